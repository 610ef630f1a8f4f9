#!/usr/bin/env python3
"""Benchmark of the EA Heisenberg spin-glass sweep on one MI355X.

A step is one full sweep (1 heat-bath + 4 over-relaxation half-sweep pairs, the
fused float64 energy, one tempering pass) of every replica of the workload.
Default workload: L = 32, 64 disorder samples x 2 copies x 32 temperatures
(geometric in [0.10, 0.30]), Gaussian couplings, zero field, float32 spins:
4096 replicas, 134,217,728 spins. Inputs are seeded and synthetic.

Prints one JSON line: ns per spin update (t / (steps x 5 x spins), the paper's
per-update time), the roofline of the dominant kernel from HIP events on the
library's stream, and the float64 oracle timed on a bounded sample of the same
workload on host cores. The dominant kernel is the over-relaxation work: for
lattices up to L = 32 two over-relaxation pairs run as one z-march (four
half-sweeps per read and write of the spins); larger lattices run each pair
separately. Both lie below the roofline ridge, so their roofline is HBM's.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Published FP32 vector peak of the MI355X (TFLOP/s, an FMA counting two flops).
PEAK_FP32_TFLOPS = 157.3
# FP32 flops one over-relaxation update needs as written (Eq. (3)): the local
# field 18 FMA (36); h.h and s.h 5 each; 2 (s.h) / (h.h) 2; the reflection 3 FMA
# (6); the compensated renormalisation 36 (three squares with their rounding
# errors 9, two error-free sums 12, the deviation from 1 6, the second-order
# correction 3, the rescaling 6).
OR_FLOPS_PER_UPDATE = 36 + 5 + 5 + 2 + 6 + 36
METRIC = "ns per spin update (HB+OR) & achieved HBM GB/s, FP32 vs batched+compressed"
STORE_BYTES = {"f32": 12, "f16": 6, "bf16": 6, "qangle": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fused(g):
    """Both half-sweeps of a pair run as one z-march when the plane fits a work-group."""
    return g.L % 4 == 0 and g.L * g.L // 4 <= 256


def or_bytes_two_pairs(groups, storage):
    """HBM bytes two over-relaxation pairs fused into one z-march must move: every
    stored spin read and written once (2 b_s per site), the couplings (and field)
    once per sample per half-sweep."""
    bs = STORE_BYTES[storage]
    total = 0.0
    for g in groups:
        coupling = 1 if g.coupling_kind == 1 else 6 * 4
        shared = coupling + (12 if g.H is not None else 0)
        total += g.n_slots * g.N * 2.0 * bs + 2 * g.n_samples * g.N * shared
    return total


def algorithmic_bytes(groups, storage, kind):
    """HBM bytes one pair of half-sweeps (parity 0 then 1) must move, all replicas.

    Fused pair (one z-march): every stored spin is written once; over-relaxation
    also reads every spin once (2 b_s per site); the heat bath reads only the
    parity-1 spins it does not overwrite first (1.5 b_s per site). Two separate
    passes (larger lattices): per update b_s written, the other parity read once,
    and over-relaxation also reads the old spin (3 b_s per pair site, 2 b_s for
    the heat bath). Couplings (six float32 per site, or one byte of sign bits for
    +-1) and fields are read once per sample per half-sweep, shared by all
    R_O R_T replicas of the sample.
    """
    bs = STORE_BYTES[storage]
    total = 0.0
    for g in groups:
        if fused(g):
            spin = (2.0 if kind == 1 else 1.5) * bs
        else:
            spin = (3.0 if kind == 1 else 2.0) * bs
        coupling = 1 if g.coupling_kind == 1 else 6 * 4
        shared = coupling + (12 if g.H is not None else 0)
        total += g.n_slots * g.N * spin + g.n_samples * g.N * shared
    return total


def time_kernel(lat, kind, n, torch):
    """Average duration of one pair of half-sweeps (one fused launch for lattices
    up to L = 32; kind 3: two over-relaxation pairs as inside a sweep, one launch
    where they fuse), from HIP events on the stream the library launches on
    (torch's current stream)."""
    stream = torch.cuda.current_stream()
    call = (lambda: lat.or_pairs(2)) if kind == 3 else (lambda: lat.pair_sweep(kind))
    call()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(n):
        call()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / n * 1e-3  # seconds per call


def time_analysis(lat, inst, torch, reps=5):
    """Mean time of one call of each measurement (HIP events on the current
    stream), with the HBM bytes they must read (every spin of copies 0 and 1, or
    of all copies for the pair sums, once; six neighbours of each come from
    cache)."""
    out = {}
    bs = STORE_BYTES[inst.storage]
    spins01 = sum(g.n_samples * min(g.n_copies, 2) * g.n_temps * g.N for g in inst.groups) * bs
    spins_all = sum(g.n_slots * g.N for g in inst.groups) * bs
    stream = torch.cuda.current_stream()
    for name, fn, nbytes in (("overlap", lat.measure_overlap, spins01),
                             ("kmodes", lat.measure_kmodes, spins01),
                             ("pair_overlaps", lat.measure_pair_overlaps, spins_all),
                             ("energy", lat.measure_energy, spins_all)):
        fn()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(reps):
            fn()
        stop.record(stream)
        stop.synchronize()
        t = start.elapsed_time(stop) / reps * 1e-3
        out[f"{name}_us"] = t * 1e6
        out[f"{name}_gbs"] = nbytes / t / 1e9
    return out


def copy_bandwidth(torch, mib=1024, reps=10):
    """Read+write GB/s of a plain device-to-device copy (the practical HBM ceiling
    next to the published 8 TB/s)."""
    n = mib << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.copy_(a)
    stop.record()
    stop.synchronize()
    t = start.elapsed_time(stop) / reps * 1e-3
    del a, b
    torch.cuda.empty_cache()
    return 2 * n / t / 1e9


def measured_traffic(build_id, workload, storage, kernel):
    """HBM bytes per launch of the dominant kernel from the hardware counters, as
    recorded in a profile summary under profiles/ by a line

        traffic: build_id=<id> workload=<name> storage=<codec> kernel=<name> bytes_per_launch=<B> ...

    (FETCH_SIZE and WRITE_SIZE of the same build, workload, spin storage and
    kernel, each scaled by what it reads for a plain copy of known size). None
    when no summary was taken with this build and launch, since counters of
    other code say nothing about it."""
    import glob
    for fn in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(fn) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                kv = dict(tok.split("=", 1) for tok in line[len("traffic:"):].split() if "=" in tok)
                if (kv.get("build_id") == build_id and kv.get("workload") == workload
                        and kv.get("storage") == storage and kv.get("kernel") == kernel):
                    return float(kv["bytes_per_launch"]), os.path.relpath(fn, ROOT)
    return None, None


def cpu_baseline(inst, sweeps, log_fn):
    """The float64 oracle, as it stands, on one sample of the workload (every
    replica of that sample), single-threaded on the host."""
    import oracle
    from paper_1204_6192_amd import inputs
    g = inst.groups[0]
    sub = inputs.Group(L=g.L, n_samples=1, n_copies=g.n_copies, temps=g.temps, J=g.J[:1],
                       H=None if g.H is None else g.H[:1], spins0=g.spins0[:1],
                       sample_uid_base=g.sample_uid_base)
    o = oracle.Oracle.from_group(sub, seed=inst.seed, n_hb=inst.n_hb, n_or=inst.n_or,
                                 pt_every=inst.pt_every)
    t0 = time.perf_counter()
    o.sweep(sweeps)
    dt = time.perf_counter() - t0
    updates = sweeps * (inst.n_hb + inst.n_or) * sub.n_slots * sub.N
    log_fn(f"oracle: {sweeps} sweeps of 1 sample ({sub.n_slots} replicas, L={g.L}) in {dt:.1f} s")
    return {"value": dt / updates * 1e9, "unit": "ns/update", "cores": 1, "kind": "oracle",
            "sample": f"1 of {g.n_samples} samples (all {sub.n_slots} replicas, L={g.L}), "
                      f"{sweeps} sweeps, {updates} updates, {dt:.1f} s"}


def roofline(inst, quad, t_or, b_or, t_quad, b_quad, t_hb, b_hb, t_hb_hw, traffic, traffic_src,
             copy_gbs):
    """HBM roofline of the dominant kernel: the over-relaxation work, two pairs in
    one z-march for lattices up to L = 32 (else one pair per launch). Its
    arithmetic intensity (OR_FLOPS_PER_UPDATE flops per update against the
    algorithmic bytes) lies below the ridge of the published peaks (157.3 TFLOP/s
    / 8 TB/s), so the roofline that bounds it is HBM's: achieved = algorithmic
    bytes per launch / mean launch time from HIP events, peak = 8 TB/s."""
    updates = sum(g.n_slots * g.N for g in inst.groups)  # per pair of half-sweeps
    if quad:
        t, nbytes, nupd = t_quad, b_quad, 2 * updates
        kernel = "k_or_quad_stream (two over-relaxation pairs, one launch)"
    else:
        t, nbytes, nupd = t_or, b_or, updates
        kernel = ("k_pair_stream (over-relaxation pair, one launch)" if all(fused(g) for g in inst.groups)
                  else "over-relaxation pair (z-march launches)")
    gbs = nbytes / t / 1e9
    flops = nupd * OR_FLOPS_PER_UPDATE
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_vs_algorithmic": None if traffic is None else traffic / nbytes,
            "traffic_source": traffic_src, "launch_us": t * 1e6, "bytes_per_launch": nbytes,
            "updates_per_launch": nupd, "frac_of_copy": gbs / copy_gbs, "device_copy_gbs": copy_gbs,
            "flops_per_update": OR_FLOPS_PER_UPDATE, "flop_per_byte": flops / nbytes,
            "ridge_flop_per_byte": PEAK_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9),
            "tflops": flops / t / 1e12,
            "or_pair_us": t_or * 1e6, "or_pair_gbs": b_or / t_or / 1e9,
            "or_pair_hbm_frac": b_or / t_or / 1e9 / PEAK_HBM_GBS,
            "hb_pair_us": t_hb * 1e6, "hb_gbs": b_hb / t_hb / 1e9, "hb_pair_us_hw_math": t_hb_hw * 1e6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="batched",
                    choices=["tiny", "batched", "field", "uneven", "large"])
    ap.add_argument("--storage", default=None, choices=["f32", "f16", "bf16", "qangle"])
    ap.add_argument("--field-amp", type=float, default=None,
                    help="random-field amplitude H_r of the field workload (default 0.1)")
    ap.add_argument("--overlap-every", type=int, default=None,
                    help="measure the overlap after every k-th sweep inside the timed region "
                         "(default: 1 for the large workload, else never)")
    ap.add_argument("--two-streams", type=int, default=None, choices=[0, 1],
                    help="sweep the two halves of the samples on two streams, one half's heat bath "
                         "beside the other's over-relaxation (default: the autotuner's choice; with "
                         "--autotune 0, 1 for the uneven workload, else 0)")
    ap.add_argument("--autotune", type=int, default=8,
                    help="before the timed run, time every launch choice over this many sweeps "
                         "(hsg_autotune, the state restored afterwards) and keep the fastest; "
                         "0 = the library's default choice")
    ap.add_argument("--kernel-variant", type=int, default=None, choices=[0, 1, 2, 3, 4],
                    help="fix the kernel variant (hsg_set_kernel) after any tuning")
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-launches", type=int, default=40)
    ap.add_argument("--copies", type=int, default=2,
                    help="copies per sample R_O (4 for the four-replica estimators in a field)")
    ap.add_argument("--tiles", type=str, default=None,
                    help="run the tile-local chain instead of the full-lattice one: TY,TZ,NHIT "
                         "(tiles of L x TY x TZ sites, 0 = L; NHIT repetitions per visit)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (disorder samples "
              "are independent and would shard across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1204_6192_amd import hsg, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_gen = time.perf_counter()
    inst = inputs.make_instance(args.config, storage=args.storage, field_amp=args.field_amp,
                                copies=args.copies)
    overlap_every = args.overlap_every
    if overlap_every is None:
        overlap_every = 1 if args.config == "large" else 0
    log(f"workload {args.config}: {len(inst.groups)} group(s), {inst.n_spins} spins, "
        f"storage {inst.storage}; inputs in {time.perf_counter() - t_gen:.1f} s")
    lat = hsg.Lattice(inst.groups, storage=inst.storage, n_hb=inst.n_hb, n_or=inst.n_or,
                      pt_every=inst.pt_every, seed=inst.seed)
    n_hit = 1
    if args.tiles:
        ty, tz, n_hit = (int(v) for v in args.tiles.split(","))
        lat.set_chain(1, ty, tz, n_hit)
        log(f"tile-local chain: tiles of L x {ty or 'L'} x {tz or 'L'}, {n_hit} repetition(s) per visit")
    if args.autotune > 0 and not args.tiles:
        t_tune = time.perf_counter()
        lat.autotune(n_sweeps=args.autotune, restore=True)
        log(f"autotune over {args.autotune} sweeps per choice: {time.perf_counter() - t_tune:.1f} s")
    if args.kernel_variant is not None:
        lat.set_kernel(args.kernel_variant)
    if args.two_streams is not None:
        lat.set_overlap(args.two_streams)
    elif args.autotune <= 0 and args.config == "uneven":
        lat.set_overlap(1)
    variant, slots, two_streams = lat.get_tuning()
    log(f"launch choice: kernel variant {variant} (0 = automatic, the two-pair z-march), slots per item "
        f"{slots}, two streams {two_streams}")
    torch.cuda.synchronize()

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n} bytes read, {n} bytes written")
        del src, dst

    q = torch.empty(sum(g.n_samples * g.n_temps * 10 for g in inst.groups), dtype=torch.float64,
                    device="cuda")
    lat.sweep(args.warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if overlap_every > 0:
        for step in range(args.steps):
            lat.sweep(1)
            if (step + 1) % overlap_every == 0:
                lat.measure_overlap(out=q)
    else:
        lat.sweep(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat.sync()
    updates = args.steps * n_hit * (inst.n_hb + inst.n_or) * lat.n_spins
    ns_update = dt / updates * 1e9
    log(f"{args.steps} sweeps in {dt:.3f} s: {ns_update * 1e3:.2f} ps/update")

    # the kernels of a sweep: heat-bath pair, over-relaxation pair, and two
    # over-relaxation pairs in one z-march where every lattice fuses them
    quad = inst.n_or >= 2 and all(fused(g) for g in inst.groups) and variant in (0, 4)
    t_or = time_kernel(lat, 1, args.kernel_launches, torch)
    t_hb = time_kernel(lat, 0, max(4, args.kernel_launches // 4), torch)
    t_quad = time_kernel(lat, 3, max(4, args.kernel_launches // 2), torch) if quad else None
    b_or = algorithmic_bytes(inst.groups, inst.storage, 1)
    b_hb = algorithmic_bytes(inst.groups, inst.storage, 0)
    b_quad = or_bytes_two_pairs(inst.groups, inst.storage)
    lat.set_math(1)
    t_hb_hw = time_kernel(lat, 0, max(4, args.kernel_launches // 4), torch)
    lat.set_math(0)
    gbs_or = b_or / t_or / 1e9
    log(f"HB pair with hardware transcendentals: {t_hb_hw * 1e6:.1f} us")
    log(f"OR pair: {t_or * 1e6:.1f} us, {b_or / 1e9:.3f} GB -> {gbs_or:.0f} GB/s; "
        f"HB pair: {t_hb * 1e6:.1f} us, {b_hb / 1e9:.3f} GB -> {b_hb / t_hb / 1e9:.0f} GB/s")
    if quad:
        log(f"two OR pairs in one z-march: {t_quad * 1e6:.1f} us, {b_quad / 1e9:.3f} GB -> "
            f"{b_quad / t_quad / 1e9:.0f} GB/s")
        b_sweep_or = (inst.n_or // 2) * b_quad + (inst.n_or % 2) * b_or
    else:
        b_sweep_or = inst.n_or * b_or
    eff_gbs = (inst.n_hb * b_hb + b_sweep_or) / (dt / args.steps) / 1e9

    analysis = time_analysis(lat, inst, torch)
    log("analysis: " + ", ".join(f"{k} {v:.1f}" for k, v in analysis.items()))
    dominant = "k_or_quad_stream" if quad else "k_pair_stream"
    traffic, traffic_src = measured_traffic(hsg.build_id(), args.config, inst.storage, dominant)
    copy_gbs = copy_bandwidth(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s read+write; OR pair at {gbs_or / copy_gbs:.1%} of it")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, args.cpu_sweeps, log)

    cfg = {"workload": args.config, "L": [g.L for g in inst.groups],
           "samples": [g.n_samples for g in inst.groups], "copies": inst.groups[0].n_copies,
           "temperatures": inst.groups[0].n_temps,
           "t_range": [float(inst.groups[0].temps[0]), float(inst.groups[0].temps[-1])],
           "couplings": "bimodal" if inst.groups[0].coupling_kind else "gaussian",
           "field": inst.groups[0].H is not None, "storage": inst.storage,
           "chain": ("full-lattice checkerboard" if not args.tiles else
                     f"tile-local, tiles L x {args.tiles.split(',')[0]} x {args.tiles.split(',')[1]} "
                     f"(0 = L), {n_hit} x ({inst.n_or} OR + {inst.n_hb} HB) per visit"),
           "sweep": f"{inst.n_hb} HB + {inst.n_or} OR + PT every {inst.pt_every}"
                    + (f" + overlap every {overlap_every}" if overlap_every else ""),
           "field_amp": None if inst.groups[0].H is None else float(
               args.field_amp if args.field_amp is not None else 0.1),
           "two_streams": bool(two_streams), "kernel_variant": variant, "slots_per_item": slots,
           "autotune_sweeps": args.autotune if not args.tiles else 0,
           "spins": lat.n_spins, "replicas": lat.n_replicas}
    out = {
        "metric": METRIC, "value": ns_update, "unit": "ns/update", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "build_id": hsg.build_id(),
        "data": "synthetic", "config": cfg,
        "effective_gbs": eff_gbs,
        "roofline": roofline(inst, quad, t_or, b_or, t_quad, b_quad, t_hb, b_hb, t_hb_hw, traffic,
                             traffic_src, copy_gbs),
        "cpu_baseline": cpu,
        "analysis": analysis,
    }
    if args.tiles:
        # the tile-local chain's kernel is VALU-bound; the HBM roofline above is the
        # full-lattice chain's over-relaxation pair, so it is not this run's
        out["roofline"] = None
        out["effective_gbs"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
