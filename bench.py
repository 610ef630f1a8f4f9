#!/usr/bin/env python3
"""Benchmark of the EA Heisenberg spin-glass sweep on one MI355X.

A step is one full sweep (1 heat-bath + 4 over-relaxation half-sweep pairs, the
fused float64 energy, one tempering pass) of every replica of the workload.
Default workload: L = 32, 64 disorder samples x 2 copies x 32 temperatures
(geometric in [0.10, 0.30]), Gaussian couplings, zero field, float32 spins:
4096 replicas, 134,217,728 spins. Inputs are seeded and synthetic.

Prints one JSON line: ns per spin update (t / (steps x 5 x spins), the paper's
per-update time, median of five timed windows of `steps` sweeps), the roofline
of the dominant kernel from HIP events on the library's stream, the same
figures for the compressed-storage workloads, and the float64 oracle timed on
a bounded sample of the workload on one host core and on all of them.

Bytes. The method's algorithmic traffic per update is one HBM pass per
half-sweep: a heat-bath update writes one stored spin and reads the six
neighbours, which amortise to one stored spin (2 b_s); over-relaxation also
reads the old spin (3 b_s); the couplings (six per site, float32 or one sign
bit each) and the field (three float32 per site) are read once per sample per
half-sweep and shared by its R_O R_T replicas. The fused kernels move less:
a fused pair, or two fused over-relaxation pairs, reads and writes every spin
once for two or four half-sweeps (exact z-march fusion, no update skipped).
The roofline therefore reports both: `achieved` and `frac` on the method's
bytes, as the contract of the measurement defines them, and `frac_own_bytes`
on the bytes the fused kernel itself must move (checked against the hardware
counters in `traffic`).
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FP32 vector peak of the MI355X without packed FP32 instructions (the library
# is compiled without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x
# 2.4 GHz. The published 157.3 TFLOP/s counts packed (two-wide) FMAs.
PEAK_FP32_TFLOPS = 78.6
# FP32 flops one over-relaxation update needs as written (Eq. (3)): the local
# field 18 FMA (36); h.h and s.h 5 each; 2 (s.h) / (h.h) 2; the reflection 3 FMA
# (6); the renormalisation of float32 spins 15 (|s|^2 - 1 as three FMA 6, the
# second-order correction 3, the rescaling 6; compressed storage skips it and
# renormalises on load).
OR_FLOPS_PER_UPDATE = 36 + 5 + 5 + 2 + 6 + 15
METRIC = "ns per spin update (HB+OR) & achieved HBM GB/s, FP32 vs batched+compressed"
STORE_BYTES = {"f32": 12, "f16": 6, "bf16": 6, "qangle": 4}
# The compressed-storage comparison run after the main workload: the batched
# workload at each compressed storage, the random-field workload at float16 and
# float32, the uneven batch at bfloat16 and the large system at quantised angles.
COMPRESSED = [("batched", "bf16"), ("batched", "f16"), ("batched", "qangle"), ("field", "f16"),
              ("field", "f32"), ("uneven", "bf16"), ("large", "qangle")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fused(g, variant=0):
    """Both half-sweeps of a pair run as one z-march when the kernel variant allows
    it (0 automatic, 3, 4, and 5, whose per-call passes run as 4) and the whole
    plane fits a work-group (L <= 32)."""
    return variant in (0, 3, 4, 5) and g.L % 4 == 0 and g.L * g.L // 4 <= 256


def quad(groups, variant, storage, n_or):
    """Two over-relaxation pairs run as one z-march in every group: variant 4 (or 5), or
    the automatic choice except for quantised angles (whose two-pair launch is
    slower than two fused pairs), where every pair fuses."""
    if n_or < 2 or not (variant in (4, 5) or (variant == 0 and storage != "qangle")):
        return False
    return all(fused(g, variant) for g in groups)


def _shared_bytes(g, bits_for_pm1):
    """Couplings and field per site of one sample."""
    if g.coupling_kind == 1:
        coupling = 6 / 8 if bits_for_pm1 else 1  # six sign bits (stored as one byte)
    else:
        coupling = 6 * 4
    return coupling + (12 if g.H is not None else 0)


def method_bytes_per_update(groups, storage, n_hb, n_or, kind=None):
    """The method's algorithmic bytes per single-site update (see the module
    docstring): 2 b_s per heat-bath update, 3 b_s per over-relaxation update,
    plus couplings and field once per sample per half-sweep, averaged over the
    updates of a sweep (kind None), or for one kind of update (0 HB, 1 OR)."""
    bs = STORE_BYTES[storage]
    total, updates = 0.0, 0.0
    for g in groups:
        share = _shared_bytes(g, True) / (g.n_slots / g.n_samples)
        if kind is None:
            per = (n_hb * 2 * bs + n_or * 3 * bs) / (n_hb + n_or) + share
        else:
            per = (3 if kind == 1 else 2) * bs + share
        total += per * g.n_slots * g.N
        updates += g.n_slots * g.N
    return total / updates


def or_bytes_two_pairs(groups, storage):
    """HBM bytes two over-relaxation pairs fused into one z-march must move: every
    stored spin read and written once (2 b_s per site), the couplings (and field)
    once per sample per half-sweep."""
    bs = STORE_BYTES[storage]
    total = 0.0
    for g in groups:
        total += g.n_slots * g.N * 2.0 * bs + 2 * g.n_samples * g.N * _shared_bytes(g, False)
    return total


def algorithmic_bytes(groups, storage, kind, variant=0):
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
        if fused(g, variant):
            spin = (2.0 if kind == 1 else 1.5) * bs
        else:
            spin = (3.0 if kind == 1 else 2.0) * bs
        total += g.n_slots * g.N * spin + g.n_samples * g.N * _shared_bytes(g, False)
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


def time_sweeps(lat, steps, windows, torch, overlap_every=0, q=None):
    """Seconds of each of `windows` timed windows of exactly `steps` sweeps, each
    bracketed by device synchronisations (wall clock)."""
    out = []
    for _ in range(windows):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if overlap_every > 0:
            for step in range(steps):
                lat.sweep(1)
                if (step + 1) % overlap_every == 0:
                    lat.measure_overlap(out=q)
        else:
            lat.sweep(steps)
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    lat.sync()
    return out


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


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inst, sweeps, log_fn):
    """The float64 oracle, as it stands, on the workload's samples: one sample
    (every replica of it) on one host core, then one sample per thread on all
    the host cores the process may use (each sample's chain stays serial)."""
    import oracle
    from paper_1204_6192_amd import inputs
    g = inst.groups[0]

    def sub(d):
        return inputs.Group(L=g.L, n_samples=1, n_copies=g.n_copies, temps=g.temps, J=g.J[d:d + 1],
                            H=None if g.H is None else g.H[d:d + 1], spins0=g.spins0[d:d + 1],
                            sample_uid_base=g.sample_uid_base + d)

    def make(d):
        return oracle.Oracle.from_group(sub(d), seed=inst.seed, n_hb=inst.n_hb, n_or=inst.n_or,
                                        pt_every=inst.pt_every)

    per_sample = (inst.n_hb + inst.n_or) * g.n_copies * g.n_temps * g.N
    o = make(0)
    t0 = time.perf_counter()
    o.sweep(sweeps)
    dt1 = time.perf_counter() - t0
    one = dt1 / (sweeps * per_sample) * 1e9
    log_fn(f"oracle, one core: {sweeps} sweeps of 1 sample ({g.n_copies * g.n_temps} replicas, "
           f"L={g.L}) in {dt1:.1f} s: {one:.1f} ns/update")
    threads = min(host_threads(), g.n_samples)
    orcs = [make(d) for d in range(threads)]
    t0 = time.perf_counter()
    oracle.sweep_parallel(orcs, sweeps, threads)
    dtn = time.perf_counter() - t0
    alln = dtn / (sweeps * per_sample * threads) * 1e9
    log_fn(f"oracle, {threads} threads: {sweeps} sweeps of {threads} samples in {dtn:.1f} s: "
           f"{alln:.2f} ns/update")
    return {"value": alln, "unit": "ns/update", "cores": threads, "kind": "oracle",
            "sample": f"{threads} of {g.n_samples} samples (all {g.n_copies * g.n_temps} replicas each, "
                      f"L={g.L}), one sample per thread, {sweeps} sweeps, "
                      f"{sweeps * per_sample * threads} updates, {dtn:.1f} s",
            "cpu_model": cpu_model(),
            "one_core": {"value": one, "unit": "ns/update", "cores": 1,
                         "sample": f"1 sample (all {g.n_copies * g.n_temps} replicas), {sweeps} sweeps, "
                                   f"{sweeps * per_sample} updates, {dt1:.1f} s"}}


def roofline(inst, variant, is_quad, t_or, t_quad, t_hb, t_hb_hw, traffic, traffic_src, copy_gbs,
             sweep_s):
    """HBM roofline of the dominant kernel: the over-relaxation work, two pairs in
    one z-march for lattices up to L = 32 (else one pair per launch). Its
    arithmetic intensity (OR_FLOPS_PER_UPDATE flops per update) lies below the
    ridge of the FP32 vector peak against 8 TB/s, so HBM bounds it. achieved =
    the method's algorithmic bytes per launch / mean launch time from HIP events;
    frac_own_bytes uses the bytes the fused launch itself must move."""
    groups = inst.groups
    updates = sum(g.n_slots * g.N for g in groups)  # per pair of half-sweeps
    b_pair_own = algorithmic_bytes(groups, inst.storage, 1, variant)
    if is_quad:
        t, own, nupd = t_quad, or_bytes_two_pairs(groups, inst.storage), 2 * updates
        kernel = "k_or_quad_stream (two over-relaxation pairs, one launch)"
    else:
        t, own, nupd = t_or, b_pair_own, updates
        kernel = ("k_pair_stream (over-relaxation pair, one launch)" if all(fused(g, variant) for g in groups)
                  else "over-relaxation pair (z-march launches)")
    per_or = method_bytes_per_update(groups, inst.storage, inst.n_hb, inst.n_or, kind=1)
    method = per_or * nupd
    gbs = method / t / 1e9
    own_gbs = own / t / 1e9
    sweep_bytes = method_bytes_per_update(groups, inst.storage, inst.n_hb, inst.n_or) * \
        (inst.n_hb + inst.n_or) * updates
    flops = nupd * OR_FLOPS_PER_UPDATE
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_source": traffic_src,
            "method_bytes_per_update": per_or, "updates_per_launch": nupd, "bytes_per_launch": method,
            "launch_us": t * 1e6,
            "fusion_note": ("four half-sweeps per read and write of every spin (two per launch for a fused "
                            "pair): the launch moves less than one HBM pass per half-sweep, so achieved on "
                            "the method's bytes can exceed the HBM peak; no update is skipped")
            if is_quad or all(fused(g, variant) for g in groups) else None,
            "own_bytes_per_launch": own, "own_gbs": own_gbs, "frac_own_bytes": own_gbs / PEAK_HBM_GBS,
            "traffic_vs_own_bytes": None if traffic is None else traffic / own,
            "frac_own_of_copy": own_gbs / copy_gbs, "device_copy_gbs": copy_gbs,
            "sweep_method_gbs": sweep_bytes / sweep_s / 1e9,
            "frac_sweep": sweep_bytes / sweep_s / 1e9 / PEAK_HBM_GBS,
            "flops_per_update": OR_FLOPS_PER_UPDATE, "flop_per_byte": flops / own,
            "ridge_flop_per_byte": PEAK_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9),
            "tflops": flops / t / 1e12,
            "or_pair_us": t_or * 1e6, "or_pair_own_gbs": b_pair_own / t_or / 1e9,
            "hb_pair_us": t_hb * 1e6,
            "hb_own_gbs": algorithmic_bytes(groups, inst.storage, 0, variant) / t_hb / 1e9,
            "hb_pair_us_hw_math": t_hb_hw * 1e6}


def make_lattice(hsg, inst, storage, tiles=None):
    lat = hsg.Lattice(inst.groups, storage=storage, n_hb=inst.n_hb, n_or=inst.n_or,
                      pt_every=inst.pt_every, seed=inst.seed)
    n_hit = 1
    if tiles:
        v = [int(x) for x in tiles.split(",")]
        tx, ty, tz, n_hit = v if len(v) == 4 else [0] + v
        lat.set_chain(1, ty, tz, n_hit, tile_x=tx)
    return lat, n_hit


def compressed_entry(hsg, torch, inst, storage, steps, windows, autotune):
    """ns per update and the method's HBM fraction of one workload and storage
    (median of the timed windows; the overlap every sweep for the large system)."""
    lat, _ = make_lattice(hsg, inst, storage)
    if autotune > 0:
        lat.autotune(n_sweeps=autotune, restore=True)
    variant, slots, two = lat.get_tuning()
    geometry = [list(lat.get_geometry(k)) for k in range(len(inst.groups))]
    q = None
    every = 1 if inst.name == "large" else 0
    if every:
        q = torch.empty(sum(g.n_samples * g.n_temps * 10 for g in inst.groups), dtype=torch.float64,
                        device="cuda")
    lat.sweep(10)
    ws = time_sweeps(lat, steps, windows, torch, every, q)
    t = statistics.median(ws) / steps
    updates = (inst.n_hb + inst.n_or) * lat.n_spins
    bpu = method_bytes_per_update(inst.groups, storage, inst.n_hb, inst.n_or)
    lat.close()
    del lat, q
    torch.cuda.empty_cache()
    return {"workload": inst.name, "storage": storage, "L": [g.L for g in inst.groups],
            "spins": inst.n_spins, "ns_per_update": t / updates * 1e9, "ms_per_step": t * 1e3,
            "windows_ms": [w / steps * 1e3 for w in ws], "method_bytes_per_update": bpu,
            "method_gbs": bpu * updates / t / 1e9, "frac": bpu * updates / t / 1e9 / PEAK_HBM_GBS,
            "kernel_variant": variant, "two_streams": bool(two), "geometry": geometry,
            "sweep": f"{inst.n_hb} HB + {inst.n_or} OR + PT every {inst.pt_every}"
                     + (" + overlap every sweep" if every else "")}


# The paper's Table 1 (ns per update on its GPU, float and fast_math), beside
# which the same update mixes are timed on the same workload shape: 256
# systems of L = 32 at T = 100. Rows: (label, n_hb, n_or, tile chain, paper ns
# float, paper ns fast_math); the tile rows visit 8 x 8 x 8 tiles with ten
# repetitions of (1 HB + 10 OR) per visit.
TABLE1 = [("1 HB", 1, 0, False, 2.23, 1.58), ("1 OR", 0, 1, False, 1.30, 1.30),
          ("1 HB + 10 OR", 1, 10, False, 0.45, 0.39), ("1 HB + 100 OR", 1, 100, False, 0.29, None),
          ("10 x (1 HB + 10 OR)", 1, 10, True, 0.36, 0.31)]


def table1_context(hsg, torch, inputs, sweeps=6):
    """ns per update of each Table 1 mix on its workload (context only: the
    paper's GPU, update mix and temperature differ from the benchmark's), with
    the library's default heat-bath arithmetic and with the hardware
    transcendentals (the analogue of the paper's fast_math rows)."""
    inst = inputs.make_instance("table1")
    rows = []
    for label, n_hb, n_or, tiles, paper, paper_fast in TABLE1:
        lat = hsg.Lattice(inst.groups, storage="f32", n_hb=n_hb, n_or=n_or, pt_every=0, seed=inst.seed)
        n_hit = 1
        if tiles:
            n_hit = 10
            lat.set_chain(1, 8, 8, n_hit, tile_x=8)
        row = {"update": label, "chain": "tile-local 8x8x8" if tiles else "full-lattice checkerboard",
               "paper_ns_float": paper, "paper_ns_fast_math": paper_fast}
        for mode in (0, 1):
            if mode == 1 and n_hb == 0:
                continue
            lat.set_math(mode)
            lat.sweep(2)
            ws = time_sweeps(lat, sweeps, 3, torch)
            t = statistics.median(ws) / sweeps
            row["ns_hw_math" if mode else "ns"] = t / (n_hit * (n_hb + n_or) * lat.n_spins) * 1e9
        lat.close()
        del lat
        rows.append(row)
    torch.cuda.empty_cache()
    return {"workload": "256 systems (128 samples x 2 copies) of L = 32 at T = 100, Gaussian J, float32",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps sweeps each; the median is reported")
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
    ap.add_argument("--kernel-variant", type=int, default=None, choices=[0, 1, 2, 3, 4, 5],
                    help="fix the kernel variant (hsg_set_kernel) after any tuning")
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compressed", default="all",
                    help="'all' (default): also time the compressed-storage workloads; 'none': skip; "
                         "or a comma list of workload:storage")
    ap.add_argument("--compressed-steps", type=int, default=20)
    ap.add_argument("--no-table1", action="store_true",
                    help="skip timing the paper's Table 1 update mixes on its workload (context)")
    ap.add_argument("--kernel-launches", type=int, default=40)
    ap.add_argument("--copies", type=int, default=2,
                    help="copies per sample R_O (4 for the four-replica estimators in a field)")
    ap.add_argument("--tiles", type=str, default=None,
                    help="run the tile-local chain instead of the full-lattice one: [TX,]TY,TZ,NHIT "
                         "(tiles of TX x TY x TZ sites, 0 = L; NHIT repetitions per visit)")
    ap.add_argument("--n-or", type=int, default=None,
                    help="over-relaxation pairs per sweep (default: the workload's, 4)")
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
    if args.n_or is not None:
        inst.n_or = args.n_or
    overlap_every = args.overlap_every
    if overlap_every is None:
        overlap_every = 1 if args.config == "large" else 0
    log(f"workload {args.config}: {len(inst.groups)} group(s), {inst.n_spins} spins, "
        f"storage {inst.storage}; inputs in {time.perf_counter() - t_gen:.1f} s")
    lat, n_hit = make_lattice(hsg, inst, inst.storage, args.tiles)
    if args.tiles:
        log(f"tile-local chain: tiles of L x {args.tiles}")
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
    windows = time_sweeps(lat, args.steps, max(1, args.windows), torch, overlap_every, q)
    dt = statistics.median(windows)
    updates = args.steps * n_hit * (inst.n_hb + inst.n_or) * lat.n_spins
    ns_update = dt / updates * 1e9
    log(f"{args.windows} windows of {args.steps} sweeps: " +
        ", ".join(f"{w:.4f}" for w in windows) + f" s; median {ns_update * 1e3:.2f} ps/update")

    out = {
        "metric": METRIC, "value": ns_update, "unit": "ns/update", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "build_id": hsg.build_id(), "data": "synthetic",
        "windows_ms_per_step": [w / args.steps * 1e3 for w in windows],
    }
    cfg = {"workload": args.config, "L": [g.L for g in inst.groups],
           "samples": [g.n_samples for g in inst.groups], "copies": inst.groups[0].n_copies,
           "temperatures": inst.groups[0].n_temps,
           "t_range": [float(inst.groups[0].temps[0]), float(inst.groups[0].temps[-1])],
           "couplings": "bimodal" if inst.groups[0].coupling_kind else "gaussian",
           "field": inst.groups[0].H is not None, "storage": inst.storage,
           "chain": ("full-lattice checkerboard" if not args.tiles else
                     f"tile-local, tiles {args.tiles} ([TX,]TY,TZ,NHIT; 0 = L), "
                     f"{n_hit} x ({inst.n_or} OR + {inst.n_hb} HB) per visit"),
           "sweep": f"{inst.n_hb} HB + {inst.n_or} OR + PT every {inst.pt_every}"
                    + (f" + overlap every {overlap_every}" if overlap_every else ""),
           "field_amp": None if inst.groups[0].H is None else float(
               args.field_amp if args.field_amp is not None else 0.1),
           "two_streams": bool(two_streams), "kernel_variant": variant, "slots_per_item": slots,
           "geometry": [list(lat.get_geometry(k)) for k in range(len(inst.groups))],
           "autotune_sweeps": args.autotune if not args.tiles else 0,
           "spins": lat.n_spins, "replicas": lat.n_replicas}
    out["config"] = cfg

    if args.tiles:
        # the tile-local chain's kernel is bound by instruction issue; no HBM roofline
        out["roofline"] = None
    else:
        # the kernels of a sweep: heat-bath pair, over-relaxation pair, and two
        # over-relaxation pairs in one z-march where every lattice fuses them
        is_quad = quad(inst.groups, variant, inst.storage, inst.n_or)
        t_or = time_kernel(lat, 1, args.kernel_launches, torch)
        t_hb = time_kernel(lat, 0, max(4, args.kernel_launches // 4), torch)
        t_quad = time_kernel(lat, 3, max(4, args.kernel_launches // 2), torch) if is_quad else None
        lat.set_math(1)
        t_hb_hw = time_kernel(lat, 0, max(4, args.kernel_launches // 4), torch)
        lat.set_math(0)
        log(f"OR pair {t_or * 1e6:.1f} us; HB pair {t_hb * 1e6:.1f} us (hardware transcendentals "
            f"{t_hb_hw * 1e6:.1f} us)" + (f"; two OR pairs in one launch {t_quad * 1e6:.1f} us" if is_quad else ""))
        out["analysis"] = time_analysis(lat, inst, torch)
        log("analysis: " + ", ".join(f"{k} {v:.1f}" for k, v in out["analysis"].items()))
        dominant = "k_or_quad_stream" if is_quad else "k_pair_stream"
        traffic, traffic_src = measured_traffic(hsg.build_id(), args.config, inst.storage, dominant)
        copy_gbs = copy_bandwidth(torch)
        out["roofline"] = roofline(inst, variant, is_quad, t_or, t_quad, t_hb, t_hb_hw, traffic,
                                   traffic_src, copy_gbs, dt / args.steps)
        r = out["roofline"]
        log(f"dominant kernel {r['kernel']}: {r['launch_us']:.1f} us; method bytes {r['achieved']:.0f} GB/s "
            f"({r['frac']:.3f} of 8 TB/s), own bytes {r['own_gbs']:.0f} GB/s ({r['frac_own_bytes']:.3f}); "
            f"sweep {r['sweep_method_gbs']:.0f} GB/s ({r['frac_sweep']:.3f}); device copy {copy_gbs:.0f} GB/s")
    lat.close()
    del lat, q
    torch.cuda.empty_cache()

    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_sweeps, log)

    out["compressed"] = None
    if args.compressed != "none" and args.config == "batched" and not args.tiles and args.n_or is None:
        todo = COMPRESSED if args.compressed == "all" else [
            tuple(x.split(":")) for x in args.compressed.split(",") if x]
        entries, cache = [], {}
        for name, storage in todo:
            if name not in cache:
                cache.clear()
                cache[name] = inst if name == args.config else inputs.make_instance(name)
            e = compressed_entry(hsg, torch, cache[name], storage, args.compressed_steps, max(1, args.windows),
                                 min(args.autotune, 4))
            log(f"compressed {name} {storage}: {e['ns_per_update'] * 1e3:.2f} ps/update, method bytes "
                f"{e['method_gbs']:.0f} GB/s ({e['frac']:.3f}), variant {e['kernel_variant']}")
            entries.append(e)
        out["compressed"] = entries
    out["table1_context"] = None
    if not args.no_table1 and args.config == "batched" and not args.tiles and args.n_or is None:
        out["table1_context"] = table1_context(hsg, torch, inputs)
        for r in out["table1_context"]["rows"]:
            log(f"Table 1 context {r['update']} ({r['chain']}): {r['ns'] * 1e3:.1f} ps/update"
                + (f", hardware math {r['ns_hw_math'] * 1e3:.1f}" if "ns_hw_math" in r else "")
                + f" (paper {r['paper_ns_float']} ns)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
