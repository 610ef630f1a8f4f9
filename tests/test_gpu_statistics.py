"""GPU statistics against the oracle: long-run averages, run statistics, the
per-sweep series and the four-replica estimators.

* Long runs (E and q^2 per rung, Eqs. (1), (4), (5)): the GPU and the oracle
  sample the same distribution on the ladder every workload uses,
  [0.10, 0.30], and on [0.20, 0.60]; the estimator and its calibration are in
  tests/longrun.py and tests/test_oracle_longrun.py.
* Run statistics (U_L, C_L and tempering round trips): the device sums and
  trip counts equal what the oracle's bookkeeping makes of the same chain's
  temperature maps and energies, sweep by sweep.
* The per-sweep series: every record equals the oracle's energy and overlap of
  the GPU's configuration after that sweep.
* chi_1, chi_2, chi_3 (Eqs. (9)-(11)): the oracle's double sums over site pairs
  on the GPU's configurations.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1204_6192_amd import inputs  # noqa: E402

import longrun  # noqa: E402


@pytest.fixture(scope="module")
def hsg():
    from paper_1204_6192_amd import hsg as mod
    return mod


def _split(flat, lat, per_group):
    """Cut a flat per-group output into the groups' blocks."""
    out, off = [], 0
    for g in lat.groups:
        n = per_group(g)
        out.append(flat[off:off + n])
        off += n
    return out


def _gpu_state(lat, k):
    g = lat.groups[k]
    s = _split(lat.get_spins().cpu().numpy(), lat, lambda g: g.n_slots * 3 * g.N)[k]
    m = _split(lat.get_temp_map().cpu().numpy(), lat, lambda g: g.n_slots)[k]
    return (s.reshape(g.n_samples, g.n_copies, g.n_temps, 3, g.N),
            m.reshape(g.n_samples, g.n_copies, g.n_temps))


def _oracle_at(oracle_lib, lat, k, seed):
    g = lat.groups[k]
    o = oracle_lib.Oracle.from_group(g, seed=seed)
    s, m = _gpu_state(lat, k)
    o.spins = np.ascontiguousarray(s, dtype=np.float64)
    o.slot_at_temp = np.ascontiguousarray(m, dtype=np.int32)
    return o


# ---------------------------------------------------------------- long runs
@pytest.mark.parametrize("ladder", [(0.10, 0.30), (0.20, 0.60)])
def test_gpu_long_run_statistics_vs_oracle(hsg, oracle_lib, ladder):
    """500 sweeps of 16 samples (L = 8, 2 x 8 rungs) on the GPU (energies and
    q^2 by rung recorded by the per-sweep series) and in the oracle, from the
    same start: per-rung time averages of E and q^2 after 100 sweeps agree,
    with error bars from the scatter over samples (|z| < 4 per rung, < 3.5
    averaged over rungs; t with 15 degrees of freedom)."""
    g = longrun.group(ladder)
    seed = inputs.PHILOX_KEY_BASE + 50
    lat = hsg.Lattice([g], seed=seed)
    buf = lat.set_series(longrun.SWEEPS)
    lat.sweep(longrun.SWEEPS)
    assert lat.get_series_count() == longrun.SWEEPS
    rec = buf.cpu().numpy()
    D, T = g.n_samples, g.n_temps
    Eg = rec[:, :D * 2 * T].reshape(-1, D, 2, T).mean(axis=2)
    Qg = rec[:, D * 2 * T:].reshape(-1, D, T)
    Eo, Qo = longrun.oracle_series(oracle_lib, g, seed)
    for name, A, B in (("E", Eg, Eo), ("q2", Qg, Qo)):
        z, z_all = longrun.zscores(A, B)
        print(f"ladder {ladder} {name}: z per rung {np.round(z, 2)}, all rungs {z_all:.2f}", flush=True)
        assert np.all(np.abs(z) < longrun.Z_RUNG_MAX), (name, z)
        assert abs(z_all) < longrun.Z_ALL_MAX, (name, z_all)


# ---------------------------------------------------------------- run statistics
@pytest.mark.parametrize("tiles", [None, (4, 4, 1)])
def test_run_statistics_against_oracle(hsg, oracle_lib, tiles):
    """Per-rung sums of E and E^2 and tempering round trips accumulated on the
    GPU after every sweep (replayed graphs; full-lattice and tile-local chains)
    against the oracle's bookkeeping (stats_record) of the same chain's maps and
    energies, read after each sweep; U_L and C_L from the oracle's formula; then
    reset."""
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 49))
    T = 4
    g = inputs.make_group(rng, 4, 2, 2, inputs.geometric_ladder(0.8, 1.0, T))  # close rungs: swaps
    lat = hsg.Lattice([g], seed=inputs.PHILOX_KEY_BASE + 49)
    if tiles:
        lat.set_chain(1, *tiles)
    lat.set_stats(True)
    cfg = oracle_lib.Oracle.from_group(g, seed=0).cfg
    st = oracle_lib.new_stats(g.n_samples, g.n_copies, T)
    for t in range(120):
        lat.sweep(1)
        sat = lat.get_temp_map().cpu().numpy().reshape(g.n_samples, g.n_copies, T)
        E = lat.get_energies().cpu().numpy().reshape(g.n_samples, g.n_copies, T)
        oracle_lib.stats_record(cfg, E, sat, st)
    gs, gt, n = lat.get_stats()
    assert n == 120 == st["n"]
    gs = gs.cpu().numpy().reshape(g.n_samples, g.n_copies, T, 2)
    assert np.array_equal(gs[..., 0], st["sum_e"]) and np.array_equal(gs[..., 1], st["sum_e2"])
    trips = gt.cpu().numpy().reshape(g.n_samples, g.n_copies, T)
    assert np.array_equal(trips, st["trips"].astype(np.int64))
    print(f"round trips per replica: {trips.ravel().tolist()}", flush=True)
    assert trips.sum() > 0  # hot ladder: replicas do travel
    U, Cv = oracle_lib.stats_finish(cfg, g.temps, st)
    assert np.allclose(gs[..., 0] / n, U, rtol=1e-15)
    lat.reset_stats()
    gs, gt, n = lat.get_stats()
    assert n == 0 and float(gs.abs().max()) == 0.0 and int(gt.abs().max()) == 0


def test_run_statistics_follow_the_oracle_chain(hsg, oracle_lib):
    """The tiny workload's first sweeps, where GPU and oracle still take the same
    tempering decisions: the GPU's statistics equal the oracle chain's own
    (sums to the float32 rounding of the energies, round trips exactly)."""
    inst = inputs.make_instance("tiny")
    g = inst.groups[0]
    lat = hsg.Lattice(inst.groups, seed=inst.seed)
    lat.set_stats(True)
    o = oracle_lib.Oracle.from_group(g, seed=inst.seed)
    o.enable_stats()
    for _ in range(4):
        lat.sweep(1)
        o.sweep(1)
        assert np.array_equal(lat.get_temp_map().cpu().numpy().reshape(o.slot_at_temp.shape), o.slot_at_temp)
    gs, gt, n = lat.get_stats()
    sums, trips, no, U, Cv = o.get_stats()
    assert n == no == 4
    gs = gs.cpu().numpy().reshape(sums.shape)
    assert np.allclose(gs, sums, rtol=1e-5)
    assert np.array_equal(gt.cpu().numpy().reshape(trips.shape), trips.astype(np.int64))


def test_autotune_restores_the_statistics(hsg):
    """With a backup buffer the autotuner leaves the run statistics as they were:
    sums, round trips and the count of sweeps recorded."""
    inst = inputs.make_instance("tiny")
    a = hsg.Lattice(inst.groups, seed=inst.seed)
    ref = hsg.Lattice(inst.groups, seed=inst.seed)
    for lat in (a, ref):
        lat.set_stats(True)
        lat.sweep(5)
    a.autotune(n_sweeps=1, restore=True)
    sa, ta, na = a.get_stats()
    sr, tr, nr = ref.get_stats()
    assert na == nr == 5
    assert torch.equal(sa, sr) and torch.equal(ta, tr)
    a.sweep(3)
    ref.sweep(3)
    sa, ta, na = a.get_stats()
    sr, tr, nr = ref.get_stats()
    assert na == nr == 8 and torch.equal(ta, tr)
    assert torch.allclose(sa, sr, rtol=1e-12)


# ---------------------------------------------------------------- series
@pytest.mark.parametrize("storage", ["f32", "qangle"])
def test_series_against_oracle(hsg, oracle_lib, storage):
    """Two lattice sizes in one handle (L = 6 runs the gather kernel, L = 8 the
    fused z-march), one with a single copy (energies only): after each of six
    sweeps, the series record of that sweep equals the oracle's energies (by
    rung) and overlap q^2 of the GPU's configuration. A capacity of five keeps
    five records; switching the series off stops recording."""
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 51))
    groups = [inputs.make_group(rng, 6, 2, 2, inputs.geometric_ladder(0.1, 0.3, 3)),
              inputs.make_group(rng, 8, 1, 1, inputs.geometric_ladder(0.1, 0.3, 4), sample_uid_base=2)]
    seed = inputs.PHILOX_KEY_BASE + 51
    lat = hsg.Lattice(groups, seed=seed, storage=storage)
    lat.sweep(2)
    buf = lat.set_series(5)
    for t in range(6):
        lat.sweep(1)
        assert lat.get_series_count() == min(t + 1, 5)
        if t >= 5:
            continue
        rec = buf[t].cpu().numpy()
        off = 0
        for k, g in enumerate(groups):
            o = _oracle_at(oracle_lib, lat, k, seed)
            E = o.compute_energies()  # by slot
            by_rung = np.take_along_axis(E, o.slot_at_temp, axis=2)
            n = g.n_slots
            got = rec[off:off + n].reshape(by_rung.shape)
            assert np.allclose(got, by_rung, rtol=1e-11, atol=1e-9), (t, k)
            off += n
            if g.n_copies >= 2:
                q2 = o.measure_overlap()[:, :, 9]
                got = rec[off:off + q2.size].reshape(q2.shape)
                assert np.allclose(got, q2, rtol=1e-12, atol=1e-14), (t, k)
                off += q2.size
        assert off == rec.size
    lat.set_series(0)
    lat.sweep(1)
    assert lat.get_series_count() == 0


def test_series_graph_replay_bit_identical(hsg):
    """Sweeps replayed eight at a time as a captured graph record the same series
    as single sweeps, and the same as direct launches."""
    inst = inputs.make_instance("batched", scale_samples=2, L_override=8)
    bufs = []
    for mode in ("one", "eight", "direct"):
        lat = hsg.Lattice(inst.groups, seed=inst.seed)
        if mode == "direct":
            lat.set_graphs(False)
        buf = lat.set_series(17)
        if mode == "one":
            for _ in range(17):
                lat.sweep(1)
        else:
            lat.sweep(17)
        assert lat.get_series_count() == 17
        bufs.append(buf.cpu())
    assert torch.equal(bufs[0], bufs[1]) and torch.equal(bufs[0], bufs[2])
    assert not torch.isnan(bufs[0]).any()


# ---------------------------------------------------------------- chi_1, chi_2, chi_3
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_chi_against_oracle(hsg, oracle_lib, storage):
    """Four copies per sample in a random field, three lattice sizes in one handle
    (L = 6 with odd L/2, L = 4 and 8), after sweeps with tempering: chi_1, chi_2,
    chi_3 of Eq. (10) against the oracle's double sums over site pairs of the
    same configurations."""
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 52))
    groups, uid = [], 0
    for L, D in ((4, 2), (6, 1), (8, 1)):
        groups.append(inputs.make_group(rng, L, D, 4, inputs.geometric_ladder(0.1, 0.5, 3),
                                        field=("gaussian", 0.2), sample_uid_base=uid))
        uid += D
    seed = inputs.PHILOX_KEY_BASE + 52
    lat = hsg.Lattice(groups, seed=seed, storage=storage)
    lat.sweep(4)
    chi = _split(lat.measure_chi().cpu().numpy(), lat, lambda g: g.n_samples * g.n_temps * 20)
    for k, g in enumerate(groups):
        want = _oracle_at(oracle_lib, lat, k, seed).measure_chi4()
        got = chi[k].reshape(want.shape)
        err = np.abs(got - want).max() / g.N ** 2
        print(f"L={g.L}: max |dchi| / N^2 {err:.2e}", flush=True)
        assert err < 1e-12


def test_chi_full_size_sampled(hsg, oracle_lib):
    """The random-field workload (L = 64, float16 storage) with four copies per
    sample, 16 samples x 24 rungs, after one sweep: chi_1, chi_2, chi_3 of two
    samples at three rungs from the oracle's copy-pair sums of the GPU's
    configurations, through the factorisation of the double sums (the oracle's
    pair sums are pinned to the double sums on small lattices)."""
    inst = inputs.make_instance("field", copies=4)
    g = inst.groups[0]
    lat = hsg.Lattice(inst.groups, seed=inst.seed, storage=inst.storage)
    lat.sweep(1)
    chi = lat.measure_chi().cpu().numpy().reshape(g.n_samples, g.n_temps, 4, 5)
    s, m = _gpu_state(lat, 0)
    N = g.N
    for d in (0, 11):
        for k in (0, 9, 23):
            sub = inputs.Group(L=g.L, n_samples=1, n_copies=4, temps=g.temps[:1], J=g.J[d:d + 1],
                               H=g.H[d:d + 1], spins0=np.zeros((1, 4, 1, 3, N), np.float32),
                               sample_uid_base=g.sample_uid_base + d)
            o = oracle_lib.Oracle.from_group(sub, seed=inst.seed)
            o.spins = np.ascontiguousarray(
                np.stack([s[d, a, m[d, a, k]] for a in range(4)])[None, :, None], dtype=np.float64)
            o.slot_at_temp = np.zeros((1, 4, 1), np.int32)
            A = o.measure_pair_overlaps()[0, 0]  # [6 pairs][7]

            def cplx(p, w):
                return A[p, 0] + 0j if w == 0 else A[p, 1 + 2 * (w - 1)] + 1j * A[p, 2 + 2 * (w - 1)]

            for w in range(4):
                a01, a02, a03, a13 = (cplx(p, w) for p in (0, 1, 2, 4))
                c1 = N * N * a01 * np.conj(a01)
                c2 = N * N * a02 * np.conj(a03)
                c3 = N * N * a02 * np.conj(a13)
                want = np.array([c1.real, c2.real, c2.imag, c3.real, c3.imag])
                err = np.abs(chi[d, k, w] - want).max() / N ** 2
                assert err < 1e-12, (d, k, w, err)
