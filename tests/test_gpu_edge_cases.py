"""Degenerate and extreme inputs on the GPU: one copy and one temperature, zero
couplings and field, a large single lattice."""

import numpy as np
import pytest
import torch

from paper_1204_6192_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hsg():
    from paper_1204_6192_amd import hsg as mod
    return mod


def test_one_copy_one_temperature(hsg):
    """A ladder of one rung: tempering never swaps, the map stays the identity;
    overlap measurements need two copies and are refused."""
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 70))
    g = inputs.make_group(rng, 8, 3, 1, [0.5])
    lat = hsg.Lattice([g], seed=inputs.PHILOX_KEY_BASE + 70)
    lat.sweep(5)
    assert torch.equal(lat.get_temp_map().cpu(), torch.zeros(3, dtype=torch.int32))
    assert int(lat.get_pt_accepts().numel()) in (0, 3)
    E = lat.get_energies()
    assert torch.allclose(E, lat.measure_energy(), rtol=1e-11)
    for fn in (lat.measure_overlap, lat.measure_kmodes, lat.measure_pair_overlaps):
        with pytest.raises(hsg.HSGError):
            fn()


@pytest.mark.parametrize("tiles", [None, (4, 4, 2)])
def test_zero_couplings_and_field(hsg, tiles):
    """H_eff = 0 everywhere: over-relaxation leaves every spin unchanged (bit for
    bit), the heat bath draws uniform directions (mean 0, second moment 1/3 per
    component over 1.3 * 10^5 spins), and every energy is exactly 0."""
    L, D = 16, 4
    N = L ** 3
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 71))
    g = inputs.make_group(rng, L, D, 2, inputs.geometric_ladder(0.2, 0.4, 4), couplings="zero")
    only_or = hsg.Lattice([g], seed=inputs.PHILOX_KEY_BASE + 71, n_hb=0, n_or=3)
    if tiles:
        only_or.set_chain(1, *tiles)
    s0 = only_or.get_spins().clone()
    only_or.sweep(2)
    assert torch.equal(only_or.get_spins(), s0)
    assert float(only_or.get_energies().abs().max()) == 0.0
    hb = hsg.Lattice([g], seed=inputs.PHILOX_KEY_BASE + 71, n_hb=1, n_or=0)
    if tiles:
        hb.set_chain(1, *tiles)
    hb.sweep(3)
    s = hb.get_spins().cpu().numpy().reshape(-1, 3, N)
    m1 = s.mean(axis=(0, 2))
    m2 = (s ** 2).mean(axis=(0, 2))
    n = s.shape[0] * N
    print(f"mean {m1}, second moment {m2} over {n} spins", flush=True)
    assert np.all(np.abs(m1) < 5.0 / np.sqrt(3 * n))
    assert np.all(np.abs(m2 - 1.0 / 3.0) < 5.0 * np.sqrt(4.0 / 45.0 / n))
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=3e-7)


def test_large_single_lattice_half_sweep(hsg, oracle_lib):
    """L = 256 (16.8 M sites per replica, 32-bit offsets near their working
    range), one sample, copy and temperature: one over-relaxation and one
    heat-bath half-sweep, every spin of both checked against the oracle started
    from the GPU's own spins: within 1e-4, and within a per-site bound from the
    conditioning of the update (1 / |H_eff|; for the heat bath also the frame's
    pole at n = -z)."""
    L = 256
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 72))
    g = inputs.make_group(rng, L, 1, 1, [0.3], couplings="bimodal")
    seed = inputs.PHILOX_KEY_BASE + 72
    lat = hsg.Lattice([g], seed=seed)
    o = oracle_lib.Oracle.from_group(g, seed=seed)
    J = g.J[0].reshape(3, L, L, L).astype(np.float64)  # J_a(i) couples i and i + e_a; axes z, y, x
    for kind, parity in ((1, 0), (0, 1)):
        pre = lat.get_spins().cpu().numpy().reshape(o.spins.shape).astype(np.float64)
        o.spins = pre.copy()
        lat.half_sweep(kind, parity)
        o.half_sweep(kind, parity)
        d = np.abs(lat.get_spins().cpu().numpy().reshape(o.spins.shape) - o.spins).max(axis=3)[0, 0, 0]
        # |H_eff| of every site: the new spin's direction is H_eff / |H_eff|, so
        # float32 rounding of the six-term sum (a few 1e-7) moves it by about
        # that over |H_eff|
        sp = pre[0, 0, 0].reshape(3, L, L, L)
        h = np.zeros_like(sp)
        for ax, npax in enumerate((3, 2, 1)):
            h += J[ax] * np.roll(sp, -1, axis=npax) + np.roll(J[ax], 1, axis=npax - 1) * np.roll(sp, 1, axis=npax)
        hn = np.linalg.norm(h, axis=0).reshape(-1)
        bound = 1e-5 + 4e-6 / np.maximum(hn, 1e-30)
        if kind == 0:
            # the heat bath's transverse frame (Frisvad) is singular at n = -z: within
            # a distance rho of it, rounding of n (about 1e-7) turns the frame by
            # about that over rho
            nz = h[2].reshape(-1) / np.maximum(hn, 1e-30)
            rho = np.sqrt(np.maximum(1.0 - nz * nz, 1e-30))
            bound += np.where(nz < 0, 1e-6 / rho, 0.0)
        worst = np.argmax(d / bound)
        print(f"L = {L}, kind {kind}, parity {parity}: max |ds| {d.max():.2e}; worst relative to the "
              f"bound {d[worst] / bound[worst]:.2f} at |H_eff| = {hn[worst]:.2e}", flush=True)
        assert d.max() < 1e-4
        assert np.all(d <= bound)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_compressed_store_rounds_to_nearest_even(hsg, oracle_lib, storage):
    """Spins written in float16 or bfloat16 (the codec's encoder, which for
    bfloat16 is gfx950's packed conversion) round every component to nearest
    with ties to even, as the oracle's codec emulation does: half of the
    components lie exactly half-way between two codes (both parities of the
    lower code, both signs), the rest anywhere in +-[1/8, 1). Read back, each
    spin is the renormalised rounded vector to float32 precision; one code step
    the wrong way would move a component by at least 5e-5 (float16) or 4e-4
    (bfloat16)."""
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 75))
    g = inputs.make_group(rng, 8, 2, 2, inputs.geometric_ladder(0.1, 0.3, 4))
    lat = hsg.Lattice([g], seed=inputs.PHILOX_KEY_BASE + 75, storage=storage)
    n = g.n_slots * 3 * g.N
    # float32 patterns in [1/8, 1) with a random sign
    bits = rng.integers(0x3E000000, 0x3F800000, size=n, dtype=np.uint64).astype(np.uint32)
    bits |= (rng.integers(0, 2, size=n, dtype=np.uint32) << 31).astype(np.uint32)
    tie = rng.integers(0, 2, size=n).astype(bool)
    if storage == "bf16":  # the 16 dropped bits exactly half a code step
        bits[tie] = (bits[tie] & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
        rnd = np.vectorize(oracle_lib.round_bf16)
    else:  # float16 keeps 10 of the 23 fraction bits (normal range here)
        bits[tie] = (bits[tie] & np.uint32(0xFFFFE000)) | np.uint32(0x1000)
        rnd = np.vectorize(oracle_lib.round_f16)
    v = bits.view(np.float32)
    lat.set_spins(torch.from_numpy(v.copy()).to(lat.device))
    got = lat.get_spins().cpu().numpy().astype(np.float64).reshape(g.n_slots, 3, g.N)
    want = rnd(v.astype(np.float64)).reshape(g.n_slots, 3, g.N)
    want = want / np.sqrt((want ** 2).sum(axis=1, keepdims=True))
    err = np.abs(got - want).max()
    print(f"{storage}: {int(tie.sum())} ties, max |got - want| {err:.2e}", flush=True)
    assert err < 1e-6
