"""Pins of the oracle's tile-local chain (the double checkerboard decomposition of
the paper's implementation section: tiles of one coarse parity visited with their
halo frozen, n_or over-relaxation rounds then n_hb heat-bath rounds per visit,
n_hit times). CPU only."""

import numpy as np
import pytest



def _spins(rng, D, O, T, N):
    v = rng.standard_normal((D, O, T, 3, N))
    return v / np.linalg.norm(v, axis=3, keepdims=True)


def _pair(oracle_lib, L, n_hb, n_or, tiles, n_hit=1, T=3, field=0.3, seed=11):
    rng = np.random.default_rng(seed)
    N = L ** 3
    J = rng.standard_normal((1, 3, N))
    H = field * rng.standard_normal((1, 3, N)) if field else None
    s0 = _spins(rng, 1, 2, T, N)
    temps = np.geomspace(0.2, 1.0, T)
    kw = dict(seed=1234 + seed, n_hb=n_hb, n_or=n_or, pt_every=1)
    a = oracle_lib.Oracle(L, 1, 2, temps, J, H, s0, tiles=tiles, n_hit=n_hit, **kw)
    b = oracle_lib.Oracle(L, 1, 2, temps, J, H, s0, **kw)
    return a, b


@pytest.mark.parametrize("n_hb,n_or", [(0, 3), (2, 0)])
def test_whole_lattice_tile_is_the_full_lattice_chain(oracle_lib, n_hb, n_or):
    """One tile covering the lattice is visited once per sweep; with a single kind
    of update its rounds are exactly the full-lattice half-sweep pairs, drawing
    the same random numbers: the two chains agree bit for bit."""
    L = 6
    a, b = _pair(oracle_lib, L, n_hb, n_or, (L, L, L))
    a.sweep(3)
    b.sweep(3)
    assert np.array_equal(a.spins, b.spins)
    assert np.array_equal(a.E, b.E)
    assert np.array_equal(a.slot_at_temp, b.slot_at_temp)


def test_small_tiles_differ_from_the_full_lattice_chain(oracle_lib):
    """With several tiles the visiting order changes which neighbour values each
    update sees: a different (equally valid) chain."""
    a, b = _pair(oracle_lib, 8, 1, 2, (8, 4, 4))
    a.sweep(1)
    b.sweep(1)
    assert not np.allclose(a.spins, b.spins)


@pytest.mark.parametrize("tiles", [(4, 4, 4), (8, 2, 4), (2, 8, 2)])
def test_tile_order_does_not_matter(oracle_lib, tiles):
    """Tiles of one coarse parity never share a face and their halos are frozen,
    so any visiting order gives the same bits."""
    L = 8
    a, _ = _pair(oracle_lib, L, 1, 2, tiles, n_hit=2)
    c, _ = _pair(oracle_lib, L, 1, 2, tiles, n_hit=2)
    n_tiles = (L // tiles[0]) * (L // tiles[1]) * (L // tiles[2])
    order = np.random.default_rng(3).permutation(n_tiles // 2)
    a.sweep(2)
    c.sweep(1, tile_order=order)
    c.sweep(1, tile_order=order[::-1].copy())
    assert np.array_equal(a.spins, c.spins)
    assert np.array_equal(a.slot_at_temp, c.slot_at_temp)


def test_rejects_tiles_that_break_the_coarse_checkerboard(oracle_lib):
    for tiles in ((8, 8, 3), (8, 8, 5), (8, 8, 16)):  # not dividing L, 3 tiles (odd), > L
        with pytest.raises(ValueError):
            _pair(oracle_lib, 12 if tiles[2] == 3 else 8, 1, 2, tiles)
    with pytest.raises(ValueError):  # 3 repetitions x 6 heat-bath rounds > 16 counter slots
        _pair(oracle_lib, 8, 6, 1, (8, 4, 4), n_hit=3)


def test_visiting_order_replayed_in_python(oracle_lib):
    """A plain-Python replay of one sweep of the tile chain on L = 4 with tiles of
    4 x 2 x 2 (four tiles, two per coarse parity), two repetitions of (two OR
    rounds, one HB round), built from the pinned single-site primitives: same
    bits as the oracle."""
    L, N = 4, 64
    a, _ = _pair(oracle_lib, L, 1, 2, (4, 2, 2), n_hit=2, T=2, seed=5)
    s = a.spins.copy()
    J, H = a.J[0], a.H[0]

    def site(x, y, z):
        return (x % L) + L * ((y % L) + L * (z % L))

    def field(sp, x, y, z):
        i = site(x, y, z)
        up = [site(x + 1, y, z), site(x, y + 1, z), site(x, y, z + 1)]
        dn = [site(x - 1, y, z), site(x, y - 1, z), site(x, y, z - 1)]
        h = [0.0, 0.0, 0.0]
        for ax in range(3):
            jf, jb = J[ax, i], J[ax, dn[ax]]
            for m in range(3):
                h[m] += jf * sp[m, up[ax]] + jb * sp[m, dn[ax]]
        for m in range(3):
            h[m] += H[m, i]
        return np.array(h)

    for cp in (0, 1):
        for Z in range(2):
            for Y in range(2):
                if (Y + Z) % 2 != cp:
                    continue
                for o in range(2):
                    for sl in range(2):
                        k = list(a.slot_at_temp[0, o]).index(sl)
                        beta = a.beta[k]
                        sp = s[0, o, sl]
                        for r in range(2):
                            for kind, reps in (("or", [0, 0]), ("hb", [r])):
                                for rep in reps:
                                    for p in (0, 1):
                                        for z in range(2 * Z, 2 * Z + 2):
                                            for y in range(2 * Y, 2 * Y + 2):
                                                for x in range(L):
                                                    if (x + y + z) % 2 != p:
                                                        continue
                                                    i = site(x, y, z)
                                                    h = field(sp, x, y, z)
                                                    if kind == "or":
                                                        new = oracle_lib.or_reflect(sp[:, i].copy(), h)
                                                    else:
                                                        w = a.hb_words(0, o, sl, rep, p, i)
                                                        new = oracle_lib.hb_draw(h, beta, w[0], w[1])
                                                    sp[:, i] = new
    a.sweep(1)
    assert np.array_equal(a.spins, s)


@pytest.mark.parametrize("beta", [1.0, 2.0])
def test_open_chain_bond_energy_tile_chain(oracle_lib, beta):
    """The open 1D chain closed form (mean bond energy -L(beta J)) under the tile
    chain with tiles cutting the chains (x tiled) and the rows (y, z tiled)."""
    L = 16
    N = L ** 3
    x = np.arange(N) % L
    J = np.zeros((1, 3, N))
    J[0, 0] = np.where(x == L - 1, 0.0, 1.0)
    n_bonds = L * L * (L - 1)
    rng = np.random.default_rng(8)
    o = oracle_lib.Oracle(L, 1, 1, [1.0 / beta], J, None, _spins(rng, 1, 1, 1, N),
                          seed=99 + int(beta), n_hb=1, n_or=1, pt_every=0, tiles=(4, 8, 4),
                          n_hit=2)
    o.sweep(20)
    M = 160
    es = np.empty(M)
    for m in range(M):
        o.sweep(1)
        es[m] = o.E[0, 0, 0]
    e_bond = es / n_bonds
    blocks = e_bond.reshape(16, -1).mean(axis=1)
    err = blocks.std(ddof=1) / np.sqrt(len(blocks))
    expect = -(1.0 / np.tanh(beta) - 1.0 / beta)
    assert abs(e_bond.mean() - expect) < 5 * err + 1e-4, (e_bond.mean(), expect)
