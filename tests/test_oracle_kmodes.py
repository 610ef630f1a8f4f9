"""Pins of the oracle's wave-vector dependent overlap q^{mu nu}(k) and chiral
overlap q_c^alpha(k) (the analysis quantities of the paper's model section).
CPU only."""

import numpy as np
import pytest


def _rand_spins(rng, L, T=2):
    v = rng.standard_normal((1, 2, T, 3, L ** 3))
    return v / np.linalg.norm(v, axis=3, keepdims=True)


def _oracle(oracle_lib, L, spins, T=2):
    N = L ** 3
    return oracle_lib.Oracle(L, 1, 2, np.geomspace(0.2, 0.4, T), np.zeros((1, 3, N)), None, spins,
                             seed=1, n_hb=1, n_or=1, pt_every=0)


def test_spin_modes_are_the_fourier_transform(oracle_lib):
    """q^{mu nu}(k) for k = 0 and 2 pi / L along x, y, z against numpy's FFT of
    the product field (numpy's forward transform carries exp(-i k.R); the
    paper's overlap exp(+i k.R), so q = conj(FFT) / N for a real field)."""
    L = 6
    rng = np.random.default_rng(1)
    spins = _rand_spins(rng, L)
    o = _oracle(oracle_lib, L, spins)
    q = o.measure_kmodes()
    for k in range(2):
        a, b = spins[0, 0, k], spins[0, 1, k]
        for mu in range(3):
            for nu in range(3):
                F = np.fft.fftn((a[mu] * b[nu]).reshape(L, L, L)) / L ** 3  # axes z, y, x
                assert abs(q[0, k, 3 * mu + nu] - F[0, 0, 0].real) < 1e-14
                for ax, idx in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
                    m = 9 + 18 * ax + 2 * (3 * mu + nu)
                    want = np.conj(F[idx])
                    assert abs(q[0, k, m] - want.real) < 1e-13
                    assert abs(q[0, k, m + 1] - want.imag) < 1e-13


def test_k0_spin_modes_are_the_overlap(oracle_lib):
    L = 4
    rng = np.random.default_rng(2)
    o = _oracle(oracle_lib, L, _rand_spins(rng, L, T=3), T=3)
    o.slot_at_temp[0, 0] = [2, 0, 1]
    o.slot_at_temp[0, 1] = [1, 2, 0]
    q = o.measure_kmodes()
    q0 = o.measure_overlap()
    assert np.allclose(q[0, :, :9], q0[0, :, :9], rtol=0, atol=1e-14)


def _spiral(L, phi, m, axis=0):
    """Conical spiral: cone angle phi about z, turning by theta = 2 pi m / L per
    step along `axis`."""
    N = L ** 3
    idx = np.arange(N)
    R = [idx % L, (idx // L) % L, idx // (L * L)][axis]
    t = 2 * np.pi * m / L * R
    return np.stack([np.sin(phi) * np.cos(t), np.sin(phi) * np.sin(t), np.full(N, np.cos(phi))])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_chirality_of_a_conical_spiral(oracle_lib, axis):
    """kappa = s(t + theta) . (s(t) x s(t - theta)) = -2 sin^2(phi) cos(phi)
    sin(theta) (1 - cos(theta)) along the spiral's axis (worked out by hand),
    0 along the other two (repeated spins); uniform, so no k != 0 weight."""
    L, m = 8, 1
    theta = 2 * np.pi * m / L
    phis = (0.7, 1.1)
    kap = [-2 * np.sin(p) ** 2 * np.cos(p) * np.sin(theta) * (1 - np.cos(theta)) for p in phis]
    spins = np.zeros((1, 2, 1, 3, L ** 3))
    spins[0, 0, 0] = _spiral(L, phis[0], m, axis)
    spins[0, 1, 0] = _spiral(L, phis[1], m, axis)
    q = _oracle(oracle_lib, L, spins, T=1).measure_kmodes()[0, 0]
    for al in range(3):
        base = 63 + 7 * al
        want = kap[0] * kap[1] if al == axis else 0.0
        assert abs(q[base] - want) < 1e-13, (al, q[base], want)
        assert np.all(np.abs(q[base + 1:base + 7]) < 1e-13)


def _rotation(rng, proper):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if (np.linalg.det(Q) > 0) != proper:
        Q[:, 0] = -Q[:, 0]
    return Q


def test_rotations_and_reflections_of_a_copy(oracle_lib):
    """A global O(3) transformation of copy 2 leaves sum_{mu nu} |q^{mu nu}(k)|^2
    unchanged at every k; the chiral overlap (a product of pseudoscalars) is
    unchanged by a proper rotation and flips sign under an improper one."""
    L = 6
    rng = np.random.default_rng(4)
    spins = _rand_spins(rng, L, T=1)
    q = _oracle(oracle_lib, L, spins, T=1).measure_kmodes()[0, 0]

    def q2(v):
        out = [np.sum(v[:9] ** 2)]
        for ax in range(3):
            z = v[9 + 18 * ax:27 + 18 * ax]
            out.append(np.sum(z ** 2))
        return np.array(out)

    for proper, sign in ((True, 1.0), (False, -1.0)):
        Rm = _rotation(rng, proper)
        s2 = spins.copy()
        s2[0, 1, 0] = Rm @ spins[0, 1, 0]
        qr = _oracle(oracle_lib, L, s2, T=1).measure_kmodes()[0, 0]
        assert np.allclose(q2(qr), q2(q), rtol=1e-12, atol=1e-15)
        assert np.allclose(qr[63:], sign * q[63:], rtol=1e-10, atol=1e-14)
        assert np.max(np.abs(q[63:])) > 1e-4  # the test has something to flip


def test_chiral_modes_are_the_fourier_transform(oracle_lib):
    """q_c^alpha(k) against numpy's FFT of kappa(1) kappa(2), with kappa taken
    from rolled arrays (and pinned in closed form above)."""
    L = 6
    rng = np.random.default_rng(5)
    spins = _rand_spins(rng, L, T=1)
    q = _oracle(oracle_lib, L, spins, T=1).measure_kmodes()[0, 0]
    grids = [spins[0, c, 0].reshape(3, L, L, L) for c in range(2)]  # [mu][z][y][x]
    for al, npax in enumerate((3, 2, 1)):  # x, y, z are array axes 3, 2, 1
        kap = []
        for g in grids:
            up = np.roll(g, -1, axis=npax)
            dn = np.roll(g, 1, axis=npax)
            kap.append(np.einsum("mzyx,mzyx->zyx", up, np.cross(g, dn, axis=0)))
        F = np.fft.fftn(kap[0] * kap[1]) / L ** 3
        base = 63 + 7 * al
        assert abs(q[base] - F[0, 0, 0].real) < 1e-14
        for ax, idx in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
            want = np.conj(F[idx])
            assert abs(q[base + 1 + 2 * ax] - want.real) < 1e-13
            assert abs(q[base + 2 + 2 * ax] - want.imag) < 1e-13


def _oracle4(oracle_lib, L, spins, T=1):
    N = L ** 3
    return oracle_lib.Oracle(L, 1, 4, np.geomspace(0.2, 0.4, T), np.zeros((1, 3, N)), None, spins,
                             seed=1, n_hb=1, n_or=1, pt_every=0)


def test_pair_overlaps_are_the_fourier_transform_and_the_trace(oracle_lib):
    """A_ab(k) against numpy's FFT of the local-overlap field s_i(a) . s_i(b), and
    A_01(k) against the trace of q^{mu nu}(k) for the same two copies."""
    L = 6
    rng = np.random.default_rng(7)
    v = rng.standard_normal((1, 4, 1, 3, L ** 3))
    spins = v / np.linalg.norm(v, axis=3, keepdims=True)
    o = _oracle4(oracle_lib, L, spins)
    A = o.measure_pair_overlaps()[0, 0]
    pairs = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    assert A.shape == (6, 7)
    for p, (a, b) in enumerate(pairs):
        f = np.einsum("mi,mi->i", spins[0, a, 0], spins[0, b, 0]).reshape(L, L, L)
        F = np.fft.fftn(f) / L ** 3
        assert abs(A[p, 0] - F[0, 0, 0].real) < 1e-14
        for ax, idx in enumerate(((0, 0, 1), (0, 1, 0), (1, 0, 0))):
            assert abs(A[p, 1 + 2 * ax] - F[idx].real) < 1e-13
            assert abs(A[p, 2 + 2 * ax] + F[idx].imag) < 1e-13  # exp(+ikR): conjugate
    two = oracle_lib.Oracle(L, 1, 2, [0.3], np.zeros((1, 3, L ** 3)), None, spins[:, :2].copy(), seed=1,
                            n_hb=1, n_or=1, pt_every=0)
    q = two.measure_kmodes()[0, 0]
    assert abs(A[0, 0] - (q[0] + q[4] + q[8])) < 1e-14
    for ax in range(3):
        for part in range(2):
            tr = sum(q[9 + 18 * ax + 2 * (3 * m + m) + part] for m in range(3))
            assert abs(A[0, 1 + 2 * ax + part] - tr) < 1e-14


def test_four_replica_sums_expand_into_pair_overlaps(oracle_lib):
    """The four-replica sums chi_1, chi_2, chi_3 of Eq. (9), evaluated by brute
    force over i, j, mu, nu on L = 2 and 4, equal N^2 A_12 conj(A_12),
    N^2 A_13 conj(A_14) and N^2 A_13 conj(A_24) (copies numbered from 1)."""
    rng = np.random.default_rng(8)
    for L in (2, 4):
        N = L ** 3
        v = rng.standard_normal((1, 4, 1, 3, N))
        spins = v / np.linalg.norm(v, axis=3, keepdims=True)
        A = _oracle4(oracle_lib, L, spins).measure_pair_overlaps()[0, 0]
        pid = {(a, b): p for p, (a, b) in enumerate((a, b) for a in range(4) for b in range(a + 1, 4))}

        def cA(a, b, ax):  # complex A_ab(k_ax), ax = -1 for k = 0
            r = A[pid[(a, b)]]
            return complex(r[0], 0.0) if ax < 0 else complex(r[1 + 2 * ax], r[2 + 2 * ax])

        s = [spins[0, c, 0] for c in range(4)]  # [mu][i]
        idx = np.arange(N)
        R = np.stack([idx % L, (idx // L) % L, idx // (L * L)])
        for ax in (-1, 0, 1, 2):
            ph = np.ones(N, dtype=complex) if ax < 0 else np.exp(1j * 2 * np.pi * R[ax] / L)

            E = ph[:, None] * np.conj(ph)[None, :]  # e^{ik(R_i - R_j)}

            def brute(c1, c2, c3, c4):
                """sum over i, j, mu, nu of s_i^mu(c1) s_j^nu(c2) s_i^mu(c3) s_j^nu(c4) e^{ik(R_i-R_j)},
                term by term as written."""
                tot = 0j
                for mu in range(3):
                    for nu in range(3):
                        t = (s[c1][mu][:, None] * s[c2][nu][None, :] * s[c3][mu][:, None]
                             * s[c4][nu][None, :])
                        tot += np.sum(t * E)
                return tot

            chi1, chi2, chi3 = brute(0, 0, 1, 1), brute(0, 0, 2, 3), brute(0, 1, 2, 3)
            a12, a13, a14, a24 = cA(0, 1, ax), cA(0, 2, ax), cA(0, 3, ax), cA(1, 3, ax)
            assert abs(chi1 - N ** 2 * a12 * np.conj(a12)) < 1e-9 * N ** 2
            assert abs(chi2 - N ** 2 * a13 * np.conj(a14)) < 1e-9 * N ** 2
            assert abs(chi3 - N ** 2 * a13 * np.conj(a24)) < 1e-9 * N ** 2
