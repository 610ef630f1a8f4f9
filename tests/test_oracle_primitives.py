"""Pins of the oracle's building blocks against things other than itself.

* Philox4x32-10 against rocRAND's independent implementation (host build).
* The uniform maps against their exact definitions on the integer grid.
* The Frisvad frame: orthonormality, handedness, continuity across the equator
  and accuracy next to its one singular point.
* The heat-bath draw of Eq. (2) against the von Mises-Fisher closed forms
  (Langevin function, second moments) and a KS test of the CDF.
* The over-relaxation reflection of Eq. (3): invariants.
* The energy of Eq. (1): an explicit bond list built independently here, and
  ferromagnetic / Neel ground states.
"""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def langevin(k):
    return 1.0 / np.tanh(k) - 1.0 / k


# ------------------------------------------------------------------ Philox
@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(d, "ref")
    subprocess.check_call([hipcc, "-I/opt/rocm/include", "--offload-arch=gfx950", "-x", "hip",
                           os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp"), "-o", exe])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(oracle_lib, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF,
                                  0xFFFFFFFF)]
    for _ in range(300):
        k0, k1, c0, c2, c3 = (int(v) for v in rng.integers(0, 2 ** 32, 5, dtype=np.uint64))
        c1 = int(rng.integers(0, 2 ** 30))
        cases.append((k0, k1, c0, c1, c2, c3))
    # the counter layout actually used by the heat bath and tempering
    for t in (0, 1, 999):
        cases.append((0x00000001, 0x12046192, 7, t, 3 | 1 << 8 | 1 << 16, 5))
    inp = "".join("%x %x %x %x %x %x\n" % c for c in cases)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    ref = [[int(w, 16) for w in line.split()] for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        got = oracle_lib.philox(c[2:], c[:2])
        assert [int(v) for v in got] == r, c


# ------------------------------------------------------------------ uniforms
def test_u24_grid(oracle_lib):
    assert oracle_lib.u24(0) == 2.0 ** -24
    assert oracle_lib.u24(0xFFFFFFFF) == 1.0
    assert oracle_lib.u24(0xFF) == 2.0 ** -24  # low 8 bits are dropped
    assert oracle_lib.u24(0x100) == 2.0 * 2.0 ** -24
    for x in (0x12345678, 0x80000000, 0x7FFFFFFF):
        assert oracle_lib.u24(x) == ((x >> 8) + 1) / 2.0 ** 24


def test_u53_grid(oracle_lib):
    assert oracle_lib.u53(0, 0) == 2.0 ** -53
    assert oracle_lib.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    a, b = 0x89ABCDEF, 0x01234567
    m = (a << 21) ^ (b >> 11)
    assert oracle_lib.u53(a, b) == (m + 1) / 2.0 ** 53


# ------------------------------------------------------------------ frame
def test_frame_orthonormal_right_handed(oracle_lib):
    rng = np.random.default_rng(3)
    ns = [np.array(v, dtype=float) for v in ((0, 0, 1), (0, 0, -1), (1, 0, 0), (0, 1, 0),
                                              (1, 0, -0.0), (0.6, 0.8, 0.0))]
    for eps in (1e-3, 1e-6, 1e-9):  # next to the singular point n = -z
        v = np.array([eps, -0.5 * eps, -1.0])
        ns.append(v / np.linalg.norm(v))
    v = rng.standard_normal((200, 3))
    ns += list(v / np.linalg.norm(v, axis=1, keepdims=True))
    for n in ns:
        e1, e2 = oracle_lib.frame(n)
        M = np.stack([e1, e2, n])
        assert np.abs(M @ M.T - np.eye(3)).max() < 1e-14
        assert np.abs(np.cross(e1, e2) - n).max() < 1e-14


def test_frame_continuous_away_from_south_pole(oracle_lib):
    """A small change of n moves the frame by a comparable amount everywhere
    except at n = -z, in particular across the equator n_z = 0."""
    rng = np.random.default_rng(4)
    for _ in range(2000):
        n = rng.standard_normal(3)
        if rng.random() < 0.5:
            n[2] = rng.uniform(-1e-7, 1e-7)  # straddle the equator
        n /= np.linalg.norm(n)
        if n[2] < -0.999:
            continue
        m = n + 1e-9 * rng.standard_normal(3)
        m /= np.linalg.norm(m)
        a1, a2 = oracle_lib.frame(n)
        b1, b2 = oracle_lib.frame(m)
        assert np.abs(a1 - b1).max() < 1e-6 and np.abs(a2 - b2).max() < 1e-6


# ------------------------------------------------------------------ heat bath
@pytest.mark.parametrize("kappa", [0.1, 0.5, 1.0, 2.0, 5.0, 10.0, 30.0])
def test_hb_vmf_moments(oracle_lib, kappa):
    """c = s.h/|h| has density ~exp(kappa c): E[c] = L(kappa), E[c^2] = 1 - 2L/kappa,
    E[(s.e1)^2] = E[(s.e2)^2] = L/kappa, E[s.e1] = E[s.e2] = 0."""
    rng = np.random.default_rng(int(kappa * 100))
    h = rng.standard_normal(3)
    h *= 1.7 / np.linalg.norm(h)
    beta = kappa / 1.7
    n = 200_000
    s = oracle_lib.hb_draw_many(h, beta, n)
    assert np.abs(np.linalg.norm(s, axis=1) - 1.0).max() < 1e-14
    nh = h / np.linalg.norm(h)
    e1, e2 = oracle_lib.frame(nh)
    c = s @ nh
    a1, a2 = s @ e1, s @ e2
    Lk = langevin(kappa)
    m2 = 1.0 - 2.0 * Lk / kappa
    var_c = m2 - Lk ** 2
    assert abs(c.mean() - Lk) < 5 * np.sqrt(var_c / n)
    var_c2 = (c ** 4).mean() - m2 ** 2
    assert abs((c ** 2).mean() - m2) < 5 * np.sqrt(var_c2 / n)
    t = Lk / kappa
    for a in (a1, a2):
        assert abs(a.mean()) < 5 * np.sqrt(t / n)
        assert abs((a ** 2).mean() - t) < 5 * np.sqrt(((a ** 4).mean() - t ** 2) / n)
    # the azimuth about h is uniform: E[a1 a2] = 0
    assert abs((a1 * a2).mean()) < 5 * np.sqrt(((a1 * a2) ** 2).mean() / n)


@pytest.mark.parametrize("kappa", [0.05, 3.0, 40.0])
def test_hb_cdf_ks(oracle_lib, kappa):
    from scipy import stats
    h = np.array([0.3, -0.4, 1.2])
    beta = kappa / np.linalg.norm(h)
    s = oracle_lib.hb_draw_many(h, beta, 50_000, key=(0xC0FFEE, int(kappa)))
    c = s @ (h / np.linalg.norm(h))

    def cdf(x):
        x = np.clip(x, -1.0, 1.0)
        # F(c) = (e^{kc} - e^{-k}) / (e^{k} - e^{-k}), written without overflow
        return np.exp(kappa * (x - 1.0)) * -np.expm1(-kappa * (x + 1.0)) / -np.expm1(-2.0 * kappa)

    res = stats.kstest(c, cdf)
    assert res.pvalue > 1e-4, res


def test_hb_zero_field_uniform(oracle_lib):
    s = oracle_lib.hb_draw_many([0.0, 0.0, 0.0], 3.0, 100_000)
    n = len(s)
    # uniform on S^2: E[s] = 0, E[s_mu^2] = 1/3
    assert np.abs(s.mean(axis=0)).max() < 5 * np.sqrt(1 / 3 / n)
    assert np.abs((s ** 2).mean(axis=0) - 1 / 3).max() < 5 * np.sqrt(4 / 45 / n)


def test_hb_extremes_of_u(oracle_lib):
    """u1 = 1 gives c = 1 exactly (the spin along h); the smallest u1 gives the far tail."""
    h = np.array([0.0, 0.0, 2.0])
    s = oracle_lib.hb_draw(h, 1.0, 0xFFFFFFFF, 0)
    assert np.allclose(s, [0, 0, 1], atol=1e-15)
    kappa = 2.0
    s = oracle_lib.hb_draw(h, 1.0, 0, 0)
    u = 2.0 ** -24
    c_expected = 1.0 + np.log(u + (1 - u) * np.exp(-2 * kappa)) / kappa
    assert abs(s[2] - c_expected) < 1e-12


# ------------------------------------------------------------------ over-relaxation
def test_or_invariants(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(500):
        s = rng.standard_normal(3)
        s /= np.linalg.norm(s)
        h = rng.standard_normal(3) * rng.uniform(0.01, 5)
        r = oracle_lib.or_reflect(s, h)
        assert abs(np.linalg.norm(r) - 1) < 1e-15
        assert abs(r @ h - s @ h) < 1e-13 * (1 + np.linalg.norm(h))
        # the component transverse to h flips sign
        nh = h / np.linalg.norm(h)
        assert np.allclose(r - (r @ nh) * nh, -(s - (s @ nh) * nh), atol=1e-14)
        # involution
        assert np.allclose(oracle_lib.or_reflect(r, h), s, atol=1e-14)
    s = np.array([0.6, 0.0, 0.8])
    assert np.array_equal(oracle_lib.or_reflect(s, np.zeros(3)), s)


# ------------------------------------------------------------------ energy
def _bond_list_energy(L, J, H, s):
    """Eq. (1) from an explicit list of the 3N bonds (i, j, J_ij), built here."""
    def idx(x, y, z):
        return (x % L) + L * ((y % L) + L * (z % L))
    bonds = []
    for z in range(L):
        for y in range(L):
            for x in range(L):
                i = idx(x, y, z)
                bonds.append((i, idx(x + 1, y, z), J[0, i]))
                bonds.append((i, idx(x, y + 1, z), J[1, i]))
                bonds.append((i, idx(x, y, z + 1), J[2, i]))
    assert len({(min(a, b), max(a, b), k % 3) for k, (a, b, _) in enumerate(bonds)}) == 3 * L ** 3
    e = 0.0
    for i, j, Jij in bonds:
        e -= Jij * float(s[:, i] @ s[:, j])
    if H is not None:
        e -= float((H * s).sum())
    return e


def test_energy_bond_list_L4(oracle_lib):
    rng = np.random.default_rng(5)
    L = 4
    N = L ** 3
    J = rng.standard_normal((3, N))
    H = 0.3 * rng.standard_normal((3, N))
    s = rng.standard_normal((3, N))
    s /= np.linalg.norm(s, axis=0)
    for HH in (None, H):
        ref = _bond_list_energy(L, J, HH, s)
        got = oracle_lib.energy(L, J, HH, s)
        assert abs(got - ref) < 1e-12 * N


def test_energy_ground_states(oracle_lib):
    L = 6
    N = L ** 3
    s = np.zeros((3, N))
    s[0] = 0.6
    s[2] = 0.8
    assert abs(oracle_lib.energy(L, np.ones((3, N)), None, s) + 3 * N) < 1e-12 * N
    # Neel state with antiferromagnetic bonds
    x, y, z = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="xy")
    par = ((np.arange(N) % L) + (np.arange(N) // L % L) + (np.arange(N) // L // L)) % 2
    sn = s * np.where(par == 0, 1.0, -1.0)
    assert abs(oracle_lib.energy(L, -np.ones((3, N)), None, sn) + 3 * N) < 1e-12 * N
    # a uniform field along the spins
    H = np.zeros((3, N))
    H[:] = 0.5 * s
    assert abs(oracle_lib.energy(L, np.zeros((3, N)), H, s) + 0.5 * N) < 1e-12 * N


# ------------------------------------------------------------------ storage rounding
def test_f16_bf16_rounding_against_numpy(oracle_lib):
    """numpy's float16 cast is IEEE round-to-nearest-even; bfloat16 by bit arithmetic."""
    rng = np.random.default_rng(9)
    vals = np.concatenate([rng.uniform(-1, 1, 3000), [1.0, -1.0, 2 ** -15, 2 ** -25, 0.5 + 2 ** -12,
                                                      0.5 + 3 * 2 ** -12, 1 - 2 ** -12]])
    for v in vals:
        assert oracle_lib.round_f16(v) == float(np.float16(v)), v
    f32 = rng.uniform(-1, 1, 3000).astype(np.float32)
    bits = f32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    ref = rounded.astype(np.uint32).view(np.float32)
    for v, r in zip(f32, ref):
        assert oracle_lib.round_bf16(float(v)) == float(r), v


# ------------------------------------------------------------------ quantised angle
def test_octahedral_special_points(oracle_lib):
    """+z maps to the centre, -z to a corner, the equator to the diamond's edge."""
    assert list(oracle_lib.oct_encode([0, 0, 1])) == [0, 0]
    assert list(oracle_lib.oct_encode([0, 0, -1])) == [32767, 32767]
    assert list(oracle_lib.oct_encode([1, 0, 0])) == [32767, 0]
    assert list(oracle_lib.oct_encode([0, -1, 0])) == [0, -32767]
    for v in ([0, 0, 1], [0, 0, -1], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0]):
        assert np.array_equal(oracle_lib.oct_decode(oracle_lib.oct_encode(v)), np.array(v, float))


def test_octahedral_roundtrip_error_and_idempotence(oracle_lib):
    """16-bit octahedral storage: angle error below 1e-4 everywhere on the sphere
    (cells of side 2/32767, stretched at most ~2x by the map); every stored code
    decodes to a vector that encodes back to the same code."""
    rng = np.random.default_rng(21)
    v = rng.standard_normal((20000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    err = max(np.linalg.norm(oracle_lib.oct_decode(oracle_lib.oct_encode(x)) - x) for x in v)
    assert err < 1e-4
    q = rng.integers(-32767, 32768, size=(5000, 2))
    for qq in q:
        back = oracle_lib.oct_encode(oracle_lib.oct_decode(qq))
        assert np.abs(back - qq).max() <= 1, qq


def test_octahedral_continuity_across_fold(oracle_lib):
    """Points on either side of the equator decode close to each other: the
    lower-half fold matches the upper half along the diamond's edge."""
    for phi in np.linspace(0, 2 * np.pi, 37):
        a = np.array([np.cos(phi), np.sin(phi), 1e-7])
        b = np.array([np.cos(phi), np.sin(phi), -1e-7])
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        da = oracle_lib.oct_decode(oracle_lib.oct_encode(a))
        db = oracle_lib.oct_decode(oracle_lib.oct_encode(b))
        assert np.linalg.norm(da - db) < 2e-4
