"""Host-side checks of the heat bath's float32 routines in csrc/device.h: the
constants are read from the source, and the routines' steps are replayed in
float32 with numpy (every fused multiply-add rounded once, through float64,
where the product of two float32 numbers is exact). The device runs the same
steps; a GPU test measures the device's own results. Here the error bounds
stated in the source are checked without a GPU, over the whole 2^-24 grid of
the uniforms for sine and cosine."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "paper_1204_6192_amd", "csrc", "device.h")).read()
F32 = np.float32


def _function(name):
    m = re.search(r"__device__ __forceinline__ \w+ " + name + r"\(.*?\n}\n", SRC, re.S)
    assert m, name
    return m.group(0)


def _hexfloats(text):
    return [F32(float.fromhex(h.rstrip("f"))) * (-1 if s == "-" else 1)
            for s, h in re.findall(r"(-?)(0x[0-9a-fA-F.]+p[+-]\d+)f", text)]


def _fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(F32)


def test_sincos_polynomial_error_over_the_uniform_grid():
    """sin(2 pi u), cos(2 pi u) for every u = k 2^-24, k = 1 .. 2^24: absolute
    error at most 7e-8 (the bound the source states), sin^2 + cos^2 within 2e-7
    of 1, exact at the quarter turns."""
    body = _function("sincos_2pi")
    c = _hexfloats(body)
    assert len(c) == 8, c  # three sine and four cosine coefficients, 2 pi's stand-in
    s3, s2, s1, s0, c4, c3, c2, c1 = c  # in the order the source uses them
    k = np.arange(1, 2 ** 24 + 1, dtype=np.int64)
    u = (k * 2.0 ** -24).astype(F32)
    q = np.rint(F32(4) * u).astype(F32)
    r = _fma(q, F32(-0.25), u)
    assert np.all(r.astype(np.float64) == u.astype(np.float64) - q.astype(np.float64) / 4)  # exact
    t = (r * r).astype(F32)
    p = _fma(s3, t, s2)
    p = _fma(p, t, s1)
    sr = _fma(r, s0, (r * (t * p).astype(F32)).astype(F32))
    g = _fma(c4, t, c3)
    g = _fma(g, t, c2)
    g = _fma(g, t, c1)
    cr = _fma(g, t, F32(1.0))
    n = q.astype(np.int64)
    so, co = np.where(n & 1, cr, sr), np.where(n & 1, sr, cr)
    so = np.where(n & 2, -so, so)
    co = np.where((n + 1) & 2, -co, co)
    x = 2 * np.pi * u.astype(np.float64)
    err_s, err_c = np.abs(so - np.sin(x)).max(), np.abs(co - np.cos(x)).max()
    assert err_s <= 7e-8 and err_c <= 7e-8, (err_s, err_c)
    assert np.abs(so.astype(np.float64) ** 2 + co.astype(np.float64) ** 2 - 1).max() <= 2e-7
    quarter = (k % (1 << 22)) == 0
    assert np.all(np.abs(so[quarter]) + np.abs(co[quarter]) == 1.0)


def test_extended_precision_constants():
    """The split constants of exp_nonpos and log_normal: log2(e) = H + L and
    ln 2 = H + L, each H the float32 rounding of the constant and L the float32
    rounding of the rest."""
    for name, value in (("exp_nonpos", 1.0 / np.log(2.0)), ("log_normal", np.log(2.0))):
        h, lo = _hexfloats(_function(name))[:2]
        assert h == F32(value)
        assert lo == F32(value - float(h))
        assert abs(float(h) + float(lo) - value) < 2.0 ** -50


def test_renormalisation_has_no_drift():
    """The float32 renormalisation applied after every update (renorm_unit):
    d = |s|^2 - 1 as a chain of three fused multiply-adds, then s (1 + d (3d/8
    - 1/2)). Replayed over 200 float32 reflections of 2 * 10^4 random spins
    about random fields, the mean of |s| - 1 stays at zero within its
    statistical error (the roundings are unbiased), while plain v / sqrt(v.v)
    drifts by about 3e-8 (it cannot resolve deviations below the float32
    spacing at 1). The source is checked to hold the replayed steps."""
    body = _function("renorm_unit")
    assert "fmaf(a.x, a.x, fmaf(a.y, a.y, fmaf(a.z, a.z, -1.0f)))" in body
    assert "d * fmaf(0.375f, d, -0.5f)" in body
    rng = np.random.default_rng(12)
    n = 20000

    def chain(x, y, z):
        d = _fma(x, x, _fma(y, y, _fma(z, z, np.full_like(z, -1))))
        c = d * _fma(np.full_like(d, 0.375), d, np.full_like(d, -0.5))
        return _fma(x, c, x), _fma(y, c, y), _fma(z, c, z)

    def plain(x, y, z):
        r = F32(1) / np.sqrt(x * x + y * y + z * z)
        return x * r, y * r, z * r

    means = {}
    for name, fn in (("chain", chain), ("plain", plain)):
        v = rng.normal(size=(3, n))
        v /= np.linalg.norm(v, axis=0)
        x, y, z = (c.astype(F32) for c in v)
        for _ in range(200):
            h = rng.normal(size=(3, n)).astype(F32)
            hh = _fma(h[0], h[0], _fma(h[1], h[1], h[2] * h[2]))
            f = F32(2) * _fma(x, h[0], _fma(y, h[1], z * h[2])) * (F32(1) / hh)
            x, y, z = fn(_fma(f, h[0], -x), _fma(f, h[1], -y), _fma(f, h[2], -z))
        dev = np.sqrt(x.astype(np.float64) ** 2 + y.astype(np.float64) ** 2 + z.astype(np.float64) ** 2) - 1
        means[name] = (dev.mean(), dev.std() / np.sqrt(n))
    m, se = means["chain"]
    assert abs(m) < 5 * se + 1e-11, means
    assert means["plain"][0] > 1e-8, means
