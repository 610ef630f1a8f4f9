"""The benchmark's accounting of algorithmic bytes and flops, against the
formulas the roofline figures use (written out here per workload)."""
import os
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _group(L, D, O, T, coupling_kind=0, field=False):
    return SimpleNamespace(L=L, N=L ** 3, n_samples=D, n_slots=D * O * T, coupling_kind=coupling_kind,
                           H=object() if field else None)


def test_batched_workload_bytes():
    """L = 32, 64 samples x 2 copies x 32 temperatures, float32: a fused pair
    reads and writes every spin once (24 B per site) and reads the 24 B of
    couplings per site once per sample; two fused over-relaxation pairs move the
    spins once and the couplings twice."""
    g = _group(32, 64, 2, 32)
    N, R, D = 32 ** 3, 4096, 64
    assert bench.fused(g)
    assert bench.algorithmic_bytes([g], "f32", 1) == R * N * 24 + D * N * 24  # 3.272 GB
    assert bench.algorithmic_bytes([g], "f32", 0) == R * N * 18 + D * N * 24  # heat bath: parity 0 not read
    assert bench.or_bytes_two_pairs([g], "f32") == R * N * 24 + 2 * D * N * 24  # 3.322 GB
    assert abs(bench.or_bytes_two_pairs([g], "f32") / 3.322e9 - 1) < 1e-3


def test_unfused_and_compressed_bytes():
    """Lattices that do not fuse pay 3 b_s per over-relaxation update and 2 b_s
    per heat-bath update; float16 halves b_s; +-1 couplings cost one byte per
    site and a field 12 B per site, per sample."""
    g = _group(64, 16, 2, 24, field=True)
    N, R, D = 64 ** 3, 768, 16
    assert not bench.fused(g)
    assert bench.algorithmic_bytes([g], "f16", 1) == R * N * 18 + D * N * (24 + 12)
    assert bench.algorithmic_bytes([g], "f16", 0) == R * N * 12 + D * N * (24 + 12)
    gb = _group(128, 1, 2, 32, coupling_kind=1)
    assert bench.algorithmic_bytes([gb], "qangle", 1) == 64 * 128 ** 3 * 12 + 128 ** 3 * 1


def test_method_bytes_per_update():
    """The method's bytes per update (one HBM pass per half-sweep: 2 b_s per
    heat-bath update, 3 b_s per over-relaxation update, couplings and field once
    per sample per half-sweep) for 1 HB + 4 OR: batched float32 33.975 B; the
    random field at float16 17.55 B; the uneven batch at bfloat16 17.55 B; the
    large system with quantised angles and one sign bit per bond 11.21 B; and
    36.375 B per over-relaxation update of the batched workload."""
    g = _group(32, 64, 2, 32)
    assert bench.method_bytes_per_update([g], "f32", 1, 4) == pytest.approx(33.6 + 24 / 64, rel=1e-12)
    assert bench.method_bytes_per_update([g], "f32", 1, 4, kind=1) == pytest.approx(36 + 24 / 64, rel=1e-12)
    f = _group(64, 16, 2, 24, field=True)
    assert bench.method_bytes_per_update([f], "f16", 1, 4) == pytest.approx(16.8 + 36 / 48, rel=1e-12)
    un = [_group(L, 32, 2, 16) for L in (12, 16, 24, 32, 48)]
    assert bench.method_bytes_per_update(un, "bf16", 1, 4) == pytest.approx(16.8 + 24 / 32, rel=1e-12)
    lg = _group(128, 1, 2, 32, coupling_kind=1)
    assert bench.method_bytes_per_update([lg], "qangle", 1, 4) == pytest.approx(11.2 + 0.75 / 64, rel=1e-12)


def test_fusion_follows_the_kernel_variant():
    """The fused-pair and two-pair accounting applies only where the chosen
    kernel variant runs those kernels."""
    g = _group(32, 64, 2, 32)
    assert bench.fused(g, 0) and bench.fused(g, 3) and bench.fused(g, 4)
    assert not bench.fused(g, 1) and not bench.fused(g, 2)
    assert not bench.fused(_group(36, 1, 2, 2), 4)
    assert bench.quad([g], 4, "f32", 4) and bench.quad([g], 0, "f32", 4) and bench.quad([g], 4, "qangle", 4)
    assert not bench.quad([g], 0, "qangle", 4) and not bench.quad([g], 3, "f32", 4)
    assert not bench.quad([g], 4, "f32", 1)
    N, R, D = 32 ** 3, 4096, 64
    assert bench.algorithmic_bytes([g], "f32", 1, variant=2) == R * N * 36 + D * N * 24


def test_flop_count_and_ridge():
    """69 FP32 flops per over-relaxation update (an FMA counting two): the local
    field 18 FMA, h.h and s.h (a product and two FMA each), 2 (s.h) times the
    reciprocal, the reflection 3 FMA and the renormalisation of float32 spins
    (|s|^2 - 1 as three FMA, the second-order correction, the rescaling: 15).
    The ridge uses the FP32 vector peak without packed instructions (78.6
    TFLOP/s: 256 CUs x 64 lanes x 2 flops x 2.4 GHz), as the library is built.
    Both over-relaxation kernels of the batched workload lie below it."""
    assert bench.OR_FLOPS_PER_UPDATE == 36 + 5 + 5 + 2 + 6 + 15 == 69
    assert bench.PEAK_FP32_TFLOPS == pytest.approx(256 * 64 * 2 * 2.4e9 / 1e12, rel=1e-3)
    ridge = bench.PEAK_FP32_TFLOPS * 1e12 / (bench.PEAK_HBM_GBS * 1e9)
    assert ridge == pytest.approx(9.825, rel=1e-3)
    g = _group(32, 64, 2, 32)
    upd = g.n_slots * g.N
    assert 2 * upd * 69 / bench.or_bytes_two_pairs([g], "f32") < ridge
    assert upd * 69 / bench.algorithmic_bytes([g], "f32", 1) < ridge


def test_counter_traffic_needs_matching_build_and_launch(tmp_path, monkeypatch):
    """Counter-derived bytes reach roofline.traffic only for the build, workload,
    spin storage and kernel they were taken with: counters of other code or of
    another launch say nothing about this one."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text(
        "# summary\n\ntraffic: build_id=abc workload=batched storage=f32 kernel=k_or_quad_stream "
        "bytes_per_launch=3383000000 fetch_kib=1 fetch_scale=2.0 write_kib=1 write_scale=1.0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    found = bench.measured_traffic("abc", "batched", "f32", "k_or_quad_stream")
    assert found == (3383000000.0, os.path.join("profiles", "k.md"))
    for args in (("abd", "batched", "f32", "k_or_quad_stream"), ("abc", "field", "f32", "k_or_quad_stream"),
                 ("abc", "batched", "f16", "k_or_quad_stream"), ("abc", "batched", "f32", "k_pair_stream")):
        assert bench.measured_traffic(*args) == (None, None), args


def test_committed_profile_traffic_line_is_parseable():
    """The committed summary of the dominant kernel carries one traffic line with
    every key the benchmark matches on."""
    import glob
    lines = []
    for fn in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(fn) as f:
            lines += [l for l in f if l.startswith("traffic:")]
    assert len(lines) >= 1
    for l in lines:
        kv = dict(t.split("=", 1) for t in l[len("traffic:"):].split() if "=" in t)
        assert {"build_id", "workload", "storage", "kernel", "bytes_per_launch"} <= set(kv)
        assert float(kv["bytes_per_launch"]) > 0
