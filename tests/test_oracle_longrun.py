"""Calibration and power of the long-run statistics comparison (CPU only).

The GPU parity test of long runs compares per-rung time averages of E and q^2
with the oracle's, with error bars from the scatter over disorder samples
(tests/longrun.py). Here the same estimator, on the same workload (L = 8, 16
samples, 2 x 8 temperatures geometric in [0.10, 0.30], 500 sweeps), compares
oracle chains that differ only in their seed: the z-scores must look like unit
Student-t variables (rms near 1, none beyond the GPU test's bounds). And a
chain at temperatures 1 % higher must be told apart, so the comparison can see
a plausible mistake such as a wrong inverse temperature.
"""

import numpy as np
import pytest

import longrun

pytestmark = pytest.mark.slow

LADDER = (0.10, 0.30)
SEED = 0x5EED_0000


@pytest.fixture(scope="module")
def runs(oracle_lib):
    g = longrun.group(LADDER)
    return g, [longrun.oracle_series(oracle_lib, g, SEED + k) for k in range(4)]


def test_long_run_estimator_calibrated(runs):
    _, r = runs
    zs = {"E": [], "q2": []}
    for a, b in ((0, 1), (2, 3)):
        for name, i in (("E", 0), ("q2", 1)):
            z, z_all = longrun.zscores(r[a][i], r[b][i])
            print(f"seeds {a} vs {b} {name}: z {np.round(z, 2)} all {z_all:.2f}", flush=True)
            assert np.all(np.abs(z) < longrun.Z_RUNG_MAX) and abs(z_all) < longrun.Z_ALL_MAX
            zs[name] += list(z)
    for name, z in zs.items():
        rms = float(np.sqrt(np.mean(np.square(z))))
        print(f"{name}: rms z over {len(z)} rungs {rms:.2f}", flush=True)
        assert 0.6 < rms < 1.4, (name, rms)


def test_long_run_estimator_sees_a_temperature_error(oracle_lib, runs):
    g, r = runs
    E_hot, _ = longrun.oracle_series(oracle_lib, g, SEED + 9, temps=g.temps * 1.01)
    z, z_all = longrun.zscores(E_hot, r[0][0])
    print(f"ladder 1 % hotter: E z {np.round(z, 2)} all {z_all:.2f}", flush=True)
    assert z_all > 2 * longrun.Z_ALL_MAX
