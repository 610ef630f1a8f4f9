"""Long-run statistics shared by the CPU calibration test and the GPU parity test.

Two chains on the same disorder samples (GPU and oracle, or two oracle runs
with different seeds) are compared rung by rung on their time averages of the
energy E (mean of the copies) and of the overlap q^2 of Eq. (5) after a burn-in.
The error bar comes from the scatter of the per-sample differences over the
independent disorder samples, not from time blocks: on L = 8 at T = 0.1, q^2
stays correlated over hundreds of sweeps, which blocks of 40 sweeps do not
resolve. Per rung, z = mean_d(diff) / (std_d(diff) / sqrt(D)), a Student t with
D - 1 degrees of freedom under the hypothesis that both chains sample the same
distribution; the rung-averaged z uses the per-sample mean over rungs.
"""

import os

import numpy as np

from paper_1204_6192_amd import inputs

L, SAMPLES, TEMPS, SWEEPS, BURN = 8, 16, 8, 500, 100
Z_RUNG_MAX, Z_ALL_MAX = 4.0, 3.5  # t with 15 degrees of freedom: p = 0.0012 and 0.003, two-sided


def group(ladder):
    rng = np.random.Generator(np.random.Philox(inputs.INSTANCE_SEED_BASE + 50))
    return inputs.make_group(rng, L, SAMPLES, 2, inputs.geometric_ladder(ladder[0], ladder[1], TEMPS))


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_series(oracle_lib, g, seed, temps=None):
    """E by rung (mean of the two copies) and q^2 by rung, [SWEEPS][D][T], of the
    oracle chain of every sample (one oracle per sample, run on host threads)."""
    temps = g.temps if temps is None else temps
    orcs = [oracle_lib.Oracle.from_group(
        inputs.Group(L=g.L, n_samples=1, n_copies=g.n_copies, temps=temps, J=g.J[d:d + 1], H=None,
                     spins0=g.spins0[d:d + 1], sample_uid_base=g.sample_uid_base + d), seed=seed)
        for d in range(g.n_samples)]
    D, T = g.n_samples, g.n_temps
    E, Q = np.zeros((SWEEPS, D, T)), np.zeros((SWEEPS, D, T))
    threads = host_threads()
    for t in range(SWEEPS):
        oracle_lib.sweep_parallel(orcs, 1, threads)
        for d, o in enumerate(orcs):
            sat = o.slot_at_temp[0]
            E[t, d] = 0.5 * (o.E[0, 0][sat[0]] + o.E[0, 1][sat[1]])
            Q[t, d] = o.measure_overlap()[0, :, 9]
    return E, Q


def zscores(A, B):
    """(z per rung [T], rung-averaged z) of the time averages of A and B [S][D][T]."""
    diff = A[BURN:].mean(axis=0) - B[BURN:].mean(axis=0)  # [D][T]
    D = diff.shape[0]
    z = diff.mean(axis=0) / (diff.std(axis=0, ddof=1) / np.sqrt(D))
    per_sample = diff.mean(axis=1)
    z_all = per_sample.mean() / (per_sample.std(ddof=1) / np.sqrt(D))
    return z, float(z_all)
