"""Seeded synthetic inputs for the EA Heisenberg spin-glass sweep.

This module is the only code shared by the HIP path and the CPU oracle. It draws
the quenched disorder, the starting spins and the temperature ladders. It does
none of the Monte-Carlo arithmetic: every random number the method itself
consumes comes from the Philox counter map, not from here.

Recipe (the paper's instances are private; these stand in for them):

* couplings J_a(i) between site i and i + e_a, a in {x, y, z}: Gaussian N(0, 1)
  drawn in float64 and rounded to float32 (Sec. 2, the definition of the
  model), or bimodal +-1 with p = 1/2 (a precomputed alternative distribution,
  which Sec. 2 allows);
* random field H_i: either H_r * N(0, 1) per component, or a uniform direction
  on a sphere of fixed radius |H| (the paper's own choice in Sec. 2);
* starting spins: uniform on the unit sphere (cos(theta) = 2u - 1,
  phi = 2 pi u'), normalised in float64 and stored as float32;
* temperatures: geometric ladder T_k = T_1 f^k, f = (T_max / T_1)^(1/(R_T - 1))
  (Sec. 4, the discussion of the temperature set for parallel tempering).

Array layouts are the canonical ones of the C-ABI:

* ``J``      float32 [n_samples][3][L^3], site index x + L (y + L z);
* ``H``      float32 [n_samples][3][L^3] or ``None``;
* ``spins0`` float32 [n_samples][n_copies][n_temps][3][L^3].
"""

from __future__ import annotations

from dataclasses import dataclass, field as dc_field
from typing import List, Optional

import numpy as np

INSTANCE_SEED_BASE = 1204619200
PHILOX_KEY_BASE = 0x1204_6192_0000_0000


def geometric_ladder(t_min: float, t_max: float, n: int) -> np.ndarray:
    """Geometric temperature set in float64, strictly increasing."""
    if n == 1:
        return np.array([t_min], dtype=np.float64)
    f = (t_max / t_min) ** (1.0 / (n - 1))
    temps = t_min * f ** np.arange(n, dtype=np.float64)
    temps[-1] = t_max
    return temps


def uniform_sphere(rng: np.random.Generator, shape) -> np.ndarray:
    """Unit 3-vectors uniform on S^2; returns float64 [..., 3, n] for shape (..., n)."""
    u = rng.random(shape)
    v = rng.random(shape)
    c = 2.0 * u - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    phi = 2.0 * np.pi * v
    out = np.stack([st * np.cos(phi), st * np.sin(phi), c], axis=-2)
    out /= np.sqrt((out * out).sum(axis=-2, keepdims=True))
    return out


@dataclass
class Group:
    """One lattice-size group: every sample in it shares L, copies and ladder."""

    L: int
    n_samples: int
    n_copies: int
    temps: np.ndarray
    J: np.ndarray
    H: Optional[np.ndarray]
    spins0: np.ndarray
    coupling_kind: int = 0  # 0 = real-valued float32, 1 = exactly +-1
    sample_uid_base: int = 0

    @property
    def n_temps(self) -> int:
        return int(self.temps.shape[0])

    @property
    def N(self) -> int:
        return self.L ** 3

    @property
    def has_field(self) -> bool:
        return self.H is not None

    @property
    def n_slots(self) -> int:
        return self.n_samples * self.n_copies * self.n_temps


def make_group(
    rng: np.random.Generator,
    L: int,
    n_samples: int,
    n_copies: int,
    temps: np.ndarray,
    couplings: str = "gaussian",
    field: Optional[tuple] = None,
    sample_uid_base: int = 0,
) -> Group:
    """Draw one group. ``field`` is None, ("gaussian", H_r) or ("sphere", |H|)."""
    N = L ** 3
    T = len(temps)
    if couplings == "gaussian":
        J = rng.standard_normal((n_samples, 3, N)).astype(np.float32)
        kind = 0
    elif couplings == "bimodal":
        J = np.where(rng.random((n_samples, 3, N)) < 0.5, -1.0, 1.0).astype(np.float32)
        kind = 1
    elif couplings == "zero":
        J = np.zeros((n_samples, 3, N), dtype=np.float32)
        kind = 0
    else:
        raise ValueError(f"unknown coupling distribution {couplings!r}")
    H = None
    if field is not None:
        form, amp = field
        if form == "gaussian":
            H = (amp * rng.standard_normal((n_samples, 3, N))).astype(np.float32)
        elif form == "sphere":
            H = (amp * uniform_sphere(rng, (n_samples, N))).astype(np.float32)
        else:
            raise ValueError(f"unknown field form {form!r}")
    spins0 = np.empty((n_samples, n_copies, T, 3, N), dtype=np.float32)
    for d in range(n_samples):  # per sample, to bound temporaries at large L
        spins0[d] = uniform_sphere(rng, (n_copies, T, N)).astype(np.float32)
    return Group(L=L, n_samples=n_samples, n_copies=n_copies,
                 temps=np.asarray(temps, dtype=np.float64), J=J, H=H, spins0=spins0,
                 coupling_kind=kind, sample_uid_base=sample_uid_base)


@dataclass
class Instance:
    """A batch of groups plus the per-sweep mix and the Philox key."""

    groups: List[Group]
    seed: int
    n_hb: int = 1
    n_or: int = 4
    pt_every: int = 1
    storage: str = "f32"
    name: str = ""
    sweeps: int = 0
    notes: dict = dc_field(default_factory=dict)

    @property
    def n_spins(self) -> int:
        return sum(g.n_slots * g.N for g in self.groups)


# The five workloads. Sizes, ladders, disorder and storage follow the benchmark
# definitions; "sweeps" is the nominal run length of the workload.
CONFIGS = {
    "tiny": dict(groups=[dict(L=8, n_samples=1, t=(0.10, 0.30, 8))],
                 couplings="gaussian", field=None, storage="f32", sweeps=1000, k=0),
    "batched": dict(groups=[dict(L=32, n_samples=64, t=(0.10, 0.30, 32))],
                    couplings="gaussian", field=None, storage="f32", sweeps=10000, k=1),
    "field": dict(groups=[dict(L=64, n_samples=16, t=(0.05, 0.25, 24))],
                  couplings="gaussian", field=("gaussian", 0.1), storage="f16",
                  sweeps=0, k=2),
    "uneven": dict(groups=[dict(L=L, n_samples=32, t=(0.10, 0.30, 16))
                           for L in (12, 16, 24, 32, 48)],
                   couplings="gaussian", field=None, storage="bf16", sweeps=0, k=3),
    "large": dict(groups=[dict(L=128, n_samples=1, t=(0.10, 0.30, 32))],
                  couplings="bimodal", field=None, storage="qangle", sweeps=0, k=4),
    # the paper's timing workload: 256 systems of L = 32 at T = 100 (one rung)
    "table1": dict(groups=[dict(L=32, n_samples=128, t=(100.0, 100.0, 1))],
                   couplings="gaussian", field=None, storage="f32", sweeps=0, k=5),
}


def make_instance(name: str, *, scale_samples: Optional[int] = None,
                  L_override: Optional[int] = None, storage: Optional[str] = None,
                  field_amp: Optional[float] = None, seed_offset: int = 0,
                  copies: int = 2) -> Instance:
    """Build a named workload. ``scale_samples`` caps samples per group (for tests);
    ``copies`` is R_O (4 for the four-replica estimators in a field)."""
    cfg = CONFIGS[name]
    k = cfg["k"]
    rng = np.random.Generator(np.random.Philox(INSTANCE_SEED_BASE + k + seed_offset))
    groups = []
    uid = 0
    field = cfg["field"]
    if field is not None and field_amp is not None:
        field = (field[0], field_amp)
    for gd in cfg["groups"]:
        n_s = gd["n_samples"] if scale_samples is None else min(gd["n_samples"], scale_samples)
        L = gd["L"] if L_override is None else L_override
        temps = geometric_ladder(*gd["t"])
        groups.append(make_group(rng, L, n_s, copies, temps, couplings=cfg["couplings"],
                                 field=field, sample_uid_base=uid))
        uid += n_s
    return Instance(groups=groups, seed=PHILOX_KEY_BASE + k, storage=storage or cfg["storage"],
                    name=name, sweeps=cfg["sweeps"])
