"""Float64 CPU oracle for the EA Heisenberg spin-glass sweep -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It wraps ``hsg_oracle.c`` (plain serial C,
float64, built with ``-O2 -ffp-contract=off`` and no fast-math) through ctypes,
with the same call names as the HIP library so that the tests can drive both
identically. It shares no code with the HIP path.

Functions and what pins them (details in the tests):

* ``philox``            -- rocRAND's independent Philox4x32-10 (host build);
* ``frame``             -- orthonormality and handedness;
* ``hb_draw``           -- von Mises-Fisher moments (Langevin function), the CDF;
* ``or_reflect``        -- Eq. (3) invariants: |s'| = 1, s'.h = s.h, involution;
* ``energy``            -- explicit bond list on L = 4, ferro / Neel ground states;
* ``Oracle.sweep``      -- single spin in a field, open 1D chain, OR energy
                           conservation, infinite temperature, site-order
                           independence of a half-sweep;
* ``Oracle.sweep`` with tiles (the tile-local chain) -- equal to the full-lattice
                           chain for one whole-lattice tile (OR-only and HB-only
                           mixes), tile-order independence, a plain-Python replay
                           of the visiting order on a small lattice, and the
                           closed forms above;
* ``Oracle.measure_kmodes`` -- an FFT of the product fields, the k = 0 overlap,
                           the chirality of a conical spiral in closed form,
                           O(3) behaviour (proper rotations keep, reflections
                           flip the chiral part);
* ``Oracle.measure_pair_overlaps`` -- an FFT of the local-overlap field, the
                           trace of q^{mu nu}(k) for the pair (0, 1), the
                           expansion of the four-replica sums on small lattices;
* ``Oracle.pt_exchange``-- acceptance frequency against min(1, e^Delta);
* ``Oracle.measure_overlap`` -- q^2 = 1 for identical aligned copies, O(3)
                           invariance, trace identity.
* ``stats_record`` / ``Oracle`` run statistics -- hand-built temperature-map
                           sequences with hand-counted round trips, sums of
                           listed energies, U_L and C_L of two-valued series;
* ``Oracle.measure_chi4`` -- the four-replica double sums of Eq. (10): an FFT of
                           the local-overlap fields, identical replicas (chi_1 =
                           chi_2 = chi_3, N^2 at k = 0, 0 elsewhere),
                           independent random replicas at infinite temperature
                           (chi_1 / N averages 1/3 at every k, chi_2 and chi_3
                           average 0).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STORAGE_MODES = {"f32": 0, "f16": 1, "bf16": 2, "qangle": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (serial, float64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class Tiles(C.Structure):
    _fields_ = [("tx", C.c_int32), ("ty", C.c_int32), ("tz", C.c_int32), ("n_hit", C.c_int32)]


class Cfg(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_samples", C.c_int32), ("n_copies", C.c_int32),
                ("n_temps", C.c_int32), ("n_hb", C.c_int32), ("n_or", C.c_int32),
                ("pt_every", C.c_int32), ("sample_uid_base", C.c_uint32),
                ("seed", C.c_uint64)]


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER
        u32p, dp, i32p, i64p, u64p = (P(C.c_uint32), P(C.c_double), P(C.c_int32),
                                       P(C.c_int64), P(C.c_uint64))
        L.hsgo_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.hsgo_u24.argtypes = [C.c_uint32]
        L.hsgo_u24.restype = C.c_double
        L.hsgo_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.hsgo_u53.restype = C.c_double
        L.hsgo_frame.argtypes = [dp, dp, dp]
        L.hsgo_hb_draw.argtypes = [dp, C.c_double, C.c_uint32, C.c_uint32, dp]
        L.hsgo_or_reflect.argtypes = [dp, dp, dp]
        L.hsgo_energy.argtypes = [C.c_int, dp, dp, dp]
        L.hsgo_energy.restype = C.c_double
        L.hsgo_hb_words.argtypes = [P(Cfg), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.c_uint32, C.c_int64, u32p]
        L.hsgo_half_sweep.argtypes = [P(Cfg), dp, dp, dp, i32p, dp, C.c_int, C.c_int, C.c_int,
                                      C.c_uint32, i64p]
        L.hsgo_pt_pass.argtypes = [P(Cfg), dp, i32p, dp, C.c_uint32, C.c_uint32, u64p]
        L.hsgo_energies.argtypes = [P(Cfg), dp, dp, dp, dp]
        L.hsgo_sweep.argtypes = [P(Cfg), dp, dp, dp, i32p, dp, dp, u64p, C.c_int, u64p]
        L.hsgo_overlap.argtypes = [P(Cfg), dp, i32p, dp]
        L.hsgo_tile_sweep.argtypes = [P(Cfg), P(Tiles), dp, dp, dp, i32p, dp, dp, u64p, C.c_int,
                                      u64p, i64p]
        L.hsgo_tiles_valid.argtypes = [C.c_int, P(Tiles), C.c_int]
        L.hsgo_kmodes.argtypes = [P(Cfg), dp, i32p, dp]
        L.hsgo_pair_overlaps.argtypes = [P(Cfg), dp, i32p, dp]
        L.hsgo_set_storage_mode.argtypes = [C.c_int]
        L.hsgo_store_roundtrip.argtypes = [C.c_int, dp]
        L.hsgo_round_f16.argtypes = [C.c_double]
        L.hsgo_round_f16.restype = C.c_double
        L.hsgo_round_bf16.argtypes = [C.c_double]
        L.hsgo_round_bf16.restype = C.c_double
        L.hsgo_hb_draw_many.argtypes = [dp, C.c_double, u32p, C.c_int64, dp]
        L.hsgo_set_noise.argtypes = [C.c_double, C.c_uint64]
        L.hsgo_oct_encode.argtypes = [dp, i32p]
        L.hsgo_oct_decode.argtypes = [i32p, dp]
        L.hsgo_stats_record.argtypes = [P(Cfg), dp, i32p, dp, dp, i32p, i32p, u32p]
        L.hsgo_stats_finish.argtypes = [P(Cfg), dp, dp, dp, C.c_uint64, dp, dp]
        L.hsgo_chi4.argtypes = [P(Cfg), dp, i32p, dp]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().hsgo_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def u24(x: int) -> float:
    return lib().hsgo_u24(int(x))


def u53(a: int, b: int) -> float:
    return lib().hsgo_u53(int(a), int(b))


def frame(n):
    n = np.ascontiguousarray(n, dtype=np.float64)
    e1 = np.zeros(3)
    e2 = np.zeros(3)
    lib().hsgo_frame(_p(n, C.c_double), _p(e1, C.c_double), _p(e2, C.c_double))
    return e1, e2


def hb_draw(h, beta: float, x0: int, x1: int) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.zeros(3)
    lib().hsgo_hb_draw(_p(h, C.c_double), float(beta), int(x0), int(x1), _p(out, C.c_double))
    return out


def hb_draw_many(h, beta: float, n: int, key=(0x1234567, 0x89ABCDE)) -> np.ndarray:
    """n heat-bath draws about a fixed field, Philox blocks (q, 0, 0, 0) under key."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros((n, 3))
    lib().hsgo_hb_draw_many(_p(h, C.c_double), float(beta), _p(k, C.c_uint32), int(n),
                            _p(out, C.c_double))
    return out


def or_reflect(s, h) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.zeros(3)
    lib().hsgo_or_reflect(_p(s, C.c_double), _p(h, C.c_double), _p(out, C.c_double))
    return out


def energy(L: int, J, H, s) -> float:
    """Eq. (1) for one replica; J [3][N], H [3][N] or None, s [3][N]."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    Hp = None
    if H is not None:
        H = np.ascontiguousarray(H, dtype=np.float64)
        Hp = _p(H, C.c_double)
    return lib().hsgo_energy(int(L), _p(J, C.c_double), Hp, _p(s, C.c_double))


def round_f16(v: float) -> float:
    return lib().hsgo_round_f16(float(v))


def round_bf16(v: float) -> float:
    return lib().hsgo_round_bf16(float(v))


def oct_encode(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    q = np.zeros(2, dtype=np.int32)
    lib().hsgo_oct_encode(_p(v, C.c_double), _p(q, C.c_int32))
    return q


def oct_decode(q):
    q = np.ascontiguousarray(q, dtype=np.int32)
    v = np.zeros(3)
    lib().hsgo_oct_decode(_p(q, C.c_int32), _p(v, C.c_double))
    return v


def store_roundtrip(mode: str, s) -> np.ndarray:
    s = np.array(s, dtype=np.float64)
    lib().hsgo_store_roundtrip(STORAGE_MODES[mode], _p(s, C.c_double))
    return s


def stats_record(cfg, E, slot_at_temp, st) -> None:
    """Record one sweep's energies E [D][O][T] (by slot) and maps into the
    statistics dict st (arrays made by new_stats)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    sat = np.ascontiguousarray(slot_at_temp, dtype=np.int32)
    lib().hsgo_stats_record(C.byref(cfg), _p(E, C.c_double), _p(sat, C.c_int32),
                            _p(st["sum_e"], C.c_double), _p(st["sum_e2"], C.c_double),
                            _p(st["end"], C.c_int32), _p(st["seen_low"], C.c_int32),
                            _p(st["trips"], C.c_uint32))
    st["n"] += 1


def new_stats(n_samples, n_copies, n_temps):
    shape = (n_samples, n_copies, n_temps)
    return {"sum_e": np.zeros(shape), "sum_e2": np.zeros(shape),
            "end": np.full(shape, -1, dtype=np.int32), "seen_low": np.zeros(shape, dtype=np.int32),
            "trips": np.zeros(shape, dtype=np.uint32), "n": 0}


def stats_finish(cfg, temps, st):
    """(U_L, C_L) per ladder and rung, [D][O][T], from the recorded sums."""
    temps = np.ascontiguousarray(temps, dtype=np.float64)
    U = np.zeros_like(st["sum_e"])
    Cv = np.zeros_like(st["sum_e"])
    lib().hsgo_stats_finish(C.byref(cfg), _p(temps, C.c_double), _p(st["sum_e"], C.c_double),
                            _p(st["sum_e2"], C.c_double), int(st["n"]), _p(U, C.c_double),
                            _p(Cv, C.c_double))
    return U, Cv


def sweep_parallel(oracles, n_sweeps: int, threads: int) -> None:
    """n_sweeps of several full-lattice, float32-storage oracles without noise
    probes (each an independent chain) on `threads` host threads at once (the
    C sweeps release the interpreter lock). The storage and noise settings are
    global to the C library and stay at their defaults throughout."""
    import concurrent.futures
    for o in oracles:
        if o.tiles is not None or o.storage != "f32" or o.noise[0] != 0.0 or o.stats is not None:
            raise ValueError("sweep_parallel takes plain float32 full-lattice chains only")
    lib().hsgo_set_storage_mode(0)
    lib().hsgo_set_noise(0.0, 0)

    def run(o):
        t = np.array([o.t], dtype=np.uint64)
        Jp, Hp = o._args()
        rc = lib().hsgo_sweep(C.byref(o.cfg), Jp, Hp, _p(o.spins, C.c_double),
                              _p(o.slot_at_temp, C.c_int32), _p(o.beta, C.c_double),
                              _p(o.E, C.c_double), _p(t, C.c_uint64), int(n_sweeps),
                              _p(o.accepts, C.c_uint64))
        if rc != 0:
            raise RuntimeError("oracle sweep failed")
        o.t = int(t[0])

    with concurrent.futures.ThreadPoolExecutor(max(1, int(threads))) as ex:
        list(ex.map(run, oracles))


# ---------------------------------------------------------------- group model
class Oracle:
    """Serial float64 model of one lattice-size group; mirrors the C-ABI calls.

    ``spins`` has the canonical layout [d][o][slot][3][N] in float64;
    ``slot_at_temp`` is [d][o][k] int32; ``E`` holds the energy of each slot after
    the last sweep, [d][o][slot].
    """

    def __init__(self, L, n_samples, n_copies, temps, J, H, spins0, *, seed, n_hb=1, n_or=4,
                 pt_every=1, sample_uid_base=0, storage="f32", tiles=None, n_hit=1):
        self.cfg = Cfg(L=L, n_samples=n_samples, n_copies=n_copies, n_temps=len(temps),
                       n_hb=n_hb, n_or=n_or, pt_every=pt_every,
                       sample_uid_base=sample_uid_base, seed=seed)
        self.L = L
        self.N = L ** 3
        self.temps = np.asarray(temps, dtype=np.float64)
        self.beta = np.ascontiguousarray(1.0 / self.temps)
        self.J = np.ascontiguousarray(J, dtype=np.float64).reshape(n_samples, 3, self.N)
        self.H = None if H is None else np.ascontiguousarray(H, dtype=np.float64).reshape(
            n_samples, 3, self.N)
        self.spins = np.ascontiguousarray(spins0, dtype=np.float64).reshape(
            n_samples, n_copies, len(temps), 3, self.N).copy()
        self.storage = storage
        # tiles = (tx, ty, tz): the tile-local chain of the double checkerboard
        # decomposition; None: the full-lattice checkerboard
        self.tiles = None
        if tiles is not None:
            self.tiles = Tiles(tx=int(tiles[0]), ty=int(tiles[1]), tz=int(tiles[2]), n_hit=int(n_hit))
            if not lib().hsgo_tiles_valid(L, C.byref(self.tiles), n_hb):
                raise ValueError(f"tiles {tiles} x {n_hit} do not fit L = {L}")
        if STORAGE_MODES[storage] != 0:
            self._apply_storage_to_all()
        T = len(temps)
        self.slot_at_temp = np.ascontiguousarray(
            np.broadcast_to(np.arange(T, dtype=np.int32), (n_samples, n_copies, T))).copy()
        self.E = np.zeros((n_samples, n_copies, T), dtype=np.float64)
        self.accepts = np.zeros((n_samples, n_copies, max(T - 1, 1)), dtype=np.uint64)
        self.t = 0
        self.pt_calls = 0
        self.noise = (0.0, 0)  # sensitivity probe: (relative amplitude, stream seed)
        self.stats = None      # run statistics (enable_stats)

    @classmethod
    def from_group(cls, g, *, seed, n_hb=1, n_or=4, pt_every=1, storage="f32", tiles=None,
                   n_hit=1):
        return cls(g.L, g.n_samples, g.n_copies, g.temps, g.J, g.H, g.spins0, seed=seed,
                   n_hb=n_hb, n_or=n_or, pt_every=pt_every, sample_uid_base=g.sample_uid_base,
                   storage=storage, tiles=tiles, n_hit=n_hit)

    def _apply_storage_to_all(self):
        mode = STORAGE_MODES[self.storage]
        flat = np.moveaxis(self.spins, 3, -1).reshape(-1, 3).copy()
        for r in range(flat.shape[0]):
            row = np.ascontiguousarray(flat[r])
            lib().hsgo_store_roundtrip(mode, _p(row, C.c_double))
            flat[r] = row
        self.spins = np.ascontiguousarray(
            np.moveaxis(flat.reshape(self.spins.shape[:3] + (self.N, 3)), -1, 3))

    def _args(self):
        Hp = None if self.H is None else _p(self.H, C.c_double)
        return _p(self.J, C.c_double), Hp

    def set_noise(self, eps: float, seed: int) -> None:
        """Test-only sensitivity probe: perturb every update by relative eps."""
        self.noise = (float(eps), int(seed))

    def _noise_on(self):
        eps, seed = self.noise
        if eps > 0.0:
            # advance the stream per call so that successive calls differ
            lib().hsgo_set_noise(eps, (seed * 1_000_003 + self.t * 7919 + self.pt_calls)
                                 & 0xFFFFFFFFFFFFFFFF)

    def enable_stats(self) -> None:
        """Record run statistics (per-rung sums of E and E^2, round trips) after
        every following sweep."""
        self.stats = new_stats(self.cfg.n_samples, self.cfg.n_copies, self.cfg.n_temps)

    def get_stats(self):
        """(sums [D][O][T][2] of E and E^2 by rung, round trips [D][O][T] by slot,
        sweeps recorded, U_L [D][O][T], C_L [D][O][T])."""
        st = self.stats
        U, Cv = stats_finish(self.cfg, self.temps, st)
        return np.stack([st["sum_e"], st["sum_e2"]], axis=-1), st["trips"].copy(), st["n"], U, Cv

    def sweep(self, n_sweeps: int = 1, tile_order=None) -> None:
        """n_sweeps sweeps of the full-lattice checkerboard chain, or of the
        tile-local chain when the oracle was made with tiles (then tile_order
        optionally permutes the visits of each coarse parity's tiles). With
        statistics enabled, each sweep is recorded after its tempering pass."""
        if self.stats is not None and n_sweeps > 1:
            for _ in range(n_sweeps):
                self.sweep(1, tile_order)
            return
        lib().hsgo_set_storage_mode(STORAGE_MODES[self.storage])
        self._noise_on()
        t = np.array([self.t], dtype=np.uint64)
        Jp, Hp = self._args()
        if self.tiles is None:
            rc = lib().hsgo_sweep(C.byref(self.cfg), Jp, Hp, _p(self.spins, C.c_double),
                                  _p(self.slot_at_temp, C.c_int32), _p(self.beta, C.c_double),
                                  _p(self.E, C.c_double), _p(t, C.c_uint64), int(n_sweeps),
                                  _p(self.accepts, C.c_uint64))
        else:
            op = None
            if tile_order is not None:
                tile_order = np.ascontiguousarray(tile_order, dtype=np.int64)
                op = _p(tile_order, C.c_int64)
            rc = lib().hsgo_tile_sweep(C.byref(self.cfg), C.byref(self.tiles), Jp, Hp,
                                       _p(self.spins, C.c_double),
                                       _p(self.slot_at_temp, C.c_int32), _p(self.beta, C.c_double),
                                       _p(self.E, C.c_double), _p(t, C.c_uint64), int(n_sweeps),
                                       _p(self.accepts, C.c_uint64), op)
        lib().hsgo_set_storage_mode(0)
        lib().hsgo_set_noise(0.0, 0)
        if rc != 0:
            raise RuntimeError("oracle sweep failed: temperature map is not a permutation")
        self.t = int(t[0])
        if self.stats is not None and n_sweeps == 1:
            stats_record(self.cfg, self.E, self.slot_at_temp, self.stats)

    def half_sweep(self, kind: int, parity: int, rep: int = 0, order=None) -> None:
        lib().hsgo_set_storage_mode(STORAGE_MODES[self.storage])
        Jp, Hp = self._args()
        op = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int64)
            op = _p(order, C.c_int64)
        rc = lib().hsgo_half_sweep(C.byref(self.cfg), Jp, Hp, _p(self.spins, C.c_double),
                                   _p(self.slot_at_temp, C.c_int32), _p(self.beta, C.c_double),
                                   int(kind), int(rep), int(parity), self.t & 0xFFFFFFFF, op)
        lib().hsgo_set_storage_mode(0)
        if rc != 0:
            raise RuntimeError("oracle half-sweep failed")

    def compute_energies(self) -> np.ndarray:
        Jp, Hp = self._args()
        E = np.zeros_like(self.E)
        lib().hsgo_energies(C.byref(self.cfg), Jp, Hp, _p(self.spins, C.c_double),
                            _p(E, C.c_double))
        return E

    def measure_energy(self) -> np.ndarray:
        return self.compute_energies()

    def pt_exchange(self, energies=None) -> None:
        """Standalone tempering pass (purpose 2, counter = number of standalone calls)."""
        E = np.ascontiguousarray(self.E if energies is None else energies, dtype=np.float64)
        lib().hsgo_pt_pass(C.byref(self.cfg), _p(E, C.c_double),
                           _p(self.slot_at_temp, C.c_int32), _p(self.beta, C.c_double),
                           self.pt_calls & 0xFFFFFFFF, 2, _p(self.accepts, C.c_uint64))
        self.pt_calls += 1

    def measure_overlap(self) -> np.ndarray:
        q = np.zeros((self.cfg.n_samples, self.cfg.n_temps, 10), dtype=np.float64)
        lib().hsgo_overlap(C.byref(self.cfg), _p(self.spins, C.c_double),
                           _p(self.slot_at_temp, C.c_int32), _p(q, C.c_double))
        return q

    def measure_kmodes(self) -> np.ndarray:
        """[n_samples][n_temps][84]: q^{mu nu}(k) and the chiral overlaps
        q_c^alpha(k) between copies 0 and 1 at each rung, for k = 0 and the three
        smallest wave vectors (layout in hsg_oracle.c)."""
        q = np.zeros((self.cfg.n_samples, self.cfg.n_temps, 84), dtype=np.float64)
        lib().hsgo_kmodes(C.byref(self.cfg), _p(self.spins, C.c_double),
                          _p(self.slot_at_temp, C.c_int32), _p(q, C.c_double))
        return q

    def measure_pair_overlaps(self) -> np.ndarray:
        """[n_samples][n_temps][P][7], P = O (O - 1) / 2 copy pairs: the local-overlap
        Fourier sums A_ab(k) behind the four-replica estimators (layout in
        hsg_oracle.c)."""
        O = self.cfg.n_copies
        q = np.zeros((self.cfg.n_samples, self.cfg.n_temps, O * (O - 1) // 2, 7), dtype=np.float64)
        lib().hsgo_pair_overlaps(C.byref(self.cfg), _p(self.spins, C.c_double),
                                 _p(self.slot_at_temp, C.c_int32), _p(q, C.c_double))
        return q

    def measure_chi4(self) -> np.ndarray:
        """[n_samples][n_temps][4][5]: the four-replica double sums chi_1, chi_2,
        chi_3 of Eq. (10) (copies 0..3 at each rung) for k = 0, k_x, k_y, k_z:
        Re chi_1, Re chi_2, Im chi_2, Re chi_3, Im chi_3. O(N^2): small L only."""
        if self.cfg.n_copies < 4:
            raise ValueError("the four-replica estimators need n_copies >= 4")
        out = np.zeros((self.cfg.n_samples, self.cfg.n_temps, 4, 5), dtype=np.float64)
        lib().hsgo_chi4(C.byref(self.cfg), _p(self.spins, C.c_double),
                        _p(self.slot_at_temp, C.c_int32), _p(out, C.c_double))
        return out

    def hb_words(self, d, o, slot, rep, parity, i):
        w = np.zeros(2, dtype=np.uint32)
        lib().hsgo_hb_words(C.byref(self.cfg), d, o, slot, rep, parity, self.t & 0xFFFFFFFF,
                            int(i), _p(w, C.c_uint32))
        return w
