"""Thin ctypes binding of libhsg.so (see include/hsg.h for the contract).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
the library. PyTorch supplies device memory and the stream. Importing this
module fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
import re
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsg.so")
HEADER_PATH = os.path.join(_HERE, "..", "include", "hsg.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (or paper_1204_6192_amd/build.py); there is no fallback path")

OK, E_INVALID, E_SIZE, E_UNSUPPORTED, E_DEVICE, E_STATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f32": 0, "f16": 1, "bf16": 2, "qangle": 3}


class HSGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hsg status {status}: {msg}")
        self.status = status


class GroupDesc(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_samples", C.c_int32), ("n_copies", C.c_int32),
                ("n_temps", C.c_int32), ("temps", C.POINTER(C.c_double)),
                ("sample_uid_base", C.c_uint32), ("has_field", C.c_int32),
                ("coupling_kind", C.c_int32), ("reserved", C.c_int32)]


class Desc(C.Structure):
    _fields_ = [("groups", C.POINTER(GroupDesc)), ("n_groups", C.c_int32), ("storage", C.c_int32),
                ("n_hb", C.c_int32), ("n_or", C.c_int32), ("pt_every", C.c_int32),
                ("reserved", C.c_int32), ("seed", C.c_uint64)]


class Sizes(C.Structure):
    _fields_ = [("state_bytes", C.c_uint64), ("coupling_bytes", C.c_uint64),
                ("field_bytes", C.c_uint64), ("scratch_bytes", C.c_uint64),
                ("n_replicas", C.c_uint64), ("n_spins", C.c_uint64)]


# The process must hold one HIP runtime. libhsg.so needs libamdhip64.so.7; torch
# (used for device memory and streams) brings its own copy with that soname, so
# importing torch first makes the loader bind libhsg.so to torch's runtime.
import torch  # noqa: E402,F401  (must precede the CDLL below)

lib = C.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({line.split()[-1] for line in f if "libamdhip64" in line})
    except OSError:
        return []


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process (%s); import torch before "
                      "anything else loads libamdhip64" % ", ".join(_hip_runtimes()))
_vp, _i32, _i64, _u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
_SIG = {
    "hsg_query_sizes": [C.POINTER(Desc), C.POINTER(Sizes)],
    "hsg_init_lattice": [C.POINTER(Desc), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)],
    "hsg_sweep": [_vp, _i32, _vp],
    "hsg_half_sweep": [_vp, _i32, _i32, _i32, _vp],
    "hsg_pair_sweep": [_vp, _i32, _i32, _vp],
    "hsg_or_pairs": [_vp, _i32, _vp],
    "hsg_pt_exchange": [_vp, _vp],
    "hsg_measure_energy": [_vp, _vp, _vp],
    "hsg_measure_energy_static": [_vp, _vp, _vp],
    "hsg_get_energies": [_vp, _vp, _vp],
    "hsg_measure_overlap": [_vp, _vp, _vp],
    "hsg_get_spins": [_vp, _vp, _vp],
    "hsg_set_spins": [_vp, _vp, _vp],
    "hsg_get_temp_map": [_vp, _vp, _vp],
    "hsg_set_temp_map": [_vp, _vp, _vp],
    "hsg_get_pt_accepts": [_vp, _vp, _vp],
    "hsg_get_state": [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64)],
    "hsg_set_state": [_vp, _u64, _u64, _vp],
    "hsg_set_tuning": [_vp, _i32],
    "hsg_set_kernel": [_vp, _i32],
    "hsg_set_overlap": [_vp, _i32],
    "hsg_get_tuning": [_vp, _vp, _vp, _vp],
    "hsg_autotune": [_vp, _i32, _vp, _vp, _vp, _vp],
    "hsg_measure_pair_overlaps": [_vp, _vp, _vp],
    "hsg_measure_kmodes": [_vp, _vp, _vp],
    "hsg_measure_chi": [_vp, _vp, _vp],
    "hsg_set_series": [_vp, _vp, _i64, _vp],
    "hsg_get_series_count": [_vp, _vp],
    "hsg_set_batch": [_vp, _i64],
    "hsg_set_stats": [_vp, _i32],
    "hsg_reset_stats": [_vp, _vp],
    "hsg_get_stats": [_vp, _vp, _vp, _vp, _vp],
    "hsg_set_chain": [_vp, _i32, _i32, _i32, _i32, _i32],
    "hsg_set_math": [_vp, _i32],
    "hsg_set_geometry": [_vp, _i32, _i32, _i32],
    "hsg_get_geometry": [_vp, _i32, _vp, _vp],
    "hsg_set_graphs": [_vp, _i32],
    "hsg_sync": [_vp, _vp],
    "hsg_debug_philox": [_vp, _vp, _vp, _i64, _vp],
    "hsg_debug_hw_math": [_vp, _vp, _i64, _vp],
}
for _name, _args in _SIG.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int32
lib.hsg_destroy.argtypes = [_vp]
lib.hsg_destroy.restype = None
lib.hsg_last_error.argtypes = []
lib.hsg_last_error.restype = C.c_char_p
lib.hsg_build_id.argtypes = []
lib.hsg_build_id.restype = C.c_char_p


def build_id() -> str:
    return lib.hsg_build_id().decode()


def declared_symbols() -> List[str]:
    """Names of the functions declared in include/hsg.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsg_[a-z_0-9]+)\s*\(", text)))


def check(status: int) -> None:
    if status != OK:
        raise HSGError(status, lib.hsg_last_error().decode())


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t) -> int:
    return t.data_ptr()


def make_desc(groups, storage: str, n_hb: int, n_or: int, pt_every: int, seed: int):
    """Build the ctypes description; returns (desc, keep-alive list)."""
    keep = []
    arr = (GroupDesc * len(groups))()
    for k, g in enumerate(groups):
        temps = np.ascontiguousarray(g.temps, dtype=np.float64)
        keep.append(temps)
        arr[k] = GroupDesc(L=g.L, n_samples=g.n_samples, n_copies=g.n_copies, n_temps=len(temps),
                           temps=temps.ctypes.data_as(C.POINTER(C.c_double)),
                           sample_uid_base=g.sample_uid_base, has_field=int(g.H is not None),
                           coupling_kind=g.coupling_kind, reserved=0)
    keep.append(arr)
    d = Desc(groups=arr, n_groups=len(groups), storage=STORAGE[storage], n_hb=n_hb, n_or=n_or,
             pt_every=pt_every, reserved=0, seed=seed & 0xFFFFFFFFFFFFFFFF)
    return d, keep


def query_sizes(desc: Desc) -> Sizes:
    out = Sizes()
    check(lib.hsg_query_sizes(C.byref(desc), C.byref(out)))
    return out


class Lattice:
    """One handle of the library plus the caller-owned device buffers (torch)."""

    def __init__(self, groups: Sequence, *, storage: str = "f32", n_hb: int = 1, n_or: int = 4,
                 pt_every: int = 1, seed: int = 0, device: str = "cuda", stream=None):
        import torch
        self.torch = torch
        self.groups = list(groups)
        self.device = torch.device(device)
        self.desc, self._keep = make_desc(self.groups, storage, n_hb, n_or, pt_every, seed)
        self.sizes = query_sizes(self.desc)
        self.n_replicas = int(self.sizes.n_replicas)
        self.n_spins = int(self.sizes.n_spins)

        def buf(nbytes):
            return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)

        self.state = buf(self.sizes.state_bytes)
        self.couplings = buf(self.sizes.coupling_bytes)
        self.field = buf(self.sizes.field_bytes) if self.sizes.field_bytes else None
        self.scratch = buf(self.sizes.scratch_bytes)
        spins0 = torch.cat([torch.from_numpy(np.ascontiguousarray(g.spins0)).reshape(-1)
                            for g in self.groups]).to(self.device)
        J = torch.cat([torch.from_numpy(np.ascontiguousarray(g.J)).reshape(-1)
                       for g in self.groups]).to(self.device)
        Hs = [g.H for g in self.groups]
        H = None
        if any(h is not None for h in Hs):
            H = torch.cat([torch.from_numpy(np.ascontiguousarray(
                h if h is not None else np.zeros_like(g.J))).reshape(-1)
                for g, h in zip(self.groups, Hs)]).to(self.device)
        self.stream = stream
        handle = C.c_void_p()
        check(lib.hsg_init_lattice(C.byref(self.desc), _ptr(spins0), _ptr(J),
                                   _ptr(H) if H is not None else None, _ptr(self.state),
                                   _ptr(self.couplings),
                                   _ptr(self.field) if self.field is not None else None,
                                   _ptr(self.scratch), _stream(stream), C.byref(handle)))
        self.h = handle

    # -- the calls of the ABI, same names ------------------------------------
    def sweep(self, n: int = 1) -> None:
        check(lib.hsg_sweep(self.h, int(n), _stream(self.stream)))

    def half_sweep(self, kind: int, parity: int, rep: int = 0) -> None:
        check(lib.hsg_half_sweep(self.h, int(kind), int(parity), int(rep), _stream(self.stream)))

    def pair_sweep(self, kind: int, rep: int = 0) -> None:
        check(lib.hsg_pair_sweep(self.h, int(kind), int(rep), _stream(self.stream)))

    def or_pairs(self, n_pairs: int) -> None:
        """n_pairs over-relaxation pairs as inside a sweep (two by two where fused)."""
        check(lib.hsg_or_pairs(self.h, int(n_pairs), _stream(self.stream)))

    def pt_exchange(self) -> None:
        check(lib.hsg_pt_exchange(self.h, _stream(self.stream)))

    def measure_energy(self):
        E = self.torch.empty(self.n_replicas, dtype=self.torch.float64, device=self.device)
        check(lib.hsg_measure_energy(self.h, _ptr(E), _stream(self.stream)))
        return E

    def measure_energy_static(self, out=None):
        """hsg_measure_energy through the library's fixed device scratch (no
        caller scratch, no allocation inside the call)."""
        E = out if out is not None else self.torch.empty(self.n_replicas, dtype=self.torch.float64,
                                                          device=self.device)
        check(lib.hsg_measure_energy_static(self.h, _ptr(E), _stream(self.stream)))
        return E

    def get_energies(self):
        E = self.torch.empty(self.n_replicas, dtype=self.torch.float64, device=self.device)
        check(lib.hsg_get_energies(self.h, _ptr(E), _stream(self.stream)))
        return E

    def measure_overlap(self, out=None):
        n = sum(g.n_samples * g.n_temps * 10 for g in self.groups)
        q = out if out is not None else self.torch.empty(n, dtype=self.torch.float64,
                                                          device=self.device)
        assert q.dtype == self.torch.float64 and q.numel() == n and q.is_contiguous()
        check(lib.hsg_measure_overlap(self.h, _ptr(q), _stream(self.stream)))
        return q

    def measure_kmodes(self, out=None):
        """[sum over groups of n_samples * n_temps * 84] float64: q^{mu nu}(k) and
        q_c^alpha(k) for k = 0 and the three smallest wave vectors (layout in
        hsg_measure_kmodes)."""
        n = sum(g.n_samples * g.n_temps * 84 for g in self.groups)
        q = out if out is not None else self.torch.empty(n, dtype=self.torch.float64,
                                                          device=self.device)
        check(lib.hsg_measure_kmodes(self.h, _ptr(q), _stream(self.stream)))
        return q

    def measure_pair_overlaps(self, out=None):
        """[sum over groups of n_samples * n_temps * P * 7] float64, P = O (O - 1) / 2:
        the local-overlap Fourier sums of every copy pair (layout in
        hsg_measure_pair_overlaps)."""
        n = sum(g.n_samples * g.n_temps * 7 * (g.n_copies * (g.n_copies - 1) // 2)
                for g in self.groups)
        q = out if out is not None else self.torch.empty(n, dtype=self.torch.float64,
                                                          device=self.device)
        check(lib.hsg_measure_pair_overlaps(self.h, _ptr(q), _stream(self.stream)))
        return q

    def measure_chi(self, out=None):
        """[sum over groups of n_samples * n_temps * 4 * 5] float64: chi_1, Re chi_2,
        Im chi_2, Re chi_3, Im chi_3 of Eq. (10) for k = 0, k_x, k_y, k_z (copies
        0..3; layout in hsg_measure_chi)."""
        n = sum(g.n_samples * g.n_temps * 20 for g in self.groups)
        q = out if out is not None else self.torch.empty(n, dtype=self.torch.float64,
                                                          device=self.device)
        check(lib.hsg_measure_chi(self.h, _ptr(q), _stream(self.stream)))
        return q

    def set_series(self, capacity: int):
        """Record every following sweep (energies by rung, q^2 by rung) into a new
        device buffer of `capacity` records; 0 switches the series off. Returns
        the buffer, [capacity, record] float64, or None."""
        if capacity <= 0:
            check(lib.hsg_set_series(self.h, None, 0, None))
            self.series = None
            return None
        rec = sum(g.n_samples * g.n_copies * g.n_temps + (g.n_samples * g.n_temps if g.n_copies >= 2 else 0)
                  for g in self.groups)
        buf = self.torch.full((int(capacity), rec), float("nan"), dtype=self.torch.float64,
                              device=self.device)
        n = C.c_int64()
        check(lib.hsg_set_series(self.h, _ptr(buf), int(capacity), C.byref(n)))
        assert n.value == rec
        self.series = buf
        return buf

    def get_series_count(self) -> int:
        n = C.c_int64()
        check(lib.hsg_get_series_count(self.h, C.byref(n)))
        return int(n.value)

    def get_spins(self):
        s = self.torch.empty(self.n_spins * 3, dtype=self.torch.float32, device=self.device)
        check(lib.hsg_get_spins(self.h, _ptr(s), _stream(self.stream)))
        return s

    def set_spins(self, s) -> None:
        assert s.dtype == self.torch.float32 and s.numel() == self.n_spins * 3 and s.is_contiguous()
        check(lib.hsg_set_spins(self.h, _ptr(s), _stream(self.stream)))

    def get_temp_map(self):
        m = self.torch.empty(self.n_replicas, dtype=self.torch.int32, device=self.device)
        check(lib.hsg_get_temp_map(self.h, _ptr(m), _stream(self.stream)))
        return m

    def set_temp_map(self, m) -> None:
        assert m.dtype == self.torch.int32 and m.numel() == self.n_replicas and m.is_contiguous()
        check(lib.hsg_set_temp_map(self.h, _ptr(m), _stream(self.stream)))

    def get_pt_accepts(self):
        n = sum(g.n_samples * g.n_copies * (g.n_temps - 1) for g in self.groups)
        a = self.torch.zeros(max(n, 1), dtype=self.torch.int64, device=self.device)
        check(lib.hsg_get_pt_accepts(self.h, _ptr(a), _stream(self.stream)))
        return a[:n]

    def get_state(self):
        t, n, s = C.c_uint64(), C.c_uint64(), C.c_uint64()
        check(lib.hsg_get_state(self.h, C.byref(t), C.byref(n), C.byref(s)))
        return int(t.value), int(n.value), int(s.value)

    def set_state(self, sweep_counter: int, pt_calls: int = 0) -> None:
        check(lib.hsg_set_state(self.h, int(sweep_counter), int(pt_calls), _stream(self.stream)))

    def set_tuning(self, slots_per_item: int) -> None:
        check(lib.hsg_set_tuning(self.h, int(slots_per_item)))

    def set_graphs(self, enable: bool) -> None:
        check(lib.hsg_set_graphs(self.h, int(bool(enable))))

    def set_kernel(self, variant: int) -> None:
        check(lib.hsg_set_kernel(self.h, int(variant)))

    def set_overlap(self, enable: bool) -> None:
        """Sweeps of the two halves of the samples on two streams (1) or one (0, default)."""
        check(lib.hsg_set_overlap(self.h, int(bool(enable))))

    def get_tuning(self):
        """(kernel variant, slots per work item, overlapped sweeps) in force."""
        v, c, o = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib.hsg_get_tuning(self.h, C.byref(v), C.byref(c), C.byref(o)))
        return v.value, c.value, o.value

    def autotune(self, n_sweeps: int = 4, restore: bool = True):
        """Time each kernel variant over n_sweeps real sweeps and keep the fastest.
        With restore, the state is saved to a temporary device buffer and put back,
        so the chain is unchanged; otherwise it advances by the trial sweeps.
        Returns (variant, slots_per_item)."""
        backup = None
        if restore:
            backup = torch.empty(self.sizes.state_bytes, dtype=torch.uint8, device=self.device)
        v, c = C.c_int32(), C.c_int32()
        check(lib.hsg_autotune(self.h, int(n_sweeps), None if backup is None else backup.data_ptr(),
                               C.byref(v), C.byref(c), _stream(self.stream)))
        del backup
        return v.value, c.value

    def set_chain(self, chain: int, tile_y: int = 0, tile_z: int = 0, n_hit: int = 1, tile_x: int = 0) -> None:
        """0: full-lattice checkerboard (default); 1: the tile-local chain with tiles
        of tile_x x tile_y x tile_z sites (0 = L) and n_hit repetitions per visit."""
        check(lib.hsg_set_chain(self.h, int(chain), int(tile_x), int(tile_y), int(tile_z), int(n_hit)))

    def set_batch(self, replicas: int) -> None:
        """Replicas per sweep batch: -1 off, 0 automatic, > 0 explicit."""
        check(lib.hsg_set_batch(self.h, int(replicas)))

    def set_stats(self, enable: bool = True) -> None:
        """Accumulate per-rung sums of E, E^2 and tempering round trips after every sweep."""
        check(lib.hsg_set_stats(self.h, int(bool(enable))))

    def reset_stats(self) -> None:
        check(lib.hsg_reset_stats(self.h, _stream(self.stream)))

    def get_stats(self):
        """(sums [n_replicas, 2] float64 by (sample, copy, rung): E, E^2;
        round trips [n_replicas] int32 by (sample, copy, slot); sweeps counted)."""
        sums = self.torch.empty((self.n_replicas, 2), dtype=self.torch.float64, device=self.device)
        trips = self.torch.empty(self.n_replicas, dtype=self.torch.int32, device=self.device)
        n = C.c_uint64()
        check(lib.hsg_get_stats(self.h, _ptr(sums), _ptr(trips), C.byref(n), _stream(self.stream)))
        return sums, trips, int(n.value)

    def set_geometry(self, group: int, tile_y: int = 0, z_slabs: int = 0) -> None:
        """z-march rows per work-group and z-slabs of group `group` (0, 0: default)."""
        check(lib.hsg_set_geometry(self.h, int(group), int(tile_y), int(z_slabs)))

    def get_geometry(self, group: int):
        """(rows per work-group, z-slabs) of the z-march of group `group`."""
        ty, zs = C.c_int32(), C.c_int32()
        check(lib.hsg_get_geometry(self.h, int(group), C.byref(ty), C.byref(zs)))
        return ty.value, zs.value

    def set_math(self, mode: int) -> None:
        """0: library transcendentals in the heat bath (default); 1: hardware ones."""
        check(lib.hsg_set_math(self.h, int(mode)))

    def sync(self) -> None:
        check(lib.hsg_sync(self.h, _stream(self.stream)))

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.hsg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_philox(ctr, key):
    """Device Philox4x32-10 on n blocks: ctr [n, 4], key [n, 2] (uint32 numpy)."""
    import torch
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    n = ctr.shape[0]
    dc = torch.from_numpy(ctr.view(np.int32)).cuda()
    dk = torch.from_numpy(key.view(np.int32)).cuda()
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    check(lib.hsg_debug_philox(_ptr(dc), _ptr(dk), _ptr(out), n, _stream(None)))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def debug_hw_math(x):
    """Hardware sin(2 pi x), cos(2 pi x), ln x, e^-x, 1/x, 1/sqrt(x), then the
    polynomial sin(2 pi x), cos(2 pi x) and the refined sqrt(x), 1/sqrt(x) of the
    default heat bath, and the heat bath's e^-x and ln x, on the device: an
    (n, 12) array."""
    import torch
    x = np.ascontiguousarray(x, dtype=np.float32)
    dx = torch.from_numpy(x).cuda()
    out = torch.empty((x.size, 12), dtype=torch.float32, device="cuda")
    check(lib.hsg_debug_hw_math(_ptr(dx), _ptr(out), x.size, _stream(None)))
    torch.cuda.synchronize()
    return out.cpu().numpy()
