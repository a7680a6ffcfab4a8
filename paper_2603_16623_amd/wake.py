"""Thin ctypes binding of ``libwake.so`` (C ABI declared in include/wake.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Functions carry the C names; ``WakeSolver`` and ``WakeBatch``
wrap a context / batch handle and raise ``WakeError`` on a negative status.
Host arrays are numpy float64; device arrays may be any object with
``data_ptr()`` (e.g. torch CUDA tensors), passed with ``device=True``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwake.so")

WAKE_OK, WAKE_EINVAL, WAKE_ENOMEM, WAKE_EDEVICE = 0, -1, -2, -3
WAKE_ESTATE, WAKE_EBREAKDOWN, WAKE_ENOTREC = -4, -5, -6
WAKE_BEAM_PARTICLES, WAKE_BEAM_GAUSSIAN, WAKE_LASER_GAUSSIAN = 1, 2, 3


class WakeError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class _Plasma(C.Structure):
    _fields_ = [("n_rings", C.c_int32), ("r0", C.c_void_p), ("dr", C.c_void_p),
                ("dens", C.c_void_p)]


class _Domain(C.Structure):
    _fields_ = [("dxi", C.c_double), ("n_xi", C.c_int32), ("record_stride", C.c_int32)]


class _Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q", C.c_double), ("n", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("xi", C.c_void_p), ("w", C.c_void_p),
                ("n_peak", C.c_double), ("sigma_r", C.c_double), ("sigma_xi", C.c_double),
                ("xi_c", C.c_double), ("a0", C.c_double), ("w0", C.c_double), ("L", C.c_double),
                ("xi_l", C.c_double)]


TUNE_BUCKETS = 8


class _Tuning(C.Structure):
    _fields_ = [("n_buckets", C.c_int32), ("lo", C.c_int32 * TUNE_BUCKETS),
                ("threads", C.c_int32 * TUNE_BUCKETS),
                ("rings_per_thread", C.c_int32 * TUNE_BUCKETS), ("rate", C.c_double * TUNE_BUCKETS)]


class _ServerConfig(C.Structure):
    _fields_ = [("threads", C.c_int32), ("slices_per_step", C.c_int32), ("max_active", C.c_int32),
                ("device_bytes", C.c_int64), ("ring_slices_per_step", C.c_int64),
                ("step_us", C.c_int32)]


_I, _P, _D, _I64 = C.c_int32, C.c_void_p, C.c_double, C.c_int64
_SIGS = {
    "wake_create": (_I, [C.POINTER(_P), C.POINTER(_Plasma), C.POINTER(_Domain), _P]),
    "wake_create_mobile_ions": (_I, [C.POINTER(_P), C.POINTER(_Plasma), C.c_double,
                                     C.POINTER(_Domain), _P]),
    "wake_species_fields": (_I, [_P, _I, _I, _P, _P, _P, _P, _P, _P, _I]),
    "wake_get_species_state": (_I, [_P, _I, C.POINTER(_I), _P, _P, _P, _P, _I]),
    "wake_set_species_state": (_I, [_P, _I, _I, _P, _P, _P, _P, _I]),
    "wake_add_beam": (_I, [_P, C.POINTER(_Source)]),
    "wake_prepare": (_I, [_P]),
    "wake_prepare_noalloc": (_I, [_P, _P, _I64]),
    "wake_solve": (_I, [_P, _I, _I]),
    "wake_fields": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _I]),
    "wake_lineout": (_I, [_P, _P, _P, _I]),
    "wake_set_grid": (_I, [_P, _I, C.c_double]),
    "wake_grid_fields": (_I, [_P, _I, _P, _P, _P, _P, _I]),
    "wake_set_grid_radii": (_I, [_P, _I64, _P, _P]),
    "wake_set_grid_beam": (_I, [_P]),
    "wake_grid_nodes": (_I, [_P, _I, C.POINTER(_I64), _P]),
    "wake_grid_chi": (_I, [_P, _I, _P, _I]),
    "wake_set_grid_chi": (_I, [_P, _I]),
    "wake_get_state": (_I, [_P, C.POINTER(_I), _P, _P, _P, _P, _I]),
    "wake_set_state": (_I, [_P, _I, _P, _P, _P, _P, _I]),
    "wake_reset": (_I, [_P]),
    "wake_status": (_I, [_P, C.POINTER(_I), C.POINTER(_I)]),
    "wake_sync": (_I, [_P]),
    "wake_autotune": (_I, [C.POINTER(_Plasma), C.POINTER(_Domain), C.POINTER(C.POINTER(_Source)),
                           C.POINTER(_I), _I, _I, _P, C.POINTER(_Tuning)]),
    "wake_set_tuning": (_I, [C.POINTER(_Tuning)]),
    "wake_get_tuning": (_I, [C.POINTER(_Tuning)]),
    "wake_get_threads": (_I, [_P, C.POINTER(_I)]),
    "wake_counters": (_I, [_P, C.POINTER(_I64), _I, _I]),
    "wake_footprint": (_I64, [_I, _I, _I64, _I]),
    "wake_destroy": (None, [_P]),
    "wake_strerror": (C.c_char_p, [_I]),
    "wake_tiling_count": (_I, []),
    "wake_tiling_get": (_I, [_I, C.POINTER(_I), C.POINTER(_I)]),
    "wake_set_tiling": (_I, [_I, _I]),
    "wake_set_cluster": (_I, [_I, _I]),
    "wake_get_layout": (_I, [C.c_void_p, C.POINTER(_I), C.POINTER(_I)]),
    "wake_get_tiling": (_I, [C.POINTER(_I), C.POINTER(_I)]),
    "wake_tiling_occupancy": (_I, [_I, _I]),
    "wake_batch_create": (_I, [C.POINTER(_P), C.POINTER(_P), _I, _P]),
    "wake_batch_solve": (_I, [_P, _I]),
    "wake_batch_capture": (_I, [_P, _I]),
    "wake_batch_replay": (_I, [_P]),
    "wake_batch_sync": (_I, [_P]),
    "wake_batch_destroy": (None, [_P]),
    "wake_server_create": (_I, [C.POINTER(_P), C.POINTER(_ServerConfig), _P]),
    "wake_server_submit": (_I, [_P, C.POINTER(_Plasma), C.POINTER(_Domain), C.POINTER(_Source), _I,
                                C.POINTER(_I64)]),
    "wake_server_step": (_I, [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)]),
    "wake_server_result": (_I, [_P, _I64, C.POINTER(_I), _P, _P, _P, _P, _P, _P, _P, _P]),
    "wake_server_stats": (_I, [_P, C.POINTER(_I64), C.POINTER(_I), C.POINTER(_I), C.POINTER(_I),
                               C.POINTER(_I64)]),
    "wake_server_ready": (_I, [_P, C.POINTER(_I64), _I, C.POINTER(_I)]),
    "wake_server_destroy": (None, [_P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built: there is
    no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2603_16623_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().wake_strerror(code).decode()


def _check(code: int, what: str):
    if code != WAKE_OK:
        raise WakeError(code, what)


def _host(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _source_struct(src) -> tuple:
    """Marshal one workload source object into a wake_source (keeps arrays alive)."""
    s = _Source()
    keep = []
    kind = getattr(src, "kind")
    if kind == "particles":
        s.kind = WAKE_BEAM_PARTICLES
        s.q = float(src.q)
        arrs = [_host(getattr(src, f)) for f in ("x", "y", "xi", "w")]
        s.n = len(arrs[0])
        s.x, s.y, s.xi, s.w = (a.ctypes.data for a in arrs)
        keep = arrs
    elif kind == "gaussian":
        s.kind = WAKE_BEAM_GAUSSIAN
        s.q, s.n_peak = float(src.q), float(src.n_peak)
        s.sigma_r, s.sigma_xi, s.xi_c = float(src.sigma_r), float(src.sigma_xi), float(src.xi_c)
    elif kind == "laser":
        s.kind = WAKE_LASER_GAUSSIAN
        s.a0, s.w0, s.L, s.xi_l = float(src.a0), float(src.w0), float(src.L), float(src.xi_l)
    else:
        raise ValueError(f"unknown source kind {kind!r}")
    return s, keep


def wake_footprint(n_rings: int, n_xi: int, n_particles: int, record_stride: int = 0) -> int:
    return int(load().wake_footprint(n_rings, n_xi, n_particles, record_stride))


def _tuning_dict(t) -> dict:
    n = t.n_buckets
    return dict(lo=list(t.lo[:n]), threads=list(t.threads[:n]),
                rings_per_thread=list(t.rings_per_thread[:n]), rate=list(t.rate[:n]))


def wake_autotune(insts, slices: int, stream=None) -> dict:
    """Measure and install the layout per ring-count bucket on these
    instances (see wake.h); returns the tuning as a dict."""
    n = len(insts)
    pls = (_Plasma * n)()
    dms = (_Domain * n)()
    srcp = (C.POINTER(_Source) * n)()
    nsrc = (_I * n)()
    keep = []
    for i, inst in enumerate(insts):
        r0, dr = _host(inst.r0), _host(inst.dr)
        dens = None if inst.dens is None else _host(inst.dens)
        keep += [r0, dr, dens]
        pls[i] = _Plasma(len(r0), r0.ctypes.data, dr.ctypes.data, None if dens is None else dens.ctypes.data)
        dms[i] = _Domain(float(inst.dxi), int(inst.n_xi), 0)
        arr = (_Source * max(1, len(inst.sources)))()
        for k, src in enumerate(inst.sources):
            st, kp = _source_struct(src)
            arr[k] = st
            keep.append(kp)
        keep.append(arr)
        srcp[i] = C.cast(arr, C.POINTER(_Source))
        nsrc[i] = len(inst.sources)
    t = _Tuning()
    _check(load().wake_autotune(pls, dms, srcp, nsrc, n, int(slices), stream, C.byref(t)), "wake_autotune")
    del keep
    return _tuning_dict(t)


def wake_set_tuning(tuning):
    """Install a tuning (a dict as wake_autotune returns), or remove it (None)."""
    if tuning is None:
        _check(load().wake_set_tuning(None), "wake_set_tuning")
        return
    t = _Tuning()
    n = len(tuning["lo"])
    t.n_buckets = n
    for b in range(n):
        t.lo[b] = tuning["lo"][b]
        t.threads[b] = tuning["threads"][b]
        t.rings_per_thread[b] = tuning["rings_per_thread"][b]
        t.rate[b] = tuning.get("rate", [0.0] * n)[b]
    _check(load().wake_set_tuning(C.byref(t)), "wake_set_tuning")


def wake_get_tuning():
    """The installed tuning as a dict, or None."""
    t = _Tuning()
    r = load().wake_get_tuning(C.byref(t))
    if r == WAKE_ESTATE:
        return None
    _check(r, "wake_get_tuning")
    return _tuning_dict(t)


def wake_tiling_count() -> int:
    return int(load().wake_tiling_count())


def wake_tiling_get(i: int):
    a, b = _I(), _I()
    _check(load().wake_tiling_get(i, C.byref(a), C.byref(b)), "wake_tiling_get")
    return a.value, b.value


def wake_set_tiling(threads: int, wgs_per_cu: int = 0):
    """Workgroup threads for contexts created from now on, and workgroups per
    compute unit of persistent launches (0: as many as fit)."""
    _check(load().wake_set_tiling(threads, wgs_per_cu), "wake_set_tiling")


def wake_set_cluster(rings_per_thread: int = 0, min_rings: int = 0):
    """Cooperative (multi-workgroup) layout for contexts created from now on:
    rings per thread of their members (0: 8) and the ring count from which
    contexts are cooperative (0: beyond one workgroup's LDS)."""
    _check(load().wake_set_cluster(rings_per_thread, min_rings), "wake_set_cluster")


def wake_get_tiling():
    a, b = _I(), _I()
    _check(load().wake_get_tiling(C.byref(a), C.byref(b)), "wake_get_tiling")
    return a.value, b.value


def wake_tiling_occupancy(threads: int, wgs_per_cu: int = 0) -> int:
    r = int(load().wake_tiling_occupancy(threads, wgs_per_cu))
    if r < 0:
        raise WakeError(r, "wake_tiling_occupancy")
    return r


class WakeSolver:
    """One context: a ring column, a window and its sources."""

    def __init__(self, r0, dr, dxi: float, n_xi: int, sources: Sequence = (), dens=None,
                 record_stride: int = 0, stream: Optional[int] = None,
                 ion_mass: Optional[float] = None):
        """ion_mass (electron masses): a two-species context whose ions move
        (wake_create_mobile_ions); None: immobile ions (wake_create)."""
        lib = load()
        self._lib = lib
        self.r0, self.dr = _host(r0), _host(dr)
        self.dens = None if dens is None else _host(dens)
        self.N, self.n_xi, self.dxi = len(self.r0), int(n_xi), float(dxi)
        self.record_stride = int(record_stride)
        pl = _Plasma(self.N, self.r0.ctypes.data, self.dr.ctypes.data,
                     None if self.dens is None else self.dens.ctypes.data)
        dm = _Domain(self.dxi, self.n_xi, self.record_stride)
        h = _P()
        self.ion_mass = None if ion_mass is None else float(ion_mass)
        if self.ion_mass is None:
            _check(lib.wake_create(C.byref(h), C.byref(pl), C.byref(dm), stream), "wake_create")
        else:
            _check(lib.wake_create_mobile_ions(C.byref(h), C.byref(pl), self.ion_mass, C.byref(dm),
                                               stream), "wake_create_mobile_ions")
        self.h = h
        for s in sources:
            self.wake_add_beam(s)

    @classmethod
    def from_instance(cls, inst, record_stride: int = 0, stream=None):
        return cls(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens,
                   record_stride, stream)

    def threads(self) -> int:
        """Workgroup threads of this context's layout."""
        t = _I()
        _check(self._lib.wake_get_threads(self.h, C.byref(t)), "wake_get_threads")
        return t.value

    def layout(self):
        """(workgroups, rings per thread) of this context's layout."""
        g, c = _I(), _I()
        _check(self._lib.wake_get_layout(self.h, C.byref(g), C.byref(c)), "wake_get_layout")
        return g.value, c.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._lib.wake_destroy(self.h)
            self.h = None

    __del__ = close

    def wake_add_beam(self, src):
        s, keep = _source_struct(src)
        _check(self._lib.wake_add_beam(self.h, C.byref(s)), "wake_add_beam")
        del keep

    def wake_prepare(self):
        _check(self._lib.wake_prepare(self.h), "wake_prepare")

    COUNTERS = ("slices", "fixups", "general_fixups", "member_local_rounds", "all_member_rounds",
                "segment_sorts", "bitonic_fallbacks", "meetings")

    def wake_counters(self, reset: bool = False) -> dict:
        """Event counters of this context's marches (see wake.h)."""
        out = (_I64 * 8)()
        _check(self._lib.wake_counters(self.h, out, 8, int(reset)), "wake_counters")
        return dict(zip(self.COUNTERS, (int(x) for x in out)))

    def wake_prepare_noalloc(self, table_ptr: int, table_bytes: int):
        """Beam table built into caller-owned device memory, no allocation."""
        _check(self._lib.wake_prepare_noalloc(self.h, table_ptr, int(table_bytes)),
               "wake_prepare_noalloc")

    def wake_solve(self, first: int = 0, count: Optional[int] = None):
        if count is None:
            count = self.n_xi - first
        _check(self._lib.wake_solve(self.h, first, count), "wake_solve")

    def wake_sync(self):
        _check(self._lib.wake_sync(self.h), "wake_sync")

    def wake_reset(self):
        _check(self._lib.wake_reset(self.h), "wake_reset")

    def wake_status(self):
        b, n = _I(), _I()
        _check(self._lib.wake_status(self.h, C.byref(b), C.byref(n)), "wake_status")
        return b.value, n.value

    def wake_fields(self, slice_: int = -1, out=None, device: bool = False):
        """dict of psi, er_bt, ez, bt, rho, ur (by ring id) at a slice."""
        names = ("psi", "er_bt", "ez", "bt", "rho", "ur")
        if out is None:
            out = {k: np.empty(self.N) for k in names}
        ptrs = [_ptr(out.get(k)) for k in names]
        _check(self._lib.wake_fields(self.h, slice_, *ptrs, int(device)), "wake_fields")
        return out

    def wake_set_grid(self, n_r: int, r_max: float = 0.0):
        """Uniform radial field grid of n_r cell-centred nodes to r_max."""
        _check(self._lib.wake_set_grid(self.h, int(n_r), float(r_max)), "wake_set_grid")
        self.grid_n = int(n_r)
        self.grid_r_max = float(r_max)

    def wake_set_grid_radii(self, radii, slice_off=None):
        """Field grid at given radii: the same ascending radii every slice, or
        (slice_off: n_xi + 1 offsets) slice n's radii[slice_off[n]:slice_off[n+1]]."""
        r = _host(radii)
        off = None if slice_off is None else np.ascontiguousarray(slice_off, dtype=np.int64)
        _check(self._lib.wake_set_grid_radii(self.h, len(r), _ptr(r), _ptr(off)),
               "wake_set_grid_radii")
        self.grid_n = len(r) if off is None else None

    def wake_set_grid_beam(self):
        """Field grid at every beam-table entry (the particles' own radii)."""
        _check(self._lib.wake_set_grid_beam(self.h), "wake_set_grid_beam")
        self.grid_n = None

    def grid_nodes(self, slice_: int = 0):
        """Radii of a slice's grid nodes."""
        n = _I64()
        _check(self._lib.wake_grid_nodes(self.h, slice_, C.byref(n), None), "wake_grid_nodes")
        r = np.empty(n.value)
        if n.value:
            _check(self._lib.wake_grid_nodes(self.h, slice_, C.byref(n), r.ctypes.data),
                   "wake_grid_nodes")
        return r

    def grid_radii(self):
        """The grid's node radii (every slice the same)."""
        return self.grid_nodes(0)

    def wake_grid_fields(self, slice_: int = -1, out=None, device: bool = False):
        """dict of psi, er_bt, ez, bt at the grid nodes of a slice."""
        names = ("psi", "er_bt", "ez", "bt")
        if out is None:
            at = slice_ if slice_ >= 0 else max(self.wake_status()[1] - 1, 0)
            n = _I64()
            _check(self._lib.wake_grid_nodes(self.h, at, C.byref(n), None), "wake_grid_nodes")
            out = {k: np.empty(n.value) for k in names}
        ptrs = [_ptr(out.get(k)) for k in names]
        _check(self._lib.wake_grid_fields(self.h, slice_, *ptrs, int(device)), "wake_grid_fields")
        return out

    def wake_set_grid_chi(self, on: bool = True):
        """Deposit chi = n/gamma on the context's grids (off by default)."""
        _check(self._lib.wake_set_grid_chi(self.h, int(bool(on))), "wake_set_grid_chi")

    def wake_grid_chi(self, slice_: int = -1):
        """chi = n/gamma at the grid nodes of a slice (uniform or fixed radii)."""
        at = slice_ if slice_ >= 0 else max(self.wake_status()[1] - 1, 0)
        n = _I64()
        _check(self._lib.wake_grid_nodes(self.h, at, C.byref(n), None), "wake_grid_nodes")
        out = np.empty(n.value)
        _check(self._lib.wake_grid_chi(self.h, slice_, out.ctypes.data, 0), "wake_grid_chi")
        return out

    def wake_lineout(self):
        psi, ez = np.empty(self.n_xi), np.empty(self.n_xi)
        _check(self._lib.wake_lineout(self.h, psi.ctypes.data, ez.ctypes.data, 0), "wake_lineout")
        return psi, ez

    def wake_get_state(self):
        names = ("rho", "ur", "f_rho", "f_u")
        out = {k: np.empty(self.N) for k in names}
        sl = _I()
        _check(self._lib.wake_get_state(self.h, C.byref(sl), *[out[k].ctypes.data for k in names], 0),
               "wake_get_state")
        out["slice"] = sl.value
        return out

    def wake_species_fields(self, species: int, slice_: int = -1, out=None, device: bool = False):
        """wake_fields of species 0 (electrons) or 1 (mobile ions)."""
        names = ("psi", "er_bt", "ez", "bt", "rho", "ur")
        if out is None:
            out = {k: np.empty(self.N) for k in names}
        ptrs = [_ptr(out.get(k)) for k in names]
        _check(self._lib.wake_species_fields(self.h, int(species), slice_, *ptrs, int(device)),
               "wake_species_fields")
        return out

    def wake_get_species_state(self, species: int):
        names = ("rho", "ur", "f_rho", "f_u")
        out = {k: np.empty(self.N) for k in names}
        sl = _I()
        _check(self._lib.wake_get_species_state(self.h, int(species), C.byref(sl),
                                                *[out[k].ctypes.data for k in names], 0),
               "wake_get_species_state")
        out["slice"] = sl.value
        return out

    def wake_set_species_state(self, species: int, slice_: int, rho, ur, f_rho=None, f_u=None):
        arrs = [_host(rho), _host(ur), None if f_rho is None else _host(f_rho),
                None if f_u is None else _host(f_u)]
        _check(self._lib.wake_set_species_state(self.h, int(species), slice_,
                                                *[_ptr(a) for a in arrs], 0),
               "wake_set_species_state")

    def wake_set_state(self, slice_: int, rho, ur, f_rho=None, f_u=None):
        arrs = [_host(rho), _host(ur), None if f_rho is None else _host(f_rho),
                None if f_u is None else _host(f_u)]
        _check(self._lib.wake_set_state(self.h, slice_, *[_ptr(a) for a in arrs], 0),
               "wake_set_state")


class WakeBatch:
    """Many contexts marched by one persistent launch."""

    def __init__(self, solvers: Sequence[WakeSolver], stream: Optional[int] = None):
        lib = load()
        self._lib = lib
        self.solvers = list(solvers)
        arr = (_P * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = _P()
        _check(lib.wake_batch_create(C.byref(h), arr, len(self.solvers), stream), "wake_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._lib.wake_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def wake_batch_solve(self, n_slices: int = -1):
        _check(self._lib.wake_batch_solve(self.h, n_slices), "wake_batch_solve")

    def wake_batch_capture(self, grid: int = 0):
        _check(self._lib.wake_batch_capture(self.h, grid), "wake_batch_capture")

    def wake_batch_replay(self):
        _check(self._lib.wake_batch_replay(self.h), "wake_batch_replay")

    def wake_batch_sync(self):
        _check(self._lib.wake_batch_sync(self.h), "wake_batch_sync")


class WakeServer:
    """Continuous batching of independent solves (wake_server_*)."""

    def __init__(self, device_bytes: int, slices_per_step: int = 100, threads: int = 0,
                 max_active: int = 0, ring_slices_per_step: int = 0, step_us: int = 0,
                 stream: Optional[int] = None):
        lib = load()
        self._lib = lib
        cfg = _ServerConfig(int(threads), int(slices_per_step), int(max_active), int(device_bytes),
                            int(ring_slices_per_step), int(step_us))
        h = _P()
        _check(lib.wake_server_create(C.byref(h), C.byref(cfg), stream), "wake_server_create")
        self.h = h
        self.meta = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._lib.wake_server_destroy(self.h)
            self.h = None

    __del__ = close

    def submit(self, r0, dr, dxi: float, n_xi: int, sources: Sequence = (), dens=None) -> int:
        r0, dr = _host(r0), _host(dr)
        dens = None if dens is None else _host(dens)
        pl = _Plasma(len(r0), r0.ctypes.data, dr.ctypes.data, None if dens is None else dens.ctypes.data)
        dm = _Domain(float(dxi), int(n_xi), 0)
        structs, keep = [], []
        for src in sources:
            st, k = _source_struct(src)
            structs.append(st)
            keep.append(k)
        arr = (_Source * max(1, len(structs)))(*structs)
        t = _I64()
        _check(self._lib.wake_server_submit(self.h, C.byref(pl), C.byref(dm), arr, len(structs),
                                            C.byref(t)), "wake_server_submit")
        del keep
        self.meta[t.value] = (len(r0), int(n_xi))
        return t.value

    def submit_instance(self, inst) -> int:
        return self.submit(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)

    def step(self):
        a, q, d = _I(), _I(), _I()
        _check(self._lib.wake_server_step(self.h, C.byref(a), C.byref(q), C.byref(d)), "wake_server_step")
        return a.value, q.value, d.value

    def result(self, ticket: int):
        """dict with status, breakdown, psi_axis, ez_axis and the final fields (or
        None while the request is not finished)."""
        N, n_xi = self.meta[ticket]
        out = {k: np.empty(n_xi) for k in ("psi_axis", "ez_axis")}
        out.update({k: np.empty(N) for k in ("psi", "er_bt", "ez", "bt", "rho", "ur")})
        brk = _I()
        r = self._lib.wake_server_result(self.h, ticket, C.byref(brk),
                                         *[out[k].ctypes.data for k in ("psi_axis", "ez_axis", "psi",
                                                                        "er_bt", "ez", "bt", "rho",
                                                                        "ur")])
        if r == WAKE_ESTATE:
            return None
        del self.meta[ticket]
        out["status"] = r
        out["breakdown"] = brk.value
        return out

    def ready(self, cap: int = 4096):
        """Tickets whose results are waiting to be fetched."""
        buf = (_I64 * cap)()
        n = _I()
        _check(self._lib.wake_server_ready(self.h, buf, cap, C.byref(n)), "wake_server_ready")
        return [buf[i] for i in range(n.value)]

    def stats(self):
        b, a, q, n, w = _I64(), _I(), _I(), _I(), _I64()
        _check(self._lib.wake_server_stats(self.h, C.byref(b), C.byref(a), C.byref(q), C.byref(n),
                                           C.byref(w)), "wake_server_stats")
        return dict(bytes_in_use=b.value, active=a.value, queued=q.value, results=n.value,
                    ring_slices=w.value)
