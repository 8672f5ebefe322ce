"""Python binding of libsu3hb.so, the MI355X checkerboard SU(3) heatbath.

Argument marshalling only: every step of the Monte Carlo runs in the HIP
kernels behind the C ABI (include/su3hb.h).  The ``su3hb_*`` functions keep
the C names; :class:`Lattice` and :class:`Batch` add torch-owned device
memory and the current torch stream.  There is no CPU fallback: importing
works without the library, but every call raises if it was not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import workloads  # noqa: F401  (seeded inputs, presets)
from .workloads import COLD, FP32_12, FP32_18, FP64_12, FP64_18, HOT  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsu3hb.so")
MAX_D = 8

OK, EINVAL, ENOMEM, EHIP, ENOTSU3, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BYTES_PER_LINK = {FP64_18: 144, FP32_18: 72, FP32_12: 48, FP64_12: 96}


class su3hb_params(C.Structure):
    _fields_ = [("nd", C.c_int), ("extents", C.c_int * MAX_D), ("nlat", C.c_int), ("dlt_mask", C.c_uint),
                ("lat2test", C.c_int), ("precision", C.c_int), ("start", C.c_int), ("seed", C.c_uint64),
                ("device_links", C.c_void_p), ("device_bytes", C.c_size_t), ("hip_stream", C.c_void_p)]


class su3hb_stats(C.Structure):
    _fields_ = [("attempts", C.c_uint64 * 3), ("accepts", C.c_uint64 * 3), ("link_updates", C.c_uint64),
                ("dtrace", C.c_double)]

    def as_dict(self) -> dict:
        return {"attempts": list(self.attempts), "accepts": list(self.accepts),
                "link_updates": int(self.link_updates), "dtrace": float(self.dtrace)}


class su3hb_replica_desc(C.Structure):
    _fields_ = [("extents", C.c_int * MAX_D), ("beta", C.c_double), ("seed", C.c_uint64), ("start", C.c_int)]


class SU3HBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"su3hb error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes); restype None means void
_SIGS = {
    "su3hb_links_bytes": (C.c_int, [C.POINTER(su3hb_params), C.POINTER(C.c_size_t)]),
    "su3hb_init_lattice": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(su3hb_params)]),
    "su3hb_free": (None, [C.c_void_p]),
    "su3hb_sweep": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int, C.POINTER(su3hb_stats)]),
    "su3hb_overrelax": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int, C.POINTER(su3hb_stats)]),
    "su3hb_sweep_measure": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int,
                                      C.POINTER(C.c_double), C.POINTER(su3hb_stats)]),
    "su3hb_plaquette": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_double)]),
    "su3hb_get_links": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "su3hb_set_links": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "su3hb_get_state": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "su3hb_set_state": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64]),
    "su3hb_set_launch": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "su3hb_get_launch": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "su3hb_autotune": (C.c_int, [C.c_void_p, C.c_int]),
    "su3hb_sweep_timed": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "su3hb_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(su3hb_replica_desc), C.c_int,
                                     C.c_int, C.c_void_p]),
    "su3hb_batch_sweep": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(su3hb_stats)]),
    "su3hb_batch_plaquette": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "su3hb_batch_get_links": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
    "su3hb_batch_set_links": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
    "su3hb_batch_free": (None, [C.c_void_p]),
    "su3hb_sweep_measure_static": (C.c_int, [C.POINTER(su3hb_params), C.c_double, C.c_double, C.c_int, C.c_int,
                                             C.c_uint64, C.c_void_p]),
    "su3hb_last_error": (C.c_char_p, []),
}


def lib() -> C.CDLL:
    """Load libsu3hb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (or "
                              f"python -m paper_0904_0642_amd.build) first; there is no fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names() -> list:
    return list(_SIGS)


def last_error() -> str:
    return lib().su3hb_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise SU3HBError(rc, last_error())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------------------
# same-name wrappers (marshalling only)

def make_params(extents, nlat=1, dlt_mask=0, lat2test=False, precision=FP64_18, start=HOT, seed=1,
                device_links=None, device_bytes=0, hip_stream=None) -> su3hb_params:
    p = su3hb_params()
    ext = list(extents)
    p.nd = len(ext)
    for i, e in enumerate(ext[:MAX_D]):
        p.extents[i] = int(e)
    p.nlat = int(nlat)
    p.dlt_mask = int(dlt_mask)
    p.lat2test = int(bool(lat2test))
    p.precision = int(precision)
    p.start = int(start)
    p.seed = int(seed) & (2**64 - 1)
    p.device_links = device_links
    p.device_bytes = int(device_bytes)
    p.hip_stream = hip_stream
    return p


def su3hb_links_bytes(params: su3hb_params) -> int:
    n = C.c_size_t(0)
    _check(lib().su3hb_links_bytes(C.byref(params), C.byref(n)))
    return n.value


def su3hb_init_lattice(params: su3hb_params) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().su3hb_init_lattice(C.byref(h), C.byref(params)))
    return h


def su3hb_free(h):
    lib().su3hb_free(h)


def su3hb_sweep(h, beta0, beta1, n_hit, n_sweeps, want_stats=False):
    st = su3hb_stats() if want_stats else None
    _check(lib().su3hb_sweep(h, float(beta0), float(beta1), int(n_hit), int(n_sweeps),
                             C.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def su3hb_overrelax(h, beta0, beta1, n_sweeps, want_stats=False):
    st = su3hb_stats() if want_stats else None
    _check(lib().su3hb_overrelax(h, float(beta0), float(beta1), int(n_sweeps),
                                 C.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def su3hb_sweep_measure(h, beta0, beta1, n_hit, n_sweeps, want_stats=False):
    series = np.zeros((int(n_sweeps), 6))
    st = su3hb_stats() if want_stats else None
    _check(lib().su3hb_sweep_measure(h, float(beta0), float(beta1), int(n_hit), int(n_sweeps),
                                     _dp(series), C.byref(st) if st is not None else None))
    return (series, st.as_dict()) if st is not None else series


def su3hb_plaquette(h, beta0=0.0, beta1=None) -> np.ndarray:
    out = np.zeros(6)
    _check(lib().su3hb_plaquette(h, float(beta0), float(beta0 if beta1 is None else beta1), _dp(out)))
    return out


def su3hb_get_links(h, n_links: int) -> np.ndarray:
    out = np.empty(int(n_links) * 18)
    _check(lib().su3hb_get_links(h, _dp(out), out.size))
    return out


def su3hb_set_links(h, flat: np.ndarray):
    a = np.ascontiguousarray(flat, dtype=np.float64).reshape(-1)
    _check(lib().su3hb_set_links(h, _dp(a), a.size))


def su3hb_get_state(h):
    s, w = C.c_uint64(), C.c_uint64()
    _check(lib().su3hb_get_state(h, C.byref(s), C.byref(w)))
    return s.value, w.value


def su3hb_set_state(h, seed, sweep):
    _check(lib().su3hb_set_state(h, int(seed) & (2**64 - 1), int(sweep)))


def su3hb_set_launch(h, block, order, waves=2):
    _check(lib().su3hb_set_launch(h, int(block), int(order), int(waves)))


def su3hb_get_launch(h):
    b, o, w = C.c_int(), C.c_int(), C.c_int()
    _check(lib().su3hb_get_launch(h, C.byref(b), C.byref(o), C.byref(w)))
    return b.value, o.value, w.value


def su3hb_autotune(h, budget_ms=200):
    _check(lib().su3hb_autotune(h, int(budget_ms)))


def su3hb_sweep_timed(h, beta0, beta1, n_hit, n_sweeps, measure=False):
    timing = np.zeros(4)
    series = np.zeros((max(int(n_sweeps), 1), 6))
    _check(lib().su3hb_sweep_timed(h, float(beta0), float(beta1), int(n_hit), int(n_sweeps), int(bool(measure)),
                                   _dp(series) if measure else None, _dp(timing)))
    return timing, (series[: int(n_sweeps)] if measure else None)


def su3hb_batch_create(nd, replicas, precision, hip_stream=None) -> C.c_void_p:
    arr = (su3hb_replica_desc * len(replicas))()
    for i, (ext, beta, seed, start) in enumerate(replicas):
        for d, e in enumerate(ext):
            arr[i].extents[d] = int(e)
        arr[i].beta = float(beta)
        arr[i].seed = int(seed) & (2**64 - 1)
        arr[i].start = int(start)
    h = C.c_void_p()
    _check(lib().su3hb_batch_create(C.byref(h), int(nd), arr, len(replicas), int(precision), hip_stream))
    return h


def su3hb_batch_sweep(h, n_hit, n_sweeps, mode=0, want_stats=False):
    st = su3hb_stats() if want_stats else None
    _check(lib().su3hb_batch_sweep(h, int(n_hit), int(n_sweeps), int(mode),
                                   C.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def su3hb_batch_plaquette(h, nrep) -> np.ndarray:
    out = np.zeros(int(nrep) * 6)
    _check(lib().su3hb_batch_plaquette(h, _dp(out), out.size))
    return out.reshape(int(nrep), 6)


def su3hb_batch_get_links(h, replica, n_links) -> np.ndarray:
    out = np.empty(int(n_links) * 18)
    _check(lib().su3hb_batch_get_links(h, int(replica), _dp(out), out.size))
    return out


def su3hb_batch_set_links(h, replica, flat):
    a = np.ascontiguousarray(flat, dtype=np.float64).reshape(-1)
    _check(lib().su3hb_batch_set_links(h, int(replica), _dp(a), a.size))


def su3hb_batch_free(h):
    lib().su3hb_batch_free(h)


def su3hb_sweep_measure_static(params: su3hb_params, beta0, beta1, n_hit, n_sweeps, sweep0=0, series_ptr=None):
    """Measured sweeps with no allocation: params.device_links holds the
    links, series_ptr is a device address of 6 * n_sweeps doubles (or None).
    Asynchronous on params.hip_stream."""
    _check(lib().su3hb_sweep_measure_static(C.byref(params), float(beta0), float(beta1), int(n_hit),
                                            int(n_sweeps), int(sweep0), series_ptr))


# ---------------------------------------------------------------------------
# torch-facing handles

def _torch_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Lattice:
    """One lattice on the current GPU; links live in a torch uint8 tensor."""

    def __init__(self, extents, nlat=1, dlt_mask=0, lat2test=False, precision=FP64_18, start=HOT, seed=1,
                 device=None):
        import torch
        lib()
        self.extents = tuple(int(e) for e in extents)
        self.nd = len(self.extents)
        self.nlat = int(nlat)
        self.precision = int(precision)
        self.volume = int(np.prod(self.extents))
        probe = make_params(self.extents, nlat, dlt_mask, lat2test, precision, start, seed)
        nbytes = su3hb_links_bytes(probe)
        dev = torch.device("cuda" if device is None else device)
        self.buffer = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=dev)
        p = make_params(self.extents, nlat, dlt_mask, lat2test, precision, start, seed,
                        device_links=C.c_void_p(self.buffer.data_ptr()), device_bytes=self.buffer.numel(),
                        hip_stream=_torch_stream())
        self._h = su3hb_init_lattice(p)

    @property
    def handle(self):
        return self._h

    @property
    def n_links(self) -> int:
        return self.nlat * self.volume * self.nd

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            su3hb_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, beta0, beta1=None, n_hit=8, n_sweeps=1, stats=False):
        return su3hb_sweep(self._h, beta0, beta0 if beta1 is None else beta1, n_hit, n_sweeps, stats)

    def overrelax(self, beta0, beta1=None, n_sweeps=1, stats=False):
        return su3hb_overrelax(self._h, beta0, beta0 if beta1 is None else beta1, n_sweeps, stats)

    def sweep_measure(self, beta0, beta1=None, n_hit=8, n_sweeps=1, stats=False):
        return su3hb_sweep_measure(self._h, beta0, beta0 if beta1 is None else beta1, n_hit, n_sweeps, stats)

    def sweep_timed(self, beta0, beta1=None, n_hit=8, n_sweeps=1, measure=False):
        return su3hb_sweep_timed(self._h, beta0, beta0 if beta1 is None else beta1, n_hit, n_sweeps, measure)

    def plaquette(self, beta0=0.0, beta1=None) -> np.ndarray:
        return su3hb_plaquette(self._h, beta0, beta1)

    def get_links(self) -> np.ndarray:
        flat = su3hb_get_links(self._h, self.n_links)
        return flat.view(np.complex128).reshape(self.nlat, self.volume, self.nd, 3, 3)

    def set_links(self, links: np.ndarray):
        a = np.ascontiguousarray(np.asarray(links, dtype=np.complex128)).view(np.float64).reshape(-1)
        su3hb_set_links(self._h, a)

    def get_state(self):
        return su3hb_get_state(self._h)

    def set_state(self, seed, sweep):
        su3hb_set_state(self._h, seed, sweep)

    def set_launch(self, block, order, waves=2):
        su3hb_set_launch(self._h, block, order, waves)

    def get_launch(self):
        return su3hb_get_launch(self._h)

    def autotune(self, budget_ms=200):
        su3hb_autotune(self._h, budget_ms)


class Batch:
    """Independent periodic lattices (one D) updated together."""

    def __init__(self, nd, replicas, precision=FP32_18):
        lib()
        self.nd = int(nd)
        self.replicas = list(replicas)
        self.precision = int(precision)
        self._h = su3hb_batch_create(nd, self.replicas, precision, _torch_stream())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            su3hb_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def links_per_sweep(self) -> int:
        return int(sum(len(r[0]) * np.prod(r[0]) for r in self.replicas))

    def sweep(self, n_hit=8, n_sweeps=1, mode=0, stats=False):
        return su3hb_batch_sweep(self._h, n_hit, n_sweeps, mode, stats)

    def plaquette(self) -> np.ndarray:
        return su3hb_batch_plaquette(self._h, len(self.replicas))

    def get_links(self, r) -> np.ndarray:
        ext = self.replicas[r][0]
        V = int(np.prod(ext))
        flat = su3hb_batch_get_links(self._h, r, V * self.nd)
        return flat.view(np.complex128).reshape(1, V, self.nd, 3, 3)

    def set_links(self, r, links):
        a = np.ascontiguousarray(np.asarray(links, dtype=np.complex128)).view(np.float64).reshape(-1)
        su3hb_batch_set_links(self._h, r, a)

    def set_launch(self, block, order, waves=2):
        su3hb_set_launch(self._h, block, order, waves)

    def autotune(self, budget_ms=200):
        su3hb_autotune(self._h, budget_ms)
