"""TEST INFRASTRUCTURE: ctypes shim over the plain FP64 C oracle.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
in ``paper_0904_0642_amd``; see ``su3_oracle.c`` for the paper passages each
function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "su3_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_MAXD = 8


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc -O2 (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-lm", "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # SU3HB_ORACLE_LIB names another build of su3_oracle.c; the mutation
        # tests use it to run the pins against copies with planted mistakes
        path = os.environ.get("SU3HB_ORACLE_LIB", "")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(path)
        u32p = C.POINTER(C.c_uint32)
        dp = C.POINTER(C.c_double)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_uniform.argtypes = [C.c_uint32]
        L.or_uniform.restype = C.c_double
        L.or_reunitarize.argtypes = [dp]
        L.or_kp_draw.argtypes = [C.c_double, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int,
                                 dp, C.POINTER(C.c_uint64)]
        L.or_kp_draw.restype = C.c_int
        L.or_reflect_matrix.argtypes = [dp, dp]
        L.or_cm_update_matrix.argtypes = [dp, dp, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                          C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.or_create.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, C.c_uint, C.c_int, C.c_uint64]
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_set_threads.argtypes = [C.c_void_p, C.c_int]
        L.or_volume.argtypes = [C.c_void_p]
        L.or_volume.restype = C.c_long
        L.or_get_sweep.argtypes = [C.c_void_p]
        L.or_get_sweep.restype = C.c_uint32
        L.or_set_sweep.argtypes = [C.c_void_p, C.c_uint32]
        L.or_site_index.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.or_site_index.restype = C.c_long
        L.or_site_coords.argtypes = [C.c_void_p, C.c_long, C.POINTER(C.c_int)]
        L.or_parity.argtypes = [C.c_void_p, C.c_long]
        L.or_parity.restype = C.c_int
        L.or_neighbor.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_int, C.c_int,
                                  C.POINTER(C.c_int), C.POINTER(C.c_long)]
        L.or_cold_start.argtypes = [C.c_void_p]
        L.or_hot_start.argtypes = [C.c_void_p]
        L.or_get_links.argtypes = [C.c_void_p, dp, C.c_size_t]
        L.or_get_links.restype = C.c_int
        L.or_set_links.argtypes = [C.c_void_p, dp, C.c_size_t]
        L.or_set_links.restype = C.c_int
        L.or_staple.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_int, C.c_double, C.c_double, dp]
        L.or_update_link.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_int, C.c_double, C.c_double,
                                     C.c_int]
        L.or_update_link.restype = C.c_double
        L.or_link_margin.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_int, C.c_double, C.c_double,
                                     C.c_int]
        L.or_link_margin.restype = C.c_double
        L.or_update_slice.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                      C.POINTER(C.c_long)]
        L.or_update_slice.restype = C.c_double
        L.or_sweep.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int, dp]
        L.or_plaquette.argtypes = [C.c_void_p, C.c_double, C.c_double, dp]
        L.or_get_link.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_int, dp]
        L.or_put_link.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_int, dp]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11)."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(r: int) -> float:
    return lib().or_uniform(r)


def reunitarize(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt reunitarisation of one 3x3 complex matrix (returns a copy)."""
    m = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(3, 3)).view(np.float64).copy()
    lib().or_reunitarize(_dptr(m))
    return m.view(np.complex128).reshape(3, 3)


def kp_draw(alpha: float, nhit: int, seed: int, lid: int, sweep: int, sub: int):
    """Multi-hit Kennedy-Pendleton draw: returns (hit or -1, x0, attempts)."""
    x0 = C.c_double(np.nan)
    att = C.c_uint64(0)
    hit = lib().or_kp_draw(alpha, nhit, seed, lid, sweep, sub, C.byref(x0), C.byref(att))
    return hit, x0.value, att.value


def cm_update_matrix(u: np.ndarray, a: np.ndarray, nhit: int, seed: int, lid: int, sweep: int):
    """One CM update of matrix u for staple a (beta folded into a)."""
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(3, 3)).view(np.float64).copy()
    aa = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(3, 3)).view(np.float64).copy()
    at = (C.c_uint64 * 3)()
    ac = (C.c_uint64 * 3)()
    lib().or_cm_update_matrix(_dptr(uu), _dptr(aa), nhit, seed, lid, sweep, at, ac)
    return uu.view(np.complex128).reshape(3, 3), list(at), list(ac)


def reflect_matrix(u: np.ndarray, a: np.ndarray) -> np.ndarray:
    """One overrelaxation step of matrix u for staple a (three subgroup reflections)."""
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(3, 3)).view(np.float64).copy()
    aa = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(3, 3)).view(np.float64).copy()
    lib().or_reflect_matrix(_dptr(uu), _dptr(aa))
    return uu.view(np.complex128).reshape(3, 3)


class Lattice:
    """FP64 oracle lattice (canonical layout [layer][site][mu][3][3] complex)."""

    def __init__(self, extents, nlat=1, dlt_mask=0, lat2test=False, seed=1, threads=1):
        self.extents = [int(e) for e in extents]
        self.nd = len(self.extents)
        self.nlat = int(nlat)
        self.dlt_mask = int(dlt_mask)
        self.lat2test = bool(lat2test)
        self.seed = int(seed)
        n = (C.c_int * _MAXD)(*self.extents)
        h = lib().or_create(self.nd, n, self.nlat, self.dlt_mask, int(self.lat2test), self.seed)
        if not h:
            raise ValueError("oracle rejected lattice parameters")
        self._h = C.c_void_p(h)
        self.V = lib().or_volume(self._h)
        self.set_threads(threads)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_destroy(h)
            self._h = None

    def set_threads(self, n: int):
        lib().or_set_threads(self._h, int(n))

    @property
    def n_links(self) -> int:
        return self.nlat * self.V * self.nd

    @property
    def sweep_counter(self) -> int:
        return lib().or_get_sweep(self._h)

    @sweep_counter.setter
    def sweep_counter(self, v: int):
        lib().or_set_sweep(self._h, int(v))

    def cold_start(self):
        lib().or_cold_start(self._h)

    def hot_start(self):
        lib().or_hot_start(self._h)

    def get_links(self) -> np.ndarray:
        out = np.empty((self.nlat, self.V, self.nd, 3, 3), dtype=np.complex128)
        flat = out.view(np.float64).reshape(-1)
        if lib().or_get_links(self._h, _dptr(flat), flat.size) != 0:
            raise RuntimeError("get_links size mismatch")
        return out

    def set_links(self, links: np.ndarray):
        a = np.ascontiguousarray(np.asarray(links, dtype=np.complex128)).view(np.float64).reshape(-1)
        if lib().or_set_links(self._h, _dptr(a), a.size) != 0:
            raise ValueError("set_links size mismatch")

    def get_link(self, layer, s, mu) -> np.ndarray:
        out = np.zeros(18)
        lib().or_get_link(self._h, int(layer), int(s), int(mu), _dptr(out))
        return out.view(np.complex128).reshape(3, 3)

    def put_link(self, layer, s, mu, u):
        a = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(3, 3)).view(np.float64).reshape(-1)
        lib().or_put_link(self._h, int(layer), int(s), int(mu), _dptr(np.ascontiguousarray(a)))

    def site_index(self, x) -> int:
        xx = (C.c_int * _MAXD)(*[int(v) for v in x])
        return lib().or_site_index(self._h, xx)

    def site_coords(self, s: int):
        xx = (C.c_int * _MAXD)()
        lib().or_site_coords(self._h, int(s), xx)
        return list(xx)[: self.nd]

    def parity(self, s: int) -> int:
        return lib().or_parity(self._h, int(s))

    def neighbor(self, layer: int, s: int, direction: int, sign: int):
        lo = C.c_int()
        so = C.c_long()
        lib().or_neighbor(self._h, int(layer), int(s), int(direction), int(sign), C.byref(lo), C.byref(so))
        return lo.value, so.value

    def staple(self, layer, s, mu, beta0, beta1=None) -> np.ndarray:
        beta1 = beta0 if beta1 is None else beta1
        a = np.zeros(18)
        lib().or_staple(self._h, int(layer), int(s), int(mu), float(beta0), float(beta1), _dptr(a))
        return a.view(np.complex128).reshape(3, 3)

    def update_link(self, layer, s, mu, beta0, beta1=None, nhit=8) -> float:
        beta1 = beta0 if beta1 is None else beta1
        return lib().or_update_link(self._h, int(layer), int(s), int(mu), float(beta0), float(beta1),
                                    int(nhit))

    def link_margin(self, layer, s, mu, beta0, beta1=None, nhit=8) -> float:
        """Smallest |R4^2 - (1 - delta/2)| over the proposals the update of
        this link would evaluate now (the lattice is not changed)."""
        beta1 = beta0 if beta1 is None else beta1
        return lib().or_link_margin(self._h, int(layer), int(s), int(mu), float(beta0), float(beta1), int(nhit))

    def update_slice(self, p, mu, beta0, beta1=None, nhit=8, order=None) -> float:
        beta1 = beta0 if beta1 is None else beta1
        optr = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int64)
            assert order.size == self.V
            optr = order.ctypes.data_as(C.POINTER(C.c_long))
        return lib().or_update_slice(self._h, int(p), int(mu), float(beta0), float(beta1), int(nhit), optr)

    def sweep(self, beta0, beta1=None, nhit=8, nsweeps=1) -> dict:
        beta1 = beta0 if beta1 is None else beta1
        st = np.zeros(7)
        lib().or_sweep(self._h, float(beta0), float(beta1), int(nhit), int(nsweeps), _dptr(st))
        return {"attempts": st[0:3].astype(np.int64), "accepts": st[3:6].astype(np.int64),
                "dtrace": float(st[6])}

    def overrelax(self, beta0, beta1=None, nsweeps=1) -> dict:
        """Overrelaxation sweeps (a sweep with no heatbath hits)."""
        return self.sweep(beta0, beta1, nhit=0, nsweeps=nsweeps)

    def plaquette(self, beta0=0.0, beta1=None) -> np.ndarray:
        """[total, spacelike, timelike, layer0, layer1, beta-weighted trace sum]."""
        beta1 = beta0 if beta1 is None else beta1
        out = np.zeros(6)
        lib().or_plaquette(self._h, float(beta0), float(beta1), _dptr(out))
        return out
