"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke check and the
benchmark's cpu_baseline leg, never by the product path.  It imports nothing
from the HIP package; callers hand it a workload description (any object with
the attributes of ``Workload``) and numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the same oracle built with multiply-add contraction: a second roundoff
# sample for the parity floor, never a reference
LIB_FMA_PATH = os.path.join(HERE, "liboracle_fma.so")
NV = 9


class Params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("nx", ctypes.c_int), ("ng", ctypes.c_int),
        ("nstages", ctypes.c_int), ("reflux", ctypes.c_int),
        ("fix_small_values", ctypes.c_int), ("nthreads", ctypes.c_int),
        ("base_blocks", ctypes.c_int * 3), ("bc_lo", ctypes.c_int * 3),
        ("bc_hi", ctypes.c_int * 3), ("xmin", ctypes.c_double * 3),
        ("xmax", ctypes.c_double * 3), ("bc_fixed_prim", ctypes.c_double * (3 * 2 * NV)),
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("glm_alpha", ctypes.c_double),
        ("small_density", ctypes.c_double), ("small_pressure", ctypes.c_double),
        ("limiter", ctypes.c_int), ("flux", ctypes.c_int),
    ]


_libs = {}


def lib(fma: bool = False):
    """The oracle library (fma=True: its contracted build, see LIB_FMA_PATH)."""
    path = LIB_FMA_PATH if fma else LIB_PATH
    if path not in _libs:
        if not os.path.exists(path):
            from . import build as _build
            _build.build()
        _libs[path] = _setup(ctypes.CDLL(path))
    return _libs[path]


def _setup(_lib):
    if True:
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        _lib.oracle_create.restype = ctypes.c_void_p
        _lib.oracle_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ip, ip, dp]
        _lib.oracle_destroy.argtypes = [ctypes.c_void_p]
        _lib.oracle_regrid.restype = ctypes.c_void_p
        _lib.oracle_regrid.argtypes = [ctypes.c_void_p, ctypes.c_int, ip, ip]
        _lib.oracle_steps.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        _lib.oracle_steps_to_time.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        _lib.oracle_euler_stage.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        _lib.oracle_cfl.argtypes = [ctypes.c_void_p, dp, dp, dp]
        _lib.oracle_flags.argtypes = [ctypes.c_void_p]
        _lib.oracle_fix_count.restype = ctypes.c_long
        _lib.oracle_fix_count.argtypes = [ctypes.c_void_p]
        _lib.oracle_get_cons.argtypes = [ctypes.c_void_p, dp]
        _lib.oracle_set_cons.argtypes = [ctypes.c_void_p, dp]
        _lib.oracle_fill_padded.argtypes = [ctypes.c_void_p, dp]
        _lib.oracle_last_error.restype = ctypes.c_char_p
        _lib.oracle_prim_to_cons.argtypes = [dp, ctypes.c_double, dp]
        _lib.oracle_cons_to_prim.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        _lib.oracle_fast_speed.restype = ctypes.c_double
        _lib.oracle_fast_speed.argtypes = [dp, ctypes.c_int, ctypes.c_double]
        _lib.oracle_face_increments.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        _lib.oracle_weno5_face.restype = ctypes.c_double
        _lib.oracle_weno5_face.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int, ctypes.c_double]
        _lib.oracle_mp5_face.restype = ctypes.c_double
        _lib.oracle_mp5_face.argtypes = [ctypes.c_double] * 5
        _lib.oracle_vanleer.restype = ctypes.c_double
        _lib.oracle_vanleer.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib.oracle_minmod.restype = ctypes.c_double
        _lib.oracle_minmod.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib.oracle_glm_interface.argtypes = [ctypes.c_double] * 5 + [dp]
        _lib.oracle_face_flux.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        _lib.oracle_phys_flux.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp]
        _lib.oracle_face_flux_kind.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def make_params(w, nthreads: Optional[int] = None, nstages: Optional[int] = None) -> Params:
    p = Params()
    p.ndim = w.ndim
    p.nx = w.nx
    p.ng = w.ng
    p.nstages = w.nstages if nstages is None else nstages
    p.reflux = w.reflux
    p.fix_small_values = w.fix_small_values
    p.nthreads = default_threads() if nthreads is None else nthreads
    for d in range(3):
        p.base_blocks[d] = int(w.base_blocks[d]) if d < w.ndim else 1
        p.bc_lo[d] = int(w.bc_lo[d])
        p.bc_hi[d] = int(w.bc_hi[d])
        p.xmin[d] = float(w.xmin[d])
        p.xmax[d] = float(w.xmax[d])
    fixed = np.ascontiguousarray(np.asarray(w.bc_fixed_prim, dtype=np.float64).reshape(-1))
    for i in range(3 * 2 * NV):
        p.bc_fixed_prim[i] = fixed[i]
    p.gamma = w.gamma
    p.cfl = w.cfl
    p.glm_alpha = w.glm_alpha
    p.small_density = w.small_density
    p.small_pressure = w.small_pressure
    p.limiter = int(getattr(w, "limiter", 0))
    p.flux = int(getattr(w, "flux", 0))
    return p


class OracleSim:
    """One oracle simulation; state lives in the C++ library."""

    def __init__(self, w, nthreads: Optional[int] = None, nstages: Optional[int] = None, fma: bool = False):
        self._lib = lib(fma)
        self.w = w
        self.params = make_params(w, nthreads, nstages)
        self.level = np.ascontiguousarray(w.level, dtype=np.int32)
        self.ijk = np.ascontiguousarray(w.ijk, dtype=np.int32)
        prim = np.ascontiguousarray(w.prim, dtype=np.float64)
        self.h = self._lib.oracle_create(ctypes.byref(self.params), len(self.level), _ip(self.level),
                                     _ip(self.ijk), _dp(prim))
        if not self.h:
            raise ValueError("oracle_create: " + self._lib.oracle_last_error().decode())
        self.shape = (len(self.level), NV) + (w.nx,) * w.ndim

    def regrid(self, level, ijk) -> "OracleSim":
        """A new simulation on the leaf set (level, ijk), every block of which
        is an old block, a child of an old leaf or the parent of old leaves,
        holding the old state copied, prolonged or restricted
        (oracle_regrid)."""
        import dataclasses
        level = np.ascontiguousarray(level, dtype=np.int32)
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        w = dataclasses.replace(self.w, level=level, ijk=ijk,
                                prim=np.zeros((len(level), NV) + (self.w.nx,) * self.w.ndim))
        new = OracleSim.__new__(OracleSim)
        new._lib = self._lib
        new.w, new.params, new.level, new.ijk = w, self.params, level, ijk
        new.h = self._lib.oracle_regrid(self.h, len(level), _ip(level), _ip(ijk))
        if not new.h:
            raise ValueError("oracle_regrid: " + self._lib.oracle_last_error().decode())
        new.shape = (len(level), NV) + (w.nx,) * w.ndim
        return new

    def close(self):
        if self.h:
            self._lib.oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def steps(self, n: int, check: bool = True) -> np.ndarray:
        """Advance n SSPRK steps; returns [n, 4] (dt, c_h, kappa, flags)."""
        diag = np.zeros((max(n, 1), 4))
        rc = self._lib.oracle_steps(self.h, n, _dp(diag))
        if rc == -1:
            raise RuntimeError("oracle: " + self._lib.oracle_last_error().decode())
        if rc != 0 and check:
            raise FloatingPointError("oracle: non-physical state or invalid dt (flags=%d)" % self.flags())
        return diag[:n]

    def steps_to_time(self, t_end: float, max_steps: int = 1000000) -> int:
        n = self._lib.oracle_steps_to_time(self.h, t_end, max_steps)
        if n == -1:
            raise RuntimeError("oracle: " + self._lib.oracle_last_error().decode())
        if n < 0:
            raise FloatingPointError("oracle: non-physical state or invalid dt (flags=%d)" % self.flags())
        return n

    def euler_stage(self, dt: float, ch: float, kappa: float):
        if self._lib.oracle_euler_stage(self.h, dt, ch, kappa) != 0:
            raise RuntimeError("oracle: " + self._lib.oracle_last_error().decode())

    def cfl(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        fl = self._lib.oracle_cfl(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value, fl

    def flags(self) -> int:
        return self._lib.oracle_flags(self.h)

    def fix_count(self) -> int:
        return self._lib.oracle_fix_count(self.h)

    def cons(self) -> np.ndarray:
        out = np.empty(self.shape)
        self._lib.oracle_get_cons(self.h, _dp(out))
        return out

    def set_cons(self, u: np.ndarray):
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == self.shape
        self._lib.oracle_set_cons(self.h, _dp(u))

    def padded(self) -> np.ndarray:
        pn = self.w.nx + 2 * self.w.ng
        out = np.empty((len(self.level), NV) + (pn,) * self.w.ndim)
        if self._lib.oracle_fill_padded(self.h, _dp(out)) != 0:
            raise RuntimeError("oracle: " + self._lib.oracle_last_error().decode())
        return out


def lohner_indicator(w, padded: np.ndarray, weights, wavefilter: float = 0.01) -> np.ndarray:
    """Loehner's (1987) second-derivative error indicator per block, in its
    per-direction form, from ghost-filled blocks (OracleSim.padded(); only
    face neighbours are read).  For every interior cell and conserved
    variable q, with a, b, e the lower neighbour, the cell and the upper
    neighbour along direction d:
        E_q = sqrt(sum_d (a - 2b + e)^2
                   / sum_d (|e - b| + |b - a| + wavefilter (|e| + 2|b| + |a|))^2),
    0 where the denominator is 0; the block's indicator is the largest
    sum_q weights[q] E_q over its cells."""
    g, n, nd = w.ng, w.nx, w.ndim
    out = np.zeros(padded.shape[0])
    inner = slice(g, g + n)
    for b in range(padded.shape[0]):
        total = np.zeros((n,) * nd)
        for q in range(NV):
            if not weights[q] > 0.0:
                continue
            u = padded[b, q]
            num = np.zeros((n,) * nd)
            den = np.zeros((n,) * nd)
            for d in range(nd):
                ax = nd - 1 - d  # array axes run [.., z, y, x]
                def shifted(o):
                    sl = [inner] * nd
                    sl[ax] = slice(g + o, g + o + n)
                    return u[tuple(sl)]
                a, c, e = shifted(-1), shifted(0), shifted(1)
                num += (a - 2.0 * c + e) ** 2
                den += (np.abs(e - c) + np.abs(c - a) + wavefilter * (np.abs(e) + 2.0 * np.abs(c) + np.abs(a))) ** 2
            pos = den > 0.0
            est = np.zeros_like(num)
            est[pos] = np.sqrt(num[pos] / den[pos])
            total += weights[q] * est
        out[b] = total.max()
    return out


def run(w, nsteps: Optional[int] = None, nthreads: Optional[int] = None, check: bool = True, fma: bool = False):
    """Run a workload for nsteps (default w.nsteps); returns (cons, diag).
    fma=True runs the contracted build (a roundoff sample, not a reference)."""
    sim = OracleSim(w, nthreads, fma=fma)
    try:
        diag = sim.steps(w.nsteps if nsteps is None else nsteps, check=check)
        return sim.cons(), diag
    finally:
        sim.close()


# --- point functions -------------------------------------------------------

def prim_to_cons(w, gamma: float) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.empty(NV)
    lib().oracle_prim_to_cons(_dp(w), gamma, _dp(u))
    return u


def cons_to_prim(u, gamma: float, small_rho: float = 0.0, small_p: float = 0.0, fix: int = 0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = np.empty(NV)
    bad = lib().oracle_cons_to_prim(_dp(u), gamma, small_rho, small_p, fix, _dp(w))
    return w, bad


def fast_speed(w, d: int, gamma: float) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    return lib().oracle_fast_speed(_dp(w), d, gamma)


def weno5_face(vm2, vm1, v0, vp1, vp2, z: bool = False, zp: bool = False, lam: float = 0.0) -> float:
    """WENO value at the face between cells i and i+1 from cells i-2 .. i+2
    (z: the WENO-Z weights; zp: the WENO-Z+ weights with lambda = lam)."""
    return lib().oracle_weno5_face(vm2, vm1, v0, vp1, vp2, 2 if zp else (1 if z else 0), lam)


def mp5_face(vm2, vm1, v0, vp1, vp2) -> float:
    """Monotonicity-preserving fifth-order value at the face between cells i
    and i+1 from cells i-2 .. i+2."""
    return lib().oracle_mp5_face(vm2, vm1, v0, vp1, vp2)


def face_increments(lim: int, dm: float, dp: float):
    """(inc_right, inc_left): a cell's face values are w + inc_right/2 and
    w - inc_left/2 for backward / forward differences dm, dp."""
    r, l = ctypes.c_double(), ctypes.c_double()
    if lib().oracle_face_increments(lim, dm, dp, ctypes.byref(r), ctypes.byref(l)) != 0:
        raise ValueError("unknown limiter %d" % lim)
    return r.value, l.value


def vanleer(dm: float, dp: float) -> float:
    return lib().oracle_vanleer(dm, dp)


def minmod(a: float, b: float) -> float:
    return lib().oracle_minmod(a, b)


def glm_interface(bnl, bnr, psl, psr, ch):
    out = np.empty(2)
    lib().oracle_glm_interface(bnl, bnr, psl, psr, ch, _dp(out))
    return out[0], out[1]


def face_flux(wl, wr, d: int, ch: float, gamma: float, flux: int = 0) -> np.ndarray:
    """Interface flux of the primitive states wl, wr along d: GLM interface
    values, then HLL (flux = 0), HLLD (flux = 1) or HLLC (flux = 2)."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    F = np.empty(NV)
    if flux == 0:
        lib().oracle_face_flux(_dp(wl), _dp(wr), d, ch, gamma, _dp(F))
    elif lib().oracle_face_flux_kind(_dp(wl), _dp(wr), d, ch, gamma, flux, _dp(F)) != 0:
        raise ValueError("unknown flux scheme %d" % flux)
    return F


def phys_flux(w, d: int, gamma: float) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    F = np.empty(NV)
    lib().oracle_phys_flux(_dp(w), d, gamma, _dp(F))
    return F
