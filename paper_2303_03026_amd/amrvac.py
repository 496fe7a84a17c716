"""Python binding of the HIP library ``libamrvac.so`` (C ABI in include/amrvac.h).

Argument marshalling only: torch provides device memory and the stream, every
step of the scheme runs in the library's kernels.  There is no fallback: if
the library is missing or no HIP device is present, construction raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrvac.so")
NV = 9

FP64, FP32_MIXED = 0, 1
LIM_VANLEER, LIM_KOREN, LIM_CADA3, LIM_WENO5, LIM_WENOZ5, LIM_MP5, LIM_WENOZP5 = 0, 1, 2, 3, 4, 5, 6
FLUX_HLL, FLUX_HLLD, FLUX_HLLC = 0, 1, 2
PATH_PLAIN, PATH_FUSED = 0, 1
FLAG_SMALL_RHO, FLAG_SMALL_P, FLAG_BAD_DT = 1, 2, 4
E_OK, E_ARG, E_HIP, E_NOMEM, E_NONPHYSICAL, E_STATE = 0, -1, -2, -3, -4, -5

# every entry point declared in include/amrvac.h
ABI_SYMBOLS = ("amrvac_slot_bytes", "amrvac_init_blocks", "amrvac_set_primitive", "amrvac_get_conserved",
               "amrvac_fill_ghosts", "amrvac_cfl_dt", "amrvac_stage", "amrvac_advance", "amrvac_set_path",
               "amrvac_sync_flags", "amrvac_reset_flags", "amrvac_last_error", "amrvac_destroy",
               "amrvac_batch_create", "amrvac_batch_add_job", "amrvac_batch_step", "amrvac_batch_job_info",
               "amrvac_batch_get_job", "amrvac_batch_remove_job", "amrvac_batch_free_blocks",
               "amrvac_set_tune", "amrvac_get_tune", "amrvac_autotune", "amrvac_stage_cfl", "amrvac_combine",
               "amrvac_regrid_plan", "amrvac_regrid", "amrvac_lohner", "amrvac_stage_noalloc")
TUNE_MAX_CANDIDATES = 12
SLOT_LEAD_FP64 = 16  # bytes before the first block of an FP64 slot


def slot_lead(precision: int) -> int:
    return SLOT_LEAD_FP64 if precision == FP64 else 0


class AmrvacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("amrvac status %d: %s" % (code, msg))
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("block_nx", ctypes.c_int), ("nghost", ctypes.c_int),
        ("precision", ctypes.c_int), ("base_blocks", ctypes.c_int * 3), ("bc_lo", ctypes.c_int * 3),
        ("bc_hi", ctypes.c_int * 3), ("fix_small_values", ctypes.c_int), ("reflux", ctypes.c_int),
        ("xmin", ctypes.c_double * 3), ("xmax", ctypes.c_double * 3), ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double), ("glm_alpha", ctypes.c_double), ("small_density", ctypes.c_double),
        ("small_pressure", ctypes.c_double), ("bc_fixed_prim", ctypes.c_double * (3 * 2 * NV)),
        ("limiter", ctypes.c_int), ("flux", ctypes.c_int),
    ]


class Tune(ctypes.Structure):
    """Launch shape of the fused stage (amrvac_tune)."""
    _fields_ = [("zseg", ctypes.c_int), ("rotate", ctypes.c_int), ("xcd", ctypes.c_int)]

    def as_tuple(self):
        return (self.zseg, self.rotate, self.xcd)


def tune_candidates(ndim: int):
    """The autotuner's candidates in its enumeration order."""
    zs = (1, 2, 4) if ndim == 3 else (1,)
    return [(z, r, x) for z in zs for r in (0, 1) for x in (0, 1)]


_lib = None


def load_library():
    """Load libamrvac.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libamrvac.so is not built (run __graft_entry__.build() or "
                          "python paper_2303_03026_amd/build.py)")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (one runtime per process; loaded the other way round, two runtimes
    # would each initialise the device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    lib.amrvac_slot_bytes.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.amrvac_init_blocks.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(GridDesc), ctypes.c_int, ip, ip,
                                       ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.amrvac_set_primitive.argtypes = [vp, ctypes.c_int, vp]
    lib.amrvac_get_conserved.argtypes = [vp, ctypes.c_int, vp]
    lib.amrvac_fill_ghosts.argtypes = [vp, ctypes.c_int]
    lib.amrvac_cfl_dt.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.amrvac_stage.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp, vp, vp]
    lib.amrvac_stage_cfl.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp, vp, vp]
    lib.amrvac_stage_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp, vp, vp]
    lib.amrvac_combine.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.amrvac_regrid_plan.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_int, ip, ip, ip, ctypes.c_int, ctypes.c_int,
                                       ip, ip, ip]
    lib.amrvac_regrid.argtypes = [vp, ctypes.c_int, ctypes.c_int, ip, ip, ctypes.POINTER(vp), ctypes.c_int,
                                  ctypes.POINTER(vp)]
    lib.amrvac_lohner.argtypes = [vp, ctypes.c_int, dp, ctypes.c_double, vp]
    lib.amrvac_advance.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.amrvac_set_path.argtypes = [vp, ctypes.c_int]
    lib.amrvac_sync_flags.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_longlong), dp]
    lib.amrvac_reset_flags.argtypes = [vp]
    lib.amrvac_last_error.argtypes = [vp]
    lib.amrvac_last_error.restype = ctypes.c_char_p
    lib.amrvac_destroy.argtypes = [vp]
    lib.amrvac_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(GridDesc), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.POINTER(vp), vp]
    lib.amrvac_batch_add_job.argtypes = [vp, ctypes.POINTER(GridDesc), ctypes.c_int, ip, ip, vp, ctypes.c_int, ip]
    lib.amrvac_batch_step.argtypes = [vp]
    lib.amrvac_batch_job_info.argtypes = [vp, ctypes.c_int, ip, ip, ip]
    lib.amrvac_batch_get_job.argtypes = [vp, ctypes.c_int, vp]
    lib.amrvac_batch_remove_job.argtypes = [vp, ctypes.c_int]
    lib.amrvac_batch_free_blocks.argtypes = [vp, ip, ip]
    lib.amrvac_set_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    lib.amrvac_get_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    lib.amrvac_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Tune),
                                    ctypes.POINTER(ctypes.c_float), ip]
    _lib = lib
    return lib


def make_desc(w, precision: int = FP64) -> GridDesc:
    """Grid description of a workload (see paper_2303_03026_amd.inputs.Workload)."""
    g = GridDesc()
    g.ndim, g.block_nx, g.nghost, g.precision = w.ndim, w.nx, w.ng, precision
    for d in range(3):
        g.base_blocks[d] = int(w.base_blocks[d]) if d < w.ndim else 1
        g.bc_lo[d] = int(w.bc_lo[d])
        g.bc_hi[d] = int(w.bc_hi[d])
        g.xmin[d] = float(w.xmin[d])
        g.xmax[d] = float(w.xmax[d])
    g.fix_small_values, g.reflux = int(w.fix_small_values), int(w.reflux)
    g.gamma, g.cfl, g.glm_alpha = w.gamma, w.cfl, w.glm_alpha
    g.small_density, g.small_pressure = w.small_density, w.small_pressure
    fixed = np.ascontiguousarray(np.asarray(w.bc_fixed_prim, dtype=np.float64).reshape(-1))
    for i in range(3 * 2 * NV):
        g.bc_fixed_prim[i] = fixed[i]
    g.limiter = int(getattr(w, "limiter", LIM_VANLEER))
    g.flux = int(getattr(w, "flux", FLUX_HLL))
    return g


def regrid_plan(w, flags, max_level: int = 12, precision: int = FP64, level=None, ijk=None):
    """New leaf set (level, ijk) for workload w's grid from per-block flags:
    > 0 refine, < 0 coarsen (complete sibling sets only), 0 keep; 2:1 nesting
    restored (amrvac_regrid_plan; host only, no device needed)."""
    lib = load_library()
    desc = make_desc(w, precision)
    level = np.ascontiguousarray(w.level if level is None else level, dtype=np.int32).reshape(-1)
    ijk = np.ascontiguousarray(w.ijk if ijk is None else ijk, dtype=np.int32).reshape(-1, 3)
    flags = np.ascontiguousarray(flags, dtype=np.int32).reshape(-1)
    if flags.shape[0] != level.shape[0]:
        raise ValueError("one flag per block")
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))  # noqa: E731
    nb_new = ctypes.c_int()
    # every old leaf ends as at most 2^ndim new ones (one level change per
    # block), so this capacity always suffices and one call does
    cap = len(level) << w.ndim
    lv = np.empty(cap, dtype=np.int32)
    ij = np.empty((cap, 3), dtype=np.int32)
    rc = lib.amrvac_regrid_plan(ctypes.byref(desc), len(level), P(level), P(ijk), P(flags), max_level, cap,
                                ctypes.byref(nb_new), P(lv), P(ij))
    if rc != 0:
        raise AmrvacError(rc, lib.amrvac_last_error(None).decode())
    return lv[:nb_new.value].copy(), ij[:nb_new.value].copy()


class Simulation:
    """One block hierarchy resident on the device, driven through the C ABI.

    Slots are torch uint8 tensors on ``device``; all work goes to one torch
    stream (default priority) that is handed to the library.
    """

    def __init__(self, w, nslots: Optional[int] = None, precision: int = FP64, path: int = PATH_PLAIN,
                 device: str = "cuda", stream=None, set_initial: bool = True):
        import torch
        if nslots is None:  # SSPRK(5,4) steps need a fourth slot
            nslots = 4 if w.nstages == 5 else 3
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the MI355X path has no CPU fallback")
        self.torch = torch
        self.lib = load_library()
        self.w = w
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.desc = make_desc(w, precision)
        self.nb = int(w.level.shape[0])
        size = ctypes.c_size_t()
        self._check(self.lib.amrvac_slot_bytes(ctypes.byref(self.desc), self.nb, ctypes.byref(size)), None)
        self.slot_bytes = size.value
        with torch.cuda.stream(self.stream):
            self.slots = [torch.empty(self.slot_bytes, dtype=torch.uint8, device=self.device)
                          for _ in range(nslots)]
            self.scal = torch.zeros(4, dtype=torch.float64, device=self.device)
        self.level = np.ascontiguousarray(w.level, dtype=np.int32)
        self.ijk = np.ascontiguousarray(w.ijk, dtype=np.int32)
        ptrs = (ctypes.c_void_p * nslots)(*[s.data_ptr() for s in self.slots])
        ctx = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        rc = self.lib.amrvac_init_blocks(
            ctypes.byref(ctx), ctypes.byref(self.desc), self.nb,
            self.level.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            self.ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ptrs, nslots,
            ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise AmrvacError(rc, self.lib.amrvac_last_error(None).decode())
        self.ctx = ctx
        if path != PATH_PLAIN:
            try:
                self.set_path(path)
            except AmrvacError:
                self.close()
                raise
        if set_initial:
            self.set_primitive(w.prim)

    # -- plumbing -------------------------------------------------------------
    def _check(self, rc: int, ctx) -> int:
        if rc != 0:
            msg = self.lib.amrvac_last_error(ctx).decode() if ctx is not None else "invalid argument"
            raise AmrvacError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.amrvac_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dt_ptr(self):
        return ctypes.c_void_p(self.scal.data_ptr())

    @property
    def ch_ptr(self):
        return ctypes.c_void_p(self.scal.data_ptr() + 8)

    @property
    def kappa_ptr(self):
        return ctypes.c_void_p(self.scal.data_ptr() + 16)

    # -- ABI calls ------------------------------------------------------------
    def set_primitive(self, prim: np.ndarray, slot: int = 0):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            t = torch.from_numpy(np.ascontiguousarray(prim, dtype=np.float64)).to(self.device, non_blocking=False)
            self._check(self.lib.amrvac_set_primitive(self.ctx, slot, ctypes.c_void_p(t.data_ptr())), self.ctx)
            self.stream.synchronize()

    def cons(self, slot: int = 0) -> np.ndarray:
        torch = self.torch
        shape = (self.nb, NV) + (self.w.nx,) * self.w.ndim
        with torch.cuda.stream(self.stream):
            t = torch.empty(shape, dtype=torch.float64, device=self.device)
            self._check(self.lib.amrvac_get_conserved(self.ctx, slot, ctypes.c_void_p(t.data_ptr())), self.ctx)
            out = t.cpu().numpy()
        self.stream.synchronize()
        return out

    def padded(self, slot: int = 0) -> np.ndarray:
        """Raw FP64 slot contents, [block][var][padded cells] (test helper)."""
        return self.padded_view(slot).cpu().numpy()

    def padded_view(self, slot: int = 0):
        """Device view of an FP64 slot as [block][var][padded cells] (test
        helper; skips the slot's lead bytes)."""
        pn = self.w.nx + 2 * self.w.ng
        self.stream.synchronize()
        raw = self.slots[slot][slot_lead(self.desc.precision):]
        return raw.view(self.torch.float64).view((self.nb, NV) + (pn,) * self.w.ndim)

    def fill(self, slot: int):
        self._check(self.lib.amrvac_fill_ghosts(self.ctx, slot), self.ctx)

    def cfl(self, slot: int = 0):
        self._check(self.lib.amrvac_cfl_dt(self.ctx, slot, self.dt_ptr, self.ch_ptr, self.kappa_ptr), self.ctx)

    def scalars(self):
        self.stream.synchronize()
        return tuple(self.scal[:3].cpu().tolist())

    def set_scalars(self, dt: float, ch: float, kappa: float):
        with self.torch.cuda.stream(self.stream):
            self.scal[:3] = self.torch.tensor([dt, ch, kappa], dtype=self.torch.float64)
        self.stream.synchronize()

    def stage(self, in_slot: int, base_slot: int, out_slot: int, weight: float, cfl: bool = False):
        """One stage; with cfl=True (amrvac_stage_cfl) the output's CFL rate
        is folded in for the next cfl() on out_slot."""
        fn = self.lib.amrvac_stage_cfl if cfl else self.lib.amrvac_stage
        self._check(fn(self.ctx, in_slot, base_slot, out_slot, weight, self.dt_ptr, self.ch_ptr, self.kappa_ptr),
                    self.ctx)

    def stage_noalloc(self, in_slot: int, base_slot: int, out_slot: int, weight: float):
        """amrvac_stage_noalloc: the per-kernel FP64 stage on the library's
        static device scratch (no allocation)."""
        self._check(self.lib.amrvac_stage_noalloc(self.ctx, in_slot, base_slot, out_slot, weight, self.dt_ptr,
                                                  self.ch_ptr, self.kappa_ptr), self.ctx)

    def combine(self, a_slot: int, b_slot: int, coef: float, out_slot: int):
        """out = a + coef (b - a) on the leaf interior cells (amrvac_combine)."""
        self._check(self.lib.amrvac_combine(self.ctx, a_slot, b_slot, coef, out_slot), self.ctx)

    def lohner(self, weights=(1.0, 0, 0, 0, 0, 0, 0, 0, 0), wavefilter: float = 0.01, slot: int = 0) -> np.ndarray:
        """Loehner's error indicator of every block (amrvac_lohner), weights
        over the conserved variables (default: density only)."""
        torch = self.torch
        wts = np.ascontiguousarray(weights, dtype=np.float64)
        if wts.shape != (NV,):
            raise ValueError("weights must have 9 entries")
        with torch.cuda.stream(self.stream):
            ind = torch.empty(self.nb, dtype=torch.float64, device=self.device)
        self._check(self.lib.amrvac_lohner(self.ctx, slot, wts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           float(wavefilter), ctypes.c_void_p(ind.data_ptr())), self.ctx)
        self.stream.synchronize()
        return ind.cpu().numpy()

    def lohner_flags(self, refine: float = 0.2, coarsen_ratio: float = 0.125, **kw) -> np.ndarray:
        """Per-block regrid flags from the Loehner indicator: 1 above refine,
        -1 below refine * coarsen_ratio, else 0."""
        ind = self.lohner(**kw)
        return np.where(ind > refine, 1, np.where(ind < refine * coarsen_ratio, -1, 0)).astype(np.int32)

    def regrid_plan(self, flags, max_level: int = 12):
        """New leaf set (level, ijk) from per-block flags (see regrid_plan)."""
        return regrid_plan(self.w, flags, max_level, precision=self.desc.precision, level=self.level, ijk=self.ijk)

    def regrid(self, level, ijk, slot: int = 0, nslots: Optional[int] = None) -> "Simulation":
        """A new Simulation on the leaf set (level, ijk) holding the state of
        slot moved over (copied, prolonged or restricted per block;
        amrvac_regrid).  This one stays usable."""
        import dataclasses
        torch = self.torch
        level = np.ascontiguousarray(level, dtype=np.int32).reshape(-1)
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        nslots = len(self.slots) if nslots is None else nslots
        new = Simulation.__new__(Simulation)
        new.torch, new.lib, new.device, new.stream, new.desc = torch, self.lib, self.device, self.stream, self.desc
        new.w = dataclasses.replace(self.w, level=level, ijk=ijk,
                                    prim=np.zeros((len(level), NV) + (self.w.nx,) * self.w.ndim))
        new.nb = len(level)
        size = ctypes.c_size_t()
        self._check(self.lib.amrvac_slot_bytes(ctypes.byref(self.desc), new.nb, ctypes.byref(size)), None)
        new.slot_bytes = size.value
        with torch.cuda.stream(self.stream):
            new.slots = [torch.empty(new.slot_bytes, dtype=torch.uint8, device=self.device) for _ in range(nslots)]
            new.scal = torch.zeros(4, dtype=torch.float64, device=self.device)
        new.level, new.ijk = level, ijk
        ptrs = (ctypes.c_void_p * nslots)(*[t.data_ptr() for t in new.slots])
        ctx = ctypes.c_void_p()
        self._check(self.lib.amrvac_regrid(self.ctx, slot, new.nb, level.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                           ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ptrs, nslots,
                                           ctypes.byref(ctx)), self.ctx)
        new.ctx = ctx
        return new

    def euler_stage(self, in_slot: int = 0, out_slot: int = 1):
        self.fill(in_slot)
        self.stage(in_slot, in_slot, out_slot, 1.0)

    def advance(self, nsteps: int, nstages: Optional[int] = None, graph: bool = False):
        ns = self.w.nstages if nstages is None else nstages
        self._check(self.lib.amrvac_advance(self.ctx, nsteps, ns, 1 if graph else 0), self.ctx)

    def set_path(self, path: int):
        self._check(self.lib.amrvac_set_path(self.ctx, path), self.ctx)

    def sync_flags(self, raise_on_error: bool = True):
        fl = ctypes.c_int()
        nfix = ctypes.c_longlong()
        dt = ctypes.c_double()
        rc = self.lib.amrvac_sync_flags(self.ctx, ctypes.byref(fl), ctypes.byref(nfix), ctypes.byref(dt))
        if rc != 0 and raise_on_error:
            raise AmrvacError(rc, self.lib.amrvac_last_error(self.ctx).decode())
        return fl.value, nfix.value, dt.value, rc

    def reset_flags(self):
        self._check(self.lib.amrvac_reset_flags(self.ctx), self.ctx)

    def set_tune(self, zseg: int, rotate: int, xcd: int):
        t = Tune(zseg, rotate, xcd)
        self._check(self.lib.amrvac_set_tune(self.ctx, ctypes.byref(t)), self.ctx)

    def get_tune(self):
        t = Tune()
        self._check(self.lib.amrvac_get_tune(self.ctx, ctypes.byref(t)), self.ctx)
        return t.as_tuple()

    def autotune(self, in_slot: int = 0, out_slot: int = 1, reps: int = 5, cache: Optional[str] = None):
        """Pick the fused stage's launch shape by timing every candidate on
        this grid (amrvac_autotune) and keep it.  With ``cache`` (a JSON file
        path) a shape measured before for the same grid shape is reused
        without timing, and a new measurement is added to the file.  Returns
        (shape, {candidate: ms per launch}); the times are empty on a hit."""
        key = tune_key(self.w, self.desc.precision)
        if cache is not None:
            hit = _cache_load(cache).get(key)
            if hit is not None:
                self.set_tune(*hit)
                return tuple(hit), {}
        best = Tune()
        ms = (ctypes.c_float * TUNE_MAX_CANDIDATES)()
        n = ctypes.c_int()
        self._check(self.lib.amrvac_autotune(self.ctx, in_slot, out_slot, reps, ctypes.byref(best), ms,
                                             ctypes.byref(n)), self.ctx)
        times = dict(zip(tune_candidates(self.w.ndim), [float(ms[k]) for k in range(n.value)]))
        if cache is not None:
            _cache_store(cache, key, best.as_tuple())
        return best.as_tuple(), times

    def synchronize(self):
        self.stream.synchronize()


def tune_key(w, precision: int) -> str:
    """Autotune cache key: dimension, precision, level count and leaf blocks
    per level (the launch shape's speed depends on these, not on the data)."""
    levels = np.bincount(np.asarray(w.level, dtype=np.int64))[1:]
    return "d%d-p%d-%s" % (w.ndim, precision, ".".join(str(int(n)) for n in levels))


def _cache_load(path: str) -> dict:
    import json
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _cache_store(path: str, key: str, shape) -> None:
    import json
    d = _cache_load(path)
    d[key] = list(shape)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def run(w, nsteps: Optional[int] = None, graph: bool = False, path: int = PATH_PLAIN) -> np.ndarray:
    """Advance a workload on the device and return the interior conserved state."""
    sim = Simulation(w, path=path)
    try:
        sim.advance(w.nsteps if nsteps is None else nsteps, graph=graph)
        sim.sync_flags()
        return sim.cons()
    finally:
        sim.close()


class Batch:
    """A batch (serving) context: a device block pool shared by many jobs of
    one block shape, precision and physics, advanced together."""

    def __init__(self, shape, capacity_blocks: int, max_jobs: int, nstages: int = 3, precision: int = FP64,
                 device: str = "cuda", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the MI355X path has no CPU fallback")
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.shape = shape
        self.desc = make_desc(shape, precision)
        self.precision = precision
        self.capacity = capacity_blocks
        size = ctypes.c_size_t()
        if self.lib.amrvac_slot_bytes(ctypes.byref(self.desc), capacity_blocks, ctypes.byref(size)) != 0:
            raise AmrvacError(E_ARG, "bad batch shape")
        self.block_bytes = (size.value - slot_lead(precision)) // capacity_blocks
        nslots = 4 if nstages >= 5 else (3 if nstages >= 3 else 2)
        with torch.cuda.stream(self.stream):
            self.slots = [torch.empty(size.value, dtype=torch.uint8, device=self.device) for _ in range(nslots)]
        torch.cuda.synchronize(self.device)
        ptrs = (ctypes.c_void_p * nslots)(*[t.data_ptr() for t in self.slots])
        ctx = ctypes.c_void_p()
        rc = self.lib.amrvac_batch_create(ctypes.byref(ctx), ctypes.byref(self.desc), capacity_blocks, max_jobs,
                                          nstages, ptrs, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise AmrvacError(rc, self.lib.amrvac_last_error(None).decode())
        self.ctx = ctx
        self.jobs = {}

    def _err(self, rc):
        raise AmrvacError(rc, self.lib.amrvac_last_error(self.ctx).decode())

    def add_job(self, w, nsteps: Optional[int] = None):
        """Admit workload w; returns the job id, or None when the pool or the
        job table is full (the caller keeps the job queued)."""
        torch = self.torch
        desc = make_desc(w, self.precision)
        level = np.ascontiguousarray(w.level, dtype=np.int32)
        ijk = np.ascontiguousarray(w.ijk, dtype=np.int32)
        jid = ctypes.c_int()
        with torch.cuda.stream(self.stream):
            if isinstance(w.prim, torch.Tensor):
                # pinned host or device tensor: queued on this stream without a
                # host wait
                prim = w.prim.to(self.device, dtype=torch.float64, non_blocking=True)
            else:
                prim = torch.from_numpy(np.ascontiguousarray(w.prim, dtype=np.float64)).to(self.device)
            rc = self.lib.amrvac_batch_add_job(
                self.ctx, ctypes.byref(desc), len(level), level.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.c_void_p(prim.data_ptr()),
                w.nsteps if nsteps is None else nsteps, ctypes.byref(jid))
        if rc == E_NOMEM:
            return None
        if rc != 0:
            self._err(rc)
        self.jobs[jid.value] = (w.nx, w.ndim, len(level))
        return jid.value

    def step(self):
        rc = self.lib.amrvac_batch_step(self.ctx)
        if rc != 0:
            self._err(rc)

    def job_info(self, job: int):
        done, left, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rc = self.lib.amrvac_batch_job_info(self.ctx, job, ctypes.byref(done), ctypes.byref(left), ctypes.byref(nb))
        if rc != 0:
            self._err(rc)
        return done.value, left.value, nb.value

    def get_job(self, job: int) -> np.ndarray:
        torch = self.torch
        nx, ndim, nb = self.jobs[job]
        with torch.cuda.stream(self.stream):
            t = torch.empty((nb, NV) + (nx,) * ndim, dtype=torch.float64, device=self.device)
            rc = self.lib.amrvac_batch_get_job(self.ctx, job, ctypes.c_void_p(t.data_ptr()))
            if rc != 0:
                self._err(rc)
            out = t.cpu().numpy()
        return out

    def remove_job(self, job: int):
        rc = self.lib.amrvac_batch_remove_job(self.ctx, job)
        if rc != 0:
            self._err(rc)
        self.jobs.pop(job, None)

    def set_tune(self, zseg: int, rotate: int, xcd: int):
        t = Tune(zseg, rotate, xcd)
        rc = self.lib.amrvac_set_tune(self.ctx, ctypes.byref(t))
        if rc != 0:
            self._err(rc)

    def get_tune(self):
        t = Tune()
        rc = self.lib.amrvac_get_tune(self.ctx, ctypes.byref(t))
        if rc != 0:
            self._err(rc)
        return t.as_tuple()

    def free_blocks(self):
        big, tot = ctypes.c_int(), ctypes.c_int()
        rc = self.lib.amrvac_batch_free_blocks(self.ctx, ctypes.byref(big), ctypes.byref(tot))
        if rc != 0:
            self._err(rc)
        return big.value, tot.value

    def sync_flags(self, raise_on_error: bool = True):
        fl, nfix, dt = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_double()
        rc = self.lib.amrvac_sync_flags(self.ctx, ctypes.byref(fl), ctypes.byref(nfix), ctypes.byref(dt))
        if rc != 0 and raise_on_error:
            self._err(rc)
        return fl.value, nfix.value, rc

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.amrvac_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
