"""Seeded synthetic inputs: block hierarchies and primitive initial states.

This module is shared by the HIP path and the CPU oracle and therefore holds
none of the scheme's arithmetic: it only lays out leaf blocks and samples
primitive variables (rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi) at cell
centres.  Each side converts primitives to conserved variables itself.

Workloads are shaped like the paper's MHD tests (Orszag-Tang type 2D vortex,
random-mode turbulence, a shock hitting a dense cloud on a static AMR
hierarchy as in the "Shock-cloud in MHD" section, and a thin low-beta current
sheet as in "Divergence control in MHD"); the paper's own data files are not
used, every field is drawn from numpy's PCG64 with a fixed draw order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

NV = 9
RHO, VX, VY, VZ, PR, BX, BY, BZ, PSI = range(NV)
BC_PERIODIC, BC_ZEROGRAD, BC_REFLECT, BC_FIXED = 0, 1, 2, 3


@dataclasses.dataclass
class Workload:
    """A leaf-block hierarchy plus its primitive initial state.

    ``prim`` has shape (nblocks, 9, nx, nx) in 2D ([block][var][j][i]) or
    (nblocks, 9, nx, nx, nx) in 3D ([block][var][k][j][i]); ``level`` is
    1-based and ``ijk`` holds each block's integer position on its level.
    """

    name: str
    ndim: int
    nx: int
    base_blocks: Tuple[int, int, int]
    xmin: Tuple[float, float, float]
    xmax: Tuple[float, float, float]
    bc_lo: Tuple[int, int, int]
    bc_hi: Tuple[int, int, int]
    level: np.ndarray
    ijk: np.ndarray
    prim: np.ndarray
    gamma: float = 5.0 / 3.0
    cfl: float = 0.8
    glm_alpha: float = 0.5
    nstages: int = 3
    nsteps: int = 1
    small_density: float = 0.0
    small_pressure: float = 0.0
    fix_small_values: int = 0
    reflux: int = 1
    ng: int = 2
    limiter: int = 0  # 0 'vanleer', 1 'koren', 2 'cada3'; 3 'weno5', 4 'wenoz5', 5 'mp5', 6 'wenozp5' (these need ng = 3)
    flux: int = 0     # 0 HLL, 1 HLLD, 2 HLLC
    bc_fixed_prim: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((3, 2, NV)))

    @property
    def nblocks(self) -> int:
        return int(self.level.shape[0])

    @property
    def interior_cells(self) -> int:
        return self.nblocks * self.nx ** self.ndim

    @property
    def max_level(self) -> int:
        return int(self.level.max())

    def with_prim(self, prim: np.ndarray, **kw) -> "Workload":
        return dataclasses.replace(self, prim=prim, **kw)


# ---------------------------------------------------------------------------
# geometry helpers


def uniform_blocks(ndim: int, base: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """All level-1 blocks, lexicographic with the x position fastest."""
    nbz = base[2] if ndim == 3 else 1
    ijk = np.array([(i, j, k) for k in range(nbz) for j in range(base[1]) for i in range(base[0])],
                   dtype=np.int32)
    return np.ones(len(ijk), dtype=np.int32), ijk


def cell_centres(ndim: int, nx: int, base: Sequence[int], xmin, xmax,
                 level: np.ndarray, ijk: np.ndarray):
    """Cell-centre coordinates of every interior cell, shaped like one
    variable of ``prim`` (x, y, z arrays)."""
    nb = len(level)
    shape = (nb,) + (nx,) * ndim
    out = []
    for d in range(3):
        if d >= ndim:
            out.append(np.zeros(shape))
            continue
        ncell = (base[d] * nx) * (2.0 ** (level - 1))            # per block
        h = (xmax[d] - xmin[d]) / ncell                          # [nb]
        loc = np.arange(nx) + 0.5
        g = ijk[:, d][:, None] * nx + loc[None, :]               # [nb, nx]
        c = xmin[d] + g * h[:, None]
        # broadcast along the right axis: axis order is [.., k, j, i]
        ax = ndim - d          # position in shape counting from block axis
        view = [nb] + [1] * ndim
        view[ax] = nx
        out.append(np.broadcast_to(c.reshape(view), shape).copy())
    return out


def global_to_blocks(arr: np.ndarray, ndim: int, nx: int) -> np.ndarray:
    """[..., z, y, x] global array on a uniform level-1 grid -> [..., block, k, j, i]
    with lexicographic block order."""
    lead = arr.shape[:-ndim]
    if ndim == 2:
        ny, nxx = arr.shape[-2:]
        a = arr.reshape(lead + (ny // nx, nx, nxx // nx, nx))
        n = len(lead)
        a = a.transpose(tuple(range(n)) + (n, n + 2, n + 1, n + 3))
        return a.reshape(lead + ((ny // nx) * (nxx // nx), nx, nx))
    nz, ny, nxx = arr.shape[-3:]
    a = arr.reshape(lead + (nz // nx, nx, ny // nx, nx, nxx // nx, nx))
    n = len(lead)
    a = a.transpose(tuple(range(n)) + (n, n + 2, n + 4, n + 1, n + 3, n + 5))
    return a.reshape(lead + ((nz // nx) * (ny // nx) * (nxx // nx), nx, nx, nx))


def blocks_to_global(arr: np.ndarray, ndim: int, nx: int, base: Sequence[int]) -> np.ndarray:
    """Inverse of :func:`global_to_blocks` for a uniform level-1 grid."""
    lead = arr.shape[:-(ndim + 1)]
    n = len(lead)
    if ndim == 2:
        a = arr.reshape(lead + (base[1], base[0], nx, nx))
        a = a.transpose(tuple(range(n)) + (n, n + 2, n + 1, n + 3))
        return a.reshape(lead + (base[1] * nx, base[0] * nx))
    a = arr.reshape(lead + (base[2], base[1], base[0], nx, nx, nx))
    a = a.transpose(tuple(range(n)) + (n, n + 3, n + 1, n + 4, n + 2, n + 5))
    return a.reshape(lead + (base[2] * nx, base[1] * nx, base[0] * nx))


# ---------------------------------------------------------------------------
# random divergence-free Fourier mode sums


def _wavevectors(ndim: int, kmax: int) -> np.ndarray:
    r = range(-kmax, kmax + 1)
    out = []
    for kx in r:
        for ky in r:
            for kz in (r if ndim == 3 else [0]):
                k = (kx, ky, kz)
                n2 = kx * kx + ky * ky + kz * kz
                if n2 < 1 or n2 > kmax * kmax:
                    continue
                # half space: first non-zero component positive
                first = next(c for c in k if c != 0)
                if first > 0:
                    out.append(k)
    return np.array(out, dtype=np.int64)


def _mode_draw(rng: np.random.Generator, ndim: int, nmodes: int, kmax: int, vector: bool):
    cand = _wavevectors(ndim, kmax)
    nmodes = min(nmodes, len(cand))   # 2D has only 24 half-plane vectors with |k| <= 4
    ks = cand[rng.choice(len(cand), size=nmodes, replace=False)]
    phases = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    dirs = None
    if vector:
        dirs = np.empty((nmodes, 3))
        for m in range(nmodes):
            k = ks[m].astype(np.float64)
            while True:
                a = rng.normal(size=3)
                a -= (a @ k) / (k @ k) * k
                nrm = np.linalg.norm(a)
                if nrm > 1e-3:
                    break
            dirs[m] = a / nrm
    return ks, phases, dirs


def _mode_sum(n: int, ndim: int, ks: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """Re sum_m coef_m exp(2 pi i k_m . x) at the cell centres of an n^ndim
    periodic unit grid, as a [z][y][x] array (complex matrix product)."""
    x = (np.arange(n) + 0.5) / n
    ax = np.exp(2j * math.pi * np.outer(x, ks[:, 0]))                   # [x, m]
    if ndim == 2:
        by = coef[None, :] * np.exp(2j * math.pi * np.outer(x, ks[:, 1]))  # [y, m]
        return (by @ ax.T).real                                          # [y, x]
    ey = np.exp(2j * math.pi * np.outer(x, ks[:, 1]))                   # [y, m]
    ez = np.exp(2j * math.pi * np.outer(x, ks[:, 2]))                   # [z, m]
    byz = (ez[:, None, :] * ey[None, :, :]).reshape(n * n, -1) * coef[None, :]
    return (byz @ ax.T).real.reshape(n, n, n)


def random_mode_fields(n: int, ndim: int, seed: int, nmodes: int = 32, kmax: int = 4,
                       rho_amp: float = 0.1, v_amp: float = 0.1, b_amp: float = 1.0,
                       b0=(1.0, 0.0, 0.0)) -> np.ndarray:
    """Global [var][z][y][x] primitive arrays of the random-mode state:
    rho = 1 + rho_amp*S, p = 1, divergence-free v and B mode sums with RMS
    v_amp and b_amp, plus a uniform B0; psi = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n,) * ndim
    out = np.zeros((NV,) + shape)
    ks, ph, _ = _mode_draw(rng, ndim, nmodes, kmax, vector=False)
    norm = math.sqrt(2.0 / len(ks))
    out[RHO] = 1.0 + rho_amp * _mode_sum(n, ndim, ks, norm * np.exp(1j * ph))
    out[PR] = 1.0
    ks, ph, dv = _mode_draw(rng, ndim, nmodes, kmax, vector=True)
    for c in range(3):
        out[VX + c] = v_amp * _mode_sum(n, ndim, ks, norm * dv[:, c] * np.exp(1j * ph))
    ks, ph, db = _mode_draw(rng, ndim, nmodes, kmax, vector=True)
    for c in range(3):
        out[BX + c] = b0[c] + b_amp * _mode_sum(n, ndim, ks, norm * db[:, c] * np.exp(1j * ph))
    return out


# ---------------------------------------------------------------------------
# named workloads


def orszag_tang_2d(seed: int = 0, n: int = 64, nx: int = 16, nsteps: int = 100) -> Workload:
    """2D Orszag-Tang type vortex on periodic [0, 2pi]^2 with seeded density
    noise of amplitude 1e-3; SSPRK(2,2), CFL 0.8."""
    gamma = 5.0 / 3.0
    base = (n // nx, n // nx, 1)
    level, ijk = uniform_blocks(2, base)
    L = 2.0 * math.pi
    x, y, _ = cell_centres(2, nx, base, (0, 0, 0), (L, L, 1), level, ijk)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = global_to_blocks(rng.uniform(0.0, 1.0, size=(n, n)), 2, nx)
    prim = np.zeros((len(level), NV, nx, nx))
    prim[:, RHO] = gamma * gamma + 1e-3 * (2.0 * u - 1.0)
    prim[:, VX] = -np.sin(y)
    prim[:, VY] = np.sin(x)
    prim[:, PR] = gamma
    prim[:, BX] = -np.sin(y)
    prim[:, BY] = np.sin(2.0 * x)
    return Workload("orszag_tang_2d_%d" % n, 2, nx, base, (0.0, 0.0, 0.0), (L, L, 1.0),
                    (0, 0, 0), (0, 0, 0), level, ijk, prim, gamma=gamma, nstages=2,
                    nsteps=nsteps)


def random_modes(n: int = 256, ndim: int = 3, seed: int = 1, nx: int = 16, nsteps: int = 50,
                 nstages: int = 3) -> Workload:
    """Periodic unit box with the random-mode state of :func:`random_mode_fields`."""
    base = (n // nx, n // nx, n // nx if ndim == 3 else 1)
    level, ijk = uniform_blocks(ndim, base)
    g = random_mode_fields(n, ndim, seed)
    prim = np.ascontiguousarray(global_to_blocks(g, ndim, nx).swapaxes(0, 1))
    return Workload("random_modes_%dd_%d" % (ndim, n), ndim, nx, base, (0.0, 0.0, 0.0),
                    (1.0, 1.0, 1.0), (0, 0, 0), (0, 0, 0), level, ijk, prim,
                    nstages=nstages, nsteps=nsteps)


def _box_dist(lo, hi, c):
    """min and max distance from point c to the axis-aligned box [lo, hi]."""
    dmin = np.sqrt(sum(np.maximum(0.0, np.maximum(lo[d] - c[d], c[d] - hi[d])) ** 2 for d in range(3)))
    dmax = np.sqrt(sum(np.maximum(np.abs(lo[d] - c[d]), np.abs(hi[d] - c[d])) ** 2 for d in range(3)))
    return dmin, dmax


def nest_2to1(ndim: int, base: Sequence[int], leaves: dict, periodic=(False, False, False)) -> dict:
    """Refine coarse leaves until every leaf's face/edge/corner neighbours are
    at most one level coarser.  ``leaves`` maps (level, i, j, k) -> True."""
    def nblk(l, d):
        return base[d] << (l - 1) if d < ndim else 1

    def covering_leaf(l, p):
        # leaf covering slot p on level l, at level <= l
        q = list(p)
        for m in range(l, 0, -1):
            if (m, q[0], q[1], q[2]) in leaves:
                return (m, q[0], q[1], q[2])
            q = [c >> 1 for c in q]
        return None

    changed = True
    while changed:
        changed = False
        for key in sorted(leaves.keys(), key=lambda t: -t[0]):
            if key not in leaves:
                continue
            l, i, j, k = key
            if l <= 2:
                continue
            offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1)
                    for c in ((-1, 0, 1) if ndim == 3 else (0,)) if (a, b, c) != (0, 0, 0)]
            for o in offs:
                p = [i + o[0], j + o[1], k + o[2]]
                ok = True
                for d in range(ndim):
                    n = nblk(l, d)
                    if p[d] < 0 or p[d] >= n:
                        if periodic[d]:
                            p[d] %= n
                        else:
                            ok = False
                if not ok:
                    continue
                cov = covering_leaf(l, p)
                if cov is not None and cov[0] < l - 1:
                    # refine the too-coarse leaf into its 2^d children
                    del leaves[cov]
                    cl, ci, cj, ck = cov
                    for a in (0, 1):
                        for b in (0, 1):
                            for c in ((0, 1) if ndim == 3 else (0,)):
                                leaves[(cl + 1, 2 * ci + a, 2 * cj + b, 2 * ck + c if ndim == 3 else 0)] = True
                    changed = True
    return leaves


def shock_cloud_amr(seed: int = 2, nsteps: int = 100, nx: int = 16, base_n: int = 128,
                    r_cloud: float = 0.25, r_shell: float = 0.2) -> Workload:
    """3-level static AMR (ratio 2) on a base_n^3 unit cube: level 2 covers a
    seeded sphere of radius r_cloud, level 3 its shell r_shell..r_cloud, with
    2:1 nesting enforced.  A dense cloud (rho = 10) sits in rho = 1, p = 1,
    B = (1, 0, 0); a v_x = 2 inflow enters through the x-min face, the other
    faces are zero-gradient."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.3, 0.7, size=3)
    nb1 = base_n // nx
    base = (nb1, nb1, nb1)
    leaves = {}
    for k in range(nb1):
        for j in range(nb1):
            for i in range(nb1):
                lo = np.array([i, j, k]) / nb1
                hi = lo + 1.0 / nb1
                dmin, _ = _box_dist(lo, hi, c)
                if dmin <= r_cloud:
                    for a in (0, 1):
                        for b in (0, 1):
                            for e in (0, 1):
                                p2 = (2 * i + a, 2 * j + b, 2 * k + e)
                                lo2 = np.array(p2) / (2 * nb1)
                                hi2 = lo2 + 0.5 / nb1
                                dmin2, dmax2 = _box_dist(lo2, hi2, c)
                                if dmin2 <= r_cloud and dmax2 >= r_shell:
                                    for a3 in (0, 1):
                                        for b3 in (0, 1):
                                            for e3 in (0, 1):
                                                leaves[(3, 2 * p2[0] + a3, 2 * p2[1] + b3, 2 * p2[2] + e3)] = True
                                else:
                                    leaves[(2,) + p2] = True
                else:
                    leaves[(1, i, j, k)] = True
    leaves = nest_2to1(3, base, leaves)
    keys = sorted(leaves.keys())
    level = np.array([t[0] for t in keys], dtype=np.int32)
    ijk = np.array([t[1:] for t in keys], dtype=np.int32)
    x, y, z = cell_centres(3, nx, base, (0, 0, 0), (1, 1, 1), level, ijk)
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    prim = np.zeros((len(level), NV, nx, nx, nx))
    prim[:, RHO] = np.where(r <= r_cloud, 10.0, 1.0)
    prim[:, PR] = 1.0
    prim[:, BX] = 1.0
    fixed = np.zeros((3, 2, NV))
    fixed[0, 0, RHO] = 1.0
    fixed[0, 0, VX] = 2.0
    fixed[0, 0, PR] = 1.0
    fixed[0, 0, BX] = 1.0
    return Workload("shock_cloud_amr3", 3, nx, base, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    (BC_FIXED, BC_ZEROGRAD, BC_ZEROGRAD), (BC_ZEROGRAD,) * 3, level, ijk, prim,
                    nstages=3, nsteps=nsteps, bc_fixed_prim=fixed)


def current_sheet(n: int = 192, seed: int = 3, nx: int = 16, nsteps: int = 200,
                  width: float = 0.05) -> Workload:
    """Low-beta (beta = 0.01) Harris-like sheet on [-0.5, 0.5]^3:
    B = (tanh(y/w), 0, sech(y/w)) so |B| = 1 and p + |B|^2/2 is uniform,
    rho = 1, p = 0.005, seeded 1e-2 random velocity per cell and component;
    periodic in x and z, reflective in y."""
    base = (n // nx,) * 3
    level, ijk = uniform_blocks(3, base)
    x, y, z = cell_centres(3, nx, base, (-0.5,) * 3, (0.5,) * 3, level, ijk)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = global_to_blocks(rng.uniform(0.0, 1.0, size=(3, n, n, n)), 3, nx)
    prim = np.zeros((len(level), NV, nx, nx, nx))
    prim[:, RHO] = 1.0
    prim[:, PR] = 0.005
    for c in range(3):
        prim[:, VX + c] = 1e-2 * (2.0 * u[c] - 1.0)
    prim[:, BX] = np.tanh(y / width)
    prim[:, BZ] = 1.0 / np.cosh(y / width)
    return Workload("current_sheet_%d" % n, 3, nx, base, (-0.5,) * 3, (0.5,) * 3,
                    (BC_PERIODIC, BC_REFLECT, BC_PERIODIC), (BC_PERIODIC, BC_REFLECT, BC_PERIODIC),
                    level, ijk, prim, nstages=3, nsteps=nsteps)


# ---------------------------------------------------------------------------
# test problems


def sod(n: int, ndim: int = 2, nx: int = 16, axis: int = 0) -> Workload:
    """Sod shock tube along ``axis`` on [0, 1]: (rho, v, p) = (1, 0, 1) left of
    x = 0.5 and (0.125, 0, 0.1) right, gamma = 1.4, B = 0, zero-gradient ends,
    one block thick and periodic in the other directions."""
    base = [1, 1, 1]
    base[axis] = n // nx
    base = tuple(base)
    level, ijk = uniform_blocks(ndim, base)
    xmax = [1.0, 1.0, 1.0]
    xmax[axis] = 1.0
    xmin = (0.0, 0.0, 0.0)
    cs = cell_centres(ndim, nx, base, xmin, xmax, level, ijk)
    s = cs[axis]
    prim = np.zeros((len(level), NV) + (nx,) * ndim)
    left = s < 0.5
    prim[:, RHO] = np.where(left, 1.0, 0.125)
    prim[:, PR] = np.where(left, 1.0, 0.1)
    lo = [BC_PERIODIC] * 3
    hi = [BC_PERIODIC] * 3
    lo[axis] = BC_ZEROGRAD
    hi[axis] = BC_ZEROGRAD
    return Workload("sod_%d" % n, ndim, nx, base, xmin, tuple(xmax), tuple(lo), tuple(hi),
                    level, ijk, prim, gamma=1.4, nstages=3)


def shu_osher(n: int = 256, nx: int = 16, limiter: int = 6) -> Workload:
    """Shu and Osher's shock / entropy-wave test as the paper runs it: x in
    [-4.5, 4.5], a Mach-3 shock at x = -4 moving right into rho = 1 + 0.2
    sin(5 x), v = 0, p = 1; left state (rho, v, p) = (3.857143, 2.629369,
    10.333333) (the paper prints these rounded to 3.86, 2.63, 10.33);
    gamma = 1.4, B = 0, HLL, SSPRK3, zero-gradient ends, final time 1.8.
    One block thick (periodic) in y; 3 ghost layers for the five-cell
    reconstructions (default 'wenozp5', the paper's choice)."""
    base = (n // nx, 1, 1)
    level, ijk = uniform_blocks(2, base)
    xmin, xmax = (-4.5, 0.0, 0.0), (4.5, 9.0 / n * nx, 1.0)
    x, _, _ = cell_centres(2, nx, base, xmin, xmax, level, ijk)
    prim = np.zeros((len(level), NV, nx, nx))
    left = x < -4.0
    prim[:, RHO] = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    prim[:, VX] = np.where(left, 2.629369, 0.0)
    prim[:, PR] = np.where(left, 10.333333, 1.0)
    return Workload("shu_osher_%d" % n, 2, nx, base, xmin, xmax, (BC_ZEROGRAD, BC_PERIODIC, BC_PERIODIC),
                    (BC_ZEROGRAD, BC_PERIODIC, BC_PERIODIC), level, ijk, prim, gamma=1.4, nstages=3,
                    ng=3 if limiter >= 3 else 2, limiter=limiter, flux=0)


def kelvin_helmholtz(seed: int = 7, base: Tuple[int, int] = (8, 4), nx: int = 16, max_level: int = 1,
                     band: float = 0.05, limiter: int = 6, flux: int = 2, nsteps: int = 10) -> Workload:
    """The paper's 2D hydrodynamic Kelvin-Helmholtz shear layer: (x, y) in
    [-1.5, 1.5] x [-0.75, 0.75], a sharp interface at y = 0 with rho = 1.5,
    v_x = dV / 2.5 above and rho = 1, v_x = -1.5 dV / 2.5 below (dV = 0.2),
    p = 1 / gamma, gamma = 5/3, B = 0, and v_y white noise of amplitude 1e-3
    (uniform in [-1e-3, 1e-3), seeded, one draw per leaf cell in leaf order).
    Base grid base * nx cells (the paper's 128 x 64); blocks whose y-range
    comes within ``band`` of the interface are refined up to ``max_level``
    with 2:1 nesting.  Periodic in x; reflective walls in y.  HLLC with
    'wenozp5' on 3 ghost layers by default, as in the paper's run."""
    b3 = (base[0], base[1], 1)
    xmin, xmax = (-1.5, -0.75, 0.0), (1.5, 0.75, 1.0)
    leaves = {(1, i, j, 0): True for j in range(base[1]) for i in range(base[0])}
    for l in range(1, max_level):
        hy = (xmax[1] - xmin[1]) / (base[1] << (l - 1))
        for key in [k for k in leaves if k[0] == l]:
            y0 = xmin[1] + key[2] * hy
            if y0 - band <= 0.0 <= y0 + hy + band:
                del leaves[key]
                for a in (0, 1):
                    for c in (0, 1):
                        leaves[(l + 1, 2 * key[1] + a, 2 * key[2] + c, 0)] = True
    leaves = nest_2to1(2, b3, leaves, periodic=(True, False, False))
    keys = sorted(leaves.keys(), key=lambda t: (t[0], t[3], t[2], t[1]))  # x fastest within a level
    level = np.array([t[0] for t in keys], dtype=np.int32)
    ijk = np.array([t[1:] for t in keys], dtype=np.int32)
    _, y, _ = cell_centres(2, nx, b3, xmin, xmax, level, ijk)
    rng = np.random.Generator(np.random.PCG64(seed))
    gamma, dv = 5.0 / 3.0, 0.2
    prim = np.zeros((len(level), NV, nx, nx))
    up = y > 0.0
    prim[:, RHO] = np.where(up, 1.5, 1.0)
    prim[:, VX] = np.where(up, dv / 2.5, -1.5 * dv / 2.5)
    prim[:, VY] = 1e-3 * rng.uniform(-1.0, 1.0, size=y.shape)
    prim[:, PR] = 1.0 / gamma
    return Workload("kelvin_helmholtz_%dx%d_l%d" % (base[0] * nx, base[1] * nx, max_level), 2, nx, b3, xmin, xmax,
                    (BC_PERIODIC, BC_REFLECT, BC_PERIODIC), (BC_PERIODIC, BC_REFLECT, BC_PERIODIC), level, ijk,
                    prim, gamma=gamma, nstages=3, nsteps=nsteps, ng=3 if limiter >= 3 else 2, limiter=limiter,
                    flux=flux)


def alfven_shock_states(delta: float = 2.5, beta: float = 0.1, theta_deg: float = 40.0,
                        gamma: float = 5.0 / 3.0):
    """The paper's planar intermediate ('Alfven') shock: upstream at rest with
    rho = 1, p = 1/gamma, plasma beta 2p/B^2 = beta and field (-B cos theta,
    B sin theta); compression ratio delta.  In the shock frame (normal x,
    upstream normal velocity -s) mass, tangential momentum and tangential
    induction give u2 = s (1 - 1/delta), B_y2 = B_y1 (s^2 - v_A^2) /
    (s^2/delta - v_A^2) with v_A^2 = B_x^2 / rho_1, v_2 = B_x (B_y2 - B_y1) /
    (-rho_1 s), and normal momentum gives p_2; the energy jump leaves one
    equation in s, solved by bisection on the intermediate branch v_A^2 <
    s^2 < delta v_A^2 (where B_y changes sign).  Returns (upstream prim,
    downstream prim, shock speed s); the shock moves towards +x."""
    rho1, p1 = 1.0, 1.0 / gamma
    b = math.sqrt(2.0 * p1 / beta)
    th = math.radians(theta_deg)
    bx, b1y = -b * math.cos(th), b * math.sin(th)
    va2 = bx * bx / rho1
    rho2 = delta * rho1

    def downstream(sp):
        j = -rho1 * sp
        w1, w2 = -sp, -sp / delta
        b2y = b1y * (sp * sp - va2) / (sp * sp / delta - va2)
        v2 = bx * (b2y - b1y) / j
        p2 = p1 + rho1 * sp * sp * (1.0 - 1.0 / delta) + 0.5 * (b1y * b1y - b2y * b2y)
        e_in = j * (0.5 * w1 * w1 + gamma * p1 / ((gamma - 1.0) * rho1)) + w1 * b1y * b1y
        e_out = j * (0.5 * (w2 * w2 + v2 * v2) + gamma * p2 / ((gamma - 1.0) * rho2)) + w2 * b2y * b2y - bx * v2 * b2y
        return e_out - e_in, (rho2, sp * (1.0 - 1.0 / delta), v2, p2, b2y)

    lo, hi = math.sqrt(va2) * (1.0 + 1e-9), math.sqrt(delta * va2) * (1.0 - 1e-9)
    grid = np.linspace(lo, hi, 2001)
    f = [downstream(x)[0] for x in grid]
    brackets = [(grid[i], grid[i + 1]) for i in range(len(grid) - 1) if f[i] * f[i + 1] <= 0.0]
    if len(brackets) != 1:
        raise ValueError("no unique intermediate shock for these parameters")
    a, c = brackets[0]
    fa = downstream(a)[0]
    for _ in range(200):
        m = 0.5 * (a + c)
        fm = downstream(m)[0]
        if fm == 0.0 or m in (a, c):
            break
        if (fm < 0.0) == (fa < 0.0):
            a, fa = m, fm
        else:
            c = m
    sp = 0.5 * (a + c)
    r2, u2, v2, p2, b2y = downstream(sp)[1]
    up = np.array([rho1, 0.0, 0.0, 0.0, p1, bx, b1y, 0.0, 0.0])
    down = np.array([r2, u2, v2, 0.0, p2, bx, b2y, 0.0, 0.0])
    return up, down, sp


def alfven_shock_cloud(seed: int = 12, base: Tuple[int, int] = (8, 8), nx: int = 16, max_level: int = 1,
                       limiter: int = 1, flux: int = 0, nsteps: int = 10, cloud: bool = True) -> Workload:
    """The paper's 2D MHD shock-cloud test ("Alfven hits Alfven"): (x, y) in
    [-0.5, 3] x [-1, 2.5], the intermediate shock of alfven_shock_states at
    x = -0.3 moving into the static medium (rho = 1, p = 1/gamma, gamma =
    5/3), whose density in [0, 1] x [0, 1.5] is 1 + 0.5 I(x, y) with I in
    [0, 256].  The paper's I is an image of Alfven; here it is a seeded
    stand-in of the same range: 12 Gaussian blobs (centres uniform in the
    rectangle, widths 0.03 .. 0.15, amplitudes 0.3 .. 1), their sum clipped
    to 1 and scaled by 256.  Zero-gradient boundaries; SSPRK3 with 'koren'
    by default.  Base grid base * nx cells (the paper's 128^2); blocks that
    meet the cloud rectangle or the shock are refined up to ``max_level``
    with 2:1 nesting."""
    b3 = (base[0], base[1], 1)
    xmin, xmax = (-0.5, -1.0, 0.0), (3.0, 2.5, 1.0)
    leaves = {(1, i, j, 0): True for j in range(base[1]) for i in range(base[0])}
    for l in range(1, max_level):
        hx = (xmax[0] - xmin[0]) / (base[0] << (l - 1))
        hy = (xmax[1] - xmin[1]) / (base[1] << (l - 1))
        for key in [k for k in leaves if k[0] == l]:
            x0, y0 = xmin[0] + key[1] * hx, xmin[1] + key[2] * hy
            meets_cloud = cloud and x0 <= 1.0 and x0 + hx >= 0.0 and y0 <= 1.5 and y0 + hy >= 0.0
            meets_shock = x0 <= -0.3 <= x0 + hx
            if meets_cloud or meets_shock:
                del leaves[key]
                for a in (0, 1):
                    for c in (0, 1):
                        leaves[(l + 1, 2 * key[1] + a, 2 * key[2] + c, 0)] = True
    leaves = nest_2to1(2, b3, leaves)
    keys = sorted(leaves.keys(), key=lambda t: (t[0], t[3], t[2], t[1]))  # x fastest within a level
    level = np.array([t[0] for t in keys], dtype=np.int32)
    ijk = np.array([t[1:] for t in keys], dtype=np.int32)
    x, y, _ = cell_centres(2, nx, b3, xmin, xmax, level, ijk)
    up, down, _ = alfven_shock_states()
    prim = np.zeros((len(level), NV, nx, nx))
    post = x < -0.3
    for q in range(NV):
        prim[:, q] = np.where(post, down[q], up[q])
    if cloud:
        rng = np.random.Generator(np.random.PCG64(seed))
        img = np.zeros_like(x)
        for _ in range(12):
            cx, cy = rng.uniform(0.0, 1.0), rng.uniform(0.0, 1.5)
            wdt, amp = rng.uniform(0.03, 0.15), rng.uniform(0.3, 1.0)
            img += amp * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * wdt * wdt))
        inside = (x >= 0.0) & (x <= 1.0) & (y >= 0.0) & (y <= 1.5)
        prim[:, RHO] = np.where(inside, 1.0 + 0.5 * 256.0 * np.minimum(img, 1.0), prim[:, RHO])
    zg = (BC_ZEROGRAD, BC_ZEROGRAD, BC_PERIODIC)
    return Workload("alfven_shock_cloud_%dx%d_l%d" % (base[0] * nx, base[1] * nx, max_level), 2, nx, b3, xmin, xmax,
                    zg, zg, level, ijk, prim, gamma=5.0 / 3.0, nstages=3, nsteps=nsteps, limiter=limiter, flux=flux)


def alfven_wave(n: int, ndim: int = 2, nx: int = 16, amp: float = 1e-6) -> Workload:
    """Small-amplitude linear Alfven wave on the periodic unit box with
    k = 2 pi (1, 1[, 1]), rho = 1, p = 1, B0 = unit vector along k, and a
    transverse perturbation dB = amp*sin(k.x) e_perp, dv = -dB (propagating
    along +k at the Alfven speed 1).  e_perp = z in 2D, (1, -1, 0)/sqrt 2 in 3D."""
    base = (n // nx, n // nx, n // nx if ndim == 3 else 1)
    level, ijk = uniform_blocks(ndim, base)
    x, y, z = cell_centres(ndim, nx, base, (0, 0, 0), (1, 1, 1), level, ijk)
    if ndim == 2:
        kvec = np.array([1.0, 1.0, 0.0])
        eperp = np.array([0.0, 0.0, 1.0])
        phase = 2.0 * math.pi * (x + y)
    else:
        kvec = np.array([1.0, 1.0, 1.0])
        eperp = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
        phase = 2.0 * math.pi * (x + y + z)
    khat = kvec / np.linalg.norm(kvec)
    prim = np.zeros((len(level), NV) + (nx,) * ndim)
    prim[:, RHO] = 1.0
    prim[:, PR] = 1.0
    db = amp * np.sin(phase)
    for c in range(3):
        prim[:, BX + c] = khat[c] + db * eperp[c]
        prim[:, VX + c] = -db * eperp[c]
    return Workload("alfven_%dd_%d" % (ndim, n), ndim, nx, base, (0.0,) * 3, (1.0,) * 3,
                    (0, 0, 0), (0, 0, 0), level, ijk, prim, nstages=3)


def uniform_state(ndim: int, base: Sequence[int], w: Sequence[float], nx: int = 16,
                  bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), level=None, ijk=None) -> Workload:
    """A constant primitive state ``w`` (9 values) on the given blocks."""
    if level is None:
        level, ijk = uniform_blocks(ndim, base)
    prim = np.empty((len(level), NV) + (nx,) * ndim)
    for q in range(NV):
        prim[:, q] = w[q]
    return Workload("uniform", ndim, nx, tuple(base), (0.0,) * 3, (1.0,) * 3, tuple(bc_lo),
                    tuple(bc_hi), level, ijk, prim)


def amr_test_hierarchy(ndim: int = 2, nb1: int = 4, seed: int = 5, nx: int = 16,
                       periodic: bool = True):
    """Small 3-level hierarchy for tests: refine a seeded subset of base blocks,
    refine a seeded subset of their children, then enforce 2:1 nesting."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = (nb1, nb1, nb1 if ndim == 3 else 1)
    leaves = {}
    coords = [(i, j, k) for k in range(base[2]) for j in range(nb1) for i in range(nb1)]
    ref1 = set(tuple(c) for c in np.array(coords)[rng.random(len(coords)) < 0.35].tolist())
    for c in coords:
        if c in ref1:
            kids = [(2 * c[0] + a, 2 * c[1] + b, 2 * c[2] + e) for e in ((0, 1) if ndim == 3 else (0,))
                    for b in (0, 1) for a in (0, 1)]
            for kd in kids:
                if rng.random() < 0.3:
                    for e in ((0, 1) if ndim == 3 else (0,)):
                        for b in (0, 1):
                            for a in (0, 1):
                                leaves[(3, 2 * kd[0] + a, 2 * kd[1] + b, 2 * kd[2] + e if ndim == 3 else 0)] = True
                else:
                    leaves[(2,) + kd] = True
        else:
            leaves[(1,) + c] = True
    leaves = nest_2to1(ndim, base, leaves, periodic=(periodic,) * 3)
    keys = sorted(leaves.keys())
    level = np.array([t[0] for t in keys], dtype=np.int32)
    ijk = np.array([t[1:] for t in keys], dtype=np.int32)
    return base, level, ijk


def smooth_amr_state(ndim: int = 2, nb1: int = 4, seed: int = 5, nx: int = 16) -> Workload:
    """A smooth periodic MHD state on :func:`amr_test_hierarchy` (used for AMR
    conservation and parity tests)."""
    base, level, ijk = amr_test_hierarchy(ndim, nb1, seed, nx)
    x, y, z = cell_centres(ndim, nx, base, (0, 0, 0), (1, 1, 1), level, ijk)
    tp = 2.0 * math.pi
    prim = np.zeros((len(level), NV) + (nx,) * ndim)
    prim[:, RHO] = 1.0 + 0.3 * np.sin(tp * x) * np.cos(tp * y) + (0.1 * np.sin(tp * z) if ndim == 3 else 0.0)
    prim[:, VX] = 0.5 * np.sin(tp * y)
    prim[:, VY] = -0.4 * np.sin(tp * x)
    prim[:, VZ] = 0.2 * np.cos(tp * (x + y))
    prim[:, PR] = 1.0 + 0.2 * np.cos(tp * x)
    prim[:, BX] = 0.8 - 0.3 * np.sin(tp * y)
    prim[:, BY] = 0.4 * np.sin(tp * x)
    prim[:, BZ] = 0.3 * np.cos(tp * x) + (0.2 * np.sin(tp * y) if ndim == 3 else 0.0)
    prim[:, PSI] = 0.01 * np.sin(tp * (x - y))
    return Workload("smooth_amr_%dd" % ndim, ndim, nx, base, (0.0,) * 3, (1.0,) * 3,
                    (0, 0, 0), (0, 0, 0), level, ijk, prim, nstages=3)


def serving_jobs(njobs: int = 2000, seed: int = 4, rate: float = 1.0) -> list:
    """Job descriptors of the serving stream: Poisson arrival times (mean gap
    1/rate), 2D/3D with equal odds, log-uniform linear size rounded to 16
    (2D 32..256, 3D 32..128), steps uniform in 20..500, FP32-mixed or FP64
    with equal odds, and a per-job field seed.  Fields are built on demand
    with :func:`serving_job_workload`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for jid in range(njobs):
        t += rng.exponential(1.0 / rate)
        ndim = 2 if rng.random() < 0.5 else 3
        lo, hi = (32, 256) if ndim == 2 else (32, 128)
        n = int(16 * round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 16.0))
        n = max(lo, min(hi, n))
        steps = int(rng.integers(20, 501))
        mixed = bool(rng.random() < 0.5)
        jobs.append(dict(id=jid, arrival=t, ndim=ndim, n=n, steps=steps, mixed=mixed,
                         seed=int(rng.integers(0, 2 ** 31 - 1))))
    return jobs


def serving_job_workload(job: dict) -> Workload:
    w = random_modes(job["n"], job["ndim"], seed=job["seed"], nsteps=job["steps"])
    w.name = "job%d" % job["id"]
    return w
