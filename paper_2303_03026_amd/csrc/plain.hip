// Plain (one kernel per phase) FP64 path: ghost filling, conserved ->
// primitive, per-direction reconstruction + GLM + HLL face fluxes, coarse/fine
// flux correction, flux-difference update with the SSPRK combination, and the
// CFL reduction.
//
// Storage: block-major slots [block][var][padded cell], padded index
// ((k+ng)*pn + (j+ng))*pn + (i+ng) (2D drops k).  Face fluxes per direction
// are [block][var][face cell] with the face coordinate along the direction
// (extent nx+1) and x the fastest index:
//   x faces: (k*nx + j)*(nx+1) + f,  y faces: (k*(nx+1) + f)*nx + i,
//   z faces: (f*nx + j)*nx + i.
#include "kernels.h"

namespace amrvac {

namespace {

__device__ __forceinline__ long pidx(const GridConst& G, int i, int j, int k) {
  const int kk = G.ndim == 3 ? k + G.ng : 0;
  return ((long)kk * G.pn + (j + G.ng)) * G.pn + (i + G.ng);
}

// ---------------------------------------------------------------------------
// ghost filling: one thread per ghost cell of a (block, face) task
//
// Every load a ghost cell needs is issued before any of its stores.  Sources
// and destination lie in the same slot, so a store the compiler cannot tell
// apart from the loads after it would cost one memory round trip per
// variable.

template <int NDIM>
__device__ __forceinline__ long pidx_n(const GridConst& G, int i, int j, int k) {
  const int kk = NDIM == 3 ? k + G.ng : 0;
  return ((long)kk * G.pn + (j + G.ng)) * G.pn + (i + G.ng);
}

// UNI: a task's ghost cells are a multiple of 64, so each wave lies in one
// task and its block, face, links and positions are wave-uniform (scalar
// loads, no divergence between the kinds of task).
template <int NDIM, class SP, bool UNI>
__global__ void __launch_bounds__(256) k_fill_faces(GridConst G, const int* __restrict__ tasks, int ntasks, Tables T,
                                                   void* __restrict__ slot, PhysConst P, FixedBC fixed) {
  const int* __restrict__ link = T.link;
  const int nx = G.nx, ng = G.ng;
  const int ncell = NDIM == 3 ? ng * nx * nx : ng * nx;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)ntasks * ncell) return;
  int task = (int)(gid / ncell);
  if (UNI) task = __builtin_amdgcn_readfirstlane(task);
  const int t = (int)(gid - (long)task * ncell);
  const int b = tasks[2 * task];
  const int face = tasks[2 * task + 1];
  const int d = face >> 1, side = face & 1;
  const int* L = link + ((long)b * 6 + face) * LINK_INTS;
  const int kind = L[0];
  const int ta = d == 0 ? 1 : 0;  // first transverse axis
  const int tb = d == 2 ? 1 : 2;  // second transverse axis (z in 2D: unused)
  const long pc = G.pcells;
  void* dst = block_ptr<SP>(slot, b, pc);

  int a, t1, t2;
  if (d == 0) {
    a = t % ng;
    t1 = (t / ng) % nx;
    t2 = t / (ng * nx);
  } else {
    t1 = t % nx;
    a = (t / nx) % ng;
    t2 = t / (nx * ng);
  }
  const int gd = side ? nx + a : a - ng;  // ghost coordinate along d
  int c[3] = {0, 0, 0};
  c[d] = gd;
  c[ta] = t1;
  if (NDIM == 3) c[tb] = t2;
  const long di = pidx_n<NDIM>(G, c[0], c[1], c[2]);

  double out[NV];
  if (kind == LINK_SAME) {
    const void* src = block_ptr<SP>(slot, L[1], pc);
    int s[3] = {c[0], c[1], c[2]};
    s[d] = side ? gd - nx : gd + nx;
    const long si = pidx_n<NDIM>(G, s[0], s[1], s[2]);
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = SP::ld(src, q, si, pc);
  } else if (kind == LINK_FINE) {
    // restriction: fine cells under this coarse ghost cell, all in one fine
    // leaf (chosen by the transverse half)
    int fc[3] = {0, 0, 0};
    fc[d] = side ? 2 * gd - 2 * nx : 2 * gd + nx;
    const int oa = (2 * c[ta]) >= nx ? 1 : 0;
    fc[ta] = 2 * c[ta] - oa * nx;
    int ob = 0;
    if (NDIM == 3) {
      ob = (2 * c[tb]) >= nx ? 1 : 0;
      fc[tb] = 2 * c[tb] - ob * nx;
    }
    const void* src = block_ptr<SP>(slot, L[1 + ob * 2 + oa], pc);
    if (NDIM == 2) {
      const long i00 = pidx_n<2>(G, fc[0], fc[1], 0), i10 = pidx_n<2>(G, fc[0] + 1, fc[1], 0);
      const long i01 = pidx_n<2>(G, fc[0], fc[1] + 1, 0), i11 = pidx_n<2>(G, fc[0] + 1, fc[1] + 1, 0);
#pragma unroll
      for (int q = 0; q < NV; ++q)
        out[q] = ((SP::ld(src, q, i00, pc) + SP::ld(src, q, i10, pc)) +
                  (SP::ld(src, q, i01, pc) + SP::ld(src, q, i11, pc))) * 0.25;
    } else {
      // the 2x2x2 fine cells are two x-pairs in each of two z planes
      const long i000 = pidx_n<3>(G, fc[0], fc[1], fc[2]);
      const long sy = G.pn, sz = (long)G.pn * G.pn;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        auto v = [&](int e, int bb, int aa) { return SP::ld(src, q, i000 + e * sz + bb * sy + aa, pc); };
        out[q] = (((v(0, 0, 0) + v(0, 0, 1)) + (v(0, 1, 0) + v(0, 1, 1))) +
                  ((v(1, 0, 0) + v(1, 0, 1)) + (v(1, 1, 0) + v(1, 1, 1)))) * 0.125;
      }
    }
  } else if (kind == LINK_PHYS) {
    const int bc = L[1];
    if (bc == 3) {  // fixed inflow state
      double w[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) w[q] = fixed.prim[d][side][q];
      prim_to_cons(w, out, P);
    } else {
      int s[3] = {c[0], c[1], c[2]};
      if (bc == 1)
        s[d] = side ? nx - 1 : 0;
      else
        s[d] = side ? 2 * nx - 1 - gd : -1 - gd;
      const long si = pidx_n<NDIM>(G, s[0], s[1], s[2]);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double v = SP::ld(dst, q, si, pc);
        out[q] = (bc == 2 && (q == I_MX + d || q == I_BX + d)) ? -v : v;
      }
    }
  } else {
    return;  // faces towards coarser leaves: k_prolong_faces
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) SP::st(dst, q, di, pc, out[q]);
}

// Prolongation of the ghost cells of faces towards coarser leaves (the
// COARSE tasks of k_fill_faces, same arithmetic): one thread per (fine
// ghost layer, coarse cell across the face), writing the 2^(d-1) fine ghost
// cells of that layer over the coarse cell, so the coarse cell and its
// slope neighbours are read once for all of them.  Threads per task:
// ng (nx/2)^(d-1).
template <int NDIM, class SP, bool UNI>
__global__ void __launch_bounds__(256) k_prolong_faces(GridConst G, const int* __restrict__ tasks, int ntasks,
                                                      Tables T, void* __restrict__ slot) {
  const int* __restrict__ link = T.link;
  const int* __restrict__ pos = T.pos;
  const int nx = G.nx, ng = G.ng, hx = nx / 2;
  const int ncell = NDIM == 3 ? ng * hx * hx : ng * hx;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)ntasks * ncell) return;
  int task = (int)(gid / ncell);
  if (UNI) task = __builtin_amdgcn_readfirstlane(task);
  const int t = (int)(gid - (long)task * ncell);
  const int b = tasks[2 * task];
  const int face = tasks[2 * task + 1];
  const int d = face >> 1, side = face & 1;
  const int* L = link + ((long)b * 6 + face) * LINK_INTS;
  const int ta = d == 0 ? 1 : 0;  // first transverse axis
  const int tb = d == 2 ? 1 : 2;  // second transverse axis (z in 2D: unused)
  const long pc = G.pcells;
  void* dst = block_ptr<SP>(slot, b, pc);
  // fine ghost layer a along d, coarse transverse indices c1 (along ta), c2
  const int a = t % ng, c1 = (t / ng) % hx, c2 = NDIM == 3 ? t / (ng * hx) : 0;
  const int gd = side ? nx + a : a - ng;  // ghost coordinate along d
  int c[3] = {0, 0, 0};  // the first of the fine cells (even transverse offsets)
  c[d] = gd;
  c[ta] = 2 * c1;
  if (NDIM == 3) c[tb] = 2 * c2;
  const int cb = L[1];
  const void* src = block_ptr<SP>(slot, cb, pc);
  int lc[3] = {0, 0, 0};
  int odd_d = 0;
#pragma unroll
  for (int ax = 0; ax < NDIM; ++ax) {
    const long n = T.wrap[3 * b + ax];
    long g = (long)pos[3 * b + ax] * nx + c[ax];
    g = (g + n) % n;
    if (ax == d) odd_d = (int)(g & 1);
    lc[ax] = (int)((g >> 1) - (long)pos[3 * cb + ax] * nx);
  }
  // slope neighbours of lc as in k_fill_faces: in place across same-level
  // faces of cb, else cb's own ghost cells (filled before this pass)
  const long i0 = pidx_n<NDIM>(G, lc[0], lc[1], lc[2]);
  int lk[2 * NDIM], ln[2 * NDIM];
#pragma unroll
  for (int f = 0; f < 2 * NDIM; ++f) {
    lk[f] = link[((long)cb * 6 + f) * LINK_INTS];
    ln[f] = link[((long)cb * 6 + f) * LINK_INTS + 1];
  }
  int bm[3], bp[3];
  long im[3], ip[3];
#pragma unroll
  for (int ax = 0; ax < NDIM; ++ax) {
    int m[3] = {lc[0], lc[1], lc[2]}, p[3] = {lc[0], lc[1], lc[2]};
    m[ax] -= 1;
    p[ax] += 1;
    bm[ax] = cb;
    bp[ax] = cb;
    if (m[ax] < 0 && lk[2 * ax] == LINK_SAME) {
      bm[ax] = ln[2 * ax];
      m[ax] += nx;
    }
    if (p[ax] >= nx && lk[2 * ax + 1] == LINK_SAME) {
      bp[ax] = ln[2 * ax + 1];
      p[ax] -= nx;
    }
    im[ax] = pidx_n<NDIM>(G, m[0], m[1], m[2]);
    ip[ax] = pidx_n<NDIM>(G, p[0], p[1], p[2]);
  }
  // fine cell k: offsets (k & 1) along ta and (k >> 1) along tb; its parity
  // along a transverse axis is its offset (the block's first cell sits at an
  // even global index), along d that of its ghost coordinate
  constexpr int NF = NDIM == 3 ? 4 : 2;
  long di[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    int f3[3] = {c[0], c[1], c[2]};
    f3[ta] += k & 1;
    if (NDIM == 3) f3[tb] += k >> 1;
    di[k] = pidx_n<NDIM>(G, f3[0], f3[1], f3[2]);
  }
  // every load before the first store (sources and destination share the
  // slot)
  double uc[NV], sl[NV][3];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    uc[q] = SP::ld(src, q, i0, pc);
#pragma unroll
    for (int ax = 0; ax < NDIM; ++ax) {
      const double um = SP::ld(block_ptr<SP>(static_cast<const void*>(slot), bm[ax], pc), q, im[ax], pc);
      const double up = SP::ld(block_ptr<SP>(static_cast<const void*>(slot), bp[ax], pc), q, ip[ax], pc);
      sl[q][ax] = minmod2(uc[q] - um, up - uc[q]);
    }
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double r = uc[q];
#pragma unroll
      for (int ax = 0; ax < NDIM; ++ax) {
        const int odd = ax == d ? odd_d : (ax == ta ? (k & 1) : (k >> 1));
        const double sg = odd ? 0.25 : -0.25;
        r = r + sg * sl[q][ax];
      }
      SP::st(dst, q, di[k], pc, r);
    }
  }
}

// ---------------------------------------------------------------------------
// conserved -> primitive on interior + face ghost cells

__global__ void __launch_bounds__(256) k_prim(GridConst G, const double* __restrict__ slot, double* __restrict__ prim,
                                             PhysConst P, DevStatus* st) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)G.nb * G.pcells;
  if (gid >= total) return;
  const int b = (int)(gid / G.pcells);
  const long c = gid - (long)b * G.pcells;
  const int i = (int)(c % G.pn) - G.ng;
  const int j = (int)((c / G.pn) % G.pn) - G.ng;
  const int k = G.ndim == 3 ? (int)(c / ((long)G.pn * G.pn)) - G.ng : 0;
  const int outside = (i < 0 || i >= G.nx) + (j < 0 || j >= G.nx) + (G.ndim == 3 && (k < 0 || k >= G.nx));
  if (outside > 1) return;
  const double* u0 = slot + (long)b * NV * G.pcells + c;
  double u[NV], w[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) u[q] = u0[q * G.pcells];
  const int bad = cons_to_prim(u, w, P);
  double* w0 = prim + (long)b * NV * G.pcells + c;
#pragma unroll
  for (int q = 0; q < NV; ++q) w0[q * G.pcells] = w[q];
  if (bad) {
    atomicOr(&st->flags, (unsigned)bad);
    if (P.fix) atomicAdd(&st->nfix, 1ull);
  }
}

// ---------------------------------------------------------------------------
// face fluxes along D: one thread per face

template <int D>
__global__ void __launch_bounds__(256) k_flux(GridConst G, const double* __restrict__ prim, double* __restrict__ flux,
                                             const double* __restrict__ ch_dev, PhysConst P,
                                             const double* __restrict__ inv_dx) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)G.nb * G.nfaces;
  if (gid >= total) return;
  const int b = (int)(gid / G.nfaces);
  const int fi = (int)(gid - (long)b * G.nfaces);
  const int nx = G.nx, n1 = nx + 1;
  int i, j, k, f;
  if (D == 0) {
    f = fi % n1;
    j = (fi / n1) % nx;
    k = fi / (n1 * nx);
    i = 0;
  } else if (D == 1) {
    i = fi % nx;
    f = (fi / nx) % n1;
    k = fi / (nx * n1);
    j = 0;
  } else {
    i = fi % nx;
    j = (fi / nx) % nx;
    f = fi / (nx * nx);
    k = 0;
  }
  const double* base = prim + (long)b * NV * G.pcells;
  double wl[NV], wr[NV], F[NV];
  if (G.ng == 3) {  // six-cell stencil f-3 .. f+2
    double c6[6][NV];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int a = f - 3 + s;
      const long ix = D == 0 ? pidx(G, a, j, k) : (D == 1 ? pidx(G, i, a, k) : pidx(G, i, j, a));
#pragma unroll
      for (int q = 0; q < NV; ++q) c6[s][q] = base[q * G.pcells + ix];
    }
    // WENO-Z+'s lambda = dx^(2/3) of this block along D
    const double lambda = P.limiter == LIM_WENOZP5 ? 1.0 / cbrt(inv_dx[3 * b + D] * inv_dx[3 * b + D]) : 0.0;
    reconstruct_face6(P.limiter, c6, lambda, wl, wr);
  } else {
    double wm[NV], wa[NV], wb[NV], wp[NV];
    long idx[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int a = f - 2 + s;
      idx[s] = D == 0 ? pidx(G, a, j, k) : (D == 1 ? pidx(G, i, a, k) : pidx(G, i, j, a));
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double* p = base + q * G.pcells;
      wm[q] = p[idx[0]];
      wa[q] = p[idx[1]];
      wb[q] = p[idx[2]];
      wp[q] = p[idx[3]];
    }
    reconstruct_face(P.limiter, wm, wa, wb, wp, wl, wr);
  }
  const double ch = *ch_dev;
  face_flux_rt<D, double>(P.flux, wl, wr, ch, 0.5 / ch, P.gamma, P.inv_gm1, F);
  double* out = flux + (long)b * NV * G.nfaces + fi;
#pragma unroll
  for (int q = 0; q < NV; ++q) out[(long)q * G.nfaces] = F[q];
}

__device__ __forceinline__ int face_index(const GridConst& G, int d, int f, int t1, int t2) {
  // t1/t2: the transverse coordinates in axis order (x before y before z)
  const int nx = G.nx, n1 = nx + 1;
  if (d == 0) return (t2 * nx + t1) * n1 + f;   // t1 = j, t2 = k
  if (d == 1) return (t2 * n1 + f) * nx + t1;   // t1 = i, t2 = k
  return (f * nx + t2) * nx + t1;               // t1 = i, t2 = j
}

// coarse/fine flux correction: one thread per coarse boundary face cell
__global__ void __launch_bounds__(256) k_reflux(GridConst G, const int* __restrict__ tasks, int ntasks,
                                               const int* __restrict__ link, FluxPtrs flux) {
  const int nx = G.nx;
  const int per = G.ndim == 3 ? nx * nx : nx;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)ntasks * per) return;
  const int task = (int)(gid / per);
  const int t = (int)(gid - (long)task * per);
  const int b = tasks[2 * task], face = tasks[2 * task + 1];
  const int d = face >> 1, side = face & 1;
  const int* L = link + ((long)b * 6 + face) * LINK_INTS;
  const int t1 = t % nx, t2 = G.ndim == 3 ? t / nx : 0;
  const int ff = side ? 0 : nx;  // fine face along d
  const int cf = side ? nx : 0;  // coarse face along d
  double* F = flux.f[d];
  double acc[NV];
  double v[2][2][NV];
  const int ne = G.ndim == 3 ? 2 : 1;
  // (unrolled: a run-time index into v would place it in scratch memory)
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (e >= ne) continue;
      const int g1 = 2 * t1 + a, g2 = 2 * t2 + e;
      const int o1 = g1 >= nx ? 1 : 0, o2 = g2 >= nx ? 1 : 0;
      const int fb = L[1 + (G.ndim == 3 ? o2 * 2 : 0) + o1];
      const int fidx = face_index(G, d, ff, g1 - o1 * nx, G.ndim == 3 ? g2 - o2 * nx : 0);
      const double* src = F + (long)fb * NV * G.nfaces + fidx;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[e][a][q] = src[(long)q * G.nfaces];
    }
#pragma unroll
  for (int q = 0; q < NV; ++q)
    acc[q] = G.ndim == 3 ? ((v[0][0][q] + v[0][1][q]) + (v[1][0][q] + v[1][1][q])) * 0.25
                         : (v[0][0][q] + v[0][1][q]) * 0.5;
  double* dst = F + (long)b * NV * G.nfaces + face_index(G, d, cf, t1, t2);
#pragma unroll
  for (int q = 0; q < NV; ++q) dst[(long)q * G.nfaces] = acc[q];
}

// flux-difference update + SSPRK combination: one thread per interior cell
__global__ void __launch_bounds__(256) k_update(GridConst G, Tables T, const double* __restrict__ in,
                                               const double* base,
                                               double* out, double w, FluxPtrs flux,
                                               const double* __restrict__ dt_dev, double dt_scale,
                                               const double* __restrict__ kappa_dev) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)G.nb * G.icells;
  if (gid >= total) return;
  const int b = (int)(gid / G.icells);
  const int c = (int)(gid - (long)b * G.icells);
  const int nx = G.nx;
  const int i = c % nx, j = (c / nx) % nx, k = G.ndim == 3 ? c / (nx * nx) : 0;
  const long pc = pidx(G, i, j, k);
  const double dt = dt_scale * *dt_dev, kappa = *kappa_dev;
  double L[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) L[q] = 0.0;
  for (int d = 0; d < G.ndim; ++d) {
    int f, t1, t2;
    if (d == 0) { f = i; t1 = j; t2 = k; }
    else if (d == 1) { f = j; t1 = i; t2 = k; }
    else { f = k; t1 = i; t2 = j; }
    const double* F = flux.f[d] + (long)b * NV * G.nfaces;
    const int lo = face_index(G, d, f, t1, t2), hi = face_index(G, d, f + 1, t1, t2);
    const double idx = T.inv_dx[3 * b + d];
#pragma unroll
    for (int q = 0; q < NV; ++q) L[q] = L[q] + (F[(long)q * G.nfaces + hi] - F[(long)q * G.nfaces + lo]) * idx;
  }
  const double* u = in + (long)b * NV * G.pcells + pc;
  double* o = out + (long)b * NV * G.pcells + pc;
  const double psi = u[I_PSI * G.pcells];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double lq = -L[q];
    if (q == I_PSI) lq = lq - kappa * psi;
    const double t = u[q * G.pcells] + dt * lq;
    if (w == 1.0) {
      o[q * G.pcells] = t;
    } else {
      const double u0 = base[(long)b * NV * G.pcells + pc + q * G.pcells];
      o[q * G.pcells] = u0 + w * (t - u0);
    }
  }
}

// Flux correction after a fused stage, direction D only (so no two tasks
// touch one cell): for each coarse cell next to finer leaves, replace the
// coarse face flux the stage used with the pairwise mean of the fine face
// fluxes, i.e. out += w*dt*dL.  The fluxes come from the flux registers the
// fused stage filled as it evaluated those faces: one thread per (task,
// coarse face cell) reads the coarse face flux and the fluxes of the
// 2^(d-1) fine faces behind it (those fine blocks' registers on the
// opposite face).
template <int D, class SP, int NFINE>
__global__ void __launch_bounds__(256) k_reflux_apply(GridConst G, Tables T, JobScalars J,
                                                     const int* __restrict__ tasks, int ntasks,
                                                     const typename SP::R* __restrict__ freg, void* out, double w) {
  using R = typename SP::R;
  const int* __restrict__ link = T.link;
  const int nx = G.nx;
  const int nfc = G.ndim == 3 ? nx * nx : nx;  // face cells per register
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)ntasks * nfc) return;
  const int task = (int)(gid / nfc);
  const int t = (int)(gid - (long)task * nfc);
  const int b = tasks[2 * task], face = tasks[2 * task + 1];
  if ((face >> 1) != D) return;
  const int side = face & 1;
  const int* L = link + ((long)b * 6 + face) * LINK_INTS;
  const int t1 = t % nx, t2 = G.ndim == 3 ? t / nx : 0;
  auto reg = [&](int blk, int f) { return freg + (long)(blk * 6 + f) * NV * nfc; };
  R F[NV], v[NFINE][NV];
  const R* rc = reg(b, face);
#pragma unroll
  for (int q = 0; q < NV; ++q) F[q] = rc[q * nfc + t];
#pragma unroll
  for (int k = 0; k < NFINE; ++k) {
    const int a = k & 1, e = k >> 1;
    const int g1 = 2 * t1 + a, g2 = 2 * t2 + e;
    const int o1 = g1 >= nx ? 1 : 0, o2 = g2 >= nx ? 1 : 0;
    const int fb = L[1 + (G.ndim == 3 ? o2 * 2 : 0) + o1];
    const R* rf = reg(fb, face ^ 1);
    const int cf = (G.ndim == 3 ? (g2 - o2 * nx) * nx : 0) + (g1 - o1 * nx);
#pragma unroll
    for (int q = 0; q < NV; ++q) v[k][q] = rf[q * nfc + cf];
  }
  const int job = T.job[b];
  const double dt = J.dt_scale * J.dt[job];
  R Ff[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if constexpr (NFINE == 4)
      Ff[q] = ((v[0][q] + v[1][q]) + (v[2][q] + v[3][q])) * R(0.25);
    else
      Ff[q] = (v[0][q] + v[1][q]) * R(0.5);
  }
  const int cell_d = side ? nx - 1 : 0;
  long c;
  if (D == 0) c = pidx(G, cell_d, t1, t2);
  else if (D == 1) c = pidx(G, t1, cell_d, t2);
  else c = pidx(G, t1, t2, cell_d);
  const double idx = T.inv_dx[3 * b + D];
  void* o = block_ptr<SP>(out, b, G.pcells);
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double df = (double)Ff[q] - (double)F[q];
    const double dl = side ? -df * idx : df * idx;
    SP::st(o, q, c, G.pcells, SP::ld(o, q, c, G.pcells) + w * dt * dl);
  }
}

// CFL rate of the cells a flux correction changed (the coarse cells next to
// each task's face), after all corrections: one thread per (task, cell),
// folded into the job's accumulators as the stage folds the others.
template <class SP>
__global__ void __launch_bounds__(256) k_cfl_reflux_cells(GridConst G, Tables T, const int* __restrict__ tasks,
                                                         int ntasks, const void* __restrict__ slot, PhysConst P,
                                                         DevStatus* st, JobCfl C) {
  const int nx = G.nx;
  const int nfc = G.ndim == 3 ? nx * nx : nx;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = gid < (long)ntasks * nfc;
  double rate = 0.0;
  int bad = 0, nan_seen = 0, job = 0;
  if (live) {
    const int task = (int)(gid / nfc);
    const int t = (int)(gid - (long)task * nfc);
    const int b = tasks[2 * task], face = tasks[2 * task + 1];
    const int d = face >> 1, cd = (face & 1) ? nx - 1 : 0;
    const int t1 = t % nx, t2 = G.ndim == 3 ? t / nx : 0;
    long c;
    if (d == 0) c = pidx(G, cd, t1, t2);
    else if (d == 1) c = pidx(G, t1, cd, t2);
    else c = pidx(G, t1, t2, cd);
    job = T.job[b];
    const void* blk = block_ptr<SP>(slot, b, G.pcells);
    double u[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) u[q] = SP::ld(blk, q, c, G.pcells);
    const double ix = T.inv_dx[3 * b], iy = T.inv_dx[3 * b + 1], iz = T.inv_dx[3 * b + 2];
    const double r = G.ndim == 3 ? cell_rate<3>(u, P, ix, iy, iz, bad) : cell_rate<2>(u, P, ix, iy, iz, bad);
    if (isnan(r))
      nan_seen = 1;
    else
      rate = r;
  }
  // when every live lane of the wave is in one job (always in a single-job
  // context; in batch pools unless a wave spans two jobs' tasks): wave max,
  // one atomic; else one atomic per lane.  Lane 0 is live whenever any lane
  // is (live lanes come first).
  const int jw = __shfl(job, 0, 64);
  if (__all(!live || job == jw)) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rate = fmax(rate, __shfl_xor(rate, off, 64));
    const int anynan = __any(nan_seen);
    if (live && (threadIdx.x & 63) == 0) {
      atomicMax(&C.rate_bits[jw], (unsigned long long)__double_as_longlong(rate));
      if (anynan) atomicOr(&C.nan[jw], 1u);
    }
  } else if (live) {
    atomicMax(&C.rate_bits[job], (unsigned long long)__double_as_longlong(rate));
    if (nan_seen) atomicOr(&C.nan[job], 1u);
  }
  if (bad) atomicOr(&st->flags, (unsigned)bad);
}

// ---------------------------------------------------------------------------
// Regrid transfer: one thread per interior cell of a block of the new leaf
// set.  Tasks are REGRID_TASK_INTS ints: kind, new block, sources.
//   COPY:     s0 = the same block in the old set;
//   PROLONG:  s0 = the old parent, s1..s3 = the child's octant (x, y, z):
//             parent cell plus a quarter of the minmod-limited slope per
//             direction towards the child's side; slope neighbours outside
//             the parent come from a same-level neighbour's interior in
//             place, else from the parent's own ghost cells (filled before);
//   RESTRICT: s0..s7 = the old children by octant x + 2y + 4z: the pairwise
//             mean of the 2^d cells under the new cell.

template <int NDIM, class SP>
__global__ void __launch_bounds__(256) k_regrid(GridConst G, Tables Told, const int* __restrict__ tasks, int ntasks,
                                               const void* __restrict__ old_slot, void* __restrict__ new_slot) {
  const int* __restrict__ link = Told.link;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)ntasks * G.icells) return;
  const int tk = (int)(gid / G.icells);
  const int c = (int)(gid - (long)tk * G.icells);
  const int* T = tasks + (long)tk * REGRID_TASK_INTS;
  const int kind = T[0];
  const int nx = G.nx;
  const long pc = G.pcells;
  const int i = c % nx, j = (c / nx) % nx, k = NDIM == 3 ? c / (nx * nx) : 0;
  const long di = pidx_n<NDIM>(G, i, j, k);
  double out[NV];
  if (kind == REGRID_COPY) {
    const void* src = block_ptr<SP>(old_slot, T[2], pc);
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = SP::ld(src, q, di, pc);
  } else if (kind == REGRID_PROLONG) {
    const int pb = T[2];
    const int o[3] = {T[3], T[4], T[5]};
    const int g[3] = {o[0] * nx + i, o[1] * nx + j, o[2] * nx + k};
    int lc[3] = {g[0] >> 1, g[1] >> 1, NDIM == 3 ? g[2] >> 1 : 0};
    const void* src = block_ptr<SP>(old_slot, pb, pc);
    const long i0 = pidx_n<NDIM>(G, lc[0], lc[1], lc[2]);
    int lk[2 * NDIM], ln[2 * NDIM];
#pragma unroll
    for (int f = 0; f < 2 * NDIM; ++f) {
      lk[f] = link[((long)pb * 6 + f) * LINK_INTS];
      ln[f] = link[((long)pb * 6 + f) * LINK_INTS + 1];
    }
    int bm[3], bp[3];
    long im[3], ip[3];
#pragma unroll
    for (int ax = 0; ax < NDIM; ++ax) {
      int m[3] = {lc[0], lc[1], lc[2]}, p[3] = {lc[0], lc[1], lc[2]};
      m[ax] -= 1;
      p[ax] += 1;
      bm[ax] = pb;
      bp[ax] = pb;
      if (m[ax] < 0 && lk[2 * ax] == LINK_SAME) {
        bm[ax] = ln[2 * ax];
        m[ax] += nx;
      }
      if (p[ax] >= nx && lk[2 * ax + 1] == LINK_SAME) {
        bp[ax] = ln[2 * ax + 1];
        p[ax] -= nx;
      }
      im[ax] = pidx_n<NDIM>(G, m[0], m[1], m[2]);
      ip[ax] = pidx_n<NDIM>(G, p[0], p[1], p[2]);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double uc = SP::ld(src, q, i0, pc);
      double r = uc;
#pragma unroll
      for (int ax = 0; ax < NDIM; ++ax) {
        const double sg = (g[ax] & 1) ? 0.25 : -0.25;
        const double um = SP::ld(block_ptr<SP>(old_slot, bm[ax], pc), q, im[ax], pc);
        const double up = SP::ld(block_ptr<SP>(old_slot, bp[ax], pc), q, ip[ax], pc);
        r = r + sg * minmod2(uc - um, up - uc);
      }
      out[q] = r;
    }
  } else {  // REGRID_RESTRICT
    const int ox = 2 * i >= nx, oy = 2 * j >= nx, oz = NDIM == 3 && 2 * k >= nx;
    const void* src = block_ptr<SP>(old_slot, T[2 + ox + 2 * oy + 4 * oz], pc);
    const int fi = 2 * i - ox * nx, fj = 2 * j - oy * nx, fk = NDIM == 3 ? 2 * k - oz * nx : 0;
    const long i000 = pidx_n<NDIM>(G, fi, fj, fk);
    const long sy = G.pn, sz = (long)G.pn * G.pn;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      auto v = [&](int e, int bb, int aa) { return SP::ld(src, q, i000 + e * sz + bb * sy + aa, pc); };
      if (NDIM == 2)
        out[q] = ((v(0, 0, 0) + v(0, 0, 1)) + (v(0, 1, 0) + v(0, 1, 1))) * 0.25;
      else
        out[q] = (((v(0, 0, 0) + v(0, 0, 1)) + (v(0, 1, 0) + v(0, 1, 1))) +
                  ((v(1, 0, 0) + v(1, 0, 1)) + (v(1, 1, 0) + v(1, 1, 1)))) * 0.125;
    }
  }
  void* dst = block_ptr<SP>(new_slot, T[1], pc);
#pragma unroll
  for (int q = 0; q < NV; ++q) SP::st(dst, q, di, pc, out[q]);
}

// ---------------------------------------------------------------------------
// Loehner's error indicator per block, one workgroup per active block.  For
// every interior cell and every conserved variable q with weight w_q > 0,
// E_q = sqrt(sum_d (a - 2b + e)^2 / sum_d (|e - b| + |b - a| + eps (|e| +
// 2|b| + |a|))^2) over the directions d with (a, b, e) = the cell's
// neighbours along d and itself; the block's indicator is the largest
// sum_q w_q E_q.  Face neighbours across a same-level face are read in
// place, all others from the block's own ghost cells (filled before).

template <int NDIM, class SP>
__global__ void __launch_bounds__(256) k_lohner(GridConst G, Tables T, const void* __restrict__ slot, LohnerParams L,
                                               double* __restrict__ ind) {
  const int blk = T.order[blockIdx.x];
  const int nx = G.nx;
  const long pc = G.pcells;
  int lk[2 * NDIM], ln[2 * NDIM];
#pragma unroll
  for (int f = 0; f < 2 * NDIM; ++f) {
    lk[f] = T.link[((long)blk * 6 + f) * LINK_INTS];
    ln[f] = T.link[((long)blk * 6 + f) * LINK_INTS + 1];
  }
  const void* own = block_ptr<SP>(slot, blk, pc);
  double r = 0.0;
  for (int c = threadIdx.x; c < (int)G.icells; c += blockDim.x) {
    const int i = c % nx, j = (c / nx) % nx, k = NDIM == 3 ? c / (nx * nx) : 0;
    const long ic = pidx_n<NDIM>(G, i, j, k);
    const void* bm[NDIM];
    const void* bp[NDIM];
    long im[NDIM], ip[NDIM];
#pragma unroll
    for (int ax = 0; ax < NDIM; ++ax) {
      int m[3] = {i, j, k}, p[3] = {i, j, k};
      m[ax] -= 1;
      p[ax] += 1;
      bm[ax] = own;
      bp[ax] = own;
      if (m[ax] < 0 && lk[2 * ax] == LINK_SAME) {
        bm[ax] = block_ptr<SP>(slot, ln[2 * ax], pc);
        m[ax] += nx;
      }
      if (p[ax] >= nx && lk[2 * ax + 1] == LINK_SAME) {
        bp[ax] = block_ptr<SP>(slot, ln[2 * ax + 1], pc);
        p[ax] -= nx;
      }
      im[ax] = pidx_n<NDIM>(G, m[0], m[1], m[2]);
      ip[ax] = pidx_n<NDIM>(G, p[0], p[1], p[2]);
    }
    double e_sum = 0.0;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (!(L.weight[q] > 0.0)) continue;  // uniform over the launch
      const double b = SP::ld(own, q, ic, pc);
      double num = 0.0, den = 0.0;
#pragma unroll
      for (int ax = 0; ax < NDIM; ++ax) {
        const double a = SP::ld(bm[ax], q, im[ax], pc), e = SP::ld(bp[ax], q, ip[ax], pc);
        const double d2 = a - 2.0 * b + e;
        const double dd = fabs(e - b) + fabs(b - a) + L.wavefilter * (fabs(e) + 2.0 * fabs(b) + fabs(a));
        num += d2 * d2;
        den += dd * dd;
      }
      e_sum += L.weight[q] * (den > 0.0 ? sqrt(num / den) : 0.0);
    }
    r = fmax(r, e_sum);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
  __shared__ double smax[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) smax[wave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smax[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, smax[q]);
    ind[blk] = m;
  }
}

// ---------------------------------------------------------------------------
// out = a + coef (b - a) on the leaf interior cells, one thread per cell.
// Both loads of a cell come before its store, so out may be a or b.

template <class SP>
__global__ void __launch_bounds__(256) k_combine(GridConst G, Tables T, const void* a, const void* b, double coef,
                                                void* out) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)T.nactive * G.icells) return;
  const int n = (int)(gid / G.icells);
  const int c = (int)(gid - (long)n * G.icells);
  const int blk = T.order[n];
  const int nx = G.nx;
  const int i = c % nx, j = (c / nx) % nx, k = G.ndim == 3 ? c / (nx * nx) : 0;
  const long pc = pidx(G, i, j, k);
  const void* pa = block_ptr<SP>(a, blk, G.pcells);
  const void* pb = block_ptr<SP>(b, blk, G.pcells);
  void* po = block_ptr<SP>(out, blk, G.pcells);
  double r[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double x = SP::ld(pa, q, pc, G.pcells);
    r[q] = x + coef * (SP::ld(pb, q, pc, G.pcells) - x);
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) SP::st(po, q, pc, G.pcells, r[q]);
}

// ---------------------------------------------------------------------------
// CFL: max over leaf interior cells of sum_d (|v_d| + c_f,d)/dx_d

template <class SP>
__global__ void __launch_bounds__(256) k_cfl(GridConst G, Tables T, const void* __restrict__ slot, PhysConst P,
                                            DevStatus* st, JobCfl C) {
  const int b = T.order[blockIdx.x];
  const int job = T.job[b];
  const void* blk = block_ptr<SP>(slot, b, G.pcells);
  const double ix = T.inv_dx[3 * b], iy = T.inv_dx[3 * b + 1], iz = T.inv_dx[3 * b + 2];
  double r = 0.0;
  int bad = 0, nan_seen = 0;
  const int nx = G.nx;
  for (int c = threadIdx.x; c < (int)G.icells; c += blockDim.x) {
    const int i = c % nx, j = (c / nx) % nx, k = G.ndim == 3 ? c / (nx * nx) : 0;
    const long pc = pidx(G, i, j, k);
    double u[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) u[q] = SP::ld(blk, q, pc, G.pcells);
    const double rate = G.ndim == 3 ? cell_rate<3>(u, P, ix, iy, iz, bad) : cell_rate<2>(u, P, ix, iy, iz, bad);
    if (isnan(rate))
      nan_seen = 1;
    else
      r = fmax(r, rate);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
  __shared__ double smax[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) smax[wave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smax[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, smax[q]);
    atomicMax(&C.rate_bits[job], (unsigned long long)__double_as_longlong(m));
  }
  if (bad) atomicOr(&st->flags, (unsigned)bad);
  if (nan_seen) atomicOr(&C.nan[job], 1u);
}

// Empty the per-job rate accumulators (a kernel rather than a memset, so
// that the clear can sit in a captured graph).
__global__ void k_cfl_clear(JobCfl C) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= C.njobs) return;
  C.rate_bits[j] = 0ull;
  C.nan[j] = 0u;
}

// dt = C / max rate, c_h = C / (dt sum_d 1/dx_d), kappa = alpha c_h / min dx
// (finest level of the job); one thread per job slot, unused slots skipped.
__global__ void k_cfl_finalize(JobCfl C, DevStatus* st) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= C.njobs) return;
  const double* g = C.geom + 4 * j;
  if (!(g[2] > 0.0)) return;
  const double rmax = __longlong_as_double((long long)C.rate_bits[j]);
  const unsigned nan_seen = C.nan[j];
  C.rate_bits[j] = 0ull;
  C.nan[j] = 0u;
  double dt = 0.0, ch = 0.0, kappa = 0.0;
  if (nan_seen || !(rmax > 0.0) || !isfinite(rmax)) {
    atomicOr(&st->flags, (unsigned)F_BAD_DT);
  } else {
    dt = g[2] / rmax;
    ch = g[2] / (dt * g[0]);
    kappa = g[3] * ch / g[1];
  }
  C.dt[j] = dt;
  C.ch[j] = ch;
  C.kappa[j] = kappa;
  if (j == 0) st->last_dt = dt;
}

// ---------------------------------------------------------------------------
// conversions

template <class SP>
__global__ void __launch_bounds__(256) k_set_prim(GridConst G, int first, int count, const double* __restrict__ prim,
                                                 void* __restrict__ slot, PhysConst P) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)count * G.icells) return;
  const int lb = (int)(gid / G.icells);
  const int b = first + lb;
  const int c = (int)(gid - (long)lb * G.icells);
  const int nx = G.nx;
  const int i = c % nx, j = (c / nx) % nx, k = G.ndim == 3 ? c / (nx * nx) : 0;
  double w[NV], u[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) w[q] = prim[((long)lb * NV + q) * G.icells + c];
  prim_to_cons(w, u, P);
  void* o = block_ptr<SP>(slot, b, G.pcells);
  const long c0 = pidx(G, i, j, k);
#pragma unroll
  for (int q = 0; q < NV; ++q) SP::st(o, q, c0, G.pcells, u[q]);
}

template <class SP>
__global__ void __launch_bounds__(256) k_get_cons(GridConst G, int first, int count, const void* __restrict__ slot,
                                                 double* __restrict__ cons) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)count * G.icells) return;
  const int lb = (int)(gid / G.icells);
  const int b = first + lb;
  const int c = (int)(gid - (long)lb * G.icells);
  const int nx = G.nx;
  const int i = c % nx, j = (c / nx) % nx, k = G.ndim == 3 ? c / (nx * nx) : 0;
  const void* s = block_ptr<SP>(slot, b, G.pcells);
  const long c0 = pidx(G, i, j, k);
#pragma unroll
  for (int q = 0; q < NV; ++q) cons[((long)lb * NV + q) * G.icells + c] = SP::ld(s, q, c0, G.pcells);
}

__global__ void k_reset_status(DevStatus* st) {
  if (threadIdx.x == 0) {
    st->flags = 0u;
    st->cfl_nan = 0u;
    st->nfix = 0ull;
    st->rate_bits = 0ull;
  }
}

inline unsigned nblocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_fill_faces(hipStream_t s, const GridConst& G, const int* tasks, int ntasks, const Tables& T,
                             void* slot, const PhysConst& P, const FixedBC& fixed) {
  if (ntasks <= 0) return hipSuccess;
  const long ncell = (long)G.ng * G.nx * (G.ndim == 3 ? G.nx : 1);
  const unsigned nbk = nblocks_for((long)ntasks * ncell, 256);
  const bool uni = ncell % 64 == 0;
  if (G.ndim == 3) {
    if (G.precision == 0) {
      if (uni)
        k_fill_faces<3, StoreF64, true><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot, P, fixed);
      else
        k_fill_faces<3, StoreF64, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot, P, fixed);
    } else {
      if (uni)
        k_fill_faces<3, StoreMixed, true><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot, P, fixed);
      else
        k_fill_faces<3, StoreMixed, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot, P, fixed);
    }
  } else {
    if (G.precision == 0)
      k_fill_faces<2, StoreF64, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot, P, fixed);
    else
      k_fill_faces<2, StoreMixed, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot, P, fixed);
  }
  return hipGetLastError();
}

hipError_t launch_prolong_faces(hipStream_t s, const GridConst& G, const int* tasks, int ntasks, const Tables& T,
                                void* slot) {
  if (ntasks <= 0) return hipSuccess;
  const long hx = G.nx / 2;
  const long ncell = (long)G.ng * hx * (G.ndim == 3 ? hx : 1);
  const unsigned nbk = nblocks_for((long)ntasks * ncell, 256);
  const bool uni = ncell % 64 == 0;
  if (G.ndim == 3) {
    if (G.precision == 0) {
      if (uni)
        k_prolong_faces<3, StoreF64, true><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot);
      else
        k_prolong_faces<3, StoreF64, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot);
    } else {
      if (uni)
        k_prolong_faces<3, StoreMixed, true><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot);
      else
        k_prolong_faces<3, StoreMixed, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot);
    }
  } else {
    if (G.precision == 0)
      k_prolong_faces<2, StoreF64, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot);
    else
      k_prolong_faces<2, StoreMixed, false><<<nbk, 256, 0, s>>>(G, tasks, ntasks, T, slot);
  }
  return hipGetLastError();
}

hipError_t launch_prim(hipStream_t s, const GridConst& G, const void* slot, double* prim, const PhysConst& P,
                       DevStatus* st) {
  const long n = (long)G.nb * G.pcells;
  k_prim<<<nblocks_for(n, 256), 256, 0, s>>>(G, static_cast<const double*>(slot), prim, P, st);
  return hipGetLastError();
}

hipError_t launch_flux(hipStream_t s, const GridConst& G, int dir, const double* prim, double* flux,
                       const double* ch_dev, const PhysConst& P, const double* inv_dx) {
  const long n = (long)G.nb * G.nfaces;
  const unsigned nbk = nblocks_for(n, 256);
  if (dir == 0)
    k_flux<0><<<nbk, 256, 0, s>>>(G, prim, flux, ch_dev, P, inv_dx);
  else if (dir == 1)
    k_flux<1><<<nbk, 256, 0, s>>>(G, prim, flux, ch_dev, P, inv_dx);
  else
    k_flux<2><<<nbk, 256, 0, s>>>(G, prim, flux, ch_dev, P, inv_dx);
  return hipGetLastError();
}

hipError_t launch_reflux(hipStream_t s, const GridConst& G, const int* tasks, int ntasks, const Tables& T,
                         FluxPtrs flux) {
  if (ntasks <= 0) return hipSuccess;
  const long per = G.ndim == 3 ? (long)G.nx * G.nx : G.nx;
  k_reflux<<<nblocks_for(ntasks * per, 256), 256, 0, s>>>(G, tasks, ntasks, T.link, flux);
  return hipGetLastError();
}

hipError_t launch_reflux_apply(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                               const int* tasks, const int first[3], const int count[3], void* out, double w,
                               const void* freg) {
  // one launch per direction, in order: a coarse cell next to finer leaves
  // across faces of two directions is corrected once per direction
  const long per = G.ndim == 3 ? (long)G.nx * G.nx : G.nx;
  if (!freg && (count[0] > 0 || count[1] > 0 || count[2] > 0)) return hipErrorInvalidValue;
#define AMRVAC_REFLUX_LAUNCH(D, SPT)                                                                       \
  if (count[D] > 0) {                                                                                     \
    if (G.ndim == 3)                                                                                      \
      k_reflux_apply<D, SPT, 4><<<nblocks_for(count[D] * per, 256), 256, 0, s>>>(                         \
          G, T, J, tasks + 2 * first[D], count[D], static_cast<const SPT::R*>(freg), out, w);              \
    else                                                                                                  \
      k_reflux_apply<D, SPT, 2><<<nblocks_for(count[D] * per, 256), 256, 0, s>>>(                         \
          G, T, J, tasks + 2 * first[D], count[D], static_cast<const SPT::R*>(freg), out, w);              \
  }
  if (G.precision == 0) {
    AMRVAC_REFLUX_LAUNCH(0, StoreF64);
    AMRVAC_REFLUX_LAUNCH(1, StoreF64);
    if (G.ndim == 3) AMRVAC_REFLUX_LAUNCH(2, StoreF64);
  } else {
    AMRVAC_REFLUX_LAUNCH(0, StoreMixed);
    AMRVAC_REFLUX_LAUNCH(1, StoreMixed);
    if (G.ndim == 3) AMRVAC_REFLUX_LAUNCH(2, StoreMixed);
  }
#undef AMRVAC_REFLUX_LAUNCH
  return hipGetLastError();
}

hipError_t launch_cfl_reflux_cells(hipStream_t s, const GridConst& G, const Tables& T, const int* tasks,
                                   int ntasks, const void* slot, const PhysConst& P, DevStatus* st,
                                   const JobCfl& C) {
  if (ntasks <= 0) return hipSuccess;
  const long n = (long)ntasks * (G.ndim == 3 ? G.nx * G.nx : G.nx);
  if (G.precision == 0)
    k_cfl_reflux_cells<StoreF64><<<nblocks_for(n, 256), 256, 0, s>>>(G, T, tasks, ntasks, slot, P, st, C);
  else
    k_cfl_reflux_cells<StoreMixed><<<nblocks_for(n, 256), 256, 0, s>>>(G, T, tasks, ntasks, slot, P, st, C);
  return hipGetLastError();
}

hipError_t launch_update(hipStream_t s, const GridConst& G, const Tables& T, const void* in, const void* base,
                         void* out, double w, FluxPtrs flux, const double* dt_dev, double dt_scale,
                         const double* kappa_dev) {
  const long n = (long)G.nb * G.icells;
  k_update<<<nblocks_for(n, 256), 256, 0, s>>>(G, T, static_cast<const double*>(in), static_cast<const double*>(base),
                                                static_cast<double*>(out), w, flux, dt_dev, dt_scale, kappa_dev);
  return hipGetLastError();
}

hipError_t launch_cfl_accumulate(hipStream_t s, const GridConst& G, const Tables& T, const void* slot,
                                 const PhysConst& P, DevStatus* st, const JobCfl& C) {
  if (T.nactive <= 0) return hipSuccess;
  if (G.precision == 0)
    k_cfl<StoreF64><<<T.nactive, 256, 0, s>>>(G, T, slot, P, st, C);
  else
    k_cfl<StoreMixed><<<T.nactive, 256, 0, s>>>(G, T, slot, P, st, C);
  return hipGetLastError();
}

hipError_t launch_cfl_finalize(hipStream_t s, DevStatus* st, const JobCfl& C) {
  k_cfl_finalize<<<nblocks_for(C.njobs, 64), 64, 0, s>>>(C, st);
  return hipGetLastError();
}

hipError_t launch_cfl(hipStream_t s, const GridConst& G, const Tables& T, const void* slot, const PhysConst& P,
                      DevStatus* st, const JobCfl& C) {
  hipError_t e = launch_cfl_accumulate(s, G, T, slot, P, st, C);
  if (e != hipSuccess) return e;
  return launch_cfl_finalize(s, st, C);
}

hipError_t launch_regrid(hipStream_t s, const GridConst& G, const Tables& Told, const int* tasks, int ntasks,
                         const void* old_slot, void* new_slot) {
  const long n = (long)ntasks * G.icells;
  if (n <= 0) return hipSuccess;
  const unsigned nbk = nblocks_for(n, 256);
  if (G.ndim == 3) {
    if (G.precision == 0)
      k_regrid<3, StoreF64><<<nbk, 256, 0, s>>>(G, Told, tasks, ntasks, old_slot, new_slot);
    else
      k_regrid<3, StoreMixed><<<nbk, 256, 0, s>>>(G, Told, tasks, ntasks, old_slot, new_slot);
  } else {
    if (G.precision == 0)
      k_regrid<2, StoreF64><<<nbk, 256, 0, s>>>(G, Told, tasks, ntasks, old_slot, new_slot);
    else
      k_regrid<2, StoreMixed><<<nbk, 256, 0, s>>>(G, Told, tasks, ntasks, old_slot, new_slot);
  }
  return hipGetLastError();
}

hipError_t launch_lohner(hipStream_t s, const GridConst& G, const Tables& T, const void* slot, const LohnerParams& L,
                         double* ind) {
  if (T.nactive <= 0) return hipSuccess;
  if (G.ndim == 3) {
    if (G.precision == 0)
      k_lohner<3, StoreF64><<<T.nactive, 256, 0, s>>>(G, T, slot, L, ind);
    else
      k_lohner<3, StoreMixed><<<T.nactive, 256, 0, s>>>(G, T, slot, L, ind);
  } else {
    if (G.precision == 0)
      k_lohner<2, StoreF64><<<T.nactive, 256, 0, s>>>(G, T, slot, L, ind);
    else
      k_lohner<2, StoreMixed><<<T.nactive, 256, 0, s>>>(G, T, slot, L, ind);
  }
  return hipGetLastError();
}

hipError_t launch_combine(hipStream_t s, const GridConst& G, const Tables& T, const void* a, const void* b,
                          double coef, void* out) {
  const long n = (long)T.nactive * G.icells;
  if (n <= 0) return hipSuccess;
  if (G.precision == 0)
    k_combine<StoreF64><<<nblocks_for(n, 256), 256, 0, s>>>(G, T, a, b, coef, out);
  else
    k_combine<StoreMixed><<<nblocks_for(n, 256), 256, 0, s>>>(G, T, a, b, coef, out);
  return hipGetLastError();
}

hipError_t launch_cfl_clear(hipStream_t s, const JobCfl& C) {
  k_cfl_clear<<<nblocks_for(C.njobs, 64), 64, 0, s>>>(C);
  return hipGetLastError();
}

hipError_t launch_set_prim(hipStream_t s, const GridConst& G, int first, int count, const double* prim, void* slot,
                           const PhysConst& P) {
  const long n = (long)count * G.icells;
  if (n <= 0) return hipSuccess;
  if (G.precision == 0)
    k_set_prim<StoreF64><<<nblocks_for(n, 256), 256, 0, s>>>(G, first, count, prim, slot, P);
  else
    k_set_prim<StoreMixed><<<nblocks_for(n, 256), 256, 0, s>>>(G, first, count, prim, slot, P);
  return hipGetLastError();
}

hipError_t launch_get_cons(hipStream_t s, const GridConst& G, int first, int count, const void* slot,
                           double* cons) {
  const long n = (long)count * G.icells;
  if (n <= 0) return hipSuccess;
  if (G.precision == 0)
    k_get_cons<StoreF64><<<nblocks_for(n, 256), 256, 0, s>>>(G, first, count, slot, cons);
  else
    k_get_cons<StoreMixed><<<nblocks_for(n, 256), 256, 0, s>>>(G, first, count, slot, cons);
  return hipGetLastError();
}

hipError_t launch_reset_status(hipStream_t s, DevStatus* st) {
  k_reset_status<<<1, 64, 0, s>>>(st);
  return hipGetLastError();
}

}  // namespace amrvac
