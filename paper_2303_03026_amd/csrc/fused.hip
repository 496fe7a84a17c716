// Fused FP64 stage kernel for 16^ndim blocks: conserved -> primitive, van Leer
// reconstruction, GLM interface + HLL fluxes in every direction, flux
// difference, psi damping and the SSPRK combination, in one launch.
//
// One 256-thread workgroup per block; thread t owns the (x, y) column
// i = t % 16, j = t / 16.  In 3D the workgroup marches through the z planes:
// the z stencil lives in a per-thread register queue (primitives of planes
// k and k+1, the left face state of the next z face and the previous z
// flux), while the x and y stencils of the current plane go through LDS:
// one plane of primitives with its 2-deep x/y halo, plus one buffer that
// holds first the slopes and then the face fluxes of one direction.
// Halo cells across faces shared with a same-level leaf are read directly
// from that neighbour's interior; only faces towards finer or coarser
// leaves and physical boundaries need filled ghost cells.
#include "kernels.h"

namespace amrvac {

namespace {

constexpr int BN = 16;          // block cells per direction
constexpr int BP = BN + 4;      // padded extent
constexpr int SLOPE_ROW = BN + 2;

template <int NDIM>
struct Pad {
  static constexpr long cells = NDIM == 3 ? (long)BP * BP * BP : (long)BP * BP;
  __device__ static constexpr long at(int i, int j, int k) {
    return ((long)(NDIM == 3 ? k + 2 : 0) * BP + (j + 2)) * BP + (i + 2);
  }
};

__device__ __forceinline__ void load_cons(const double* __restrict__ U, long pc, long c, double u[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) u[q] = U[q * pc + c];
}

// Reconstruct the face between LDS cells (line, f-1) and (line, f) along DIR
// from the plane primitives and the slopes of the two cells; first-order
// fallback when rho or p is not positive on either side.
template <int DIR>
__device__ __forceinline__ void face_states(const double (*Wp)[BP * BP], const double (*Sl)[SLOPE_ROW * BN],
                                            int line, int f, double wl[NV], double wr[NV]) {
  double wm[NV], wp[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if (DIR == 0) {
      wm[q] = Wp[q][(line + 2) * BP + f + 1];
      wp[q] = Wp[q][(line + 2) * BP + f + 2];
    } else {
      wm[q] = Wp[q][(f + 1) * BP + line + 2];
      wp[q] = Wp[q][(f + 2) * BP + line + 2];
    }
    wl[q] = wm[q] + 0.5 * Sl[q][line * SLOPE_ROW + f];
    wr[q] = wp[q] - 0.5 * Sl[q][line * SLOPE_ROW + f + 1];
  }
  if (!((wl[I_RHO] > 0.0) && (wl[4] > 0.0) && (wr[I_RHO] > 0.0) && (wr[4] > 0.0))) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      wl[q] = wm[q];
      wr[q] = wp[q];
    }
  }
}

// van Leer slope along DIR of LDS cell (line, a), a in -1..16
template <int DIR>
__device__ __forceinline__ void cell_slope(const double (*Wp)[BP * BP], double (*Sl)[SLOPE_ROW * BN], int line,
                                           int a) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double m, c, p;
    if (DIR == 0) {
      m = Wp[q][(line + 2) * BP + a + 1];
      c = Wp[q][(line + 2) * BP + a + 2];
      p = Wp[q][(line + 2) * BP + a + 3];
    } else {
      m = Wp[q][(a + 1) * BP + line + 2];
      c = Wp[q][(a + 2) * BP + line + 2];
      p = Wp[q][(a + 3) * BP + line + 2];
    }
    Sl[q][line * SLOPE_ROW + a + 1] = vl_slope(c - m, p - c);
  }
}

// One in-plane direction: slopes -> sync -> face fluxes -> sync -> flux
// difference of this thread's cell added to acc (scaled by 1/dx).
template <int DIR>
__device__ __forceinline__ void plane_direction(const double (*Wp)[BP * BP], double (*Sl)[SLOPE_ROW * BN],
                                                double (*Fl)[(BN + 1) * BN], int t, int i, int j, double ch,
                                                double hic, double inv_dx, const PhysConst& P, double acc[NV]) {
  const int line = DIR == 0 ? j : i;
  const int f = DIR == 0 ? i : j;
  cell_slope<DIR>(Wp, Sl, line, f);
  if (t < 32) cell_slope<DIR>(Wp, Sl, t & 15, t < 16 ? -1 : BN);
  __syncthreads();
  {
    double wl[NV], wr[NV], F[NV];
    face_states<DIR>(Wp, Sl, line, f, wl, wr);
    hll_glm_flux<DIR>(wl, wr, ch, hic, P, F);
#pragma unroll
    for (int q = 0; q < NV; ++q) Fl[q][line * (BN + 1) + f] = F[q];
  }
  if (t < 16) {  // the 17th face of line t
    double wl[NV], wr[NV], F[NV];
    face_states<DIR>(Wp, Sl, t, BN, wl, wr);
    hll_glm_flux<DIR>(wl, wr, ch, hic, P, F);
#pragma unroll
    for (int q = 0; q < NV; ++q) Fl[q][t * (BN + 1) + BN] = F[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q)
    acc[q] = acc[q] + (Fl[q][line * (BN + 1) + f + 1] - Fl[q][line * (BN + 1) + f]) * inv_dx;
}

template <int NDIM>
__global__ void __launch_bounds__(256, 2)
k_stage_fused(GridConst G, LevelConst Lc, const int* __restrict__ level, const int* __restrict__ link,
              const int* __restrict__ order, int per_xcd, const double* __restrict__ in, const double* base,
              double* out, double wgt, const double* __restrict__ dt_dev, const double* __restrict__ ch_dev,
              const double* __restrict__ kappa_dev, PhysConst P, DevStatus* st) {
  using PD = Pad<NDIM>;
  constexpr long PC = PD::cells;
  __shared__ double Wp[NV][BP * BP];          // primitives of the current plane (+ x/y halo)
  __shared__ double Sl[NV][SLOPE_ROW * BN];   // slopes of one direction, cells -1..16 per line
  __shared__ double Fl[NV][(BN + 1) * BN];    // face fluxes of one direction, faces 0..16 per line

  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of the Morton-ordered block list so that neighbouring
  // blocks run together on one L2.
  const int slot = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (slot >= G.nb) return;
  const int b = order[slot];
  const int t = threadIdx.x;
  const int i = t & 15, j = t >> 4;
  const long boff = (long)b * NV * PC;
  const double* __restrict__ U = in + boff;
  // Halo source per face: a same-level neighbour is read in place (its
  // interior, shifted by one block); other faces use this block's ghost
  // cells, filled by the ghost kernels.
  int srcb[6], sh[6];
#pragma unroll
  for (int f = 0; f < 2 * NDIM; ++f) {
    const int* Lk = link + ((long)b * 6 + f) * LINK_INTS;
    const bool same = Lk[0] == LINK_SAME;
    srcb[f] = same ? Lk[1] : b;
    sh[f] = same ? ((f & 1) ? -BN : BN) : 0;
  }
  const int lev = level[b];
  const double dt = *dt_dev, ch = *ch_dev, kappa = *kappa_dev;
  const double hic = 0.5 / ch;
  const double idx = Lc.inv_dx[lev][0], idy = Lc.inv_dx[lev][1], idz = Lc.inv_dx[lev][2];
  int bad = 0;
  unsigned nfix = 0;

  // halo cell of this thread for the x/y stencil of a plane (threads 0..127)
  int hx = 0, hy = 0;
  const bool has_halo = t < 128;
  if (t < 64) {
    hy = t >> 2;
    const int o = t & 3;
    hx = o < 2 ? o - 2 : BN + o - 2;
  } else if (t < 128) {
    hx = t & 15;
    const int o = (t >> 4) & 3;
    hy = o < 2 ? o - 2 : BN + o - 2;
  }
  const int hf = hx < 0 ? 0 : (hx >= BN ? 1 : (hy < 0 ? 2 : 3));
  const double* __restrict__ Uh = in + (long)srcb[hf] * NV * PC;
  const int hxs = hx + (hf < 2 ? sh[hf] : 0), hys = hy + (hf >= 2 ? sh[hf] : 0);
  // z ghost planes come from faces 4 (below) and 5 (above)
  const double* __restrict__ Uzlo = in + (long)srcb[NDIM == 3 ? 4 : 0] * NV * PC;
  const double* __restrict__ Uzhi = in + (long)srcb[NDIM == 3 ? 5 : 0] * NV * PC;
  const int shzlo = NDIM == 3 ? sh[4] : 0, shzhi = NDIM == 3 ? sh[5] : 0;

  auto convert = [&](const double u[NV], double w[NV]) {
    const int bb = cons_to_prim(u, w, P);
    if (bb) {
      bad |= bb;
      if (P.fix) ++nfix;
    }
  };

  // z pipeline (3D): wa = W(k), wb = W(k+1), wla = left state of face k+1/2
  // (W(k) + sigma(k)/2), fzlo = z flux at face k-1/2.
  double wa[NV], wb[NV], wla[NV], fzlo[NV];
  if (NDIM == 3) {
    double u[NV], wm2[NV], wm1[NV];
    load_cons(Uzlo, PC, PD::at(i, j, -2 + shzlo), u);
    convert(u, wm2);
    load_cons(Uzlo, PC, PD::at(i, j, -1 + shzlo), u);
    convert(u, wm1);
    load_cons(U, PC, PD::at(i, j, 0), u);
    convert(u, wa);
    load_cons(U, PC, PD::at(i, j, 1), u);
    convert(u, wb);
    double wl[NV], wr[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double sm = vl_slope(wm1[q] - wm2[q], wa[q] - wm1[q]);
      const double s0 = vl_slope(wa[q] - wm1[q], wb[q] - wa[q]);
      wl[q] = wm1[q] + 0.5 * sm;
      wr[q] = wa[q] - 0.5 * s0;
      wla[q] = wa[q] + 0.5 * s0;
    }
    if (!((wl[I_RHO] > 0.0) && (wl[4] > 0.0) && (wr[I_RHO] > 0.0) && (wr[4] > 0.0))) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        wl[q] = wm1[q];
        wr[q] = wa[q];
      }
    }
    hll_glm_flux<2>(wl, wr, ch, hic, P, fzlo);
  } else {
    double u[NV];
    load_cons(U, PC, PD::at(i, j, 0), u);
    convert(u, wa);
  }

  constexpr int NK = NDIM == 3 ? BN : 1;
  for (int k = 0; k < NK; ++k) {
    // prefetch the conserved state of plane k+2 (consumed by the z step)
    double uc[NV];
    if (NDIM == 3) {
      if (k + 2 < BN)
        load_cons(U, PC, PD::at(i, j, k + 2), uc);
      else
        load_cons(Uzhi, PC, PD::at(i, j, k + 2 + shzhi), uc);
    }

    // ---- plane k primitives into LDS (interior from the queue, halo loaded)
#pragma unroll
    for (int q = 0; q < NV; ++q) Wp[q][(j + 2) * BP + (i + 2)] = wa[q];
    if (has_halo) {
      double u[NV], w[NV];
      load_cons(Uh, PC, PD::at(hxs, hys, k), u);
      convert(u, w);
#pragma unroll
      for (int q = 0; q < NV; ++q) Wp[q][(hy + 2) * BP + (hx + 2)] = w[q];
    }
    __syncthreads();

    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    plane_direction<0>(Wp, Sl, Fl, t, i, j, ch, hic, idx, P, acc);
    plane_direction<1>(Wp, Sl, Fl, t, i, j, ch, hic, idy, P, acc);

    // ---- z direction (registers)
    if (NDIM == 3) {
      double wc[NV];
      convert(uc, wc);
      double wl[NV], wr[NV], fz[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double s1 = vl_slope(wb[q] - wa[q], wc[q] - wb[q]);
        wl[q] = wla[q];
        wr[q] = wb[q] - 0.5 * s1;
        wla[q] = wb[q] + 0.5 * s1;
      }
      if (!((wl[I_RHO] > 0.0) && (wl[4] > 0.0) && (wr[I_RHO] > 0.0) && (wr[4] > 0.0))) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          wl[q] = wa[q];
          wr[q] = wb[q];
        }
      }
      hll_glm_flux<2>(wl, wr, ch, hic, P, fz);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        acc[q] = acc[q] + (fz[q] - fzlo[q]) * idz;
        fzlo[q] = fz[q];
        wa[q] = wb[q];
        wb[q] = wc[q];
      }
    }

    // ---- update: L = -(sum_d dF_d / dx_d) - kappa psi; SSPRK combination
    const long c = PD::at(i, j, k);
    double u[NV];
    load_cons(U, PC, c, u);
    double* __restrict__ o = out + boff + c;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double lq = -acc[q];
      if (q == I_PSI) lq = lq - kappa * u[I_PSI];
      const double tq = u[q] + dt * lq;
      if (wgt == 1.0) {
        o[q * PC] = tq;
      } else {
        const double u0 = base[boff + c + q * PC];
        o[q * PC] = u0 + wgt * (tq - u0);
      }
    }
  }
  if (bad) atomicOr(&st->flags, (unsigned)bad);
  if (nfix) atomicAdd(&st->nfix, (unsigned long long)nfix);
}

}  // namespace

hipError_t launch_fused_stage(hipStream_t s, const GridConst& G, const LevelConst& L, const int* level,
                              const int* link, const int* order, const void* in, const void* base, void* out,
                              double w, const double* dt_dev, const double* ch_dev, const double* kappa_dev,
                              const PhysConst& P, DevStatus* st) {
  if (G.nx != BN) return hipErrorInvalidValue;
  const int per_xcd = (G.nb + 7) / 8;
  const unsigned grid = 8u * (unsigned)per_xcd;
  if (G.ndim == 3)
    k_stage_fused<3><<<grid, 256, 0, s>>>(G, L, level, link, order, per_xcd, static_cast<const double*>(in),
                                          static_cast<const double*>(base), static_cast<double*>(out), w, dt_dev,
                                          ch_dev, kappa_dev, P, st);
  else
    k_stage_fused<2><<<grid, 256, 0, s>>>(G, L, level, link, order, per_xcd, static_cast<const double*>(in),
                                          static_cast<const double*>(base), static_cast<double*>(out), w, dt_dev,
                                          ch_dev, kappa_dev, P, st);
  return hipGetLastError();
}

}  // namespace amrvac
