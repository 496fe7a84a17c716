// Fused stage kernel for 2D 16^2 blocks with three ghost layers (the
// five-cell reconstructions 'weno5', 'wenoz5', 'wenozp5' and 'mp5'), FP64:
// conserved -> primitive, the fifth-order face states, GLM interface + HLL
// (or HLLD, HLLC) fluxes in both directions, flux difference, psi damping
// and the SSPRK combination in one launch.
//
// One 256-thread workgroup per block; thread t owns cell (i, j) = (t % 16,
// t / 16).  The block's primitives with a 3-deep x/y halo (22 x 22 cells,
// corners unused) live in LDS; halo cells across a face shared with a
// same-level leaf are read in place from that neighbour's interior, the
// others from this block's ghost cells (filled by the ghost kernels).  Each
// thread evaluates one x face and one y face; neighbouring face fluxes come
// by lane shuffles.  The arithmetic is the per-kernel path's step for step (same
// primitive conversion, face states, flux and update order), so on grids
// without coarse/fine faces the two paths agree bit for bit.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_mhd.h"
#include "kernels.h"

namespace amrvac {
namespace {

constexpr int BN5 = 16;             // cells per block side
constexpr int NG5 = 3;              // ghost layers
constexpr int P5 = BN5 + 2 * NG5;   // LDS cells per row / column
constexpr int S5 = P5 + 1;          // LDS row stride (odd, against bank conflicts on column reads)
constexpr int NF5 = BN5 + 1;        // faces per line

// padded 2D cell index in a block of the slot layout
__device__ __forceinline__ long cell5(const GridConst& G, int x, int y) { return (long)(y + NG5) * G.pn + (x + NG5); }

template <bool W1>
__global__ void __launch_bounds__(256, 3) k_stage_fused5(GridConst G, Tables T, JobScalars J, const void* __restrict__ in,
                                                         const void* base, void* out, double wgt, PhysConst P,
                                                         DevStatus* st) {
  // primitives, cell (x, y) at (y + 3) * S5 + (x + 3); once all faces are
  // evaluated the same storage carries the y flux differences to the cells'
  // owners, cell (x, y) at y * NF5 + x
  __shared__ double W[NV][P5 * S5];
  __shared__ double Ex[NV][BN5];  // the 17th x face of each row
  __shared__ double Ey[NV][BN5];  // the 17th y face of each column
  const int b = T.order[blockIdx.x];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const long PC = G.pcells;
  const void* own = block_ptr<StoreF64>(in, b, PC);
  int lk[4], ln[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    lk[f] = T.link[((long)b * 6 + f) * LINK_INTS];
    ln[f] = T.link[((long)b * 6 + f) * LINK_INTS + 1];
  }
  int bad = 0;
  unsigned nfix = 0;
  // conserved state of cell (x, y) of this block, -3 <= x, y < 19 with at
  // most one coordinate outside 0..15, as primitives into LDS
  auto fetch = [&](int x, int y) {
    const void* blk = own;
    int xs = x, ys = y, f = -1;
    if (x < 0) f = 0;
    else if (x >= BN5) f = 1;
    else if (y < 0) f = 2;
    else if (y >= BN5) f = 3;
    if (f >= 0 && lk[f] == LINK_SAME) {
      blk = block_ptr<StoreF64>(in, ln[f], PC);
      if (f == 0) xs += BN5;
      else if (f == 1) xs -= BN5;
      else if (f == 2) ys += BN5;
      else ys -= BN5;
    }
    const long c = cell5(G, xs, ys);
    double u[NV], w[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) u[q] = StoreF64::ld(blk, q, c, PC);
    const int bb = cons_to_prim(u, w, P);
    if (bb) {
      bad |= bb;
      if (P.fix) ++nfix;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) W[q][(y + NG5) * S5 + (x + NG5)] = w[q];
  };
  fetch(i, j);
  if (t < 4 * NG5 * BN5) {  // the 192 halo cells: 48 per side, 3 layers of 16
    const int side = t / (NG5 * BN5), r = t - side * (NG5 * BN5);
    if (side < 2) {
      const int y = r / NG5, a = r - y * NG5;
      fetch(side == 0 ? a - NG5 : BN5 + a, y);
    } else {
      const int x = r % BN5, a = r / BN5;
      fetch(x, side == 2 ? a - NG5 : BN5 + a);
    }
  }
  __syncthreads();

  const int job = T.job[b];
  const double ch = J.ch[job];
  const double idx = T.inv_dx[3 * b], idy = T.inv_dx[3 * b + 1];
  const int lim = P.limiter;
  const double lamx = lim == LIM_WENOZP5 ? 1.0 / cbrt(idx * idx) : 0.0;
  const double lamy = lim == LIM_WENOZP5 ? 1.0 / cbrt(idy * idy) : 0.0;

  // face f of line `line` along DIR (between cells f-1 and f of the line).
  // The five-cell reconstructions act on one variable at a time, so each
  // variable's six cells are read from LDS just before use (a few live
  // registers instead of all 54 values); the arithmetic is that of the
  // shared six-cell reconstruction.
  auto face = [&](auto dir, int line, int f, double lambda, double Fq[NV]) {
    constexpr int DIR = decltype(dir)::value;
    auto at = [&](int s) {
      const int a = f - NG5 + s;
      return DIR == 0 ? (line + NG5) * S5 + (a + NG5) : (a + NG5) * S5 + (line + NG5);
    };
    double wl[NV], wr[NV];
    if (lim >= LIM_WENO5) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double v0 = W[q][at(0)], v1 = W[q][at(1)], v2 = W[q][at(2)];
        const double v3 = W[q][at(3)], v4 = W[q][at(4)], v5 = W[q][at(5)];
        if (lim == LIM_MP5) {
          wl[q] = mp5_face(v0, v1, v2, v3, v4);
          wr[q] = mp5_face(v5, v4, v3, v2, v1);
        } else {
          wl[q] = weno5_face(v0, v1, v2, v3, v4, lim, lambda);
          wr[q] = weno5_face(v5, v4, v3, v2, v1, lim, lambda);
        }
      }
      double cl[NV], cr[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        cl[q] = W[q][at(2)];
        cr[q] = W[q][at(3)];
      }
      positivity_fallback(wl, wr, cl, cr);
    } else {
      double c1[NV], c2[NV], c3[NV], c4[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        c1[q] = W[q][at(1)];
        c2[q] = W[q][at(2)];
        c3[q] = W[q][at(3)];
        c4[q] = W[q][at(4)];
      }
      reconstruct_face(lim, c1, c2, c3, c4, wl, wr);
    }
    face_flux_rt<DIR, double>(P.flux, wl, wr, ch, 0.5 / ch, P.gamma, P.inv_gm1, Fq);
  };
  using X = std::integral_constant<int, 0>;
  using Y = std::integral_constant<int, 1>;

  // 2 x 16 x 17 faces on 4 waves.  Along x thread t = (i, j) evaluates the
  // left face of cell (i, j); along y it evaluates the lower face of cell
  // (j, i) (transposed), so that in both directions the face above a thread's
  // lies in the next lane of the same wave and reaches it by a lane shuffle.
  // The 17th faces of the rows go to the first wave's lanes 0..15 and those
  // of the columns to the second wave's, through LDS: no wave takes more
  // than three face evaluations.
  double fx[NV], fy[NV];
  face(X{}, j, i, lamx, fx);
  face(Y{}, j, i, lamy, fy);
  if (t < BN5 || (t >= 64 && t < 64 + BN5)) {
    double fe[NV];
    if (t < BN5) {
      face(X{}, t, BN5, lamx, fe);
#pragma unroll
      for (int q = 0; q < NV; ++q) Ex[q][t] = fe[q];
    } else {
      face(Y{}, t - 64, BN5, lamy, fe);
#pragma unroll
      for (int q = 0; q < NV; ++q) Ey[q][t - 64] = fe[q];
    }
  }
  __syncthreads();  // every face evaluated: W is free, Ex / Ey written
  const int up = (t & 63) + 1;
  double dx[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double nx_ = __shfl(fx[q], up, 64), ny_ = __shfl(fy[q], up, 64);
    dx[q] = (i < BN5 - 1 ? nx_ : Ex[q][j]) - fx[q];
    // y difference of cell (j, i), handed to the thread that owns it
    W[q][i * NF5 + j] = (i < BN5 - 1 ? ny_ : Ey[q][j]) - fy[q];
  }
  __syncthreads();
  double L[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    L[q] = 0.0;
    L[q] = L[q] + dx[q] * idx;
    L[q] = L[q] + W[q][j * NF5 + i] * idy;
  }

  // update: L = -(sum_d dF_d / dx_d) - kappa psi; SSPRK combination
  const long c = cell5(G, i, j);
  const double dt = J.dt_scale * J.dt[job], kappa = J.kappa[job];
  const double psi = StoreF64::ld(own, I_PSI, c, PC);
  void* o = block_ptr<StoreF64>(out, b, PC);
  const void* bs = block_ptr<StoreF64>(base, b, PC);
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double lq = -L[q];
    if (q == I_PSI) lq = lq - kappa * psi;
    const double tq = StoreF64::ld(own, q, c, PC) + dt * lq;
    if (W1) {
      StoreF64::st(o, q, c, PC, tq);
    } else {
      const double u0 = StoreF64::ld(bs, q, c, PC);
      StoreF64::st(o, q, c, PC, u0 + wgt * (tq - u0));
    }
  }
  if (bad) atomicOr(&st->flags, (unsigned)bad);
  if (nfix) atomicAdd(&st->nfix, (unsigned long long)nfix);
}

}  // namespace

hipError_t launch_fused5_stage(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J, const void* in,
                               const void* base, void* out, double w, const PhysConst& P, DevStatus* st) {
  if (G.ndim != 2 || G.nx != BN5 || G.ng != NG5 || G.precision != 0) return hipErrorInvalidValue;
  if (T.nactive <= 0) return hipSuccess;
  if (w == 1.0)
    k_stage_fused5<true><<<T.nactive, 256, 0, s>>>(G, T, J, in, base, out, w, P, st);
  else
    k_stage_fused5<false><<<T.nactive, 256, 0, s>>>(G, T, J, in, base, out, w, P, st);
  return hipGetLastError();
}

}  // namespace amrvac
