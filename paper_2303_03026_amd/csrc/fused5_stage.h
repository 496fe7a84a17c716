// Fused stage kernel for 16^ndim blocks with three ghost layers (the
// five-cell reconstructions 'weno5', 'wenoz5', 'wenozp5' and 'mp5'), FP64 or
// FP32-mixed: conserved -> primitive, the fifth-order face states, GLM
// interface + HLL (or HLLD, HLLC) fluxes in every direction, flux
// difference, psi damping and the SSPRK combination in one launch.
//
// FP32-mixed: FP32 storage, primitives, face states and fluxes; the
// nonlinear weights of the five-cell values in FP64 (from the FP32 cells);
// the energy's flux differences and update, the pressure recovery and the
// small-value check in FP64 -- the split of the two-ghost-layer mixed stage.
//
// One 256-thread workgroup per block; thread t owns cell (i, j) = (t % 16,
// t / 16) of a plane.  A plane's primitives with a 3-deep in-plane halo
// (22 x 22 cells, corners unused) live in LDS; halo cells across a face
// shared with a same-level leaf are read in place from that neighbour's
// interior, the others from this block's ghost cells (filled by the ghost
// kernels).  Each thread evaluates one face per in-plane direction;
// neighbouring face fluxes come by lane shuffles.
//
// 2D: the block is one x-y plane.  3D: the workgroup first sweeps the 16 x-y
// planes, leaving each cell's x and y flux differences in a per-block
// scratch array, then sweeps the 16 x-z planes, where the z faces take the
// place of the y faces, and updates.  (A z register queue would hold six
// planes of primitives per thread, more than the register file holds at
// any useful occupancy.)  The arithmetic is the per-kernel path's step for
// step (same primitive conversion, face states, flux and the x, y, z order
// of the flux differences), so on grids without coarse/fine faces the two
// paths agree bit for bit.
//
// The reconstruction (LIM: one of the five-cell limiters, or -1 for the
// two-ghost-layer limiters chosen at run time) and the Riemann solver (FLX)
// are template parameters, so that an instance holds the code of one scheme
// only; the instances are spread over three translation units, one per
// flux (fused5.hip: HLL and the dispatch; fused5_hllc.hip; fused5_hlld.hip).
#pragma once
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

// padded cell index in a block of the slot layout
__device__ __forceinline__ long cell5(const GridConst& G, int x, int y, int z = 0) {
  return ((long)(G.ndim == 3 ? z + NG5 : 0) * G.pn + (y + NG5)) * G.pn + (x + NG5);
}

// freg (grids with a coarse/fine flux correction; else null): the face
// fluxes evaluated on block faces towards finer or coarser leaves are stored
// in these flux registers ([block][face][var][face cell], face cell t1 + 16
// t2 with t1 along the face's first transverse axis: y for x faces, x
// otherwise) for the correction pass.  One instance serves both cases: a
// separate instance without the register stores was measured slower (its
// register allocation spills 448 against 176 B per lane in 3D FP64, and a
// c1 step with 'wenozp5' + HLLC took 19.3 against 16.5 ms).
// CFL: also fold the CFL rate of every output cell into the job's running
// maximum (C.rate_bits, C.nan), leaving out the cells next to faces towards
// finer leaves when C.skip_fine (the flux correction changes them later).
// Three workgroups per CU (at most 168 VGPRs; the 3D instances spill a few
// hundred bytes per lane): a plane's 17th faces leave some waves idle at
// the barrier after the face evaluations (in the x-z sweep a single wave
// works through them), and a third resident workgroup fills those slots.
// With two per CU (256 VGPRs, little spilling) the 3D stage took 12% (FP64)
// and 24% (FP32-mixed) longer; with four, FP64 lost that gain again.
template <int NDIM, class SP, bool W1, bool CFL, int LIM, int FLX>
__global__ void __launch_bounds__(256, 3) k_stage_fused5(GridConst G, Tables T, JobScalars J, const void* __restrict__ in,
                                                         const void* base, void* out, double wgt, PhysConst P,
                                                         DevStatus* st, double* __restrict__ part,
                                                         typename SP::R* __restrict__ freg, JobCfl C) {
  using R = typename SP::R;
  // primitives of a plane, cell (a, c) of its two axes at (c + 3) * S5 + (a + 3);
  // once all faces of the plane are evaluated the same storage carries the
  // second axis' flux differences to the cells' owners, cell (a, c) at
  // c * NF5 + a
  __shared__ R W[NV][P5 * S5];
  __shared__ R Ex[NV][BN5];  // the 17th face of each line along the first axis
  __shared__ R Ey[NV][BN5];  // the 17th face of each line along the second axis
  // mixed: the energy's second-axis differences on their way
  __shared__ double De[std::is_same<typename SP::R, double>::value ? 1 : BN5 * NF5];
  const int b = T.order[blockIdx.x];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const long PC = G.pcells;
  const void* own = block_ptr<SP>(in, b, PC);
  int lk[2 * NDIM], ln[2 * NDIM];
#pragma unroll
  for (int f = 0; f < 2 * NDIM; ++f) {
    lk[f] = T.link[((long)b * 6 + f) * LINK_INTS];
    ln[f] = T.link[((long)b * 6 + f) * LINK_INTS + 1];
  }
  int bad = 0;
  unsigned nfix = 0;
  // conserved state of cell (x, y, z) of this block (at most one coordinate
  // outside 0..15), as primitives into the plane's LDS cell (a, c); count:
  // whether a small-value fix is counted here (each cell once per stage)
  auto fetch = [&](int x, int y, int z, int a, int c, bool count) {
    const void* blk = own;
    int xs = x, ys = y, zs = z, f = -1;
    if (x < 0) f = 0;
    else if (x >= BN5) f = 1;
    else if (y < 0) f = 2;
    else if (y >= BN5) f = 3;
    else if (NDIM == 3 && z < 0) f = 4;
    else if (NDIM == 3 && z >= BN5) f = 5;
    if (f >= 0 && lk[f] == LINK_SAME) {
      blk = block_ptr<SP>(in, ln[f], PC);
      if (f == 0) xs += BN5;
      else if (f == 1) xs -= BN5;
      else if (f == 2) ys += BN5;
      else if (f == 3) ys -= BN5;
      else if (f == 4) zs += BN5;
      else zs -= BN5;
    }
    const long ci = cell5(G, xs, ys, zs);
    double u[NV];
    R w[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) u[q] = SP::ld(blk, q, ci, PC);
    const int bb = cons_to_prim(u, w, P);
    if (bb) {
      bad |= bb;
      if (P.fix && count) ++nfix;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) W[q][(c + NG5) * S5 + (a + NG5)] = w[q];
  };

  // faces with flux registers (bit f: block face f)
  constexpr int NFC = NDIM == 3 ? BN5 * BN5 : BN5;
  unsigned regs = 0, skips = 0;
  if (freg) {
#pragma unroll
    for (int f = 0; f < 2 * NDIM; ++f)
      if (lk[f] == LINK_FINE || lk[f] == LINK_COARSE) regs |= 1u << f;
  }
  if constexpr (CFL) {
#pragma unroll
    for (int f = 0; f < 2 * NDIM; ++f)
      if (C.skip_fine && lk[f] == LINK_FINE) skips |= 1u << f;
  }
  double rmax = 0.0;  // CFL: running max of this thread's output cells
  int rnan = 0;
  // store the NV fluxes of one face cell (the address is formed here: the
  // empty asm keeps the compiler from hoisting it out of the plane loops)
  auto put_reg = [&](int f, int cell, const R Fv[NV]) {
    R* p = freg + ((long)b * 6 + f) * NV * NFC + cell;
    asm volatile("" : "+v"(p));
#pragma unroll
    for (int q = 0; q < NV; ++q) p[q * NFC] = Fv[q];
  };
  const int job = T.job[b];
  const double ch = J.ch[job];
  const double idx = T.inv_dx[3 * b], idy = T.inv_dx[3 * b + 1], idz = T.inv_dx[3 * b + 2];
  const int lim = LIM >= 0 ? LIM : P.limiter;  // LIM < 0: a two-ghost-layer limiter
  const double lamx = lim == LIM_WENOZP5 ? 1.0 / cbrt(idx * idx) : 0.0;
  const double lamy = lim == LIM_WENOZP5 ? 1.0 / cbrt(idy * idy) : 0.0;
  const double lamz = (NDIM == 3 && lim == LIM_WENOZP5) ? 1.0 / cbrt(idz * idz) : 0.0;

  // face f (between cells f-1 and f) of line `line` along the plane's axis
  // AX, a face of direction D.  The five-cell reconstructions act on one
  // variable at a time, so each variable's six cells are read from LDS just
  // before use (a few live registers instead of all 54 values); the
  // arithmetic is that of the shared six-cell reconstruction.
  auto face = [&](auto ax, auto dir, int line, int f, double lambda, R Fq[NV]) {
    constexpr int AX = decltype(ax)::value;
    constexpr int D = decltype(dir)::value;
    auto at = [&](int s) {
      const int a = f - NG5 + s;
      return AX == 0 ? (line + NG5) * S5 + (a + NG5) : (a + NG5) * S5 + (line + NG5);
    };
    R wl[NV], wr[NV];
    if constexpr (LIM >= LIM_WENO5) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const R v0 = W[q][at(0)], v1 = W[q][at(1)], v2 = W[q][at(2)];
        const R v3 = W[q][at(3)], v4 = W[q][at(4)], v5 = W[q][at(5)];
        if constexpr (LIM == LIM_MP5) {
          wl[q] = mp5_face_r(v0, v1, v2, v3, v4);
          wr[q] = mp5_face_r(v5, v4, v3, v2, v1);
        } else {
          wl[q] = weno5_face_r(v0, v1, v2, v3, v4, lim, lambda);
          wr[q] = weno5_face_r(v5, v4, v3, v2, v1, lim, lambda);
        }
      }
      R cl[NV], cr[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        cl[q] = W[q][at(2)];
        cr[q] = W[q][at(3)];
      }
      positivity_fallback(wl, wr, cl, cr);
    } else {
      R c1[NV], c2[NV], c3[NV], c4[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        c1[q] = W[q][at(1)];
        c2[q] = W[q][at(2)];
        c3[q] = W[q][at(3)];
        c4[q] = W[q][at(4)];
      }
      reconstruct_face(lim, c1, c2, c3, c4, wl, wr);
    }
    face_flux<FLX, D, R>(wl, wr, (R)ch, (R)(0.5 / ch), (R)P.gamma, (R)P.inv_gm1, Fq);
  };
  using A0 = std::integral_constant<int, 0>;
  using A1 = std::integral_constant<int, 1>;
  using DX = std::integral_constant<int, 0>;
  using DY = std::integral_constant<int, 1>;
  using DZ = std::integral_constant<int, 2>;

  // Flux differences of one plane along its second axis (direction D2) and,
  // with FIRST, along its first axis (x): 16 x 17 faces per axis on 4 waves.
  // Along the first axis thread t = (i, j) evaluates the left face of cell
  // (i, j); along the second it evaluates the lower face of cell (j, i)
  // (transposed), so that in both directions the next face of a thread's
  // lies in the next lane of the same wave and reaches it by a lane shuffle.
  // The 17th faces go to lanes 0..15 of two waves that change with the
  // plane (first axis and second axis), through LDS: no wave takes more than
  // three face evaluations.  d1 (first axis) and d2 (second axis) are the
  // differences F(f+1) - F(f) of cell (i, j).
  // next - this of two face fluxes: at face precision, the energy's in FP64
  auto diff = [&](int q, R next, R f) -> double {
    return q == I_EN ? (double)next - (double)f : (double)(next - f);
  };
  constexpr bool kMixed = !std::is_same<R, double>::value;
  // pl: the plane's index along its normal (register cells pl * 16 + line)
  auto plane_differences = [&](auto first, auto dir2, double lam2, int pl, double d1[NV], double d2[NV]) {
    constexpr bool FIRST = decltype(first)::value;
    constexpr int D2 = decltype(dir2)::value;
    const int rofs = NDIM == 3 ? pl * BN5 : 0;
    R f1[NV], f2[NV];
    if constexpr (FIRST) {
      face(A0{}, DX{}, j, i, lamx, f1);
      if ((regs & 1u) && i == 0) put_reg(0, rofs + j, f1);
    }
    face(A1{}, dir2, j, i, lam2, f2);
    if ((regs & (1u << (2 * D2))) && i == 0) put_reg(2 * D2, rofs + j, f2);
    {
      // the 17th faces: first axis on wave pl % 4, second axis on wave
      // (pl + 2) % 4, so that the extra pass moves between the SIMDs from
      // plane to plane (with it always on waves 0 and 1 the 3D stage took
      // 3% (FP64) and 5% (FP32-mixed) longer)
      const int wv = t >> 6, ln = t & 63;
      const int xw = FIRST ? (pl & 3) : -1, yw = (pl + 2) & 3;
      if ((wv == xw || wv == yw) && ln < BN5) {
        R fe[NV];
        if (wv == xw) {
          if constexpr (FIRST) {
            face(A0{}, DX{}, ln, BN5, lamx, fe);
#pragma unroll
            for (int q = 0; q < NV; ++q) Ex[q][ln] = fe[q];
            if (regs & 2u) put_reg(1, rofs + ln, fe);
          }
        } else {
          face(A1{}, dir2, ln, BN5, lam2, fe);
#pragma unroll
          for (int q = 0; q < NV; ++q) Ey[q][ln] = fe[q];
          if (regs & (2u << (2 * D2))) put_reg(2 * D2 + 1, rofs + ln, fe);
        }
      }
    }
    __syncthreads();  // every face evaluated: W is free, Ex / Ey written
    const int up = (t & 63) + 1;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if constexpr (FIRST) {
        const R n1 = __shfl(f1[q], up, 64);
        d1[q] = diff(q, i < BN5 - 1 ? n1 : Ex[q][j], f1[q]);
      }
      const R n2 = __shfl(f2[q], up, 64);
      // second-axis difference of cell (j, i), handed to the thread that owns
      // it (the mixed energy's through a double array)
      const double dd = diff(q, i < BN5 - 1 ? n2 : Ey[q][j], f2[q]);
      if (kMixed && q == I_EN)
        De[i * NF5 + j] = dd;
      else
        W[q][i * NF5 + j] = (R)dd;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) d2[q] = (kMixed && q == I_EN) ? De[j * NF5 + i] : (double)W[q][j * NF5 + i];
  };
  // L + d / dx at face precision (the energy in FP64)
  auto accum = [&](int q, double Lq, double d, double id) -> double {
    if (!kMixed || q == I_EN) return Lq + d * id;
    return (double)((R)Lq + (R)d * (R)id);
  };
  using Yes = std::integral_constant<bool, true>;
  using No = std::integral_constant<bool, false>;

  // update of cell (x, y, z): L = -(sum_d dF_d / dx_d) - kappa psi; SSPRK combination
  const double dt = J.dt_scale * J.dt[job], kappa = J.kappa[job];
  void* o = block_ptr<SP>(out, b, PC);
  const void* bs = block_ptr<SP>(base, b, PC);
  // (the energy in FP64, the rest at face precision)
  auto update = [&](int x, int y, int z, const double L[NV]) {
    const long c = cell5(G, x, y, z);
    const double psi = SP::ld(own, I_PSI, c, PC);
    double un[NV];  // CFL: the output cell as a later load would see it
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double uq = SP::ld(own, q, c, PC);
      double res;
      if (q == I_EN) {
        const double tq = uq + dt * (-L[q]);
        if (W1) {
          res = tq;
        } else {
          const double u0 = SP::ld(bs, q, c, PC);
          res = u0 + wgt * (tq - u0);
        }
      } else {
        R lq = -(R)L[q];
        if (q == I_PSI) lq = lq - (R)kappa * (R)psi;
        const R tq = (R)uq + (R)dt * lq;
        if (W1) {
          res = (double)tq;
        } else {
          const R u0 = (R)SP::ld(bs, q, c, PC);
          res = (double)(u0 + (R)wgt * (tq - u0));
        }
      }
      SP::st(o, q, c, PC, res);
      if (CFL) un[q] = SP::as_stored(q, res);
    }
    if (CFL) {
      const unsigned cell_faces = (x == 0 ? 1u : 0u) | (x == BN5 - 1 ? 2u : 0u) | (y == 0 ? 4u : 0u) |
                                  (y == BN5 - 1 ? 8u : 0u) | (NDIM == 3 && z == 0 ? 16u : 0u) |
                                  (NDIM == 3 && z == BN5 - 1 ? 32u : 0u);
      if (!(cell_faces & skips)) {
        const double rate = cell_rate<NDIM>(un, P, idx, idy, idz, bad);
        if (isnan(rate))
          rnan = 1;
        else
          rmax = fmax(rmax, rate);
      }
    }
  };
  // the 192 in-plane halo cells of an x-y plane z: 48 per side, 3 layers of 16
  auto fetch_xy_halo = [&](int z, bool count) {
    if (t < 4 * NG5 * BN5) {
      const int side = t / (NG5 * BN5), r = t - side * (NG5 * BN5);
      if (side < 2) {
        const int y = r / NG5, a = r - y * NG5;
        const int x = side == 0 ? a - NG5 : BN5 + a;
        fetch(x, y, z, x, y, count);
      } else {
        const int x = r % BN5, a = r / BN5;
        const int y = side == 2 ? a - NG5 : BN5 + a;
        fetch(x, y, z, x, y, count);
      }
    }
  };

  if constexpr (NDIM == 2) {
    fetch(i, j, 0, i, j, true);
    fetch_xy_halo(0, true);
    __syncthreads();
    double d1[NV], d2[NV], L[NV];
    plane_differences(Yes{}, DY{}, lamy, 0, d1, d2);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      L[q] = 0.0;
      L[q] = accum(q, L[q], d1[q], idx);
      L[q] = accum(q, L[q], d2[q], idy);
    }
    update(i, j, 0, L);
  } else {
    // x-y planes: x and y differences of every cell into the scratch array
    // part[block][var][cell] (interior cells, x fastest)
    double* pb = part + (long)b * NV * (BN5 * BN5 * BN5);
    for (int k = 0; k < BN5; ++k) {
      fetch(i, j, k, i, j, true);
      fetch_xy_halo(k, false);
      __syncthreads();
      double d1[NV], d2[NV];
      plane_differences(Yes{}, DY{}, lamy, k, d1, d2);
      const int ci = (k * BN5 + j) * BN5 + i;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        double L = 0.0;
        L = accum(q, L, d1[q], idx);
        L = accum(q, L, d2[q], idy);
        pb[q * (BN5 * BN5 * BN5) + ci] = L;
      }
      __syncthreads();  // the plane's LDS is read before the next plane loads
    }
    // x-z planes: the z faces (the plane's second axis), then the update;
    // thread (i, j) of plane y owns cell (i, y, j)
    for (int y = 0; y < BN5; ++y) {
      fetch(i, y, j, i, j, false);
      if (t < 2 * NG5 * BN5) {  // the 96 z-halo cells: 3 layers of 16 below and above
        const int side = t / (NG5 * BN5), r = t - side * (NG5 * BN5);
        const int x = r % BN5, a = r / BN5;
        const int z = side == 0 ? a - NG5 : BN5 + a;
        fetch(x, y, z, x, z, false);
      }
      __syncthreads();
      double d1[NV], d2[NV], L[NV];
      plane_differences(No{}, DZ{}, lamz, y, d1, d2);
      const int ci = (j * BN5 + y) * BN5 + i;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        L[q] = pb[q * (BN5 * BN5 * BN5) + ci];
        L[q] = accum(q, L[q], d2[q], idz);
      }
      update(i, y, j, L);
      __syncthreads();
    }
  }
  if (CFL) {
    // workgroup max (wave max, then over the four waves in LDS), one atomic
    // per workgroup on the job's word (non-negative doubles order as their
    // bit patterns)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
    __shared__ double wmax[4];
    __shared__ int wnan[4];
    const int lane = t & 63, wave = t >> 6;
    const int anynan = __any(rnan);
    if (lane == 0) {
      wmax[wave] = rmax;
      wnan[wave] = anynan;
    }
    __syncthreads();
    if (t == 0) {
      const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
      atomicMax(&C.rate_bits[job], (unsigned long long)__double_as_longlong(m));
      if (wnan[0] | wnan[1] | wnan[2] | wnan[3]) atomicOr(&C.nan[job], 1u);
    }
  }
  if (bad) atomicOr(&st->flags, (unsigned)bad);
  if (nfix) atomicAdd(&st->nfix, (unsigned long long)nfix);
}

template <int ND, class SPT, bool W1, bool CF, int LIM, int FLX>
hipError_t f5_launch(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J, const void* in,
                     const void* base, void* out, double w, const PhysConst& P, DevStatus* st, double* pt,
                     void* freg, const JobCfl& C) {
  k_stage_fused5<ND, SPT, W1, CF, LIM, FLX><<<T.nactive, 256, 0, s>>>(
      G, T, J, in, base, out, w, P, st, pt, static_cast<typename SPT::R*>(freg), C);
  return hipGetLastError();
}

// the instance for (w == 1, CFL fold); the 3D stage does not fold the CFL
// rate (the runtime never asks it to), so those instances are not built
template <int ND, class SPT, int LIM, int FLX>
hipError_t f5_dispatch(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J, const void* in,
                       const void* base, void* out, double w, const PhysConst& P, DevStatus* st, double* pt,
                       void* freg, const JobCfl* cfl) {
  const JobCfl C = cfl ? *cfl : JobCfl{};
  const bool w1 = w == 1.0;
#define AMRVAC_F5_ARGS s, G, T, J, in, base, out, w, P, st, pt, freg, C
  if constexpr (ND == 3) {
    if (cfl) return hipErrorInvalidValue;
    return w1 ? f5_launch<3, SPT, true, false, LIM, FLX>(AMRVAC_F5_ARGS)
              : f5_launch<3, SPT, false, false, LIM, FLX>(AMRVAC_F5_ARGS);
  } else {
    if (w1)
      return cfl ? f5_launch<2, SPT, true, true, LIM, FLX>(AMRVAC_F5_ARGS)
                 : f5_launch<2, SPT, true, false, LIM, FLX>(AMRVAC_F5_ARGS);
    return cfl ? f5_launch<2, SPT, false, true, LIM, FLX>(AMRVAC_F5_ARGS)
               : f5_launch<2, SPT, false, false, LIM, FLX>(AMRVAC_F5_ARGS);
  }
#undef AMRVAC_F5_ARGS
}

template <int LIM, int FLX>
hipError_t f5_dispatch_lim(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                           const void* in, const void* base, void* out, double w, const PhysConst& P,
                           DevStatus* st, double* pt, void* freg, const JobCfl* cfl) {
  if (G.precision == 0)
    return G.ndim == 3 ? f5_dispatch<3, StoreF64, LIM, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl)
                       : f5_dispatch<2, StoreF64, LIM, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
  return G.ndim == 3 ? f5_dispatch<3, StoreMixed, LIM, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl)
                     : f5_dispatch<2, StoreMixed, LIM, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
}

// launch_fused5_stage for one flux: the limiter picks the instance
template <int FLX>
hipError_t launch_fused5_flux(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                              const void* in, const void* base, void* out, double w, const PhysConst& P,
                              DevStatus* st, double* part, void* freg, const JobCfl* cfl) {
  if (G.nx != BN5 || G.ng != NG5) return hipErrorInvalidValue;
  if (G.ndim == 3 && !part) return hipErrorInvalidValue;
  if (T.nactive <= 0) return hipSuccess;
  double* const pt = G.ndim == 3 ? part : nullptr;
  switch (P.limiter) {
    case LIM_WENO5:
      return f5_dispatch_lim<LIM_WENO5, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
    case LIM_WENOZ5:
      return f5_dispatch_lim<LIM_WENOZ5, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
    case LIM_MP5:
      return f5_dispatch_lim<LIM_MP5, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
    case LIM_WENOZP5:
      return f5_dispatch_lim<LIM_WENOZP5, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
    default:
      return f5_dispatch_lim<-1, FLX>(s, G, T, J, in, base, out, w, P, st, pt, freg, cfl);
  }
}

}  // namespace

// the per-flux launchers of fused5_hllc.hip and fused5_hlld.hip
hipError_t launch_fused5_hllc(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                              const void* in, const void* base, void* out, double w, const PhysConst& P,
                              DevStatus* st, double* part, void* freg, const JobCfl* cfl);
hipError_t launch_fused5_hlld(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                              const void* in, const void* base, void* out, double w, const PhysConst& P,
                              DevStatus* st, double* part, void* freg, const JobCfl* cfl);

}  // namespace amrvac
