// Fused stage kernel for 16^ndim blocks: conserved -> primitive, limited
// linear reconstruction (van Leer, Koren or Cada-Torrilhon), GLM interface +
// HLL (or HLLD, HLLC) fluxes in every direction, flux difference, psi damping and the SSPRK
// combination, in one launch.
//
// One 256-thread workgroup per block (or per z segment of a block); thread t
// owns the (x, y) column i = t % 16, j = t / 16, so that an x line of the
// block is one 16-lane row of a wave and a wave holds four lines.  In 3D
// the workgroup marches through the z planes: the z stencil lives in a
// per-thread register queue (primitives of plane k+1, the left face state of
// the next z face and the accumulated flux difference), while the x and y
// stencils of the current plane read one LDS plane of primitives with its
// 2-deep x/y halo.  Each face reads its four cells from the plane and forms
// the limited differences of its two cells itself.  Thread (i, j) evaluates
// the left x face and the lower y face of its cell; the right x face comes
// from the next lane of its row (a DPP row shift) and the upper y face from
// the same lane of the next line of its wave (a wave shuffle), so neither
// face fluxes nor slopes go through LDS.  Only the faces that leave a wave
// are exchanged in LDS: the 17th face of every x line and y column (done by
// two waves per plane) and the y faces of the first line of each wave.  Two
// workgroup barriers per plane: the plane is complete, the faces are done.
// Halo cells across faces shared with a same-level leaf are read directly
// from that neighbour's interior; only faces towards finer or coarser
// leaves and physical boundaries need filled ghost cells.
#include "kernels.h"

namespace amrvac {

namespace {

constexpr int BN = 16;          // block cells per direction
constexpr int BP = BN + 4;      // padded extent
// LDS row stride of the plane, one value longer than the data so that the
// strided 17th-face accesses of 16 lanes hit distinct banks
constexpr int WROW = BP + 1;
constexpr int PLANE = BP * WROW;  // LDS values per variable of one plane

// Workgroup barrier that orders LDS accesses only.  Every exchange between
// the threads of a workgroup in this kernel goes through LDS, so global loads
// in flight (the z-plane prefetch, the halo staging) stay in flight across it
// instead of being drained as a full fence would.
// (The compiler-level memory clobbers keep LDS accesses on their side; the
// wait makes this wave's LDS writes complete before it arrives.)
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt untouched
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int NDIM>
struct Pad {
  static constexpr long cells = NDIM == 3 ? (long)BP * BP * BP : (long)BP * BP;
  __device__ static constexpr long at(int i, int j, int k) {
    return ((long)(NDIM == 3 ? k + 2 : 0) * BP + (j + 2)) * BP + (i + 2);
  }
};

template <class SP>
__device__ __forceinline__ void load_cons(const void* __restrict__ U, long pc, long c, double u[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) u[q] = SP::ld(U, q, c, pc);
}

// Interface flux along DIR of the face between the LDS plane cells base + s
// and base + 2 s, from the four cells base, base + s, base + 2 s, base + 3 s
// of its line (i-2 .. i+1): both cells' limited differences, the face
// states, the first-order fallback where rho or p is not positive on either
// side (the two cells are re-read only in waves where some lane needs
// them), then the GLM + HLL / HLLD / HLLC flux.
template <int DIR, int LIM, int FLX, class R>
__device__ __forceinline__ void lds_face(const R (*__restrict__ Wp)[PLANE], int base, int s,
                                         R ch, R hic, R gamma, R inv_gm1, R F[NV]) {
  R wl[NV], wr[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const R a = Wp[q][base], b = Wp[q][base + s], c = Wp[q][base + 2 * s], d = Wp[q][base + 3 * s];
    R rb, lb, rc, lc;
    cell_increments<LIM>(b - a, c - b, rb, lb);
    cell_increments<LIM>(c - b, d - c, rc, lc);
    wl[q] = b + R(0.5) * rb;
    wr[q] = c - R(0.5) * lc;
  }
  const bool bad = !((wl[I_RHO] > R(0)) && (wl[4] > R(0)) && (wr[I_RHO] > R(0)) && (wr[4] > R(0)));
  if (__any(bad)) {
    asm volatile("");  // keeps the branch wave-uniform
    if (bad) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        wl[q] = Wp[q][base + s];
        wr[q] = Wp[q][base + 2 * s];
      }
    }
  }
  face_flux<FLX, DIR, R>(wl, wr, ch, hic, gamma, inv_gm1, F);
}

// The value of the next lane of this lane's 16-lane row (a DPP row shift;
// the last lane of a row gets 0).
__device__ __forceinline__ float row_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, false));
}
__device__ __forceinline__ double row_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x101, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Halo cell h (0..127) of a plane's x/y stencil: h < 64 are the x-halo
// cells (x = -2, -1, 16, 17 of row h / 4), the rest the y-halo rows
// (y = -2, -1, 16, 17, x = h % 16).  Cells 2m and 2m+1 are neighbours in x.
struct HaloXY {
  int x, y;
};
__device__ __forceinline__ HaloXY halo_cell(int h) {
  const bool xh = h < 64;
  const int o = xh ? (h & 3) : ((h >> 4) & 3);
  const int edge = o < 2 ? o - 2 : BN + o - 2;
  return HaloXY{xh ? edge : (h & 15), xh ? (h >> 2) : edge};
}

// LDS address of a __shared__ object, for the direct global->LDS loads
template <class T>
__device__ __forceinline__ __attribute__((address_space(3))) void* lds_addr(T* p) {
  return (__attribute__((address_space(3))) void*)p;
}

// Face-arithmetic constants of one launch, in the face precision.
template <class R>
struct FaceConst {
  R ch, hic, gamma, inv_gm1;
};

// Waves per SIMD the stage is built for: FP64 3D holds the z queue beside a
// face evaluation (two waves, 230-256 VGPRs); in 2D there is no z queue and
// three waves fit (at most 168 VGPRs; measured on the 6-level Alfven
// shock-cloud grid with HLLD, 0.79 against 0.83 ms per step, HLL and HLLC
// unchanged).
template <class SP>
constexpr int kWavesPerEU2D = SP::kWavesPerEU < 3 ? 3 : SP::kWavesPerEU;

// W1: the stage weight is 1 (out = in + dt L(in)), so base is not read.
// CFL: also fold the CFL rate of every output cell into the job's running
// maximum (C.rate_bits, C.nan), as the time-step pass would from out.
// Work item w (one z segment of one block) is run by workgroup g with
// w = (g % 8) * per_xcd + g / 8 when tune.xcd is set (each XCD gets a
// contiguous run of the Morton-ordered list), else w = g.
template <int NDIM, class SP, bool W1, bool CFL, int LIM, int FLX, bool REG>
__global__ void __launch_bounds__(256, NDIM == 2 ? kWavesPerEU2D<SP> : SP::kWavesPerEU)
k_stage_fused(GridConst G, Tables T, JobScalars J, FusedTune tune, int per_xcd, const void* __restrict__ in,
              const void* base, void* out, double wgt, PhysConst P, DevStatus* st, JobCfl C,
              typename SP::R* __restrict__ freg) {
  using R = typename SP::R;
  using PD = Pad<NDIM>;
  constexpr long PC = PD::cells;
  __shared__ R Wp[NV][PLANE];    // primitives of the current plane (+ x/y halo)
  __shared__ R Xf[NV][2 * BN];   // 17th faces: x face 16 of line j at j, y face 16 of column i at 16 + i
  __shared__ R Bd[3][NV][BN];    // y faces of the first line of waves 1..3 (the next line of waves 0..2)
  // LDS staging of the next plane's 128 halo cells (3D; conserved, storage
  // precision), written by direct global->LDS loads (global_load_lds) of one
  // wave while the current plane is computed, so the halo's memory latency
  // is off the critical path.  One such load of a wave writes 64 consecutive
  // lane slots: 16 bytes (cells 2m, 2m+1 of a double array) or 4 bytes (cell
  // m of a float array).
  // (Only the arrays of the instantiation's storage are referenced; the
  // others are dropped.  Their sizes are not template-dependent, which
  // clang's host pass needs for the 16-byte form of the builtin.)
  constexpr bool kF64 = SP::kBytesPerCell == 72;
  __shared__ double HsD[NV * 128];     // FP64 state, [var][cell]
  __shared__ float HsF[(NV - 1) * 128];  // mixed: rho, m, B, psi
  __shared__ double HsE[128];          // mixed: e

  // Workgroups are dealt to the 8 XCDs round-robin; with tune.xcd each XCD
  // gets a contiguous run of the Morton-ordered block list so that
  // neighbouring blocks (and the segments of one block) share one L2.
  const int wi = tune.xcd ? (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  const int nseg = NDIM == 3 ? tune.zseg : 1;
  const int slot = wi / nseg;
  if (slot >= T.nactive) return;
  const int seg = wi - slot * nseg;
  const int b = T.order[slot];
  const int t = threadIdx.x;
  const int i = t & 15, j = t >> 4;
  const void* __restrict__ U = block_ptr<SP>(in, b, PC);
  // Halo source per face: a same-level neighbour is read in place (its
  // interior, shifted by one block); other faces use this block's ghost
  // cells, filled by the ghost kernels.
  // (named scalars, not arrays: the per-lane selects below would otherwise
  // turn an array into scratch memory)
  auto face_src = [&](int f) {
    const int* Lk = T.link + ((long)b * 6 + f) * LINK_INTS;
    return Lk[0] == LINK_SAME ? Lk[1] : b;
  };
  auto face_shift = [&](int f) {
    const int* Lk = T.link + ((long)b * 6 + f) * LINK_INTS;
    return Lk[0] == LINK_SAME ? ((f & 1) ? -BN : BN) : 0;
  };
  const int sb0 = face_src(0), sb1 = face_src(1), sb2 = face_src(2), sb3 = face_src(3);
  const int sh0 = face_shift(0), sh1 = face_shift(1), sh2 = face_shift(2), sh3 = face_shift(3);
  // Flux registers of the faces towards finer or coarser leaves (freg is
  // null when no coarse/fine correction follows): the face fluxes evaluated
  // there are stored for the correction pass, [face][var][face cell] of this
  // block; bit f of regs marks face f.  With CFL and C.skip_fine the cells
  // next to faces towards finer leaves (bit f of skips) are left to the pass
  // after that correction.
  constexpr int NFC = NDIM == 3 ? BN * BN : BN;
  // (REG: the instantiation for grids with coarse/fine correction; freg is
  // then not null)
  unsigned regs = 0, skips = 0;
  if constexpr (REG) {
#pragma unroll
    for (int f = 0; f < 2 * NDIM; ++f) {
      const int kd = T.link[((long)b * 6 + f) * LINK_INTS];
      if (kd == LINK_FINE || kd == LINK_COARSE) regs |= 1u << f;
      if (CFL && C.skip_fine && kd == LINK_FINE) skips |= 1u << f;
    }
  }
  R* const rgb = freg + (long)b * 6 * NV * NFC;
  // store the NV fluxes of one face cell; the address is formed here (the
  // empty asm keeps the compiler from hoisting nine addresses per face out
  // of the plane loop, which would cost registers the stage does not have)
  auto put_reg = [&](int f, int cell, const R Fv[NV]) {
    R* p = rgb + f * NV * NFC + cell;
    asm volatile("" : "+v"(p));
#pragma unroll
    for (int q = 0; q < NV; ++q) p[q * NFC] = Fv[q];
  };
  const int job = T.job[b];
  const double dt = J.dt_scale * J.dt[job], kappa = J.kappa[job], chd = J.ch[job];
  const FaceConst<R> K{(R)chd, (R)(0.5 / chd), (R)P.gamma, (R)P.inv_gm1};
  const double idx = T.inv_dx[3 * b], idy = T.inv_dx[3 * b + 1], idz = T.inv_dx[3 * b + 2];
  const R idzr = (R)idz;
  int bad = 0;
  unsigned nfix = 0;
  double rmax = 0.0;  // CFL: running max of this thread's output cells
  int rnan = 0;

  // Halo cell of this thread for the x/y stencil of a plane: 128 cells, done
  // by threads 0..127 on planes of parity 0 and by threads 128..255 on planes
  // of parity 1, where a plane's parity is 0 unless tune.rot is set.
  const HaloXY hc = halo_cell(t & 127);
  const int hx = hc.x, hy = hc.y;
  const int hpar = t >> 7;
  // source block of halo cell (x, y) and the cell's index there in plane p
  struct HaloSrc {
    const void* blk;
    long cell0;  // padded index of the cell in plane 0
  };
  auto halo_src = [&](HaloXY c) {
    const bool xlo = c.x < 0, xhi = c.x >= BN, ylo = c.y < 0;
    const int sb = xlo ? sb0 : (xhi ? sb1 : (ylo ? sb2 : sb3));
    const int xs = c.x + (xlo ? sh0 : (xhi ? sh1 : 0));
    const int ys = c.y + (xlo || xhi ? 0 : (ylo ? sh2 : sh3));
    return HaloSrc{block_ptr<SP>(in, sb, PC), PD::at(xs, ys, 0)};
  };
  // padded cells between consecutive z planes
  constexpr long PLANE = (long)BP * BP;
  const HaloSrc hs = halo_src(hc);
  // wave 3 stages the next plane's halo (3D).  Lane m's sources in plane 0:
  // FP64, the pair 2m, 2m+1 of every variable; mixed, float cells m and
  // 64 + m and the energy pair 2m, 2m+1.
  const double* stg_d = nullptr;
  const float *stg_f1 = nullptr, *stg_f2 = nullptr;
  if (NDIM == 3) {
    const int m = t & 63;
    const HaloSrc a = halo_src(halo_cell(2 * m));
    if constexpr (kF64) {
      stg_d = static_cast<const double*>(a.blk) + a.cell0;
    } else {
      const HaloSrc s1 = halo_src(halo_cell(m)), s2 = halo_src(halo_cell(64 + m));
      stg_f1 = static_cast<const float*>(s1.blk) + s1.cell0;
      stg_f2 = static_cast<const float*>(s2.blk) + s2.cell0;
      stg_d = reinterpret_cast<const double*>(static_cast<const char*>(a.blk) + 32 * PC) + a.cell0;
    }
  }
  const bool stager = NDIM == 3 && t >= 192;
  auto stage_halo = [&](int p) {
    const long off = p * PLANE;
    if constexpr (kF64) {
#pragma unroll
      for (int q = 0; q < NV; ++q)
        __builtin_amdgcn_global_load_lds(stg_d + off + q * PC, lds_addr(&HsD[q * 128]), 16, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < NV - 1; ++q) {
        __builtin_amdgcn_global_load_lds(stg_f1 + off + q * PC, lds_addr(&HsF[q * 128]), 4, 0, 0);
        __builtin_amdgcn_global_load_lds(stg_f2 + off + q * PC, lds_addr(&HsF[q * 128 + 64]), 4, 0, 0);
      }
      __builtin_amdgcn_global_load_lds(stg_d + off, lds_addr(&HsE[0]), 16, 0, 0);
    }
  };
  // staged conserved values of halo cell h
  auto staged = [&](int h, double u[NV]) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if constexpr (kF64)
        u[q] = HsD[q * 128 + h];
      else
        u[q] = q == I_EN ? HsE[h] : (double)HsF[StoreMixed::fidx(q) * 128 + h];
    }
  };
  // z ghost planes come from faces 4 (below) and 5 (above)
  const void* __restrict__ Uzlo = block_ptr<SP>(in, NDIM == 3 ? face_src(4) : b, PC);
  const void* __restrict__ Uzhi = block_ptr<SP>(in, NDIM == 3 ? face_src(5) : b, PC);
  const int shzlo = NDIM == 3 ? face_shift(4) : 0, shzhi = NDIM == 3 ? face_shift(5) : 0;

  auto convert = [&](const double u[NV], R w[NV]) {
    const int bb = cons_to_prim(u, w, P);
    if (bb) {
      bad |= bb;
      if (P.fix) ++nfix;
    }
  };

  // z pipeline (3D).  Registers carry wb = W(k+1), wla = the left state of
  // face k+1/2 (W(k) + sigma(k)/2) and acc, which enters plane k already
  // holding the contribution -F_z(k-1/2)/dz of the face below; W(k) itself
  // sits in this thread's cell of the LDS plane.
  // This workgroup marches planes k0 .. k1-1 (the whole block unless the z
  // range is split into segments).
  const int klen = BN / nseg;
  const int k0 = NDIM == 3 ? seg * klen : 0;
  const int k1 = NDIM == 3 ? k0 + klen : 1;
  // conserved state of this thread's column at plane p, -2 <= p < BN + 2
  auto load_z = [&](int p, double u[NV]) {
    if (p < 0)
      load_cons<SP>(Uzlo, PC, PD::at(i, j, p + shzlo), u);
    else if (p >= BN)
      load_cons<SP>(Uzhi, PC, PD::at(i, j, p + shzhi), u);
    else
      load_cons<SP>(U, PC, PD::at(i, j, p), u);
  };
  R wb[NV], wla[NV], acc[NV];
  double acc_e = 0.0;
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = R(0);
  {
    double u[NV];
    R wa[NV];
    load_cons<SP>(U, PC, PD::at(i, j, k0), u);
    convert(u, wa);
#pragma unroll
    for (int q = 0; q < NV; ++q) Wp[q][(j + 2) * WROW + (i + 2)] = wa[q];
    if (NDIM == 3) {
      R wm2[NV], wm1[NV];
      load_z(k0 - 2, u);
      convert(u, wm2);
      load_z(k0 - 1, u);
      convert(u, wm1);
      load_z(k0 + 1, u);
      convert(u, wb);
      R wl[NV], wr[NV], fz[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        R rm, lm, r0, l0;
        cell_increments<LIM>(wm1[q] - wm2[q], wa[q] - wm1[q], rm, lm);
        cell_increments<LIM>(wa[q] - wm1[q], wb[q] - wa[q], r0, l0);
        wl[q] = wm1[q] + R(0.5) * rm;
        wr[q] = wa[q] - R(0.5) * l0;
        wla[q] = wa[q] + R(0.5) * r0;
      }
      positivity_fallback(wl, wr, wm1, wa);
      face_flux<FLX, 2, R>(wl, wr, K.ch, K.hic, K.gamma, K.inv_gm1, fz);
      if ((regs & 16u) && k0 == 0) put_reg(4, j * BN + i, fz);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        if (q == I_EN) {
          const double d = (double)fz[q] * idz;
          acc_e = -d;
        } else {
          const R d = fz[q] * idzr;
          acc[q] = -d;
        }
      }
    }
  }

  // halo parity of plane k: halo cells are converted by threads 0..127 on
  // planes of parity 0 and by 128..255 on planes of parity 1
  auto parity = [&](int k) { return tune.rot ? ((k + slot) & 1) : 0; };
  // plane k0's halo straight from memory
  if (hpar == parity(k0)) {
    double u[NV];
    R w[NV];
    load_cons<SP>(hs.blk, PC, hs.cell0 + k0 * PLANE, u);
    convert(u, w);
#pragma unroll
    for (int q = 0; q < NV; ++q) Wp[q][(hy + 2) * WROW + (hx + 2)] = w[q];
  }

  for (int k = k0; k < k1; ++k) {
    // prefetch the conserved state of plane k+2 (consumed by the z step)
    double uc[NV];
    if (NDIM == 3) load_z(k + 2, uc);

    // who does this plane's extra work: the halo cells of the next plane go
    // to the threads of that plane's parity (waves 0, 1 or 2, 3), the 17th x
    // faces to wave xw and the 17th y faces to wave yw, the other two waves;
    // with tune.rot the pairs alternate with the plane
    const int xw = parity(k + 1) ? 0 : 2, yw = xw + 1;
    const int wave = t >> 6;
    const int kofs = NDIM == 3 ? k * BN : 0;  // register cells of this plane's x and y faces

    // plane k's primitives (own cells and halo) are complete in LDS, and the
    // staging buffer and the previous plane's exchanged faces have been read
    lds_barrier();
    const bool staging = stager && k + 1 < k1;
    if (staging) stage_halo(k + 1);

    // the 17th faces: x face 16 of line l (cells 14 .. 17) by lane l of wave
    // xw, y face 16 of column l by lane l of wave yw
    {
      const int l = t & 63;
      if (wave == xw && l < BN) {
        R F[NV];
        lds_face<0, LIM, FLX, R>(Wp, (l + 2) * WROW + BN, 1, K.ch, K.hic, K.gamma, K.inv_gm1, F);
#pragma unroll
        for (int q = 0; q < NV; ++q) Xf[q][l] = F[q];
        if (regs & 2u) put_reg(1, kofs + l, F);
      }
      if (wave == yw && l < BN) {
        R F[NV];
        lds_face<1, LIM, FLX, R>(Wp, BN * WROW + l + 2, WROW, K.ch, K.hic, K.gamma, K.inv_gm1, F);
#pragma unroll
        for (int q = 0; q < NV; ++q) Xf[q][BN + l] = F[q];
        if (regs & 8u) put_reg(3, kofs + l, F);
      }
    }
    // x: the left face of this cell (cells i-2 .. i+1 of line j); its right
    // face is the next lane's left face (lane 15: the 17th face, from LDS).
    // dX = F(i+1) - F(i) (the energy's in double); lane 15 holds -F(i)
    // until the barrier, then adds F(16): the same difference, bit for bit.
    R dX[NV];
    double dXe;
    {
      R F[NV];
      lds_face<0, LIM, FLX, R>(Wp, (j + 2) * WROW + i, 1, K.ch, K.hic, K.gamma, K.inv_gm1, F);
      if ((regs & 1u) && i == 0) put_reg(0, kofs + j, F);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const R hi = row_next(F[q]);
        if (q == I_EN)
          dXe = (double)hi - (double)F[q];
        else
          dX[q] = hi - F[q];
      }
    }
    // y: the lower face of this cell (cells j-2 .. j+1 of column i); its
    // upper face is the lower face of the same lane of the next line of the
    // wave, or for a wave's last line that of the next wave's first line
    // (exchanged in LDS) or the 17th face; that line holds -F(j) until the
    // barrier
    R dY[NV];
    double dYe;
    {
      R F[NV];
      lds_face<1, LIM, FLX, R>(Wp, j * WROW + i + 2, WROW, K.ch, K.hic, K.gamma, K.inv_gm1, F);
      if ((regs & 4u) && j == 0) put_reg(2, kofs + i, F);
      const bool last = (j & 3) == 3;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const R up = __shfl_down(F[q], BN, 64);
        const R hi = last ? R(0) : up;
        if (q == I_EN)
          dYe = (double)hi - (double)F[q];
        else
          dY[q] = hi - F[q];
      }
      if ((j & 3) == 0 && wave > 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Bd[wave - 1][q][i] = F[q];
      }
    }
    // a wave with direct global->LDS loads in flight completes them before the
    // barrier that publishes them (vmcnt(0); expcnt and lgkmcnt untouched)
    if (staging) __builtin_amdgcn_s_waitcnt(0x0F70);
    // every face of the plane is done and exchanged
    lds_barrier();
    if (i == BN - 1) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        if (q == I_EN)
          dXe = (double)Xf[q][j] + dXe;
        else
          dX[q] = Xf[q][j] + dX[q];
      }
    }
    if ((j & 3) == 3) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const R hi = wave < 3 ? Bd[wave][q][i] : Xf[q][BN + i];
        if (q == I_EN)
          dYe = (double)hi + dYe;
        else
          dY[q] = hi + dY[q];
      }
    }
    // flux differences over dx, x then y (the energy in double)
    {
      const R idxr = (R)idx, idyr = (R)idy;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        if (q == I_EN) {
          acc_e = acc_e + dXe * idx;
          acc_e = acc_e + dYe * idy;
        } else {
          acc[q] = acc[q] + dX[q] * idxr;
          acc[q] = acc[q] + dY[q] * idyr;
        }
      }
    }

    // this plane's conserved state and the stage base, issued as one group
    const long c = PD::at(i, j, k);
    double u[NV], ub[NV];

    // ---- z direction (registers; W(k) from this thread's LDS cell, which
    // no other thread reads after the last barrier of the plane)
    R fz[NV];
    double fze = 0.0;
    if (NDIM == 3) {
      R wa[NV], wc[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) wa[q] = Wp[q][(j + 2) * WROW + (i + 2)];
      convert(uc, wc);
      R wl[NV], wr[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        R r1, l1;
        cell_increments<LIM>(wb[q] - wa[q], wc[q] - wb[q], r1, l1);
        wl[q] = wla[q];
        wr[q] = wb[q] - R(0.5) * l1;
        wla[q] = wb[q] + R(0.5) * r1;
      }
      positivity_fallback(wl, wr, wa, wb);
      face_flux<FLX, 2, R>(wl, wr, K.ch, K.hic, K.gamma, K.inv_gm1, fz);
      if ((regs & 32u) && k == BN - 1) put_reg(5, j * BN + i, fz);
      // fz becomes F_z(k+1/2)/dz (the energy term in double, in fze); it is
      // added here and its negative seeds the next plane's accumulator
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        if (q == I_EN) {
          fze = (double)fz[q] * idz;
          acc_e = acc_e + fze;
        } else {
          fz[q] = fz[q] * idzr;
          acc[q] = acc[q] + fz[q];
        }
        // W(k+1) goes into this thread's LDS cell for the next plane
        Wp[q][(j + 2) * WROW + (i + 2)] = wb[q];
        wb[q] = wc[q];
      }
    }

    // ---- update: L = -(sum_d dF_d / dx_d) - kappa psi; SSPRK combination
    // (the energy in double, the rest in the face precision)
    load_cons<SP>(U, PC, c, u);
    if (!W1) load_cons<SP>(block_ptr<SP>(base, b, PC), PC, c, ub);
    // (out may be the base slot: each cell is read before it is written, by
    // the same thread)
    void* o = block_ptr<SP>(out, b, PC);
    double un[NV];  // CFL: the output cell as a later load would see it
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double res;
      if (q == I_EN) {
        const double tq = u[q] + dt * (-acc_e);
        res = W1 ? tq : ub[q] + wgt * (tq - ub[q]);
      } else {
        R lq = -acc[q];
        if (q == I_PSI) lq = lq - (R)kappa * (R)u[I_PSI];
        const R tq = (R)u[q] + (R)dt * lq;
        if (W1) {
          res = (double)tq;
        } else {
          const R u0 = (R)ub[q];
          res = (double)(u0 + (R)wgt * (tq - u0));
        }
      }
      SP::st(o, q, c, PC, res);
      if (CFL) un[q] = SP::as_stored(q, res);
    }
    // (bit f of the cell's faces: the block faces it touches)
    const unsigned cell_faces = (i == 0 ? 1u : 0u) | (i == BN - 1 ? 2u : 0u) | (j == 0 ? 4u : 0u) |
                                (j == BN - 1 ? 8u : 0u) | (NDIM == 3 && k == 0 ? 16u : 0u) |
                                (NDIM == 3 && k == BN - 1 ? 32u : 0u);
    if (CFL && !(cell_faces & skips)) {
      const double rate = cell_rate<NDIM>(un, P, idx, idy, idz, bad);
      if (isnan(rate))
        rnan = 1;
      else
        rmax = fmax(rmax, rate);
    }
    if (NDIM == 3) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        if (q == I_EN)
          acc_e = -fze;
        else
          acc[q] = -fz[q];
      }
      // ---- plane k+1 halo: staged conserved values -> primitives in LDS
      // (no thread reads this plane's halo after its last barrier)
      if (k + 1 < k1 && hpar == parity(k + 1)) {
        double uh[NV];
        R w[NV];
        staged(t & 127, uh);
        convert(uh, w);
#pragma unroll
        for (int q = 0; q < NV; ++q) Wp[q][(hy + 2) * WROW + (hx + 2)] = w[q];
      }
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
    lds_barrier();
    if (t == 0) {
      const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
      atomicMax(&C.rate_bits[job], (unsigned long long)__double_as_longlong(m));
      if (wnan[0] | wnan[1] | wnan[2] | wnan[3]) atomicOr(&C.nan[job], 1u);
    }
  }
  if (bad) atomicOr(&st->flags, (unsigned)bad);
  if (nfix) atomicAdd(&st->nfix, (unsigned long long)nfix);
}

}  // namespace

hipError_t launch_fused_stage(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                              const FusedTune& tune, const void* in, const void* base, void* out, double w,
                              const PhysConst& P, DevStatus* st, const JobCfl* cfl, void* freg) {
  if (G.nx != BN || G.ng != 2) return hipErrorInvalidValue;
  if (tune.zseg != 1 && tune.zseg != 2 && tune.zseg != 4) return hipErrorInvalidValue;
  if (T.nactive <= 0) return hipSuccess;
  const long items = (long)T.nactive * (G.ndim == 3 ? tune.zseg : 1);
  const int per_xcd = (int)((items + 7) / 8);
  const unsigned grid = tune.xcd ? 8u * (unsigned)per_xcd : (unsigned)items;
  const JobCfl C = cfl ? *cfl : JobCfl{};
#define AMRVAC_FUSED_KERNEL(ND, SPT, W1, CF, LM, FX)                                                         \
  do {                                                                                                      \
    if (freg)                                                                                               \
      k_stage_fused<ND, SPT, W1, CF, LM, FX, true><<<grid, 256, 0, s>>>(G, T, J, tune, per_xcd, in, base, out, w, \
                                                                         P, st, C, static_cast<SPT::R*>(freg)); \
    else                                                                                                    \
      k_stage_fused<ND, SPT, W1, CF, LM, FX, false><<<grid, 256, 0, s>>>(G, T, J, tune, per_xcd, in, base, out,  \
                                                                          w, P, st, C, nullptr);            \
  } while (0)
#define AMRVAC_FUSED_LAUNCH(ND, SPT, LM, FX)               \
  do {                                                     \
    if (cfl) {                                             \
      if (w == 1.0)                                        \
        AMRVAC_FUSED_KERNEL(ND, SPT, true, true, LM, FX);  \
      else                                                 \
        AMRVAC_FUSED_KERNEL(ND, SPT, false, true, LM, FX); \
    } else {                                               \
      if (w == 1.0)                                        \
        AMRVAC_FUSED_KERNEL(ND, SPT, true, false, LM, FX); \
      else                                                 \
        AMRVAC_FUSED_KERNEL(ND, SPT, false, false, LM, FX); \
    }                                                      \
  } while (0)
#define AMRVAC_FUSED_FLUX(ND, SPT, LM)                 \
  do {                                                 \
    if (P.flux == FLUX_HLLD)                           \
      AMRVAC_FUSED_LAUNCH(ND, SPT, LM, FLUX_HLLD);     \
    else if (P.flux == FLUX_HLLC)                      \
      AMRVAC_FUSED_LAUNCH(ND, SPT, LM, FLUX_HLLC);     \
    else                                               \
      AMRVAC_FUSED_LAUNCH(ND, SPT, LM, FLUX_HLL);      \
  } while (0)
#define AMRVAC_FUSED_LIMITER(ND, SPT)                 \
  do {                                                \
    if (P.limiter == LIM_KOREN)                       \
      AMRVAC_FUSED_FLUX(ND, SPT, LIM_KOREN);          \
    else if (P.limiter == LIM_CADA3)                  \
      AMRVAC_FUSED_FLUX(ND, SPT, LIM_CADA3);          \
    else                                              \
      AMRVAC_FUSED_FLUX(ND, SPT, LIM_VANLEER);        \
  } while (0)
  if (G.precision == 0) {
    if (G.ndim == 3)
      AMRVAC_FUSED_LIMITER(3, StoreF64);
    else
      AMRVAC_FUSED_LIMITER(2, StoreF64);
  } else {
    if (G.ndim == 3)
      AMRVAC_FUSED_LIMITER(3, StoreMixed);
    else
      AMRVAC_FUSED_LIMITER(2, StoreMixed);
  }
#undef AMRVAC_FUSED_LIMITER
#undef AMRVAC_FUSED_FLUX
#undef AMRVAC_FUSED_LAUNCH
#undef AMRVAC_FUSED_KERNEL
  return hipGetLastError();
}

}  // namespace amrvac
