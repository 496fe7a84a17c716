// Device-side ideal GLM-MHD arithmetic for gfx950 (register-resident, fully
// unrolled; the face direction is a template parameter so component
// selection costs nothing).
//
// Scheme (MPI-AMRVAC 3.0, arXiv 2303.03026): conservative finite volumes
// ("Schemes and limiters for HD and MHD"), 'vanleer' slopes on primitive
// variables (Table t:limiters), HLL fluxes (Table tab:schemes_space), 'glm'
// divergence control after Dedner et al. 2002 (Table t:divb), small-value
// checks on entry to conserved->primitive ("Bootstrapping" section).
#pragma once

#include <hip/hip_runtime.h>

namespace amrvac {

constexpr int NV = 9;
// conserved slots; primitives reuse them with v in 1..3 and p in 4
enum { I_RHO = 0, I_MX = 1, I_MY = 2, I_MZ = 3, I_EN = 4, I_BX = 5, I_BY = 6, I_BZ = 7, I_PSI = 8 };
enum { F_SMALL_RHO = 1, F_SMALL_P = 2, F_BAD_DT = 4 };

// Per-launch physical constants (by value in kernel arguments).
struct PhysConst {
  double gamma;
  double gm1;      // gamma - 1
  double inv_gm1;  // 1 / (gamma - 1)
  double small_rho;
  double small_p;
  int fix;
};

// Library-owned device status record.
struct DevStatus {
  unsigned int flags;
  unsigned int cfl_nan;  // a NaN rate was met by the running CFL reduction
  unsigned long long nfix;
  unsigned long long rate_bits;  // max CFL rate (non-negative double bits)
  double last_dt;
};

// Lean FP64 reciprocal, quotient and square root for the normal-range
// operands of this scheme (no denormal or overflow scaling): a hardware
// seed (v_rcp_f64 / v_rsq_f64) refined by Newton steps to about one ulp.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(e, r, r);
  e = fma(-x, r, 1.0);
  return fma(e, r, r);
}

__device__ __forceinline__ double div64(double a, double b) {
  const double r = rcp64(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

__device__ __forceinline__ double sqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, x), h, g);
  return x > 0.0 ? g : 0.0;
}

// conserved -> primitive; returns the small-value bits of this cell.  With
// the fix on, density is floored first (velocity uses the floored value),
// then pressure; conserved values and B are never changed.
__device__ __forceinline__ int cons_to_prim(const double u[NV], double w[NV], const PhysConst& P) {
  int bad = 0;
  double rho = u[I_RHO];
  if (!(rho > P.small_rho)) {
    bad |= F_SMALL_RHO;
    if (P.fix) rho = P.small_rho;
  }
  const double ri = rcp64(rho);
  w[I_RHO] = rho;
  w[1] = u[I_MX] * ri;
  w[2] = u[I_MY] * ri;
  w[3] = u[I_MZ] * ri;
  const double m2 = u[I_MX] * u[I_MX] + u[I_MY] * u[I_MY] + u[I_MZ] * u[I_MZ];
  const double b2 = u[I_BX] * u[I_BX] + u[I_BY] * u[I_BY] + u[I_BZ] * u[I_BZ];
  double p = P.gm1 * (u[I_EN] - 0.5 * m2 * ri - 0.5 * b2);
  if (!(p > P.small_p)) {
    bad |= F_SMALL_P;
    if (P.fix) p = P.small_p;
  }
  w[4] = p;
  w[I_BX] = u[I_BX];
  w[I_BY] = u[I_BY];
  w[I_BZ] = u[I_BZ];
  w[I_PSI] = u[I_PSI];
  return bad;
}

__device__ __forceinline__ void prim_to_cons(const double w[NV], double u[NV], const PhysConst& P) {
  const double rho = w[I_RHO];
  u[I_RHO] = rho;
  u[I_MX] = rho * w[1];
  u[I_MY] = rho * w[2];
  u[I_MZ] = rho * w[3];
  const double v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  const double b2 = w[I_BX] * w[I_BX] + w[I_BY] * w[I_BY] + w[I_BZ] * w[I_BZ];
  u[I_EN] = w[4] * P.inv_gm1 + 0.5 * rho * v2 + 0.5 * b2;
  u[I_BX] = w[I_BX];
  u[I_BY] = w[I_BY];
  u[I_BZ] = w[I_BZ];
  u[I_PSI] = w[I_PSI];
}

// van Leer's harmonic-mean slope
__device__ __forceinline__ double vl_slope(double dm, double dp) {
  const double q = dm * dp;
  return q > 0.0 ? div64(2.0 * q, dm + dp) : 0.0;
}

__device__ __forceinline__ double minmod2(double a, double b) {
  return a * b > 0.0 ? (fabs(a) < fabs(b) ? a : b) : 0.0;
}

// Fast magnetosonic speed along D from a primitive state (1/rho given).
template <int D>
__device__ __forceinline__ double cfast(const double w[NV], double ri, double b2, const PhysConst& P) {
  const double a2 = P.gamma * w[4] * ri;
  const double bb = b2 * ri;
  const double bn2 = w[I_BX + D] * w[I_BX + D] * ri;
  const double s = a2 + bb;
  double disc = s * s - 4.0 * a2 * bn2;
  disc = disc < 0.0 ? 0.0 : disc;
  return sqrt64(0.5 * (s + sqrt64(disc)));
}

// Interface flux along D from reconstructed left/right primitive states:
// GLM interface values of (B_n, psi) from the exact solution of the linear
// subsystem, then HLL (Davis bounds) on rho, m, e and the tangential B,
// with B_n replaced on both sides.  half_inv_ch = 0.5 / c_h.  The HLL
// combination is formed one component at a time so that only the two
// primitive states and a few per-side scalars stay live.
template <int D>
__device__ __forceinline__ void hll_glm_flux(double wl[NV], double wr[NV], double ch, double half_inv_ch,
                                             const PhysConst& P, double F[NV]) {
  constexpr int N = I_BX + D;
  const double bn = 0.5 * (wl[N] + wr[N]) - (wr[I_PSI] - wl[I_PSI]) * half_inv_ch;
  const double ps = 0.5 * (wl[I_PSI] + wr[I_PSI]) - 0.5 * ch * (wr[N] - wl[N]);
  wl[N] = bn;
  wr[N] = bn;

  const double rl = wl[I_RHO], rr = wr[I_RHO];
  const double b2l = wl[I_BX] * wl[I_BX] + wl[I_BY] * wl[I_BY] + wl[I_BZ] * wl[I_BZ];
  const double b2r = wr[I_BX] * wr[I_BX] + wr[I_BY] * wr[I_BY] + wr[I_BZ] * wr[I_BZ];
  const double cl = cfast<D>(wl, rcp64(rl), b2l, P);
  const double cr = cfast<D>(wr, rcp64(rr), b2r, P);
  const double vnl = wl[1 + D], vnr = wr[1 + D];
  const double sl = fmin(vnl - cl, vnr - cr);
  const double sr = fmax(vnl + cl, vnr + cr);
  const double inv = rcp64(sr - sl);
  const double slsr = sl * sr;
  const bool use_l = sl >= 0.0, use_r = sr <= 0.0;
  auto hll = [&](double ul, double ur, double fl, double fr) {
    const double h = (sr * fl - sl * fr + slsr * (ur - ul)) * inv;
    return use_l ? fl : (use_r ? fr : h);
  };
  // mass
  const double mnl = rl * vnl, mnr = rr * vnr;
  F[I_RHO] = hll(rl, rr, mnl, mnr);
  // energy
  {
    const double v2l = wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3];
    const double v2r = wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3];
    const double el = wl[4] * P.inv_gm1 + 0.5 * rl * v2l + 0.5 * b2l;
    const double er = wr[4] * P.inv_gm1 + 0.5 * rr * v2r + 0.5 * b2r;
    const double vbl = wl[1] * wl[I_BX] + wl[2] * wl[I_BY] + wl[3] * wl[I_BZ];
    const double vbr = wr[1] * wr[I_BX] + wr[2] * wr[I_BY] + wr[3] * wr[I_BZ];
    const double ptl = wl[4] + 0.5 * b2l, ptr = wr[4] + 0.5 * b2r;
    F[I_EN] = hll(el, er, (el + ptl) * vnl - bn * vbl, (er + ptr) * vnr - bn * vbr);
    // momentum
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double ml = rl * wl[1 + c], mr = rr * wr[1 + c];
      double fl = ml * vnl - wl[I_BX + c] * bn;
      double fr = mr * vnr - wr[I_BX + c] * bn;
      if (c == D) {
        fl += ptl;
        fr += ptr;
      }
      F[I_MX + c] = hll(ml, mr, fl, fr);
    }
  }
  // tangential field
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c == D) continue;
    F[I_BX + c] = hll(wl[I_BX + c], wr[I_BX + c], vnl * wl[I_BX + c] - bn * wl[1 + c],
                      vnr * wr[I_BX + c] - bn * wr[1 + c]);
  }
  F[N] = ps;
  F[I_PSI] = ch * ch * bn;
}

// Reconstructed left/right states at the face between cells a (=i) and
// b (=i+1) from four primitive cells m (=i-1), a, b, p (=i+2), with the
// first-order fallback when rho or p is not positive on either side.
__device__ __forceinline__ void reconstruct_face(const double wm[NV], const double wa[NV], const double wb[NV],
                                                 const double wp[NV], double wl[NV], double wr[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double sa = vl_slope(wa[q] - wm[q], wb[q] - wa[q]);
    const double sb = vl_slope(wb[q] - wa[q], wp[q] - wb[q]);
    wl[q] = wa[q] + 0.5 * sa;
    wr[q] = wb[q] - 0.5 * sb;
  }
  const bool ok = (wl[I_RHO] > 0.0) && (wl[4] > 0.0) && (wr[I_RHO] > 0.0) && (wr[4] > 0.0);
  if (!ok) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      wl[q] = wa[q];
      wr[q] = wb[q];
    }
  }
}

}  // namespace amrvac
