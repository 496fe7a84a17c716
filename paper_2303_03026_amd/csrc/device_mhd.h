// Device-side ideal GLM-MHD arithmetic for gfx950 (register-resident, fully
// unrolled; the face direction is a template parameter so component
// selection costs nothing).  Face arithmetic is templated on the real type:
// double on the FP64 path, float on the FP32-mixed path (where the
// conserved-to-primitive step and the pressure recovery stay in double).
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
  int limiter;  // LIM_* (the fused stage takes it as a template argument)
  int flux;     // FLUX_HLL, FLUX_HLLD or FLUX_HLLC (likewise)
};

// Library-owned device status record.
struct DevStatus {
  unsigned int flags;
  unsigned int cfl_nan;  // a NaN rate was met by the running CFL reduction
  unsigned long long nfix;
  unsigned long long rate_bits;  // max CFL rate (non-negative double bits)
  double last_dt;
};

// ---------------------------------------------------------------------------
// Lean reciprocal, quotient and square root for the normal-range operands of
// this scheme (no denormal or overflow scaling).  FP64: a hardware seed
// (v_rcp_f64 / v_rsq_f64, measured on gfx950 to about 2^-24 relative) refined
// by Newton steps; the reciprocal takes two (about one ulp), the quotient one
// step plus a residual correction of the product (about one ulp).  FP32: the
// single-instruction v_rcp_f32 / v_sqrt_f32 (about one ulp).

__device__ __forceinline__ double rcp_(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(e, r, r);
  e = fma(-x, r, 1.0);
  return fma(e, r, r);
}
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double div_(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);  // ~2^-48 relative
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}
__device__ __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

__device__ __forceinline__ double sqrt_(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, x), h, g);
  return x > 0.0 ? g : 0.0;
}
__device__ __forceinline__ float sqrt_(float x) { return x > 0.0f ? __builtin_amdgcn_sqrtf(x) : 0.0f; }

// ---------------------------------------------------------------------------
// conserved -> primitive; returns the small-value bits of this cell.  The
// conserved input is double (the FP64 energy and the promoted FP32 rest on
// the mixed path) and the pressure recovery e - m^2/2rho - B^2/2 is done in
// double; the primitive is then rounded to R.  With the fix on, density is
// floored first (velocity uses the floored value), then pressure; conserved
// values and B are never changed.
template <class R>
__device__ __forceinline__ int cons_to_prim(const double u[NV], R w[NV], const PhysConst& P) {
  int bad = 0;
  double rho = u[I_RHO];
  if (!(rho > P.small_rho)) {
    bad |= F_SMALL_RHO;
    if (P.fix) rho = P.small_rho;
  }
  const double ri = rcp_(rho);
  w[I_RHO] = (R)rho;
  w[1] = (R)(u[I_MX] * ri);
  w[2] = (R)(u[I_MY] * ri);
  w[3] = (R)(u[I_MZ] * ri);
  const double m2 = u[I_MX] * u[I_MX] + u[I_MY] * u[I_MY] + u[I_MZ] * u[I_MZ];
  const double b2 = u[I_BX] * u[I_BX] + u[I_BY] * u[I_BY] + u[I_BZ] * u[I_BZ];
  double p = P.gm1 * (u[I_EN] - 0.5 * m2 * ri - 0.5 * b2);
  if (!(p > P.small_p)) {
    bad |= F_SMALL_P;
    if (P.fix) p = P.small_p;
  }
  w[4] = (R)p;
  w[I_BX] = (R)u[I_BX];
  w[I_BY] = (R)u[I_BY];
  w[I_BZ] = (R)u[I_BZ];
  w[I_PSI] = (R)u[I_PSI];
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

// van Leer's harmonic-mean slope.  The quotient is formed for every lane and
// then selected (no branch), so the nine slopes of a cell can interleave; it
// is discarded where dm * dp <= 0, which includes a zero denominator.
template <class R>
__device__ __forceinline__ R vl_slope(R dm, R dp) {
  const R q = dm * dp;
  const R v = div_(R(2) * q, dm + dp);
  return q > R(0) ? v : R(0);
}

// Limiters of Table t:limiters that work on the 2-ghost-cell stencil.  With
// d- = w_i - w_(i-1) and d+ = w_(i+1) - w_i, cell i's face values are
//   right face:  w_i + lim(d+, d-) / 2,    left face:  w_i - lim(d-, d+) / 2,
// lim(near, far) being the limited difference across the face (odd in its
// arguments).  van Leer's is symmetric: lim(d+, d-) = lim(d-, d+) = the
// harmonic slope.  Koren's and Cada-Torrilhon's third-order ones are not;
// written division-free with s = sign(near), b = |near|, a = s far, they are
//   koren:  s max(0, min(2a, (2b + a)/3, 2b))
//   cada3:  s max(0, min((2b + a)/3, max(-a/2, min(2a, (2b + a)/3, 1.6 b))))
// (the unlimited third-order value (2b + a)/3 in smooth monotone regions).
enum { LIM_VANLEER = 0, LIM_KOREN = 1, LIM_CADA3 = 2, LIM_WENO5 = 3, LIM_WENOZ5 = 4, LIM_MP5 = 5, LIM_WENOZP5 = 6 };

template <int LIM, class R>
__device__ __forceinline__ R lim_diff(R near, R far) {
  const R s = near < R(0) ? R(-1) : R(1);
  const R b = s * near, a = s * far;
  const R p3 = (R(2) * b + a) * R(1.0 / 3.0);
  if (LIM == LIM_KOREN) return s * fmax(R(0), fmin(fmin(R(2) * a, p3), R(2) * b));
  return s * fmax(R(0), fmin(p3, fmax(R(-0.5) * a, fmin(fmin(R(2) * a, p3), R(1.6) * b))));
}

// Limited differences of a cell for its right (inc_r) and left (inc_l)
// face values: w + inc_r / 2 and w - inc_l / 2.
template <int LIM, class R>
__device__ __forceinline__ void cell_increments(R dm, R dp, R& inc_r, R& inc_l) {
  if (LIM == LIM_VANLEER) {
    inc_r = vl_slope(dm, dp);
    inc_l = inc_r;
  } else {
    inc_r = lim_diff<LIM>(dp, dm);
    inc_l = lim_diff<LIM>(dm, dp);
  }
}

__device__ __forceinline__ double minmod2(double a, double b) {
  return a * b > 0.0 ? (fabs(a) < fabs(b) ? a : b) : 0.0;
}

// Fast magnetosonic speed along D from a primitive state (1/rho given).
template <int D, class R>
__device__ __forceinline__ R cfast(const R w[NV], R ri, R b2, R gamma) {
  const R a2 = gamma * w[4] * ri;
  const R bb = b2 * ri;
  const R bn2 = w[I_BX + D] * w[I_BX + D] * ri;
  const R s = a2 + bb;
  R disc = s * s - R(4) * a2 * bn2;
  disc = disc < R(0) ? R(0) : disc;
  return sqrt_(R(0.5) * (s + sqrt_(disc)));
}

// CFL rate of one cell from its conserved state (always FP64): the sum over
// directions of (|v_d| + c_fast,d) / dx_d, after the small-value check of the
// conserved-to-primitive step (its bits are or-ed into bad).  The time-step
// pass and the fused last stage both use this, so they agree bit for bit.
template <int NDIM>
__device__ __forceinline__ double cell_rate(const double u[NV], const PhysConst& P, double ix, double iy, double iz,
                                            int& bad) {
  double w[NV];
  bad |= cons_to_prim(u, w, P);
  const double ri = rcp_(w[I_RHO]);
  const double b2 = w[I_BX] * w[I_BX] + w[I_BY] * w[I_BY] + w[I_BZ] * w[I_BZ];
  double rate = (fabs(w[1]) + cfast<0>(w, ri, b2, P.gamma)) * ix;
  rate = rate + (fabs(w[2]) + cfast<1>(w, ri, b2, P.gamma)) * iy;
  if (NDIM == 3) rate = rate + (fabs(w[3]) + cfast<2>(w, ri, b2, P.gamma)) * iz;
  return rate;
}

// Interface flux along D from reconstructed left/right primitive states:
// GLM interface values of (B_n, psi) from the exact solution of the linear
// subsystem, then HLL (Davis bounds) on rho, m, e and the tangential B,
// with B_n replaced on both sides.  half_inv_ch = 0.5 / c_h.  The HLL
// combination is formed one component at a time so that only the two
// primitive states and a few per-side scalars stay live.
template <int D, class R>
__device__ __forceinline__ void hll_glm_flux(R wl[NV], R wr[NV], R ch, R half_inv_ch, R gamma, R inv_gm1,
                                             R F[NV]) {
  constexpr int N = I_BX + D;
  const R bn = R(0.5) * (wl[N] + wr[N]) - (wr[I_PSI] - wl[I_PSI]) * half_inv_ch;
  const R ps = R(0.5) * (wl[I_PSI] + wr[I_PSI]) - R(0.5) * ch * (wr[N] - wl[N]);
  wl[N] = bn;
  wr[N] = bn;

  const R rl = wl[I_RHO], rr = wr[I_RHO];
  const R b2l = wl[I_BX] * wl[I_BX] + wl[I_BY] * wl[I_BY] + wl[I_BZ] * wl[I_BZ];
  const R b2r = wr[I_BX] * wr[I_BX] + wr[I_BY] * wr[I_BY] + wr[I_BZ] * wr[I_BZ];
  const R cl = cfast<D>(wl, rcp_(rl), b2l, gamma);
  const R cr = cfast<D>(wr, rcp_(rr), b2r, gamma);
  const R vnl = wl[1 + D], vnr = wr[1 + D];
  const R sl = fmin(vnl - cl, vnr - cr);
  const R sr = fmax(vnl + cl, vnr + cr);
  // F = a fl + b fr + c (ur - ul): (S_R, -S_L, S_L S_R) / (S_R - S_L) in
  // the subsonic case, (1, 0, 0) if S_L >= 0 and (0, 1, 0) if S_R <= 0
  const bool use_l = sl >= R(0), use_r = sr <= R(0);
  const R inv = rcp_(sr - sl);
  const R ca = use_l ? R(1) : (use_r ? R(0) : sr * inv);
  const R cb = use_l ? R(0) : (use_r ? R(1) : -sl * inv);
  const R cc = (use_l || use_r) ? R(0) : sl * sr * inv;
  auto hll = [&](R ul, R ur, R fl, R fr) { return ca * fl + cb * fr + cc * (ur - ul); };
  // mass
  const R mnl = rl * vnl, mnr = rr * vnr;
  F[I_RHO] = hll(rl, rr, mnl, mnr);
  // energy
  {
    const R v2l = wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3];
    const R v2r = wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3];
    const R el = wl[4] * inv_gm1 + R(0.5) * rl * v2l + R(0.5) * b2l;
    const R er = wr[4] * inv_gm1 + R(0.5) * rr * v2r + R(0.5) * b2r;
    const R vbl = wl[1] * wl[I_BX] + wl[2] * wl[I_BY] + wl[3] * wl[I_BZ];
    const R vbr = wr[1] * wr[I_BX] + wr[2] * wr[I_BY] + wr[3] * wr[I_BZ];
    const R ptl = wl[4] + R(0.5) * b2l, ptr = wr[4] + R(0.5) * b2r;
    F[I_EN] = hll(el, er, (el + ptl) * vnl - bn * vbl, (er + ptr) * vnr - bn * vbr);
    // momentum
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R ml = rl * wl[1 + c], mr = rr * wr[1 + c];
      R fl = ml * vnl - wl[I_BX + c] * bn;
      R fr = mr * vnr - wr[I_BX + c] * bn;
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

// HLLD (Miyoshi and Kusano 2005) with the same GLM interface values as
// hll_glm_flux: B_n := B_n* on both sides, F(B_n) = psi*, F(psi) = c_h^2 B_n*,
// and HLLD on the other seven components.  S_L, S_R bracket both fast speeds
// around both normal velocities; S_M is the contact speed and p_T* the total
// pressure of the star region; the single-star states follow from the jump
// conditions across S_L / S_R (their tangential parts unchanged where
// rho (S - u)(S - S_M) - B_n^2 vanishes), the Alfven waves sit at
// S_M -/+ |B_n| / sqrt(rho*), and the double-star states between them and the
// contact.  Only the side of the contact that the interface lies on is
// assembled: F = F_a + S_a (U*_a - U_a) [+ S*_a (U**_a - U*_a) between the
// Alfven wave and the contact]; selects (not arithmetic) drop the star terms
// when every wave moves one way.
template <int D, class R>
__device__ __forceinline__ void hlld_glm_flux(R wl[NV], R wr[NV], R ch, R half_inv_ch, R gamma, R inv_gm1,
                                              R F[NV]) {
  constexpr int N = I_BX + D;
  constexpr int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;  // tangential axes
  const R bn = R(0.5) * (wl[N] + wr[N]) - (wr[I_PSI] - wl[I_PSI]) * half_inv_ch;
  const R ps = R(0.5) * (wl[I_PSI] + wr[I_PSI]) - R(0.5) * ch * (wr[N] - wl[N]);
  wl[N] = bn;
  wr[N] = bn;
  const R rl = wl[I_RHO], rr = wr[I_RHO];
  const R ul = wl[1 + D], ur = wr[1 + D];
  const R b2l = wl[I_BX] * wl[I_BX] + wl[I_BY] * wl[I_BY] + wl[I_BZ] * wl[I_BZ];
  const R b2r = wr[I_BX] * wr[I_BX] + wr[I_BY] * wr[I_BY] + wr[I_BZ] * wr[I_BZ];
  const R ptl = wl[4] + R(0.5) * b2l, ptr = wr[4] + R(0.5) * b2r;
  const R cfm = fmax(cfast<D>(wl, rcp_(rl), b2l, gamma), cfast<D>(wr, rcp_(rr), b2r, gamma));
  const R sl = fmin(ul, ur) - cfm, sr = fmax(ul, ur) + cfm;
  const R dl = (sl - ul) * rl, dr = (sr - ur) * rr;
  const R idd = rcp_(dr - dl);
  const R sm = (dr * ur - dl * ul - ptr + ptl) * idd;
  const R pts = (dr * ptl - dl * ptr + dl * dr * (ur - ul)) * idd;
  const R bn2 = bn * bn;
  // single-star density and tangential parts, both sides
  R rs[2], vs1[2], vs2[2], bs1[2], bs2[2], isb[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const R* w = a ? wr : wl;
    const R rho = a ? rr : rl, u = a ? ur : ul, sa = (a ? sr : sl) - u, sb = (a ? sr : sl) - sm;
    isb[a] = rcp_(sb);
    rs[a] = rho * sa * isb[a];
    const R den = rho * sa * sb - bn2;
    const bool deg = fabs(den) <= R(1e-12) * rho * sa * sa;
    const R iden = rcp_(den);
    const R f1 = deg ? R(0) : bn * (sm - u) * iden;
    const R f2 = deg ? R(1) : (rho * sa * sa - bn2) * iden;
    vs1[a] = w[1 + T1] - f1 * w[I_BX + T1];
    vs2[a] = w[1 + T2] - f1 * w[I_BX + T2];
    bs1[a] = f2 * w[I_BX + T1];
    bs2[a] = f2 * w[I_BX + T2];
  }
  // double-star tangential parts
  const R sql = sqrt_(rs[0]), sqr = sqrt_(rs[1]);
  const R isum = rcp_(sql + sqr);
  const R sg = bn > R(0) ? R(1) : (bn < R(0) ? R(-1) : R(0));
  const R vss1 = (sql * vs1[0] + sqr * vs1[1] + (bs1[1] - bs1[0]) * sg) * isum;
  const R vss2 = (sql * vs2[0] + sqr * vs2[1] + (bs2[1] - bs2[0]) * sg) * isum;
  const R bss1 = (sql * bs1[1] + sqr * bs1[0] + sql * sqr * (vs1[1] - vs1[0]) * sg) * isum;
  const R bss2 = (sql * bs2[1] + sqr * bs2[0] + sql * sqr * (vs2[1] - vs2[0]) * sg) * isum;
  // the side a of the contact the interface lies on, and its states
  const bool right = sr < R(0) || (!(sl > R(0)) && sm < R(0));
  const R* w = right ? wr : wl;
  const R rho = right ? rr : rl, u = right ? ur : ul, pt = right ? ptr : ptl, b2 = right ? b2r : b2l;
  const R S = right ? sr : sl, sa = S - u;
  const R rsa = right ? rs[1] : rs[0], isba = right ? isb[1] : isb[0];
  const R vs1a = right ? vs1[1] : vs1[0], vs2a = right ? vs2[1] : vs2[0];
  const R bs1a = right ? bs1[1] : bs1[0], bs2a = right ? bs2[1] : bs2[0];
  const R v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  const R e = w[4] * inv_gm1 + R(0.5) * rho * v2 + R(0.5) * b2;
  const R vb = w[1] * w[I_BX] + w[2] * w[I_BY] + w[3] * w[I_BZ];
  const R vbs = sm * bn + vs1a * bs1a + vs2a * bs2a;
  const R es = (sa * e - pt * u + pts * sm + bn * (vb - vbs)) * isba;
  const R vbss = sm * bn + vss1 * bss1 + vss2 * bss2;
  const R sqa = right ? sqr : sql, sgn_a = right ? R(1) : R(-1);
  const R ess = es + sgn_a * sqa * (vbs - vbss) * sg;
  const R sas = sm + sgn_a * fabs(bn) * rcp_(sqa);  // S*_a
  const bool super = sl > R(0) || sr < R(0);       // every wave moves one way: F = F_a
  const bool inner = sgn_a * sas > R(0);            // between the Alfven wave and the contact
  auto hlld = [&](R uq, R usq, R ussq, R fq) {
    const R fs = fq + S * (usq - uq);
    const R f = inner ? fs + sas * (ussq - usq) : fs;
    return super ? fq : f;
  };
  F[I_RHO] = hlld(rho, rsa, rsa, rho * u);
  F[1 + D] = hlld(rho * u, rsa * sm, rsa * sm, rho * u * u + pt - bn2);
  F[1 + T1] = hlld(rho * w[1 + T1], rsa * vs1a, rsa * vss1, rho * w[1 + T1] * u - w[I_BX + T1] * bn);
  F[1 + T2] = hlld(rho * w[1 + T2], rsa * vs2a, rsa * vss2, rho * w[1 + T2] * u - w[I_BX + T2] * bn);
  F[I_EN] = hlld(e, es, ess, (e + pt) * u - bn * vb);
  F[I_BX + T1] = hlld(w[I_BX + T1], bs1a, bss1, u * w[I_BX + T1] - bn * w[1 + T1]);
  F[I_BX + T2] = hlld(w[I_BX + T2], bs2a, bss2, u * w[I_BX + T2] - bn * w[1 + T2]);
  F[N] = ps;
  F[I_PSI] = ch * ch * bn;
}

// HLLC for MHD (Li 2005) with the same GLM interface values: Davis bounds
// S_L, S_R as for HLL, contact speed S_M, star-region total pressure
// pT* = rho_L (S_L - u_L)(S_M - u_L) + pT_L; both star states take the
// tangential field and velocity of the HLL average state, and their density,
// momentum and energy from the jump conditions across S_L or S_R.  Only the
// side of the contact the interface lies on is assembled; selects drop the
// star terms when every wave moves one way.
template <int D, class R>
__device__ __forceinline__ void hllc_glm_flux(R wl[NV], R wr[NV], R ch, R half_inv_ch, R gamma, R inv_gm1,
                                              R F[NV]) {
  constexpr int N = I_BX + D;
  constexpr int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;
  const R bn = R(0.5) * (wl[N] + wr[N]) - (wr[I_PSI] - wl[I_PSI]) * half_inv_ch;
  const R ps = R(0.5) * (wl[I_PSI] + wr[I_PSI]) - R(0.5) * ch * (wr[N] - wl[N]);
  wl[N] = bn;
  wr[N] = bn;
  const R rl = wl[I_RHO], rr = wr[I_RHO];
  const R ul = wl[1 + D], ur = wr[1 + D];
  const R b2l = wl[I_BX] * wl[I_BX] + wl[I_BY] * wl[I_BY] + wl[I_BZ] * wl[I_BZ];
  const R b2r = wr[I_BX] * wr[I_BX] + wr[I_BY] * wr[I_BY] + wr[I_BZ] * wr[I_BZ];
  const R ptl = wl[4] + R(0.5) * b2l, ptr = wr[4] + R(0.5) * b2r;
  const R cl = cfast<D>(wl, rcp_(rl), b2l, gamma), cr = cfast<D>(wr, rcp_(rr), b2r, gamma);
  const R sl = fmin(ul - cl, ur - cr), sr = fmax(ul + cl, ur + cr);
  // HLL average of density and of the tangential momentum and field
  const R isr = rcp_(sr - sl);
  auto havg = [&](R ql, R qr, R fql, R fqr) { return (sr * qr - sl * ql - (fqr - fql)) * isr; };
  const R rh = havg(rl, rr, rl * ul, rr * ur);
  const R m1h = havg(rl * wl[1 + T1], rr * wr[1 + T1], rl * wl[1 + T1] * ul - wl[I_BX + T1] * bn,
                     rr * wr[1 + T1] * ur - wr[I_BX + T1] * bn);
  const R m2h = havg(rl * wl[1 + T2], rr * wr[1 + T2], rl * wl[1 + T2] * ul - wl[I_BX + T2] * bn,
                     rr * wr[1 + T2] * ur - wr[I_BX + T2] * bn);
  const R b1h = havg(wl[I_BX + T1], wr[I_BX + T1], ul * wl[I_BX + T1] - bn * wl[1 + T1],
                     ur * wr[I_BX + T1] - bn * wr[1 + T1]);
  const R b2h = havg(wl[I_BX + T2], wr[I_BX + T2], ul * wl[I_BX + T2] - bn * wl[1 + T2],
                     ur * wr[I_BX + T2] - bn * wr[1 + T2]);
  const R irh = rcp_(rh);
  const R vs1 = m1h * irh, vs2 = m2h * irh;
  const R sm = (rr * ur * (sr - ur) - rl * ul * (sl - ul) + ptl - ptr) * rcp_(rr * (sr - ur) - rl * (sl - ul));
  const R pts = rl * (sl - ul) * (sm - ul) + ptl;
  const R vbs = sm * bn + vs1 * b1h + vs2 * b2h;
  // the side of the contact the interface lies on
  const bool super = sl >= R(0) || sr <= R(0);
  const bool right = sr <= R(0) || (!(sl >= R(0)) && sm < R(0));
  const R* w = right ? wr : wl;
  const R rho = right ? rr : rl, u = right ? ur : ul, pt = right ? ptr : ptl, b2 = right ? b2r : b2l;
  const R S = right ? sr : sl, sa = S - u, isb = rcp_(S - sm);
  const R v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  const R e = w[4] * inv_gm1 + R(0.5) * rho * v2 + R(0.5) * b2;
  const R vb = w[1] * w[I_BX] + w[2] * w[I_BY] + w[3] * w[I_BZ];
  const R rs = rho * sa * isb;
  const R ms1 = (rho * w[1 + T1] * sa + bn * (w[I_BX + T1] - b1h)) * isb;
  const R ms2 = (rho * w[1 + T2] * sa + bn * (w[I_BX + T2] - b2h)) * isb;
  const R es = (e * sa - pt * u + pts * sm + bn * (vb - vbs)) * isb;
  auto hllc = [&](R uq, R usq, R fq) { return super ? fq : fq + S * (usq - uq); };
  F[I_RHO] = hllc(rho, rs, rho * u);
  F[1 + D] = hllc(rho * u, rs * sm, rho * u * u + pt - bn * bn);
  F[1 + T1] = hllc(rho * w[1 + T1], ms1, rho * w[1 + T1] * u - w[I_BX + T1] * bn);
  F[1 + T2] = hllc(rho * w[1 + T2], ms2, rho * w[1 + T2] * u - w[I_BX + T2] * bn);
  F[I_EN] = hllc(e, es, (e + pt) * u - bn * vb);
  F[I_BX + T1] = hllc(w[I_BX + T1], b1h, u * w[I_BX + T1] - bn * w[1 + T1]);
  F[I_BX + T2] = hllc(w[I_BX + T2], b2h, u * w[I_BX + T2] - bn * w[1 + T2]);
  F[N] = ps;
  F[I_PSI] = ch * ch * bn;
}

enum { FLUX_HLL = 0, FLUX_HLLD = 1, FLUX_HLLC = 2 };

// interface flux of the scheme chosen at compile time
template <int FLX, int D, class R>
__device__ __forceinline__ void face_flux(R wl[NV], R wr[NV], R ch, R half_inv_ch, R gamma, R inv_gm1, R F[NV]) {
  if (FLX == FLUX_HLLD)
    hlld_glm_flux<D, R>(wl, wr, ch, half_inv_ch, gamma, inv_gm1, F);
  else if (FLX == FLUX_HLLC)
    hllc_glm_flux<D, R>(wl, wr, ch, half_inv_ch, gamma, inv_gm1, F);
  else
    hll_glm_flux<D, R>(wl, wr, ch, half_inv_ch, gamma, inv_gm1, F);
}

// ... and at run time (the per-kernel path)
template <int D, class R>
__device__ __forceinline__ void face_flux_rt(int flux, R wl[NV], R wr[NV], R ch, R half_inv_ch, R gamma, R inv_gm1,
                                             R F[NV]) {
  if (flux == FLUX_HLLD)
    hlld_glm_flux<D, R>(wl, wr, ch, half_inv_ch, gamma, inv_gm1, F);
  else if (flux == FLUX_HLLC)
    hllc_glm_flux<D, R>(wl, wr, ch, half_inv_ch, gamma, inv_gm1, F);
  else
    hll_glm_flux<D, R>(wl, wr, ch, half_inv_ch, gamma, inv_gm1, F);
}

// First-order fallback at a face: where rho or p of either reconstructed
// state is not positive, both states become the two cell states (cl, cr).
// It is rare, so the selects run only in waves where some lane needs them
// (a wave-uniform branch on the vote).
template <class R>
__device__ __forceinline__ void positivity_fallback(R wl[NV], R wr[NV], const R cl[NV], const R cr[NV]) {
  const bool bad = !((wl[I_RHO] > R(0)) && (wl[4] > R(0)) && (wr[I_RHO] > R(0)) && (wr[4] > R(0)));
  if (__any(bad)) {
    asm volatile("");  // keeps the branch: the compiler would otherwise select unconditionally
    if (bad) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        wl[q] = cl[q];
        wr[q] = cr[q];
      }
    }
  }
}

// Reconstructed left/right states at the face between cells a (=i) and
// b (=i+1) from four primitive cells m (=i-1), a, b, p (=i+2), with the
// first-order fallback when rho or p is not positive on either side.
template <int LIM, class R>
__device__ __forceinline__ void reconstruct_face_lim(const R wm[NV], const R wa[NV], const R wb[NV], const R wp[NV],
                                                     R wl[NV], R wr[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    R ra, la, rb, lb;
    cell_increments<LIM>(wa[q] - wm[q], wb[q] - wa[q], ra, la);
    cell_increments<LIM>(wb[q] - wa[q], wp[q] - wb[q], rb, lb);
    wl[q] = wa[q] + R(0.5) * ra;
    wr[q] = wb[q] - R(0.5) * lb;
  }
  positivity_fallback(wl, wr, wa, wb);
}

// Fifth-order WENO value at the face between cells i and i+1 seen from cell i
// (cells i-2 .. i+2; 3 ghost layers): candidate polynomials q_k, smoothness
// indicators beta_k, optimal weights (0.1, 0.6, 0.3).  Weights by limiter:
// 'weno5' (Jiang-Shu) d_k / (1e-6 + beta_k)^2; 'wenoz5' (Borges et al.)
// d_k (1 + tau5 / (beta_k + 1e-40)) with tau5 = |beta_0 - beta_2|;
// 'wenozp5' (Acker et al.) d_k (1 + (tau5 / (beta_k + 1e-40))^2 + lambda
// (beta_k + 1e-40) / (tau5 + 1e-40)) with lambda = dx^(2/3).
__device__ __forceinline__ double weno5_face(double vm2, double vm1, double v0, double vp1, double vp2, int lim,
                                             double lambda) {
  const double q0 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) * (1.0 / 6.0);
  const double q1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) * (1.0 / 6.0);
  const double q2 = (2.0 * v0 + 5.0 * vp1 - vp2) * (1.0 / 6.0);
  const double a0 = vm2 - 2.0 * vm1 + v0, b0 = vm2 - 4.0 * vm1 + 3.0 * v0;
  const double a1 = vm1 - 2.0 * v0 + vp1, b1 = vm1 - vp1;
  const double a2 = v0 - 2.0 * vp1 + vp2, b2 = 3.0 * v0 - 4.0 * vp1 + vp2;
  const double be0 = (13.0 / 12.0) * a0 * a0 + 0.25 * b0 * b0;
  const double be1 = (13.0 / 12.0) * a1 * a1 + 0.25 * b1 * b1;
  const double be2 = (13.0 / 12.0) * a2 * a2 + 0.25 * b2 * b2;
  // the three reciprocals of the weights come from one reciprocal of their
  // product (the refined hardware reciprocal is the costly operation here);
  // the factors are at least 1e-40 (1e-12 for 'weno5'), so the product does
  // not underflow, and it overflows only for cell values beyond about 1e50
  auto rcp3 = [](double x0, double x1, double x2, double& r0, double& r1, double& r2) {
    const double x01 = x0 * x1;
    const double r = rcp_(x01 * x2);
    r0 = r * (x1 * x2);
    r1 = r * (x0 * x2);
    r2 = r * x01;
  };
  double al0, al1, al2;
  if (lim == LIM_WENOZ5 || lim == LIM_WENOZP5) {
    const double tau5 = fabs(be0 - be2);
    const double e0 = be0 + 1e-40, e1 = be1 + 1e-40, e2 = be2 + 1e-40;
    double i0, i1, i2;
    rcp3(e0, e1, e2, i0, i1, i2);
    const double r0 = tau5 * i0, r1 = tau5 * i1, r2 = tau5 * i2;
    if (lim == LIM_WENOZ5) {
      al0 = 0.1 * (1.0 + r0);
      al1 = 0.6 * (1.0 + r1);
      al2 = 0.3 * (1.0 + r2);
    } else {
      // the weights times tau5 + 1e-40 (their ratios are what counts), which
      // takes the quotient lambda / (tau5 + 1e-40) out
      const double tp = tau5 + 1e-40;
      al0 = 0.1 * (tp + (tp * r0) * r0 + lambda * e0);
      al1 = 0.6 * (tp + (tp * r1) * r1 + lambda * e1);
      al2 = 0.3 * (tp + (tp * r2) * r2 + lambda * e2);
    }
  } else {
    const double e0 = 1e-6 + be0, e1 = 1e-6 + be1, e2 = 1e-6 + be2;
    double i0, i1, i2;
    rcp3(e0 * e0, e1 * e1, e2 * e2, i0, i1, i2);
    al0 = 0.1 * i0;
    al1 = 0.6 * i1;
    al2 = 0.3 * i2;
  }
  return div_(al0 * q0 + al1 * q1 + al2 * q2, al0 + al1 + al2);
}

__device__ __forceinline__ double mm2(double a, double b) {
  return (a > 0.0 && b > 0.0) ? fmin(a, b) : ((a < 0.0 && b < 0.0) ? fmax(a, b) : 0.0);
}

__device__ __forceinline__ double mm4(double a, double b, double c, double d) {
  const double lo = fmin(fmin(a, b), fmin(c, d)), hi = fmax(fmax(a, b), fmax(c, d));
  return lo > 0.0 ? lo : (hi < 0.0 ? hi : 0.0);
}

// Monotonicity-preserving fifth-order face value ('mp5', Suresh and Huynh):
// the fifth-order interpolant unless it leaves the interval between u_i and
// u_i + minmod(u_{i+1} - u_i, 4 (u_i - u_{i-1})); then its median with the
// bounds u_min, u_max built from curvature-limited second differences.
__device__ __forceinline__ double mp5_face(double vm2, double vm1, double v0, double vp1, double vp2) {
  const double u_or = (2.0 * vm2 - 13.0 * vm1 + 47.0 * v0 + 27.0 * vp1 - 3.0 * vp2) * (1.0 / 60.0);
  const double back = v0 - vm1;
  const double u_mp = v0 + mm2(vp1 - v0, 4.0 * back);
  if ((u_or - v0) * (u_or - u_mp) <= 0.0) return u_or;
  const double dm1 = vm2 - 2.0 * vm1 + v0, d0 = vm1 - 2.0 * v0 + vp1, dp1 = v0 - 2.0 * vp1 + vp2;
  const double cp = mm4(4.0 * d0 - dp1, 4.0 * dp1 - d0, d0, dp1);
  const double cm = mm4(4.0 * d0 - dm1, 4.0 * dm1 - d0, d0, dm1);
  const double u_ul = v0 + 4.0 * back;
  const double u_md = 0.5 * (v0 + vp1) - 0.5 * cp;
  const double u_lc = v0 + 0.5 * back + (4.0 / 3.0) * cm;
  const double u_min = fmax(fmin(fmin(v0, vp1), u_md), fmin(fmin(v0, u_ul), u_lc));
  const double u_max = fmin(fmax(fmax(v0, vp1), u_md), fmax(fmax(v0, u_ul), u_lc));
  return u_or + mm2(u_min - u_or, u_max - u_or);
}

// the same with the limiter chosen at run time (the per-kernel path, and the
// fused stage with three ghost layers run with a two-ghost-layer limiter)
template <class R>
__device__ __forceinline__ void reconstruct_face(int lim, const R wm[NV], const R wa[NV], const R wb[NV],
                                                 const R wp[NV], R wl[NV], R wr[NV]) {
  if (lim == LIM_KOREN)
    reconstruct_face_lim<LIM_KOREN>(wm, wa, wb, wp, wl, wr);
  else if (lim == LIM_CADA3)
    reconstruct_face_lim<LIM_CADA3>(wm, wa, wb, wp, wl, wr);
  else
    reconstruct_face_lim<LIM_VANLEER>(wm, wa, wb, wp, wl, wr);
}

// The five-cell face values at face precision R: the stored (R) cell
// values are promoted and the value is computed in FP64, then rounded to R.
// (In FP32 the WENO-Z+ term (tau5 / (beta + 1e-40))^2 overflows and 1e-40
// is not representable, so the nonlinear weights stay FP64 on the mixed
// path too.)
template <class R>
__device__ __forceinline__ R weno5_face_r(R vm2, R vm1, R v0, R vp1, R vp2, int lim, double lambda) {
  return (R)weno5_face((double)vm2, (double)vm1, (double)v0, (double)vp1, (double)vp2, lim, lambda);
}
template <class R>
__device__ __forceinline__ R mp5_face_r(R vm2, R vm1, R v0, R vp1, R vp2) {
  return (R)mp5_face((double)vm2, (double)vm1, (double)v0, (double)vp1, (double)vp2);
}

// Face states from the six cells c[0..5] around the face between c[2] and
// c[3] (3 ghost layers): the fifth-order values of 'weno5' / 'wenoz5' /
// 'wenozp5' (lambda = dx^(2/3) of the block) or 'mp5', else the
// two-ghost-layer reconstruction from c[1..4]; first-order fallback as
// always.
template <class R>
__device__ __forceinline__ void reconstruct_face6(int lim, const R c[6][NV], double lambda, R wl[NV], R wr[NV]) {
  if (lim == LIM_MP5) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      wl[q] = mp5_face_r(c[0][q], c[1][q], c[2][q], c[3][q], c[4][q]);
      wr[q] = mp5_face_r(c[5][q], c[4][q], c[3][q], c[2][q], c[1][q]);
    }
    positivity_fallback(wl, wr, c[2], c[3]);
  } else if (lim >= LIM_WENO5) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      wl[q] = weno5_face_r(c[0][q], c[1][q], c[2][q], c[3][q], c[4][q], lim, lambda);
      wr[q] = weno5_face_r(c[5][q], c[4][q], c[3][q], c[2][q], c[1][q], lim, lambda);
    }
    positivity_fallback(wl, wr, c[2], c[3]);
  } else {
    reconstruct_face(lim, c[1], c[2], c[3], c[4], wl, wr);
  }
}

// ---------------------------------------------------------------------------
// Slot storage policies.  A slot is [block][...] with pc padded cells per
// block.  FP64: 9 double arrays.  Mixed: 8 float arrays (rho, m_x, m_y, m_z,
// B_x, B_y, B_z, psi) then one double array (e).  Values move as double.

struct StoreF64 {
  using R = double;  // face arithmetic type
  static constexpr int kBytesPerCell = 72;
  static constexpr int kWavesPerEU = 2;  // fused-stage occupancy target
  __device__ static double ld(const void* blk, int q, long c, long pc) {
    return static_cast<const double*>(blk)[q * pc + c];
  }
  __device__ static void st(void* blk, int q, long c, long pc, double v) {
    static_cast<double*>(blk)[q * pc + c] = v;
  }
  // the value a later load of variable q returns after st(v)
  __device__ static double as_stored(int, double v) { return v; }
};

struct StoreMixed {
  using R = float;
  static constexpr int kBytesPerCell = 40;
  static constexpr int kWavesPerEU = 3;
  __device__ static int fidx(int q) { return q < I_EN ? q : q - 1; }
  __device__ static double ld(const void* blk, int q, long c, long pc) {
    if (q == I_EN) return reinterpret_cast<const double*>(static_cast<const char*>(blk) + 32 * pc)[c];
    return (double)static_cast<const float*>(blk)[fidx(q) * pc + c];
  }
  __device__ static void st(void* blk, int q, long c, long pc, double v) {
    if (q == I_EN)
      reinterpret_cast<double*>(static_cast<char*>(blk) + 32 * pc)[c] = v;
    else
      static_cast<float*>(blk)[fidx(q) * pc + c] = (float)v;
  }
  __device__ static double as_stored(int q, double v) { return q == I_EN ? v : (double)(float)v; }
};

template <class SP>
__device__ __forceinline__ const void* block_ptr(const void* slot, long b, long pc) {
  return static_cast<const char*>(slot) + b * pc * SP::kBytesPerCell;
}
template <class SP>
__device__ __forceinline__ void* block_ptr(void* slot, long b, long pc) {
  return static_cast<char*>(slot) + b * pc * SP::kBytesPerCell;
}

}  // namespace amrvac
