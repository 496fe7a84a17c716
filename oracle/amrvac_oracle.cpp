// Plain FP64 CPU oracle of the explicit ideal GLM-MHD block update.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
// this file: only the tests, the package smoke check and the benchmark's
// cpu_baseline leg use it.  It shares no code, header, table or helper with the
// HIP library; both sides read the same seeded primitive input arrays and
// nothing else.
//
// What it computes (MPI-AMRVAC 3.0, arXiv 2303.03026):
//   * conservative cell-centred finite volumes inside a multistage SSP
//     Runge-Kutta step ("Schemes and limiters for HD and MHD", Table
//     tab:schemes_time: SSPRK(2,2), SSPRK(3,3), SSPRK(4,3) and SSPRK(5,4));
//   * limited linear reconstruction of primitive variables giving a left and
//     a right state per face, with the 'vanleer', 'koren' or 'cada3'
//     limiter and 2 ghost cells, or the fifth-order 'weno5' / 'wenoz5' /
//     'wenozp5' / 'mp5' reconstructions with 3 ghost cells (Table
//     t:limiters);
//   * the HLL flux (Table tab:schemes_space; Harten et al. 1983), or HLLD
//     (Miyoshi and Kusano 2005), or HLLC (Li 2005);
//   * the 'glm' divergence control of Dedner et al. 2002 (Table t:divb);
//   * the CFL coupling of the time step to the grid spacing ("Schemes and
//     limiters for HD and MHD");
//   * small-value checking on entry to the conserved-to-primitive step, with
//     the optional replacement fix ("Bootstrapping" section);
//   * a static block-based octree/quadtree AMR hierarchy with refinement
//     ratio 2 where only leaf blocks are advanced ("Open source strategy"
//     section and the AMR statement in "Schemes and limiters"); ghost cells
//     come from same-level neighbours, restriction of finer neighbours,
//     prolongation of coarser neighbours or physical boundaries.
//
// The paper prints none of these formulas; they are written here from the
// cited textbook definitions in the readings listed in the repository's
// design notes.  Where the paper is silent the oracle takes these readings:
//   magnetic units with p_mag = |B|^2/2 (plasma beta 2p/B^2, Alfven shock
//   section); GLM without the extended source terms, with psi damping as the
//   explicit source -kappa*psi; c_h and kappa fixed per step from dt;
//   "max of sum" CFL; Davis wave-speed bounds; van Leer's harmonic slope,
//   Koren's limiter function, Cada and Torrilhon's third-order limiter
//   function without its smooth-extremum switch;
//   first-order fallback per face on non-positive reconstructed rho or p;
//   delta-form SSPRK; pairwise restriction sums; minmod-limited conservative
//   linear prolongation of conserved variables; flux correction (reflux) at
//   coarse/fine faces; one global dt; face ghost slabs only (the
//   dimension-by-dimension stencil never reads edge or corner ghosts).
//
// Plain loops, no blocking or fusion.  Built with -O2 -ffp-contract=off.
// OpenMP runs independent blocks of one phase on several threads; the
// results do not depend on the thread count.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <initializer_list>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int NV = 9;
// conserved: rho, m_x, m_y, m_z, e, B_x, B_y, B_z, psi
enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4, BX = 5, BY = 6, BZ = 7, PSI = 8 };
// primitive: rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi
enum { VX = 1, VY = 2, VZ = 3, PR = 4 };
enum { BC_PERIODIC = 0, BC_ZEROGRAD = 1, BC_REFLECT = 2, BC_FIXED = 3 };
enum { FLAG_SMALL_RHO = 1, FLAG_SMALL_P = 2, FLAG_BAD_DT = 4 };

struct Cell {
  double v[NV];
};

struct Phys {
  double gamma;
  double small_rho;
  double small_p;
  int fix;
};

// ---------------------------------------------------------------------------
// Equation of state and variable conversion (ideal MHD, total energy form,
// Table tab:eqs "mhd"; magnetic pressure |B|^2/2).

Cell prim_to_cons(const Cell& w, double gamma) {
  Cell u;
  const double rho = w.v[RHO];
  u.v[RHO] = rho;
  u.v[MX] = rho * w.v[VX];
  u.v[MY] = rho * w.v[VY];
  u.v[MZ] = rho * w.v[VZ];
  const double v2 = w.v[VX] * w.v[VX] + w.v[VY] * w.v[VY] + w.v[VZ] * w.v[VZ];
  const double b2 = w.v[BX] * w.v[BX] + w.v[BY] * w.v[BY] + w.v[BZ] * w.v[BZ];
  u.v[EN] = w.v[PR] / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * b2;
  u.v[BX] = w.v[BX];
  u.v[BY] = w.v[BY];
  u.v[BZ] = w.v[BZ];
  u.v[PSI] = w.v[PSI];
  return u;
}

// Conserved -> primitive with the small-value check of the Bootstrapping
// section: a cell whose density is not above small_rho or whose pressure is
// not above small_p is reported; with the fix on, the primitive density is
// replaced first (velocity then uses it), then the primitive pressure.  The
// conserved state is never modified and B is never touched.
int cons_to_prim(const Cell& u, const Phys& ph, Cell& w) {
  int bad = 0;
  double rho = u.v[RHO];
  if (!(rho > ph.small_rho)) {
    bad |= FLAG_SMALL_RHO;
    if (ph.fix) rho = ph.small_rho;
  }
  w.v[RHO] = rho;
  w.v[VX] = u.v[MX] / rho;
  w.v[VY] = u.v[MY] / rho;
  w.v[VZ] = u.v[MZ] / rho;
  const double m2 = u.v[MX] * u.v[MX] + u.v[MY] * u.v[MY] + u.v[MZ] * u.v[MZ];
  const double b2 = u.v[BX] * u.v[BX] + u.v[BY] * u.v[BY] + u.v[BZ] * u.v[BZ];
  double p = (ph.gamma - 1.0) * (u.v[EN] - 0.5 * m2 / rho - 0.5 * b2);
  if (!(p > ph.small_p)) {
    bad |= FLAG_SMALL_P;
    if (ph.fix) p = ph.small_p;
  }
  w.v[PR] = p;
  w.v[BX] = u.v[BX];
  w.v[BY] = u.v[BY];
  w.v[BZ] = u.v[BZ];
  w.v[PSI] = u.v[PSI];
  return bad;
}

// Fast magnetosonic speed along direction d.
double fast_speed(const Cell& w, int d, double gamma) {
  const double rho = w.v[RHO];
  const double a2 = gamma * w.v[PR] / rho;
  const double b2 = (w.v[BX] * w.v[BX] + w.v[BY] * w.v[BY] + w.v[BZ] * w.v[BZ]) / rho;
  const double bn2 = w.v[BX + d] * w.v[BX + d] / rho;
  const double s = a2 + b2;
  double disc = s * s - 4.0 * a2 * bn2;
  if (disc < 0.0) disc = 0.0;
  return std::sqrt(0.5 * (s + std::sqrt(disc)));
}

// van Leer (1974) slope: harmonic mean of the one-sided differences when they
// share a sign, zero otherwise (the 'vanleer' row of Table t:limiters).
double vanleer(double dm, double dp) {
  const double prod = dm * dp;
  if (prod > 0.0) return 2.0 * prod / (dm + dp);
  return 0.0;
}

double minmod(double a, double b) {
  if (a * b > 0.0) return std::fabs(a) < std::fabs(b) ? a : b;
  return 0.0;
}

// Koren (1993) limiter function (the 'koren' row of Table t:limiters) of
// r = d+/d-, the ratio of the forward to the backward difference; the face
// value on the forward side is w + phi(r) d- / 2, which is the kappa = 1/3
// third-order value w + d-/6 + d+/3 for 0.4 <= r <= 4.
double koren_phi(double r) { return std::max(0.0, std::min(std::min(2.0 * r, (1.0 + 2.0 * r) / 3.0), 2.0)); }

// Cada and Torrilhon (2009) third-order limiter function (the 'cada3' row of
// Table t:limiters) of theta = d-/d+; the face value on the forward side is
// w + phi(theta) d+ / 2.  It follows the unlimited third-order polynomial
// (2 + theta)/3 where that lies between the lower bounds -theta/2 (which lets
// extrema keep a slope) and the upper bounds 2 theta and 1.6.
double cada3_phi(double th) {
  const double p3 = (2.0 + th) / 3.0;
  return std::max(0.0, std::min(p3, std::max(-0.5 * th, std::min(std::min(2.0 * th, p3), 1.6))));
}

enum { LIM_VANLEER = 0, LIM_KOREN = 1, LIM_CADA3 = 2, LIM_WENO5 = 3, LIM_WENOZ5 = 4, LIM_MP5 = 5, LIM_WENOZP5 = 6 };
enum { WENO_JS = 0, WENO_Z = 1, WENO_ZP = 2 };

bool five_cell_limiter(int lim) { return lim >= LIM_WENO5 && lim <= LIM_WENOZP5; }

// Fifth-order WENO value at the face between cells i and i+1, seen from cell
// i, from cells i-2 .. i+2 (the 'weno5' and 'wenoz5' rows of Table
// t:limiters, 3 ghost cells): the three third-order candidate polynomials
// q_k, their smoothness indicators beta_k and the optimal weights
// (0.1, 0.6, 0.3).  'weno5' (Jiang and Shu 1996): alpha_k = d_k / (eps +
// beta_k)^2 with eps = 1e-6.  'wenoz5' (Borges et al. 2008): alpha_k = d_k
// (1 + tau5 / (beta_k + eps)) with tau5 = |beta_0 - beta_2|, eps = 1e-40.
// 'wenozp5' (Acker et al. 2016): alpha_k = d_k (1 + (tau5 / (beta_k +
// eps))^2 + lambda (beta_k + eps) / (tau5 + eps)) with lambda = dx^(2/3),
// eps = 1e-40.
double weno5_face(double vm2, double vm1, double v0, double vp1, double vp2, int kind, double lambda) {
  const double q0 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0;
  const double q1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0;
  const double q2 = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0;
  const double a0 = vm2 - 2.0 * vm1 + v0, b0 = vm2 - 4.0 * vm1 + 3.0 * v0;
  const double a1 = vm1 - 2.0 * v0 + vp1, b1 = vm1 - vp1;
  const double a2 = v0 - 2.0 * vp1 + vp2, b2 = 3.0 * v0 - 4.0 * vp1 + vp2;
  const double beta[3] = {13.0 / 12.0 * a0 * a0 + 0.25 * b0 * b0, 13.0 / 12.0 * a1 * a1 + 0.25 * b1 * b1,
                          13.0 / 12.0 * a2 * a2 + 0.25 * b2 * b2};
  const double d[3] = {0.1, 0.6, 0.3};
  double alpha[3];
  if (kind == WENO_Z) {
    const double tau5 = std::fabs(beta[0] - beta[2]);
    for (int k = 0; k < 3; ++k) alpha[k] = d[k] * (1.0 + tau5 / (beta[k] + 1e-40));
  } else if (kind == WENO_ZP) {
    const double tau5 = std::fabs(beta[0] - beta[2]);
    for (int k = 0; k < 3; ++k) {
      const double r = tau5 / (beta[k] + 1e-40);
      alpha[k] = d[k] * (1.0 + r * r + lambda * (beta[k] + 1e-40) / (tau5 + 1e-40));
    }
  } else {
    for (int k = 0; k < 3; ++k) alpha[k] = d[k] / ((1e-6 + beta[k]) * (1e-6 + beta[k]));
  }
  const double sum = alpha[0] + alpha[1] + alpha[2];
  return (alpha[0] * q0 + alpha[1] * q1 + alpha[2] * q2) / sum;
}

double minmod2(double a, double b) {
  if (a > 0.0 && b > 0.0) return std::min(a, b);
  if (a < 0.0 && b < 0.0) return std::max(a, b);
  return 0.0;
}

double minmod4(double a, double b, double c, double d) {
  if (a > 0.0 && b > 0.0 && c > 0.0 && d > 0.0) return std::min(std::min(a, b), std::min(c, d));
  if (a < 0.0 && b < 0.0 && c < 0.0 && d < 0.0) return std::max(std::max(a, b), std::max(c, d));
  return 0.0;
}

// Monotonicity-preserving fifth-order value at the face between cells i and
// i+1 seen from cell i, from cells i-2 .. i+2 (the 'mp5' row of Table
// t:limiters; Suresh and Huynh 1997).  The fifth-order interpolant u_or is
// kept when it lies between u_i and the monotonicity bound u_mp = u_i +
// minmod(u_{i+1} - u_i, 4 (u_i - u_{i-1})); otherwise it is limited to the
// interval [u_min, u_max] built from the upper limit u_ul, the median u_md
// and the large-curvature value u_lc, with the curvatures d measured by the
// four-argument minmod of neighbouring second differences.  The acceptance
// test is taken without a round-off epsilon.
double mp5_face(double vm2, double vm1, double v0, double vp1, double vp2) {
  const double alpha = 4.0;
  const double u_or = (2.0 * vm2 - 13.0 * vm1 + 47.0 * v0 + 27.0 * vp1 - 3.0 * vp2) / 60.0;
  const double u_mp = v0 + minmod2(vp1 - v0, alpha * (v0 - vm1));
  if ((u_or - v0) * (u_or - u_mp) <= 0.0) return u_or;
  const double dm1 = vm2 - 2.0 * vm1 + v0;  // second differences at i-1, i, i+1
  const double d0 = vm1 - 2.0 * v0 + vp1;
  const double dp1 = v0 - 2.0 * vp1 + vp2;
  const double dm4_plus = minmod4(4.0 * d0 - dp1, 4.0 * dp1 - d0, d0, dp1);
  const double dm4_minus = minmod4(4.0 * d0 - dm1, 4.0 * dm1 - d0, d0, dm1);
  const double u_ul = v0 + alpha * (v0 - vm1);
  const double u_av = 0.5 * (v0 + vp1);
  const double u_md = u_av - 0.5 * dm4_plus;
  const double u_lc = v0 + 0.5 * (v0 - vm1) + 4.0 / 3.0 * dm4_minus;
  const double u_min = std::max(std::min(std::min(v0, vp1), u_md), std::min(std::min(v0, u_ul), u_lc));
  const double u_max = std::min(std::max(std::max(v0, vp1), u_md), std::max(std::max(v0, u_ul), u_lc));
  // the median of u_or, u_min and u_max
  return u_or + minmod2(u_min - u_or, u_max - u_or);
}

// One of the fifth-order face values above by limiter id.
double five_cell_face(int lim, double vm2, double vm1, double v0, double vp1, double vp2, double lambda) {
  if (lim == LIM_MP5) return mp5_face(vm2, vm1, v0, vp1, vp2);
  const int kind = lim == LIM_WENOZ5 ? WENO_Z : (lim == LIM_WENOZP5 ? WENO_ZP : WENO_JS);
  return weno5_face(vm2, vm1, v0, vp1, vp2, kind, lambda);
}

// The two face values of a cell with backward and forward differences dm, dp:
// right face w + inc_right/2, left face w - inc_left/2.  The left face is the
// right face of the mirrored stencil (dm, dp -> -dp, -dm).  A zero difference
// in a ratio's denominator gives a zero increment (its limit).
void face_increments(int lim, double dm, double dp, double* inc_right, double* inc_left) {
  if (lim == LIM_KOREN) {
    *inc_right = dm != 0.0 ? koren_phi(dp / dm) * dm : 0.0;
    *inc_left = dp != 0.0 ? koren_phi(dm / dp) * dp : 0.0;
  } else if (lim == LIM_CADA3) {
    *inc_right = dp != 0.0 ? cada3_phi(dm / dp) * dp : 0.0;
    *inc_left = dm != 0.0 ? cada3_phi(dp / dm) * dm : 0.0;
  } else {
    *inc_right = vanleer(dm, dp);
    *inc_left = *inc_right;
  }
}

// Physical ideal-MHD flux along d for every component except B_d and psi,
// which the GLM interface solve supplies.
void phys_flux(const Cell& w, const Cell& u, int d, double f[NV]) {
  const double vn = w.v[VX + d];
  const double bn = w.v[BX + d];
  const double b2 = w.v[BX] * w.v[BX] + w.v[BY] * w.v[BY] + w.v[BZ] * w.v[BZ];
  const double ptot = w.v[PR] + 0.5 * b2;
  const double vb = w.v[VX] * w.v[BX] + w.v[VY] * w.v[BY] + w.v[VZ] * w.v[BZ];
  f[RHO] = u.v[MX + d];
  for (int j = 0; j < 3; ++j) {
    f[MX + j] = u.v[MX + j] * vn - w.v[BX + j] * bn;
    if (j == d) f[MX + j] += ptot;
  }
  f[EN] = (u.v[EN] + ptot) * vn - bn * vb;
  for (int j = 0; j < 3; ++j) f[BX + j] = (j == d) ? 0.0 : vn * w.v[BX + j] - bn * w.v[VX + j];
  f[PSI] = 0.0;
}

// Exact solution of the linear (B_n, psi) Riemann problem of the mixed GLM
// system d_t B_n + d_n psi = 0, d_t psi + c_h^2 d_n B_n = 0 (Dedner 2002).
void glm_interface(double bnl, double bnr, double psl, double psr, double ch, double* bn,
                   double* ps) {
  *bn = 0.5 * (bnl + bnr) - (psr - psl) / (2.0 * ch);
  *ps = 0.5 * (psl + psr) - 0.5 * ch * (bnr - bnl);
}

enum { FLUX_HLL = 0, FLUX_HLLD = 1, FLUX_HLLC = 2 };

// HLLD (Miyoshi and Kusano 2005; the 'hlld' entry of Table
// tab:schemes_space, used there with glm) on the seven components other than
// B_n and psi; bx is the normal field, the same on both sides.  Notation: u
// the normal velocity, pT = p + |B|^2/2 the total pressure, t the two
// tangential directions.  Wave speeds: S_L, S_R bracket both fast speeds
// around both normal velocities; S_M is the contact (entropy) speed; S*_L,
// S*_R the rotational (Alfven) waves S_M -/+ |bx| / sqrt(rho*).
void hlld_flux(const Cell& wl, const Cell& wr, const Cell& ul, const Cell& ur, const double fl[NV],
               const double fr[NV], int d, double bx, double gamma, double F[NV]) {
  const int MN = MX + d;
  int tan[2], k = 0;
  for (int j = 0; j < 3; ++j)
    if (j != d) tan[k++] = j;
  const double rho[2] = {wl.v[RHO], wr.v[RHO]};
  const double un[2] = {wl.v[VX + d], wr.v[VX + d]};
  double pt[2];
  for (int a = 0; a < 2; ++a) {
    const Cell& w = a ? wr : wl;
    pt[a] = w.v[PR] + 0.5 * (w.v[BX] * w.v[BX] + w.v[BY] * w.v[BY] + w.v[BZ] * w.v[BZ]);
  }
  const double cfmax = std::max(fast_speed(wl, d, gamma), fast_speed(wr, d, gamma));
  const double S[2] = {std::min(un[0], un[1]) - cfmax, std::max(un[0], un[1]) + cfmax};
  auto copy7 = [&](const double* f) {
    for (int q = 0; q < NV; ++q)
      if (q != BX + d && q != PSI) F[q] = f[q];
  };
  if (S[0] > 0.0) { copy7(fl); return; }
  if (S[1] < 0.0) { copy7(fr); return; }
  // contact speed and the total pressure of the star region
  const double dl = (S[0] - un[0]) * rho[0], dr = (S[1] - un[1]) * rho[1];
  const double sm = (dr * un[1] - dl * un[0] - pt[1] + pt[0]) / (dr - dl);
  const double pts = (dr * pt[0] - dl * pt[1] + rho[0] * rho[1] * (S[1] - un[1]) * (S[0] - un[0]) * (un[1] - un[0])) /
                     (dr - dl);
  // single-star states U*_L, U*_R
  Cell us[2];
  double rs[2], vs[2][2], bs[2][2];
  for (int a = 0; a < 2; ++a) {
    const Cell& w = a ? wr : wl;
    const Cell& u = a ? ur : ul;
    const double sa = S[a] - un[a], sb = S[a] - sm;
    rs[a] = rho[a] * sa / sb;
    const double den = rho[a] * sa * sb - bx * bx;
    const bool degenerate = std::fabs(den) <= 1e-12 * rho[a] * sa * sa;
    for (int t = 0; t < 2; ++t) {
      const double vt = w.v[VX + tan[t]], bt = w.v[BX + tan[t]];
      if (degenerate) {
        vs[a][t] = vt;
        bs[a][t] = bt;
      } else {
        vs[a][t] = vt - bx * bt * (sm - un[a]) / den;
        bs[a][t] = bt * (rho[a] * sa * sa - bx * bx) / den;
      }
    }
    const double vb = un[a] * bx + w.v[VX + tan[0]] * w.v[BX + tan[0]] + w.v[VX + tan[1]] * w.v[BX + tan[1]];
    const double vbs = sm * bx + vs[a][0] * bs[a][0] + vs[a][1] * bs[a][1];
    Cell& x = us[a];
    x = u;  // B_n and psi are not HLLD components
    x.v[RHO] = rs[a];
    x.v[MN] = rs[a] * sm;
    x.v[EN] = (sa * u.v[EN] - pt[a] * un[a] + pts * sm + bx * (vb - vbs)) / sb;
    for (int t = 0; t < 2; ++t) {
      x.v[MX + tan[t]] = rs[a] * vs[a][t];
      x.v[BX + tan[t]] = bs[a][t];
    }
  }
  // the side of the contact the interface lies on
  const int a = sm >= 0.0 ? 0 : 1;
  const Cell& ua = a ? ur : ul;
  const double* fa = a ? fr : fl;
  double Fs[NV];
  for (int q = 0; q < NV; ++q) Fs[q] = fa[q] + S[a] * (us[a].v[q] - ua.v[q]);
  const double sql = std::sqrt(rs[0]), sqr = std::sqrt(rs[1]);
  const double sas = a == 0 ? sm - std::fabs(bx) / sql : sm + std::fabs(bx) / sqr;  // S*_L or S*_R
  const bool inner = a == 0 ? sas < 0.0 : sas > 0.0;  // between the Alfven wave and the contact
  if (!inner) { copy7(Fs); return; }
  // double-star state U**_a
  const double sg = bx > 0.0 ? 1.0 : (bx < 0.0 ? -1.0 : 0.0);
  double vss[2], bss[2];
  for (int t = 0; t < 2; ++t) {
    vss[t] = (sql * vs[0][t] + sqr * vs[1][t] + (bs[1][t] - bs[0][t]) * sg) / (sql + sqr);
    bss[t] = (sql * bs[1][t] + sqr * bs[0][t] + sql * sqr * (vs[1][t] - vs[0][t]) * sg) / (sql + sqr);
  }
  const double vbs_a = sm * bx + vs[a][0] * bs[a][0] + vs[a][1] * bs[a][1];
  const double vbss = sm * bx + vss[0] * bss[0] + vss[1] * bss[1];
  Cell uss = us[a];
  uss.v[EN] = a == 0 ? us[0].v[EN] - sql * (vbs_a - vbss) * sg : us[1].v[EN] + sqr * (vbs_a - vbss) * sg;
  for (int t = 0; t < 2; ++t) {
    uss.v[MX + tan[t]] = rs[a] * vss[t];
    uss.v[BX + tan[t]] = bss[t];
  }
  double Fss[NV];
  for (int q = 0; q < NV; ++q) Fss[q] = Fs[q] + sas * (uss.v[q] - us[a].v[q]);
  copy7(Fss);
}

// HLLC for MHD (Li 2005; the 'hllc' entry of Table tab:schemes_space) on the
// seven components other than B_n and psi; bx is the normal field on both
// sides.  S_L, S_R are the Davis bounds of the HLL flux and S_M the contact
// speed.  The tangential field and velocity of both star states are those of
// the HLL average state; density, momentum and energy of each star state
// follow from the jump conditions across S_L or S_R with normal velocity
// S_M and total pressure pT* = rho_L (S_L - u_L)(S_M - u_L) + pT_L.
void hllc_flux(const Cell& wl, const Cell& wr, const Cell& ul, const Cell& ur, const double fl[NV],
               const double fr[NV], int d, double bx, double gamma, double F[NV]) {
  const int MN = MX + d;
  int tan[2], k = 0;
  for (int j = 0; j < 3; ++j)
    if (j != d) tan[k++] = j;
  auto copy7 = [&](const double* f) {
    for (int q = 0; q < NV; ++q)
      if (q != BX + d && q != PSI) F[q] = f[q];
  };
  const double cl = fast_speed(wl, d, gamma), cr = fast_speed(wr, d, gamma);
  const double uln = wl.v[VX + d], urn = wr.v[VX + d];
  const double S[2] = {std::min(uln - cl, urn - cr), std::max(uln + cl, urn + cr)};
  if (S[0] >= 0.0) { copy7(fl); return; }
  if (S[1] <= 0.0) { copy7(fr); return; }
  // HLL average state
  double uh[NV];
  for (int q = 0; q < NV; ++q) uh[q] = (S[1] * ur.v[q] - S[0] * ul.v[q] - (fr[q] - fl[q])) / (S[1] - S[0]);
  double pt[2];
  for (int a = 0; a < 2; ++a) {
    const Cell& w = a ? wr : wl;
    pt[a] = w.v[PR] + 0.5 * (w.v[BX] * w.v[BX] + w.v[BY] * w.v[BY] + w.v[BZ] * w.v[BZ]);
  }
  const double rho[2] = {wl.v[RHO], wr.v[RHO]}, un[2] = {uln, urn};
  const double sm = (rho[1] * un[1] * (S[1] - un[1]) - rho[0] * un[0] * (S[0] - un[0]) + pt[0] - pt[1]) /
                    (rho[1] * (S[1] - un[1]) - rho[0] * (S[0] - un[0]));
  const double pts = rho[0] * (S[0] - un[0]) * (sm - un[0]) + pt[0];
  double bs[2], vs[2];
  for (int t = 0; t < 2; ++t) {
    bs[t] = uh[BX + tan[t]];
    vs[t] = uh[MX + tan[t]] / uh[RHO];
  }
  const double vbs = sm * bx + vs[0] * bs[0] + vs[1] * bs[1];
  const int a = sm >= 0.0 ? 0 : 1;
  const Cell& w = a ? wr : wl;
  const Cell& u = a ? ur : ul;
  const double* f = a ? fr : fl;
  const double sa = S[a] - un[a], sb = S[a] - sm;
  Cell us = u;  // B_n and psi are not HLLC components
  us.v[RHO] = rho[a] * sa / sb;
  us.v[MN] = us.v[RHO] * sm;
  for (int t = 0; t < 2; ++t) {
    us.v[MX + tan[t]] = (rho[a] * w.v[VX + tan[t]] * sa + bx * (w.v[BX + tan[t]] - bs[t])) / sb;
    us.v[BX + tan[t]] = bs[t];
  }
  const double vb = un[a] * bx + w.v[VX + tan[0]] * w.v[BX + tan[0]] + w.v[VX + tan[1]] * w.v[BX + tan[1]];
  us.v[EN] = (u.v[EN] * sa - pt[a] * un[a] + pts * sm + bx * (vb - vbs)) / sb;
  double Fs[NV];
  for (int q = 0; q < NV; ++q) Fs[q] = f[q] + S[a] * (us.v[q] - u.v[q]);
  copy7(Fs);
}

// Interface flux from the reconstructed left/right primitive states: GLM
// interface values for (B_n, psi), then HLL with Davis speed bounds (or
// HLLD) on the other seven components, built from the states with B_n
// replaced.
void face_flux(Cell wl, Cell wr, int d, double ch, double gamma, double F[NV], int flux = FLUX_HLL) {
  double bn, ps;
  glm_interface(wl.v[BX + d], wr.v[BX + d], wl.v[PSI], wr.v[PSI], ch, &bn, &ps);
  wl.v[BX + d] = bn;
  wr.v[BX + d] = bn;
  const Cell ul = prim_to_cons(wl, gamma);
  const Cell ur = prim_to_cons(wr, gamma);
  double fl[NV], fr[NV];
  phys_flux(wl, ul, d, fl);
  phys_flux(wr, ur, d, fr);
  F[BX + d] = ps;
  F[PSI] = ch * ch * bn;
  if (flux == FLUX_HLLD) {
    hlld_flux(wl, wr, ul, ur, fl, fr, d, bn, gamma, F);
    return;
  }
  if (flux == FLUX_HLLC) {
    hllc_flux(wl, wr, ul, ur, fl, fr, d, bn, gamma, F);
    return;
  }
  const double cl = fast_speed(wl, d, gamma);
  const double cr = fast_speed(wr, d, gamma);
  const double sl = std::min(wl.v[VX + d] - cl, wr.v[VX + d] - cr);
  const double sr = std::max(wl.v[VX + d] + cl, wr.v[VX + d] + cr);
  for (int q = 0; q < NV; ++q) {
    if (q == BX + d || q == PSI) continue;
    if (sl >= 0.0) {
      F[q] = fl[q];
    } else if (sr <= 0.0) {
      F[q] = fr[q];
    } else {
      F[q] = (sr * fl[q] - sl * fr[q] + sl * sr * (ur.v[q] - ul.v[q])) / (sr - sl);
    }
  }
  F[BX + d] = ps;
  F[PSI] = ch * ch * bn;
}

// ---------------------------------------------------------------------------
// Block hierarchy.

struct Key {
  int l;
  long i, j, k;
  bool operator==(const Key& o) const { return l == o.l && i == o.i && j == o.j && k == o.k; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = (uint64_t)k.l * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.i + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.j + 0x8CB92BA72F3D8DD7ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.k + 0x52DCE729DA3ED8FBull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

using Idx = std::array<long, 3>;
using BlockData = std::vector<Cell>;

}  // namespace

extern "C" {

// Parameter record shared with the Python test wrapper (ctypes mirror).
typedef struct {
  int ndim;
  int nx;
  int ng;
  int nstages;  // 1 = forward Euler, 2 = SSPRK(2,2), 3 = SSPRK(3,3), 4 = SSPRK(4,3), 5 = SSPRK(5,4)
  int reflux;
  int fix_small_values;
  int nthreads;
  int base_blocks[3];
  int bc_lo[3];
  int bc_hi[3];
  double xmin[3];
  double xmax[3];
  double bc_fixed_prim[3][2][NV];
  double gamma;
  double cfl;
  double glm_alpha;
  double small_density;
  double small_pressure;
  int limiter;  // 0 'vanleer', 1 'koren', 2 'cada3', 3 'weno5', 4 'wenoz5', 5 'mp5', 6 'wenozp5'
  int flux;     // 0 = HLL, 1 = HLLD, 2 = HLLC
} oracle_params;

}  // extern "C"

namespace {

struct Sim {
  oracle_params P;
  Phys ph;
  int ndim, nx, ng, pn;
  long pcells;  // padded cells per block (corners included, unused)
  long icells;  // interior cells per block
  int nb;
  int finest;
  std::vector<int> lev;
  std::vector<Idx> pos;
  std::unordered_map<Key, int, KeyHash> leaf;
  std::unordered_set<Key, KeyHash> refined;
  Cell fixedU[3][2];
  std::vector<BlockData> S0, S1, S2;            // state slots
  std::vector<BlockData> S3, S4, L3;            // SSPRK(5,4) only: u3, u4 and L(u3)
  std::vector<BlockData> Lb;                    // L of the current stage input
  std::vector<std::array<BlockData, 3>> flux;  // face fluxes per block and direction
  int flags = 0;
  long nfix = 0;
  double last_dt = 0, last_ch = 0, last_kappa = 0;

  long ncell(int l, int d) const { return d < ndim ? ((long)P.base_blocks[d] * nx) << (l - 1) : 1; }
  double dx(int l, int d) const { return (P.xmax[d] - P.xmin[d]) / (double)ncell(l, d); }

  // padded index, i/j/k in [-ng, nx+ng)
  long pidx(long i, long j, long k) const {
    const long kk = ndim == 3 ? k + ng : 0;
    return (kk * pn + (j + ng)) * pn + (i + ng);
  }
  long pidx(const Idx& c) const { return pidx(c[0], c[1], c[2]); }

  // Conserved value of the level-l cell with global index g, defined from the
  // leaf interiors alone: same-level leaf copy, periodic wrap, physical
  // boundary, restriction of the finer leaves covering it, or prolongation of
  // the coarser leaf covering it.
  Cell lookup(const std::vector<BlockData>& S, int l, Idx g, bool allow_prolong) const {
    for (int d = 0; d < ndim; ++d) {
      const long n = ncell(l, d);
      if (g[d] >= 0 && g[d] < n) continue;
      const int side = g[d] < 0 ? 0 : 1;
      const int bc = side ? P.bc_hi[d] : P.bc_lo[d];
      if (bc == BC_PERIODIC) {
        g[d] = ((g[d] % n) + n) % n;
        continue;
      }
      Idx h = g;
      if (bc == BC_ZEROGRAD) {
        h[d] = side ? n - 1 : 0;
        return lookup(S, l, h, allow_prolong);
      }
      if (bc == BC_REFLECT) {
        h[d] = side ? 2 * n - 1 - g[d] : -1 - g[d];
        Cell c = lookup(S, l, h, allow_prolong);
        c.v[MX + d] = -c.v[MX + d];
        c.v[BX + d] = -c.v[BX + d];
        return c;
      }
      if (bc == BC_FIXED) return fixedU[d][side];
      throw std::logic_error("unknown boundary kind");
    }
    Key key{l, g[0] / nx, ndim > 1 ? g[1] / nx : 0, ndim > 2 ? g[2] / nx : 0};
    auto it = leaf.find(key);
    if (it != leaf.end()) {
      const Idx loc{g[0] - key.i * nx, g[1] - key.j * nx, ndim > 2 ? g[2] - key.k * nx : 0};
      return S[it->second][pidx(loc)];
    }
    if (refined.count(key)) return restrict_cell(S, l, g);
    if (!allow_prolong) throw std::logic_error("ghost stencil needs a prolongation of a prolongation (hierarchy not 2:1 nested)");
    return prolong_cell(S, l, g);
  }

  Cell fine_leaf_cell(const std::vector<BlockData>& S, int l, const Idx& g) const {
    Key key{l, g[0] / nx, ndim > 1 ? g[1] / nx : 0, ndim > 2 ? g[2] / nx : 0};
    auto it = leaf.find(key);
    if (it == leaf.end()) throw std::logic_error("restriction source is not a leaf (hierarchy not 2:1 nested)");
    const Idx loc{g[0] - key.i * nx, g[1] - key.j * nx, ndim > 2 ? g[2] - key.k * nx : 0};
    return S[it->second][pidx(loc)];
  }

  // Volume average of the 2^d children, summed pairwise (x pairs, then y,
  // then z) and scaled by 2^-d.
  Cell restrict_cell(const std::vector<BlockData>& S, int l, const Idx& g) const {
    Cell r;
    if (ndim == 2) {
      Cell c[2][2];
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) c[b][a] = fine_leaf_cell(S, l + 1, Idx{2 * g[0] + a, 2 * g[1] + b, 0});
      for (int q = 0; q < NV; ++q)
        r.v[q] = ((c[0][0].v[q] + c[0][1].v[q]) + (c[1][0].v[q] + c[1][1].v[q])) * 0.25;
    } else {
      Cell c[2][2][2];
      for (int e = 0; e < 2; ++e)
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a)
            c[e][b][a] = fine_leaf_cell(S, l + 1, Idx{2 * g[0] + a, 2 * g[1] + b, 2 * g[2] + e});
      for (int q = 0; q < NV; ++q)
        r.v[q] = (((c[0][0][0].v[q] + c[0][0][1].v[q]) + (c[0][1][0].v[q] + c[0][1][1].v[q])) +
                  ((c[1][0][0].v[q] + c[1][0][1].v[q]) + (c[1][1][0].v[q] + c[1][1][1].v[q]))) *
                 0.125;
    }
    return r;
  }

  // Conservative linear prolongation: parent value plus a quarter of the
  // minmod-limited parent slope per direction, towards the child's side.
  Cell prolong_cell(const std::vector<BlockData>& S, int l, const Idx& g) const {
    if (l <= 1) throw std::logic_error("prolongation requested on the base level");
    Idx gc{g[0] >> 1, ndim > 1 ? g[1] >> 1 : 0, ndim > 2 ? g[2] >> 1 : 0};
    Key pk{l - 1, gc[0] / nx, ndim > 1 ? gc[1] / nx : 0, ndim > 2 ? gc[2] / nx : 0};
    if (!leaf.count(pk)) throw std::logic_error("prolongation parent is not a leaf (hierarchy not 2:1 nested)");
    const Cell uc = lookup(S, l - 1, gc, false);
    Cell r = uc;
    for (int d = 0; d < ndim; ++d) {
      Idx lo = gc, hi = gc;
      lo[d] -= 1;
      hi[d] += 1;
      const Cell um = lookup(S, l - 1, lo, false);
      const Cell up = lookup(S, l - 1, hi, false);
      const double s = (g[d] & 1) ? 0.25 : -0.25;
      for (int q = 0; q < NV; ++q) r.v[q] = r.v[q] + s * minmod(uc.v[q] - um.v[q], up.v[q] - uc.v[q]);
    }
    return r;
  }

  // Fill the face ghost slabs of every block of slot S (all 2*ndim faces,
  // ng deep, interior-wide in the other directions).
  void fill_ghosts(std::vector<BlockData>& S) {
    const std::vector<BlockData>& cS = S;
    std::vector<std::vector<std::pair<long, Cell>>> out(nb);
#pragma omp parallel for schedule(dynamic) num_threads(P.nthreads)
    for (int b = 0; b < nb; ++b) {
      const int l = lev[b];
      for (int d = 0; d < ndim; ++d) {
        for (int side = 0; side < 2; ++side) {
          const long a0 = side ? nx : -ng, a1 = side ? nx + ng : 0;
          const long kmax = ndim == 3 ? nx : 1;
          for (long k = 0; k < kmax; ++k)
            for (long j = 0; j < nx; ++j)
              for (long a = a0; a < a1; ++a) {
                Idx loc;
                // loc along d is a; the remaining interior directions are j, k
                if (d == 0) loc = Idx{a, j, k};
                else if (d == 1) loc = Idx{j, a, k};
                else loc = Idx{j, k, a};
                if (ndim == 2) loc[2] = 0;
                Idx g{pos[b][0] * nx + loc[0], pos[b][1] * nx + loc[1], ndim == 3 ? pos[b][2] * nx + loc[2] : 0};
                out[b].emplace_back(pidx(loc), lookup(cS, l, g, true));
              }
        }
      }
    }
    for (int b = 0; b < nb; ++b)
      for (auto& pc : out[b]) S[b][pc.first] = pc.second;
  }

  // Time step, c_h and kappa from the leaf interior cells of S.
  void cfl(const std::vector<BlockData>& S, double* dt, double* ch, double* kappa) {
    double rmax = 0.0;
    bool nan_seen = false;
    int f = 0;
    for (int b = 0; b < nb; ++b) {
      const int l = lev[b];
      const long kmax = ndim == 3 ? nx : 1;
      for (long k = 0; k < kmax; ++k)
        for (long j = 0; j < nx; ++j)
          for (long i = 0; i < nx; ++i) {
            Cell w;
            f |= cons_to_prim(S[b][pidx(i, j, k)], ph, w);
            double r = 0.0;
            for (int d = 0; d < ndim; ++d)
              r += (std::fabs(w.v[VX + d]) + fast_speed(w, d, ph.gamma)) / dx(l, d);
            if (std::isnan(r)) nan_seen = true;
            else if (r > rmax) rmax = r;
          }
    }
    double sum_inv = 0.0, min_dx = 0.0;
    for (int d = 0; d < ndim; ++d) {
      sum_inv += 1.0 / dx(finest, d);
      min_dx = d == 0 ? dx(finest, d) : std::min(min_dx, dx(finest, d));
    }
    if (nan_seen || !(rmax > 0.0) || !std::isfinite(rmax)) {
      f |= FLAG_BAD_DT;
      *dt = 0.0;
      *ch = 0.0;
      *kappa = 0.0;
    } else {
      *dt = P.cfl / rmax;
      *ch = P.cfl / (*dt * sum_inv);
      *kappa = P.glm_alpha * *ch / min_dx;
    }
    flags |= f;
  }

  // L(in) on the interior cells of every block: ghost fill, primitives,
  // reconstructed face states, face fluxes, the flux correction at
  // coarse/fine faces, then minus the flux difference over dx plus the psi
  // damping source (the right-hand side of the method-of-lines form).
  void rhs(std::vector<BlockData>& in, std::vector<BlockData>& L_out, double ch, double kappa) {
    if (L_out.size() != (size_t)nb) L_out.assign(nb, BlockData(pcells));
    fill_ghosts(in);
    const long kmax = ndim == 3 ? nx : 1;
    int fl = 0;
    long nf = 0;
#pragma omp parallel for schedule(dynamic) num_threads(P.nthreads) reduction(| : fl) reduction(+ : nf)
    for (int b = 0; b < nb; ++b) {
      // primitives on interior and face ghost cells
      std::vector<Cell> W(pcells);
      for (long k = (ndim == 3 ? -ng : 0); k < (ndim == 3 ? nx + ng : 1); ++k)
        for (long j = -ng; j < nx + ng; ++j)
          for (long i = -ng; i < nx + ng; ++i) {
            int out_i = (i < 0 || i >= nx), out_j = (j < 0 || j >= nx),
                out_k = ndim == 3 && (k < 0 || k >= nx);
            if (out_i + out_j + out_k > 1) continue;  // edge/corner cells are never read
            const int bad = cons_to_prim(in[b][pidx(i, j, k)], ph, W[pidx(i, j, k)]);
            fl |= bad;
            if (bad && ph.fix) ++nf;
          }
      for (int d = 0; d < ndim; ++d) {
        BlockData& F = flux[b][d];
        // faces f = 0..nx along d, f between cells f-1 and f
        for (long t2 = 0; t2 < kmax; ++t2)
          for (long t1 = 0; t1 < nx; ++t1)
            for (long f = 0; f <= nx; ++f) {
              auto at = [&](long a) -> const Cell& {
                if (d == 0) return W[pidx(a, t1, t2)];
                if (d == 1) return W[pidx(t1, a, t2)];
                return W[pidx(t1, t2, a)];
              };
              const Cell& wmm = at(f - 2);
              const Cell& wm = at(f - 1);
              const Cell& wp = at(f);
              const Cell& wpp = at(f + 1);
              Cell wl, wr;
              if (five_cell_limiter(P.limiter)) {
                // five-point stencils f-3 .. f+1 (left state) and f+2 .. f-2
                // (right state, mirrored)
                const double lambda = std::pow(dx(lev[b], d), 2.0 / 3.0);
                const Cell& wm3 = at(f - 3);
                const Cell& wp2 = at(f + 2);
                for (int q = 0; q < NV; ++q) {
                  wl.v[q] = five_cell_face(P.limiter, wm3.v[q], wmm.v[q], wm.v[q], wp.v[q], wpp.v[q], lambda);
                  wr.v[q] = five_cell_face(P.limiter, wp2.v[q], wpp.v[q], wp.v[q], wm.v[q], wmm.v[q], lambda);
                }
              } else {
                for (int q = 0; q < NV; ++q) {
                  double rm, lm, rp, lp;
                  face_increments(P.limiter, wm.v[q] - wmm.v[q], wp.v[q] - wm.v[q], &rm, &lm);
                  face_increments(P.limiter, wp.v[q] - wm.v[q], wpp.v[q] - wp.v[q], &rp, &lp);
                  wl.v[q] = wm.v[q] + 0.5 * rm;
                  wr.v[q] = wp.v[q] - 0.5 * lp;
                }
              }
              if (!(wl.v[RHO] > 0.0) || !(wl.v[PR] > 0.0) || !(wr.v[RHO] > 0.0) || !(wr.v[PR] > 0.0)) {
                wl = wm;
                wr = wp;
              }
              face_flux(wl, wr, d, ch, ph.gamma, F[(t2 * nx + t1) * (nx + 1) + f].v, P.flux);
            }
      }
    }
    flags |= fl;
    nfix += nf;
    if (P.reflux) do_reflux();
#pragma omp parallel for schedule(dynamic) num_threads(P.nthreads)
    for (int b = 0; b < nb; ++b) {
      const int l = lev[b];
      for (long k = 0; k < kmax; ++k)
        for (long j = 0; j < nx; ++j)
          for (long i = 0; i < nx; ++i) {
            const long c = pidx(i, j, k);
            const Cell& u = in[b][c];
            double L[NV];
            for (int q = 0; q < NV; ++q) L[q] = 0.0;
            for (int d = 0; d < ndim; ++d) {
              long f, t1, t2;
              if (d == 0) { f = i; t1 = j; t2 = k; }
              else if (d == 1) { f = j; t1 = i; t2 = k; }
              else { f = k; t1 = i; t2 = j; }
              const Cell& flo = flux[b][d][(t2 * nx + t1) * (nx + 1) + f];
              const Cell& fhi = flux[b][d][(t2 * nx + t1) * (nx + 1) + f + 1];
              const double h = dx(l, d);
              for (int q = 0; q < NV; ++q) L[q] = L[q] + (fhi.v[q] - flo.v[q]) / h;
            }
            for (int q = 0; q < NV; ++q) L[q] = -L[q];
            L[PSI] = L[PSI] - kappa * u.v[PSI];
            for (int q = 0; q < NV; ++q) L_out[b][c].v[q] = L[q];
          }
    }
  }

  // One explicit stage: out = base + w*((in + dt*L(in)) - base), or
  // out = in + dt*L(in) when w == 1 (the advect1 statement of the IMEX
  // implementation section with the SSPRK combination folded in).
  void stage(std::vector<BlockData>& in, const std::vector<BlockData>* base,
             std::vector<BlockData>& out, double w, double dt, double ch, double kappa) {
    rhs(in, Lb, ch, kappa);
    const long kmax = ndim == 3 ? nx : 1;
#pragma omp parallel for schedule(dynamic) num_threads(P.nthreads)
    for (int b = 0; b < nb; ++b)
      for (long k = 0; k < kmax; ++k)
        for (long j = 0; j < nx; ++j)
          for (long i = 0; i < nx; ++i) {
            const long c = pidx(i, j, k);
            const Cell& u = in[b][c];
            const Cell& L = Lb[b][c];
            Cell& o = out[b][c];
            for (int q = 0; q < NV; ++q) {
              const double t = u.v[q] + dt * L.v[q];
              if (w == 1.0) {
                o.v[q] = t;
              } else {
                const double u0 = (*base)[b][c].v[q];
                o.v[q] = u0 + w * (t - u0);
              }
            }
          }
  }

  // One row of a Shu-Osher scheme whose state weights sum to one, evaluated
  // around u0 (delta form, so a uniform state stays exact):
  //   out = u0 + sum_j a_j (u_j - u0) + sum_j b_j dt L_j   (interior cells)
  using Term = std::pair<double, const std::vector<BlockData>*>;
  void shu_osher(std::vector<BlockData>& out, const std::vector<BlockData>& u0, std::initializer_list<Term> us,
                 std::initializer_list<Term> ls, double dt) {
    const long kmax = ndim == 3 ? nx : 1;
#pragma omp parallel for schedule(dynamic) num_threads(P.nthreads)
    for (int b = 0; b < nb; ++b)
      for (long k = 0; k < kmax; ++k)
        for (long j = 0; j < nx; ++j)
          for (long i = 0; i < nx; ++i) {
            const long c = pidx(i, j, k);
            for (int q = 0; q < NV; ++q) {
              const double z = u0[b][c].v[q];
              double acc = 0.0;
              for (const Term& t : us) acc = acc + t.first * ((*t.second)[b][c].v[q] - z);
              for (const Term& t : ls) acc = acc + t.first * (dt * (*t.second)[b][c].v[q]);
              out[b][c].v[q] = z + acc;
            }
          }
  }

  // Flux correction at coarse/fine faces: the coarse face flux becomes the
  // pairwise mean of the 2^(d-1) fine face fluxes covering it.
  void do_reflux() {
    const long kmax = ndim == 3 ? nx : 1;
    for (int b = 0; b < nb; ++b) {
      const int l = lev[b];
      for (int d = 0; d < ndim; ++d)
        for (int side = 0; side < 2; ++side) {
          Idx nbp = pos[b];
          nbp[d] += side ? 1 : -1;
          const long nblk = (long)P.base_blocks[d] << (l - 1);
          if (nbp[d] < 0 || nbp[d] >= nblk) {
            if ((side ? P.bc_hi[d] : P.bc_lo[d]) != BC_PERIODIC) continue;
            nbp[d] = (nbp[d] + nblk) % nblk;
          }
          if (!refined.count(Key{l, nbp[0], nbp[1], nbp[2]})) continue;
          // fine face index along d, and fine block position along d
          const long fine_blk_d = side ? 2 * nbp[d] : 2 * nbp[d] + 1;
          const long ff = side ? 0 : nx;
          const long cf = side ? nx : 0;
          for (long t2 = 0; t2 < kmax; ++t2)
            for (long t1 = 0; t1 < nx; ++t1) {
              // global coarse transverse cell indices
              const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
              Idx gct{0, 0, 0};
              gct[ta] = pos[b][ta] * nx + t1;
              if (ndim == 3) gct[tb] = pos[b][tb] * nx + t2;
              Cell fv[2][2];
              for (int e = 0; e < (ndim == 3 ? 2 : 1); ++e)
                for (int a = 0; a < 2; ++a) {
                  Idx gf{0, 0, 0};
                  gf[ta] = 2 * gct[ta] + a;
                  if (ndim == 3) gf[tb] = 2 * gct[tb] + e;
                  Idx fb{0, 0, 0};
                  fb[d] = fine_blk_d;
                  fb[ta] = gf[ta] / nx;
                  if (ndim == 3) fb[tb] = gf[tb] / nx;
                  auto it = leaf.find(Key{l + 1, fb[0], fb[1], fb[2]});
                  if (it == leaf.end()) throw std::logic_error("reflux partner is not a leaf");
                  const long ft1 = gf[ta] - fb[ta] * nx;
                  const long ft2 = ndim == 3 ? gf[tb] - fb[tb] * nx : 0;
                  fv[e][a] = flux[it->second][d][(ft2 * nx + ft1) * (nx + 1) + ff];
                }
              Cell& cflux = flux[b][d][(t2 * nx + t1) * (nx + 1) + cf];
              for (int q = 0; q < NV; ++q) {
                if (ndim == 2)
                  cflux.v[q] = (fv[0][0].v[q] + fv[0][1].v[q]) * 0.5;
                else
                  cflux.v[q] = ((fv[0][0].v[q] + fv[0][1].v[q]) + (fv[1][0].v[q] + fv[1][1].v[q])) * 0.25;
              }
            }
        }
    }
  }

  // One full step.  dt_cap > 0 clamps dt (c_h and kappa keep the CFL value).
  void step(double dt_cap = 0.0) {
    double dt, ch, kappa;
    cfl(S0, &dt, &ch, &kappa);
    if (dt_cap > 0.0 && dt > dt_cap) dt = dt_cap;
    last_dt = dt;
    last_ch = ch;
    last_kappa = kappa;
    if (flags & FLAG_BAD_DT) return;
    const int s = P.nstages;
    if (s == 1) {
      stage(S0, nullptr, S1, 1.0, dt, ch, kappa);
      std::swap(S0, S1);
    } else if (s == 2) {
      stage(S0, nullptr, S1, 1.0, dt, ch, kappa);
      stage(S1, &S0, S0, 0.5, dt, ch, kappa);
    } else if (s == 3) {
      stage(S0, nullptr, S1, 1.0, dt, ch, kappa);
      stage(S1, &S0, S2, 0.25, dt, ch, kappa);
      stage(S2, &S0, S0, 2.0 / 3.0, dt, ch, kappa);
    } else if (s == 4) {
      // SSPRK(4,3) (Table tab:schemes_time): four forward-Euler stages of
      // dt/2; the third returns to u0 with weight 1/3:
      //   u1 = u0 + h L(u0), u2 = u1 + h L(u1),
      //   u3 = 2/3 u0 + 1/3 (u2 + h L(u2)), u4 = u3 + h L(u3),  h = dt/2
      const double h = 0.5 * dt;
      stage(S0, nullptr, S1, 1.0, h, ch, kappa);
      stage(S1, nullptr, S2, 1.0, h, ch, kappa);
      stage(S2, &S0, S1, 1.0 / 3.0, h, ch, kappa);
      stage(S1, nullptr, S0, 1.0, h, ch, kappa);
    } else {
      // SSPRK(5,4) (five-step row of Table tab:schemes_time; Spiteri and
      // Ruuth 2002), Shu-Osher form with their published coefficients:
      //   u1 = u0 + b10 dt L(u0)
      //   u2 = a20 u0 + a21 u1 + b21 dt L(u1)
      //   u3 = a30 u0 + a32 u2 + b32 dt L(u2)
      //   u4 = a40 u0 + a43 u3 + b43 dt L(u3)
      //   u5 = a52 u2 + a53 u3 + b53 dt L(u3) + a54 u4 + b54 dt L(u4)
      // (a_k0 = 1 - the other state weights of the row: the delta form).
      const double b10 = 0.391752226571890;
      const double a21 = 0.555629506348765, b21 = 0.368410593050371;
      const double a32 = 0.379898148511597, b32 = 0.251891774271694;
      const double a43 = 0.821920045606868, b43 = 0.544974750228521;
      const double a52 = 0.517231671970585, a53 = 0.096059710526147, b53 = 0.063692468666290;
      const double a54 = 0.386708617503269, b54 = 0.226007483236906;
      if (S3.size() != (size_t)nb) {
        S3.assign(nb, BlockData(pcells));
        S4.assign(nb, BlockData(pcells));
      }
      rhs(S0, Lb, ch, kappa);
      shu_osher(S1, S0, {}, {{b10, &Lb}}, dt);
      rhs(S1, Lb, ch, kappa);
      shu_osher(S2, S0, {{a21, &S1}}, {{b21, &Lb}}, dt);
      rhs(S2, Lb, ch, kappa);
      shu_osher(S3, S0, {{a32, &S2}}, {{b32, &Lb}}, dt);
      rhs(S3, L3, ch, kappa);
      shu_osher(S4, S0, {{a43, &S3}}, {{b43, &L3}}, dt);
      rhs(S4, Lb, ch, kappa);
      shu_osher(S1, S0, {{a52, &S2}, {a53, &S3}, {a54, &S4}}, {{b53, &L3}, {b54, &Lb}}, dt);
      std::swap(S0, S1);
    }
  }
};

Sim* build_sim(const oracle_params* p, int nblocks, const int* level, const int* ijk, const double* prim) {
  Sim* s = new Sim();
  s->P = *p;
  s->ph = Phys{p->gamma, p->small_density, p->small_pressure, p->fix_small_values};
  s->ndim = p->ndim;
  s->nx = p->nx;
  s->ng = p->ng;
  if (s->ndim != 2 && s->ndim != 3) throw std::invalid_argument("ndim must be 2 or 3");
  if (s->ng != 2 && s->ng != 3) throw std::invalid_argument("ghost layers must be 2 or 3");
  if (s->nx < 4 || (s->nx & 1)) throw std::invalid_argument("nx must be even and >= 4");
  if (2 * s->ng > s->nx) throw std::invalid_argument("nx must be at least twice the ghost depth (restriction)");
  if (p->nstages < 1 || p->nstages > 5) throw std::invalid_argument("nstages must be 1 .. 5");
  if (p->limiter < LIM_VANLEER || p->limiter > LIM_WENOZP5) throw std::invalid_argument("unknown limiter");
  if (five_cell_limiter(p->limiter) && p->ng != 3)
    throw std::invalid_argument("the fifth-order reconstructions need 3 ghost layers");
  if (p->flux != FLUX_HLL && p->flux != FLUX_HLLD && p->flux != FLUX_HLLC) throw std::invalid_argument("unknown flux scheme");
  if (s->P.nthreads < 1) s->P.nthreads = 1;
  for (int d = 0; d < s->ndim; ++d)
    if ((p->bc_lo[d] == BC_PERIODIC) != (p->bc_hi[d] == BC_PERIODIC))
      throw std::invalid_argument("periodic boundaries must be periodic on both sides");
  s->pn = s->nx + 2 * s->ng;
  s->pcells = (long)s->pn * s->pn * (s->ndim == 3 ? s->pn : 1);
  s->icells = (long)s->nx * s->nx * (s->ndim == 3 ? s->nx : 1);
  s->nb = nblocks;
  s->finest = 1;
  for (int b = 0; b < nblocks; ++b) {
    const int l = level[b];
    if (l < 1) throw std::invalid_argument("levels are 1-based");
    Idx q{ijk[3 * b], ijk[3 * b + 1], s->ndim == 3 ? ijk[3 * b + 2] : 0};
    for (int d = 0; d < s->ndim; ++d)
      if (q[d] < 0 || q[d] >= ((long)p->base_blocks[d] << (l - 1))) throw std::invalid_argument("block outside the domain");
    s->lev.push_back(l);
    s->pos.push_back(q);
    if (!s->leaf.emplace(Key{l, q[0], q[1], q[2]}, b).second) throw std::invalid_argument("duplicate block");
    s->finest = std::max(s->finest, l);
    Idx a = q;
    for (int m = l - 1; m >= 1; --m) {
      for (int d = 0; d < 3; ++d) a[d] >>= 1;
      s->refined.insert(Key{m, a[0], a[1], a[2]});
    }
  }
  for (const auto& kv : s->leaf)
    if (s->refined.count(kv.first)) throw std::invalid_argument("a leaf overlaps a refined block");
  for (int d = 0; d < 3; ++d)
    for (int side = 0; side < 2; ++side) {
      Cell w;
      for (int q = 0; q < NV; ++q) w.v[q] = p->bc_fixed_prim[d][side][q];
      s->fixedU[d][side] = prim_to_cons(w, p->gamma);
    }
  s->S0.assign(nblocks, BlockData(s->pcells));
  s->S1.assign(nblocks, BlockData(s->pcells));
  s->S2.assign(nblocks, BlockData(s->pcells));
  s->flux.resize(nblocks);
  const long nfaces = (long)(s->nx + 1) * s->nx * (s->ndim == 3 ? s->nx : 1);
  for (int b = 0; b < nblocks; ++b)
    for (int d = 0; d < s->ndim; ++d) s->flux[b][d].assign(nfaces, Cell{});
  const long ic = s->icells;
  for (int b = 0; b < nblocks; ++b) {
    for (long c = 0; c < ic; ++c) {
      const long i = c % s->nx, j = (c / s->nx) % s->nx, k = s->ndim == 3 ? c / ((long)s->nx * s->nx) : 0;
      Cell w;
      for (int q = 0; q < NV; ++q) w.v[q] = prim[((long)b * NV + q) * ic + c];
      s->S0[b][s->pidx(i, j, k)] = prim_to_cons(w, p->gamma);
    }
  }
  return s;
}

thread_local std::string g_err;

}  // namespace

extern "C" {

const char* oracle_last_error() { return g_err.c_str(); }

void* oracle_create(const oracle_params* p, int nblocks, const int* level, const int* ijk, const double* prim) {
  try {
    return build_sim(p, nblocks, level, ijk, prim);
  } catch (const std::exception& e) {
    g_err = e.what();
    return nullptr;
  }
}

void oracle_destroy(void* h) { delete static_cast<Sim*>(h); }

// Regrid: a new simulation on another leaf set whose every block is a block
// of the old one, a child of an old leaf (refinement) or the parent of 2^d
// old leaves (coarsening).  Its state: copies of unchanged blocks; for a
// child, the conservative linear prolongation of its parent (parent value
// plus a quarter of the minmod-limited slope per direction, the slope
// neighbours taken from the parent's ghost-filled block); for a parent, the
// volume average of its children (the restriction of the ghost fill).  The
// old simulation's state slot 0 has its ghosts filled as a side effect.
void* oracle_regrid(void* h, int nblocks, const int* level, const int* ijk) {
  try {
    Sim* o = static_cast<Sim*>(h);
    o->fill_ghosts(o->S0);
    const int nd = o->ndim;
    const long nxo = o->nx;
    std::vector<double> zero((size_t)nblocks * NV * (size_t)o->icells, 0.0);
    Sim* s = build_sim(&o->P, nblocks, level, ijk, zero.data());
    const long kmax = nd == 3 ? nxo : 1;
    for (int b = 0; b < nblocks; ++b) {
      const int l = level[b];
      const Idx bi{ijk[3 * b], ijk[3 * b + 1], nd > 2 ? ijk[3 * b + 2] : 0};
      const Key same{l, bi[0], bi[1], bi[2]};
      const Key par{l - 1, bi[0] >> 1, bi[1] >> 1, bi[2] >> 1};
      auto it = o->leaf.find(same);
      auto ip = l > 1 ? o->leaf.find(par) : o->leaf.end();
      const bool coarsened = o->refined.count(same) > 0;
      if (it == o->leaf.end() && ip == o->leaf.end() && !coarsened)
        throw std::invalid_argument("regrid block is not an old block, child or parent of old leaves");
      for (long k = 0; k < kmax; ++k)
        for (long j = 0; j < nxo; ++j)
          for (long i = 0; i < nxo; ++i) {
            const long c = s->pidx(i, j, k);
            const Idx g{bi[0] * nxo + i, bi[1] * nxo + j, nd > 2 ? bi[2] * nxo + k : 0};
            Cell v;
            if (it != o->leaf.end()) {
              v = o->S0[it->second][o->pidx(i, j, k)];
            } else if (ip != o->leaf.end()) {
              const BlockData& P = o->S0[ip->second];
              const Idx lc{(g[0] >> 1) - par.i * nxo, (g[1] >> 1) - par.j * nxo, nd > 2 ? (g[2] >> 1) - par.k * nxo : 0};
              const Cell uc = P[o->pidx(lc)];
              v = uc;
              for (int d = 0; d < nd; ++d) {
                Idx lo = lc, hi = lc;
                lo[d] -= 1;
                hi[d] += 1;
                const Cell& um = P[o->pidx(lo)];
                const Cell& up = P[o->pidx(hi)];
                const double sg = (g[d] & 1) ? 0.25 : -0.25;
                for (int q = 0; q < NV; ++q) v.v[q] = v.v[q] + sg * minmod(uc.v[q] - um.v[q], up.v[q] - uc.v[q]);
              }
            } else {
              v = o->restrict_cell(o->S0, l, g);
            }
            s->S0[b][c] = v;
          }
    }
    return s;
  } catch (const std::exception& e) {
    g_err = e.what();
    return nullptr;
  }
}

// Advance nsteps full SSPRK steps; diag receives (dt, c_h, kappa, flags) per
// step.  Returns 0, or -1 on an exception (message in oracle_last_error), or
// -4 if a step met a non-physical state or an invalid dt (the run stops there).
int oracle_steps(void* h, int nsteps, double* diag) {
  Sim* s = static_cast<Sim*>(h);
  try {
    for (int n = 0; n < nsteps; ++n) {
      s->step();
      if (diag) {
        diag[4 * n + 0] = s->last_dt;
        diag[4 * n + 1] = s->last_ch;
        diag[4 * n + 2] = s->last_kappa;
        diag[4 * n + 3] = (double)s->flags;
      }
      if (s->flags & FLAG_BAD_DT) return -4;
      if ((s->flags & (FLAG_SMALL_RHO | FLAG_SMALL_P)) && !s->P.fix_small_values) return -4;
    }
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
  return 0;
}

// Advance until time t_end (the last dt clamped so the run ends on it),
// at most max_steps steps.  Returns the number of steps taken, or a negative
// status as oracle_steps.
int oracle_steps_to_time(void* h, double t_end, int max_steps) {
  Sim* s = static_cast<Sim*>(h);
  double t = 0.0;
  int n = 0;
  try {
    while (t < t_end && n < max_steps) {
      s->step(t_end - t);
      if (s->flags & FLAG_BAD_DT) return -4;
      if ((s->flags & (FLAG_SMALL_RHO | FLAG_SMALL_P)) && !s->P.fix_small_values) return -4;
      t += s->last_dt;
      ++n;
    }
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
  return n;
}

// One stage with caller-given dt, c_h, kappa, from slot 0 into slot 0
// (forward Euler, w = 1).
int oracle_euler_stage(void* h, double dt, double ch, double kappa) {
  Sim* s = static_cast<Sim*>(h);
  try {
    s->stage(s->S0, nullptr, s->S1, 1.0, dt, ch, kappa);
    std::swap(s->S0, s->S1);
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
  return 0;
}

int oracle_cfl(void* h, double* dt, double* ch, double* kappa) {
  Sim* s = static_cast<Sim*>(h);
  s->cfl(s->S0, dt, ch, kappa);
  return s->flags;
}

int oracle_flags(void* h) { return static_cast<Sim*>(h)->flags; }
long oracle_fix_count(void* h) { return static_cast<Sim*>(h)->nfix; }

// Interior conserved state of slot 0, [block][var][k][j][i].
void oracle_get_cons(void* h, double* out) {
  Sim* s = static_cast<Sim*>(h);
  const long ic = s->icells;
  for (int b = 0; b < s->nb; ++b)
    for (long c = 0; c < ic; ++c) {
      const long i = c % s->nx, j = (c / s->nx) % s->nx, k = s->ndim == 3 ? c / ((long)s->nx * s->nx) : 0;
      const Cell& u = s->S0[b][s->pidx(i, j, k)];
      for (int q = 0; q < NV; ++q) out[((long)b * NV + q) * ic + c] = u.v[q];
    }
}

// Replace the interior conserved state of slot 0.
void oracle_set_cons(void* h, const double* in) {
  Sim* s = static_cast<Sim*>(h);
  const long ic = s->icells;
  for (int b = 0; b < s->nb; ++b)
    for (long c = 0; c < ic; ++c) {
      const long i = c % s->nx, j = (c / s->nx) % s->nx, k = s->ndim == 3 ? c / ((long)s->nx * s->nx) : 0;
      Cell& u = s->S0[b][s->pidx(i, j, k)];
      for (int q = 0; q < NV; ++q) u.v[q] = in[((long)b * NV + q) * ic + c];
    }
}

// Fill the face ghosts of slot 0 and return the padded state,
// [block][var][pk][pj][pi] with (nx+2ng)^ndim cells; edge and corner cells
// are returned as NaN.
int oracle_fill_padded(void* h, double* out) {
  Sim* s = static_cast<Sim*>(h);
  try {
    s->fill_ghosts(s->S0);
  } catch (const std::exception& e) {
    g_err = e.what();
    return -1;
  }
  const int ng = s->ng, nx = s->nx, pn = s->pn;
  for (int b = 0; b < s->nb; ++b)
    for (long c = 0; c < s->pcells; ++c) {
      const long i = c % pn - ng, j = (c / pn) % pn - ng, k = s->ndim == 3 ? c / ((long)pn * pn) - ng : 0;
      const int o = (i < 0 || i >= nx) + (j < 0 || j >= nx) + (s->ndim == 3 && (k < 0 || k >= nx));
      for (int q = 0; q < NV; ++q)
        out[((long)b * NV + q) * s->pcells + c] = o > 1 ? NAN : s->S0[b][c].v[q];
    }
  return 0;
}

// Point functions, exposed for the unit pins.
void oracle_prim_to_cons(const double* w, double gamma, double* u) {
  Cell c;
  std::memcpy(c.v, w, sizeof(c.v));
  Cell r = prim_to_cons(c, gamma);
  std::memcpy(u, r.v, sizeof(r.v));
}
int oracle_cons_to_prim(const double* u, double gamma, double small_rho, double small_p, int fix, double* w) {
  Cell c, r;
  std::memcpy(c.v, u, sizeof(c.v));
  const int bad = cons_to_prim(c, Phys{gamma, small_rho, small_p, fix}, r);
  std::memcpy(w, r.v, sizeof(r.v));
  return bad;
}
double oracle_fast_speed(const double* w, int d, double gamma) {
  Cell c;
  std::memcpy(c.v, w, sizeof(c.v));
  return fast_speed(c, d, gamma);
}
double oracle_vanleer(double dm, double dp) { return vanleer(dm, dp); }
double oracle_minmod(double a, double b) { return minmod(a, b); }
double oracle_weno5_face(double vm2, double vm1, double v0, double vp1, double vp2, int kind, double lambda) {
  return weno5_face(vm2, vm1, v0, vp1, vp2, kind, lambda);
}

double oracle_mp5_face(double vm2, double vm1, double v0, double vp1, double vp2) {
  return mp5_face(vm2, vm1, v0, vp1, vp2);
}
int oracle_face_increments(int lim, double dm, double dp, double* inc_right, double* inc_left) {
  if (lim < LIM_VANLEER || lim > LIM_CADA3) return -1;
  face_increments(lim, dm, dp, inc_right, inc_left);
  return 0;
}
void oracle_glm_interface(double bnl, double bnr, double psl, double psr, double ch, double* out) {
  glm_interface(bnl, bnr, psl, psr, ch, &out[0], &out[1]);
}
void oracle_face_flux(const double* wl, const double* wr, int d, double ch, double gamma, double* F) {
  Cell a, b;
  std::memcpy(a.v, wl, sizeof(a.v));
  std::memcpy(b.v, wr, sizeof(b.v));
  face_flux(a, b, d, ch, gamma, F);
}
int oracle_face_flux_kind(const double* wl, const double* wr, int d, double ch, double gamma, int flux, double* F) {
  if (flux != FLUX_HLL && flux != FLUX_HLLD && flux != FLUX_HLLC) return -1;
  Cell a, b;
  std::memcpy(a.v, wl, sizeof(a.v));
  std::memcpy(b.v, wr, sizeof(b.v));
  face_flux(a, b, d, ch, gamma, F, flux);
  return 0;
}
void oracle_phys_flux(const double* w, int d, double gamma, double* F) {
  Cell c;
  std::memcpy(c.v, w, sizeof(c.v));
  const Cell u = prim_to_cons(c, gamma);
  phys_flux(c, u, d, F);
}

}  // extern "C"
