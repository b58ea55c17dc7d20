// Device-side numerics of the ideal-MHD step (gfx950).
//
// Everything here is a __device__ inline function templated on the face
// scalar R (double, or float in the mixed-precision path) so that the
// reconstruction / Riemann / EMF chain is instantiated twice from one source.
// Primitive recovery and all accumulation stay in double.
//
// Paper: arXiv 2511.20337 (gPLUTO). Sec. 2.1 Eqs. (mhd), (Energy): state,
// flux and EOS; Sec. 2.2: primitive inversion, reconstruction (Eq.
// reconstruct), Riemann flux, constrained transport; Secs. 4.1/4.2 cite the
// HLLD solver of Miyoshi & Kusano (2005), written out below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Every floating-point operation is evaluated as written: no automatic fusion
// of a multiply and an add into an FMA (explicit __builtin_fma calls stay).
// The adjoint re-evaluates reconstruction and the Riemann solver in other
// kernels and in dual numbers; with contraction left to the compiler, the same
// source could round differently there than in the forward kernels, and at
// near-ties (a limiter at a local extremum, min/max of equal wave speeds,
// the sign of the contact speed) take the other branch. This pragma applies
// to every function defined after it in the translation unit.
#pragma clang fp contract(off)

namespace mhd {

enum : int { F_RHO = 0, F_MX = 1, F_MY = 2, F_MZ = 3, F_EN = 4, F_BX = 5, F_BY = 6, F_BZ = 7 };

// Workgroup order of the WENO-Z kernels, of the mixed-mode EMF and update
// kernels and of the adjoint's gather kernels: the hardware deals workgroups
// round-robin to the 8 XCDs, each with its own L2. Within every full group of
// 512 workgroups, XCD x is given the 64 consecutive ones x*64 .. x*64+63, so
// that neighbouring rows (the stencil's reach along y) are mostly read through
// the same L2, while all XCDs still advance together through the domain and
// share the Infinity Cache. A permutation of 0 .. nb-1; a last partial group
// keeps its order. (Measured slower for the z-marching face kernel, whose
// neighbouring columns share the Infinity Cache better round-robin.)
__device__ __forceinline__ unsigned xcd_grouped(unsigned b, unsigned nb) {
  const unsigned grp = b / 512u;
  if ((grp + 1u) * 512u > nb) return b;
  const unsigned w = b % 512u;
  return grp * 512u + (w % 8u) * 64u + w / 8u;
}

// Per-face record slots (one array of N values per slot, per direction):
// fluxes of the cell-averaged fields, then the quantities the edge EMF needs.
// With the UCT-HLLD average, S_AP holds its weight om, S_AM its diffusion
// coefficient d^L and S_DR d^R, and S_V1/S_V2 the om-weighted velocities.
enum : int {
  S_RHO = 0, S_MX = 1, S_MY = 2, S_MZ = 3, S_EN = 4, S_BZ = 5,  // S_BZ: 2D only
  S_AP = 6, S_AM = 7, S_V1 = 8, S_V2 = 9, S_DR = 10, NSLOT = 11
};

struct Geom {
  int nx, ny, nz;
  int64_t n;            // cells
  double dx, dy, dz;    // spacings
  double gamma;
};

// FP64 reciprocal, quotient and square root from the hardware estimates
// (v_rcp_f64 / v_rsq_f64, about 5e-8 relative), refined by Newton steps and
// a residual correction: on 2^20 random operands the quotient and the square
// root reproduce the IEEE result bit for bit, at well under the instruction
// count of the IEEE sequences. Operands: finite, nonzero divisors and
// non-negative radicands in the normal range.
__device__ __forceinline__ double rcp_r(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
}
// Quotient a/b; r receives the refined reciprocal of b it was formed with.
__device__ __forceinline__ double div_r_rcp(double a, double b, double& r) {
  r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
  const double q = a * r;
  return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
__device__ __forceinline__ double div_r(double a, double b) {
  double r;
  return div_r_rcp(a, b, r);
}
// Square root of x >= 0; h receives about 1/(2 sqrt(x)) (one Newton step).
__device__ __forceinline__ double sqrt_r_half(double x, double& h) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y;
  h = 0.5 * y;
  const double t = __builtin_fma(-s, h, 0.5);
  s = __builtin_fma(s, t, s);
  h = __builtin_fma(h, t, h);
  const double r = __builtin_fma(__builtin_fma(-s, s, x), h, s);
  return x > 0.0 ? r : 0.0;  // the estimate is infinite at 0
}
__device__ __forceinline__ double sqrt_r(double x) {
  double h;
  return sqrt_r_half(x, h);
}
// a * b + c with one rounding. With contraction off, these are the only fused
// multiply-adds; the adjoint's dual numbers overload fma_r with the same value.
__device__ __forceinline__ double fma_r(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fma_r(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
// FP32 (mixed precision): the one-ulp hardware reciprocal and square root.
__device__ __forceinline__ float rcp_r(float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  return __builtin_fmaf(r, __builtin_fmaf(-b, r, 1.0f), r);
}
__device__ __forceinline__ float div_r(float a, float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  const float q = a * r;
  return __builtin_fmaf(__builtin_fmaf(-b, q, a), r, q);
}
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double abs_r(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float abs_r(float x) { return __builtin_fabsf(x); }
template <class R> __device__ __forceinline__ R max_r(R a, R b) { return (b > a) ? b : a; }
template <class R> __device__ __forceinline__ R min_r(R a, R b) { return (b < a) ? b : a; }

// Limited slope of piecewise-linear reconstruction: minmod (LIM 0) or the
// harmonic van Leer limiter (LIM 1); zero at extrema.
template <int LIM, class R>
__device__ __forceinline__ R plm_slope(R dm, R dp) {
  const R pr = dm * dp;
  if (LIM == 0) return (pr <= R(0)) ? R(0) : ((abs_r(dm) <= abs_r(dp)) ? dm : dp);
  const R q = div_r(R(2) * dm * dp, dm + dp);  // unused (maybe not finite) at extrema
  return (pr <= R(0)) ? R(0) : q;
}

// Fifth-order WENO-Z reconstruction (Borges et al. 2008, one of the operators
// R+- cited with Eq. (reconstruct)), FP64: the value at the upper interface of
// the middle cell of v0..v4 (cells i-2..i+2), a convex combination of the three
// third-order candidate values with Z weights d_k (1 + tau5 / (beta_k + eps)),
// Jiang-Shu smoothness indicators beta_k, tau5 = |beta0 - beta2|, ideal
// weights (1, 6, 3)/10, eps = 1e-40. The lower interface value is the same
// function of the cells in reverse order. The weights are formed over a common
// denominator, which moves the result by a few ulps from the textbook order of
// operations, and so do the fused multiply-adds.
__device__ __forceinline__ double wenoz_upper(double v0, double v1, double v2, double v3,
                                              double v4) {
  // six times the three candidate values (fused multiply-adds throughout:
  // this reconstruction has no adjoint whose roundings must match)
  const double q0 = __builtin_fma(2.0, v0, __builtin_fma(-7.0, v1, 11.0 * v2));
  const double q1 = __builtin_fma(5.0, v2, __builtin_fma(2.0, v3, -v1));
  const double q2 = __builtin_fma(2.0, v2, __builtin_fma(5.0, v3, -v4));
  const double c1 = 13.0 / 12.0, c2 = 1.0 / 4.0;
  const double a0 = __builtin_fma(-2.0, v1, v0 + v2);
  const double b0 = __builtin_fma(-4.0, v1, __builtin_fma(3.0, v2, v0));
  const double a1 = __builtin_fma(-2.0, v2, v1 + v3), b1 = v1 - v3;
  const double a2 = __builtin_fma(-2.0, v3, v2 + v4);
  const double b2 = __builtin_fma(3.0, v2, __builtin_fma(-4.0, v3, v4));
  const double eps = 1e-40;
  const double beta0 = __builtin_fma(c1 * a0, a0, __builtin_fma(c2 * b0, b0, eps));
  const double beta1 = __builtin_fma(c1 * a1, a1, __builtin_fma(c2 * b1, b1, eps));
  const double beta2 = __builtin_fma(c1 * a2, a2, __builtin_fma(c2 * b2, b2, eps));
  const double tau5 = __builtin_fabs(beta0 - beta2);
  // d_k (1 + tau5 / beta_k) times beta0 beta1 beta2 (> 0, which the
  // normalisation cancels), so that one division remains instead of seven;
  // beta_k >= eps keeps the products normal, and they stay finite while the
  // differences of the five values are below about 1e50
  const double al0 = 0.1 * (beta0 + tau5) * (beta1 * beta2);
  const double al1 = 0.6 * (beta1 + tau5) * (beta0 * beta2);
  const double al2 = 0.3 * (beta2 + tau5) * (beta0 * beta1);
  return div_r(__builtin_fma(al0, q0, __builtin_fma(al1, q1, al2 * q2)), 6.0 * (al0 + al1 + al2));
}

// Face-frame primitive state: (rho, u_n, v_t1, v_t2, B_t1, B_t2, p).
template <class R> struct FState { R w[7]; };

template <class R> struct RiemannOut {
  R f[7];        // flux of (rho, m_n, m_t1, m_t2, B_t1, B_t2, E)
  R ap, am;      // max(0, S_R), max(0, -S_L)
  R v1, v2;      // HLL-weighted transverse velocities (EM 1: om-weighted)
  R om, dl, dr;  // EM 1: UCT-HLLD weight of the left state, diffusion coefficients
};

// Fast magnetosonic speed along the normal.
template <class R>
__device__ __forceinline__ R cfast(R g, R rho, R p, R bn, R b1, R b2) {
  const R gp = g * p;
  const R bn2 = bn * bn;
  const R bb = fma_r(b2, b2, fma_r(b1, b1, bn2));
  const R a = gp + bb;
  const R disc = max_r(R(0), fma_r(a, a, -(R(4) * gp) * bn2));
  return sqrt_r(div_r(a + sqrt_r(disc), R(2) * rho));
}

// Conserved vector, normal flux and total pressure of a face-frame state.
template <class R>
__device__ __forceinline__ void phys(R igm1, const R* w, R bn, R* u, R* f, R& pt) {
  const R rho = w[0], vn = w[1], v1 = w[2], v2 = w[3], b1 = w[4], b2 = w[5], p = w[6];
  const R bb = fma_r(b2, b2, fma_r(b1, b1, bn * bn));
  pt = fma_r(R(0.5), bb, p);
  const R v2s = fma_r(v2, v2, fma_r(v1, v1, vn * vn));
  const R en = fma_r(R(0.5), bb, fma_r(R(0.5) * rho, v2s, p * igm1));
  const R mn = rho * vn;
  u[0] = rho; u[1] = mn; u[2] = rho * v1; u[3] = rho * v2; u[4] = b1; u[5] = b2; u[6] = en;
  const R vb = fma_r(v2, b2, fma_r(v1, b1, vn * bn));
  f[0] = mn;
  f[1] = fma_r(mn, vn, fma_r(-bn, bn, pt));
  f[2] = fma_r(mn, v1, -bn * b1);
  f[3] = fma_r(mn, v2, -bn * b2);
  f[4] = fma_r(vn, b1, -v1 * bn);
  f[5] = fma_r(vn, b2, -v2 * bn);
  f[6] = fma_r(en + pt, vn, -bn * vb);
}

// Relative tolerance below which the HLLD star state is treated as
// degenerate: 1e-12 in FP64; the same number of units of the working
// precision in FP32 (1e-12 * 2^29), where D = rho (S-u)(S-S_M) - bn^2 is
// the small difference of two large terms at low plasma beta.
template <class R> struct DegenerateTol { static constexpr double value = 1e-12; };
template <> struct DegenerateTol<float> { static constexpr double value = 1e-12 * 536870912.0; };

// Intermediate values of one Riemann solve, recorded for the hand-written
// reverse sweep of the adjoint (RiemannTape) or not at all (NoTape, which the
// forward kernels use; the compiler drops every store).
struct NoTape {
  static constexpr bool on = false;
};
struct RiemannTape {
  static constexpr bool on = true;
  // region: 0 F_L, 1 F_R (outside the fan), 2 HLL fan, 3 F*_L, 4 F**_L,
  // 5 F**_R, 6 F*_R
  int region;
  double ul[7], fl[7], ur[7], fr[7], ptl, ptr, cl, cr, sl, sr, ap, am, isum, v1, v2;
  double idn;                                     // HLL fan
  double dl, dr, ml, mr, iden, sm, pts;           // HLLD contact
  double ism[2], rs[2], big[2], den[2], iden2[2], fv[2], fb[2];
  double vs[2], ws[2], b1s[2], b2s[2], vb[2], vbs[2], es[2];
  bool deg[2];
  double sql, sqr, abn, sls, srs, sgn, isq, ssq, vss, wss, b1ss, b2ss, vbss, ess;
};

// HLL (RS 1) or HLLD (RS 0) flux between face-frame states wl | wr with
// continuous normal field bn. Wave-speed bounds: S_L = min(u_L,u_R) - c,
// S_R = max(u_L,u_R) + c, c = max(c_f,L, c_f,R). HLLD: the four-state solver
// of Miyoshi & Kusano (contact S_M, Alfven fronts S*_L, S*_R); when
// rho (S-u)(S-S_M) - bn^2 vanishes (relative DegenerateTol) the tangential
// fields of that side's star state are left unchanged. Region ties go left.
//
// EM 1 also gives the coefficients of the UCT-HLLD edge average. At the wave
// structure of the face the flux of each transverse field component is
// linear in the outer transverse fields and velocities,
//   F[B_t] = chiL B_t^L + chiR B_t^R - bn (om v_t^L + (1 - om) v_t^R);
// the EMF takes om, 1 - om as the weights of v_n B_t on either side,
// d^L = chiL - om u_L and d^R = (1 - om) u_R - chiR as its diffusion
// coefficients, and v1, v2 become the om-weighted velocities. Per region
// (B*_t = zeta B_t and v*_t = v_t - eta B_t on each side; w = 1/(sql + sqr)):
//   F_L, F*_L:  om = 1, chiL = u_L + S_L (zeta_L - 1), chiR = 0;
//   F**_L:      om = 1 + S*_L w sql sqr / |bn|,
//               chiL = u_L + S_L (zeta_L - 1) + S*_L (w (sqr zeta_L + s sql sqr eta_L) - zeta_L),
//               chiR = S*_L w (sql zeta_R - s sql sqr eta_R), s = sign(bn);
//   F**_R, F*_R, F_R: the mirror images. For HLL: om = alpha+/(alpha+ + alpha-),
//   d^L = d^R = alpha+ alpha-/(alpha+ + alpha-).
template <int RS, class R, class T, int EM = 0>
__device__ __forceinline__ void riemann_core(R g, const R* wl, const R* wr, R bn,
                                             RiemannOut<R>& o, T& tp) {
  R ul[7], fl[7], ur[7], fr[7], ptl, ptr;
  const R igm1 = rcp_r(g - R(1));  // 1/(gamma-1)
  phys(igm1, wl, bn, ul, fl, ptl);
  phys(igm1, wr, bn, ur, fr, ptr);
  const R cl = cfast(g, wl[0], wl[6], bn, wl[4], wl[5]);
  const R cr = cfast(g, wr[0], wr[6], bn, wr[4], wr[5]);
  const R cm = max_r(cl, cr);
  const R sl = min_r(wl[1], wr[1]) - cm;
  const R sr = max_r(wl[1], wr[1]) + cm;
  o.ap = max_r(R(0), sr);
  o.am = max_r(R(0), -sl);
  const R isum = rcp_r(o.ap + o.am);
  o.v1 = fma_r(o.ap, wl[2], o.am * wr[2]) * isum;
  o.v2 = fma_r(o.ap, wl[3], o.am * wr[3]) * isum;
  if constexpr (T::on) {
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      tp.ul[q] = ul[q]; tp.fl[q] = fl[q]; tp.ur[q] = ur[q]; tp.fr[q] = fr[q];
    }
    tp.ptl = ptl; tp.ptr = ptr; tp.cl = cl; tp.cr = cr; tp.sl = sl; tp.sr = sr;
    tp.ap = o.ap; tp.am = o.am; tp.isum = isum; tp.v1 = o.v1; tp.v2 = o.v2;
  }
  if (EM == 1 && RS == 1) {
    o.om = o.ap * isum;
    o.dl = o.ap * o.am * isum;
    o.dr = o.dl;
  }
  if (RS == 1) {
    if (sl >= R(0)) {
      if constexpr (T::on) tp.region = 0;
#pragma unroll
      for (int q = 0; q < 7; ++q) o.f[q] = fl[q];
    } else if (sr <= R(0)) {
      if constexpr (T::on) tp.region = 1;
#pragma unroll
      for (int q = 0; q < 7; ++q) o.f[q] = fr[q];
    } else {
      const R idn = rcp_r(sr - sl);
      if constexpr (T::on) { tp.region = 2; tp.idn = idn; }
#pragma unroll
      for (int q = 0; q < 7; ++q)
        o.f[q] = fma_r(sl * sr, ur[q] - ul[q], fma_r(sr, fl[q], -sl * fr[q])) * idn;
    }
    return;
  }
  if (sl > R(0)) {
    if constexpr (T::on) tp.region = 0;
#pragma unroll
    for (int q = 0; q < 7; ++q) o.f[q] = fl[q];
    if (EM == 1) { o.om = R(1); o.dl = R(0); o.dr = R(0); o.v1 = wl[2]; o.v2 = wl[3]; }
    return;
  }
  if (sr < R(0)) {
    if constexpr (T::on) tp.region = 1;
#pragma unroll
    for (int q = 0; q < 7; ++q) o.f[q] = fr[q];
    if (EM == 1) { o.om = R(0); o.dl = R(0); o.dr = R(0); o.v1 = wr[2]; o.v2 = wr[3]; }
    return;
  }
  const R dl = sl - wl[1], dr = sr - wr[1];
  const R ml = dl * wl[0], mr = dr * wr[0];          // mass fluxes through the outer fronts
  const R iden = rcp_r(mr - ml);
  const R sm = fma_r(mr, wr[1], fma_r(-ml, wl[1], ptl - ptr)) * iden;
  const R pts = fma_r(ml * mr, wr[1] - wl[1], fma_r(mr, ptl, -ml * ptr)) * iden;
  const R bn2 = bn * bn;
  if constexpr (T::on) {
    tp.dl = dl; tp.dr = dr; tp.ml = ml; tp.mr = mr; tp.iden = iden; tp.sm = sm; tp.pts = pts;
  }

  // star states, one side at a time: s = 0 left, 1 right
  R rs[2], vs[2], ws[2], b1s[2], b2s[2], es[2];
  R zeta[2], eta[2];  // EM 1: B*_t = zeta B_t, v*_t = v_t - eta B_t
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const R* w = s ? wr : wl;
    const R d = s ? dr : dl;
    const R m = s ? mr : ml;
    const R S = s ? sr : sl;
    const R pt = s ? ptr : ptl;
    const R en = s ? ur[6] : ul[6];
    const R ism = rcp_r(S - sm);
    rs[s] = m * ism;
    const R big = m * (S - sm);
    const R den = big - bn2;
    const bool deg = abs_r(den) <= R(DegenerateTol<R>::value) * (abs_r(big) + bn2);
    if (deg) {
      vs[s] = w[2]; ws[s] = w[3]; b1s[s] = w[4]; b2s[s] = w[5];
      zeta[s] = R(1);
      eta[s] = R(0);
    } else {
      const R iden2 = rcp_r(den);
      const R fv = bn * (sm - w[1]) * iden2;
      vs[s] = fma_r(-w[4], fv, w[2]);
      ws[s] = fma_r(-w[5], fv, w[3]);
      const R fb = fma_r(m, d, -bn2) * iden2;
      b1s[s] = w[4] * fb;
      b2s[s] = w[5] * fb;
      zeta[s] = fb;
      eta[s] = fv;
      if constexpr (T::on) { tp.iden2[s] = iden2; tp.fv[s] = fv; tp.fb[s] = fb; }
    }
    const R vb = fma_r(w[3], w[5], fma_r(w[2], w[4], w[1] * bn));
    const R vbs = fma_r(ws[s], b2s[s], fma_r(vs[s], b1s[s], sm * bn));
    es[s] = fma_r(bn, vb - vbs, fma_r(pts, sm, fma_r(d, en, -pt * w[1]))) * ism;
    if constexpr (T::on) {
      tp.ism[s] = ism; tp.rs[s] = rs[s]; tp.big[s] = big; tp.den[s] = den; tp.deg[s] = deg;
      tp.vs[s] = vs[s]; tp.ws[s] = ws[s]; tp.b1s[s] = b1s[s]; tp.b2s[s] = b2s[s];
      tp.vb[s] = vb; tp.vbs[s] = vbs; tp.es[s] = es[s];
    }
  }
  const R sql = sqrt_r(rs[0]), sqr = sqrt_r(rs[1]);
  const R abn = abs_r(bn);
  const R sls = sm - div_r(abn, sql);
  const R srs = sm + div_r(abn, sqr);
  if constexpr (T::on) { tp.sql = sql; tp.sqr = sqr; tp.abn = abn; tp.sls = sls; tp.srs = srs; }

  if (sls >= R(0)) {  // F*_L
    if constexpr (T::on) tp.region = 3;
    if (EM == 1) {
      o.om = R(1);
      o.dl = sl * (zeta[0] - R(1));
      o.dr = R(0);
      o.v1 = wl[2];
      o.v2 = wl[3];
    }
    const R us[7] = {rs[0], rs[0] * sm, rs[0] * vs[0], rs[0] * ws[0], b1s[0], b2s[0], es[0]};
#pragma unroll
    for (int q = 0; q < 7; ++q) o.f[q] = fma_r(sl, us[q] - ul[q], fl[q]);
    return;
  }
  const R sgn = (bn > R(0)) ? R(1) : ((bn < R(0)) ? R(-1) : R(0));
  const R isq = rcp_r(sql + sqr);
  const R ssq = sgn * sql * sqr;
  const R vss = fma_r(sgn, b1s[1] - b1s[0], fma_r(sql, vs[0], sqr * vs[1])) * isq;
  const R wss = fma_r(sgn, b2s[1] - b2s[0], fma_r(sql, ws[0], sqr * ws[1])) * isq;
  const R b1ss = fma_r(ssq, vs[1] - vs[0], fma_r(sql, b1s[1], sqr * b1s[0])) * isq;
  const R b2ss = fma_r(ssq, ws[1] - ws[0], fma_r(sql, b2s[1], sqr * b2s[0])) * isq;
  const R vbss = fma_r(vss, b1ss, wss * b2ss);
  if constexpr (T::on) {
    tp.sgn = sgn; tp.isq = isq; tp.ssq = ssq; tp.vss = vss; tp.wss = wss; tp.b1ss = b1ss;
    tp.b2ss = b2ss; tp.vbss = vbss;
  }
  if (EM == 1) {
    // F**_L or F**_R (|bn| > 0 there: S*_L < 0 <= S_M or S_M < 0 <= S*_R)
    const R ww = isq * sql * sqr;
    const R cl = fma_r(sgn * sql * sqr, eta[0], sqr * zeta[0]) * isq;  // B** per B_t^L
    const R cr = fma_r(-sgn * sql * sqr, eta[1], sql * zeta[1]) * isq;  // B** per B_t^R
    R chiL, chiR;
    if (sm >= R(0)) {
      o.om = R(1) - div_r(-sls * ww, abn);
      chiL = fma_r(sls, cl - zeta[0], fma_r(sl, zeta[0] - R(1), wl[1]));
      chiR = sls * cr;
    } else {
      o.om = div_r(srs * ww, abn);
      chiR = fma_r(srs, cr - zeta[1], fma_r(sr, zeta[1] - R(1), wr[1]));
      chiL = srs * cl;
    }
    const R omr = R(1) - o.om;
    o.dl = fma_r(-o.om, wl[1], chiL);
    o.dr = fma_r(omr, wr[1], -chiR);
    o.v1 = fma_r(o.om, wl[2], omr * wr[2]);
    o.v2 = fma_r(o.om, wl[3], omr * wr[3]);
  }
  if (sm >= R(0)) {  // F**_L
    const R ess = fma_r(-sgn * sql, fma_r(vs[0], b1s[0], ws[0] * b2s[0]) - vbss, es[0]);
    if constexpr (T::on) { tp.region = 4; tp.ess = ess; }
    const R us[7] = {rs[0], rs[0] * sm, rs[0] * vs[0], rs[0] * ws[0], b1s[0], b2s[0], es[0]};
    const R uss[7] = {rs[0], rs[0] * sm, rs[0] * vss, rs[0] * wss, b1ss, b2ss, ess};
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const R fs = fma_r(sl, us[q] - ul[q], fl[q]);
      o.f[q] = fma_r(sls, uss[q] - us[q], fs);
    }
    return;
  }
  const R us[7] = {rs[1], rs[1] * sm, rs[1] * vs[1], rs[1] * ws[1], b1s[1], b2s[1], es[1]};
  if (srs >= R(0)) {  // F**_R
    const R ess = fma_r(sgn * sqr, fma_r(vs[1], b1s[1], ws[1] * b2s[1]) - vbss, es[1]);
    if constexpr (T::on) { tp.region = 5; tp.ess = ess; }
    const R uss[7] = {rs[1], rs[1] * sm, rs[1] * vss, rs[1] * wss, b1ss, b2ss, ess};
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const R fs = fma_r(sr, us[q] - ur[q], fr[q]);
      o.f[q] = fma_r(srs, uss[q] - us[q], fs);
    }
    return;
  }
  if constexpr (T::on) tp.region = 6;
  if (EM == 1) {
    o.om = R(0);
    o.dl = R(0);
    o.dr = -sr * (zeta[1] - R(1));
    o.v1 = wr[2];
    o.v2 = wr[3];
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) o.f[q] = fma_r(sr, us[q] - ur[q], fr[q]);  // F*_R
}

template <int RS, class R, int EM = 0>
__device__ __forceinline__ void riemann(R g, const R* wl, const R* wr, R bn, RiemannOut<R>& o) {
  NoTape tp;
  riemann_core<RS, R, NoTape, EM>(g, wl, wr, bn, o, tp);
}

// Upwind edge EMF for component c with cyclic pair (a, b); the exact value
// is v_b B_a - v_a B_b. a-bracket: v_a B_b upwinded along a from the two
// b-faces (W, E) reconstructed toward the edge, with the largest alpha+-
// of the two a-faces touching the edge; b-bracket likewise along b.
template <class R>
__device__ __forceinline__ R uct(R apa, R ama, R vW, R bW, R vE, R bE,
                                 R apb, R amb, R vS, R bS, R vN, R bN) {
  const R ta = div_r(apa * vW * bW + ama * vE * bE - apa * ama * (bE - bW), apa + ama);
  const R tb = div_r(apb * vS * bS + amb * vN * bN - apb * amb * (bN - bS), apb + amb);
  return tb - ta;
}

// UCT-HLLD edge EMF for component c with cyclic pair (a, b): the weights
// (aa, 1 - aa) and diffusion coefficients dla, dra (averaged over the two
// a-faces touching the edge) act on v_a B_b from the two b-faces
// reconstructed along a (W, E); the b-bracket likewise.
template <class R>
__device__ __forceinline__ R uct_hlld(R aa, R dla, R dra, R vW, R bW, R vE, R bE, R ab, R dlb,
                                      R drb, R vS, R bS, R vN, R bN) {
  const R ta = aa * vW * bW + (R(1) - aa) * vE * bE - (dra * bE - dla * bW);
  const R tb = ab * vS * bS + (R(1) - ab) * vN * bN - (drb * bN - dlb * bS);
  return tb - ta;
}

// Values of a face quantity reconstructed toward an edge from the two faces
// beside it: lo = x(-1) + slope(-1)/2 (upper extrapolation of the lower face),
// hi = x(0) - slope(0)/2, from the four faces x(-2), x(-1), x(0), x(+1).
template <int LIM, class R>
__device__ __forceinline__ void edge_pair(R xm2, R xm1, R x0, R xp1, R& lo, R& hi) {
  lo = fma_r(R(0.5), plm_slope<LIM, R>(xm1 - xm2, x0 - xm1), xm1);
  hi = fma_r(R(-0.5), plm_slope<LIM, R>(x0 - xm1, xp1 - x0), x0);
}

}  // namespace mhd
