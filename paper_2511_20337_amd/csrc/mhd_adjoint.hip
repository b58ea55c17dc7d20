// Adjoint (vector-Jacobian product) of one SSP-RK2 or SSP-RK3 step, FP64,
// gather form.
//
// The RK2 step is Phi(Un) = (Un + S(S(Un)))/2 with S(U) = U + dt L(U). Reverse:
//   G2 = Ubar1/2;        U1bar = G2 + dt J_L(U1)^T G2;
//   Ubar0 = Ubar1/2 + U1bar + dt J_L(Un)^T U1bar;
//   dtbar = <G2, L(U1)> + <U1bar, L(Un)>.
// The RK3 step takes the same per-stage adjoint three times (adjoint_rk3).
// J_L^T G is assembled from the local Jacobians of each piece of L, every
// output written by exactly one thread (no atomics, deterministic):
//   k_adj_edges — the EMF cotangent from -curl E, times the partial
//                 derivatives of the upwind EMF average w.r.t. its twelve
//                 inputs (per edge, stored);
//   k_adj_faces — per face: flux cotangents from the divergence, cotangents
//                 of alpha+-, the weighted velocities and b gathered from the
//                 edges that used them (through the adjoint of their
//                 reconstruction), then the Riemann solver's vector-Jacobian
//                 product: one hand-written reverse sweep over the values the
//                 solver itself recorded;
//   k_adj_cells — per cell: adjoint of PLM (gathering the face-state
//                 cotangents of the faces each cell feeds) and of primitive
//                 recovery;
//   k_adj_final — staggered-field cotangents, the RK combination and the
//                 dtbar reduction.
// At every non-smooth point the derivative of the branch taken by the
// forward step is used (limiter at extrema, min/max, Riemann region).
#include "mhd_adjoint.hpp"
#include "mhd_grid.hpp"
#include "mhd_kernels.hpp"

namespace mhd {

namespace {

// ---------------------------------------------------------------------------
// Hand-written reverse sweep of the Riemann solver. The forward values come
// from riemann_core itself (recorded on a tape), so every branch (wave-speed
// min/max, HLL/HLLD region, degenerate star state, sign of the normal field)
// is the one the forward kernels take; the derivative of each recorded
// branch is then propagated backwards once for all fifteen inputs. At a
// square root of zero the derivative is taken as zero.

// phys(): cotangents of u[7], f[7] and pt -> added to wb[7] and bnb.
__device__ __forceinline__ void phys_vjp(double igm1, const double* w, double bn,
                                         const double* ub, const double* fb, double ptb,
                                         double* wb, double& bnb) {
  const double rho = w[0], vn = w[1], v1 = w[2], v2 = w[3], b1 = w[4], b2 = w[5], p = w[6];
  const double bb = bn * bn + b1 * b1 + b2 * b2;
  const double pt = p + 0.5 * bb;
  const double v2s = vn * vn + v1 * v1 + v2 * v2;
  const double en = p * igm1 + 0.5 * rho * v2s + 0.5 * bb;
  const double mn = rho * vn;
  const double vb = vn * bn + v1 * b1 + v2 * b2;
  double mnb = fb[0] + fb[1] * vn + fb[2] * v1 + fb[3] * v2 + ub[1];
  double vnb = fb[1] * mn + fb[4] * b1 + fb[5] * b2 + fb[6] * (en + pt);
  double v1b = fb[2] * mn - fb[4] * bn + ub[2] * rho;
  double v2b = fb[3] * mn - fb[5] * bn + ub[3] * rho;
  double b1b = -fb[2] * bn + fb[4] * vn + ub[4];
  double b2b = -fb[3] * bn + fb[5] * vn + ub[5];
  double bnl = -2.0 * bn * fb[1] - fb[2] * b1 - fb[3] * b2 - fb[4] * v1 - fb[5] * v2 - fb[6] * vb;
  const double ptt = ptb + fb[1] + fb[6] * vn;
  const double enb = ub[6] + fb[6] * vn;
  const double vbb = -fb[6] * bn;
  vnb += vbb * bn;
  bnl += vbb * vn;
  v1b += vbb * b1;
  b1b += vbb * v1;
  v2b += vbb * b2;
  b2b += vbb * v2;
  const double rhob = ub[0] + ub[2] * v1 + ub[3] * v2 + mnb * vn + enb * 0.5 * v2s;
  vnb += mnb * rho;
  const double v2sb = enb * 0.5 * rho;
  const double bbb = 0.5 * (enb + ptt);
  const double pb = enb * igm1 + ptt;
  vnb += 2.0 * vn * v2sb;
  v1b += 2.0 * v1 * v2sb;
  v2b += 2.0 * v2 * v2sb;
  bnl += 2.0 * bn * bbb;
  b1b += 2.0 * b1 * bbb;
  b2b += 2.0 * b2 * bbb;
  wb[0] += rhob; wb[1] += vnb; wb[2] += v1b; wb[3] += v2b; wb[4] += b1b; wb[5] += b2b;
  wb[6] += pb;
  bnb += bnl;
}

// cfast(): cotangent of c_f -> added to rho, p (wb[0], wb[6]), b_t (wb[4], wb[5]), bn.
// The branch values are recomputed with cfast's own expressions.
__device__ __forceinline__ void cfast_vjp(double g, const double* w, double bn, double cfb,
                                          double* wb, double& bnb) {
  const double rho = w[0], p = w[6], b1 = w[4], b2 = w[5];
  const double gp = g * p;
  const double bn2 = bn * bn;
  const double bb = fma_r(b2, b2, fma_r(b1, b1, bn2));
  const double a = gp + bb;
  const double x = fma_r(a, a, -(4.0 * gp) * bn2);
  const double disc = max_r(0.0, x);
  const double sd = sqrt_r(disc);
  const double q = div_r(a + sd, 2.0 * rho);
  const double cf = sqrt_r(q);
  // reciprocals from the refined estimate (a few ulps from the quotients);
  // the selects drop the non-finite values at cf = 0, sd = 0
  const double qb = cf > 0.0 ? cfb * 0.5 * rcp_r(cf) : 0.0;
  const double irho = rcp_r(rho);
  const double i2r = 0.5 * irho;
  double ab = qb * i2r;
  const double sdb = qb * i2r;
  const double rhob = -qb * q * irho;
  const double discb = sd > 0.0 ? sdb * 0.5 * rcp_r(sd) : 0.0;
  const double xb = (x > 0.0) ? discb : 0.0;
  ab += 2.0 * a * xb;
  const double gpb = -4.0 * bn2 * xb + ab;
  const double bn2b = -4.0 * gp * xb + ab;
  wb[0] += rhob;
  wb[6] += g * gpb;
  wb[4] += 2.0 * b1 * ab;
  wb[5] += 2.0 * b2 * ab;
  bnb += 2.0 * bn * bn2b;
}

// Cotangents of the star state U*_s = (rho*, rho* S_M, rho* v*, rho* w*,
// B*_t1, B*_t2, E*) of side s -> the per-side adjoint accumulators.
struct StarBar {
  double rs[2], vs[2], ws[2], b1s[2], b2s[2], es[2];
  double sm;
};

__device__ __forceinline__ void star_us_vjp(const RiemannTape& t, int s, const double* usb,
                                            StarBar& sb) {
  sb.rs[s] += usb[0] + usb[1] * t.sm + usb[2] * t.vs[s] + usb[3] * t.ws[s];
  sb.sm += usb[1] * t.rs[s];
  sb.vs[s] += usb[2] * t.rs[s];
  sb.ws[s] += usb[3] * t.rs[s];
  sb.b1s[s] += usb[4];
  sb.b2s[s] += usb[5];
  sb.es[s] += usb[6];
}

template <int RS>
__device__ __forceinline__ void riemann_vjp(double g, const double* wl, const double* wr, double bn,
                                            const double* fbar, double apbar, double ambar,
                                            double v1bar, double v2bar, double* wlb, double* wrb,
                                            double& bnb) {
  RiemannTape t;
  RiemannOut<double> o;
  riemann_core<RS, double, RiemannTape>(g, wl, wr, bn, o, t);
  const double igm1 = rcp_r(g - 1.0);
#pragma unroll
  for (int q = 0; q < 7; ++q) { wlb[q] = 0.0; wrb[q] = 0.0; }
  bnb = 0.0;
  double ulb[7], flb[7], urb[7], frb[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) { ulb[q] = 0.0; flb[q] = 0.0; urb[q] = 0.0; frb[q] = 0.0; }
  double ptlb = 0.0, ptrb = 0.0, slb = 0.0, srb = 0.0;
  // HLL-weighted velocities v = (ap wl + am wr) / (ap + am)
  const double n1b = v1bar * t.isum, n2b = v2bar * t.isum;
  const double sumb = -(v1bar * t.v1 + v2bar * t.v2) * t.isum;
  const double apb = apbar + n1b * wl[2] + n2b * wl[3] + sumb;
  const double amb = ambar + n1b * wr[2] + n2b * wr[3] + sumb;
  wlb[2] += n1b * t.ap;
  wrb[2] += n1b * t.am;
  wlb[3] += n2b * t.ap;
  wrb[3] += n2b * t.am;
  const int reg = t.region;
  if (reg == 0) {
#pragma unroll
    for (int q = 0; q < 7; ++q) flb[q] += fbar[q];
  } else if (reg == 1) {
#pragma unroll
    for (int q = 0; q < 7; ++q) frb[q] += fbar[q];
  } else if (RS == 1) {
    // HLL fan: f = (sl sr (ur - ul) + sr fl - sl fr) / (sr - sl)
    double db = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const double nb = fbar[q] * t.idn;
      db -= fbar[q] * o.f[q] * t.idn;
      const double du = t.ur[q] - t.ul[q];
      slb += nb * (t.sr * du - t.fr[q]);
      srb += nb * (t.sl * du + t.fl[q]);
      urb[q] += nb * t.sl * t.sr;
      ulb[q] -= nb * t.sl * t.sr;
      flb[q] += nb * t.sr;
      frb[q] -= nb * t.sl;
    }
    srb += db;
    slb -= db;
  } else {
    // HLLD fan
    StarBar sb;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      sb.rs[q] = 0.0; sb.vs[q] = 0.0; sb.ws[q] = 0.0; sb.b1s[q] = 0.0; sb.b2s[q] = 0.0;
      sb.es[q] = 0.0;
    }
    sb.sm = 0.0;
    double ptsb = 0.0, slsb = 0.0, srsb = 0.0, sqlb = 0.0, sqrb = 0.0;
    const int side = (reg == 3 || reg == 4) ? 0 : 1;
    const double S = side ? t.sr : t.sl;
    const double* uo = side ? t.ur : t.ul;
    double* uob = side ? urb : ulb;
    double* fob = side ? frb : flb;
    const double us[7] = {t.rs[side], t.rs[side] * t.sm, t.rs[side] * t.vs[side],
                          t.rs[side] * t.ws[side], t.b1s[side], t.b2s[side], t.es[side]};
    double usb[7];
    double Sb = 0.0;
    if (reg == 3 || reg == 6) {
      // F*_a = F_a + S_a (U*_a - U_a)
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        fob[q] += fbar[q];
        Sb += fbar[q] * (us[q] - uo[q]);
        usb[q] = fbar[q] * S;
        uob[q] -= fbar[q] * S;
      }
    } else {
      // F**_a = F*_a + S*_a (U**_a - U*_a)
      const double sa = side ? t.srs : t.sls;
      const double uss[7] = {t.rs[side], t.rs[side] * t.sm, t.rs[side] * t.vss,
                             t.rs[side] * t.wss, t.b1ss, t.b2ss, t.ess};
      double ussb[7], sab = 0.0;
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        sab += fbar[q] * (uss[q] - us[q]);
        ussb[q] = fbar[q] * sa;
        usb[q] = -fbar[q] * sa + fbar[q] * S;
        Sb += fbar[q] * (us[q] - uo[q]);
        uob[q] -= fbar[q] * S;
        fob[q] += fbar[q];
      }
      if (side) srsb += sab; else slsb += sab;
      // U** of this side
      sb.rs[side] += ussb[0] + ussb[1] * t.sm + ussb[2] * t.vss + ussb[3] * t.wss;
      sb.sm += ussb[1] * t.rs[side];
      double vssb = ussb[2] * t.rs[side], wssb = ussb[3] * t.rs[side];
      double b1ssb = ussb[4], b2ssb = ussb[5];
      const double essb = ussb[6];
      // E**_a = E*_a -+ sgn sq_a ((v*_a B*_1a + w*_a B*_2a) - vbss)
      sb.es[side] += essb;
      const double tt = t.vs[side] * t.b1s[side] + t.ws[side] * t.b2s[side] - t.vbss;
      const double sqa = side ? t.sqr : t.sql;
      const double cc = side ? t.sgn * sqa : -t.sgn * sqa;
      const double ttb = essb * cc;
      const double sqab = essb * tt * (side ? t.sgn : -t.sgn);
      if (side) sqrb += sqab; else sqlb += sqab;
      sb.vs[side] += ttb * t.b1s[side];
      sb.b1s[side] += ttb * t.vs[side];
      sb.ws[side] += ttb * t.b2s[side];
      sb.b2s[side] += ttb * t.ws[side];
      const double vbssb = -ttb;
      // vbss = vss b1ss + wss b2ss
      vssb += vbssb * t.b1ss;
      b1ssb += vbssb * t.vss;
      wssb += vbssb * t.b2ss;
      b2ssb += vbssb * t.wss;
      // double-star v, w, B_t: (... ) * isq
      const double nv = t.sql * t.vs[0] + t.sqr * t.vs[1] + t.sgn * (t.b1s[1] - t.b1s[0]);
      const double nw = t.sql * t.ws[0] + t.sqr * t.ws[1] + t.sgn * (t.b2s[1] - t.b2s[0]);
      const double nb1 = t.sql * t.b1s[1] + t.sqr * t.b1s[0] + t.ssq * (t.vs[1] - t.vs[0]);
      const double nb2 = t.sql * t.b2s[1] + t.sqr * t.b2s[0] + t.ssq * (t.ws[1] - t.ws[0]);
      const double isqb = vssb * nv + wssb * nw + b1ssb * nb1 + b2ssb * nb2;
      const double nvb = vssb * t.isq, nwb = wssb * t.isq;
      const double nb1b = b1ssb * t.isq, nb2b = b2ssb * t.isq;
      sqlb += nvb * t.vs[0] + nwb * t.ws[0] + nb1b * t.b1s[1] + nb2b * t.b2s[1];
      sqrb += nvb * t.vs[1] + nwb * t.ws[1] + nb1b * t.b1s[0] + nb2b * t.b2s[0];
      sb.vs[0] += nvb * t.sql - nb1b * t.ssq;
      sb.vs[1] += nvb * t.sqr + nb1b * t.ssq;
      sb.ws[0] += nwb * t.sql - nb2b * t.ssq;
      sb.ws[1] += nwb * t.sqr + nb2b * t.ssq;
      sb.b1s[1] += nvb * t.sgn + nb1b * t.sql;
      sb.b1s[0] += -nvb * t.sgn + nb1b * t.sqr;
      sb.b2s[1] += nwb * t.sgn + nb2b * t.sql;
      sb.b2s[0] += -nwb * t.sgn + nb2b * t.sqr;
      const double ssqb = nb1b * (t.vs[1] - t.vs[0]) + nb2b * (t.ws[1] - t.ws[0]);
      sqlb += ssqb * t.sgn * t.sqr;
      sqrb += ssqb * t.sgn * t.sql;
      const double sumq = -isqb * t.isq * t.isq;
      sqlb += sumq;
      sqrb += sumq;
    }
    star_us_vjp(t, side, usb, sb);
    if (side) srb += Sb; else slb += Sb;
    // Alfven fronts S*_L = S_M - |bn|/sql, S*_R = S_M + |bn|/sqr
    {
      sb.sm += slsb + srsb;
      const double isl = rcp_r(t.sql), isr = rcp_r(t.sqr);
      const double ql = t.abn * isl, qr = t.abn * isr;
      const double abnb = -slsb * isl + srsb * isr;
      sqlb += slsb * ql * isl;
      sqrb -= srsb * qr * isr;
      bnb += abnb * (bn < 0.0 ? -1.0 : 1.0);
      sb.rs[0] += t.sql > 0.0 ? sqlb * 0.5 * isl : 0.0;
      sb.rs[1] += t.sqr > 0.0 ? sqrb * 0.5 * isr : 0.0;
    }
    // star states of both sides
    double bn2b = 0.0, mlb = 0.0, mrb = 0.0, dlb = 0.0, drb = 0.0;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const double* w = sd ? wr : wl;
      double* wb = sd ? wrb : wlb;
      const double d = sd ? t.dr : t.dl;
      const double m = sd ? t.mr : t.ml;
      const double Sv = sd ? t.sr : t.sl;
      const double pt = sd ? t.ptr : t.ptl;
      const double en = sd ? t.ur[6] : t.ul[6];
      const double ne = d * en - pt * w[1] + t.pts * t.sm + bn * (t.vb[sd] - t.vbs[sd]);
      const double neb = sb.es[sd] * t.ism[sd];
      double ismb = sb.es[sd] * ne;
      double db_ = neb * en;
      const double enb = neb * d;
      const double ptb = -neb * w[1];
      wb[1] -= neb * pt;
      ptsb += neb * t.sm;
      sb.sm += neb * t.pts;
      bnb += neb * (t.vb[sd] - t.vbs[sd]);
      const double vbb = neb * bn, vbsb = -neb * bn;
      sb.sm += vbsb * bn;
      bnb += vbsb * t.sm;
      double vsb = sb.vs[sd] + vbsb * t.b1s[sd];
      double b1sb = sb.b1s[sd] + vbsb * t.vs[sd];
      double wsb = sb.ws[sd] + vbsb * t.b2s[sd];
      double b2sb = sb.b2s[sd] + vbsb * t.ws[sd];
      wb[1] += vbb * bn;
      bnb += vbb * w[1];
      wb[2] += vbb * w[4];
      wb[4] += vbb * w[2];
      wb[3] += vbb * w[5];
      wb[5] += vbb * w[3];
      double mb = 0.0, Sbv = 0.0, bigb = 0.0;
      if (t.deg[sd]) {
        wb[2] += vsb;
        wb[3] += wsb;
        wb[4] += b1sb;
        wb[5] += b2sb;
      } else {
        const double fbk = t.fb[sd], fv = t.fv[sd], iden2 = t.iden2[sd];
        wb[4] += b1sb * fbk;
        wb[5] += b2sb * fbk;
        const double fbb = b1sb * w[4] + b2sb * w[5];
        const double nfb = fbb * iden2;
        double iden2b = fbb * (m * d - bn * bn);
        mb += nfb * d;
        db_ += nfb * m;
        bn2b -= nfb;
        wb[2] += vsb;
        wb[4] -= vsb * fv;
        wb[3] += wsb;
        wb[5] -= wsb * fv;
        const double fvb = -vsb * w[4] - wsb * w[5];
        bnb += fvb * (t.sm - w[1]) * iden2;
        sb.sm += fvb * bn * iden2;
        wb[1] -= fvb * bn * iden2;
        iden2b += fvb * bn * (t.sm - w[1]);
        const double denb = -iden2b * iden2 * iden2;
        bigb = denb;
        bn2b -= denb;
      }
      mb += bigb * (Sv - t.sm);
      Sbv += bigb * m;
      sb.sm -= bigb * m;
      mb += sb.rs[sd] * t.ism[sd];
      ismb += sb.rs[sd] * m;
      const double tism = -ismb * t.ism[sd] * t.ism[sd];
      Sbv += tism;
      sb.sm -= tism;
      if (sd) {
        drb += db_; mrb += mb; srb += Sbv; ptrb += ptb; urb[6] += enb;
      } else {
        dlb += db_; mlb += mb; slb += Sbv; ptlb += ptb; ulb[6] += enb;
      }
    }
    bnb += 2.0 * bn * bn2b;
    // contact speed and star total pressure
    const double dw = wr[1] - wl[1];
    const double nsm = t.mr * wr[1] - t.ml * wl[1] + t.ptl - t.ptr;
    const double npt = t.ml * t.mr * dw + t.mr * t.ptl - t.ml * t.ptr;
    const double nsmb = sb.sm * t.iden, nptb = ptsb * t.iden;
    const double idenb = sb.sm * nsm + ptsb * npt;
    mrb += nsmb * wr[1] + nptb * (t.ml * dw + t.ptl);
    mlb += -nsmb * wl[1] + nptb * (t.mr * dw - t.ptr);
    wrb[1] += nsmb * t.mr + nptb * t.ml * t.mr;
    wlb[1] += -nsmb * t.ml - nptb * t.ml * t.mr;
    ptlb += nsmb + nptb * t.mr;
    ptrb += -nsmb - nptb * t.ml;
    const double dden = -idenb * t.iden * t.iden;
    mrb += dden;
    mlb -= dden;
    dlb += mlb * wl[0];
    wlb[0] += mlb * t.dl;
    drb += mrb * wr[0];
    wrb[0] += mrb * t.dr;
    slb += dlb;
    wlb[1] -= dlb;
    srb += drb;
    wrb[1] -= drb;
  }
  // alpha+- = max(0, S_R), max(0, -S_L)
  if (t.sr > 0.0) srb += apb;
  if (-t.sl > 0.0) slb -= amb;
  // S_L = min(u_L, u_R) - c, S_R = max(u_L, u_R) + c, c = max(c_L, c_R);
  // the selected argument takes the cotangent (the first one on ties)
  if (wr[1] < wl[1]) wrb[1] += slb; else wlb[1] += slb;
  if (wr[1] > wl[1]) wrb[1] += srb; else wlb[1] += srb;
  const double cmb = srb - slb;
  {
    // one evaluation on the side whose fast speed was taken, by selects
    const bool rs = t.cr > t.cl;
    double wc[7], wcb[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 7; ++q) wc[q] = rs ? wr[q] : wl[q];
    cfast_vjp(g, wc, bn, cmb, wcb, bnb);
    constexpr int touched[4] = {0, 4, 5, 6};  // rho, B_t1, B_t2, p
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int q = touched[e];
      wrb[q] += rs ? wcb[q] : 0.0;
      wlb[q] += rs ? 0.0 : wcb[q];
    }
  }
  phys_vjp(igm1, wl, bn, ulb, flb, ptlb, wlb, bnb);
  phys_vjp(igm1, wr, bn, urb, frb, ptrb, wrb, bnb);
}

// Edge-partial slots: d E / d input times Ebar.
enum : int { E_APA = 0, E_AMA, E_VW, E_BW, E_VE, E_BE, E_APB, E_AMB, E_VS, E_BS, E_VN, E_BN, NE };

struct Bufs {
  double* EB;    // 3 components x NE x n
  double* WB;    // 3 directions x 14 x n: wL-bar (7), wR-bar (7)
  double* BF;    // 3 x n: staggered-field cotangent gathered at each face
  double* BC;    // 3 x n: cell-centred field cotangent
  double* T;     // 8 x n: J^T G of the cell-averaged fields
  double* A;     // 8 x n: cotangent of the stage-1 state
  double* PW;    // 8 x n: FP64 primitives of the state the stage adjoint linearises at
  double* FWn;   // dim x NSLOT x n: face records at U_n (kept from the stage-1 forward)
  double* EWn;   // 3 x n: edge EMFs at U_n
  // SSP-RK3 only (nullptr otherwise):
  double* FW1;   // dim x NSLOT x n: face records at U1 (kept from the stage-2 forward)
  double* EW1;   // 3 x n: edge EMFs at U1
  double* A1;    // 8 x n: cotangent of the stage-1 state
  double* part;  // (2 or 3) x nblocks: dtbar partial sums, one set per stage
};

template <int D>
__device__ __forceinline__ double delta(const Geom& g) {
  return D == 0 ? g.dx : (D == 1 ? g.dy : g.dz);
}

// ---------------------------------------------------------------------------
template <int C, int LIM>
__device__ __forceinline__ void edge_partials(const double* __restrict__ U,
                                              const double* __restrict__ FW,
                                              const double* __restrict__ G, double s,
                                              const Geom& g, int i, int j, int k, int64_t c,
                                              double* __restrict__ EB) {
  constexpr int A = (C + 1) % 3, B = (C + 2) % 3;
  const int64_t n = g.n;
  const double* fa = FW + (int64_t)A * NSLOT * n;
  const double* fb = FW + (int64_t)B * NSLOT * n;
  const int64_t cmb = shifted<B>(g, i, j, k, -1);
  const int64_t cma = shifted<A>(g, i, j, k, -1);
  // Ebar = sum over the four faces whose -curl E uses this edge
  const double* GA = G + (F_BX + A) * n;
  const double* GB = G + (F_BX + B) * n;
  const double eb = s * ((GA[c] - GA[cmb]) / delta<B>(g) - (GB[c] - GB[cma]) / delta<A>(g));
  const double apa = max_r(fa[S_AP * n + cmb], fa[S_AP * n + c]);
  const double ama = max_r(fa[S_AM * n + cmb], fa[S_AM * n + c]);
  const double apb = max_r(fb[S_AP * n + cma], fb[S_AP * n + c]);
  const double amb = max_r(fb[S_AM * n + cma], fb[S_AM * n + c]);
  const int64_t a2 = shifted<A>(g, i, j, k, -2), a1 = shifted<A>(g, i, j, k, 1);
  const int64_t b2 = shifted<B>(g, i, j, k, -2), b1 = shifted<B>(g, i, j, k, 1);
  const double* vbA = fb + S_V2 * n;
  const double* bB = U + (F_BX + B) * n;
  const double* vaB = fa + S_V1 * n;
  const double* bA = U + (F_BX + A) * n;
  double vW, vE, bW, bE, vS, vN, bS, bN;
  edge_pair<LIM, double>(vbA[a2], vbA[cma], vbA[c], vbA[a1], vW, vE);
  edge_pair<LIM, double>(bB[a2], bB[cma], bB[c], bB[a1], bW, bE);
  edge_pair<LIM, double>(vaB[b2], vaB[cmb], vaB[c], vaB[b1], vS, vN);
  edge_pair<LIM, double>(bA[b2], bA[cmb], bA[c], bA[b1], bS, bN);
  // E = tb - ta
  const double isa = 1.0 / (apa + ama), isb = 1.0 / (apb + amb);
  const double ta = (apa * vW * bW + ama * vE * bE - apa * ama * (bE - bW)) * isa;
  const double tb = (apb * vS * bS + amb * vN * bN - apb * amb * (bN - bS)) * isb;
  double* e = EB + (int64_t)C * NE * n + c;
  e[E_VW * n] = -eb * apa * bW * isa;
  e[E_BW * n] = -eb * apa * (vW + ama) * isa;
  e[E_VE * n] = -eb * ama * bE * isa;
  e[E_BE * n] = -eb * ama * (vE - apa) * isa;
  e[E_APA * n] = -eb * (vW * bW - ama * (bE - bW) - ta) * isa;
  e[E_AMA * n] = -eb * (vE * bE - apa * (bE - bW) - ta) * isa;
  e[E_VS * n] = eb * apb * bS * isb;
  e[E_BS * n] = eb * apb * (vS + amb) * isb;
  e[E_VN * n] = eb * amb * bN * isb;
  e[E_BN * n] = eb * amb * (vN - apb) * isb;
  e[E_APB * n] = eb * (vS * bS - amb * (bN - bS) - tb) * isb;
  e[E_AMB * n] = eb * (vN * bN - apb * (bN - bS) - tb) * isb;
}

template <int DIM, int LIM>
__global__ __launch_bounds__(kBlock) void k_adj_edges(const double* __restrict__ U,
                                                      const double* __restrict__ FW,
                                                      const double* __restrict__ G, double s,
                                                      Geom g, double* __restrict__ EB) {
  // XCD-grouped workgroup order: the rows above and below, which the stencil
  // reads, mostly come through the same L2 (KH 512^2 adjoint 2878 -> 3041
  // steps/s, blast 256^3 30.5 -> 31.1, for edges, faces and cells together)
  const int64_t c = (int64_t)xcd_grouped(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  if (DIM == 3) {
    edge_partials<0, LIM>(U, FW, G, s, g, i, j, k, c, EB);
    edge_partials<1, LIM>(U, FW, G, s, g, i, j, k, c, EB);
  }
  edge_partials<2, LIM>(U, FW, G, s, g, i, j, k, c, EB);
}

// ---------------------------------------------------------------------------
// Cotangents a face receives from the edges of component C that use it.
// ROLE 0: the face is an a-face of C (normal A = D), its v_B (slot V1) and
// b_D are reconstructed along B; ROLE 1: a b-face (normal B = D), its v_A
// (slot V2) and b_D along A. Split into the loads (edge_load) and the
// arithmetic (edge_apply), so that a face's loads all go out before any of
// its arithmetic waits for one.
struct EdgeIn {
  double apm, ap0, app, amm, am0, amp;  // alpha+- of the faces c-e, c, c+e
  double ea0, eap, em0, emp;            // alpha cotangents of the edges at c, c+e
  double xv[5], xb[5];                  // v and b on the faces c-2e .. c+2e
  double vp[3], vm[3], bp[3], bm[3];    // cotangents of their edge values
};

template <int C, int ROLE>
__device__ __forceinline__ void edge_load(const double* __restrict__ U,
                                          const double* __restrict__ FW,
                                          const double* __restrict__ EB, const Geom& g, int i,
                                          int j, int k, int64_t c, EdgeIn& in) {
  constexpr int A = (C + 1) % 3, B = (C + 2) % 3;
  constexpr int D = ROLE == 0 ? A : B;      // this face's normal
  constexpr int E = ROLE == 0 ? B : A;      // reconstruction / neighbour direction
  constexpr int sap = ROLE == 0 ? E_APA : E_APB, sam = ROLE == 0 ? E_AMA : E_AMB;
  constexpr int svlo = ROLE == 0 ? E_VS : E_VW, svhi = ROLE == 0 ? E_VN : E_VE;
  constexpr int sblo = ROLE == 0 ? E_BS : E_BW, sbhi = ROLE == 0 ? E_BN : E_BE;
  const int64_t n = g.n;
  const double* f = FW + (int64_t)D * NSLOT * n;
  const double* e = EB + (int64_t)C * NE * n;
  const int64_t cm1 = shifted<E>(g, i, j, k, -1), cp1 = shifted<E>(g, i, j, k, 1);
  const int64_t cm2 = shifted<E>(g, i, j, k, -2), cp2 = shifted<E>(g, i, j, k, 2);
  const double* ap = f + S_AP * n;
  const double* am = f + S_AM * n;
  in.apm = ap[cm1]; in.ap0 = ap[c]; in.app = ap[cp1];
  in.amm = am[cm1]; in.am0 = am[c]; in.amp = am[cp1];
  in.ea0 = e[sap * n + c]; in.eap = e[sap * n + cp1];
  in.em0 = e[sam * n + c]; in.emp = e[sam * n + cp1];
  const double* v = f + (ROLE == 0 ? S_V1 : S_V2) * n;
  const double* b = U + (F_BX + D) * n;
  const int64_t c5[5] = {cm2, cm1, c, cp1, cp2};
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    in.xv[s] = v[c5[s]];
    in.xb[s] = b[c5[s]];
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    in.vp[s] = e[svlo * n + c5[s + 2]];
    in.vm[s] = e[svhi * n + c5[s + 1]];
    in.bp[s] = e[sblo * n + c5[s + 2]];
    in.bm[s] = e[sbhi * n + c5[s + 1]];
  }
}

template <int LIM>
__device__ __forceinline__ void edge_apply(EdgeIn& in, double& apbar, double& ambar,
                                           double& vbar, double& bbar) {
  // the empty asm keeps the compiler from sinking the four alpha cotangent
  // loads into the branches that add them (one round trip each)
  asm volatile("" : "+v"(in.ea0), "+v"(in.eap), "+v"(in.em0), "+v"(in.emp));
  // alpha: the edge at c takes max(face c-e, face c); the edge at c+e takes
  // max(face c, face c+e); the first argument wins ties.
  apbar = (in.ap0 > in.apm) ? apbar + in.ea0 : apbar;
  apbar = !(in.app > in.ap0) ? apbar + in.eap : apbar;
  ambar = (in.am0 > in.amm) ? ambar + in.em0 : ambar;
  ambar = !(in.amp > in.am0) ? ambar + in.emp : ambar;
  // reconstructed values: upper extrapolation of face p feeds the edge at
  // p+e (as its lower value), the lower extrapolation feeds the edge at p
  vbar += plm_adjoint<LIM>(in.xv, in.vp, in.vm);
  bbar += plm_adjoint<LIM>(in.xb, in.bp, in.bm);
}

// Reconstructed face-frame states of the lower D-face of cell (i,j,k) as
// face_inputs forms them, from the recovered primitives PW of the four cells
// c-2..c+1 along D (the values primitive recovery gives, computed once per
// cell by k_adj_prim): pw_load gathers the 28 values, pw_states reconstructs.
template <int D>
__device__ __forceinline__ void pw_load(const double* __restrict__ PW, const Geom& g, int i,
                                        int j, int k, double (&v)[7][4]) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  const int64_t n = g.n;
  int64_t cs[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) cs[s] = shifted<D>(g, i, j, k, s - 2);
#pragma unroll
  for (int q = 0; q < 7; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) v[q][s] = PW[(int64_t)slot[q] * n + cs[s]];
}
template <int LIM>
__device__ __forceinline__ void pw_states(const double (&v)[7][4], double* wl, double* wr) {
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const double a = v[q][0], b = v[q][1], c = v[q][2], e = v[q][3];
    wl[q] = fma_r(0.5, plm_slope<LIM, double>(b - a, c - b), b);
    wr[q] = fma_r(-0.5, plm_slope<LIM, double>(c - b, e - c), c);
  }
}

// FP64 primitives of every cell of the stage's state, once, for the face and
// cell kernels of the stage adjoint (which read each cell's from up to
// thirteen stencils).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_adj_prim(const double* __restrict__ U,
                                                     double* __restrict__ PW, Geom g) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  double V[8];
  prim_at<DIM>(U, g, i, j, k, V);
#pragma unroll
  for (int q = 0; q < 8; ++q) PW[q * g.n + c] = V[q];
}

template <int DIM, int D, int LIM, int RS>
__device__ __forceinline__ void face_adjoint(const double* __restrict__ U,
                                             const double* __restrict__ FW,
                                             const double* __restrict__ G, double s,
                                             const double* __restrict__ EB, const Geom& g, int i,
                                             int j, int k, int64_t c, const Bufs& bf) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int C1 = (D + 2) % 3;  // this face is an a-face of C1
  constexpr int C2 = (D + 1) % 3;  // and a b-face of C2
  constexpr bool E1 = (DIM == 3 || C1 == 2), E2 = (DIM == 3 || C2 == 2);
  const int64_t n = g.n;
  const int64_t cm = shifted<D>(g, i, j, k, -1);
  const double idl = s / delta<D>(g);
  // Gather: every value the face needs, issued before any of it is used.
  constexpr int NG = (DIM == 2) ? 6 : 5;
  constexpr int gq[6] = {0, F_MX + D, F_MX + T1, F_MX + T2, F_EN, F_BZ};
  double gc[NG], gm[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    gc[q] = G[gq[q] * n + c];
    gm[q] = G[gq[q] * n + cm];
  }
  EdgeIn e1, e2;
  if (E1) edge_load<C1, 0>(U, FW, EB, g, i, j, k, c, e1);
  if (E2) edge_load<C2, 1>(U, FW, EB, g, i, j, k, c, e2);
  double pv[7][4];
  pw_load<D>(bf.PW, g, i, j, k, pv);
  const double bn = U[(F_BX + D) * n + c];
  __builtin_amdgcn_sched_barrier(0);
  // flux cotangents (face frame: rho, m_n, m_t1, m_t2, B_t1, B_t2, E)
  double fb[7];
  fb[0] = (gc[0] - gm[0]) * idl;
  fb[1] = (gc[1] - gm[1]) * idl;
  fb[2] = (gc[2] - gm[2]) * idl;
  fb[3] = (gc[3] - gm[3]) * idl;
  fb[4] = 0.0;
  fb[5] = 0.0;
  fb[6] = (gc[4] - gm[4]) * idl;
  if (DIM == 2) {
    const double bz = (gc[NG - 1] - gm[NG - 1]) * idl;
    if (D == 0) fb[5] = bz; else fb[4] = bz;   // B_z is t2 of x-faces, t1 of y-faces
  }
  // cotangents from the edges
  double apbar = 0.0, ambar = 0.0, v1bar = 0.0, v2bar = 0.0, bbar = 0.0;
  if (E1) edge_apply<LIM>(e1, apbar, ambar, v1bar, bbar);
  if (E2) edge_apply<LIM>(e2, apbar, ambar, v2bar, bbar);
  // Riemann vector-Jacobian product: one reverse sweep
  double wl[7], wr[7];
  pw_states<LIM>(pv, wl, wr);
  double* wb = bf.WB + (int64_t)D * 14 * n + c;
  double wlb[7], wrb[7], bnbar;
  riemann_vjp<RS>(g.gamma, wl, wr, bn, fb, apbar, ambar, v1bar, v2bar, wlb, wrb, bnbar);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    wb[(int64_t)q * n] = wlb[q];
    wb[(int64_t)(7 + q) * n] = wrb[q];
  }
  bf.BF[(int64_t)D * n + c] = bnbar + bbar;
}

template <int DIM, int LIM, int RS>
__global__ __launch_bounds__(kBlock) void k_adj_faces(const double* __restrict__ U,
                                                      const double* __restrict__ FW,
                                                      const double* __restrict__ G, double s,
                                                      Geom g, Bufs bf) {
  const int64_t c = (int64_t)xcd_grouped(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  face_adjoint<DIM, 0, LIM, RS>(U, FW, G, s, bf.EB, g, i, j, k, c, bf);
  face_adjoint<DIM, 1, LIM, RS>(U, FW, G, s, bf.EB, g, i, j, k, c, bf);
  if (DIM == 3) face_adjoint<DIM, 2, LIM, RS>(U, FW, G, s, bf.EB, g, i, j, k, c, bf);
}

// ---------------------------------------------------------------------------
template <int DIM, int D, int LIM>
__device__ __forceinline__ void plm_cell_adjoint(const double* __restrict__ PW,
                                                 const double* __restrict__ WB, const Geom& g,
                                                 int i, int j, int k, double* vbar) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  const int64_t n = g.n;
  int64_t cs[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) cs[s] = shifted<D>(g, i, j, k, s - 2);
  double V[5][8];
#pragma unroll
  for (int s = 0; s < 5; ++s)
#pragma unroll
    for (int q = 0; q < 7; ++q) V[s][slot[q]] = PW[(int64_t)slot[q] * n + cs[s]];
  // faces p (lower face of cell p) for p = c-1 .. c+2 along D
  int64_t fidx[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) fidx[s] = shifted<D>(g, i, j, k, s - 1);
  const double* w = WB + (int64_t)D * 14 * n;
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int sl = slot[q];
    const double x[5] = {V[0][sl], V[1][sl], V[2][sl], V[3][sl], V[4][sl]};
    // upper extrapolation of cell p = left state of face p+1;
    // lower extrapolation of cell p = right state of face p
    const double xp[3] = {w[q * n + fidx[1]], w[q * n + fidx[2]], w[q * n + fidx[3]]};
    const double xm[3] = {w[(7 + q) * n + fidx[0]], w[(7 + q) * n + fidx[1]],
                          w[(7 + q) * n + fidx[2]]};
    vbar[sl] += plm_adjoint<LIM>(x, xp, xm);
  }
}

template <int DIM, int LIM>
__global__ __launch_bounds__(kBlock) void k_adj_cells(const double* __restrict__ U, Geom g,
                                                      Bufs bf) {
  const int64_t c = (int64_t)xcd_grouped(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  const int64_t n = g.n;
  double vb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  plm_cell_adjoint<DIM, 0, LIM>(bf.PW, bf.WB, g, i, j, k, vb);
  plm_cell_adjoint<DIM, 1, LIM>(bf.PW, bf.WB, g, i, j, k, vb);
  if (DIM == 3) plm_cell_adjoint<DIM, 2, LIM>(bf.PW, bf.WB, g, i, j, k, vb);
  // primitive recovery: v = m/rho, p = (gamma-1)(E - |m|^2/(2 rho) - |Bc|^2/2)
  double V[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) V[q] = bf.PW[q * n + c];
  const double gm1 = g.gamma - 1.0;
  const double pb = vb[4] * gm1;
  const double irho = 1.0 / V[0];
  const double v2 = V[1] * V[1] + V[2] * V[2] + V[3] * V[3];
  double trho = vb[0] + 0.5 * pb * v2;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    trho -= vb[1 + d] * V[1 + d] * irho;
    bf.T[(F_MX + d) * n + c] = vb[1 + d] * irho - pb * V[1 + d];
  }
  bf.T[c] = trho;
  bf.T[F_EN * n + c] = pb;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double bcb = vb[5 + d] - pb * V[5 + d];
    if (DIM == 2 && d == 2) bf.T[F_BZ * n + c] = bcb;  // cell-centred B_z
    else bf.BC[(int64_t)d * n + c] = bcb;
  }
}

// L(U) of cell (i,j,k) from the forward records, as the update kernel forms it.
template <int DIM>
__device__ __forceinline__ void stage_rhs(const double* __restrict__ FW,
                                          const double* __restrict__ EW, const Geom& g, int i,
                                          int j, int k, int64_t c, double* L) {
  const int64_t n = g.n;
  const int64_t xp = lin(g, wrap(i + 1, g.nx), j, k);
  const int64_t yp = lin(g, i, wrap(j + 1, g.ny), k);
  const int64_t zp = (DIM == 3) ? lin(g, i, j, wrap(k + 1, g.nz)) : c;
  const double idx = 1.0 / g.dx, idy = 1.0 / g.dy, idz = 1.0 / g.dz;
  const double* fx = FW;
  const double* fy = FW + (int64_t)NSLOT * n;
  const double* fz = FW + (int64_t)2 * NSLOT * n;
  constexpr int ncell = (DIM == 3) ? 5 : 6;
#pragma unroll
  for (int q = 0; q < ncell; ++q) {
    double acc = (fx[q * n + xp] - fx[q * n + c]) * idx + (fy[q * n + yp] - fy[q * n + c]) * idy;
    if (DIM == 3) acc += (fz[q * n + zp] - fz[q * n + c]) * idz;
    L[q == 5 ? 7 : q] = -acc;
  }
  if (DIM == 3) {
    const double* ex = EW;
    const double* ey = EW + n;
    const double* ez = EW + 2 * n;
    L[5] = -((ez[yp] - ez[c]) * idy - (ey[zp] - ey[c]) * idz);
    L[6] = -((ex[zp] - ex[c]) * idz - (ez[xp] - ez[c]) * idx);
    L[7] = -((ey[xp] - ey[c]) * idx - (ex[yp] - ex[c]) * idy);
  } else {
    const double* ez = EW + 2 * n;
    L[5] = -((ez[yp] - ez[c]) * idy);
    L[6] = (ez[xp] - ez[c]) * idx;
  }
}

// ---------------------------------------------------------------------------
// out = cd * Dir + s G + dt J^T (s G); DT: also the per-block partial of
// <s G, L(U)> (L(U) from the forward records), which only dt-bar needs.
template <int DIM, bool DT>
__global__ __launch_bounds__(kBlock) void k_adj_final(const double* __restrict__ G, double s,
                                                      const double* __restrict__ Dir, double cd,
                                                      const double* __restrict__ FW,
                                                      const double* __restrict__ EW, Geom g,
                                                      double dt, Bufs bf, double* out,
                                                      double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (c < g.n) {
    int i, j, k;
    coords(g, c, i, j, k);
    const int64_t n = g.n;
    double jt[8];
#pragma unroll
    for (int q = 0; q < 5; ++q) jt[q] = bf.T[q * n + c];
    const int64_t xm = lin(g, wrap(i - 1, g.nx), j, k);
    const int64_t ym = lin(g, i, wrap(j - 1, g.ny), k);
    jt[5] = 0.5 * (bf.BC[c] + bf.BC[xm]) + bf.BF[c];
    jt[6] = 0.5 * (bf.BC[n + c] + bf.BC[n + ym]) + bf.BF[n + c];
    if (DIM == 3) {
      const int64_t zm = lin(g, i, j, wrap(k - 1, g.nz));
      jt[7] = 0.5 * (bf.BC[2 * n + c] + bf.BC[2 * n + zm]) + bf.BF[2 * n + c];
    } else {
      jt[7] = bf.T[F_BZ * n + c];
    }
    double L[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (DT) stage_rhs<DIM>(FW, EW, g, i, j, k, c, L);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double sg = s * G[q * n + c];
      double v = sg + dt * jt[q];
      if (Dir) v += cd * Dir[q * n + c];
      out[q * n + c] = v;
      if constexpr (DT) dot += sg * L[q];
    }
  }
  if constexpr (!DT) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
  __shared__ double red[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = dot;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) r += red[w];
    part[blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(1024) void k_sum_final(const double* __restrict__ part, int np,
                                                    double* __restrict__ out) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < np; b += 1024) acc += part[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 16; ++w) r += red[w];
    *out = r;
  }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

Bufs carve(double* scratch, int dim, int64_t n, int integrator) {
  Bufs b;
  double* p = scratch;
  b.EB = p; p += 3 * NE * n;
  b.WB = p; p += 3 * 14 * n;
  b.BF = p; p += 3 * n;
  b.BC = p; p += 3 * n;
  b.T = p; p += 8 * n;
  b.A = p; p += 8 * n;
  b.PW = p; p += 8 * n;
  b.FWn = p; p += (int64_t)dim * NSLOT * n;
  b.EWn = p; p += 3 * n;
  b.FW1 = b.EW1 = b.A1 = nullptr;
  if (integrator == 1) {
    b.FW1 = p; p += (int64_t)dim * NSLOT * n;
    b.EW1 = p; p += 3 * n;
    b.A1 = p; p += 8 * n;
  }
  b.part = p;
  return b;
}

// J^T of one stage, combined: out = cd Dir + s G + dt J_L(U)^T (s G); the
// forward records FW/EW must hold the face/edge data at U.
template <int DIM, int LIM, int RS>
hipError_t stage_adjoint(const AdjointArgs& a, const Bufs& bf, const double* U, const double* FW,
                         const double* EW, const double* G, double s, const double* Dir,
                         double cd, double* out, double* part) {
  const unsigned nb = blocks_for(a.g.n);
  hipLaunchKernelGGL((k_adj_prim<DIM>), dim3(nb), dim3(kBlock), 0, a.stream, U, bf.PW, a.g);
  hipLaunchKernelGGL((k_adj_edges<DIM, LIM>), dim3(nb), dim3(kBlock), 0, a.stream, U, FW, G, s,
                     a.g, bf.EB);
  hipLaunchKernelGGL((k_adj_faces<DIM, LIM, RS>), dim3(nb), dim3(kBlock), 0, a.stream, U, FW, G,
                     s, a.g, bf);
  hipLaunchKernelGGL((k_adj_cells<DIM, LIM>), dim3(nb), dim3(kBlock), 0, a.stream, U, a.g, bf);
  if (a.want_dtbar)
    hipLaunchKernelGGL((k_adj_final<DIM, true>), dim3(nb), dim3(kBlock), 0, a.stream, G, s, Dir,
                       cd, FW, EW, a.g, a.dt, bf, out, part);
  else
    hipLaunchKernelGGL((k_adj_final<DIM, false>), dim3(nb), dim3(kBlock), 0, a.stream, G, s, Dir,
                       cd, FW, EW, a.g, a.dt, bf, out, part);
  return hipGetLastError();
}

// Elementwise out = a x + b y (n doubles).
__global__ __launch_bounds__(kBlock) void k_axpby(const double* __restrict__ x, double a,
                                                  const double* __restrict__ y, double b,
                                                  double* __restrict__ out, int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c < n) out[c] = a * x[c] + b * y[c];
}

// Adjoint of one SSP-RK3 step (Eq. (RK3)): U1 = Un + dt L(Un),
// U2 = 3/4 Un + 1/4 (U1 + dt L(U1)), U3 = 1/3 Un + 2/3 (U2 + dt L(U2)).
// With G = Ubar of U3, in reverse:
//   A2 = 2/3 (G + dt J(U2)^T G)        (cotangent of U2)
//   A1 = 1/4 (A2 + dt J(U1)^T A2)      (cotangent of U1)
//   Ubar_n = 3/4 A2 + 1/3 G + A1 + dt J(Un)^T A1,
// and dtbar = sum over the stages of (s G_stage) . L(U_stage). The forward
// pass keeps the face/edge records at Un and U1 and recomputes those at U2;
// the direct term 3/4 A2 + 1/3 G goes to the space of U2, which nothing reads
// after the last stage's adjoint.
template <int DIM, int LIM, int RS>
hipError_t adjoint_rk3(const AdjointArgs& a, const Bufs& bf, StageArgs f) {
  const int64_t n = a.g.n;
  const unsigned nb = blocks_for(n);
  if (!a.U2 || !bf.FW1) return hipErrorInvalidValue;
  f.stage = 1;  // U1 = Un + dt L(Un), records at Un kept
  f.U = a.Un;
  f.U0 = nullptr;
  f.out = a.U1;
  f.FW = bf.FWn;
  f.EW = bf.EWn;
  hipError_t e = launch_stage(f);
  if (e != hipSuccess) return e;
  f.stage = 4;  // U2 = (3 Un + (U1 + dt L(U1))) / 4, records at U1 kept
  f.U = a.U1;
  f.U0 = a.Un;
  f.out = a.U2;
  f.FW = bf.FW1;
  f.EW = bf.EW1;
  e = launch_stage(f);
  if (e != hipSuccess) return e;
  f.stage = 3;  // records at U2
  f.U = a.U2;
  f.U0 = nullptr;
  f.FW = a.FW;
  f.EW = a.EW;
  e = launch_stage(f);
  if (e != hipSuccess) return e;
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.U2, a.FW, a.EW, a.Ubar1, 2.0 / 3.0, nullptr, 0.0, bf.A,
                                  bf.part);
  if (e != hipSuccess) return e;
  const unsigned n8 = (unsigned)((8 * n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_axpby, dim3(n8), dim3(kBlock), 0, a.stream, bf.A, 0.75, a.Ubar1,
                     1.0 / 3.0, a.U2, 8 * n);
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.U1, bf.FW1, bf.EW1, bf.A, 0.25, nullptr, 0.0, bf.A1,
                                  bf.part + nb);
  if (e != hipSuccess) return e;
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.Un, bf.FWn, bf.EWn, bf.A1, 1.0, a.U2, 1.0, a.Ubar0,
                                  bf.part + 2 * nb);
  if (e != hipSuccess) return e;
  if (a.want_dtbar)
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(1024), 0, a.stream, bf.part, (int)(3 * nb),
                       a.dtbar_dev);
  return hipGetLastError();
}

template <int DIM, int LIM, int RS>
hipError_t adjoint_impl(const AdjointArgs& a) {
  const int64_t n = a.g.n;
  const Bufs bf = carve(a.scratch, a.dim, n, a.integrator);
  const unsigned nb = blocks_for(n);
  StageArgs f{};
  f.dim = a.dim;
  f.limiter = a.limiter;
  f.riemann = a.riemann;
  f.precision = 0;
  f.g = a.g;
  f.FW = a.FW;
  f.EW = a.EW;
  f.dt = a.dt;
  f.dtp = nullptr;
  f.flag = a.flag;
  f.stream = a.stream;
  f.timer = nullptr;
  if (a.integrator == 1) return adjoint_rk3<DIM, LIM, RS>(a, bf, f);
  // forward stage 1: U1 = Un + dt L(Un); its face/edge records at Un are
  // kept (FWn, EWn) for the stage-1 adjoint
  f.stage = 1;
  f.U = a.Un;
  f.U0 = nullptr;
  f.out = a.U1;
  f.FW = bf.FWn;
  f.EW = bf.EWn;
  hipError_t e = launch_stage(f);
  if (e != hipSuccess) return e;
  // records at U1, then the stage-2 adjoint: A = G2 + dt J(U1)^T G2, G2 = Ubar1/2
  f.stage = 3;
  f.U = a.U1;
  f.FW = a.FW;
  f.EW = a.EW;
  e = launch_stage(f);
  if (e != hipSuccess) return e;
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.U1, a.FW, a.EW, a.Ubar1, 0.5, nullptr, 0.0, bf.A,
                                  bf.part);
  if (e != hipSuccess) return e;
  // the stage-1 adjoint at Un: Ubar0 = Ubar1/2 + A + dt J(Un)^T A
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.Un, bf.FWn, bf.EWn, bf.A, 1.0, a.Ubar1, 0.5, a.Ubar0,
                                  bf.part + nb);
  if (e != hipSuccess) return e;
  if (a.want_dtbar)
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(1024), 0, a.stream, bf.part, (int)(2 * nb),
                       a.dtbar_dev);
  return hipGetLastError();
}

template <int DIM>
hipError_t adjoint_dim(const AdjointArgs& a) {
  if (a.limiter == 0)
    return a.riemann == 0 ? adjoint_impl<DIM, 0, 0>(a) : adjoint_impl<DIM, 0, 1>(a);
  return a.riemann == 0 ? adjoint_impl<DIM, 1, 0>(a) : adjoint_impl<DIM, 1, 1>(a);
}

}  // namespace

size_t adjoint_workspace_bytes(int dim, size_t ncell, int integrator) {
  const size_t nb = (ncell + kBlock - 1) / kBlock;
  size_t per_cell = 3 * NE + 3 * 14 + 3 + 3 + 8 + 8 + 8 + (size_t)dim * NSLOT + 3;
  if (integrator == 1) per_cell += (size_t)dim * NSLOT + 3 + 8;  // FW1, EW1, A1
  return sizeof(double) * (per_cell * ncell + (integrator == 1 ? 3 : 2) * nb) + 256;
}

hipError_t launch_adjoint_step(const AdjointArgs& a) {
  return (a.dim == 3) ? adjoint_dim<3>(a) : adjoint_dim<2>(a);
}

}  // namespace mhd
