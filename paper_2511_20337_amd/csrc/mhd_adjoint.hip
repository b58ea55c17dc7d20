// Adjoint (vector-Jacobian product) of one SSP-RK2 step, FP64, gather form.
//
// The step is Phi(Un) = (Un + S(S(Un)))/2 with S(U) = U + dt L(U). Reverse:
//   G2 = Ubar1/2;        U1bar = G2 + dt J_L(U1)^T G2;
//   Ubar0 = Ubar1/2 + U1bar + dt J_L(Un)^T U1bar;
//   dtbar = <G2, L(U1)> + <U1bar, L(Un)>.
// J_L^T G is assembled from the local Jacobians of each piece of L, every
// output written by exactly one thread (no atomics, deterministic):
//   k_adj_edges — the EMF cotangent from -curl E, times the partial
//                 derivatives of the upwind EMF average w.r.t. its twelve
//                 inputs (per edge, stored);
//   k_adj_faces — per face: flux cotangents from the divergence, cotangents
//                 of alpha+-, the weighted velocities and b gathered from the
//                 edges that used them (through the adjoint of their
//                 reconstruction), then the Riemann solver's vector-Jacobian
//                 product, evaluated with the solver itself on a forward-mode
//                 dual scalar, one pass per input;
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
// Forward-mode dual scalar (value, one tangent) for the Riemann solver.
struct Dual {
  double v, d;
  __device__ __forceinline__ Dual() : v(0.0), d(0.0) {}
  __device__ __forceinline__ Dual(double x) : v(x), d(0.0) {}  // NOLINT
  __device__ __forceinline__ Dual(double x, double t) : v(x), d(t) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
  return Dual(a.v * b.v, __builtin_fma(a.d, b.v, a.v * b.d));
}
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
__device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
__device__ __forceinline__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
__device__ __forceinline__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
// Found by argument-dependent lookup from the solver template. The value
// parts use the same quotient, reciprocal and square root as the forward
// kernels, so a dual pass reproduces the forward values bit for bit and
// takes the same branches.
// (Tangents may round differently from their exact quotients; only the
// values steer branches.)
__device__ __forceinline__ Dual sqrt_r(Dual x) {
  double h;
  const double s = ::mhd::sqrt_r_half(x.v, h);
  return Dual(s, s > 0.0 ? x.d * h : 0.0);
}
__device__ __forceinline__ Dual abs_r(Dual x) { return x.v < 0.0 ? -x : x; }
__device__ __forceinline__ Dual fma_r(Dual a, Dual b, Dual c) {
  return Dual(__builtin_fma(a.v, b.v, c.v), __builtin_fma(a.d, b.v, __builtin_fma(a.v, b.d, c.d)));
}
__device__ __forceinline__ Dual rcp_r(Dual x) {
  const double r = ::mhd::rcp_r(x.v);
  return Dual(r, -x.d * r * r);
}
__device__ __forceinline__ Dual div_r(Dual a, Dual b) {
  double r;
  const double q = ::mhd::div_r_rcp(a.v, b.v, r);
  return Dual(q, __builtin_fma(-q, b.d, a.d) * r);
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
  double* part;  // 2 x nblocks: dtbar partial sums
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
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
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
// (slot V2) and b_D along A.
template <int C, int ROLE, int LIM>
__device__ __forceinline__ void edge_to_face(const double* __restrict__ U,
                                             const double* __restrict__ FW,
                                             const double* __restrict__ EB, const Geom& g, int i,
                                             int j, int k, int64_t c, double& apbar,
                                             double& ambar, double& vbar, double& bbar) {
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
  // alpha: the edge at c takes max(face c-e, face c); the edge at c+e takes
  // max(face c, face c+e); the first argument wins ties.
  {
    const double* ap = f + S_AP * n;
    const double* am = f + S_AM * n;
    if (ap[c] > ap[cm1]) apbar += e[sap * n + c];
    if (!(ap[cp1] > ap[c])) apbar += e[sap * n + cp1];
    if (am[c] > am[cm1]) ambar += e[sam * n + c];
    if (!(am[cp1] > am[c])) ambar += e[sam * n + cp1];
  }
  // reconstructed values: upper extrapolation of face p feeds the edge at
  // p+e (as its lower value), the lower extrapolation feeds the edge at p
  const double* v = f + (ROLE == 0 ? S_V1 : S_V2) * n;
  const double* b = U + (F_BX + D) * n;
  const double xv[5] = {v[cm2], v[cm1], v[c], v[cp1], v[cp2]};
  const double xb[5] = {b[cm2], b[cm1], b[c], b[cp1], b[cp2]};
  const double vp[3] = {e[svlo * n + c], e[svlo * n + cp1], e[svlo * n + cp2]};
  const double vm[3] = {e[svhi * n + cm1], e[svhi * n + c], e[svhi * n + cp1]};
  const double bp[3] = {e[sblo * n + c], e[sblo * n + cp1], e[sblo * n + cp2]};
  const double bm[3] = {e[sbhi * n + cm1], e[sbhi * n + c], e[sbhi * n + cp1]};
  vbar += plm_adjoint<LIM>(xv, vp, vm);
  bbar += plm_adjoint<LIM>(xb, bp, bm);
}

template <int DIM, int D, int LIM, int RS>
__device__ __forceinline__ void face_adjoint(const double* __restrict__ U,
                                             const double* __restrict__ FW,
                                             const double* __restrict__ G, double s,
                                             const double* __restrict__ EB, const Geom& g, int i,
                                             int j, int k, int64_t c, const Bufs& bf) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int64_t n = g.n;
  const int64_t cm = shifted<D>(g, i, j, k, -1);
  const double idl = s / delta<D>(g);
  // flux cotangents (face frame: rho, m_n, m_t1, m_t2, B_t1, B_t2, E)
  double fb[7];
  fb[0] = (G[c] - G[cm]) * idl;
  fb[1] = (G[(F_MX + D) * n + c] - G[(F_MX + D) * n + cm]) * idl;
  fb[2] = (G[(F_MX + T1) * n + c] - G[(F_MX + T1) * n + cm]) * idl;
  fb[3] = (G[(F_MX + T2) * n + c] - G[(F_MX + T2) * n + cm]) * idl;
  fb[4] = 0.0;
  fb[5] = 0.0;
  fb[6] = (G[F_EN * n + c] - G[F_EN * n + cm]) * idl;
  if (DIM == 2) {
    const double bz = (G[F_BZ * n + c] - G[F_BZ * n + cm]) * idl;
    if (D == 0) fb[5] = bz; else fb[4] = bz;   // B_z is t2 of x-faces, t1 of y-faces
  }
  // cotangents from the edges
  double apbar = 0.0, ambar = 0.0, v1bar = 0.0, v2bar = 0.0, bbar = 0.0;
  constexpr int C1 = (D + 2) % 3;  // this face is an a-face of C1
  constexpr int C2 = (D + 1) % 3;  // and a b-face of C2
  if (DIM == 3 || C1 == 2) edge_to_face<C1, 0, LIM>(U, FW, EB, g, i, j, k, c, apbar, ambar, v1bar, bbar);
  if (DIM == 3 || C2 == 2) edge_to_face<C2, 1, LIM>(U, FW, EB, g, i, j, k, c, apbar, ambar, v2bar, bbar);
  // Riemann vector-Jacobian product, one dual pass per input
  double wl[7], wr[7], bn;
  face_inputs<DIM, D, LIM>(U, g, i, j, k, wl, wr, bn);
  double* wb = bf.WB + (int64_t)D * 14 * n + c;
  double bnbar = 0.0;
#pragma unroll 1
  for (int in = 0; in < 15; ++in) {
    Dual dl[7], dr[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      dl[q] = Dual(wl[q], in == q ? 1.0 : 0.0);
      dr[q] = Dual(wr[q], in == 7 + q ? 1.0 : 0.0);
    }
    const Dual dbn(bn, in == 14 ? 1.0 : 0.0);
    RiemannOut<Dual> o;
    riemann<RS, Dual>(Dual(g.gamma), dl, dr, dbn, o);
    double acc = apbar * o.ap.d + ambar * o.am.d + v1bar * o.v1.d + v2bar * o.v2.d;
#pragma unroll
    for (int q = 0; q < 7; ++q) acc += fb[q] * o.f[q].d;
    if (in < 14) wb[(int64_t)in * n] = acc;
    else bnbar = acc;
  }
  bf.BF[(int64_t)D * n + c] = bnbar + bbar;
}

template <int DIM, int LIM, int RS>
__global__ __launch_bounds__(kBlock) void k_adj_faces(const double* __restrict__ U,
                                                      const double* __restrict__ FW,
                                                      const double* __restrict__ G, double s,
                                                      Geom g, Bufs bf) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  face_adjoint<DIM, 0, LIM, RS>(U, FW, G, s, bf.EB, g, i, j, k, c, bf);
  face_adjoint<DIM, 1, LIM, RS>(U, FW, G, s, bf.EB, g, i, j, k, c, bf);
  if (DIM == 3) face_adjoint<DIM, 2, LIM, RS>(U, FW, G, s, bf.EB, g, i, j, k, c, bf);
}

// ---------------------------------------------------------------------------
template <int DIM, int D, int LIM>
__device__ __forceinline__ void plm_cell_adjoint(const double* __restrict__ U,
                                                 const double* __restrict__ WB, const Geom& g,
                                                 int i, int j, int k, double* vbar) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  const int64_t n = g.n;
  double V[5][8];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int o = s - 2;
    prim_at<DIM>(U, g, D == 0 ? wrap(i + o, g.nx) : i, D == 1 ? wrap(j + o, g.ny) : j,
                 D == 2 ? wrap(k + o, g.nz) : k, V[s]);
  }
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
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  const int64_t n = g.n;
  double vb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  plm_cell_adjoint<DIM, 0, LIM>(U, bf.WB, g, i, j, k, vb);
  plm_cell_adjoint<DIM, 1, LIM>(U, bf.WB, g, i, j, k, vb);
  if (DIM == 3) plm_cell_adjoint<DIM, 2, LIM>(U, bf.WB, g, i, j, k, vb);
  // primitive recovery: v = m/rho, p = (gamma-1)(E - |m|^2/(2 rho) - |Bc|^2/2)
  double V[8];
  prim_at<DIM>(U, g, i, j, k, V);
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

// ---------------------------------------------------------------------------
// out = cd * Dir + s G + dt J^T (s G); per-block partial of <s G, L(U)>.
template <int DIM>
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
    // L(U) from the forward records, as in the update kernel
    const int64_t xp = lin(g, wrap(i + 1, g.nx), j, k);
    const int64_t yp = lin(g, i, wrap(j + 1, g.ny), k);
    const int64_t zp = (DIM == 3) ? lin(g, i, j, wrap(k + 1, g.nz)) : c;
    const double idx = 1.0 / g.dx, idy = 1.0 / g.dy, idz = 1.0 / g.dz;
    const double* fx = FW;
    const double* fy = FW + (int64_t)NSLOT * n;
    const double* fz = FW + (int64_t)2 * NSLOT * n;
    double L[8];
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
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double sg = s * G[q * n + c];
      double v = sg + dt * jt[q];
      if (Dir) v += cd * Dir[q * n + c];
      out[q * n + c] = v;
      dot += sg * L[q];
    }
  }
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

Bufs carve(double* scratch, int64_t n) {
  Bufs b;
  double* p = scratch;
  b.EB = p; p += 3 * NE * n;
  b.WB = p; p += 3 * 14 * n;
  b.BF = p; p += 3 * n;
  b.BC = p; p += 3 * n;
  b.T = p; p += 8 * n;
  b.A = p; p += 8 * n;
  b.part = p;
  return b;
}

// J^T of one stage, combined: out = cd Dir + s G + dt J_L(U)^T (s G); the
// forward records FW/EW must hold the face/edge data at U.
template <int DIM, int LIM, int RS>
hipError_t stage_adjoint(const AdjointArgs& a, const Bufs& bf, const double* U,
                         const double* G, double s, const double* Dir, double cd, double* out,
                         double* part) {
  const unsigned nb = blocks_for(a.g.n);
  hipLaunchKernelGGL((k_adj_edges<DIM, LIM>), dim3(nb), dim3(kBlock), 0, a.stream, U, a.FW, G, s,
                     a.g, bf.EB);
  hipLaunchKernelGGL((k_adj_faces<DIM, LIM, RS>), dim3(nb), dim3(kBlock), 0, a.stream, U, a.FW, G,
                     s, a.g, bf);
  hipLaunchKernelGGL((k_adj_cells<DIM, LIM>), dim3(nb), dim3(kBlock), 0, a.stream, U, a.g, bf);
  hipLaunchKernelGGL((k_adj_final<DIM>), dim3(nb), dim3(kBlock), 0, a.stream, G, s, Dir, cd, a.FW,
                     a.EW, a.g, a.dt, bf, out, part);
  return hipGetLastError();
}

template <int DIM, int LIM, int RS>
hipError_t adjoint_impl(const AdjointArgs& a) {
  const int64_t n = a.g.n;
  const Bufs bf = carve(a.scratch, n);
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
  // forward stage 1: U1 = Un + dt L(Un)
  f.stage = 1;
  f.U = a.Un;
  f.U0 = nullptr;
  f.out = a.U1;
  hipError_t e = launch_stage(f);
  if (e != hipSuccess) return e;
  // records at U1, then the stage-2 adjoint: A = G2 + dt J(U1)^T G2, G2 = Ubar1/2
  f.stage = 3;
  f.U = a.U1;
  e = launch_stage(f);
  if (e != hipSuccess) return e;
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.U1, a.Ubar1, 0.5, nullptr, 0.0, bf.A, bf.part);
  if (e != hipSuccess) return e;
  // records at Un, then the stage-1 adjoint: Ubar0 = Ubar1/2 + A + dt J(Un)^T A
  f.U = a.Un;
  e = launch_stage(f);
  if (e != hipSuccess) return e;
  e = stage_adjoint<DIM, LIM, RS>(a, bf, a.Un, bf.A, 1.0, a.Ubar1, 0.5, a.Ubar0, bf.part + nb);
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

size_t adjoint_workspace_bytes(int dim, size_t ncell) {
  (void)dim;
  const size_t nb = (ncell + kBlock - 1) / kBlock;
  return sizeof(double) * ((size_t)(3 * NE + 3 * 14 + 3 + 3 + 8 + 8) * ncell + 2 * nb) + 256;
}

hipError_t launch_adjoint_step(const AdjointArgs& a) {
  return (a.dim == 3) ? adjoint_dim<3>(a) : adjoint_dim<2>(a);
}

}  // namespace mhd
