// ORACLE — test infrastructure, not product code.
//
// A plain, slow, obviously-correct CPU implementation of one time step of the
// finite-volume ideal-MHD scheme on a uniform periodic Cartesian mesh:
// primitive recovery, piecewise-linear limited reconstruction, an HLL or HLLD
// Riemann solve at every interface, an upwind constrained-transport EMF
// average on cell edges, the flux-divergence / curl update, and a two-stage
// strong-stability-preserving Runge-Kutta step with a CFL time step.
//
// Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
// load this library. It shares no source, header, helper or constant with the
// GPU library; the two meet only through the seeded input generators.
//
// Paper: "The PLUTO Code on GPUs: A First Look at Eulerian MHD Methods"
// (arXiv 2511.20337). Citations name the paper's section / equation.
//   conservation law ............ Sec. 2.1, Eq. (cons_law) with S = 0
//   state, flux tensor .......... Sec. 2.1, Eq. (mhd)
//   total energy / ideal EOS .... Sec. 2.1, Eq. (Energy)
//   semi-discrete FV update ..... Sec. 2.2, Eq. (FV)
//   SSP Runge-Kutta ............. Sec. 2.2, Eq. (RK3) (two-stage member used)
//   reconstruction .............. Sec. 2.2, Eq. (reconstruct), on primitives
//   primitive inversion ......... Sec. 2.2, unnumbered equation after (reconstruct)
//   Riemann flux ................ Sec. 2.2, unnumbered flux equation; HLLD is
//                                 the Miyoshi & Kusano (2005) solver the
//                                 paper cites for both benchmarks (Sec. 4.1, 4.2)
//   constrained transport ....... Sec. 2.2 (CT keeps div B at machine precision)
//
// Every point where the paper is silent, ambiguous or garbled is taken with a
// stated reading, marked [reading] below where it applies.
//
// All arithmetic is written with a scalar template parameter:
//   S — scalar of the stored state, primitive recovery and accumulation;
//   R — scalar of reconstruction, Riemann solve and EMF.
// (S, R) = (double, double) is the FP64 oracle; (double, float) is the mixed
// variant (Riemann fluxes and EMFs rounded to double before differencing);
// (Dual, Dual) carries one forward-mode tangent through the whole step and
// serves as the exact Jacobian-vector product the adjoint is checked against.
// Build with -ffp-contract=off so that every operation rounds where written.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual number: value v and one tangent d.
// Branches (min/max/limiter/HLLD region) follow the value, which gives the
// derivative of the branch taken.
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}           // NOLINT: implicit on purpose
  Dual(double x, double t) : v(x), d(t) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }

// Operation-counting scalar: the value of a double, and a count of every
// floating-point operation (add/sub, mul, div, sqrt) charged to the current
// phase of the right-hand side. Used only to state the algorithmic flops per
// cell of each phase of the method.
enum { PH_PRIM = 0, PH_FACE, PH_EMF, PH_UPDATE, PH_N };
long long g_ops[PH_N][4];
int g_phase = 0;
struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}  // NOLINT: implicit on purpose
};
inline Cnt cnt(double x, int kind) { g_ops[g_phase][kind] += 1; return Cnt(x); }
inline Cnt operator+(Cnt a, Cnt b) { return cnt(a.v + b.v, 0); }
inline Cnt operator-(Cnt a, Cnt b) { return cnt(a.v - b.v, 0); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { return cnt(a.v * b.v, 1); }
inline Cnt operator/(Cnt a, Cnt b) { return cnt(a.v / b.v, 2); }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }

inline double val(double x) { return x; }
inline double val(float x) { return (double)x; }
inline double val(Dual x) { return x.v; }
inline double val(Cnt x) { return x.v; }

inline double Sqrt(double x) { return std::sqrt(x); }
inline float Sqrt(float x) { return std::sqrt(x); }
inline Dual Sqrt(Dual x) {
  double s = std::sqrt(x.v);
  return Dual(s, s > 0.0 ? 0.5 * x.d / s : 0.0);
}
inline double Abs(double x) { return std::fabs(x); }
inline float Abs(float x) { return std::fabs(x); }
inline Dual Abs(Dual x) { return x.v < 0.0 ? -x : x; }
inline Cnt Sqrt(Cnt x) { return cnt(std::sqrt(x.v), 3); }
inline Cnt Abs(Cnt x) { return Cnt(std::fabs(x.v)); }
// min/max return the first argument on ties.
template <class T> inline T Max(T a, T b) { return (b > a) ? b : a; }
template <class T> inline T Min(T a, T b) { return (b < a) ? b : a; }
inline bool Finite(double x) { return std::isfinite(x); }
inline bool Finite(float x) { return std::isfinite(x); }
inline bool Finite(Dual x) { return std::isfinite(x.v); }
inline bool Finite(Cnt x) { return std::isfinite(x.v); }

// Conversions between the state scalar and the face scalar.
template <class To> struct Cast;
template <> struct Cast<double> {
  static double of(double x) { return x; }
  static double of(float x) { return (double)x; }
};
template <> struct Cast<float> {
  static float of(double x) { return (float)x; }
  static float of(float x) { return x; }
};
template <> struct Cast<Dual> {
  static Dual of(Dual x) { return x; }
};
template <> struct Cast<Cnt> {
  static Cnt of(Cnt x) { return x; }
};

// ---------------------------------------------------------------------------
// Configuration (mirrors the Python-side ctypes structure of this oracle).
struct OCfg {
  int32_t dim;              // 2 or 3
  int32_t nx, ny, nz;       // cells; nz == 1 when dim == 2
  double xmin, xmax, ymin, ymax, zmin, zmax;
  double gamma;             // adiabatic index
  double cfl;               // Courant number
  int32_t limiter;          // 0 minmod, 1 van Leer (PLM); 2 WENO-Z
  int32_t riemann;          // 0 HLLD, 1 HLL
  int32_t precision;        // 0 FP64, 1 mixed (FP32 reconstruction/Riemann/EMF)
  int32_t nthreads;         // OpenMP threads (<= 0: library default)
  int32_t integrator;       // 0 SSP-RK2, 1 SSP-RK3
  int32_t emf;              // 0 UCT-HLL, 1 UCT-HLLD
};

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4, BX = 5, BY = 6, BZ = 7, NF = 8 };
// primitive slots
enum { VRHO = 0, VVX = 1, VVY = 2, VVZ = 3, VPR = 4, VBX = 5, VBY = 6, VBZ = 7 };

struct Grid {
  int dim, nx, ny, nz;
  double dx, dy, dz;
  size_t ncell;
  explicit Grid(const OCfg& c)
      : dim(c.dim), nx(c.nx), ny(c.ny), nz(c.nz),
        dx((c.xmax - c.xmin) / c.nx), dy((c.ymax - c.ymin) / c.ny),
        dz((c.zmax - c.zmin) / c.nz),
        ncell((size_t)c.nx * c.ny * c.nz) {}
  static int wrap(int i, int n) { return ((i % n) + n) % n; }
  // linear index of cell (i,j,k) with periodic wrap
  size_t at(int i, int j, int k) const {
    return ((size_t)wrap(k, nz) * ny + wrap(j, ny)) * nx + wrap(i, nx);
  }
  // cell shifted by s along direction d
  size_t shift(int i, int j, int k, int d, int s) const {
    return at(i + (d == 0 ? s : 0), j + (d == 1 ? s : 0), k + (d == 2 ? s : 0));
  }
  double delta(int d) const { return d == 0 ? dx : (d == 1 ? dy : dz); }
};

// Transverse directions of a face normal d: (t1, t2) = (y,z), (z,x), (x,y).
inline int t1_of(int d) { return (d + 1) % 3; }
inline int t2_of(int d) { return (d + 2) % 3; }

// Rows (j, k) of the mesh are independent within one sweep; they are shared
// over OpenMP threads.
template <class F> void par_for(int n, int nthreads, F&& f) {
#ifdef _OPENMP
  if (nthreads > 0) {
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int k = 0; k < n; ++k) f(k);
  } else {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) f(k);
  }
#else
  (void)nthreads;
  for (int k = 0; k < n; ++k) f(k);
#endif
}

template <class F> void par_rows(const Grid& G, int nthreads, F&& f) {
  par_for(G.nz * G.ny, nthreads, [&](int r) { f(r % G.ny, r / G.ny); });
}

// ---------------------------------------------------------------------------
// Limited slope for piecewise-linear reconstruction [reading: the paper names
// only a generic reconstruction operator R+/R- (Eq. reconstruct); PLM with a
// minmod or van Leer (harmonic) limiter, applied component-wise].
template <class R> R limited_slope(int limiter, R dm, R dp) {
  if (dm * dp <= R(0)) return R(0);
  if (limiter == 0) return (Abs(dm) <= Abs(dp)) ? dm : dp;        // minmod
  return R(2) * dm * dp / (dm + dp);                              // van Leer
}

// Fifth-order WENO-Z value at the upper interface of the middle cell of five
// (v0..v4 = cells i-2..i+2), after Borges et al. (2008), cited with Eq.
// (reconstruct) [reading: the paper gives no formulas; the three third-order
// candidate values, the Jiang-Shu smoothness indicators beta_k, the ideal
// weights (1, 6, 3)/10, tau5 = |beta0 - beta2| and the Z weights
// alpha_k = d_k (1 + tau5 / (beta_k + eps)) with the exponent 1 and
// eps = 1e-40]. The lower interface value is the same function of the cells
// in reverse order.
template <class R> R wenoz_upper(R v0, R v1, R v2, R v3, R v4) {
  const R q0 = (R(2) * v0 - R(7) * v1 + R(11) * v2) / R(6);
  const R q1 = (-v1 + R(5) * v2 + R(2) * v3) / R(6);
  const R q2 = (R(2) * v2 + R(5) * v3 - v4) / R(6);
  const R c1 = R(13) / R(12), c2 = R(1) / R(4);
  const R a0 = v0 - R(2) * v1 + v2, b0 = v0 - R(4) * v1 + R(3) * v2;
  const R a1 = v1 - R(2) * v2 + v3, b1 = v1 - v3;
  const R a2 = v2 - R(2) * v3 + v4, b2 = R(3) * v2 - R(4) * v3 + v4;
  const R beta0 = c1 * a0 * a0 + c2 * b0 * b0;
  const R beta1 = c1 * a1 * a1 + c2 * b1 * b1;
  const R beta2 = c1 * a2 * a2 + c2 * b2 * b2;
  const R tau5 = Abs(beta0 - beta2);
  const R eps = R(1e-40);
  const R al0 = R(0.1) * (R(1) + tau5 / (beta0 + eps));
  const R al1 = R(0.6) * (R(1) + tau5 / (beta1 + eps));
  const R al2 = R(0.3) * (R(1) + tau5 / (beta2 + eps));
  return (al0 * q0 + al1 * q1 + al2 * q2) / (al0 + al1 + al2);
}

// ---------------------------------------------------------------------------
// One-dimensional Riemann problem in the frame of the face normal.
// w = (rho, u, v, w, B_t1, B_t2, p); bn = normal field (continuous).
// Output: the numerical flux of (rho, m_n, m_t1, m_t2, B_t1, B_t2, E) and the
// quantities the upwind EMF needs: alpha+ = max(0,S_R), alpha- = max(0,-S_L)
// and the HLL-weighted transverse velocities.
template <class R> struct RSOut {
  R F[7];
  R ap, am, vt1, vt2;
  // UCT-HLLD coefficients (filled on request): the flux weight of the left
  // state (that of the right one is 1 - om), the diffusion coefficients of
  // the left and right transverse field, and the face velocities weighted by
  // (om, 1 - om)
  R om, dl, dr, wt1, wt2;
};

// Conserved vector, physical flux (Eq. mhd, projected on the normal) and total
// pressure of a primitive state (Eq. Energy for the total energy).
template <class R>
void state_of(R g, const R w[7], R bn, R U[7], R F[7], R& pt) {
  const R rho = w[0], u = w[1], v = w[2], ww = w[3], bt1 = w[4], bt2 = w[5], p = w[6];
  const R B2 = bn * bn + bt1 * bt1 + bt2 * bt2;
  const R v2 = u * u + v * v + ww * ww;
  pt = p + R(0.5) * B2;
  const R E = p / (g - R(1)) + R(0.5) * rho * v2 + R(0.5) * B2;
  U[0] = rho; U[1] = rho * u; U[2] = rho * v; U[3] = rho * ww;
  U[4] = bt1; U[5] = bt2; U[6] = E;
  const R vb = u * bn + v * bt1 + ww * bt2;
  F[0] = rho * u;
  F[1] = rho * u * u + pt - bn * bn;
  F[2] = rho * u * v - bn * bt1;
  F[3] = rho * u * ww - bn * bt2;
  F[4] = u * bt1 - v * bn;
  F[5] = u * bt2 - ww * bn;
  F[6] = (E + pt) * u - bn * vb;
}

// Fast magnetosonic speed along the normal.
template <class R> R fast_speed(R g, R rho, R p, R bn, R bt1, R bt2) {
  const R gp = g * p;
  const R B2 = bn * bn + bt1 * bt1 + bt2 * bt2;
  const R a = gp + B2;
  const R disc = Max(R(0), a * a - R(4) * gp * bn * bn);
  return Sqrt((a + Sqrt(disc)) / (R(2) * rho));
}

// Diagnostic counters of the HLLD degeneracy test (star sides evaluated,
// sides found degenerate), per working precision: [0] FP64, [1] FP32.
long long g_deg_sides[2], g_deg_hits[2];
bool g_count_deg = false;  // set only while oracle_count_degenerate runs
template <class R> constexpr int prec_index() { return std::is_same<R, float>::value ? 1 : 0; }

// Relative tolerance of the HLLD degeneracy test, per working precision.
template <class R> struct DegTol { static constexpr double value = 1e-12; };
template <> struct DegTol<float> { static constexpr double value = 1e-12 * 536870912.0; };

// [reading] UCT-HLLD (the CT average the paper names for its runs; its
// formulas are not in the paper). At the wave structure of a face (wave
// speeds, contact speed, star densities and the per-side factors that map
// B_t and v_t into the star states), the HLLD flux of each transverse field
// component is linear in (B_t^L, B_t^R, v_t^L, v_t^R):
//   F[B_t] = chiL B_t^L + chiR B_t^R - B_n (om v_t^L + (1 - om) v_t^R).
// The upwind EMF takes om and 1 - om as the weights of the left and right
// advective terms v_n B_t, d^L = chiL - om u_L and d^R = (1 - om) u_R - chiR
// as the diffusion coefficients, and om v_t^L + (1 - om) v_t^R as the face
// velocity, so that plane-parallel data give E = -F_HLLD[B_t] exactly. For the
// HLL flux the same construction gives om = alpha+/(alpha+ + alpha-),
// d^L = d^R = alpha+ alpha-/(alpha+ + alpha-).
template <class R>
void uct_hll_coeffs(const R wl[7], const R wr[7], RSOut<R>& o) {
  o.om = o.ap / (o.ap + o.am);
  o.dl = o.ap * o.am / (o.ap + o.am);
  o.dr = o.dl;
  o.wt1 = o.om * wl[2] + (R(1) - o.om) * wr[2];
  o.wt2 = o.om * wl[3] + (R(1) - o.om) * wr[3];
}

template <class R>
void riemann(int solver, R g, const R wl[7], const R wr[7], R bn, RSOut<R>& o,
             bool uct_hlld = false) {
  R UL[7], FL[7], UR[7], FR[7], ptl, ptr;
  state_of(g, wl, bn, UL, FL, ptl);
  state_of(g, wr, bn, UR, FR, ptr);
  const R ul = wl[1], ur = wr[1];
  const R cfl = fast_speed(g, wl[0], wl[6], bn, wl[4], wl[5]);
  const R cfr = fast_speed(g, wr[0], wr[6], bn, wr[4], wr[5]);
  // [reading] wave-speed estimate shared by HLL and HLLD
  const R cmax = Max(cfl, cfr);
  const R SL = Min(ul, ur) - cmax;
  const R SR = Max(ul, ur) + cmax;

  o.ap = Max(R(0), SR);
  o.am = Max(R(0), -SL);
  o.vt1 = (o.ap * wl[2] + o.am * wr[2]) / (o.ap + o.am);
  o.vt2 = (o.ap * wl[3] + o.am * wr[3]) / (o.ap + o.am);

  if (solver == 1) {  // HLL: single intermediate state
    if (uct_hlld) uct_hll_coeffs(wl, wr, o);
    if (SL >= R(0)) { for (int q = 0; q < 7; ++q) o.F[q] = FL[q]; return; }
    if (SR <= R(0)) { for (int q = 0; q < 7; ++q) o.F[q] = FR[q]; return; }
    for (int q = 0; q < 7; ++q)
      o.F[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (UR[q] - UL[q])) / (SR - SL);
    return;
  }

  // HLLD (Miyoshi & Kusano 2005): four intermediate states.
  if (SL > R(0)) {
    for (int q = 0; q < 7; ++q) o.F[q] = FL[q];
    if (uct_hlld) { o.om = R(1); o.dl = R(0); o.dr = R(0); o.wt1 = wl[2]; o.wt2 = wl[3]; }
    return;
  }
  if (SR < R(0)) {
    for (int q = 0; q < 7; ++q) o.F[q] = FR[q];
    if (uct_hlld) { o.om = R(0); o.dl = R(0); o.dr = R(0); o.wt1 = wr[2]; o.wt2 = wr[3]; }
    return;
  }

  // contact speed and total pressure of the star region
  const R sdl = SL - ul, sdr = SR - ur;
  const R den = sdr * wr[0] - sdl * wl[0];
  const R SM = (sdr * wr[0] * ur - sdl * wl[0] * ul - ptr + ptl) / den;
  const R pts = (sdr * wr[0] * ptl - sdl * wl[0] * ptr +
                 wl[0] * wr[0] * sdr * sdl * (ur - ul)) / den;

  // single-star states on each side
  R Us[2][7];
  R rhos[2], vs[2], ws[2], b1s[2], b2s[2];
  R zeta[2], eta[2];  // B*_t = zeta B_t, v*_t = v_t - eta B_t (per side)
  const R* wlr[2] = {wl, wr};
  const R* Ulr[2] = {UL, UR};
  const R Slr[2] = {SL, SR};
  for (int s = 0; s < 2; ++s) {
    const R* w = wlr[s];
    const R* U = Ulr[s];
    const R S = Slr[s];
    const R su = S - w[1];
    const R sm = S - SM;
    rhos[s] = w[0] * su / sm;
    const R big = w[0] * su * sm;
    const R D = big - bn * bn;
    // [reading] degenerate case (S_alpha ~ S*_alpha): tangential fields
    // unchanged when |D| is within a relative tolerance of 1e-12 in FP64
    // units, scaled to the working precision (x 2^29 in FP32)
    const bool degenerate = Abs(D) <= R(DegTol<R>::value) * (Abs(big) + bn * bn);
    if (g_count_deg) {
#pragma omp atomic
      g_deg_sides[prec_index<R>()] += 1;
      if (degenerate) {
#pragma omp atomic
        g_deg_hits[prec_index<R>()] += 1;
      }
    }
    if (degenerate) {
      vs[s] = w[2]; ws[s] = w[3]; b1s[s] = w[4]; b2s[s] = w[5];
      zeta[s] = R(1);
      eta[s] = R(0);
    } else {
      const R fv = bn * (SM - w[1]) / D;
      vs[s] = w[2] - w[4] * fv;
      ws[s] = w[3] - w[5] * fv;
      const R fb = (w[0] * su * su - bn * bn) / D;
      b1s[s] = w[4] * fb;
      b2s[s] = w[5] * fb;
      zeta[s] = fb;
      eta[s] = fv;
    }
    const R vb = w[1] * bn + w[2] * w[4] + w[3] * w[5];
    const R vbs = SM * bn + vs[s] * b1s[s] + ws[s] * b2s[s];
    const R pt = (s == 0) ? ptl : ptr;
    const R Es = (su * U[6] - pt * w[1] + pts * SM + bn * (vb - vbs)) / sm;
    Us[s][0] = rhos[s];
    Us[s][1] = rhos[s] * SM;
    Us[s][2] = rhos[s] * vs[s];
    Us[s][3] = rhos[s] * ws[s];
    Us[s][4] = b1s[s];
    Us[s][5] = b2s[s];
    Us[s][6] = Es;
  }

  // rotational (Alfven) waves
  const R sql = Sqrt(rhos[0]), sqr = Sqrt(rhos[1]);
  const R SLs = SM - Abs(bn) / sql;
  const R SRs = SM + Abs(bn) / sqr;
  const R sgn = (bn > R(0)) ? R(1) : ((bn < R(0)) ? R(-1) : R(0));  // sign(0) = 0

  // double-star state (shared v, w, B_t; energy per side)
  const R isum = R(1) / (sql + sqr);
  const R vss = (sql * vs[0] + sqr * vs[1] + sgn * (b1s[1] - b1s[0])) * isum;
  const R wss = (sql * ws[0] + sqr * ws[1] + sgn * (b2s[1] - b2s[0])) * isum;
  const R b1ss = (sql * b1s[1] + sqr * b1s[0] + sgn * sql * sqr * (vs[1] - vs[0])) * isum;
  const R b2ss = (sql * b2s[1] + sqr * b2s[0] + sgn * sql * sqr * (ws[1] - ws[0])) * isum;
  const R vbss = vss * b1ss + wss * b2ss;
  const R Essl = Us[0][6] - sgn * sql * ((vs[0] * b1s[0] + ws[0] * b2s[0]) - vbss);
  const R Essr = Us[1][6] + sgn * sqr * ((vs[1] * b1s[1] + ws[1] * b2s[1]) - vbss);

  // region: 3 F*_L, 4 F**_L, 5 F**_R, 6 F*_R; ties go to the left (the flux
  // is continuous there)
  const int region = (SLs >= R(0)) ? 3 : (SM >= R(0)) ? 4 : (SRs >= R(0)) ? 5 : 6;
  if (uct_hlld) {
    // the HLLD flux of one transverse field component at this wave
    // structure, as a function of (B_t^L, B_t^R, v_t^L, v_t^R)
    auto bt_flux = [&](R BL, R BR, R vL, R vR) {
      const R FLt = ul * BL - vL * bn, FRt = ur * BR - vR * bn;
      const R BsL = zeta[0] * BL, BsR = zeta[1] * BR;
      const R vsL = vL - eta[0] * BL, vsR = vR - eta[1] * BR;
      const R Bss = (sql * BsR + sqr * BsL + sgn * sql * sqr * (vsR - vsL)) * isum;
      if (region == 3) return FLt + SL * (BsL - BL);
      if (region == 4) return FLt + SL * (BsL - BL) + SLs * (Bss - BsL);
      if (region == 5) return FRt + SR * (BsR - BR) + SRs * (Bss - BsR);
      return FRt + SR * (BsR - BR);
    };
    const R chiL = bt_flux(R(1), R(0), R(0), R(0));
    const R chiR = bt_flux(R(0), R(1), R(0), R(0));
    // om from the coefficient of v_t^L, -B_n om; with B_n = 0 only the F* regions
    // occur and the star side alone carries the flux
    if (bn > R(0) || bn < R(0)) o.om = -bt_flux(R(0), R(0), R(1), R(0)) / bn;
    else o.om = (region == 3) ? R(1) : R(0);
    o.dl = chiL - o.om * ul;
    o.dr = (R(1) - o.om) * ur - chiR;
    o.wt1 = o.om * wl[2] + (R(1) - o.om) * wr[2];
    o.wt2 = o.om * wl[3] + (R(1) - o.om) * wr[3];
  }
  if (region == 3) {                       // F*_L
    for (int q = 0; q < 7; ++q) o.F[q] = FL[q] + SL * (Us[0][q] - UL[q]);
    return;
  }
  if (region == 4) {                       // F**_L
    const R Uss[7] = {rhos[0], rhos[0] * SM, rhos[0] * vss, rhos[0] * wss, b1ss, b2ss, Essl};
    for (int q = 0; q < 7; ++q) {
      const R Fs = FL[q] + SL * (Us[0][q] - UL[q]);
      o.F[q] = Fs + SLs * (Uss[q] - Us[0][q]);
    }
    return;
  }
  if (region == 5) {                       // F**_R
    const R Uss[7] = {rhos[1], rhos[1] * SM, rhos[1] * vss, rhos[1] * wss, b1ss, b2ss, Essr};
    for (int q = 0; q < 7; ++q) {
      const R Fs = FR[q] + SR * (Us[1][q] - UR[q]);
      o.F[q] = Fs + SRs * (Uss[q] - Us[1][q]);
    }
    return;
  }
  for (int q = 0; q < 7; ++q) o.F[q] = FR[q] + SR * (Us[1][q] - UR[q]);  // F*_R
}

// Upwind constrained-transport EMF [reading: an upwind average in the family
// of the UCT schemes the paper cites for CT; the coefficients are the HLL
// wave-speed bounds of the faces touching the edge].
// Edge component c with cyclic pair (a, b): the exact EMF is v_b B_a - v_a B_b.
//  apa/ama: alpha+-, maximised over the two a-faces touching the edge
//  vW,bW / vE,bE: v_a and B_b on the two b-faces, reconstructed along a
//  apb/amb: alpha+-, maximised over the two b-faces touching the edge
//  vS,bS / vN,bN: v_b and B_a on the two a-faces, reconstructed along b
template <class R>
R uct_emf(R apa, R ama, R vW, R bW, R vE, R bE, R apb, R amb, R vS, R bS, R vN, R bN) {
  const R ta = (apa * vW * bW + ama * vE * bE - apa * ama * (bE - bW)) / (apa + ama);
  const R tb = (apb * vS * bS + amb * vN * bN - apb * amb * (bN - bS)) / (apb + amb);
  return tb - ta;
}

// UCT-HLLD edge EMF [reading: the coefficients of the two faces touching the
// edge are averaged]. a-bracket: weights (aa, 1 - aa) and diffusion
// coefficients dla, dra from the a-faces, applied to v_a B_b on the two
// b-faces reconstructed along a (W, E); b-bracket likewise.
template <class R>
R uct_hlld_emf(R aa, R dla, R dra, R vW, R bW, R vE, R bE, R ab, R dlb, R drb, R vS, R bS, R vN,
               R bN) {
  const R ta = aa * vW * bW + (R(1) - aa) * vE * bE - (dra * bE - dla * bW);
  const R tb = ab * vS * bS + (R(1) - ab) * vN * bN - (drb * bN - dlb * bS);
  return tb - ta;
}

// ---------------------------------------------------------------------------
// Right-hand side L(U) of the semi-discrete equations (Eq. FV) for all eight
// stored fields: (rho, m_x, m_y, m_z, E) cell averages and the staggered field
// (b_x, b_y, b_z) on the lower x-, y-, z-faces; in 2D field 7 is a cell-centred
// B_z. Returns 1 if any cell held rho <= 0, p <= 0 or a non-finite value.
template <class S, class R>
int compute_rhs(const OCfg& cfg, const S* U, S* L) {
  const Grid G(cfg);
  const size_t n = G.ncell;
  const int dim = G.dim;
  const S gamma = S(cfg.gamma);
  const R gR = Cast<R>::of(S(cfg.gamma));
  int bad = 0;

  auto F = [&](int f) { return U + (size_t)f * n; };

  g_phase = PH_PRIM;
  // --- primitives (Sec. 2.2 primitive inversion), FP64 in every mode -------
  std::vector<S> V((size_t)NF * n);
  auto Vf = [&](int f) { return V.data() + (size_t)f * n; };
  std::vector<int> badk((size_t)G.nz * G.ny, 0);
  par_rows(G, cfg.nthreads, [&](int j, int k) {
      for (int i = 0; i < G.nx; ++i) {
        const size_t c = G.at(i, j, k);
        const S rho = F(RHO)[c];
        S Bc[3];
        // [reading] cell-centred field = arithmetic mean of the two faces
        Bc[0] = S(0.5) * (F(BX)[c] + F(BX)[G.at(i + 1, j, k)]);
        Bc[1] = S(0.5) * (F(BY)[c] + F(BY)[G.at(i, j + 1, k)]);
        if (dim == 3) Bc[2] = S(0.5) * (F(BZ)[c] + F(BZ)[G.at(i, j, k + 1)]);
        else Bc[2] = F(BZ)[c];
        const S vx = F(MX)[c] / rho, vy = F(MY)[c] / rho, vz = F(MZ)[c] / rho;
        const S kin = S(0.5) * (F(MX)[c] * vx + F(MY)[c] * vy + F(MZ)[c] * vz);
        const S mag = S(0.5) * (Bc[0] * Bc[0] + Bc[1] * Bc[1] + Bc[2] * Bc[2]);
        const S p = (gamma - S(1)) * (F(EN)[c] - kin - mag);
        Vf(VRHO)[c] = rho; Vf(VVX)[c] = vx; Vf(VVY)[c] = vy; Vf(VVZ)[c] = vz;
        Vf(VPR)[c] = p; Vf(VBX)[c] = Bc[0]; Vf(VBY)[c] = Bc[1]; Vf(VBZ)[c] = Bc[2];
        if (!(val(rho) > 0.0) || !(val(p) > 0.0) || !Finite(p) || !Finite(rho) ||
            !Finite(vx) || !Finite(vy) || !Finite(vz))
          badk[(size_t)k * G.ny + j] = 1;
      }
  });
  for (int r : badk) bad |= r;

  g_phase = PH_FACE;
  // --- per direction: reconstruction + Riemann solve at every lower face ---
  // Face arrays: flux of the eight stored components in the global frame
  // (promoted to S), alpha+-, and the HLL-weighted velocity (global comps).
  // With the UCT-HLLD average, Ap/Am hold its weight om and diffusion
  // coefficient d^L, Dr its d^R, and Vt the om-weighted velocities.
  const bool uh = cfg.emf == 1;
  std::vector<S> Fl[3];
  std::vector<R> Ap[3], Am[3], Vt[3], Dr[3];
  for (int d = 0; d < dim; ++d) {
    Fl[d].assign((size_t)NF * n, S(0));
    Ap[d].assign(n, R(0));
    Am[d].assign(n, R(0));
    Vt[d].assign((size_t)3 * n, R(0));
    if (uh) Dr[d].assign(n, R(0));
    const int t1 = t1_of(d), t2 = t2_of(d);
    const int vn = VVX + d, vt1 = VVX + t1, vt2 = VVX + t2;
    const int bt1 = VBX + t1, bt2 = VBX + t2;
    // reconstructed primitive slots in the face frame:
    // (rho, v_n, v_t1, v_t2, B_t1, B_t2, p)
    const int slot[7] = {VRHO, vn, vt1, vt2, bt1, bt2, VPR};
    par_rows(G, cfg.nthreads, [&](int j, int k) {
        for (int i = 0; i < G.nx; ++i) {
          const size_t cm2 = G.shift(i, j, k, d, -2), cm1 = G.shift(i, j, k, d, -1);
          const size_t c0 = G.at(i, j, k), cp1 = G.shift(i, j, k, d, +1);
          const size_t cm3 = G.shift(i, j, k, d, -3), cp2 = G.shift(i, j, k, d, +2);
          R wl[7], wr[7];
          for (int q = 0; q < 7; ++q) {
            const S* P = Vf(slot[q]);
            const R a = Cast<R>::of(P[cm2]), b = Cast<R>::of(P[cm1]);
            const R c = Cast<R>::of(P[c0]), e = Cast<R>::of(P[cp1]);
            // face i-1/2: left state from cell i-1, right state from cell i
            if (cfg.limiter == 2) {
              const R z = Cast<R>::of(P[cm3]), f = Cast<R>::of(P[cp2]);
              wl[q] = wenoz_upper(z, a, b, c, e);
              wr[q] = wenoz_upper(f, e, c, b, a);
            } else {
              wl[q] = b + R(0.5) * limited_slope(cfg.limiter, b - a, c - b);
              wr[q] = c - R(0.5) * limited_slope(cfg.limiter, c - b, e - c);
            }
          }
          const R bn = Cast<R>::of(F(BX + d)[c0]);  // staggered normal field
          RSOut<R> o;
          riemann<R>(cfg.riemann, gR, wl, wr, bn, o, uh);
          S* fl = Fl[d].data();
          fl[(size_t)RHO * n + c0] = Cast<S>::of(o.F[0]);
          fl[(size_t)(MX + d) * n + c0] = Cast<S>::of(o.F[1]);
          fl[(size_t)(MX + t1) * n + c0] = Cast<S>::of(o.F[2]);
          fl[(size_t)(MX + t2) * n + c0] = Cast<S>::of(o.F[3]);
          fl[(size_t)(BX + t1) * n + c0] = Cast<S>::of(o.F[4]);
          fl[(size_t)(BX + t2) * n + c0] = Cast<S>::of(o.F[5]);
          fl[(size_t)EN * n + c0] = Cast<S>::of(o.F[6]);
          fl[(size_t)(BX + d) * n + c0] = S(0);
          if (uh) {
            Ap[d][c0] = o.om;
            Am[d][c0] = o.dl;
            Dr[d][c0] = o.dr;
            Vt[d][(size_t)t1 * n + c0] = o.wt1;
            Vt[d][(size_t)t2 * n + c0] = o.wt2;
          } else {
            Ap[d][c0] = o.ap;
            Am[d][c0] = o.am;
            Vt[d][(size_t)t1 * n + c0] = o.vt1;
            Vt[d][(size_t)t2 * n + c0] = o.vt2;
          }
        }
    });
  }

  g_phase = PH_EMF;
  // --- upwind CT EMF on cell edges -----------------------------------------
  // Edge of component c stored at cell (i,j,k) sits at the lower a- and lower
  // b-position of that cell: E_z at (i-1/2, j-1/2, k), E_x at (i, j-1/2, k-1/2),
  // E_y at (i-1/2, j, k-1/2).
  std::vector<S> Ed[3];
  const int ncomp = (dim == 3) ? 3 : 1;
  for (int ci = 0; ci < ncomp; ++ci) {
    const int c = (dim == 3) ? ci : 2;
    const int a = (c + 1) % 3, b = (c + 2) % 3;  // (x,y)->z, (y,z)->x, (z,x)->y
    Ed[c].assign(n, S(0));
    par_rows(G, cfg.nthreads, [&](int j, int k) {
        for (int i = 0; i < G.nx; ++i) {
          const size_t c0 = G.at(i, j, k);
          // Reconstruct a face quantity X, stored at lower faces, along
          // direction e toward the edge: value from the lower side (upper
          // extrapolation of face c0-e) and from the upper side (lower
          // extrapolation of face c0).
          auto recon = [&](auto get, int e, R& lo, R& hi) {
            const R xm2 = get(G.shift(i, j, k, e, -2));
            const R xm1 = get(G.shift(i, j, k, e, -1));
            const R x0 = get(c0);
            const R xp1 = get(G.shift(i, j, k, e, +1));
            // [reading: with WENO-Z faces, the edge values use van Leer PLM]
            const int el = cfg.limiter == 2 ? 1 : cfg.limiter;
            lo = xm1 + R(0.5) * limited_slope(el, xm1 - xm2, x0 - xm1);
            hi = x0 - R(0.5) * limited_slope(el, x0 - xm1, xp1 - x0);
          };
          // a-faces touching the edge: cells c0 - e_b and c0
          const size_t ca = G.shift(i, j, k, b, -1);
          // b-faces touching the edge: cells c0 - e_a and c0
          const size_t cb = G.shift(i, j, k, a, -1);
          // W/E: on b-faces, v_a and B_b reconstructed along a
          R vW, vE, bW, bE;
          recon([&](size_t q) { return Vt[b][(size_t)a * n + q]; }, a, vW, vE);
          recon([&](size_t q) { return Cast<R>::of(F(BX + b)[q]); }, a, bW, bE);
          // S/N: on a-faces, v_b and B_a reconstructed along b
          R vS, vN, bS, bN;
          recon([&](size_t q) { return Vt[a][(size_t)b * n + q]; }, b, vS, vN);
          recon([&](size_t q) { return Cast<R>::of(F(BX + a)[q]); }, b, bS, bN);
          if (uh) {
            const R aa = R(0.5) * (Ap[a][ca] + Ap[a][c0]);
            const R dla = R(0.5) * (Am[a][ca] + Am[a][c0]);
            const R dra = R(0.5) * (Dr[a][ca] + Dr[a][c0]);
            const R ab = R(0.5) * (Ap[b][cb] + Ap[b][c0]);
            const R dlb = R(0.5) * (Am[b][cb] + Am[b][c0]);
            const R drb = R(0.5) * (Dr[b][cb] + Dr[b][c0]);
            Ed[c][c0] = Cast<S>::of(
                uct_hlld_emf<R>(aa, dla, dra, vW, bW, vE, bE, ab, dlb, drb, vS, bS, vN, bN));
          } else {
            const R apa = Max(Ap[a][ca], Ap[a][c0]);
            const R ama = Max(Am[a][ca], Am[a][c0]);
            const R apb = Max(Ap[b][cb], Ap[b][c0]);
            const R amb = Max(Am[b][cb], Am[b][c0]);
            Ed[c][c0] =
                Cast<S>::of(uct_emf<R>(apa, ama, vW, bW, vE, bE, apb, amb, vS, bS, vN, bN));
          }
        }
    });
  }

  g_phase = PH_UPDATE;
  // --- flux-divergence update of cell fields; curl update of face fields ---
  par_rows(G, cfg.nthreads, [&](int j, int k) {
      for (int i = 0; i < G.nx; ++i) {
        const size_t c0 = G.at(i, j, k);
        const size_t xp = G.at(i + 1, j, k), yp = G.at(i, j + 1, k), zp = G.at(i, j, k + 1);
        // cell-averaged fields: -(dF/dx + dG/dy [+ dH/dz]), summed x, y, z
        const int cells2d[6] = {RHO, MX, MY, MZ, EN, BZ};
        const int ncf = (dim == 3) ? 5 : 6;
        for (int qq = 0; qq < ncf; ++qq) {
          const int q = cells2d[qq];
          const S* fx = Fl[0].data() + (size_t)q * n;
          const S* fy = Fl[1].data() + (size_t)q * n;
          S acc = (fx[xp] - fx[c0]) / S(G.dx) + (fy[yp] - fy[c0]) / S(G.dy);
          if (dim == 3) {
            const S* fz = Fl[2].data() + (size_t)q * n;
            acc = acc + (fz[zp] - fz[c0]) / S(G.dz);
          }
          L[(size_t)q * n + c0] = -acc;
        }
        // face fields: dB/dt = -curl E (Stokes on each face)
        if (dim == 3) {
          const S* Ex = Ed[0].data();
          const S* Ey = Ed[1].data();
          const S* Ez = Ed[2].data();
          L[(size_t)BX * n + c0] = -((Ez[yp] - Ez[c0]) / S(G.dy) - (Ey[zp] - Ey[c0]) / S(G.dz));
          L[(size_t)BY * n + c0] = -((Ex[zp] - Ex[c0]) / S(G.dz) - (Ez[xp] - Ez[c0]) / S(G.dx));
          L[(size_t)BZ * n + c0] = -((Ey[xp] - Ey[c0]) / S(G.dx) - (Ex[yp] - Ex[c0]) / S(G.dy));
        } else {
          const S* Ez = Ed[2].data();
          L[(size_t)BX * n + c0] = -((Ez[yp] - Ez[c0]) / S(G.dy));
          L[(size_t)BY * n + c0] = (Ez[xp] - Ez[c0]) / S(G.dx);
        }
      }
  });
  return bad;
}

template <class S, class R>
int rhs_dispatch(const OCfg& cfg, const S* U, S* L);

template <>
int rhs_dispatch<double, double>(const OCfg& cfg, const double* U, double* L) {
  if (cfg.precision == 1) return compute_rhs<double, float>(cfg, U, L);
  return compute_rhs<double, double>(cfg, U, L);
}

// SSP-RK2 [reading: the two-stage member of the Shu-Osher family cited with
// Eq. (RK3)]: U1 = Un + dt L(Un); Un+1 = (Un + (U1 + dt L(U1))) / 2.
template <class S, class RhsFn>
int rk2_step(const OCfg& cfg, S* U, S dt, RhsFn rhs) {
  const Grid G(cfg);
  const size_t N = (size_t)NF * G.ncell;
  std::vector<S> L(N), U1(N);
  int bad = rhs(U, L.data());
  for (size_t q = 0; q < N; ++q) U1[q] = U[q] + dt * L[q];
  bad |= rhs(U1.data(), L.data());
  for (size_t q = 0; q < N; ++q) U[q] = S(0.5) * (U[q] + (U1[q] + dt * L[q]));
  return bad;
}

// SSP-RK3 of Shu & Osher, Sec. 2.2 Eq. (RK3) [reading: the printed last stage
// adds L** once where the scheme's third order needs it twice; L = dt times
// the right-hand side]: U* = Un + dt L(Un);
// U** = (3 Un + (U* + dt L(U*))) / 4;  Un+1 = (Un + 2 (U** + dt L(U**))) / 3.
template <class S, class RhsFn>
int rk3_step(const OCfg& cfg, S* U, S dt, RhsFn rhs) {
  const Grid G(cfg);
  const size_t N = (size_t)NF * G.ncell;
  std::vector<S> L(N), U1(N), U2(N);
  int bad = rhs(U, L.data());
  for (size_t q = 0; q < N; ++q) U1[q] = U[q] + dt * L[q];
  bad |= rhs(U1.data(), L.data());
  for (size_t q = 0; q < N; ++q) U2[q] = (S(3) * U[q] + (U1[q] + dt * L[q])) / S(4);
  bad |= rhs(U2.data(), L.data());
  for (size_t q = 0; q < N; ++q) U[q] = (U[q] + S(2) * (U2[q] + dt * L[q])) / S(3);
  return bad;
}

// One step with the configured integrator.
template <class S, class RhsFn>
int ssp_step(const OCfg& cfg, S* U, S dt, RhsFn rhs) {
  return cfg.integrator == 1 ? rk3_step<S>(cfg, U, dt, rhs) : rk2_step<S>(cfg, U, dt, rhs);
}

// CFL time step [reading: the paper gives no formula]:
// dt = C min over cells and directions of Delta_d / (|v_d| + c_f,d).
int cfl_dt(const OCfg& cfg, const double* U, double* dt_out) {
  const Grid G(cfg);
  const size_t n = G.ncell;
  const double g = cfg.gamma;
  const size_t nrow = (size_t)G.nz * G.ny;
  std::vector<double> kmin(nrow, INFINITY);
  std::vector<int> kbad(nrow, 0);
  par_rows(G, cfg.nthreads, [&](int j, int k) {
    double m = INFINITY;
    const size_t r = (size_t)k * G.ny + j;
      for (int i = 0; i < G.nx; ++i) {
        const size_t c = G.at(i, j, k);
        const double rho = U[c];
        double Bc[3];
        Bc[0] = 0.5 * (U[BX * n + c] + U[BX * n + G.at(i + 1, j, k)]);
        Bc[1] = 0.5 * (U[BY * n + c] + U[BY * n + G.at(i, j + 1, k)]);
        Bc[2] = (G.dim == 3) ? 0.5 * (U[BZ * n + c] + U[BZ * n + G.at(i, j, k + 1)]) : U[BZ * n + c];
        const double v[3] = {U[MX * n + c] / rho, U[MY * n + c] / rho, U[MZ * n + c] / rho};
        const double kin = 0.5 * (U[MX * n + c] * v[0] + U[MY * n + c] * v[1] + U[MZ * n + c] * v[2]);
        const double mag = 0.5 * (Bc[0] * Bc[0] + Bc[1] * Bc[1] + Bc[2] * Bc[2]);
        const double p = (g - 1.0) * (U[EN * n + c] - kin - mag);
        if (!(rho > 0.0) || !(p > 0.0) || !std::isfinite(p)) kbad[r] = 1;
        for (int d = 0; d < G.dim; ++d) {
          const double cf = fast_speed<double>(g, rho, p, Bc[d], Bc[(d + 1) % 3], Bc[(d + 2) % 3]);
          const double lam = std::fabs(v[d]) + cf;
          const double t = G.delta(d) / lam;
          if (t < m) m = t;
        }
      }
    kmin[r] = m;
  });
  double m = INFINITY;
  int bad = 0;
  for (size_t r = 0; r < nrow; ++r) { m = std::min(m, kmin[r]); bad |= kbad[r]; }
  *dt_out = cfg.cfl * m;
  return bad;
}

// ---------------------------------------------------------------------------
// GLM divergence cleaning (Sec. 2.1 lists it beside CT as the control of div B;
// Dedner et al. 2002) [reading: the mixed GLM form, with the energy equation
// left as in Eq. (Energy)]. Nine cell-centred fields (rho, m, E, B, psi):
//   dB/dt + div(vB - Bv) + grad psi = 0,
//   dpsi/dt + c_h^2 div B = -(c_h^2 / c_p^2) psi,
// the hyperbolic part in the finite-volume form of Eq. (FV) and the damping
// applied after each full step as psi <- psi exp(-alpha c_h dt / Delta_min).
// c_h = C Delta_min / dt: the largest speed the step's dt allows [reading];
// alpha = 0.1 [reading].
constexpr int NG = 9;
enum { PSI = 8 };
constexpr double kGlmAlpha = 0.1;

// The (B_n, psi) subsystem decouples from the rest at a face; its exact
// Riemann solution gives the interface values bn_s, psi_s, whose fluxes are
// psi_s (for B_n) and c_h^2 bn_s (for psi); the rest of the face is the MHD
// Riemann problem with the normal field bn_s on both sides.
template <class R>
void glm_face(int solver, R g, const R wl[7], const R wr[7], R bnl, R bnr, R psil, R psir, R ch,
              R F[9]) {
  const R bn_s = R(0.5) * (bnl + bnr) - (psir - psil) / (R(2) * ch);
  const R psi_s = R(0.5) * (psil + psir) - R(0.5) * ch * (bnr - bnl);
  RSOut<R> o;
  riemann<R>(solver, g, wl, wr, bn_s, o);
  for (int q = 0; q < 7; ++q) F[q] = o.F[q];
  F[7] = psi_s;
  F[8] = ch * ch * bn_s;
}

template <class S, class R>
int compute_rhs_glm(const OCfg& cfg, const S* U, S* L, double ch) {
  const Grid G(cfg);
  const size_t n = G.ncell;
  const int dim = G.dim;
  const S gamma = S(cfg.gamma);
  const R gR = Cast<R>::of(S(cfg.gamma));
  auto F = [&](int f) { return U + (size_t)f * n; };
  // primitives (rho, v, p, B, psi), FP64
  std::vector<S> V((size_t)NG * n);
  auto Vf = [&](int f) { return V.data() + (size_t)f * n; };
  std::vector<int> badk((size_t)G.nz * G.ny, 0);
  par_rows(G, cfg.nthreads, [&](int j, int k) {
      for (int i = 0; i < G.nx; ++i) {
        const size_t c = G.at(i, j, k);
        const S rho = F(RHO)[c];
        const S vx = F(MX)[c] / rho, vy = F(MY)[c] / rho, vz = F(MZ)[c] / rho;
        const S kin = S(0.5) * (F(MX)[c] * vx + F(MY)[c] * vy + F(MZ)[c] * vz);
        const S mag = S(0.5) * (F(BX)[c] * F(BX)[c] + F(BY)[c] * F(BY)[c] + F(BZ)[c] * F(BZ)[c]);
        const S p = (gamma - S(1)) * (F(EN)[c] - kin - mag);
        Vf(VRHO)[c] = rho; Vf(VVX)[c] = vx; Vf(VVY)[c] = vy; Vf(VVZ)[c] = vz; Vf(VPR)[c] = p;
        Vf(VBX)[c] = F(BX)[c]; Vf(VBY)[c] = F(BY)[c]; Vf(VBZ)[c] = F(BZ)[c];
        Vf(PSI)[c] = F(PSI)[c];
        if (!(val(rho) > 0.0) || !(val(p) > 0.0) || !Finite(p) || !Finite(rho) ||
            !Finite(vx) || !Finite(vy) || !Finite(vz))
          badk[(size_t)k * G.ny + j] = 1;
      }
  });
  int bad = 0;
  for (int r : badk) bad |= r;
  // fluxes of the nine fields through every lower face, global components
  std::vector<S> Fl[3];
  const R chR = Cast<R>::of(S(ch));
  for (int d = 0; d < dim; ++d) {
    Fl[d].assign((size_t)NG * n, S(0));
    const int t1 = t1_of(d), t2 = t2_of(d);
    // face frame (rho, v_n, v_t1, v_t2, B_t1, B_t2, p), then B_n and psi
    const int slot[9] = {VRHO, VVX + d, VVX + t1, VVX + t2, VBX + t1, VBX + t2, VPR, VBX + d, PSI};
    par_rows(G, cfg.nthreads, [&](int j, int k) {
        for (int i = 0; i < G.nx; ++i) {
          const size_t cm2 = G.shift(i, j, k, d, -2), cm1 = G.shift(i, j, k, d, -1);
          const size_t c0 = G.at(i, j, k), cp1 = G.shift(i, j, k, d, +1);
          const size_t cm3 = G.shift(i, j, k, d, -3), cp2 = G.shift(i, j, k, d, +2);
          R wl[9], wr[9];
          for (int q = 0; q < 9; ++q) {
            const S* P = Vf(slot[q]);
            const R a = Cast<R>::of(P[cm2]), b = Cast<R>::of(P[cm1]);
            const R c = Cast<R>::of(P[c0]), e = Cast<R>::of(P[cp1]);
            if (cfg.limiter == 2) {
              const R z = Cast<R>::of(P[cm3]), f = Cast<R>::of(P[cp2]);
              wl[q] = wenoz_upper(z, a, b, c, e);
              wr[q] = wenoz_upper(f, e, c, b, a);
            } else {
              wl[q] = b + R(0.5) * limited_slope(cfg.limiter, b - a, c - b);
              wr[q] = c - R(0.5) * limited_slope(cfg.limiter, c - b, e - c);
            }
          }
          R Ff[9];
          glm_face<R>(cfg.riemann, gR, wl, wr, wl[7], wr[7], wl[8], wr[8], chR, Ff);
          S* fl = Fl[d].data();
          fl[(size_t)RHO * n + c0] = Cast<S>::of(Ff[0]);
          fl[(size_t)(MX + d) * n + c0] = Cast<S>::of(Ff[1]);
          fl[(size_t)(MX + t1) * n + c0] = Cast<S>::of(Ff[2]);
          fl[(size_t)(MX + t2) * n + c0] = Cast<S>::of(Ff[3]);
          fl[(size_t)(BX + t1) * n + c0] = Cast<S>::of(Ff[4]);
          fl[(size_t)(BX + t2) * n + c0] = Cast<S>::of(Ff[5]);
          fl[(size_t)EN * n + c0] = Cast<S>::of(Ff[6]);
          fl[(size_t)(BX + d) * n + c0] = Cast<S>::of(Ff[7]);
          fl[(size_t)PSI * n + c0] = Cast<S>::of(Ff[8]);
        }
    });
  }
  // flux divergence of all nine fields
  par_rows(G, cfg.nthreads, [&](int j, int k) {
      for (int i = 0; i < G.nx; ++i) {
        const size_t c0 = G.at(i, j, k);
        const size_t xp = G.at(i + 1, j, k), yp = G.at(i, j + 1, k), zp = G.at(i, j, k + 1);
        for (int q = 0; q < NG; ++q) {
          const S* fx = Fl[0].data() + (size_t)q * n;
          const S* fy = Fl[1].data() + (size_t)q * n;
          S acc = (fx[xp] - fx[c0]) / S(G.dx) + (fy[yp] - fy[c0]) / S(G.dy);
          if (dim == 3) {
            const S* fz = Fl[2].data() + (size_t)q * n;
            acc = acc + (fz[zp] - fz[c0]) / S(G.dz);
          }
          L[(size_t)q * n + c0] = -acc;
        }
      }
  });
  return bad;
}

double glm_dmin(const Grid& G) {
  double m = std::min(G.dx, G.dy);
  return G.dim == 3 ? std::min(m, G.dz) : m;
}

// One step of the configured integrator on the nine GLM fields, then the damping.
int glm_step(const OCfg& cfg, double* U, double dt) {
  const Grid G(cfg);
  const size_t N = (size_t)NG * G.ncell;
  const double dmin = glm_dmin(G);
  const double ch = cfg.cfl * dmin / dt;
  auto rhs = [&](const double* u, double* l) {
    if (cfg.precision == 1) return compute_rhs_glm<double, float>(cfg, u, l, ch);
    return compute_rhs_glm<double, double>(cfg, u, l, ch);
  };
  std::vector<double> L(N), U1(N);
  int bad = rhs(U, L.data());
  for (size_t q = 0; q < N; ++q) U1[q] = U[q] + dt * L[q];
  bad |= rhs(U1.data(), L.data());
  if (cfg.integrator == 1) {
    std::vector<double> U2(N);
    for (size_t q = 0; q < N; ++q) U2[q] = (3.0 * U[q] + (U1[q] + dt * L[q])) / 4.0;
    bad |= rhs(U2.data(), L.data());
    for (size_t q = 0; q < N; ++q) U[q] = (U[q] + 2.0 * (U2[q] + dt * L[q])) / 3.0;
  } else {
    for (size_t q = 0; q < N; ++q) U[q] = 0.5 * (U[q] + (U1[q] + dt * L[q]));
  }
  const double decay = std::exp(-kGlmAlpha * ch * dt / dmin);
  double* psi = U + (size_t)PSI * G.ncell;
  for (size_t c = 0; c < G.ncell; ++c) psi[c] = psi[c] * decay;
  return bad;
}

// CFL time step of a GLM state (cell-centred B), same formula as cfl_dt.
int glm_cfl_dt(const OCfg& cfg, const double* U, double* dt_out) {
  const Grid G(cfg);
  const size_t n = G.ncell;
  const double g = cfg.gamma;
  double m = INFINITY;
  int bad = 0;
  for (size_t c = 0; c < n; ++c) {
    const double rho = U[c];
    const double B[3] = {U[BX * n + c], U[BY * n + c], U[BZ * n + c]};
    const double v[3] = {U[MX * n + c] / rho, U[MY * n + c] / rho, U[MZ * n + c] / rho};
    const double kin = 0.5 * (U[MX * n + c] * v[0] + U[MY * n + c] * v[1] + U[MZ * n + c] * v[2]);
    const double mag = 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const double p = (g - 1.0) * (U[EN * n + c] - kin - mag);
    if (!(rho > 0.0) || !(p > 0.0) || !std::isfinite(p)) bad = 1;
    for (int d = 0; d < G.dim; ++d) {
      const double cf = fast_speed<double>(g, rho, p, B[d], B[(d + 1) % 3], B[(d + 2) % 3]);
      const double t = G.delta(d) / (std::fabs(v[d]) + cf);
      if (t < m) m = t;
    }
  }
  *dt_out = cfg.cfl * m;
  return bad;
}

bool cfg_ok(const OCfg* c) {
  if (!c) return false;
  if (c->dim != 2 && c->dim != 3) return false;
  if (c->nx < 4 || c->ny < 4) return false;
  if (c->dim == 3 && c->nz < 4) return false;
  if (c->dim == 2 && c->nz != 1) return false;
  if (!(c->gamma > 1.0) || !(c->cfl > 0.0)) return false;
  if (c->limiter < 0 || c->limiter > 2 || c->riemann < 0 || c->riemann > 1) return false;
  if (c->precision < 0 || c->precision > 1) return false;
  if (c->integrator < 0 || c->integrator > 1) return false;
  if (c->emf < 0 || c->emf > 1) return false;
  if (!(c->xmax > c->xmin) || !(c->ymax > c->ymin) || !(c->zmax > c->zmin)) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface. Return codes: 0 ok, -1 invalid argument, -4 unphysical state
// met (rho <= 0, p <= 0 or non-finite; the computation still completes).
extern "C" {

int oracle_rhs(const OCfg* cfg, const double* U, double* L) {
  if (!cfg_ok(cfg) || !U || !L) return -1;
  return rhs_dispatch<double, double>(*cfg, U, L) ? -4 : 0;
}

int oracle_step(const OCfg* cfg, double* U, double dt) {
  if (!cfg_ok(cfg) || !U || !(dt > 0.0) || !std::isfinite(dt)) return -1;
  int bad = ssp_step<double>(*cfg, U, dt, [&](const double* u, double* l) {
    return rhs_dispatch<double, double>(*cfg, u, l);
  });
  return bad ? -4 : 0;
}

int oracle_dt(const OCfg* cfg, const double* U, double* dt) {
  if (!cfg_ok(cfg) || !U || !dt) return -1;
  return cfl_dt(*cfg, U, dt) ? -4 : 0;
}

// n steps, each with dt from the CFL condition of the state at its start.
// dts (nullable) receives the n time steps used.
int oracle_run(const OCfg* cfg, double* U, int nsteps, double* dts) {
  if (!cfg_ok(cfg) || !U || nsteps < 0) return -1;
  int bad = 0;
  for (int s = 0; s < nsteps; ++s) {
    double dt;
    bad |= cfl_dt(*cfg, U, &dt);
    if (dts) dts[s] = dt;
    bad |= ssp_step<double>(*cfg, U, dt, [&](const double* u, double* l) {
      return rhs_dispatch<double, double>(*cfg, u, l);
    });
  }
  return bad ? -4 : 0;
}

// n steps with a prescribed dt sequence.
int oracle_run_dts(const OCfg* cfg, double* U, int nsteps, const double* dts) {
  if (!cfg_ok(cfg) || !U || nsteps < 0 || !dts) return -1;
  int bad = 0;
  for (int s = 0; s < nsteps; ++s) {
    bad |= ssp_step<double>(*cfg, U, dts[s], [&](const double* u, double* l) {
      return rhs_dispatch<double, double>(*cfg, u, l);
    });
  }
  return bad ? -4 : 0;
}

// How often the HLLD star state is taken as degenerate in one right-hand
// side of U, in FP64 and in the mixed (FP32) variant: out = {FP64 sides,
// FP64 degenerate sides, FP32 sides, FP32 degenerate sides}.
int oracle_count_degenerate(const OCfg* cfg, const double* U, long long* out) {
  if (!cfg_ok(cfg) || !U || !out) return -1;
  const Grid G(*cfg);
  std::vector<double> L((size_t)NF * G.ncell);
  g_count_deg = true;
  for (int p = 0; p < 2; ++p) {
    OCfg c = *cfg;
    c.precision = p;
    g_deg_sides[p] = g_deg_hits[p] = 0;
    rhs_dispatch<double, double>(c, U, L.data());
    out[2 * p] = g_deg_sides[p];
    out[2 * p + 1] = g_deg_hits[p];
  }
  g_count_deg = false;
  return 0;
}

// GLM divergence cleaning: nine cell-centred fields (rho, m, E, B, psi).
int oracle_glm_dt(const OCfg* cfg, const double* U, double* dt) {
  if (!cfg_ok(cfg) || !U || !dt) return -1;
  return glm_cfl_dt(*cfg, U, dt) ? -4 : 0;
}

int oracle_glm_run_dts(const OCfg* cfg, double* U, int nsteps, const double* dts) {
  if (!cfg_ok(cfg) || !U || nsteps < 0 || !dts) return -1;
  int bad = 0;
  for (int s = 0; s < nsteps; ++s) bad |= glm_step(*cfg, U, dts[s]);
  return bad ? -4 : 0;
}

int oracle_glm_run(const OCfg* cfg, double* U, int nsteps, double* dts) {
  if (!cfg_ok(cfg) || !U || nsteps < 0) return -1;
  int bad = 0;
  for (int s = 0; s < nsteps; ++s) {
    double dt;
    bad |= glm_cfl_dt(*cfg, U, &dt);
    if (dts) dts[s] = dt;
    bad |= glm_step(*cfg, U, dt);
  }
  return bad ? -4 : 0;
}

// Right-hand side of the GLM system for a given c_h (no damping).
int oracle_glm_rhs(const OCfg* cfg, const double* U, double* L, double ch) {
  if (!cfg_ok(cfg) || !U || !L || !(ch > 0.0)) return -1;
  const int bad = cfg->precision == 1 ? compute_rhs_glm<double, float>(*cfg, U, L, ch)
                                      : compute_rhs_glm<double, double>(*cfg, U, L, ch);
  return bad ? -4 : 0;
}

// One GLM face: out[9] = fluxes of (rho, m_n, m_t1, m_t2, B_t1, B_t2, E, B_n, psi).
int oracle_glm_face(int solver, double gamma, const double* wl, const double* wr, double bnl,
                    double bnr, double psil, double psir, double ch, double* out) {
  if (!wl || !wr || !out || !(gamma > 1.0) || !(ch > 0.0) || solver < 0 || solver > 1) return -1;
  glm_face<double>(solver, gamma, wl, wr, bnl, bnr, psil, psir, ch, out);
  return 0;
}

// Forward-mode tangent of one step (FP64 only): on return U holds the new
// state and dU the directional derivative of the step along (dU, ddt).
int oracle_step_jvp(const OCfg* cfg, double* U, double* dU, double dt, double ddt) {
  if (!cfg_ok(cfg) || !U || !dU || !(dt > 0.0)) return -1;
  OCfg c = *cfg;
  c.precision = 0;
  const Grid G(c);
  const size_t N = (size_t)NF * G.ncell;
  std::vector<Dual> Ud(N);
  for (size_t q = 0; q < N; ++q) Ud[q] = Dual(U[q], dU[q]);
  int bad = ssp_step<Dual>(c, Ud.data(), Dual(dt, ddt), [&](const Dual* u, Dual* l) {
    return compute_rhs<Dual, Dual>(c, u, l);
  });
  for (size_t q = 0; q < N; ++q) { U[q] = Ud[q].v; dU[q] = Ud[q].d; }
  return bad ? -4 : 0;
}

// Floating-point operations of one right-hand side evaluation, single
// threaded, per phase: out[4*phase + kind], kind = add/sub, mul, div, sqrt;
// phases: primitives, faces (reconstruction + Riemann), EMF, update.
int oracle_count_ops(const OCfg* cfg, const double* U, long long* out) {
  if (!cfg_ok(cfg) || !U || !out) return -1;
  OCfg c = *cfg;
  c.nthreads = 1;
  c.precision = 0;
  const Grid G(c);
  const size_t N = (size_t)NF * G.ncell;
  std::vector<Cnt> Uc(N), Lc(N);
  for (size_t q = 0; q < N; ++q) Uc[q] = Cnt(U[q]);
  for (int p = 0; p < PH_N; ++p)
    for (int k = 0; k < 4; ++k) g_ops[p][k] = 0;
  int bad = compute_rhs<Cnt, Cnt>(c, Uc.data(), Lc.data());
  for (int p = 0; p < PH_N; ++p)
    for (int k = 0; k < 4; ++k) out[4 * p + k] = g_ops[p][k];
  return bad ? -4 : 0;
}

// Discrete divergence of the staggered field at every cell.
int oracle_divb(const OCfg* cfg, const double* U, double* div) {
  if (!cfg_ok(cfg) || !U || !div) return -1;
  const Grid G(*cfg);
  const size_t n = G.ncell;
  for (int k = 0; k < G.nz; ++k)
    for (int j = 0; j < G.ny; ++j)
      for (int i = 0; i < G.nx; ++i) {
        const size_t c = G.at(i, j, k);
        double s = (U[BX * n + G.at(i + 1, j, k)] - U[BX * n + c]) / G.dx +
                   (U[BY * n + G.at(i, j + 1, k)] - U[BY * n + c]) / G.dy;
        if (G.dim == 3) s += (U[BZ * n + G.at(i, j, k + 1)] - U[BZ * n + c]) / G.dz;
        div[c] = s;
      }
  return 0;
}

// Primitive recovery at every cell: V = (rho, vx, vy, vz, p, Bcx, Bcy, Bcz).
int oracle_prim(const OCfg* cfg, const double* U, double* V) {
  if (!cfg_ok(cfg) || !U || !V) return -1;
  const Grid G(*cfg);
  const size_t n = G.ncell;
  int bad = 0;
  for (int k = 0; k < G.nz; ++k)
    for (int j = 0; j < G.ny; ++j)
      for (int i = 0; i < G.nx; ++i) {
        const size_t c = G.at(i, j, k);
        const double rho = U[c];
        const double Bx = 0.5 * (U[BX * n + c] + U[BX * n + G.at(i + 1, j, k)]);
        const double By = 0.5 * (U[BY * n + c] + U[BY * n + G.at(i, j + 1, k)]);
        const double Bz = (G.dim == 3) ? 0.5 * (U[BZ * n + c] + U[BZ * n + G.at(i, j, k + 1)]) : U[BZ * n + c];
        const double vx = U[MX * n + c] / rho, vy = U[MY * n + c] / rho, vz = U[MZ * n + c] / rho;
        const double kin = 0.5 * (U[MX * n + c] * vx + U[MY * n + c] * vy + U[MZ * n + c] * vz);
        const double mag = 0.5 * (Bx * Bx + By * By + Bz * Bz);
        const double p = (cfg->gamma - 1.0) * (U[EN * n + c] - kin - mag);
        V[0 * n + c] = rho; V[1 * n + c] = vx; V[2 * n + c] = vy; V[3 * n + c] = vz;
        V[4 * n + c] = p; V[5 * n + c] = Bx; V[6 * n + c] = By; V[7 * n + c] = Bz;
        if (!(rho > 0.0) || !(p > 0.0)) bad = 1;
      }
  return bad ? -4 : 0;
}

// A single Riemann problem in the face frame, for unit tests.
// w = (rho, u, v, w, B_t1, B_t2, p). out[11] = F[7], alpha+, alpha-, vt1, vt2.
// precision 1 evaluates it in FP32.
int oracle_riemann(int solver, int precision, double gamma, const double* wl,
                   const double* wr, double bn, double* out) {
  if (!wl || !wr || !out || !(gamma > 1.0) || solver < 0 || solver > 1) return -1;
  if (precision == 1) {
    float l[7], r[7];
    for (int q = 0; q < 7; ++q) { l[q] = (float)wl[q]; r[q] = (float)wr[q]; }
    RSOut<float> o;
    riemann<float>(solver, (float)gamma, l, r, (float)bn, o, true);
    for (int q = 0; q < 7; ++q) out[q] = o.F[q];
    out[7] = o.ap; out[8] = o.am; out[9] = o.vt1; out[10] = o.vt2;
    out[11] = o.om; out[12] = o.dl; out[13] = o.dr; out[14] = o.wt1; out[15] = o.wt2;
    return 0;
  }
  RSOut<double> o;
  riemann<double>(solver, gamma, wl, wr, bn, o, true);
  for (int q = 0; q < 7; ++q) out[q] = o.F[q];
  out[7] = o.ap; out[8] = o.am; out[9] = o.vt1; out[10] = o.vt2;
  out[11] = o.om; out[12] = o.dl; out[13] = o.dr; out[14] = o.wt1; out[15] = o.wt2;
  return 0;
}

// Physical flux of a primitive state in the face frame (for unit tests).
int oracle_flux(double gamma, const double* w, double bn, double* U7, double* F7) {
  if (!w || !U7 || !F7) return -1;
  double pt;
  state_of<double>(gamma, w, bn, U7, F7, pt);
  return 0;
}

double oracle_slope(int limiter, double dm, double dp) {
  return limited_slope<double>(limiter, dm, dp);
}

// WENO-Z upper-interface value of the middle of five cell values (for unit tests).
double oracle_wenoz(const double* v) { return wenoz_upper<double>(v[0], v[1], v[2], v[3], v[4]); }

double oracle_fast_speed(double gamma, double rho, double p, double bn, double bt1, double bt2) {
  return fast_speed<double>(gamma, rho, p, bn, bt1, bt2);
}

double oracle_uct(const double* a12) {
  return uct_emf<double>(a12[0], a12[1], a12[2], a12[3], a12[4], a12[5], a12[6], a12[7],
                         a12[8], a12[9], a12[10], a12[11]);
}

}  // extern "C"
