// Index helpers and primitive recovery shared by the forward and adjoint
// kernels (periodic Cartesian grid, field-major SoA, x fastest).
#pragma once
#include "mhd_device.hpp"

namespace mhd {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ int64_t lin(const Geom& g, int i, int j, int k) {
  return ((int64_t)k * g.ny + j) * g.nx + i;
}

__device__ __forceinline__ void coords(const Geom& g, int64_t c, int& i, int& j, int& k) {
  i = (int)(c % g.nx);
  const int64_t r = c / g.nx;
  j = (int)(r % g.ny);
  k = (int)(r / g.ny);
}

// Cell shifted by s (|s| <= 2) along direction D, periodic.
template <int D>
__device__ __forceinline__ int64_t shifted(const Geom& g, int i, int j, int k, int s) {
  if (D == 0) return lin(g, wrap(i + s, g.nx), j, k);
  if (D == 1) return lin(g, i, wrap(j + s, g.ny), k);
  return lin(g, i, j, wrap(k + s, g.nz));
}

// The stored values primitive recovery at a cell reads: its 8 fields and
// the staggered field on its three upper faces.
struct RawCell {
  double u[8];
  double bxp, byp, bzp;
};

template <int DIM>
__device__ __forceinline__ RawCell load_raw(const double* __restrict__ U, const Geom& g, int i,
                                            int j, int k) {
  const int64_t n = g.n;
  const int64_t c = lin(g, i, j, k);
  RawCell r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r.u[q] = U[q * n + c];
  r.bxp = U[5 * n + lin(g, wrap(i + 1, g.nx), j, k)];
  r.byp = U[6 * n + lin(g, i, wrap(j + 1, g.ny), k)];
  r.bzp = (DIM == 3) ? U[7 * n + lin(g, i, j, wrap(k + 1, g.nz))] : 0.0;
  return r;
}

// Primitive recovery (always FP64): V = (rho, vx, vy, vz, p, Bx, By, Bz), B
// cell-centred as the mean of the two faces (2D: field 7 is already
// cell-centred). Returns false for an unphysical cell.
template <int DIM>
__device__ __forceinline__ bool prim_from_raw(const RawCell& r, double gamma, double* V) {
  const double rho = r.u[0];
  const double mx = r.u[1], my = r.u[2], mz = r.u[3], en = r.u[4];
  const double bx = 0.5 * (r.u[5] + r.bxp);
  const double by = 0.5 * (r.u[6] + r.byp);
  const double bz = (DIM == 3) ? 0.5 * (r.u[7] + r.bzp) : r.u[7];
  const double irho = 1.0 / rho;
  const double vx = mx * irho, vy = my * irho, vz = mz * irho;
  const double kin = 0.5 * fma_r(mz, vz, fma_r(my, vy, mx * vx));
  const double mag = 0.5 * fma_r(bz, bz, fma_r(by, by, bx * bx));
  const double p = (gamma - 1.0) * (en - kin - mag);
  V[0] = rho; V[1] = vx; V[2] = vy; V[3] = vz; V[4] = p; V[5] = bx; V[6] = by; V[7] = bz;
  return (rho > 0.0) && (p > 0.0) && __builtin_isfinite(p) && __builtin_isfinite(vx) &&
         __builtin_isfinite(vy) && __builtin_isfinite(vz);
}

// Primitive recovery at cell (i,j,k).
template <int DIM>
__device__ __forceinline__ bool prim_at(const double* __restrict__ U, const Geom& g, int i, int j,
                                        int k, double* V) {
  return prim_from_raw<DIM>(load_raw<DIM>(U, g, i, j, k), g.gamma, V);
}

// Reconstructed face-frame states of the lower D-face of cell (i,j,k):
// w = (rho, v_n, v_t1, v_t2, B_t1, B_t2, p) from PLM over cells c-2..c+1
// along D, and the staggered normal field bn (FP64).
template <int DIM, int D, int LIM>
__device__ __forceinline__ void face_inputs(const double* __restrict__ U, const Geom& g, int i,
                                            int j, int k, double* wl, double* wr, double& bn) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  double V[4][8];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int o = s - 2;
    prim_at<DIM>(U, g, D == 0 ? wrap(i + o, g.nx) : i, D == 1 ? wrap(j + o, g.ny) : j,
                 D == 2 ? wrap(k + o, g.nz) : k, V[s]);
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int s = slot[q];
    const double a = V[0][s], b = V[1][s], c = V[2][s], e = V[3][s];
    wl[q] = fma_r(0.5, plm_slope<LIM, double>(b - a, c - b), b);
    wr[q] = fma_r(-0.5, plm_slope<LIM, double>(c - b, e - c), c);
  }
  bn = U[(F_BX + D) * g.n + lin(g, i, j, k)];
}

// Partial derivatives (d slope/d dm, d slope/d dp) of the limited slope.
template <int LIM>
__device__ __forceinline__ void plm_slope_grad(double dm, double dp, double& s1, double& s2) {
  const bool ext = dm * dp <= 0.0;
  if (LIM == 0) {
    const bool left = __builtin_fabs(dm) <= __builtin_fabs(dp);
    s1 = (ext || !left) ? 0.0 : 1.0;
    s2 = (ext || left) ? 0.0 : 1.0;
  } else {
    // branch-free: at extrema (where dm + dp may vanish) the select drops the
    // value of the refined reciprocal
    const double is = rcp_r(dm + dp);
    s1 = ext ? 0.0 : 2.0 * dp * dp * is * is;
    s2 = ext ? 0.0 : 2.0 * dm * dm * is * is;
  }
}

// Adjoint of piecewise-linear extrapolation along one line. x[0..4] are the
// values at positions -2..+2 around position 0; xp[p], xm[p] (p = 0,1,2 for
// positions -1, 0, +1) are the cotangents of the upper extrapolation
// x + slope/2 and the lower one x - slope/2 at those positions. Returns the
// cotangent of x at position 0.
template <int LIM>
__device__ __forceinline__ double plm_adjoint(const double* x, const double* xp,
                                              const double* xm) {
  double s1[3], s2[3], sb[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    plm_slope_grad<LIM>(x[p + 1] - x[p], x[p + 2] - x[p + 1], s1[p], s2[p]);
    sb[p] = 0.5 * (xp[p] - xm[p]);
  }
  return xp[1] + xm[1] + sb[1] * (s1[1] - s2[1]) - sb[2] * s1[2] + sb[0] * s2[0];
}

}  // namespace mhd
