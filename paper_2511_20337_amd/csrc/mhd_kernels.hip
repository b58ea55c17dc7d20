// HIP kernels of the ideal-MHD step for gfx950, and their launchers.
//
// One stage of the SSP-RK2 step is three launches over the cell grid:
//   k_faces  — per cell, its lower x/y(/z) faces: primitive recovery of the
//              four cells along each normal, PLM, HLL/HLLD; writes the face
//              fluxes and the alpha+-, HLL-weighted velocities the EMF needs;
//   k_emf    — per cell, the upwind CT EMF on its lower edges;
//   k_update — per cell, flux divergence of the cell fields, -curl E of the
//              face fields, and the RK combination (or the bare RHS).
// The CFL time step is a per-cell minimum reduced with wave64 shuffles and a
// block LDS step into per-block partials, then one finishing block.
//
// Layout: state and workspace arrays are field-major SoA, x fastest, so a
// wavefront of 64 consecutive cells reads 512 contiguous bytes per field.
#include "mhd_device.hpp"
#include "mhd_grid.hpp"
#include "mhd_kernels.hpp"

namespace mhd {

namespace {

// One lower face of direction D at cell (i,j,k): PLM from the four cells
// c-2, c-1, c, c+1 along D (V0 is cell c), then the Riemann solve.
template <int DIM, int D, int LIM, int RS, class R>
__device__ __forceinline__ void face_dir(const double* __restrict__ U, double* __restrict__ FW,
                                         const Geom& g, int i, int j, int k, int64_t c,
                                         const double* V0) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  // primitive slots in the face frame: rho, v_n, v_t1, v_t2, B_t1, B_t2, p
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  double Vm2[8], Vm1[8], Vp1[8];
  const int sh[3] = {D == 0, D == 1, D == 2};
  prim_at<DIM>(U, g, wrap(i - 2 * sh[0], g.nx), wrap(j - 2 * sh[1], g.ny), wrap(k - 2 * sh[2], g.nz), Vm2);
  prim_at<DIM>(U, g, wrap(i - sh[0], g.nx), wrap(j - sh[1], g.ny), wrap(k - sh[2], g.nz), Vm1);
  prim_at<DIM>(U, g, wrap(i + sh[0], g.nx), wrap(j + sh[1], g.ny), wrap(k + sh[2], g.nz), Vp1);
  R wl[7], wr[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int s = slot[q];
    const R a = (R)Vm2[s], b = (R)Vm1[s], cc = (R)V0[s], e = (R)Vp1[s];
    wl[q] = b + R(0.5) * plm_slope<LIM, R>(b - a, cc - b);
    wr[q] = cc - R(0.5) * plm_slope<LIM, R>(cc - b, e - cc);
  }
  const R bn = (R)U[(F_BX + D) * g.n + c];
  RiemannOut<R> o;
  riemann<RS, R>((R)g.gamma, wl, wr, bn, o);
  const int64_t n = g.n;
  double* fw = FW + (int64_t)D * NSLOT * n + c;
  fw[S_RHO * n] = (double)o.f[0];
  fw[(S_MX + D) * n] = (double)o.f[1];
  fw[(S_MX + T1) * n] = (double)o.f[2];
  fw[(S_MX + T2) * n] = (double)o.f[3];
  fw[S_EN * n] = (double)o.f[6];
  if (DIM == 2) fw[S_BZ * n] = (double)((D == 0) ? o.f[5] : o.f[4]);  // B_z is t2 of x, t1 of y
  fw[S_AP * n] = (double)o.ap;
  fw[S_AM * n] = (double)o.am;
  fw[S_V1 * n] = (double)o.v1;
  fw[S_V2 * n] = (double)o.v2;
}

template <int DIM, int LIM, int RS, class R>
__global__ __launch_bounds__(kBlock) void k_faces(const double* __restrict__ U,
                                                  double* __restrict__ FW, Geom g,
                                                  int* __restrict__ flag) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  double V0[8];
  if (!prim_at<DIM>(U, g, i, j, k, V0)) atomicOr(flag, 1);
  face_dir<DIM, 0, LIM, RS, R>(U, FW, g, i, j, k, c, V0);
  face_dir<DIM, 1, LIM, RS, R>(U, FW, g, i, j, k, c, V0);
  if (DIM == 3) face_dir<DIM, 2, LIM, RS, R>(U, FW, g, i, j, k, c, V0);
}

// Edge EMF of component C at cell (i,j,k): the edge at the lower A- and
// lower B-position of the cell, (A, B) = (C+1, C+2) cyclic.
template <int C, int LIM, class R>
__device__ __forceinline__ double emf_comp(const double* __restrict__ U,
                                           const double* __restrict__ FW, const Geom& g, int i,
                                           int j, int k, int64_t c) {
  constexpr int A = (C + 1) % 3, B = (C + 2) % 3;
  const int64_t n = g.n;
  const double* fa = FW + (int64_t)A * NSLOT * n;  // a-faces (normal A)
  const double* fb = FW + (int64_t)B * NSLOT * n;  // b-faces (normal B)
  const int64_t cmb = shifted<B>(g, i, j, k, -1);  // a-face below the edge along B
  const int64_t cma = shifted<A>(g, i, j, k, -1);  // b-face below the edge along A
  const R apa = max_r((R)fa[S_AP * n + cmb], (R)fa[S_AP * n + c]);
  const R ama = max_r((R)fa[S_AM * n + cmb], (R)fa[S_AM * n + c]);
  const R apb = max_r((R)fb[S_AP * n + cma], (R)fb[S_AP * n + c]);
  const R amb = max_r((R)fb[S_AM * n + cma], (R)fb[S_AM * n + c]);
  // W/E: on b-faces, v_A (slot V2 of the B frame) and b_B, along A
  const int64_t a2 = shifted<A>(g, i, j, k, -2), a1 = shifted<A>(g, i, j, k, 1);
  const double* vbA = fb + S_V2 * n;
  const double* bB = U + (F_BX + B) * n;
  R vW, vE, bW, bE;
  edge_pair<LIM, R>((R)vbA[a2], (R)vbA[cma], (R)vbA[c], (R)vbA[a1], vW, vE);
  edge_pair<LIM, R>((R)bB[a2], (R)bB[cma], (R)bB[c], (R)bB[a1], bW, bE);
  // S/N: on a-faces, v_B (slot V1 of the A frame) and b_A, along B
  const int64_t b2 = shifted<B>(g, i, j, k, -2), b1 = shifted<B>(g, i, j, k, 1);
  const double* vaB = fa + S_V1 * n;
  const double* bA = U + (F_BX + A) * n;
  R vS, vN, bS, bN;
  edge_pair<LIM, R>((R)vaB[b2], (R)vaB[cmb], (R)vaB[c], (R)vaB[b1], vS, vN);
  edge_pair<LIM, R>((R)bA[b2], (R)bA[cmb], (R)bA[c], (R)bA[b1], bS, bN);
  return (double)uct<R>(apa, ama, vW, bW, vE, bE, apb, amb, vS, bS, vN, bN);
}

template <int DIM, int LIM, class R>
__global__ __launch_bounds__(kBlock) void k_emf(const double* __restrict__ U,
                                                const double* __restrict__ FW,
                                                double* __restrict__ EW, Geom g) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  if (DIM == 3) {
    EW[c] = emf_comp<0, LIM, R>(U, FW, g, i, j, k, c);
    EW[g.n + c] = emf_comp<1, LIM, R>(U, FW, g, i, j, k, c);
  }
  EW[2 * g.n + c] = emf_comp<2, LIM, R>(U, FW, g, i, j, k, c);
}

// STAGE 0: out = L(U); 1: out = U + dt L(U); 2: out = (U0 + (U + dt L(U))) / 2.
template <int DIM, int STAGE>
__global__ __launch_bounds__(kBlock) void k_update(const double* __restrict__ U,
                                                   const double* U0, double* out,
                                                   const double* __restrict__ FW,
                                                   const double* __restrict__ EW, Geom g,
                                                   double dt, const double* __restrict__ dtp) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.n) return;
  int i, j, k;
  coords(g, c, i, j, k);
  const int64_t n = g.n;
  const double h = (STAGE == 0) ? 0.0 : (dtp ? *dtp : dt);
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
  for (int qq = 0; qq < ncell; ++qq) {
    const int q = qq;  // slot == field for rho..E; slot S_BZ for the 2D B_z
    double acc = (fx[q * n + xp] - fx[q * n + c]) * idx + (fy[q * n + yp] - fy[q * n + c]) * idy;
    if (DIM == 3) acc += (fz[q * n + zp] - fz[q * n + c]) * idz;
    L[qq == 5 ? 7 : qq] = -acc;
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
    double v;
    if (STAGE == 0) v = L[q];
    else if (STAGE == 1) v = U[q * n + c] + h * L[q];
    else v = 0.5 * (U0[q * n + c] + (U[q * n + c] + h * L[q]));
    out[q * n + c] = v;
  }
}

// CFL: per-cell min over directions of dx_d / (|v_d| + c_f,d); grid-stride,
// wave64 shuffle + LDS reduction to one partial per block.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cfl(const double* __restrict__ U, Geom g,
                                                double* __restrict__ partial,
                                                int* __restrict__ flag) {
  double m = __builtin_inf();
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < g.n;
       c += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    coords(g, c, i, j, k);
    double V[8];
    if (!prim_at<DIM>(U, g, i, j, k, V)) atomicOr(flag, 1);
    const double dd[3] = {g.dx, g.dy, g.dz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double cf = cfast<double>(g.gamma, V[0], V[4], V[5 + d], V[5 + (d + 1) % 3],
                                      V[5 + (d + 2) % 3]);
      const double t = dd[d] / (__builtin_fabs(V[1 + d]) + cf);
      m = (t < m) ? t : m;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = (o < m) ? o : m;
  }
  __shared__ double red[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) r = (red[w] < r) ? red[w] : r;
    partial[blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(1024) void k_cfl_final(const double* __restrict__ partial, int np,
                                                    double cfl, double* __restrict__ dt_out) {
  double m = __builtin_inf();
  for (int b = threadIdx.x; b < np; b += 1024) m = (partial[b] < m) ? partial[b] : m;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = (o < m) ? o : m;
  }
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < 16; ++w) r = (red[w] < r) ? red[w] : r;
    *dt_out = cfl * r;
  }
}

unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int DIM, int LIM, int RS, class R>
hipError_t stage_impl(const StageArgs& a) {
  const unsigned nb = grid_for(a.g.n);
  MHD_TIMED(a, K_FACES,
            hipLaunchKernelGGL((k_faces<DIM, LIM, RS, R>), dim3(nb), dim3(kBlock), 0, a.stream,
                               a.U, a.FW, a.g, a.flag));
  MHD_TIMED(a, K_EMF,
            hipLaunchKernelGGL((k_emf<DIM, LIM, R>), dim3(nb), dim3(kBlock), 0, a.stream, a.U,
                               a.FW, a.EW, a.g));
  switch (a.stage) {
    case 3:  // face and edge records only
      break;
    case 0:
      MHD_TIMED(a, K_UPDATE,
                hipLaunchKernelGGL((k_update<DIM, 0>), dim3(nb), dim3(kBlock), 0, a.stream, a.U,
                                   a.U0, a.out, a.FW, a.EW, a.g, a.dt, a.dtp));
      break;
    case 1:
      MHD_TIMED(a, K_UPDATE,
                hipLaunchKernelGGL((k_update<DIM, 1>), dim3(nb), dim3(kBlock), 0, a.stream, a.U,
                                   a.U0, a.out, a.FW, a.EW, a.g, a.dt, a.dtp));
      break;
    default:
      MHD_TIMED(a, K_UPDATE,
                hipLaunchKernelGGL((k_update<DIM, 2>), dim3(nb), dim3(kBlock), 0, a.stream, a.U,
                                   a.U0, a.out, a.FW, a.EW, a.g, a.dt, a.dtp));
      break;
  }
  return hipGetLastError();
}

template <int DIM>
hipError_t stage_lim(const StageArgs& a) {
  const bool mixed = a.precision == 1;
  if (a.limiter == 0) {
    if (a.riemann == 0)
      return mixed ? stage_impl<DIM, 0, 0, float>(a) : stage_impl<DIM, 0, 0, double>(a);
    return mixed ? stage_impl<DIM, 0, 1, float>(a) : stage_impl<DIM, 0, 1, double>(a);
  }
  if (a.riemann == 0)
    return mixed ? stage_impl<DIM, 1, 0, float>(a) : stage_impl<DIM, 1, 0, double>(a);
  return mixed ? stage_impl<DIM, 1, 1, float>(a) : stage_impl<DIM, 1, 1, double>(a);
}

}  // namespace

hipError_t launch_stage(const StageArgs& a) {
  return (a.dim == 3) ? stage_lim<3>(a) : stage_lim<2>(a);
}

hipError_t launch_cfl(const CflArgs& a) {
  if (a.dim == 3)
    MHD_TIMED(a, K_CFL,
              hipLaunchKernelGGL((k_cfl<3>), dim3(a.nblocks), dim3(kBlock), 0, a.stream, a.U, a.g,
                                 a.partial, a.flag));
  else
    MHD_TIMED(a, K_CFL,
              hipLaunchKernelGGL((k_cfl<2>), dim3(a.nblocks), dim3(kBlock), 0, a.stream, a.U, a.g,
                                 a.partial, a.flag));
  MHD_TIMED(a, K_CFL_FINAL,
            hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, a.partial,
                               a.nblocks, a.cfl, a.dt_out));
  return hipGetLastError();
}

}  // namespace mhd
