// HIP kernels of the ideal-MHD step for gfx950, and their launchers.
//
// One stage of the SSP-RK2 step is three launches:
//   k_faces_march — 3D: 64 x 4 columns of cells marching along z, with the
//                   primitives of three planes and a cross halo in LDS; per
//                   cell its lower x/y/z faces: PLM, HLL/HLLD; writes the
//                   face fluxes and the alpha+-, HLL-weighted velocities the
//                   EMF needs (k_faces_tiled does the same on 2D tiles);
//   k_emf         — per cell, the upwind CT EMF on its lower edges;
//   k_update      — per cell, flux divergence of the cell fields, -curl E of
//                   the face fields, and the RK combination (or the bare RHS).
// The CFL time step is a per-cell minimum reduced with wave64 shuffles and a
// block LDS step into per-block partials, then one finishing block; in the 3D
// step the first stage's face kernel computes those partials itself.
//
// Layout: state and workspace arrays are field-major SoA, x fastest, so a
// wavefront of 64 consecutive cells reads 512 contiguous bytes per field.
#include <mutex>

#include "mhd_device.hpp"
#include "mhd_grid.hpp"
#include "mhd_kernels.hpp"

namespace mhd {

namespace {

// ---------------------------------------------------------------------------
// 2D face kernel on tiles: a workgroup owns 16 x 16 cells, one per thread.
// (The 3D grid uses the z-marching kernel below.)
template <int DIM>
struct Tile {
  static constexpr int TX = 16, TY = (DIM == 3) ? 4 : 16, TZ = (DIM == 3) ? 4 : 1;
  static constexpr int NCORE = TX * TY * TZ;  // also the workgroup size
  // cross-shaped halo: two cells below and one above the tile along each axis
  static constexpr int HX = 3 * TY * TZ, HY = 3 * TX * TZ, HZ = (DIM == 3) ? 3 * TX * TY : 0;
  static constexpr int NPRIM = NCORE + HX + HY + HZ;
};
static_assert(Tile<2>::NCORE % 64 == 0 && Tile<2>::NCORE <= 1024, "whole wavefronts");

// Row tiles for the kernels without LDS staging: a wavefront covers 64
// consecutive cells of one row (512 contiguous bytes per field).
struct RowTile {
  static constexpr int TX = 64, TY = 4, TZ = 1;
  static constexpr int NT = TX * TY;  // workgroup size
};

// Face records (fluxes, alpha+-, HLL-weighted velocities) and edge EMFs are
// stored in the precision they were computed in: FP64, or FP32 in the mixed
// mode (exact, and half the bytes for the kernels that read them). The
// workspace holds dim * NSLOT * n and 3 * n doubles either way.
template <class R>
__device__ __forceinline__ R* stored(double* buf) {
  return reinterpret_cast<R*>(buf);
}
template <class R>
__device__ __forceinline__ const R* stored(const double* buf) {
  return reinterpret_cast<const R*>(buf);
}

struct MarchGrid {
  int ntx, nty, nzc, lz;  // column tiles in x, y; runs of lz planes along z
  unsigned nblocks;
};

struct TileGrid {
  int ntx, nty, ntz;
  unsigned ntiles;
};

// Tiles are visited in natural order (x fastest): consecutive workgroups,
// which the dispatcher deals to the 8 XCDs in turn, then stream through
// contiguous memory; halo reuse across XCDs is served by the Infinity Cache.
// (Renumbering tiles so that each XCD owns a contiguous run measured slower
// at 256^3: face kernel 1.77 vs 1.71 ms, update 1.11 vs 0.98 ms.)
__device__ __forceinline__ int wrap_any(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

template <int DIM>
__device__ __forceinline__ void tile_origin(const TileGrid& tg, unsigned t, int& i0, int& j0,
                                            int& k0) {
  using T = Tile<DIM>;
  const int tx = (int)(t % (unsigned)tg.ntx);
  const unsigned r = t / (unsigned)tg.ntx;
  const int ty = (int)(r % (unsigned)tg.nty);
  const int tz = (int)(r / (unsigned)tg.nty);
  i0 = tx * T::TX;
  j0 = ty * T::TY;
  k0 = tz * T::TZ;
}

// Cell of this thread in the row-tile traversal; false outside the domain.
// XG: workgroups in the XCD-grouped order (xcd_grouped) instead of round-robin.
template <bool XG = false>
__device__ __forceinline__ bool row_cell(const Geom& g, const TileGrid& tg, int& i, int& j, int& k) {
  const unsigned t = XG ? xcd_grouped(blockIdx.x, gridDim.x) : blockIdx.x;
  const int tx = (int)(t % (unsigned)tg.ntx);
  const unsigned r = t / (unsigned)tg.ntx;
  const int ty = (int)(r % (unsigned)tg.nty);
  const int tz = (int)(r / (unsigned)tg.nty);
  i = tx * RowTile::TX + (int)threadIdx.x % RowTile::TX;
  j = ty * RowTile::TY + (int)threadIdx.x / RowTile::TX;
  k = tz;
  return i < g.nx && j < g.ny && k < g.nz;
}

// The record of a lower D-face: the fluxes of the cell fields (with B_z in
// 2D), then the EMF inputs, alpha+- and the HLL-weighted velocities (EM 0),
// or the UCT-HLLD weight, diffusion coefficients and weighted velocities
// (EM 1). The normal-B flux is zero and the edge EMFs replace the B_t fluxes.
template <int DIM, int D, int EM, class R>
__device__ __forceinline__ void put_record(double* __restrict__ FW, int64_t n, int64_t c,
                                           const RiemannOut<R>& o) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  R* fw = stored<R>(FW) + (int64_t)D * NSLOT * n + c;
  fw[S_RHO * n] = o.f[0];
  fw[(S_MX + D) * n] = o.f[1];
  fw[(S_MX + T1) * n] = o.f[2];
  fw[(S_MX + T2) * n] = o.f[3];
  fw[S_EN * n] = o.f[6];
  if (DIM == 2) fw[S_BZ * n] = (D == 0) ? o.f[5] : o.f[4];  // B_z is t2 of x, t1 of y
  if (EM == 1) {
    fw[S_AP * n] = o.om;
    fw[S_AM * n] = o.dl;
    fw[S_DR * n] = o.dr;
  } else {
    fw[S_AP * n] = o.ap;
    fw[S_AM * n] = o.am;
  }
  fw[S_V1 * n] = o.v1;
  fw[S_V2 * n] = o.v2;
}

// Upwind edge EMF from its inputs: alpha+- of the two a-faces touching the
// edge (below the edge along B, then the cell's own), of the two b-faces
// (below along A, then own); the face velocity v_A and the field b_B on the
// b-faces at A-offsets -2..+1, and v_B and b_A on the a-faces at B-offsets
// -2..+1, each reconstructed toward the edge.
template <int LIM, class R>
__device__ __forceinline__ R emf_core(R apa_m, R apa_c, R ama_m, R ama_c, R apb_m, R apb_c,
                                      R amb_m, R amb_c, const R* vbA, const R* bB, const R* vaB,
                                      const R* bA) {
  const R apa = max_r(apa_m, apa_c), ama = max_r(ama_m, ama_c);
  const R apb = max_r(apb_m, apb_c), amb = max_r(amb_m, amb_c);
  R vW, vE, bW, bE, vS, vN, bS, bN;
  edge_pair<LIM, R>(vbA[0], vbA[1], vbA[2], vbA[3], vW, vE);
  edge_pair<LIM, R>(bB[0], bB[1], bB[2], bB[3], bW, bE);
  edge_pair<LIM, R>(vaB[0], vaB[1], vaB[2], vaB[3], vS, vN);
  edge_pair<LIM, R>(bA[0], bA[1], bA[2], bA[3], bS, bN);
  return uct<R>(apa, ama, vW, bW, vE, bE, apb, amb, vS, bS, vN, bN);
}

// UCT-HLLD edge EMF from its inputs: om, d^L, d^R of the two a-faces (below
// the edge along B, then the cell's own) and of the two b-faces, averaged;
// the reconstructed values as for emf_core.
template <int LIM, class R>
__device__ __forceinline__ R emf_core_hlld(R oma_m, R oma_c, R dla_m, R dla_c, R dra_m, R dra_c,
                                           R omb_m, R omb_c, R dlb_m, R dlb_c, R drb_m, R drb_c,
                                           const R* vbA, const R* bB, const R* vaB,
                                           const R* bA) {
  const R aa = R(0.5) * (oma_m + oma_c), dla = R(0.5) * (dla_m + dla_c);
  const R dra = R(0.5) * (dra_m + dra_c);
  const R ab = R(0.5) * (omb_m + omb_c), dlb = R(0.5) * (dlb_m + dlb_c);
  const R drb = R(0.5) * (drb_m + drb_c);
  R vW, vE, bW, bE, vS, vN, bS, bN;
  edge_pair<LIM, R>(vbA[0], vbA[1], vbA[2], vbA[3], vW, vE);
  edge_pair<LIM, R>(bB[0], bB[1], bB[2], bB[3], bW, bE);
  edge_pair<LIM, R>(vaB[0], vaB[1], vaB[2], vaB[3], vS, vN);
  edge_pair<LIM, R>(bA[0], bA[1], bA[2], bA[3], bS, bN);
  return uct_hlld<R>(aa, dla, dra, vW, bW, vE, bE, ab, dlb, drb, vS, bS, vN, bN);
}

// Edge EMF of component C at cell (i,j,k): the edge at the lower A- and
// lower B-position of the cell, (A, B) = (C+1, C+2) cyclic. EM 0: the
// upwind average with the HLL bounds; EM 1: the UCT-HLLD average.
template <int C, int LIM, class R, int EM = 0>
__device__ __forceinline__ R emf_comp(const double* __restrict__ U,
                                      const double* __restrict__ FW, const Geom& g, int i, int j,
                                      int k, int64_t c) {
  constexpr int A = (C + 1) % 3, B = (C + 2) % 3;
  const int64_t n = g.n;
  const R* fa = stored<R>(FW) + (int64_t)A * NSLOT * n;  // a-faces (normal A)
  const R* fb = stored<R>(FW) + (int64_t)B * NSLOT * n;  // b-faces (normal B)
  const int64_t cmb = shifted<B>(g, i, j, k, -1);  // a-face below the edge along B
  const int64_t cma = shifted<A>(g, i, j, k, -1);  // b-face below the edge along A
  const int64_t a2 = shifted<A>(g, i, j, k, -2), a1 = shifted<A>(g, i, j, k, 1);
  const int64_t b2 = shifted<B>(g, i, j, k, -2), b1 = shifted<B>(g, i, j, k, 1);
  const R* vbA = fb + S_V2 * n;  // on b-faces, v_A (slot V2 of the B frame)
  const double* bBf = U + (F_BX + B) * n;
  const R* vaB = fa + S_V1 * n;  // on a-faces, v_B (slot V1 of the A frame)
  const double* bAf = U + (F_BX + A) * n;
  const R wv[4] = {vbA[a2], vbA[cma], vbA[c], vbA[a1]};
  const R wb[4] = {(R)bBf[a2], (R)bBf[cma], (R)bBf[c], (R)bBf[a1]};
  const R sv[4] = {vaB[b2], vaB[cmb], vaB[c], vaB[b1]};
  const R sb[4] = {(R)bAf[b2], (R)bAf[cmb], (R)bAf[c], (R)bAf[b1]};
  if (EM == 1)
    return emf_core_hlld<LIM, R>(fa[S_AP * n + cmb], fa[S_AP * n + c], fa[S_AM * n + cmb],
                                 fa[S_AM * n + c], fa[S_DR * n + cmb], fa[S_DR * n + c],
                                 fb[S_AP * n + cma], fb[S_AP * n + c], fb[S_AM * n + cma],
                                 fb[S_AM * n + c], fb[S_DR * n + cma], fb[S_DR * n + c], wv, wb,
                                 sv, sb);
  return emf_core<LIM, R>(fa[S_AP * n + cmb], fa[S_AP * n + c], fa[S_AM * n + cmb],
                          fa[S_AM * n + c], fb[S_AP * n + cma], fb[S_AP * n + c],
                          fb[S_AM * n + cma], fb[S_AM * n + c], wv, wb, sv, sb);
}

// 3D EMF kernel marching along z over 64 x 4 columns: the inputs of E_x and
// E_y that are offset along z (alpha+- of the y- and x-faces one plane down,
// v and b on those faces two planes down to one up) ride in registers from
// plane to plane, so each is loaded once per run instead of up to four times.
struct EmfCol {
  static constexpr int TX = 64, TY = 4;
  static constexpr int NT = TX * TY;  // workgroup size
};

// The coefficients of one face the edge average takes: alpha+ and alpha-
// (EM 0), or the UCT-HLLD weight and diffusion coefficients (EM 1).
template <int EM, class R>
struct FaceCoef {
  R c[EM == 1 ? 3 : 2];
};
template <int EM, class R>
__device__ __forceinline__ FaceCoef<EM, R> face_coef(const R* f, int64_t n, int64_t c) {
  FaceCoef<EM, R> o;
  o.c[0] = f[S_AP * n + c];
  o.c[1] = f[S_AM * n + c];
  if constexpr (EM == 1) o.c[2] = f[S_DR * n + c];
  return o;
}
// Edge EMF from the coefficients of the a-faces (below the edge along B,
// then the cell's own) and b-faces, and the reconstructed values.
template <int LIM, int EM, class R>
__device__ __forceinline__ R emf_from(const FaceCoef<EM, R>& am, const FaceCoef<EM, R>& ac,
                                      const FaceCoef<EM, R>& bm, const FaceCoef<EM, R>& bc,
                                      const R* vbA, const R* bB, const R* vaB, const R* bA) {
  if constexpr (EM == 1)
    return emf_core_hlld<LIM, R>(am.c[0], ac.c[0], am.c[1], ac.c[1], am.c[2], ac.c[2], bm.c[0],
                                 bc.c[0], bm.c[1], bc.c[1], bm.c[2], bc.c[2], vbA, bB, vaB, bA);
  else
    return emf_core<LIM, R>(am.c[0], ac.c[0], am.c[1], ac.c[1], bm.c[0], bc.c[0], bm.c[1],
                            bc.c[1], vbA, bB, vaB, bA);
}

template <int LIM, class R, int EM>
__device__ __forceinline__ void emf_march(const double* __restrict__ U,
                                          const double* __restrict__ FW, double* __restrict__ EW,
                                          Geom g, MarchGrid mg) {
  // mixed mode: the XCD-grouped order (0.523 -> 0.513 ms at 256^3; FP64 unchanged)
  const unsigned b = (sizeof(R) == 4) ? xcd_grouped(blockIdx.x, gridDim.x) : blockIdx.x;
  const int tx = (int)(b % (unsigned)mg.ntx);
  const unsigned r = b / (unsigned)mg.ntx;
  const int ty = (int)(r % (unsigned)mg.nty);
  const int zc = (int)(r / (unsigned)mg.nty);
  const int i = tx * EmfCol::TX + (int)threadIdx.x % EmfCol::TX;
  const int j = ty * EmfCol::TY + (int)threadIdx.x / EmfCol::TX;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = zc * mg.lz;
  const int k1 = min(k0 + mg.lz, g.nz);
  const int64_t n = g.n;
  const R* fx = stored<R>(FW);
  const R* fy = fx + (int64_t)NSLOT * n;
  const R* fz = fx + (int64_t)2 * NSLOT * n;
  R* ew = stored<R>(EW);
  const double* bx = U + F_BX * n;
  const double* by = U + F_BY * n;
  const double* bz = U + F_BZ * n;
  // planes k-2 .. k+1 of this column: v_z on y-faces and b_y (E_x), v_z on
  // x-faces and b_x (E_y); the coefficients of y- and x-faces on planes k-1, k
  R yv[4], yb[4], xv[4], xb[4];
  FaceCoef<EM, R> yc[2], xc[2];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int64_t cs = lin(g, i, j, wrap_any(k0 - 2 + s, g.nz));
    yv[s] = fy[S_V1 * n + cs];
    yb[s] = (R)by[cs];
    xv[s] = fx[S_V2 * n + cs];
    xb[s] = (R)bx[cs];
  }
  {
    const int64_t cm = lin(g, i, j, wrap_any(k0 - 1, g.nz));
    yc[0] = face_coef<EM, R>(fy, n, cm);
    xc[0] = face_coef<EM, R>(fx, n, cm);
  }
  const int im2 = wrap(i - 2, g.nx), im1 = wrap(i - 1, g.nx), ip1 = wrap(i + 1, g.nx);
  const int jm2 = wrap(j - 2, g.ny), jm1 = wrap(j - 1, g.ny), jp1 = wrap(j + 1, g.ny);
  for (int k = k0; k < k1; ++k) {
    const int64_t c = lin(g, i, j, k);
    const int64_t cp = lin(g, i, j, wrap(k + 1, g.nz));
    const int64_t cjm2 = lin(g, i, jm2, k), cjm1 = lin(g, i, jm1, k), cjp1 = lin(g, i, jp1, k);
    const int64_t cim2 = lin(g, im2, j, k), cim1 = lin(g, im1, j, k), cip1 = lin(g, ip1, j, k);
    // all loads of this plane first (face records in R, staggered fields in
    // FP64), then the conversions to R: the loads stay in flight together
    const R* vz2 = fz + S_V2 * n;
    const R* vz1 = fz + S_V1 * n;
    R r[14];
    double d[9];
    r[0] = fy[S_V1 * n + cp]; r[1] = fx[S_V2 * n + cp];
    yc[1] = face_coef<EM, R>(fy, n, c);
    xc[1] = face_coef<EM, R>(fx, n, c);
    r[6] = vz2[cjm2]; r[7] = vz2[cjm1]; r[8] = vz2[c]; r[9] = vz2[cjp1];
    r[10] = vz1[cim2]; r[11] = vz1[cim1]; r[12] = vz1[c]; r[13] = vz1[cip1];
    const FaceCoef<EM, R> zjm = face_coef<EM, R>(fz, n, cjm1);
    const FaceCoef<EM, R> zc0 = face_coef<EM, R>(fz, n, c);
    const FaceCoef<EM, R> zim = face_coef<EM, R>(fz, n, cim1);
    d[0] = by[cp]; d[1] = bx[cp];
    d[2] = bz[cjm2]; d[3] = bz[cjm1]; d[4] = bz[c]; d[5] = bz[cjp1];
    d[6] = bz[cim2]; d[7] = bz[cim1]; d[8] = bz[cip1];
    // E_z: (A, B) = (x, y); its inputs are loaded here too, so that no load
    // of the plane is issued after one of its EMF stores (the wait for it
    // would then wait for the store as well)
    const FaceCoef<EM, R> xjm = face_coef<EM, R>(fx, n, cjm1);
    const FaceCoef<EM, R> yim = face_coef<EM, R>(fy, n, cim1);
    const R* vyx = fy + S_V2 * n;  // v_x on y-faces
    const R* vxy = fx + S_V1 * n;  // v_y on x-faces
    const R zwv[4] = {vyx[cim2], vyx[cim1], vyx[c], vyx[cip1]};
    const R zsv[4] = {vxy[cjm2], vxy[cjm1], vxy[c], vxy[cjp1]};
    const double zwd[4] = {by[cim2], by[cim1], by[c], by[cip1]};
    const double zsd[4] = {bx[cjm2], bx[cjm1], bx[c], bx[cjp1]};
    // keep the scheduler from sinking loads into the arithmetic (the minmod
    // FP64 instantiation otherwise waited for its loads one or two at a time)
    __builtin_amdgcn_sched_barrier(0);
    yv[3] = r[0];
    yb[3] = (R)d[0];
    xv[3] = r[1];
    xb[3] = (R)d[1];
    // E_x: (A, B) = (y, z); a-faces are y-faces, b-faces z-faces
    R ex, ey, ez;
    {
      const R wv[4] = {r[6], r[7], r[8], r[9]};
      const R wb[4] = {(R)d[2], (R)d[3], (R)d[4], (R)d[5]};
      ex = emf_from<LIM, EM, R>(yc[0], yc[1], zjm, zc0, wv, wb, yv, yb);
    }
    // E_y: (A, B) = (z, x); a-faces are z-faces, b-faces x-faces
    {
      const R sv[4] = {r[10], r[11], r[12], r[13]};
      const R sb[4] = {(R)d[6], (R)d[7], (R)d[4], (R)d[8]};
      ey = emf_from<LIM, EM, R>(zim, zc0, xc[0], xc[1], xv, xb, sv, sb);
    }
    // E_z: a-faces are x-faces, b-faces y-faces
    {
      const R wb[4] = {(R)zwd[0], (R)zwd[1], (R)zwd[2], (R)zwd[3]};
      const R sb[4] = {(R)zsd[0], (R)zsd[1], (R)zsd[2], (R)zsd[3]};
      ez = emf_from<LIM, EM, R>(xjm, xc[1], yim, yc[1], zwv, wb, zsv, sb);
    }
    ew[c] = ex;
    ew[n + c] = ey;
    ew[2 * n + c] = ez;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      yv[s] = yv[s + 1];
      yb[s] = yb[s + 1];
      xv[s] = xv[s + 1];
      xb[s] = xb[s + 1];
    }
    yc[0] = yc[1];
    xc[0] = xc[1];
  }
}

// The upwind (EM 0) kernel is held to two waves per SIMD, where it keeps all
// its loads of a plane in flight without spilling; the UCT-HLLD kernel (EM 1)
// needs more registers and runs at one.
template <int LIM, class R>
__global__ __launch_bounds__(EmfCol::NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_emf_march(const double* __restrict__ U, const double* __restrict__ FW,
                 double* __restrict__ EW, Geom g, MarchGrid mg) {
  emf_march<LIM, R, 0>(U, FW, EW, g, mg);
}
template <int LIM, class R>
__global__ __launch_bounds__(EmfCol::NT)
void k_emf_march_hlld(const double* __restrict__ U, const double* __restrict__ FW,
                      double* __restrict__ EW, Geom g, MarchGrid mg) {
  emf_march<LIM, R, 1>(U, FW, EW, g, mg);
}

template <int DIM, int LIM, class R, int EM>
__global__ __launch_bounds__(RowTile::NT) void k_emf(const double* __restrict__ U,
                                                const double* __restrict__ FW,
                                                double* __restrict__ EW, Geom g, TileGrid tg) {
  int i, j, k;
  if (!row_cell(g, tg, i, j, k)) return;
  const int64_t c = lin(g, i, j, k);
  R* ew = stored<R>(EW);
  if (DIM == 3) {
    ew[c] = emf_comp<0, LIM, R, EM>(U, FW, g, i, j, k, c);
    ew[g.n + c] = emf_comp<1, LIM, R, EM>(U, FW, g, i, j, k, c);
  }
  ew[2 * g.n + c] = emf_comp<2, LIM, R, EM>(U, FW, g, i, j, k, c);
}

// STAGE 0: out = L(U); 1: out = U + dt L(U); 2: out = (U0 + (U + dt L(U))) / 2
// (SSP-RK2); 4: out = (3 U0 + (U + dt L(U))) / 4 and 5: out = (U0 + 2 (U + dt
// L(U))) / 3, the second and third stages of SSP-RK3 (Eq. (RK3)).
// R: the precision of the stored fluxes (differenced in FP64).
template <int DIM, int STAGE, class R>
__global__ __launch_bounds__(RowTile::NT) void k_update(const double* __restrict__ U,
                                                   const double* U0, double* out,
                                                   const double* __restrict__ FW,
                                                   const double* __restrict__ EW, Geom g,
                                                   TileGrid tg, double dt,
                                                   const double* __restrict__ dtp) {
  int i, j, k;
  // mixed mode (FP32 records): the XCD-grouped order, measured faster there
  // (0.777 -> 0.738 ms at 256^3) and slower in FP64
  if (!row_cell<sizeof(R) == 4>(g, tg, i, j, k)) return;
  const int64_t c = lin(g, i, j, k);
  const int64_t n = g.n;
  const double h = (STAGE == 0) ? 0.0 : (dtp ? *dtp : dt);
  const int64_t xp = lin(g, wrap(i + 1, g.nx), j, k);
  const int64_t yp = lin(g, i, wrap(j + 1, g.ny), k);
  const int64_t zp = (DIM == 3) ? lin(g, i, j, wrap(k + 1, g.nz)) : c;
  const double idx = 1.0 / g.dx, idy = 1.0 / g.dy, idz = 1.0 / g.dz;
  const R* fx = stored<R>(FW);
  const R* fy = fx + (int64_t)NSLOT * n;
  const R* fz = fx + (int64_t)2 * NSLOT * n;
  double L[8];
  constexpr int ncell = (DIM == 3) ? 5 : 6;
#pragma unroll
  for (int qq = 0; qq < ncell; ++qq) {
    const int q = qq;  // slot == field for rho..E; slot S_BZ for the 2D B_z
    double acc = ((double)fx[q * n + xp] - (double)fx[q * n + c]) * idx +
                 ((double)fy[q * n + yp] - (double)fy[q * n + c]) * idy;
    if (DIM == 3) acc += ((double)fz[q * n + zp] - (double)fz[q * n + c]) * idz;
    L[qq == 5 ? 7 : qq] = -acc;
  }
  // edge EMFs, stored in R, widened to FP64 before differencing
  const R* ex = stored<R>(EW);
  const R* ey = ex + n;
  const R* ez = ex + 2 * n;
  if (DIM == 3) {
    L[5] = -(((double)ez[yp] - (double)ez[c]) * idy - ((double)ey[zp] - (double)ey[c]) * idz);
    L[6] = -(((double)ex[zp] - (double)ex[c]) * idz - ((double)ez[xp] - (double)ez[c]) * idx);
    L[7] = -(((double)ey[xp] - (double)ey[c]) * idx - ((double)ex[yp] - (double)ex[c]) * idy);
  } else {
    L[5] = -(((double)ez[yp] - (double)ez[c]) * idy);
    L[6] = ((double)ez[xp] - (double)ez[c]) * idx;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double v;
    if (STAGE == 0) v = L[q];
    else if (STAGE == 1) v = U[q * n + c] + h * L[q];
    else if (STAGE == 4) v = (3.0 * U0[q * n + c] + (U[q * n + c] + h * L[q])) / 4.0;
    else if (STAGE == 5) v = (U0[q * n + c] + 2.0 * (U[q * n + c] + h * L[q])) / 3.0;
    else v = 0.5 * (U0[q * n + c] + (U[q * n + c] + h * L[q]));
    out[q * n + c] = v;
  }
}

// 2D EMF and update in one kernel, over the row tiles of k_update: each
// thread forms E_z at the lower corner of its cell (any thread past the grid
// at the periodic image of that corner), threads 0..68 also the corners of
// the row above and of the column to the right, all into LDS behind one
// barrier; then each cell of the grid is updated as k_update<2> does it
// (bitwise equal), and its own E_z is stored for the adjoint's records.
// cflp != nullptr (first stage of a step whose face kernel left npart CFL
// partials): every workgroup reduces the partials itself to the minimum
// k_cfl_final forms (a minimum is exact in any order), dt = cfl * min, and
// workgroup 0 writes it to *dt_out; for small grids this replaces the
// k_cfl_final launch.
template <int LIM, int STAGE, class R, int EM>
__global__ __launch_bounds__(RowTile::NT) void k_emf_update_2d(const double* __restrict__ U,
                                                               const double* U0, double* out,
                                                               const double* __restrict__ FW,
                                                               double* __restrict__ EW, Geom g,
                                                               TileGrid tg, double dt,
                                                               const double* __restrict__ dtp,
                                                               const double* __restrict__ cflp,
                                                               int npart, double cfl,
                                                               double* __restrict__ dt_out) {
  constexpr int TX = RowTile::TX, TY = RowTile::TY, SX = TX + 1;
  __shared__ R ezs[(TY + 1) * SX];
  __shared__ double red[RowTile::NT / 64];
  if (cflp) {
    double m = __builtin_inf();
    for (int b = (int)threadIdx.x; b < npart; b += RowTile::NT) m = (cflp[b] < m) ? cflp[b] : m;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(m, off, 64);
      m = (o < m) ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  }
  const unsigned t = (sizeof(R) == 4) ? xcd_grouped(blockIdx.x, gridDim.x) : blockIdx.x;
  const int i0 = (int)(t % (unsigned)tg.ntx) * TX;
  const int j0 = (int)(t / (unsigned)tg.ntx) * TY;
  const int x = (int)threadIdx.x % TX, y = (int)threadIdx.x / TX;
  const int i = i0 + x, j = j0 + y;
  const bool inside = i < g.nx && j < g.ny;
  const int64_t n = g.n;
  {
    const int iw = wrap_any(i, g.nx), jw = wrap_any(j, g.ny);
    const R ez = emf_comp<2, LIM, R, EM>(U, FW, g, iw, jw, 0, lin(g, iw, jw, 0));
    ezs[y * SX + x] = ez;
    if (inside) stored<R>(EW)[2 * n + lin(g, i, j, 0)] = ez;
  }
  if (threadIdx.x < TX + TY + 1) {
    const int h = (int)threadIdx.x;
    const int hx = (h < TX) ? h : TX, hy = (h < TX) ? TY : h - TX;  // h = TX + TY: the corner
    const int iw = wrap_any(i0 + hx, g.nx), jw = wrap_any(j0 + hy, g.ny);
    ezs[hy * SX + hx] = emf_comp<2, LIM, R, EM>(U, FW, g, iw, jw, 0, lin(g, iw, jw, 0));
  }
  __syncthreads();
  double h;
  if (STAGE == 0) {
    h = 0.0;
  } else if (cflp) {
    double m = red[0];
#pragma unroll
    for (int w = 1; w < RowTile::NT / 64; ++w) m = (red[w] < m) ? red[w] : m;
    h = cfl * m;
    if (blockIdx.x == 0 && threadIdx.x == 0) *dt_out = h;
  } else {
    h = dtp ? *dtp : dt;
  }
  if (!inside) return;
  const int64_t c = lin(g, i, j, 0);
  const int64_t xp = lin(g, wrap(i + 1, g.nx), j, 0);
  const int64_t yp = lin(g, i, wrap(j + 1, g.ny), 0);
  const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
  const R* fx = stored<R>(FW);
  const R* fy = fx + (int64_t)NSLOT * n;
  double L[8];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double acc = ((double)fx[q * n + xp] - (double)fx[q * n + c]) * idx +
                       ((double)fy[q * n + yp] - (double)fy[q * n + c]) * idy;
    L[q == 5 ? 7 : q] = -acc;
  }
  const double ezc = (double)ezs[y * SX + x];
  L[5] = -(((double)ezs[(y + 1) * SX + x] - ezc) * idy);
  L[6] = ((double)ezs[y * SX + x + 1] - ezc) * idx;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double v;
    if (STAGE == 0) v = L[q];
    else if (STAGE == 1) v = U[q * n + c] + h * L[q];
    else if (STAGE == 4) v = (3.0 * U0[q * n + c] + (U[q * n + c] + h * L[q])) / 4.0;
    else if (STAGE == 5) v = (U0[q * n + c] + 2.0 * (U[q * n + c] + h * L[q])) / 3.0;
    else v = 0.5 * (U0[q * n + c] + (U[q * n + c] + h * L[q]));
    out[q * n + c] = v;
  }
}

// k_update for an even nx, two cells along x per thread (i even, i + 1) in
// tiles of 128 x 4 cells: each array's values of the pair come as one
// two-wide load (aligned: n, the offsets and i are even), the x neighbour of
// the second cell as one more, so a wave issues half the loads and stores of
// k_update for the same bytes. The arithmetic per cell is that of k_update
// (bitwise equal results). Mixed mode (FP32 records): the XCD-grouped order.
struct PairTile {
  static constexpr int TX = 128, TY = 4, TZ = 1;
  static constexpr int NT = 256;
};
template <class T> struct Pair;
template <> struct Pair<double> { using V = double __attribute__((ext_vector_type(2))); };
template <> struct Pair<float> { using V = float __attribute__((ext_vector_type(2))); };
template <class T>
__device__ __forceinline__ typename Pair<T>::V ld2(const T* p, int64_t c) {
  return *reinterpret_cast<const typename Pair<T>::V*>(p + c);
}

template <int DIM, int STAGE, class R>
__global__ __launch_bounds__(PairTile::NT) void k_update2(const double* __restrict__ U,
                                                         const double* U0, double* out,
                                                         const double* __restrict__ FW,
                                                         const double* __restrict__ EW, Geom g,
                                                         TileGrid tg, double dt,
                                                         const double* __restrict__ dtp) {
  const unsigned t = (sizeof(R) == 4) ? xcd_grouped(blockIdx.x, gridDim.x) : blockIdx.x;
  const int tx = (int)(t % (unsigned)tg.ntx);
  const unsigned r = t / (unsigned)tg.ntx;
  const int ty = (int)(r % (unsigned)tg.nty);
  const int k = (int)(r / (unsigned)tg.nty);
  const int i = tx * PairTile::TX + 2 * ((int)threadIdx.x % 64);
  const int j = ty * PairTile::TY + (int)threadIdx.x / 64;
  if (i >= g.nx || j >= g.ny || k >= g.nz) return;
  const int64_t c = lin(g, i, j, k);
  const int64_t n = g.n;
  const double h = (STAGE == 0) ? 0.0 : (dtp ? *dtp : dt);
  const int64_t xq = lin(g, wrap(i + 2, g.nx), j, k);
  const int64_t yp = lin(g, i, wrap(j + 1, g.ny), k);
  const int64_t zp = (DIM == 3) ? lin(g, i, j, wrap(k + 1, g.nz)) : c;
  const double idx = 1.0 / g.dx, idy = 1.0 / g.dy, idz = 1.0 / g.dz;
  const R* fx = stored<R>(FW);
  const R* fy = fx + (int64_t)NSLOT * n;
  const R* fz = fx + (int64_t)2 * NSLOT * n;
  const R* ex = stored<R>(EW);
  const R* ey = ex + n;
  const R* ez = ex + 2 * n;
  double L[2][8];
  constexpr int ncell = (DIM == 3) ? 5 : 6;
#pragma unroll
  for (int qq = 0; qq < ncell; ++qq) {
    const typename Pair<R>::V ax = ld2(fx + qq * n, c), ay = ld2(fy + qq * n, c),
                              ayp = ld2(fy + qq * n, yp);
    const R axq = fx[qq * n + xq];
    typename Pair<R>::V az = {}, azp = {};
    if (DIM == 3) {
      az = ld2(fz + qq * n, c);
      azp = ld2(fz + qq * n, zp);
    }
    const double xc[3] = {(double)ax.x, (double)ax.y, (double)axq};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      double acc = (xc[e + 1] - xc[e]) * idx + ((double)(e ? ayp.y : ayp.x) - (double)(e ? ay.y : ay.x)) * idy;
      if (DIM == 3) acc += ((double)(e ? azp.y : azp.x) - (double)(e ? az.y : az.x)) * idz;
      L[e][qq == 5 ? 7 : qq] = -acc;
    }
  }
  {
    const typename Pair<R>::V zc = ld2(ez, c), zy = ld2(ez, yp);
    const R zq = ez[xq];
    const double ezc[3] = {(double)zc.x, (double)zc.y, (double)zq};
    if (DIM == 3) {
      const typename Pair<R>::V yc = ld2(ey, c), yz = ld2(ey, zp), xc2 = ld2(ex, c),
                                xy = ld2(ex, yp), xz = ld2(ex, zp);
      const R yq = ey[xq];
      const double eyc[3] = {(double)yc.x, (double)yc.y, (double)yq};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double exc = (double)(e ? xc2.y : xc2.x);
        L[e][5] = -(((double)(e ? zy.y : zy.x) - ezc[e]) * idy - ((double)(e ? yz.y : yz.x) - eyc[e]) * idz);
        L[e][6] = -(((double)(e ? xz.y : xz.x) - exc) * idz - (ezc[e + 1] - ezc[e]) * idx);
        L[e][7] = -((eyc[e + 1] - eyc[e]) * idx - ((double)(e ? xy.y : xy.x) - exc) * idy);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        L[e][5] = -(((double)(e ? zy.y : zy.x) - ezc[e]) * idy);
        L[e][6] = (ezc[e + 1] - ezc[e]) * idx;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    typename Pair<double>::V u = {}, u0 = {}, v;
    if (STAGE != 0) u = ld2(U + q * n, c);
    if (STAGE == 2 || STAGE == 4 || STAGE == 5) u0 = ld2(U0 + q * n, c);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double ue = e ? u.y : u.x, u0e = e ? u0.y : u0.x;
      double w;
      if (STAGE == 0) w = L[e][q];
      else if (STAGE == 1) w = ue + h * L[e][q];
      else if (STAGE == 4) w = (3.0 * u0e + (ue + h * L[e][q])) / 4.0;
      else if (STAGE == 5) w = (u0e + 2.0 * (ue + h * L[e][q])) / 3.0;
      else w = 0.5 * (u0e + (ue + h * L[e][q]));
      if (e) v.y = w; else v.x = w;
    }
    *reinterpret_cast<typename Pair<double>::V*>(out + q * n + c) = v;
  }
}

// LDS slot of a tile-relative cell position (at most one coordinate outside).
template <int DIM>
__device__ __forceinline__ int pslot(int x, int y, int z) {
  using T = Tile<DIM>;
  if (x < 0 || x >= T::TX) return T::NCORE + ((x < 0 ? x + 2 : 2) * T::TZ + z) * T::TY + y;
  if (y < 0 || y >= T::TY) return T::NCORE + T::HX + ((y < 0 ? y + 2 : 2) * T::TZ + z) * T::TX + x;
  if (DIM == 3 && (z < 0 || z >= T::TZ))
    return T::NCORE + T::HX + T::HY + ((z < 0 ? z + 2 : 2) * T::TY + y) * T::TX + x;
  return (z * T::TY + y) * T::TX + x;
}

// Inverse of pslot for the load loop.
template <int DIM>
__device__ __forceinline__ void pslot_pos(int e, int& x, int& y, int& z) {
  using T = Tile<DIM>;
  if (e < T::NCORE) {
    x = e % T::TX;
    y = (e / T::TX) % T::TY;
    z = e / (T::TX * T::TY);
    return;
  }
  e -= T::NCORE;
  if (e < T::HX) {
    y = e % T::TY;
    z = (e / T::TY) % T::TZ;
    const int s = e / (T::TY * T::TZ);
    x = (s == 0) ? -2 : (s == 1 ? -1 : T::TX);
    return;
  }
  e -= T::HX;
  if (e < T::HY) {
    x = e % T::TX;
    z = (e / T::TX) % T::TZ;
    const int s = e / (T::TX * T::TZ);
    y = (s == 0) ? -2 : (s == 1 ? -1 : T::TY);
    return;
  }
  e -= T::HY;
  x = e % T::TX;
  y = (e / T::TX) % T::TY;
  const int s = e / (T::TX * T::TY);
  z = (s == 0) ? -2 : (s == 1 ? -1 : T::TZ);
}

// One lower face of direction D of the tile cell (x,y,z) from LDS primitives.
template <int DIM, int D, int LIM, int RS, class R, int EM>
__device__ __forceinline__ void tile_face(const R (*sp)[Tile<DIM>::NPRIM], R bn,
                                          double* __restrict__ FW, const Geom& g, int x, int y,
                                          int z, int64_t c) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  int e[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int o = s - 2;
    e[s] = pslot<DIM>(x + (D == 0 ? o : 0), y + (D == 1 ? o : 0), z + (D == 2 ? o : 0));
  }
  R wl[7], wr[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const R* P = sp[slot[q]];
    const R a = P[e[0]], b = P[e[1]], cc = P[e[2]], d = P[e[3]];
    wl[q] = fma_r(R(0.5), plm_slope<LIM, R>(b - a, cc - b), b);
    wr[q] = fma_r(R(-0.5), plm_slope<LIM, R>(cc - b, d - cc), cc);
  }
  RiemannOut<R> o;
  riemann<RS, R, EM>((R)g.gamma, wl, wr, bn, o);
  put_record<DIM, D, EM, R>(FW, g.n, c, o);
}

// ---------------------------------------------------------------------------
// CFL bound of one cell from its FP64 primitives: min over directions of
// dx_d / (|v_d| + c_f,d), the expression of k_cfl.
__device__ __forceinline__ double cfl_bound(const Geom& g, const double* W, double m) {
  const double dd[3] = {g.dx, g.dy, g.dz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double cf = cfast<double>(g.gamma, W[0], W[4], W[5 + d], W[5 + (d + 1) % 3],
                                    W[5 + (d + 2) % 3]);
    const double t = dd[d] / (__builtin_fabs(W[1 + d]) + cf);
    m = (t < m) ? t : m;
  }
  return m;
}

// Minimum of v over the kBlock threads of the workgroup, stored by thread 0
// to *out. Every thread of the workgroup must call it.
__device__ __forceinline__ void workgroup_min_store(double v, double* __restrict__ out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = (o < v) ? o : v;
  }
  __shared__ double red[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) r = (red[w] < r) ? red[w] : r;
    *out = r;
  }
}

// Face kernel: primitives of the tile and its cross halo are recovered once
// (in FP64) into LDS, held in the reconstruction precision R, then each
// thread solves the lower x/y(/z) faces of its cell. cflp != nullptr: also
// the CFL bound of the state over the tile's own cells (the core, each cell
// the own cell of exactly one tile) into cflp[blockIdx.x]; k_cfl_final
// finishes it.
template <int DIM, int LIM, int RS, class R, int EM>
__global__ __launch_bounds__(Tile<DIM>::NCORE) void k_faces_tiled(const double* __restrict__ U,
                                                        double* __restrict__ FW, Geom g,
                                                        TileGrid tg, int* __restrict__ flag,
                                                        double* __restrict__ cflp) {
  static_assert(DIM == 2, "the 3D grid uses k_faces_march");
  using T = Tile<DIM>;
  static_assert(T::NCORE == kBlock, "workgroup_min_store reduces over kBlock threads");
  __shared__ R sp[8][T::NPRIM];
  int i0, j0, k0;
  tile_origin<DIM>(tg, blockIdx.x, i0, j0, k0);
  const int x = threadIdx.x % T::TX, y = (threadIdx.x / T::TX) % T::TY,
            z = threadIdx.x / (T::TX * T::TY);
  const int i = i0 + x, j = j0 + y, k = k0 + z;
  const bool inside = i < g.nx && j < g.ny && k < g.nz;
  // The normal fields of the cell's faces first (any in-bounds cell for a
  // thread outside the grid): loaded after the x-face records, waiting for
  // them would wait for those stores too.
  const int64_t c = lin(g, min(i, g.nx - 1), min(j, g.ny - 1), min(k, g.nz - 1));
  R bn[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) bn[d] = (R)U[(F_BX + d) * g.n + c];
  bool bad = false;
  double cmin = __builtin_inf();  // CFL bound of this thread's own cell
  for (int e = threadIdx.x; e < T::NPRIM; e += T::NCORE) {
    int x, y, z;
    pslot_pos<DIM>(e, x, y, z);
    double V[8];
    bad |= !prim_at<DIM>(U, g, wrap_any(i0 + x, g.nx), wrap_any(j0 + y, g.ny),
                         wrap_any(k0 + z, g.nz), V);
#pragma unroll
    for (int q = 0; q < 8; ++q) sp[q][e] = (R)V[q];
    // the core comes first, thread t's first entry is its own cell
    if (cflp && inside && e == (int)threadIdx.x) cmin = cfl_bound(g, V, cmin);
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  if (inside) {
    tile_face<DIM, 0, LIM, RS, R, EM>(sp, bn[0], FW, g, x, y, z, c);
    tile_face<DIM, 1, LIM, RS, R, EM>(sp, bn[1], FW, g, x, y, z, c);
    if (DIM == 3) tile_face<DIM, 2, LIM, RS, R, EM>(sp, bn[DIM - 1], FW, g, x, y, z, c);
  }
  if (cflp) workgroup_min_store(cmin, cflp + blockIdx.x);
}

// Cell of this thread when each workgroup of kBlock threads takes kBlock
// consecutive cells in storage order (x fastest; workgroups in the
// XCD-grouped order of xcd_grouped), so that no lane idles
// whatever nx is (row tiles of 64 leave 8% of the lanes idle at nx = 352).
// The configuration check keeps n below 2^32.
__device__ __forceinline__ bool linear_cell(const Geom& g, int& i, int& j, int& k, int64_t& c) {
  const uint32_t t = xcd_grouped(blockIdx.x, gridDim.x) * (uint32_t)kBlock + threadIdx.x;
  if ((int64_t)t >= g.n) return false;
  const uint32_t r = t / (uint32_t)g.nx;
  i = (int)(t - r * (uint32_t)g.nx);
  k = (int)(r / (uint32_t)g.ny);
  j = (int)(r - (uint32_t)k * (uint32_t)g.ny);
  c = t;
  return true;
}

// Primitive recovery for WENO-Z (FP64): every cell's primitives, in the order
// of prim_at, into PW[8][n], so that the face kernel reads each of the six
// cells of a stencil instead of recovering it again (each cell is in 18
// stencils in 3D). cflp != nullptr (3D): also the CFL bound of the state,
// reduced over the workgroup into cflp[blockIdx.x]; k_cfl_final finishes it.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_prim_weno(const double* __restrict__ U,
                                                 double* __restrict__ PW, Geom g,
                                                 int* __restrict__ flag,
                                                 double* __restrict__ cflp) {
  int i, j, k;
  int64_t c;
  const bool inside = linear_cell(g, i, j, k, c);
  double cmin = __builtin_inf();
  if (inside) {
    double V[8];
    const bool ok = prim_at<DIM>(U, g, i, j, k, V);
#pragma unroll
    for (int q = 0; q < 8; ++q) PW[q * g.n + c] = V[q];
    if (!ok) atomicOr(flag, 1);
    if (DIM == 3 && cflp) cmin = cfl_bound(g, V, cmin);
  }
  if (DIM == 3 && cflp) workgroup_min_store(cmin, cflp + blockIdx.x);
}

// Lower face of direction D of cell (i,j,k) with WENO-Z reconstruction (FP64)
// from the primitives PW of the six cells along D (offsets -3..+2): the left
// state is the upper value of cell -1 (cells -3..+1), the right state the
// lower value of cell 0 (cells +2..-2 in reverse). One quantity at a time, so
// that only its six values are live beside the reconstructed states.
template <int DIM, int D, int RS, int EM>
__device__ __forceinline__ void weno_face(const double* __restrict__ PW,
                                          const double* __restrict__ U, double* __restrict__ FW,
                                          const Geom& g, int i, int j, int k, int64_t c) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
  const int64_t n = g.n;
  int64_t cs[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int o = s - 3;
    cs[s] = lin(g, D == 0 ? wrap_any(i + o, g.nx) : i, D == 1 ? wrap_any(j + o, g.ny) : j,
                D == 2 ? wrap_any(k + o, g.nz) : k);
  }
  double v[7][6];
#pragma unroll
  for (int q = 0; q < 7; ++q)
#pragma unroll
    for (int s = 0; s < 6; ++s) v[q][s] = PW[slot[q] * n + cs[s]];
  const double bn = U[(F_BX + D) * n + c];
  __builtin_amdgcn_sched_barrier(0);
  double wl[7], wr[7];
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    wl[q] = wenoz_upper(v[q][0], v[q][1], v[q][2], v[q][3], v[q][4]);
    wr[q] = wenoz_upper(v[q][5], v[q][4], v[q][3], v[q][2], v[q][1]);
  }
  RiemannOut<double> o;
  riemann<RS, double, EM>(g.gamma, wl, wr, bn, o);
  put_record<DIM, D, EM, double>(FW, n, c, o);
}

// Face kernel for WENO-Z (2D and 3D, FP64), one cell per thread, kBlock
// consecutive cells per workgroup: its +-3-cell stencils are gathered from the
// primitives PW through the caches rather than staged in LDS (a z-march ring
// would need six planes and a 3-cell halo).
template <int DIM, int RS, int EM>
__global__ __launch_bounds__(kBlock) void k_faces_weno(const double* __restrict__ PW,
                                                  const double* __restrict__ U,
                                                  double* __restrict__ FW, Geom g) {
  int i, j, k;
  int64_t c;
  if (!linear_cell(g, i, j, k, c)) return;
  weno_face<DIM, 0, RS, EM>(PW, U, FW, g, i, j, k, c);
  weno_face<DIM, 1, RS, EM>(PW, U, FW, g, i, j, k, c);
  if (DIM == 3) weno_face<DIM, 2, RS, EM>(PW, U, FW, g, i, j, k, c);
}

// ---------------------------------------------------------------------------
// 3D face kernel marching along z. A workgroup owns a 64 x 4 column of cells
// and walks a run of planes k0 <= k < k1, one cell of each plane per thread.
// LDS holds the primitives of planes k-1, k, k+1 of the column (a ring of
// three) and the x/y cross halo (two cells below, one above) of planes k and
// k+1 (two buffers). The lower z-face of cell k takes its left state
// V_{k-1} + slope_{k-1}/2 from the previous plane's step, where the thread
// computed slope_{k-1} for the right state of the face below; each z slope is
// thus evaluated once. Per plane only the core of plane k+2 and the halo of
// plane k+1 are recovered. Their raw values are loaded before any face of
// plane k is solved, so that their latency hides behind the solves, and
// waiting for them never waits for the face records stored after them (the
// vector-memory counter retires in issue order); the normal fields of the
// faces come from raw cells loaded two planes earlier. Neighbours read only
// plane k of the ring and the current halo buffer, and a thread alone reads
// its own cells of planes k-1 and k+1, so the recovered plane k+2 (into the
// slot of plane k-1) and the halo of plane k+1 (into the other buffer) are
// written without waiting, and one barrier per plane publishes them.
// (Measured at 256^3 in FP64: 1.53 ms per launch against 1.65 ms for the
// same arithmetic with the loads issued after the records of the plane and
// two barriers per plane; 64 x 4 columns beat 16 x 16 ones, and dealing
// x-neighbour columns to one XCD is slower than the natural order.)
struct March {
  static constexpr int TX = 64, TY = 4, NCORE = TX * TY;
  static constexpr int NHALO = 3 * TY + 3 * TX;  // x-halo then y-halo
  static constexpr int NQ = 8;                   // primitives per cell: V slots 0..7
};
static_assert(March::NCORE == kBlock, "one column cell per thread");
static_assert(March::NHALO <= March::NCORE, "at most one halo cell per thread");

// Planes per run: the prologue costs two extra planes per run, shorter runs
// give more workgroups (4096 at 256^3 with 16; 16 measured faster than 32).
constexpr int kMarchRun = 16;
// Most CFL partials (2D tiles) that every workgroup of the first stage's
// update reduces itself instead of a k_cfl_final launch (1024: KH 512^2).
constexpr unsigned kUpdateCflMax = 1024;

// 73.5 KB in FP64: two workgroups (eight waves) per CU.
template <class R>
struct MarchLds {
  R ring[3][March::NQ][March::NCORE];   // planes by (k - k0 + 1) % 3
  R halo[2][March::NQ][March::NHALO];   // planes by (k - k0) & 1
};
// flat offsets (in R) of the parts
constexpr int kRingQ = March::NCORE;              // quantity stride in the ring
constexpr int kRingP = March::NQ * March::NCORE;  // plane stride in the ring
constexpr int kHaloOff = 3 * kRingP;
constexpr int kHaloB = March::NQ * March::NHALO;  // halo buffer stride

// Position of halo entry h of a plane, relative to the column origin;
// s = 0, 1, 2: two cells below the column, then one above.
__device__ __forceinline__ void march_halo_pos(int h, int& x, int& y) {
  if (h < 3 * March::TY) {
    const int s = h / March::TY;
    y = h % March::TY;
    x = (s < 2) ? s - 2 : March::TX;
  } else {
    h -= 3 * March::TY;
    const int s = h / March::TX;
    x = h % March::TX;
    y = (s < 2) ? s - 2 : March::TY;
  }
}

// Byte offsets within a plane of one field (FP64) of the values the primitive
// recovery of cell (i, j) reads (indices wrapped): the cell, and its upper x
// and y neighbours (staggered B_x, B_y). The staggered B_z above is the
// cell's own offset in the next plane. 32 bits: a plane holds fewer than
// 2^29 cells.
struct PlaneOffs {
  uint32_t c, xp, yp;
};
__device__ __forceinline__ PlaneOffs plane_offs(const Geom& g, int i, int j) {
  const int iw = wrap_any(i, g.nx), jw = wrap_any(j, g.ny);
  PlaneOffs p;
  p.c = (uint32_t)(jw * g.nx + iw) * 8u;
  p.xp = (uint32_t)(jw * g.nx + wrap(iw + 1, g.nx)) * 8u;
  p.yp = (uint32_t)(wrap(jw + 1, g.ny) * g.nx + iw) * 8u;
  return p;
}
// The value at byte offset off of the uniform base b.
__device__ __forceinline__ double ld_at(const double* __restrict__ b, uint32_t off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(b) + off);
}
// Raw values of the cell at offsets p in plane kw; the staggered B_z above
// from plane kw1 (both wrapped into 0..nz-1).
__device__ __forceinline__ RawCell load_raw_plane(const double* __restrict__ U, const Geom& g,
                                                  int64_t nxy, int kw, int kw1,
                                                  const PlaneOffs& p) {
  const double* pl = U + kw * nxy;
  RawCell r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r.u[q] = ld_at(pl + q * g.n, p.c);
  r.bxp = ld_at(pl + 5 * g.n, p.xp);
  r.byp = ld_at(pl + 6 * g.n, p.yp);
  r.bzp = ld_at(U + 7 * g.n + kw1 * nxy, p.c);
  return r;
}

// Primitives of a raw cell (FP64 recovery) rounded to R, into LDS at lds[o]
// with quantity stride st.
template <class R>
__device__ __forceinline__ bool march_recover(const RawCell& raw, double gamma, R* lds, int o,
                                              int st, double* W) {
  const bool ok = prim_from_raw<3>(raw, gamma, W);
#pragma unroll
  for (int q = 0; q < March::NQ; ++q) lds[o + q * st] = (R)W[q];
  return ok;
}

// Offsets of plane-k cell (xx, yy) (at most one coordinate outside the
// column): quantity q at lds[o + q * st]; r is the ring plane of k, hb its
// halo buffer.
__device__ __forceinline__ void march_xy(int r, int hb, int xx, int yy, int& o, int& st) {
  if (xx < 0 || xx >= March::TX || yy < 0 || yy >= March::TY) {
    const int h = (xx < 0 || xx >= March::TX)
                      ? ((xx < 0) ? xx + 2 : 2) * March::TY + yy
                      : 3 * March::TY + ((yy < 0) ? yy + 2 : 2) * March::TX + xx;
    o = kHaloOff + hb * kHaloB + h;
    st = March::NHALO;
  } else {
    o = r * kRingP + yy * March::TX + xx;
    st = kRingQ;
  }
}

// Writes the nine records of a lower face of the plane whose records start
// at fwp (slot 0 of direction 0), the cell at byte offset boff.
template <int D, int EM, class R>
__device__ __forceinline__ void put_record_at(R* __restrict__ fwp, int64_t n, uint32_t boff,
                                              const RiemannOut<R>& o) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  auto put = [&](int slot, R v) {
    *reinterpret_cast<R*>(reinterpret_cast<char*>(fwp + ((int64_t)D * NSLOT + slot) * n) +
                          boff) = v;
  };
  put(S_RHO, o.f[0]);
  put(S_MX + D, o.f[1]);
  put(S_MX + T1, o.f[2]);
  put(S_MX + T2, o.f[3]);
  put(S_EN, o.f[6]);
  if (EM == 1) {
    put(S_AP, o.om);
    put(S_AM, o.dl);
    put(S_DR, o.dr);
  } else {
    put(S_AP, o.ap);
    put(S_AM, o.am);
  }
  put(S_V1, o.v1);
  put(S_V2, o.v2);
}

template <int D, int RS, class R, int EM>
__device__ __forceinline__ void march_solve(const R* wl, const R* wr, R bn, R gamma,
                                            R* __restrict__ fwp, int64_t n, uint32_t boff) {
  RiemannOut<R> o;
  riemann<RS, R, EM>(gamma, wl, wr, bn, o);
  put_record_at<D, EM, R>(fwp, n, boff, o);
}

// Reconstructed states of the lower x (D = 0) or y (D = 1) face of a cell of
// plane k: PLM over the four stencil cells (offsets o*, strides s*).
template <int D, int LIM, class R>
__device__ __forceinline__ void march_recon_xy(const R* lds, const int* o, const int* st, R* wl,
                                               R* wr) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr int slot[7] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4};
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int sq = slot[q];
    R v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = lds[o[s] + sq * st[s]];
    wl[q] = fma_r(R(0.5), plm_slope<LIM, R>(v[1] - v[0], v[2] - v[1]), v[1]);
    wr[q] = fma_r(R(-0.5), plm_slope<LIM, R>(v[2] - v[1], v[3] - v[2]), v[2]);
  }
}

// cflp != nullptr: also the CFL bound of the state, reduced over the cells
// of this workgroup's column and run (each cell is the own cell of exactly
// one workgroup and plane) into cflp[blockIdx.x]; k_cfl_final finishes it.
// FULL: every column lies inside the grid (nx % 64 == 0, ny % 4 == 0), so no
// thread skips the faces. Then every path through a plane issues the same
// loads and stores, and the waits for the prefetched cells count exactly the
// stores issued after them (no skipped-faces path forces waiting for the
// stores as well).
template <int LIM, int RS, class R, int EM, bool FULL>
__global__ __launch_bounds__(kBlock)
void k_faces_march(const double* __restrict__ U, double* __restrict__ FW, Geom g, MarchGrid mg,
                   int* __restrict__ flag, double* __restrict__ cflp) {
  // slots of the z-face frame (rho, v_z, v_x, v_y, B_x, B_y, p)
  constexpr int zslot[7] = {0, 3, 1, 2, 5, 6, 4};
  __shared__ MarchLds<R> L;
  R* lds = &L.ring[0][0][0];
  const unsigned b = blockIdx.x;
  const int tx = (int)(b % (unsigned)mg.ntx);
  const unsigned r = b / (unsigned)mg.ntx;
  const int ty = (int)(r % (unsigned)mg.nty);
  const int zc = (int)(r / (unsigned)mg.nty);
  const int i0 = tx * March::TX, j0 = ty * March::TY;
  const int k0 = zc * mg.lz;
  const int k1 = min(k0 + mg.lz, g.nz);
  const int x = (int)threadIdx.x % March::TX, y = (int)threadIdx.x / March::TX;
  const int cidx = y * March::TX + x;
  const int i = i0 + x, j = j0 + y;
  const bool inside = FULL || ((i < g.nx) && (j < g.ny));
  const int64_t nxy = (int64_t)g.nx * g.ny;
  const R gam = (R)g.gamma;
  // own cell; halo cell (threads past the halo load a valid cell and drop it)
  const PlaneOffs po = plane_offs(g, i, j);
  const bool haloer = (int)threadIdx.x < March::NHALO;
  int hx, hy;
  march_halo_pos(haloer ? (int)threadIdx.x : March::NHALO - 1, hx, hy);
  const PlaneOffs ph = plane_offs(g, i0 + hx, j0 + hy);
  bool bad = false;
  // Prologue: own cells of planes k0-2 .. k0+1, the ring gets k0-1, k0,
  // k0+1 (slots 0, 1, 2), halo buffer 0 the halo of plane k0; the left state
  // of the first z-face. The staggered normal fields of the own cell (the
  // raw B of its lower faces) of planes k and k+1 are carried in registers:
  // each plane's are taken from the raw cell loaded two planes earlier.
  R zl[7];
  double cmin = __builtin_inf();  // CFL bound over this thread's own cells
  double bn0[3], bn1[3];          // normal fields of planes k, k+1
  {
    const int km2 = wrap_any(k0 - 2, g.nz), km1 = wrap_any(k0 - 1, g.nz);
    const int kp1 = wrap_any(k0 + 1, g.nz), kp2 = wrap_any(k0 + 2, g.nz);
    double Wm2[8], Wm1[8], W[8];
    bad |= !prim_from_raw<3>(load_raw_plane(U, g, nxy, km2, km1, po), g.gamma, Wm2);
    bad |= !march_recover<R>(load_raw_plane(U, g, nxy, km1, k0, po), g.gamma, lds,
                             0 * kRingP + cidx, kRingQ, Wm1);
    R zm2[7], zm1[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      zm2[q] = (R)Wm2[zslot[q]];
      zm1[q] = (R)Wm1[zslot[q]];
    }
    const RawCell c0 = load_raw_plane(U, g, nxy, k0, kp1, po);
    bad |= !march_recover<R>(c0, g.gamma, lds, 1 * kRingP + cidx, kRingQ, W);
    if (cflp && inside) cmin = cfl_bound(g, W, cmin);
#pragma unroll
    for (int q = 0; q < 7; ++q)
      zl[q] = fma_r(R(0.5), plm_slope<LIM, R>(zm1[q] - zm2[q], (R)W[zslot[q]] - zm1[q]), zm1[q]);
    const RawCell c1 = load_raw_plane(U, g, nxy, kp1, kp2, po);
    bad |= !march_recover<R>(c1, g.gamma, lds, 2 * kRingP + cidx, kRingQ, W);
    if (cflp && inside && k0 + 1 < k1) cmin = cfl_bound(g, W, cmin);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      bn0[d] = c0.u[5 + d];
      bn1[d] = c1.u[5 + d];
    }
    if (haloer)
      bad |= !march_recover<R>(load_raw_plane(U, g, nxy, k0, kp1, ph), g.gamma, lds,
                               kHaloOff + (int)threadIdx.x, March::NHALO, W);
  }
  __syncthreads();
  int rm = 0, r0 = 1, rp = 2, hb = 0;
  R* const fw0 = stored<R>(FW);
  const uint32_t boff = (uint32_t)(j * g.nx + i) * (uint32_t)sizeof(R);  // valid when inside
  for (int k = k0; k < k1; ++k) {
    const bool more = k + 1 < k1;
    // The raw halo cell of plane k+1 and the raw own cell of plane k+2,
    // loaded by every thread (in-bounds, wrapped indices) before any face
    // record of this plane is stored.
    const int ka = wrap_any(k + 1, g.nz), kb = wrap_any(k + 2, g.nz), kc = wrap_any(k + 3, g.nz);
    const RawCell hr = load_raw_plane(U, g, nxy, ka, kb, ph);
    const RawCell nxt = load_raw_plane(U, g, nxy, kb, kc, po);
    R* const fwp = fw0 + k * nxy;
    R wl[7], wr[7];
    int o[4], st[4];
    if (inside) {
      march_xy(r0, hb, x - 2, y, o[0], st[0]);
      march_xy(r0, hb, x - 1, y, o[1], st[1]);
      march_xy(r0, hb, x, y, o[2], st[2]);
      march_xy(r0, hb, x + 1, y, o[3], st[3]);
      march_recon_xy<0, LIM, R>(lds, o, st, wl, wr);
    }
    // the halo of plane k+1 into the other buffer (read by no one before the
    // barrier below), once the x reconstruction has covered its latency
    if (more && haloer) {
      double W[8];
      bad |= !march_recover<R>(hr, g.gamma, lds, kHaloOff + (hb ^ 1) * kHaloB + (int)threadIdx.x,
                               March::NHALO, W);
    }
    if (inside) {
      march_solve<0, RS, R, EM>(wl, wr, (R)bn0[0], gam, fwp, g.n, boff);
      march_xy(r0, hb, x, y - 2, o[0], st[0]);
      march_xy(r0, hb, x, y - 1, o[1], st[1]);
      march_xy(r0, hb, x, y + 1, o[3], st[3]);
      march_recon_xy<1, LIM, R>(lds, o, st, wl, wr);
      march_solve<1, RS, R, EM>(wl, wr, (R)bn0[1], gam, fwp, g.n, boff);
      // z face: left state carried from the plane below; the slope of cell k
      // gives the right state and the next plane's left state
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        const int sq = zslot[q];
        const R a = lds[rm * kRingP + sq * kRingQ + cidx];
        const R bb = lds[r0 * kRingP + sq * kRingQ + cidx];
        const R cc = lds[rp * kRingP + sq * kRingQ + cidx];
        const R dlt = plm_slope<LIM, R>(bb - a, cc - bb);
        wl[q] = zl[q];
        wr[q] = fma_r(R(-0.5), dlt, bb);
        zl[q] = fma_r(R(0.5), dlt, bb);
      }
      march_solve<2, RS, R, EM>(wl, wr, (R)bn0[2], gam, fwp, g.n, boff);
    }
    if (more) {
      // plane k+2 into the ring slot of plane k-1 (own cell, read by no
      // other thread)
      double W[8];
      bad |= !march_recover<R>(nxt, g.gamma, lds, rm * kRingP + cidx, kRingQ, W);
      if (cflp && inside && k + 2 < k1) cmin = cfl_bound(g, W, cmin);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bn0[d] = bn1[d];
        bn1[d] = nxt.u[5 + d];
      }
      __syncthreads();
    }
    const int t = rm;
    rm = r0;
    r0 = rp;
    rp = t;
    hb ^= 1;
  }
  if (cflp) workgroup_min_store(cmin, cflp + blockIdx.x);
  if (bad) atomicOr(flag, 1);
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

// ---------------------------------------------------------------------------
// GLM divergence cleaning (Sec. 2.1 lists it beside CT; Dedner et al. 2002),
// mixed form: nine cell-centred fields (rho, m_x, m_y, m_z, E, B_x, B_y, B_z,
// psi), psi coupled to B by dB/dt + grad psi and dpsi/dt + c_h^2 div B, its
// damping applied after each full step. One stage is three launches over
// kBlock consecutive cells per workgroup: primitives of every cell (and the
// CFL partials), faces (each cell's three lower faces from the primitives of
// its stencil), update (flux divergence of the nine fields, RK combination,
// the damping of psi in the last stage).
constexpr int kGlmFields = 9;

template <int DIM>
__device__ __forceinline__ double cfl_bound_dim(const Geom& g, const double* W, double m) {
  const double dd[3] = {g.dx, g.dy, g.dz};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double cf = cfast<double>(g.gamma, W[0], W[4], W[5 + d], W[5 + (d + 1) % 3],
                                    W[5 + (d + 2) % 3]);
    const double t = dd[d] / (__builtin_fabs(W[1 + d]) + cf);
    m = (t < m) ? t : m;
  }
  return m;
}

// Primitives (rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi) of every cell into
// PW[9][n] (FP64; the field is already cell-centred), the workgroup's CFL
// partial into cflp[blockIdx.x] (nullable).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_glm_prim(const double* __restrict__ U,
                                                double* __restrict__ PW, Geom g,
                                                int* __restrict__ flag,
                                                double* __restrict__ cflp) {
  int i, j, k;
  int64_t c;
  const bool inside = linear_cell(g, i, j, k, c);
  double cmin = __builtin_inf();
  if (inside) {
    const int64_t n = g.n;
    const double rho = U[c];
    const double mx = U[n + c], my = U[2 * n + c], mz = U[3 * n + c], en = U[4 * n + c];
    const double bx = U[5 * n + c], by = U[6 * n + c], bz = U[7 * n + c];
    const double irho = 1.0 / rho;
    const double vx = mx * irho, vy = my * irho, vz = mz * irho;
    const double kin = 0.5 * fma_r(mz, vz, fma_r(my, vy, mx * vx));
    const double mag = 0.5 * fma_r(bz, bz, fma_r(by, by, bx * bx));
    const double p = (g.gamma - 1.0) * (en - kin - mag);
    const double V[9] = {rho, vx, vy, vz, p, bx, by, bz, U[8 * n + c]};
#pragma unroll
    for (int q = 0; q < kGlmFields; ++q) PW[q * n + c] = V[q];
    const bool ok = (rho > 0.0) && (p > 0.0) && __builtin_isfinite(p) &&
                    __builtin_isfinite(vx) && __builtin_isfinite(vy) && __builtin_isfinite(vz);
    if (!ok) atomicOr(flag, 1);
    if (cflp) cmin = cfl_bound_dim<DIM>(g, V, cmin);
  }
  if (cflp) workgroup_min_store(cmin, cflp + blockIdx.x);
}

// Lower D-face of cell (i,j,k): the nine quantities reconstructed from the
// primitives along D (PLM over offsets -2..+1, or WENO-Z over -3..+2), then
// the (B_n, psi) subsystem's exact interface values
//   bn* = (bn_L + bn_R)/2 - (psi_R - psi_L)/(2 c_h),
//   psi* = (psi_L + psi_R)/2 - c_h (bn_R - bn_L)/2,
// the MHD Riemann flux with the normal field bn*, and the fluxes psi* of B_n
// and c_h^2 bn* of psi; written in global components to FW[D][9][n].
template <int DIM, int D, int LIM, int RS, class R>
__device__ __forceinline__ void glm_face(const double* __restrict__ PW, double* __restrict__ FW,
                                         const Geom& g, int i, int j, int k, int64_t c, R ch) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  // face frame (rho, v_n, v_t1, v_t2, B_t1, B_t2, p), then B_n and psi
  constexpr int slot[9] = {0, 1 + D, 1 + T1, 1 + T2, 5 + T1, 5 + T2, 4, 5 + D, 8};
  constexpr int NS = (LIM == 2) ? 6 : 4, O0 = (LIM == 2) ? 3 : 2;
  const int64_t n = g.n;
  int64_t cs[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int o = s - O0;
    cs[s] = lin(g, D == 0 ? wrap_any(i + o, g.nx) : i, D == 1 ? wrap_any(j + o, g.ny) : j,
                D == 2 ? wrap_any(k + o, g.nz) : k);
  }
  // the stencil's 9 x NS primitives are all loaded before a scheduling
  // barrier (one wait per face instead of one per quantity)
  double pv[9][NS];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int s = 0; s < NS; ++s) pv[q][s] = PW[slot[q] * n + cs[s]];
  __builtin_amdgcn_sched_barrier(0);
  R wl[9], wr[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double* v8 = pv[q];
    if constexpr (LIM == 2) {
      wl[q] = (R)wenoz_upper(v8[0], v8[1], v8[2], v8[3], v8[4]);
      wr[q] = (R)wenoz_upper(v8[5], v8[4], v8[3], v8[2], v8[1]);
    } else {
      R v[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = (R)v8[s];
      wl[q] = fma_r(R(0.5), plm_slope<LIM, R>(v[1] - v[0], v[2] - v[1]), v[1]);
      wr[q] = fma_r(R(-0.5), plm_slope<LIM, R>(v[2] - v[1], v[3] - v[2]), v[2]);
    }
  }
  const R bns = R(0.5) * (wl[7] + wr[7]) - div_r(wr[8] - wl[8], R(2) * ch);
  const R psis = R(0.5) * (wl[8] + wr[8]) - R(0.5) * ch * (wr[7] - wl[7]);
  RiemannOut<R> o;
  riemann<RS, R>((R)g.gamma, wl, wr, bns, o);
  R* fw = stored<R>(FW) + (int64_t)D * kGlmFields * n + c;
  fw[0 * n] = o.f[0];
  fw[(1 + D) * n] = o.f[1];
  fw[(1 + T1) * n] = o.f[2];
  fw[(1 + T2) * n] = o.f[3];
  fw[4 * n] = o.f[6];
  fw[(5 + T1) * n] = o.f[4];
  fw[(5 + T2) * n] = o.f[5];
  fw[(5 + D) * n] = psis;
  fw[8 * n] = ch * ch * bns;
}

// c_h = C Delta_min / dt, the largest speed the step's time step allows.
template <int DIM, int LIM, int RS, class R>
__global__ __launch_bounds__(kBlock) void k_glm_faces(const double* __restrict__ PW,
                                                 double* __restrict__ FW, Geom g, double cfl,
                                                 double dmin, double dt,
                                                 const double* __restrict__ dtp) {
  int i, j, k;
  int64_t c;
  if (!linear_cell(g, i, j, k, c)) return;
  const double h = dtp ? *dtp : dt;
  const R ch = (R)(cfl * dmin / h);
  glm_face<DIM, 0, LIM, RS, R>(PW, FW, g, i, j, k, c, ch);
  glm_face<DIM, 1, LIM, RS, R>(PW, FW, g, i, j, k, c, ch);
  if (DIM == 3) glm_face<DIM, 2, LIM, RS, R>(PW, FW, g, i, j, k, c, ch);
}

// STAGE as in k_update (0: out = L(U); 1, 2: SSP-RK2; 1, 4, 5: SSP-RK3); in
// the last stage of a step (2 or 5) psi is multiplied by the damping factor
// exp(-alpha c_h dt / Delta_min).
template <int DIM, int STAGE, class R>
__global__ __launch_bounds__(kBlock) void k_glm_update(const double* __restrict__ U,
                                                  const double* U0, double* out,
                                                  const double* __restrict__ FW, Geom g,
                                                  double dt, const double* __restrict__ dtp,
                                                  double decay) {
  int i, j, k;
  int64_t c;
  if (!linear_cell(g, i, j, k, c)) return;
  const int64_t n = g.n;
  const double h = (STAGE == 0) ? 0.0 : (dtp ? *dtp : dt);
  const int64_t xp = lin(g, wrap(i + 1, g.nx), j, k);
  const int64_t yp = lin(g, i, wrap(j + 1, g.ny), k);
  const int64_t zp = (DIM == 3) ? lin(g, i, j, wrap(k + 1, g.nz)) : c;
  const double idx = 1.0 / g.dx, idy = 1.0 / g.dy, idz = 1.0 / g.dz;
  const R* fx = stored<R>(FW);
  const R* fy = fx + (int64_t)kGlmFields * n;
  const R* fz = fx + (int64_t)2 * kGlmFields * n;
#pragma unroll
  for (int q = 0; q < kGlmFields; ++q) {
    double acc = ((double)fx[q * n + xp] - (double)fx[q * n + c]) * idx +
                 ((double)fy[q * n + yp] - (double)fy[q * n + c]) * idy;
    if (DIM == 3) acc += ((double)fz[q * n + zp] - (double)fz[q * n + c]) * idz;
    const double Lq = -acc;
    double v;
    if (STAGE == 0) v = Lq;
    else if (STAGE == 1) v = U[q * n + c] + h * Lq;
    else if (STAGE == 4) v = (3.0 * U0[q * n + c] + (U[q * n + c] + h * Lq)) / 4.0;
    else if (STAGE == 5) v = (U0[q * n + c] + 2.0 * (U[q * n + c] + h * Lq)) / 3.0;
    else v = 0.5 * (U0[q * n + c] + (U[q * n + c] + h * Lq));
    if ((STAGE == 2 || STAGE == 5) && q == 8) v = v * decay;
    out[q * n + c] = v;
  }
}

template <int DIM, int LIM, int RS, class R>
hipError_t glm_stage_impl(const StageArgs& a) {
  const unsigned nl = (unsigned)((a.g.n + kBlock - 1) / kBlock);
  if (!a.PW) return hipErrorInvalidValue;
  MHD_TIMED(a, K_PRIM,
            hipLaunchKernelGGL((k_glm_prim<DIM>), dim3(nl), dim3(kBlock), 0, a.stream, a.U, a.PW,
                               a.g, a.flag, a.cfl_partial));
  if (a.cfl_partial)  // dt of the state U, before the faces read it
    MHD_TIMED(a, K_CFL_FINAL,
              hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, a.cfl_partial,
                                 (int)nl, a.cfl, a.dt_out));
  MHD_TIMED(a, K_FACES,
            hipLaunchKernelGGL((k_glm_faces<DIM, LIM, RS, R>), dim3(nl), dim3(kBlock), 0, a.stream,
                               a.PW, a.FW, a.g, a.cfl, a.glm_dmin, a.dt, a.dtp));
#define MHD_GLM_UPD(ST)                                                                      \
  MHD_TIMED(a, K_UPDATE,                                                                     \
            hipLaunchKernelGGL((k_glm_update<DIM, ST, R>), dim3(nl), dim3(kBlock), 0, a.stream, \
                               a.U, a.U0, a.out, a.FW, a.g, a.dt, a.dtp, a.glm_decay))
  switch (a.stage) {
    case 0: MHD_GLM_UPD(0); break;
    case 1: MHD_GLM_UPD(1); break;
    case 4: MHD_GLM_UPD(4); break;
    case 5: MHD_GLM_UPD(5); break;
    default: MHD_GLM_UPD(2); break;
  }
#undef MHD_GLM_UPD
  return hipGetLastError();
}

template <int DIM>
hipError_t glm_stage_lim(const StageArgs& a) {
  const bool mixed = a.precision == 1;
  if (a.limiter == 2) {
    if (mixed) return hipErrorInvalidValue;
    return a.riemann == 0 ? glm_stage_impl<DIM, 2, 0, double>(a)
                          : glm_stage_impl<DIM, 2, 1, double>(a);
  }
  if (a.limiter == 0) {
    if (a.riemann == 0)
      return mixed ? glm_stage_impl<DIM, 0, 0, float>(a) : glm_stage_impl<DIM, 0, 0, double>(a);
    return mixed ? glm_stage_impl<DIM, 0, 1, float>(a) : glm_stage_impl<DIM, 0, 1, double>(a);
  }
  if (a.riemann == 0)
    return mixed ? glm_stage_impl<DIM, 1, 0, float>(a) : glm_stage_impl<DIM, 1, 0, double>(a);
  return mixed ? glm_stage_impl<DIM, 1, 1, float>(a) : glm_stage_impl<DIM, 1, 1, double>(a);
}


template <class T>
TileGrid tile_grid(const Geom& g) {
  TileGrid tg;
  tg.ntx = (g.nx + T::TX - 1) / T::TX;
  tg.nty = (g.ny + T::TY - 1) / T::TY;
  tg.ntz = (g.nz + T::TZ - 1) / T::TZ;
  tg.ntiles = (unsigned)tg.ntx * (unsigned)tg.nty * (unsigned)tg.ntz;
  return tg;
}

MarchGrid march_grid(const Geom& g) {
  MarchGrid mg;
  mg.ntx = (g.nx + March::TX - 1) / March::TX;
  mg.nty = (g.ny + March::TY - 1) / March::TY;
  mg.lz = g.nz < kMarchRun ? g.nz : kMarchRun;
  mg.nzc = (g.nz + mg.lz - 1) / mg.lz;
  mg.nblocks = (unsigned)mg.ntx * (unsigned)mg.nty * (unsigned)mg.nzc;
  return mg;
}

template <int DIM, int LIM, int RS, class R, int EM>
hipError_t stage_impl(const StageArgs& a) {
  // LIM 2 (WENO-Z, FP64): faces by k_faces_weno, edge values by van Leer PLM
  constexpr int ELIM = (LIM == 2) ? 1 : LIM;
  const TileGrid rg = tile_grid<RowTile>(a.g);
  const unsigned nb = rg.ntiles;
  if constexpr (LIM == 2) {
    static_assert(sizeof(R) == 8, "WENO-Z runs in FP64");
    if (!a.PW || (DIM == 2 && a.cfl_partial)) return hipErrorInvalidValue;
    const unsigned nl = (unsigned)((a.g.n + kBlock - 1) / kBlock);
    MHD_TIMED(a, K_PRIM,
              hipLaunchKernelGGL((k_prim_weno<DIM>), dim3(nl), dim3(kBlock), 0, a.stream, a.U,
                                 a.PW, a.g, a.flag, a.cfl_partial));
    if (a.cfl_partial)  // dt of the state U, before the update kernel reads it
      MHD_TIMED(a, K_CFL_FINAL,
                hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, a.cfl_partial,
                                   (int)nl, a.cfl, a.dt_out));
    MHD_TIMED(a, K_FACES,
              hipLaunchKernelGGL((k_faces_weno<DIM, RS, EM>), dim3(nl), dim3(kBlock), 0, a.stream,
                                 a.PW, a.U, a.FW, a.g));
  } else if constexpr (DIM == 3) {
    const MarchGrid mg = march_grid(a.g);
    if (a.g.nx % March::TX == 0 && a.g.ny % March::TY == 0)
      MHD_TIMED(a, K_FACES,
                hipLaunchKernelGGL((k_faces_march<LIM, RS, R, EM, true>), dim3(mg.nblocks),
                                   dim3(kBlock), 0, a.stream, a.U, a.FW, a.g, mg, a.flag,
                                   a.cfl_partial));
    else
      MHD_TIMED(a, K_FACES,
                hipLaunchKernelGGL((k_faces_march<LIM, RS, R, EM, false>), dim3(mg.nblocks),
                                   dim3(kBlock), 0, a.stream, a.U, a.FW, a.g, mg, a.flag,
                                   a.cfl_partial));
    if (a.cfl_partial)  // dt of the state U, before the update kernels read it
      MHD_TIMED(a, K_CFL_FINAL,
                hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, a.cfl_partial,
                                   (int)mg.nblocks, a.cfl, a.dt_out));
  } else {
    const TileGrid tg = tile_grid<Tile<DIM>>(a.g);
    MHD_TIMED(a, K_FACES,
              hipLaunchKernelGGL((k_faces_tiled<DIM, LIM, RS, R, EM>), dim3(tg.ntiles),
                                 dim3(Tile<DIM>::NCORE), 0, a.stream, a.U, a.FW, a.g, tg, a.flag,
                                 a.cfl_partial));
    // dt of the state U before the update reads it: for a few partials the
    // update's workgroups reduce them themselves, else k_cfl_final
    if (a.cfl_partial && tg.ntiles > kUpdateCflMax)
      MHD_TIMED(a, K_CFL_FINAL,
                hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, a.cfl_partial,
                                   (int)tg.ntiles, a.cfl, a.dt_out));
  }
  if constexpr (DIM == 3) {
    MarchGrid eg;
    eg.ntx = (a.g.nx + EmfCol::TX - 1) / EmfCol::TX;
    eg.nty = (a.g.ny + EmfCol::TY - 1) / EmfCol::TY;
    eg.lz = a.g.nz < kMarchRun ? a.g.nz : kMarchRun;
    eg.nzc = (a.g.nz + eg.lz - 1) / eg.lz;
    eg.nblocks = (unsigned)eg.ntx * (unsigned)eg.nty * (unsigned)eg.nzc;
    if constexpr (EM == 1)
      MHD_TIMED(a, K_EMF,
                hipLaunchKernelGGL((k_emf_march_hlld<ELIM, R>), dim3(eg.nblocks),
                                   dim3(EmfCol::NT), 0, a.stream, a.U, a.FW, a.EW, a.g, eg));
    else
      MHD_TIMED(a, K_EMF,
                hipLaunchKernelGGL((k_emf_march<ELIM, R>), dim3(eg.nblocks), dim3(EmfCol::NT), 0,
                                   a.stream, a.U, a.FW, a.EW, a.g, eg));
  } else if (a.stage == 3) {  // 2D records only; the 2D stages fuse the EMF into the update
    MHD_TIMED(a, K_EMF,
              hipLaunchKernelGGL((k_emf<DIM, ELIM, R, EM>), dim3(nb), dim3(RowTile::NT), 0, a.stream, a.U,
                                 a.FW, a.EW, a.g, rg));
  }
  if constexpr (DIM == 2) {
    // the stage-1 CFL partials of the tiled face kernel, when few
    const unsigned ntile = tile_grid<Tile<DIM>>(a.g).ntiles;
    const double* ucfl = (a.cfl_partial && ntile <= kUpdateCflMax) ? a.cfl_partial : nullptr;
    const int unp = (int)ntile;
    switch (a.stage) {
      case 3:
        break;
      case 0:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_emf_update_2d<ELIM, 0, R, EM>), dim3(nb), dim3(RowTile::NT),
                                     0, a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt,
                                     a.dtp, ucfl, unp, a.cfl, a.dt_out));
        break;
      case 1:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_emf_update_2d<ELIM, 1, R, EM>), dim3(nb), dim3(RowTile::NT),
                                     0, a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt,
                                     a.dtp, ucfl, unp, a.cfl, a.dt_out));
        break;
      case 4:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_emf_update_2d<ELIM, 4, R, EM>), dim3(nb), dim3(RowTile::NT),
                                     0, a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt,
                                     a.dtp, ucfl, unp, a.cfl, a.dt_out));
        break;
      case 5:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_emf_update_2d<ELIM, 5, R, EM>), dim3(nb), dim3(RowTile::NT),
                                     0, a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt,
                                     a.dtp, ucfl, unp, a.cfl, a.dt_out));
        break;
      default:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_emf_update_2d<ELIM, 2, R, EM>), dim3(nb), dim3(RowTile::NT),
                                     0, a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt,
                                     a.dtp, ucfl, unp, a.cfl, a.dt_out));
        break;
    }
    return hipGetLastError();
  } else {
    if (a.g.nx % 2 == 0 && a.stage != 3) {
      // even nx: the two-cell update (measured 0.979 -> 0.959 ms at 256^3 and
      // 2.74 -> 2.56 ms at 352^3, FP64)
      const TileGrid pg = tile_grid<PairTile>(a.g);
      const unsigned pb = pg.ntiles;
      switch (a.stage) {
        case 0:
          MHD_TIMED(a, K_UPDATE,
                    hipLaunchKernelGGL((k_update2<DIM, 0, R>), dim3(pb), dim3(PairTile::NT), 0,
                                       a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, pg, a.dt, a.dtp));
          break;
        case 1:
          MHD_TIMED(a, K_UPDATE,
                    hipLaunchKernelGGL((k_update2<DIM, 1, R>), dim3(pb), dim3(PairTile::NT), 0,
                                       a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, pg, a.dt, a.dtp));
          break;
        case 4:
          MHD_TIMED(a, K_UPDATE,
                    hipLaunchKernelGGL((k_update2<DIM, 4, R>), dim3(pb), dim3(PairTile::NT), 0,
                                       a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, pg, a.dt, a.dtp));
          break;
        case 5:
          MHD_TIMED(a, K_UPDATE,
                    hipLaunchKernelGGL((k_update2<DIM, 5, R>), dim3(pb), dim3(PairTile::NT), 0,
                                       a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, pg, a.dt, a.dtp));
          break;
        default:
          MHD_TIMED(a, K_UPDATE,
                    hipLaunchKernelGGL((k_update2<DIM, 2, R>), dim3(pb), dim3(PairTile::NT), 0,
                                       a.stream, a.U, a.U0, a.out, a.FW, a.EW, a.g, pg, a.dt, a.dtp));
          break;
      }
      return hipGetLastError();
    }
    switch (a.stage) {
      case 3:  // face and edge records only (the adjoint's forward recompute)
        break;
      case 0:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_update<DIM, 0, R>), dim3(nb), dim3(RowTile::NT), 0, a.stream, a.U,
                                     a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt, a.dtp));
        break;
      case 1:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_update<DIM, 1, R>), dim3(nb), dim3(RowTile::NT), 0, a.stream, a.U,
                                     a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt, a.dtp));
        break;
      case 4:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_update<DIM, 4, R>), dim3(nb), dim3(RowTile::NT), 0, a.stream, a.U,
                                     a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt, a.dtp));
        break;
      case 5:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_update<DIM, 5, R>), dim3(nb), dim3(RowTile::NT), 0, a.stream, a.U,
                                     a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt, a.dtp));
        break;
      default:
        MHD_TIMED(a, K_UPDATE,
                  hipLaunchKernelGGL((k_update<DIM, 2, R>), dim3(nb), dim3(RowTile::NT), 0, a.stream, a.U,
                                     a.U0, a.out, a.FW, a.EW, a.g, rg, a.dt, a.dtp));
        break;
    }
    return hipGetLastError();
  }
}

template <int DIM, int EM>
hipError_t stage_lim(const StageArgs& a) {
  const bool mixed = a.precision == 1;
  if (a.limiter == 2) {  // WENO-Z: FP64 only
    if (mixed) return hipErrorInvalidValue;
    return a.riemann == 0 ? stage_impl<DIM, 2, 0, double, EM>(a)
                          : stage_impl<DIM, 2, 1, double, EM>(a);
  }
  if (a.limiter == 0) {
    if (a.riemann == 0)
      return mixed ? stage_impl<DIM, 0, 0, float, EM>(a) : stage_impl<DIM, 0, 0, double, EM>(a);
    return mixed ? stage_impl<DIM, 0, 1, float, EM>(a) : stage_impl<DIM, 0, 1, double, EM>(a);
  }
  if (a.riemann == 0)
    return mixed ? stage_impl<DIM, 1, 0, float, EM>(a) : stage_impl<DIM, 1, 0, double, EM>(a);
  return mixed ? stage_impl<DIM, 1, 1, float, EM>(a) : stage_impl<DIM, 1, 1, double, EM>(a);
}

}  // namespace

size_t stage_cfl_blocks(const Geom& g, int limiter, bool glm) {
  if (glm || limiter == 2) return (size_t)((g.n + kBlock - 1) / kBlock);
  if (g.nz == 1) return tile_grid<Tile<2>>(g).ntiles;  // 2D (3D grids have nz >= 4)
  return march_grid(g).nblocks;
}

hipError_t launch_glm_cfl(const CflArgs& a, double* PW) {
  const unsigned nl = (unsigned)((a.g.n + kBlock - 1) / kBlock);
  if (a.dim == 3)
    MHD_TIMED(a, K_CFL,
              hipLaunchKernelGGL((k_glm_prim<3>), dim3(nl), dim3(kBlock), 0, a.stream, a.U, PW,
                                 a.g, a.flag, a.partial));
  else
    MHD_TIMED(a, K_CFL,
              hipLaunchKernelGGL((k_glm_prim<2>), dim3(nl), dim3(kBlock), 0, a.stream, a.U, PW,
                                 a.g, a.flag, a.partial));
  MHD_TIMED(a, K_CFL_FINAL,
            hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, a.partial, (int)nl,
                               a.cfl, a.dt_out));
  return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& a) {
  if (a.glm) return (a.dim == 3) ? glm_stage_lim<3>(a) : glm_stage_lim<2>(a);
  if (a.emf == 1) return (a.dim == 3) ? stage_lim<3, 1>(a) : stage_lim<2, 1>(a);
  return (a.dim == 3) ? stage_lim<3, 0>(a) : stage_lim<2, 0>(a);
}

// ---------------------------------------------------------------------------
// Allocation-free CFL time step (mhd_dt_device_noalloc). Its per-block
// partials and the unphysical flag live in this file-scope device array
// instead of the caller's workspace: kNoAllocPartials doubles, then the flag
// (an int) in the next double. Every device holds its own copy at its own
// address, found with hipGetSymbolAddress on the first call made with that
// device current; host code uses only that address, never the array's name.
// Calls that overlap on one device share the array and race.
static __device__ __align__(256) double scratch[kNoAllocPartials + 32];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

hipError_t scratch_here(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// The flag must start each call at zero: a kernel clears it (no memset, so
// that a captured graph replays the clear correctly).
__global__ void k_flag_clear(int* __restrict__ flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ void k_flag_copy(const int* __restrict__ flag, int32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = *flag;
}

}  // namespace

hipError_t launch_cfl_noalloc(const CflArgs& a, int32_t* flag_out) {
  if (a.nblocks < 1 || a.nblocks > kNoAllocPartials) return hipErrorInvalidValue;
  double* base = nullptr;
  hipError_t e = scratch_here(&base);
  if (e != hipSuccess) return e;
  int* flag = reinterpret_cast<int*>(base + kNoAllocPartials);
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, a.stream, flag);
  if (a.dim == 3)
    MHD_TIMED(a, K_CFL,
              hipLaunchKernelGGL((k_cfl<3>), dim3(a.nblocks), dim3(kBlock), 0, a.stream, a.U, a.g,
                                 base, flag));
  else
    MHD_TIMED(a, K_CFL,
              hipLaunchKernelGGL((k_cfl<2>), dim3(a.nblocks), dim3(kBlock), 0, a.stream, a.U, a.g,
                                 base, flag));
  MHD_TIMED(a, K_CFL_FINAL,
            hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, a.stream, base, a.nblocks,
                               a.cfl, a.dt_out));
  if (flag_out) hipLaunchKernelGGL(k_flag_copy, dim3(1), dim3(64), 0, a.stream, flag, flag_out);
  return hipGetLastError();
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
