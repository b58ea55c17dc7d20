// The C ABI used on its own (include/mhd.h and the HIP runtime, no PyTorch):
// reads an FP64 state, runs `nsteps` calls of mhd_step_cfl on device 0 and
// writes the state followed by the last time step. The GPU test that runs it
// checks that the bare ABI and the Python binding give the same bits.
//
// usage: step_cli IN OUT NSTEPS DIM NX NY NZ XMIN XMAX YMIN YMAX ZMIN ZMAX
//                 GAMMA CFL LIMITER RIEMANN PRECISION INTEGRATOR
// IN holds 8 nz ny nx doubles (field-major, x fastest); OUT receives the same
// layout and then one double, dt of the last step. Exit status 0 on success.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mhd.h"

namespace {

int hip_fail(const char* what, hipError_t e) {
  std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return 1;
}

int mhd_fail(const char* what, mhd_status s, const mhd_ctx* ctx) {
  std::fprintf(stderr, "%s: %s (%s)\n", what, mhd_strerror(s), ctx ? mhd_last_error(ctx) : "");
  return 1;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 20) {
    std::fprintf(stderr, "usage: %s IN OUT NSTEPS DIM NX NY NZ XMIN XMAX YMIN YMAX ZMIN ZMAX "
                         "GAMMA CFL LIMITER RIEMANN PRECISION INTEGRATOR\n", argv[0]);
    return 2;
  }
  const int nsteps = std::atoi(argv[3]);
  mhd_config cfg{};
  cfg.dim = std::atoi(argv[4]);
  cfg.nx = std::atoi(argv[5]);
  cfg.ny = std::atoi(argv[6]);
  cfg.nz = std::atoi(argv[7]);
  cfg.xmin = std::atof(argv[8]);
  cfg.xmax = std::atof(argv[9]);
  cfg.ymin = std::atof(argv[10]);
  cfg.ymax = std::atof(argv[11]);
  cfg.zmin = std::atof(argv[12]);
  cfg.zmax = std::atof(argv[13]);
  cfg.gamma = std::atof(argv[14]);
  cfg.cfl = std::atof(argv[15]);
  cfg.limiter = std::atoi(argv[16]);
  cfg.riemann = std::atoi(argv[17]);
  cfg.precision = std::atoi(argv[18]);
  cfg.integrator = std::atoi(argv[19]);
  mhd_ctx* ctx = nullptr;
  mhd_status st = mhd_init(&cfg, &ctx);
  if (st != MHD_OK) return mhd_fail("mhd_init", st, nullptr);
  const size_t count = 8 * (size_t)cfg.nx * cfg.ny * cfg.nz;
  std::vector<double> U(count + 1);
  FILE* in = std::fopen(argv[1], "rb");
  if (!in || std::fread(U.data(), sizeof(double), count, in) != count) {
    std::fprintf(stderr, "cannot read %zu doubles from %s\n", count, argv[1]);
    return 1;
  }
  std::fclose(in);
  const size_t ws_bytes = mhd_workspace_bytes(ctx, 0);
  double* dU = nullptr;
  double* dt_dev = nullptr;
  void* ws = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&dU), count * sizeof(double));
  if (e != hipSuccess) return hip_fail("hipMalloc state", e);
  e = hipMalloc(&ws, ws_bytes);  // hipMalloc returns 256-byte aligned memory
  if (e != hipSuccess) return hip_fail("hipMalloc workspace", e);
  e = hipMalloc(reinterpret_cast<void**>(&dt_dev), sizeof(double));
  if (e != hipSuccess) return hip_fail("hipMalloc dt", e);
  hipStream_t stream = nullptr;
  e = hipStreamCreate(&stream);
  if (e != hipSuccess) return hip_fail("hipStreamCreate", e);
  e = hipMemcpy(dU, U.data(), count * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail("hipMemcpy in", e);
  for (int s = 0; s < nsteps; ++s) {
    st = mhd_step_cfl(ctx, dU, dt_dev, ws, ws_bytes, stream);
    if (st != MHD_OK) return mhd_fail("mhd_step_cfl", st, ctx);
  }
  st = mhd_check(ctx, ws, ws_bytes, stream);  // synchronises; reports an unphysical state
  if (st != MHD_OK) return mhd_fail("mhd_check", st, ctx);
  e = hipMemcpy(U.data(), dU, count * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail("hipMemcpy out", e);
  e = hipMemcpy(U.data() + count, dt_dev, sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail("hipMemcpy dt", e);
  FILE* out = std::fopen(argv[2], "wb");
  if (!out || std::fwrite(U.data(), sizeof(double), count + 1, out) != count + 1) {
    std::fprintf(stderr, "cannot write %s\n", argv[2]);
    return 1;
  }
  std::fclose(out);
  (void)hipStreamDestroy(stream);
  (void)hipFree(dt_dev);
  (void)hipFree(ws);
  (void)hipFree(dU);
  mhd_destroy(ctx);
  return 0;
}
