// Sanitizer driver for the host side of the C ABI (include/mhd.h), without a
// GPU: configuration checks (valid and invalid fields), workspace sizes for
// every mode, error texts, null arguments. No call here reaches the device.
#include <cstdio>
#include <cstring>

#include "mhd.h"

static mhd_config base() {
  mhd_config c;
  std::memset(&c, 0, sizeof c);
  c.dim = 3; c.nx = 12; c.ny = 10; c.nz = 9;
  c.xmin = 0; c.xmax = 1; c.ymin = 0; c.ymax = 1; c.zmin = 0; c.zmax = 1;
  c.gamma = 5.0 / 3.0; c.cfl = 0.3; c.limiter = MHD_LIM_VANLEER; c.riemann = MHD_RS_HLLD;
  return c;
}

int main() {
  int bad = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int lim = 0; lim <= 2; ++lim)
      for (int prec = 0; prec <= 1; ++prec)
        for (int integ = 0; integ <= 1; ++integ)
          for (int mode = 0; mode <= 2; ++mode) {
            mhd_config c = base();
            c.dim = dim;
            if (dim == 2) c.nz = 1;
            c.limiter = lim; c.precision = prec; c.integrator = integ;
            c.emf = mode == 1 ? MHD_EMF_UCT_HLLD : MHD_EMF_UCT_HLL;
            c.divb = mode == 2 ? MHD_DIVB_GLM : MHD_DIVB_CT;
            mhd_ctx* ctx = nullptr;
            const mhd_status st = mhd_init(&c, &ctx);
            const bool expect_ok = !(lim == 2 && prec == 1);
            if ((st == MHD_OK) != expect_ok) ++bad;
            if (st == MHD_OK) {
              const size_t f = mhd_workspace_bytes(ctx, 0), a = mhd_workspace_bytes(ctx, 1);
              if (f == 0 || a < f) ++bad;
              if (mhd_last_error(ctx)[0] != '\0') ++bad;
              mhd_destroy(ctx);
            }
          }
  // invalid configurations and arguments
  const int nbadcfg = 8;
  for (int t = 0; t < nbadcfg; ++t) {
    mhd_config c = base();
    switch (t) {
      case 0: c.dim = 4; break;
      case 1: c.nx = 3; break;
      case 2: c.gamma = 1.0; break;
      case 3: c.cfl = -1.0; break;
      case 4: c.emf = 7; break;
      case 5: c.divb = 3; break;
      case 6: c.divb = MHD_DIVB_GLM; c.emf = MHD_EMF_UCT_HLLD; break;
      default: c.xmax = c.xmin; break;
    }
    mhd_ctx* ctx = nullptr;
    if (mhd_init(&c, &ctx) != MHD_ERR_INVALID || ctx != nullptr) ++bad;
  }
  mhd_config c = base();
  if (mhd_init(&c, nullptr) != MHD_ERR_INVALID) ++bad;
  if (mhd_init(nullptr, nullptr) != MHD_ERR_INVALID) ++bad;
  if (mhd_workspace_bytes(nullptr, 0) != 0) ++bad;
  mhd_destroy(nullptr);
  for (int s = 0; s >= -6; --s)
    if (!mhd_strerror((mhd_status)s) || !mhd_strerror((mhd_status)s)[0]) ++bad;
  if (std::strcmp(mhd_last_error(nullptr), "") != 0) ++bad;
  if (bad) {
    std::printf("host driver: %d failures\n", bad);
    return 1;
  }
  std::printf("host driver ok\n");
  return 0;
}
