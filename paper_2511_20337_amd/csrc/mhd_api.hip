// C ABI of libmhd (declared in include/mhd.h): configuration checks,
// workspace layout and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mhd.h"
#include "mhd_adjoint.hpp"
#include "mhd_kernels.hpp"

namespace {

const char* const kKernelNames[mhd::K_COUNT] = {"faces", "emf", "update", "cfl", "cfl_final",
                                                "adjoint", "prim"};

// Per-kernel HIP-event timing: an event pair per launch, read back on demand.
struct EventTimer final : mhd::Timer {
  struct Rec {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipError_t err = hipSuccess;
  hipEvent_t open_[mhd::K_COUNT] = {};
  double ms[mhd::K_COUNT] = {};
  int64_t count[mhd::K_COUNT] = {};

  void note(hipError_t r) {
    if (r != hipSuccess) err = r;
  }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) err = r;
    return e;
  }
  void begin(int kid, hipStream_t s) override {
    open_[kid] = get();
    if (open_[kid]) note(hipEventRecord(open_[kid], s));
  }
  void end(int kid, hipStream_t s) override {
    hipEvent_t b = get();
    if (b && open_[kid]) {
      note(hipEventRecord(b, s));
      recs.push_back({kid, open_[kid], b});
    }
    open_[kid] = nullptr;
  }
  hipError_t collect() {
    for (Rec& r : recs) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e != hipSuccess) return e;
      float t = 0.f;
      e = hipEventElapsedTime(&t, r.a, r.b);
      if (e != hipSuccess) return e;
      ms[r.kid] += t;
      count[r.kid] += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
    return err;
  }
  void reset() {
    for (int k = 0; k < mhd::K_COUNT; ++k) {
      ms[k] = 0.0;
      count[k] = 0;
    }
  }
  ~EventTimer() override {
    for (Rec& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct mhd_ctx {
  mhd_config cfg;
  EventTimer* timer;
  mhd::Geom g;
  // workspace layout (byte offsets from the 256-aligned base)
  size_t off_partial, off_u1, off_fw, off_ew, off_u2, off_pw, off_adj, bytes_fwd, bytes_adj;
  int cfl_blocks;
  char err[256];
};

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kCtl = 256;      // control block: [0] dt (double), [8] flag (int)
constexpr int kCflBlocks = 2048;  // CFL partials (grid-stride reduction)
// GLM damping rate alpha (psi <- psi exp(-alpha c_h dt / Delta_min) per step)
constexpr double kGlmAlpha = 0.1;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool cfg_valid(const mhd_config* c) {
  if (!c) return false;
  if (c->dim != 2 && c->dim != 3) return false;
  if (c->nx < 4 || c->ny < 4) return false;
  if (c->dim == 3 && c->nz < 4) return false;
  if (c->dim == 2 && c->nz != 1) return false;
  if (!(c->xmax > c->xmin) || !(c->ymax > c->ymin) || !(c->zmax > c->zmin)) return false;
  if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) return false;
  if (!(c->cfl > 0.0) || !std::isfinite(c->cfl)) return false;
  if (c->limiter < 0 || c->limiter > 2 || c->riemann < 0 || c->riemann > 1) return false;
  if (c->limiter == MHD_LIM_WENOZ && c->precision != MHD_PREC_FP64) return false;
  if (c->precision < 0 || c->precision > 1) return false;
  if (c->integrator != MHD_SSP_RK2 && c->integrator != MHD_SSP_RK3) return false;
  if (c->emf != MHD_EMF_UCT_HLL && c->emf != MHD_EMF_UCT_HLLD) return false;
  if (c->divb != MHD_DIVB_CT && c->divb != MHD_DIVB_GLM) return false;
  if (c->divb == MHD_DIVB_GLM && c->emf != MHD_EMF_UCT_HLL) return false;  // no EMF in GLM
  // 64-bit cell count; per-axis sizes bounded so index arithmetic stays in int
  const double cells = (double)c->nx * c->ny * c->nz;
  if (cells > 4.0e9) return false;
  // the 3D z-marching kernels address a plane of one field with 32-bit byte
  // offsets: fewer than 2^29 cells per plane
  if (c->dim == 3 && (double)c->nx * c->ny >= 536870912.0) return false;
  return true;
}

mhd_status device_fail(mhd_ctx* ctx, hipError_t e, const char* where) {
  std::snprintf(ctx->err, sizeof ctx->err, "%s: %s", where, hipGetErrorString(e));
  return MHD_ERR_DEVICE;
}

bool ws_ok(const mhd_ctx* ctx, const void* ws, size_t bytes, bool adj) {
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return false;
  return bytes >= (adj ? ctx->bytes_adj : ctx->bytes_fwd);
}

char* base(void* ws) { return static_cast<char*>(ws); }
double* ws_dt(void* ws) { return reinterpret_cast<double*>(base(ws)); }
int* ws_flag(void* ws) { return reinterpret_cast<int*>(base(ws) + 8); }

mhd::StageArgs stage_args(mhd_ctx* ctx, void* ws, hipStream_t s) {
  mhd::StageArgs a{};
  a.dim = ctx->cfg.dim;
  a.limiter = ctx->cfg.limiter;
  a.riemann = ctx->cfg.riemann;
  a.precision = ctx->cfg.precision;
  a.emf = ctx->cfg.emf;
  a.g = ctx->g;
  a.FW = reinterpret_cast<double*>(base(ws) + ctx->off_fw);
  a.EW = reinterpret_cast<double*>(base(ws) + ctx->off_ew);
  a.glm = ctx->cfg.divb == MHD_DIVB_GLM;
  a.PW = (ctx->cfg.limiter == MHD_LIM_WENOZ || a.glm)
             ? reinterpret_cast<double*>(base(ws) + ctx->off_pw) : nullptr;
  if (a.glm) {
    // c_h = C Delta_min / dt; the damping per step exp(-alpha c_h dt / Delta_min)
    a.glm_dmin = std::min(ctx->g.dx, ctx->g.dy);
    if (ctx->cfg.dim == 3) a.glm_dmin = std::min(a.glm_dmin, ctx->g.dz);
    a.cfl = ctx->cfg.cfl;
    a.glm_decay = std::exp(-kGlmAlpha * ctx->cfg.cfl);
  }
  a.flag = ws_flag(ws);
  a.stream = s;
  a.timer = ctx->timer;
  return a;
}

// One SSP-RK2 or SSP-RK3 step. dt_cfl (not for 2D WENO-Z): dt is the CFL step of U,
// reduced by the stage-1 face kernel and written to dt_cfl, which is also dtp.
mhd_status run_step(mhd_ctx* ctx, double* U, double dt, const double* dtp, void* ws,
                    hipStream_t s, double* dt_cfl = nullptr) {
  double* U1 = reinterpret_cast<double*>(base(ws) + ctx->off_u1);
  mhd::StageArgs a = stage_args(ctx, ws, s);
  a.dt = dt;
  a.dtp = dtp;
  a.stage = 1;
  a.U = U;
  a.U0 = nullptr;
  a.out = U1;
  if (dt_cfl) {
    a.cfl_partial = reinterpret_cast<double*>(base(ws) + ctx->off_partial);
    a.cfl = ctx->cfg.cfl;
    a.dt_out = dt_cfl;
  }
  hipError_t e = mhd::launch_stage(a);
  if (e != hipSuccess) return device_fail(ctx, e, "stage 1");
  a.cfl_partial = nullptr;
  if (ctx->cfg.integrator == MHD_SSP_RK3) {
    double* U2 = reinterpret_cast<double*>(base(ws) + ctx->off_u2);
    a.stage = 4;  // U2 = (3 U + (U1 + dt L(U1))) / 4
    a.U = U1;
    a.U0 = U;
    a.out = U2;
    e = mhd::launch_stage(a);
    if (e != hipSuccess) return device_fail(ctx, e, "stage 2");
    a.stage = 5;  // U <- (U + 2 (U2 + dt L(U2))) / 3
    a.U = U2;
    a.U0 = U;
    a.out = U;
    e = mhd::launch_stage(a);
    if (e != hipSuccess) return device_fail(ctx, e, "stage 3");
    return MHD_OK;
  }
  a.stage = 2;
  a.U = U1;
  a.U0 = U;
  a.out = U;
  e = mhd::launch_stage(a);
  if (e != hipSuccess) return device_fail(ctx, e, "stage 2");
  return MHD_OK;
}

mhd_status cfl_to(mhd_ctx* ctx, const double* U, void* ws, double* dt_dev, hipStream_t s) {
  if (ctx->cfg.divb == MHD_DIVB_GLM) {  // through the GLM primitive kernel
    mhd::CflArgs a{};
    a.dim = ctx->cfg.dim;
    a.g = ctx->g;
    a.U = U;
    a.partial = reinterpret_cast<double*>(base(ws) + ctx->off_partial);
    a.cfl = ctx->cfg.cfl;
    a.dt_out = dt_dev;
    a.flag = ws_flag(ws);
    a.stream = s;
    a.timer = ctx->timer;
    hipError_t e = mhd::launch_glm_cfl(a, reinterpret_cast<double*>(base(ws) + ctx->off_pw));
    if (e != hipSuccess) return device_fail(ctx, e, "cfl");
    return MHD_OK;
  }
  mhd::CflArgs a{};
  a.dim = ctx->cfg.dim;
  a.g = ctx->g;
  a.U = U;
  a.partial = reinterpret_cast<double*>(base(ws) + ctx->off_partial);
  a.nblocks = ctx->cfl_blocks;
  a.cfl = ctx->cfg.cfl;
  a.dt_out = dt_dev;
  a.flag = ws_flag(ws);
  a.stream = s;
  a.timer = ctx->timer;
  hipError_t e = mhd::launch_cfl(a);
  if (e != hipSuccess) return device_fail(ctx, e, "cfl");
  return MHD_OK;
}

mhd_status read_flag(mhd_ctx* ctx, void* ws, hipStream_t s, int* flag) {
  hipError_t e = hipMemcpyAsync(flag, ws_flag(ws), sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_fail(ctx, e, "read flag");
  if (*flag) {
    // clear with a tiny kernel-free copy from a zero on the host
    static const int zero = 0;
    e = hipMemcpyAsync(ws_flag(ws), &zero, sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(ctx, e, "clear flag");
  }
  return MHD_OK;
}

}  // namespace

extern "C" {

mhd_status mhd_init(const mhd_config* cfg, mhd_ctx** out) {
  if (!out) return MHD_ERR_INVALID;
  *out = nullptr;
  if (!cfg_valid(cfg)) return MHD_ERR_INVALID;
  mhd_ctx* c = new (std::nothrow) mhd_ctx();
  if (!c) return MHD_ERR_INVALID;
  c->cfg = *cfg;
  c->g.nx = cfg->nx;
  c->g.ny = cfg->ny;
  c->g.nz = cfg->nz;
  c->g.n = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  c->g.dx = (cfg->xmax - cfg->xmin) / cfg->nx;
  c->g.dy = (cfg->ymax - cfg->ymin) / cfg->ny;
  c->g.dz = (cfg->zmax - cfg->zmin) / cfg->nz;
  c->g.gamma = cfg->gamma;
  const size_t n = (size_t)c->g.n;
  const bool glm = cfg->divb == MHD_DIVB_GLM;
  const size_t nf = glm ? 9 : 8;  // stored fields
  c->cfl_blocks = kCflBlocks;
  // CFL partials: of k_cfl, or (3D) one per face (WENO-Z: primitive) workgroup
  // of the fused step; GLM: one per primitive workgroup in 2D and 3D
  size_t npart = kCflBlocks;
  if (cfg->dim == 3 || glm)
    npart = std::max(npart, mhd::stage_cfl_blocks(c->g, cfg->limiter, glm));
  size_t off = kCtl;
  c->off_partial = off;
  off = align_up(off + sizeof(double) * npart);
  c->off_u1 = off;
  off = align_up(off + sizeof(double) * nf * n);
  c->off_fw = off;  // face records (CT) or the nine face fluxes per direction (GLM)
  off = align_up(off + sizeof(double) * (size_t)cfg->dim * (glm ? 9 : mhd::NSLOT) * n);
  c->off_ew = off;
  if (!glm) off = align_up(off + sizeof(double) * 3 * n);
  c->off_u2 = off;  // SSP-RK3: the second-stage state
  if (cfg->integrator == MHD_SSP_RK3) off = align_up(off + sizeof(double) * nf * n);
  c->off_pw = off;  // WENO-Z and GLM: the primitives of every cell
  if (cfg->limiter == MHD_LIM_WENOZ || glm) off = align_up(off + sizeof(double) * nf * n);
  c->bytes_fwd = off;
  c->off_adj = off;
  c->bytes_adj = off + mhd::adjoint_workspace_bytes(cfg->dim, n, cfg->integrator);
  c->err[0] = '\0';
  *out = c;
  return MHD_OK;
}

void mhd_destroy(mhd_ctx* ctx) {
  if (!ctx) return;
  delete ctx->timer;
  delete ctx;
}

size_t mhd_workspace_bytes(const mhd_ctx* ctx, int32_t with_adjoint) {
  if (!ctx) return 0;
  return with_adjoint ? ctx->bytes_adj : ctx->bytes_fwd;
}

mhd_status mhd_dt_device(mhd_ctx* ctx, const double* U, void* ws, size_t ws_bytes, double* dt_dev,
                         void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !dt_dev) return MHD_ERR_INVALID;
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  return cfl_to(ctx, U, ws, dt_dev, static_cast<hipStream_t>(stream));
}

mhd_status mhd_dt_device_noalloc(mhd_ctx* ctx, const double* U, double* dt_dev,
                                 int32_t* flag_dev, void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !dt_dev) return MHD_ERR_INVALID;
  if (ctx->cfg.divb == MHD_DIVB_GLM) return MHD_ERR_UNSUPPORTED;
  mhd::CflArgs a{};
  a.dim = ctx->cfg.dim;
  a.g = ctx->g;
  a.U = U;
  // the reduction strides over the grid, so every valid grid fits in the
  // array's partials; small grids take fewer blocks
  const int64_t need = (ctx->g.n + 255) / 256;
  a.nblocks = (int)std::min<int64_t>(need, mhd::kNoAllocPartials);
  a.cfl = ctx->cfg.cfl;
  a.dt_out = dt_dev;
  a.stream = static_cast<hipStream_t>(stream);
  a.timer = ctx->timer;
  hipError_t e = mhd::launch_cfl_noalloc(a, flag_dev);
  if (e != hipSuccess) return device_fail(ctx, e, "cfl (no workspace)");
  return MHD_OK;
}

mhd_status mhd_dt(mhd_ctx* ctx, const double* U, void* ws, size_t ws_bytes, double* dt_out,
                  void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !dt_out) return MHD_ERR_INVALID;
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  mhd_status st = cfl_to(ctx, U, ws, ws_dt(ws), s);
  if (st != MHD_OK) return st;
  hipError_t e = hipMemcpyAsync(dt_out, ws_dt(ws), sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return device_fail(ctx, e, "dt copy");
  int flag = 0;
  st = read_flag(ctx, ws, s, &flag);
  if (st != MHD_OK) return st;
  return flag ? MHD_ERR_UNPHYSICAL : MHD_OK;
}

mhd_status mhd_step(mhd_ctx* ctx, double* U, double dt, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !(dt > 0.0) || !std::isfinite(dt)) return MHD_ERR_INVALID;
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  return run_step(ctx, U, dt, nullptr, ws, static_cast<hipStream_t>(stream));
}

mhd_status mhd_step_device_dt(mhd_ctx* ctx, double* U, const double* dt_dev, void* ws,
                              size_t ws_bytes, void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !dt_dev) return MHD_ERR_INVALID;
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  return run_step(ctx, U, 0.0, dt_dev, ws, static_cast<hipStream_t>(stream));
}

mhd_status mhd_step_cfl(mhd_ctx* ctx, double* U, double* dt_dev, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !dt_dev) return MHD_ERR_INVALID;
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->cfg.dim == 3 || ctx->cfg.divb == MHD_DIVB_GLM || ctx->cfg.limiter != MHD_LIM_WENOZ)
    return run_step(ctx, U, 0.0, dt_dev, ws, s, dt_dev);
  mhd_status st = cfl_to(ctx, U, ws, dt_dev, s);  // 2D WENO-Z: the separate CFL pass
  if (st != MHD_OK) return st;
  return run_step(ctx, U, 0.0, dt_dev, ws, s);
}

mhd_status mhd_rhs(mhd_ctx* ctx, const double* U, double* L, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U || !L || U == L) return MHD_ERR_INVALID;
  if (ctx->cfg.divb == MHD_DIVB_GLM) return MHD_ERR_UNSUPPORTED;  // c_h needs the step's dt
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  mhd::StageArgs a = stage_args(ctx, ws, static_cast<hipStream_t>(stream));
  a.stage = 0;
  a.U = U;
  a.U0 = nullptr;
  a.out = L;
  hipError_t e = mhd::launch_stage(a);
  if (e != hipSuccess) return device_fail(ctx, e, "rhs");
  return MHD_OK;
}

// Shared body of the two adjoint entry points: dt-bar goes to the device
// double dtbar_dev when want_dtbar (nullptr: the workspace slot).
static mhd_status adjoint_impl(mhd_ctx* ctx, const double* U_n, double dt, const double* Ubar_np1,
                               double* Ubar_n, bool want_dtbar, double* dtbar_dev, void* ws,
                               size_t ws_bytes, hipStream_t s) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!U_n || !Ubar_np1 || !Ubar_n || !(dt > 0.0) || !std::isfinite(dt)) return MHD_ERR_INVALID;
  if (Ubar_n == Ubar_np1 || Ubar_n == U_n) return MHD_ERR_INVALID;
  if (ctx->cfg.precision != MHD_PREC_FP64 || ctx->cfg.limiter == MHD_LIM_WENOZ ||
      ctx->cfg.emf != MHD_EMF_UCT_HLL || ctx->cfg.divb != MHD_DIVB_CT)
    return MHD_ERR_UNSUPPORTED;
  if (!ws_ok(ctx, ws, ws_bytes, true)) return MHD_ERR_WORKSPACE;
  mhd::AdjointArgs a{};
  a.dim = ctx->cfg.dim;
  a.limiter = ctx->cfg.limiter;
  a.riemann = ctx->cfg.riemann;
  a.integrator = ctx->cfg.integrator == MHD_SSP_RK3 ? 1 : 0;
  a.g = ctx->g;
  a.Un = U_n;
  a.Ubar1 = Ubar_np1;
  a.Ubar0 = Ubar_n;
  a.dt = dt;
  a.U1 = reinterpret_cast<double*>(base(ws) + ctx->off_u1);
  a.U2 = ctx->cfg.integrator == MHD_SSP_RK3
             ? reinterpret_cast<double*>(base(ws) + ctx->off_u2) : nullptr;
  a.FW = reinterpret_cast<double*>(base(ws) + ctx->off_fw);
  a.EW = reinterpret_cast<double*>(base(ws) + ctx->off_ew);
  a.scratch = reinterpret_cast<double*>(base(ws) + ctx->off_adj);
  a.dtbar_dev = dtbar_dev ? dtbar_dev : ws_dt(ws);
  a.want_dtbar = want_dtbar;
  a.flag = ws_flag(ws);
  a.stream = s;
  hipError_t e = mhd::launch_adjoint_step(a);
  if (e == hipErrorNotSupported) return MHD_ERR_UNSUPPORTED;
  if (e != hipSuccess) return device_fail(ctx, e, "adjoint");
  return MHD_OK;
}

mhd_status mhd_adjoint_step(mhd_ctx* ctx, const double* U_n, double dt, const double* Ubar_np1,
                            double* Ubar_n, double* dtbar, void* ws, size_t ws_bytes,
                            void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  mhd_status st = adjoint_impl(ctx, U_n, dt, Ubar_np1, Ubar_n, dtbar != nullptr, nullptr, ws,
                               ws_bytes, s);
  if (st != MHD_OK || !dtbar) return st;
  hipError_t e = hipMemcpyAsync(dtbar, ws_dt(ws), sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_fail(ctx, e, "dtbar copy");
  return MHD_OK;
}

mhd_status mhd_adjoint_step_device(mhd_ctx* ctx, const double* U_n, double dt,
                                   const double* Ubar_np1, double* Ubar_n, double* dtbar_dev,
                                   void* ws, size_t ws_bytes, void* stream) {
  return adjoint_impl(ctx, U_n, dt, Ubar_np1, Ubar_n, dtbar_dev != nullptr, dtbar_dev, ws,
                      ws_bytes, static_cast<hipStream_t>(stream));
}

mhd_status mhd_check(mhd_ctx* ctx, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return MHD_ERR_INVALID;
  if (!ws_ok(ctx, ws, ws_bytes, false)) return MHD_ERR_WORKSPACE;
  int flag = 0;
  mhd_status st = read_flag(ctx, ws, static_cast<hipStream_t>(stream), &flag);
  if (st != MHD_OK) return st;
  return flag ? MHD_ERR_UNPHYSICAL : MHD_OK;
}

mhd_status mhd_timing(mhd_ctx* ctx, int32_t enable) {
  if (!ctx) return MHD_ERR_INVALID;
  if (enable) {
    if (!ctx->timer) ctx->timer = new (std::nothrow) EventTimer();
    if (!ctx->timer) return MHD_ERR_INVALID;
    ctx->timer->reset();
  } else {
    delete ctx->timer;
    ctx->timer = nullptr;
  }
  return MHD_OK;
}

mhd_status mhd_timing_read(mhd_ctx* ctx, int32_t kernel, const char** name, double* total_ms,
                           int64_t* launches) {
  if (!ctx || !ctx->timer || kernel < 0 || kernel >= mhd::K_COUNT) return MHD_ERR_INVALID;
  hipError_t e = ctx->timer->collect();
  if (e != hipSuccess) return device_fail(ctx, e, "timing");
  if (name) *name = kKernelNames[kernel];
  if (total_ms) *total_ms = ctx->timer->ms[kernel];
  if (launches) *launches = ctx->timer->count[kernel];
  return MHD_OK;
}

const char* mhd_strerror(mhd_status s) {
  switch (s) {
    case MHD_OK: return "ok";
    case MHD_ERR_INVALID: return "invalid argument";
    case MHD_ERR_UNSUPPORTED: return "unsupported configuration";
    case MHD_ERR_DEVICE: return "device error";
    case MHD_ERR_UNPHYSICAL: return "unphysical state (rho <= 0, p <= 0 or non-finite)";
    case MHD_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
  }
  return "unknown status";
}

const char* mhd_last_error(const mhd_ctx* ctx) { return ctx ? ctx->err : ""; }

}  // extern "C"
