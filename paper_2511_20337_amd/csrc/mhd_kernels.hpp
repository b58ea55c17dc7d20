// Host-side launch interface between the C ABI and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mhd_device.hpp"

namespace mhd {

// Kernel identities for the optional per-kernel event timing.
enum KernelId : int { K_FACES = 0, K_EMF, K_UPDATE, K_CFL, K_CFL_FINAL, K_ADJ, K_PRIM, K_COUNT };

// Records a pair of HIP events around each launch on the launch stream.
struct Timer {
  virtual void begin(int kid, hipStream_t s) = 0;
  virtual void end(int kid, hipStream_t s) = 0;
  virtual ~Timer() = default;
};

// One RK stage (or the bare right-hand side).
struct StageArgs {
  int dim, limiter, riemann, precision;
  int emf;                // 0: upwind average with the HLL bounds; 1: UCT-HLLD
  bool glm;               // GLM divergence cleaning: nine cell-centred fields, no CT
  double glm_dmin;        // GLM: the smallest cell spacing (c_h = cfl dmin / dt)
  double glm_decay;       // GLM: damping factor of psi per step, exp(-alpha cfl)
  int stage;              // 0: out = L(U); 1: out = U + dt L; 2: out = (U0 + U + dt L)/2;
                          // 3: face/edge records only; SSP-RK3 stages 2 and 3:
                          // 4: out = (3 U0 + (U + dt L))/4; 5: out = (U0 + 2 (U + dt L))/3
  Geom g;
  const double* U;        // state the right-hand side is evaluated at
  const double* U0;       // stage 2: state at the start of the step
  double* out;
  double* FW;             // face records: dim * NSLOT * n doubles
  double* EW;             // edge EMFs: 3 * n doubles
  double* PW;             // WENO-Z only: primitives of every cell, 8 * n doubles
  double dt;
  const double* dtp;      // device dt (nullptr: use dt)
  int* flag;              // sticky unphysical flag
  hipStream_t stream;
  Timer* timer;           // nullable
  // 3D stage 1 only, optional: the face kernel (with WENO-Z, the primitive
  // kernel) also reduces the CFL bound of U
  // into cfl_partial (stage_cfl_blocks(g, limiter) doubles), and *dt_out = cfl * min
  // is written before the update reads dtp (which then must be dt_out)
  double* cfl_partial;
  double cfl;
  double* dt_out;
};

struct CflArgs {
  int dim;
  Geom g;
  const double* U;
  double* partial;        // nblocks doubles
  int nblocks;
  double cfl;
  double* dt_out;         // device double
  int* flag;
  hipStream_t stream;
  Timer* timer;           // nullable
};

#define MHD_TIMED(args, kid, ...)                              \
  do {                                                         \
    if ((args).timer) (args).timer->begin((kid), (args).stream); \
    __VA_ARGS__;                                               \
    if ((args).timer) (args).timer->end((kid), (args).stream);   \
  } while (0)

hipError_t launch_stage(const StageArgs& a);
// number of CFL partials the 3D face kernel (WENO-Z, GLM: primitive kernel)
// writes (one per workgroup)
size_t stage_cfl_blocks(const Geom& g, int limiter, bool glm);
// GLM: the CFL time step of U through its primitive kernel (writes PW too)
hipError_t launch_glm_cfl(const CflArgs& a, double* PW);
hipError_t launch_cfl(const CflArgs& a);
// Partials of the allocation-free CFL time step (a file-scope device array of
// that many doubles plus the flag; nblocks must not exceed it).
constexpr int kNoAllocPartials = 2048;
// The CFL time step with the partials and the flag in that array (a.partial
// and a.flag are ignored); flag_out (device int32, nullable) receives 1 if
// any cell was unphysical in this call, else 0.
hipError_t launch_cfl_noalloc(const CflArgs& a, int32_t* flag_out);

}  // namespace mhd
