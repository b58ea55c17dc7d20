// Host-side launch interface of the adjoint (vector-Jacobian product) of one
// SSP-RK2 step.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mhd_device.hpp"

namespace mhd {

struct AdjointArgs {
  int dim, limiter, riemann;
  int integrator;        // 0: SSP-RK2, 1: SSP-RK3
  Geom g;
  const double* Un;      // state at the start of the step (unchanged)
  const double* Ubar1;   // adjoint of the step's output
  double* Ubar0;         // adjoint of the step's input (written)
  double dt;
  double* U1;            // forward scratch: stage-1 state
  double* U2;            // forward scratch (SSP-RK3): stage-2 state
  double* FW;            // forward scratch: face records
  double* EW;            // forward scratch: edge EMFs
  double* scratch;       // adjoint scratch (adjoint_workspace_bytes)
  double* dtbar_dev;     // device double receiving dt-bar
  bool want_dtbar;
  int* flag;
  hipStream_t stream;
};

// Extra workspace bytes the adjoint needs beyond the forward workspace.
size_t adjoint_workspace_bytes(int dim, size_t ncell, int integrator);

// Enqueue the adjoint step; hipErrorNotSupported if not available.
hipError_t launch_adjoint_step(const AdjointArgs& a);

}  // namespace mhd
