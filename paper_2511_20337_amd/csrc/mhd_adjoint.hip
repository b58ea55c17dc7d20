// Adjoint of one SSP-RK2 step (placeholder until the reverse kernels land).
#include "mhd_adjoint.hpp"

namespace mhd {

size_t adjoint_workspace_bytes(int dim, size_t ncell) {
  (void)dim;
  (void)ncell;
  return 0;
}

hipError_t launch_adjoint_step(const AdjointArgs& a) {
  (void)a;
  return hipErrorNotSupported;
}

}  // namespace mhd
