// Parameter-derivative (adjoint) kernels of the JVB library.
#include "vbqmc_internal.h"

namespace vbqmc {

size_t param_grad_ws_doubles(const DevWF& wf, int64_t W) {
  (void)wf;
  (void)W;
  return 0;
}

hipError_t launch_param_grad(const DevWF& wf, const DevWF* dwf, int nt, int64_t W, const double* R, double* dlogpsi, double* deloc,
                             double* ws, size_t ws_doubles, hipStream_t s) {
  (void)wf; (void)dwf; (void)nt; (void)W; (void)R; (void)dlogpsi; (void)deloc; (void)ws; (void)ws_doubles; (void)s;
  return hipErrorNotSupported;
}

}  // namespace vbqmc
