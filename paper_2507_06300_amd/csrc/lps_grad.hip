// Adjoint of the batched forward pass (placeholder until the adjoint kernels land).
#include "lps_internal.hpp"

namespace lps {

size_t grad_workspace_bytes(const lps_ctx* ctx) { (void)ctx; return 256; }

hipError_t launch_grad(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL, double* dparams,
                       double* dkx, double* dky, uint32_t* status, hipStream_t s) {
  (void)ctx; (void)st; (void)prec; (void)logL; (void)dparams; (void)dkx; (void)dky; (void)status; (void)s;
  return hipErrorNotSupported;
}

}  // namespace lps
