// Multi-RHS gather on MFMA with split-BF16 operands (placeholder until the
// MFMA kernel lands).
#include <hip/hip_runtime.h>

#include "bvc_internal.hpp"

namespace bvc {

int gather_multi_mfma(int dim, int64_t n_cache, const float* cx, const float* cn, int nf, const float* A,
                      const float* B, int64_t n_eval, const float* ex, float* U, hipStream_t st) {
  (void)dim; (void)n_cache; (void)cx; (void)cn; (void)nf; (void)A; (void)B; (void)n_eval; (void)ex; (void)U; (void)st;
  return fail(BVC_EUNSUPPORTED, "split-BF16 multi-RHS gather is not built yet");
}

}  // namespace bvc
