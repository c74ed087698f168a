// Batched step kernels with FP16 deviation storage (lbm_batch_kernels.hpp).
#include "lbm_batch_kernels.hpp"

namespace mclbm {
void launch_batch_f16(const BatchLaunch &B, hipStream_t s, int lp, long long L, bool diag) {
    launch_batch_storage<__half>(B, s, lp, L, diag);
}
}  // namespace mclbm
