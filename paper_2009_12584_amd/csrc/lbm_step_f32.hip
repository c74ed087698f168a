// Step kernels of one simulation with FP32 deviation storage (lbm_step_kernels.hpp).
#include "lbm_step_kernels.hpp"

namespace mclbm {
void launch_step_f32(const Launch &L, dim3 g, hipStream_t s, const Inst &I, int parity, const Fields &fo,
                     double *partials) {
    launch_storage<float>(L, g, s, I, parity, fo, partials);
}
}  // namespace mclbm
