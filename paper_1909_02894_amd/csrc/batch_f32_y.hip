// Batch phase kernel, f32, direction y.
#include "batch_kernels.hpp"
#include "batch_registry.hpp"

namespace dirac {
static BatchKernelRegistrar reg_batch_f32_y(1, 1,
    reinterpret_cast<const void*>(&batch_stage_kernel<float, true>),
    [](int logn, int s) { return batch_smem_for<float, true>(logn, s); });
}  // namespace dirac
