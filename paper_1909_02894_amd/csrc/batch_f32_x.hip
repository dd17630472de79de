// Batch phase kernel, f32, direction x.
#include "batch_kernels.hpp"
#include "batch_registry.hpp"

namespace dirac {
static BatchKernelRegistrar reg_batch_f32_x(1, 0,
    reinterpret_cast<const void*>(&batch_stage_kernel<float, false>),
    [](int logn, int s) { return batch_smem_for<float, false>(logn, s); });
}  // namespace dirac
