// Batch phase kernel, f64, direction y.
#include "batch_kernels.hpp"
#include "batch_registry.hpp"

namespace dirac {
static BatchKernelRegistrar reg_batch_f64_y(0, 1,
    reinterpret_cast<const void*>(&batch_stage_kernel<double, true>),
    [](int logn, int s) { return batch_smem_for<double, true>(logn, s); });
}  // namespace dirac
