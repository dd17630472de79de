// Batch phase kernel, f64, direction x.
#include "batch_kernels.hpp"
#include "batch_registry.hpp"

namespace dirac {
static BatchKernelRegistrar reg_batch_f64_x(0, 0,
    reinterpret_cast<const void*>(&batch_stage_kernel<double, false>),
    [](int logn, int s) { return batch_smem_for<double, false>(logn, s); });
}  // namespace dirac
