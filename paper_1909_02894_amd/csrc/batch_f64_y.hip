// Batch phase kernels, f64, direction y: one per (n, schedule).
#include "batch_kernels.hpp"
#include "batch_registry.hpp"

namespace dirac {

template <int N, int S>
struct BatchReg {
    BatchReg() {
        if constexpr (bsched_valid(N, S))
            BatchKernelRegistrar(0, 1, __builtin_ctz(N), S,
                                 reinterpret_cast<const void*>(&batch_group_kernel<double, true, N, S>),
                                 batch_smem_bytes_s<double, true, N, S>());
    }
};
#define BGK(N, S) static BatchReg<N, S> DIRAC_BCAT(breg_, __LINE__);
#define DIRAC_BCAT2(a, b) a##b
#define DIRAC_BCAT(a, b) DIRAC_BCAT2(a, b)
BGK(16, 0)
BGK(16, 1)
BGK(16, 2)
BGK(16, 3)
BGK(32, 0)
BGK(32, 1)
BGK(32, 2)
BGK(32, 3)
BGK(64, 0)
BGK(64, 1)
BGK(64, 2)
BGK(64, 3)
BGK(128, 0)
BGK(128, 1)
BGK(128, 2)
BGK(128, 3)
BGK(256, 0)
BGK(256, 1)
BGK(256, 2)
BGK(256, 3)
BGK(512, 0)
BGK(512, 1)
BGK(512, 2)
BGK(512, 3)
BGK(1024, 0)
BGK(1024, 1)
BGK(1024, 2)
BGK(1024, 3)
BGK(2048, 0)
BGK(2048, 1)
BGK(2048, 2)
BGK(2048, 3)

static BatchMultiRegistrar breg_multi(0, 1, reinterpret_cast<const void*>(&batch_multi_kernel<double, true>));

}  // namespace dirac
