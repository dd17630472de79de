// batch_registry.hpp -- the batch phase kernels per (precision, direction,
// transform length, schedule), registered by the translation units that
// instantiate them.
#pragma once
#include <stddef.h>

namespace dirac {

struct BatchKernel {
    const void* fn = nullptr;
    size_t smem = 0;           // dynamic LDS bytes of one workgroup
};

// logn in [4, 11], sched in [0, 4)
BatchKernel& batch_kernel(int prec, int dir, int logn, int sched);
// the kernel that covers several size groups in one launch
const void*& batch_multi_kernel_fn(int prec, int dir);

struct BatchMultiRegistrar {
    BatchMultiRegistrar(int prec, int dir, const void* fn) { batch_multi_kernel_fn(prec, dir) = fn; }
};

struct BatchKernelRegistrar {
    BatchKernelRegistrar(int prec, int dir, int logn, int sched, const void* fn, size_t smem) {
        batch_kernel(prec, dir, logn, sched).fn = fn;
        batch_kernel(prec, dir, logn, sched).smem = smem;
    }
};

}  // namespace dirac
