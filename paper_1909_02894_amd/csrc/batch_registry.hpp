// batch_registry.hpp -- the batch phase kernels per (precision, direction).
#pragma once
#include <stddef.h>

namespace dirac {

struct BatchKernel {
    const void* fn = nullptr;
    size_t (*smem)(int logn, int sched) = nullptr;
};

BatchKernel& batch_kernel(int prec, int dir);

struct BatchKernelRegistrar {
    BatchKernelRegistrar(int prec, int dir, const void* fn, size_t (*smem)(int, int)) {
        batch_kernel(prec, dir).fn = fn;
        batch_kernel(prec, dir).smem = smem;
    }
};

}  // namespace dirac
