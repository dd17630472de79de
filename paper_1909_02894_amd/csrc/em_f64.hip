// em_f64.hip -- instantiations of the direction kernels with in-kernel
// time-dependent half-step exponentials (double).
#include <hip/hip_runtime.h>

#include "em_kernels.hpp"

namespace dirac {

#define EMK(N, DIR) \
    EmEntry{0, N, DIR, em_lines(N, DIR == 1), em_threads(N, DIR == 1), reinterpret_cast<const void*>(&em_stage_kernel<double, N, DIR == 1>)}

const EmEntry* em_entries_f64(int* count) {
    static const EmEntry e[] = {EMK(16, 0),  EMK(32, 0),  EMK(64, 0),  EMK(128, 0), EMK(256, 0),  EMK(512, 0),
                                EMK(1024, 0), EMK(2048, 0), EMK(16, 1), EMK(32, 1),  EMK(64, 1),   EMK(128, 1),
                                EMK(256, 1), EMK(512, 1), EMK(1024, 1), EMK(2048, 1)};
    *count = (int)(sizeof e / sizeof e[0]);
    return e;
}

hipError_t launch_em_exp(const double* in, double* out, const double* rec, size_t npts, int times, const double* fA,
                         const double* fV, hipStream_t s) {
    if (times < 1 || times > 2) return hipErrorInvalidValue;
    EmExpParams<double> p{in, out, rec, npts, times, {fA[0], fA[1]}, {fV[0], fV[1]}};
    hipLaunchKernelGGL(em_exp_kernel<double>, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

const void* em_exp_fn(int prec) {
    return prec == 0 ? reinterpret_cast<const void*>(&em_exp_kernel<double>)
                     : reinterpret_cast<const void*>(&em_exp_kernel<float>);
}

}  // namespace dirac
