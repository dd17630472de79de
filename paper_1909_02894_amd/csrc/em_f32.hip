// em_f32.hip -- instantiations of the direction kernels with in-kernel
// time-dependent half-step exponentials (float).
#include <hip/hip_runtime.h>

#include "em_kernels.hpp"

namespace dirac {

#define EMK(N, DIR) \
    EmEntry{1, N, DIR, em_lines(N, DIR == 1), em_threads(N, DIR == 1), reinterpret_cast<const void*>(&em_stage_kernel<float, N, DIR == 1>)}

const EmEntry* em_entries_f32(int* count) {
    static const EmEntry e[] = {EMK(16, 0),  EMK(32, 0),  EMK(64, 0),  EMK(128, 0), EMK(256, 0),  EMK(512, 0),
                                EMK(1024, 0), EMK(2048, 0), EMK(16, 1), EMK(32, 1),  EMK(64, 1),   EMK(128, 1),
                                EMK(256, 1), EMK(512, 1), EMK(1024, 1), EMK(2048, 1)};
    *count = (int)(sizeof e / sizeof e[0]);
    return e;
}

}  // namespace dirac
