// bis_f64.hip -- instantiations of the second-order directional kernels (double).
#include <hip/hip_runtime.h>

#include "bis_kernels.hpp"

namespace dirac {

#define BIS(N, DIR)                                                                                    \
    BisEntry{0, N, DIR, bis_lines(N, DIR == 1), bis_threads(N, DIR == 1),                              \
             {reinterpret_cast<const void*>(&bis_stage_kernel<double, N, DIR == 1, 1>),                   \
              reinterpret_cast<const void*>(&bis_stage_kernel<double, N, DIR == 1, 2>)}}

const BisEntry* bis_entries_f64(int* count) {
    static const BisEntry e[] = {BIS(16, 0),  BIS(32, 0),  BIS(64, 0),  BIS(128, 0), BIS(256, 0),  BIS(512, 0),
                                 BIS(1024, 0), BIS(2048, 0), BIS(16, 1), BIS(32, 1),  BIS(64, 1),   BIS(128, 1),
                                 BIS(256, 1), BIS(512, 1), BIS(1024, 1), BIS(2048, 1)};
    *count = (int)(sizeof e / sizeof e[0]);
    return e;
}

}  // namespace dirac
