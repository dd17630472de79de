// d3_f32.hip -- instantiations of the 3-D, 4-spinor direction kernels (float).
#include <hip/hip_runtime.h>

#include "d3_kernels.hpp"

namespace dirac {

#define D3K(N, DIR)                                                                                  \
    D3Entry{1, N, DIR, d3_lines<float>(N), d3_threads<float>(N),                                          \
            {reinterpret_cast<const void*>(&d3_stage_kernel<float, N, DIR, 0>),                         \
             reinterpret_cast<const void*>(&d3_stage_kernel<float, N, DIR, 1>),                         \
             reinterpret_cast<const void*>(&d3_stage_kernel<float, N, DIR, 2>)}}
#define D3ALL(DIR) D3K(16, DIR), D3K(32, DIR), D3K(64, DIR), D3K(128, DIR), D3K(256, DIR), D3K(512, DIR), D3K(1024, DIR)

const D3Entry* d3_entries_f32(int* count) {
    static const D3Entry e[] = {D3ALL(0), D3ALL(1), D3ALL(2)};
    *count = (int)(sizeof e / sizeof e[0]);
    return e;
}

}  // namespace dirac
