// d3_f64.hip -- instantiations of the 3-D, 4-spinor direction kernels (double).
#include <hip/hip_runtime.h>

#include "d3_kernels.hpp"

namespace dirac {

#define D3K(N, DIR)                                                                                  \
    D3Entry{0, N, DIR, d3_lines<double>(N), d3_threads<double>(N),                                          \
            {reinterpret_cast<const void*>(&d3_stage_kernel<double, N, DIR, 0>),                         \
             reinterpret_cast<const void*>(&d3_stage_kernel<double, N, DIR, 1>),                         \
             reinterpret_cast<const void*>(&d3_stage_kernel<double, N, DIR, 2>)}}
#define D3ALL(DIR) D3K(16, DIR), D3K(32, DIR), D3K(64, DIR), D3K(128, DIR), D3K(256, DIR), D3K(512, DIR), D3K(1024, DIR)

const D3Entry* d3_entries_f64(int* count) {
    static const D3Entry e[] = {D3ALL(0), D3ALL(1), D3ALL(2)};
    *count = (int)(sizeof e / sizeof e[0]);
    return e;
}

}  // namespace dirac
