// Direction-y (columns) kernel schedules, FP32, n = 512..8192: REG(n, radix,
// lines per workgroup, spinor components per thread).  The first entry per n is
// the default schedule and also carries the observable kernel.
#include "stage_kernels.hpp"
#include "registry.hpp"
#define DIRAC_T float
#define DIRAC_PREC 1
#define DIRAC_COLS true
#define DIRAC_DIR 1
REGO(512, 8, 4, 2)
REG(512, 8, 4, 1)
REG(512, 8, 2, 1)
REG(512, 8, 8, 2)
REG(512, 16, 8, 2)
REGO(1024, 8, 4, 1)
REG(1024, 8, 4, 2)
REG(1024, 16, 4, 2)
REGO(2048, 8, 2, 2)
REG(2048, 16, 4, 1)
REG(2048, 16, 4, 2)
REG(2048, 8, 4, 2)
REGO(4096, 16, 2, 2)
REG(4096, 16, 2, 1)
REG(4096, 8, 2, 2)
REGO(8192, 16, 1, 2)
REG(8192, 16, 1, 1)
REG(8192, 16, 2, 2)
