// Direction-y (columns) kernel schedules, FP64, n = 512..4096: REG(n, radix,
// lines per workgroup, spinor components per thread).  The first entry per n is
// the default schedule and also carries the observable kernel.
#include "stage_kernels.hpp"
#include "registry.hpp"
#define DIRAC_T double
#define DIRAC_PREC 0
#define DIRAC_COLS true
#define DIRAC_DIR 1
REGO(512, 8, 2, 1)
REG(512, 4, 2, 2)
REG(512, 8, 2, 2)
REG(512, 8, 4, 2)
REG(512, 8, 4, 1)
REG(512, 8, 1, 1)
REGO(1024, 8, 4, 2)
REG(1024, 8, 4, 1)
REG(1024, 8, 2, 2)
REGO(2048, 8, 2, 2)
REG(2048, 8, 1, 2)
REG(2048, 8, 2, 1)
REG(2048, 16, 2, 2)
REGO(4096, 8, 1, 2)
REG(4096, 8, 1, 1)
REG(4096, 8, 2, 2)
