// Direction-x (rows) kernel schedules, FP64, n = 16..256: REG(n, radix,
// lines per workgroup, spinor components per thread).  The first entry per n is
// the default schedule and also carries the observable kernel.
#include "stage_kernels.hpp"
#include "registry.hpp"
#define DIRAC_T double
#define DIRAC_PREC 0
#define DIRAC_COLS false
#define DIRAC_DIR 0
REGO(16, 4, 16, 2)
REG(16, 4, 8, 1)
REG(16, 4, 16, 1)
REGO(32, 4, 8, 2)
REG(32, 4, 4, 1)
REG(32, 4, 8, 1)
REGO(64, 4, 4, 2)
REG(64, 4, 2, 1)
REG(64, 8, 8, 2)
REGO(128, 4, 2, 2)
REG(128, 4, 1, 1)
REG(128, 8, 4, 2)
REG(128, 8, 2, 1)
REGO(256, 4, 1, 2)
REG(256, 4, 1, 1)
REG(256, 8, 2, 2)
REG(256, 8, 1, 1)
