// Direction-y (columns) kernel schedules, FP64, n = 16..256.  The first entry per n
// is the default schedule and also carries the observable kernel.
#include "stage_kernels.hpp"
#include "registry.hpp"
#define DIRAC_T double
#define DIRAC_PREC 0
#define DIRAC_COLS true
#define DIRAC_DIR 1
REGO(16, 4, 16)
REG(16, 4, 8)
REGO(32, 4, 8)
REG(32, 4, 4)
REGO(64, 4, 4)
REG(64, 8, 4)
REG(64, 8, 8)
REGO(128, 4, 4)
REG(128, 8, 4)
REG(128, 8, 8)
REGO(256, 8, 4)
REG(256, 8, 8)
REG(256, 4, 4)
