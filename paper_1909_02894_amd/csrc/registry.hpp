// registry.hpp -- compiled kernel variants of the direction and observable
// kernels, registered per (precision, n, direction, schedule) by the
// translation units that instantiate them.
#pragma once
#include <vector>

namespace dirac {

struct KernelEntry {
    int prec;       // 0 = FP64, 1 = FP32
    int n;          // transform length
    int dir;        // 0 = x (rows), 1 = y (columns)
    int radix;      // values per thread per component
    int lines;      // lines per workgroup
    int cpt;        // spinor components per thread (1 or 2)
    int nthreads;   // workgroup size
    const void* stage_fn[3];   // by mode: 0 flat, 1 flat + layer, 2 curved
    const void* obs_fn;
};

std::vector<KernelEntry>& kernel_registry();

struct Registrar {
    Registrar(const KernelEntry& e) { kernel_registry().push_back(e); }
};

}  // namespace dirac

// REG(N, R, L, CPT) inside a translation unit that defines DIRAC_T (double /
// float), DIRAC_PREC (0/1), DIRAC_COLS (false/true), DIRAC_DIR (0/1).
#define DIRAC_CAT2(a, b) a##b
#define DIRAC_CAT(a, b) DIRAC_CAT2(a, b)
#define DIRAC_REG_IMPL(N, R, L, CPT, OBS)                                                             \
    static ::dirac::Registrar DIRAC_CAT(reg_, __LINE__)(::dirac::KernelEntry{                        \
        DIRAC_PREC, N, DIRAC_DIR, R, L, CPT,                                                          \
        ::dirac::LineFFT<DIRAC_T, N, R, L, DIRAC_COLS, CPT>::NT,                                       \
        {reinterpret_cast<const void*>(&::dirac::stage_kernel<DIRAC_T, N, R, L, DIRAC_COLS, 0, CPT>), \
         reinterpret_cast<const void*>(&::dirac::stage_kernel<DIRAC_T, N, R, L, DIRAC_COLS, 1, CPT>), \
         reinterpret_cast<const void*>(&::dirac::stage_kernel<DIRAC_T, N, R, L, DIRAC_COLS, 2, CPT>)},\
        OBS});
// REG: a direction-kernel schedule.  REGO: the same plus the observable kernel
// with that schedule (one per precision, n and direction).
#define REG(N, R, L, CPT) DIRAC_REG_IMPL(N, R, L, CPT, nullptr)
#define REGO(N, R, L, CPT) \
    DIRAC_REG_IMPL(N, R, L, CPT, reinterpret_cast<const void*>(&::dirac::obs_kernel<DIRAC_T, N, R, L, DIRAC_COLS, CPT>))
