// solver.hpp -- host-side state of one solve.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <vector>

#include "../../include/dirac.h"
#include "registry.hpp"

namespace dirac {

// Byte offsets of every region inside the caller's device buffer (256-aligned).
// SIZE_MAX marks a region the solve does not need.
struct Layout {
    size_t psi;        // state, n1 n2 points x 2 components x complex (T)
    size_t a;          // a(x) per point (T), curved metrics only
    size_t aT;         // the same, transposed ([n1][n2]: contiguous along columns), for the y direction
    size_t E;          // Step-1 exponential per point, 4 T (curved only)
    size_t da;         // (d_x a, d_y a) per point, 2 T (second-order directional step, curved only)
    size_t em;         // per-point record of the time-dependent exponential, 8 T (potentials only)
    size_t obs;        // 5 FP64 planes for the observables
    size_t fields;     // FIELDS metric staging, 6 FP64 planes
    size_t scratch;    // n1 n2 x 32 bytes: complex128 staging / autotune save
    size_t inv_s[2];   // 1/S per axis (T)
    size_t K[2];       // directional symbols per axis (complex T)
    size_t D[2];       // derivative symbols per axis (T)
    size_t tw[2];      // FFT twiddles per axis (complex T)
    size_t cn_vec;     // Scheme I: 2 sets of gmres_restart + 4 FP64 vectors (rhs, operator product x / y
                       // parts, basis), then a second state vector
    size_t cn_part;    // Scheme I: reduction partials
    size_t cn_coef;    // Scheme I: 2 sets of the device solve state and Arnoldi coefficient records
    size_t cn_vecbytes;
    size_t partials;   // reduction partials (FP64)
    size_t out;        // small reduction outputs (FP64)
    size_t total;      // footprint including alignment slack
};

dirac_status fail(dirac_status st, const char* fmt, ...);
dirac_status validate(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec,
                      const dirac_scheme* sc, const dirac_em* em);
Layout make_layout(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec,
                   const dirac_scheme* sc, const dirac_em* em);
double envelope_at(const dirac_envelope& e, double t);
dirac_scheme scheme_or_default(const dirac_scheme* sc);
dirac_status cn_step_n(dirac_solver* s, int64_t nsteps);
// Whether a solve with potentials runs its exponentials as a pointwise pass
// (plain direction kernels) rather than inside the direction kernels.
bool em_pass(const dirac_solver* s);
const KernelEntry* pick_entry(int prec, int n, int dir, int other, int mode);

}  // namespace dirac

struct dirac_solver {
    dirac_grid g{};
    dirac_metric metric{};
    dirac_pml pmlp{};
    int32_t prec = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    dirac::Layout lay{};
    bool curved = false, pml = false;
    double e0u_re = 1, e0u_im = 0;   // flat Step-1 factor e^{-i dt m c^2 / 2}
    int device = 0;
    double b_min = 1, b_max = 1;
    int64_t step = 0;
    bool has_state = false;
    const dirac::KernelEntry* sched[2] = {nullptr, nullptr};
    bool store_wt[2] = {false, false};   // write-through state stores, x / y direction kernels
    bool use_graph = true;
    int graph_chunk = 32;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<hipEvent_t> events;
    dirac_scheme scheme{};
    int64_t cn_iters = 0;
    double cn_last_res = 0;
    int cn_cycle_len = 0;             // Arnoldi columns of the last GMRES cycle (batch size hint)
    void* cn_head = nullptr;          // pinned host copies of the two GMRES state heads
    hipEvent_t cn_ev[2] = {nullptr, nullptr};
    bool has_em = false;             // time-dependent potentials
    int em_form = 0;                 // 0: by size, 1: exponentials inside the x / y kernels, 2: a pointwise pass
    double em_charge = 0;
    dirac_envelope env_V{}, env_A{};
};
