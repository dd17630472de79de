// runtime.hip -- the C ABI of libdirac: validation, device-buffer layout,
// setup, the step launcher (direct or HIP-graph replay), observables,
// conversions, schedules, timing and the autotuner.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cassert>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dirac.h"
#include "fft_line.hpp"
#include "registry.hpp"
#include "setup_kernels.hpp"
#include "solver.hpp"
#include "stage_kernels.hpp"
#include "cn_kernels.hpp"
#include "bis_kernels.hpp"
#include "em_kernels.hpp"

namespace dirac {

const EmEntry* em_entries_f64(int* count);
const EmEntry* em_entries_f32(int* count);

const EmEntry* em_entry(int prec, int n, int dir) {
    int cnt = 0;
    const EmEntry* e = prec == DIRAC_FP64 ? em_entries_f64(&cnt) : em_entries_f32(&cnt);
    for (int i = 0; i < cnt; ++i)
        if (e[i].n == n && e[i].dir == dir) return &e[i];
    return nullptr;
}

double envelope_at(const dirac_envelope& e, double t) {
    const double g = e.tau > 0 ? std::exp(-((t - e.t0) / e.tau) * ((t - e.t0) / e.tau)) : 1.0;
    return e.c0 + e.c1 * std::sin(e.omega * t + e.phase) * g;
}

const BisEntry* bis_entries_f64(int* count);
const BisEntry* bis_entries_f32(int* count);

const BisEntry* bis_entry(int prec, int n, int dir) {
    int cnt = 0;
    const BisEntry* e = prec == DIRAC_FP64 ? bis_entries_f64(&cnt) : bis_entries_f32(&cnt);
    for (int i = 0; i < cnt; ++i)
        if (e[i].n == n && e[i].dir == dir) return &e[i];
    return nullptr;
}

std::vector<KernelEntry>& kernel_registry() {
    static std::vector<KernelEntry> r;
    return r;
}

static thread_local std::string g_last_error;

dirac_status fail(dirac_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

static dirac_status hip_fail(hipError_t e, const char* what) {
    return fail(DIRAC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}
#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return hip_fail(e_, (what));    \
    } while (0)

static bool is_pow2_in_range(int n) { return n >= 16 && n <= 8192 && (n & (n - 1)) == 0; }
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------- validation

dirac_scheme scheme_or_default(const dirac_scheme* sc) {
    dirac_scheme d{};
    if (sc) d = *sc;
    if (d.scheme == DIRAC_SCHEME_CN_GMRES) {
        if (d.gmres_restart == 0) d.gmres_restart = 20;
        if (d.gmres_max_iter == 0) d.gmres_max_iter = 400;
        if (d.gmres_rtol == 0) d.gmres_rtol = 1e-13;
    }
    return d;
}

static bool envelope_ok(const dirac_envelope& e) {
    return std::isfinite(e.c0) && std::isfinite(e.c1) && std::isfinite(e.omega) && std::isfinite(e.phase) &&
           std::isfinite(e.t0) && std::isfinite(e.tau) && e.tau >= 0;
}

dirac_status validate(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec,
                      const dirac_scheme* scp, const dirac_em* em) {
    if (!g || !m || !pml) return fail(DIRAC_E_ARG, "null grid, metric or pml");
    if (em) {
        if (!std::isfinite(em->charge)) return fail(DIRAC_E_ARG, "charge must be finite");
        if (!envelope_ok(em->fV) || !envelope_ok(em->fA))
            return fail(DIRAC_E_ARG, "envelope parameters must be finite with tau >= 0");
        if (scp && scp->scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS)
            return fail(DIRAC_E_ARG, "potentials are built for the plain and printed directional steps and Scheme I");
        if (g->n1 > 2048 || g->n2 > 2048) return fail(DIRAC_E_SIZE, "solves with potentials need n1, n2 <= 2048");
    }
    const dirac_scheme sc = scheme_or_default(scp);
    if (sc.scheme < DIRAC_SCHEME_EXP_SPLIT || sc.scheme > DIRAC_SCHEME_EXP_SPLIT_2BIS)
        return fail(DIRAC_E_ARG, "unknown scheme %d", sc.scheme);
    if (sc.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS && (g->n1 > 2048 || g->n2 > 2048))
        return fail(DIRAC_E_SIZE, "the second-order directional step is built for n1, n2 <= 2048");
    if (sc.scheme == DIRAC_SCHEME_CN_GMRES) {
        if (prec != DIRAC_FP64) return fail(DIRAC_E_ARG, "Scheme I is built in FP64 only");
        if (g->n1 > 2048 || g->n2 > 2048) return fail(DIRAC_E_SIZE, "Scheme I needs n1, n2 <= 2048");
        if (sc.gmres_restart < 2 || sc.gmres_restart > 63) return fail(DIRAC_E_ARG, "gmres_restart must be in [2, 63]");
        if (sc.gmres_max_iter < 1) return fail(DIRAC_E_ARG, "gmres_max_iter must be >= 1");
        if (!(sc.gmres_rtol > 0) || !std::isfinite(sc.gmres_rtol)) return fail(DIRAC_E_ARG, "gmres_rtol must be > 0");
    }
    if (prec != DIRAC_FP64 && prec != DIRAC_FP32) return fail(DIRAC_E_ARG, "precision must be 0 (FP64) or 1 (FP32)");
    if (!is_pow2_in_range(g->n1) || !is_pow2_in_range(g->n2))
        return fail(DIRAC_E_SIZE, "n1 = %d, n2 = %d: each must be a power of two in [16, 8192]", g->n1, g->n2);
    if ((size_t)g->n1 * g->n2 * 4 * (prec == DIRAC_FP32 ? 4 : 8) >= (size_t(1) << 31))
        return fail(DIRAC_E_SIZE, "state of %d x %d points does not fit 2 GiB of 32-bit offsets", g->n1, g->n2);
    if (!(g->a1 > 0) || !(g->a2 > 0) || !std::isfinite(g->a1) || !std::isfinite(g->a2))
        return fail(DIRAC_E_ARG, "half-widths a1, a2 must be finite and > 0");
    if (!(g->dt > 0) || !std::isfinite(g->dt)) return fail(DIRAC_E_ARG, "dt must be finite and > 0");
    if (!(g->c > 0) || !std::isfinite(g->c)) return fail(DIRAC_E_ARG, "c must be finite and > 0");
    if (!(g->m >= 0) || !std::isfinite(g->m)) return fail(DIRAC_E_ARG, "m must be finite and >= 0");
    if (sc.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS_PRINTED) {
        // per-mode factor b (1 - theta^2) e^{-i theta} + 1 - b stays in the unit
        // disk for every b in [0, 1] iff |1 - theta^2| <= 1
        const double th1 = g->c * g->dt * M_PI * (g->n1 / 2) / g->a1;
        const double th2 = g->c * g->dt * M_PI * (g->n2 / 2) / g->a2;
        if (std::max(th1, th2) > std::sqrt(2.0))
            return fail(DIRAC_E_UNSTABLE, "eq. (step2bis) as printed needs c dt max|xi| <= sqrt(2); got %.6g",
                        std::max(th1, th2));
    }
    if (m->kind < 0 || m->kind > 3) return fail(DIRAC_E_ARG, "unknown metric kind %d", m->kind);
    if (m->spin < 0 || m->spin > 2) return fail(DIRAC_E_ARG, "unknown spin selector %d", m->spin);
    if (m->kind == DIRAC_METRIC_GAUSS_BUMP && (!(m->bump_s > 0) || !std::isfinite(m->bump_s) || !std::isfinite(m->bump_A)))
        return fail(DIRAC_E_ARG, "bump_s must be finite and > 0, bump_A finite");
    if (m->kind == DIRAC_METRIC_FIELDS &&
        (!m->phi || !m->psi || !m->dphi_dx || !m->dphi_dy || !m->dpsi_dx || !m->dpsi_dy))
        return fail(DIRAC_E_ARG, "FIELDS metric needs all six host arrays");
    if (pml->width_pts < 0 || pml->width_pts > std::min(g->n1, g->n2) / 2)
        return fail(DIRAC_E_ARG, "pml width %d outside [0, min(n1, n2)/2]", pml->width_pts);
    if (pml->width_pts > 0) {
        if (pml->type < 1 || pml->type > 6) return fail(DIRAC_E_ARG, "pml type must be 1..6");
        if (!std::isfinite(pml->sigma0) || pml->sigma0 < 0) return fail(DIRAC_E_ARG, "pml sigma0 must be finite and >= 0");
        if (!std::isfinite(pml->theta)) return fail(DIRAC_E_ARG, "pml theta must be finite");
        if (std::fabs(std::sin(pml->theta)) > 0 && pml->sigma0 > 0 && sc.scheme == DIRAC_SCHEME_CN_GMRES)
            return fail(DIRAC_E_ARG, "Scheme I is built for a real stretch S (theta = %g has sin != 0)", pml->theta);
        if (std::fabs(std::sin(pml->theta)) > 0 && pml->sigma0 > 0)
            return fail(DIRAC_E_UNSTABLE,
                        "complex stretch (theta = %g) makes the blend coefficient complex; the directional "
                        "step is stable only for real b in [0, 1]", pml->theta);
    }
    return DIRAC_OK;
}

Layout make_layout(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec,
                   const dirac_scheme* scp, const dirac_em* em) {
    Layout L{};
    const dirac_scheme sc = scheme_or_default(scp);
    const size_t N = (size_t)g->n1 * g->n2;
    const size_t sz = prec == DIRAC_FP32 ? 4 : 8;
    const bool curved = m->kind != DIRAC_METRIC_FLAT;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.psi = take(N * 4 * sz);
    L.a = curved ? take(N * sz) : SIZE_MAX;
    L.aT = curved ? take(N * sz) : SIZE_MAX;
    L.E = curved ? take(N * 4 * sz) : SIZE_MAX;
    L.da = curved && sc.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS ? take(N * 2 * sz) : SIZE_MAX;
    L.em = em ? take(N * 8 * sz) : SIZE_MAX;
    L.obs = take((em ? 8 : 5) * N * 8);
    L.fields = m->kind == DIRAC_METRIC_FIELDS ? take(6 * N * 8) : SIZE_MAX;
    L.scratch = take(N * 4 * 8);
    for (int ax = 0; ax < 2; ++ax) {
        const size_t n = ax == 0 ? g->n1 : g->n2;
        L.inv_s[ax] = take(n * sz);
        L.K[ax] = take(n * 2 * sz);
        L.D[ax] = take(n * sz);
        L.tw[ax] = take(n * 2 * sz);
    }
    const size_t setup_parts = ((N + 255) / 256) * 3;
    const size_t obs_parts = ((size_t)g->n1 + g->n2) * 8;
    if (sc.scheme == DIRAC_SCHEME_CN_GMRES) {
        // two sets (consecutive steps alternate) of: rhs, the two parts of an
        // operator product and the m + 1 basis vectors; then the second state
        L.cn_vecbytes = align256(N * 32);
        L.cn_vec = take(L.cn_vecbytes * (2 * (size_t)(sc.gmres_restart + 4) + 1));
        L.cn_part = take((size_t)kCnDotBlocks * (kCnMaxRestart + 2) * 2 * 8);
        // per set: the device-resident solve state, then one coefficient record per iteration
        L.cn_coef = take(2 * (align256(sizeof(CnCtrl)) + (size_t)sc.gmres_restart * kCnRecDoubles * 8));
    } else {
        L.cn_vec = L.cn_part = L.cn_coef = SIZE_MAX;
        L.cn_vecbytes = 0;
    }
    L.partials = take(std::max(setup_parts, obs_parts) * 8);
    L.out = take(64 * 8);
    L.total = off + 256;     // slack so that an unaligned caller buffer can be aligned up
    (void)pml;
    return L;
}

// ---------------------------------------------------------------- schedules

const KernelEntry* find_entry(int prec, int n, int dir, const dirac_schedule& s) {
    for (const auto& e : kernel_registry())
        if (e.prec == prec && e.n == n && e.dir == dir && e.radix == s.radix && e.lines == s.lines_per_wg &&
            e.cpt == s.components_per_thread)
            return &e;
    return nullptr;
}
const KernelEntry* default_entry(int prec, int n, int dir) {
    for (const auto& e : kernel_registry())
        if (e.prec == prec && e.n == n && e.dir == dir) return &e;
    return nullptr;
}
const KernelEntry* obs_entry(int prec, int n, int dir) {
    for (const auto& e : kernel_registry())
        if (e.prec == prec && e.n == n && e.dir == dir && e.obs_fn) return &e;
    return nullptr;
}

struct TuneKey {
    int prec, n, dir, other, mode;
    bool operator<(const TuneKey& o) const {
        return std::tie(prec, n, dir, other, mode) < std::tie(o.prec, o.n, o.dir, o.other, o.mode);
    }
};
struct TuneVal { int radix, lines, cpt; double ms; int wt; };
static std::map<TuneKey, TuneVal>& tune_cache() { static std::map<TuneKey, TuneVal> c; return c; }
static std::mutex& tune_mutex() { static std::mutex m; return m; }

int solver_mode(const dirac_solver* s) { return (s->curved ? 2 : 0) + (s->pml ? 1 : 0); }
// Tuning-cache mode: the kernel mode plus the kernel family (the corrected
// second-order step and the potential kernels are tuned apart).
int tune_mode(const dirac_solver* s) {
    return solver_mode(s) + (s->scheme.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS ? 4 : 0) +
           (s->has_em && !em_pass(s) ? 8 : 0);
}

// Whether the direction kernel carries the write-through store path (every
// row kernel; column kernels up to kStoreWtMaxColN points, stage_tile).
bool store_wt_compiled(const dirac_solver* s, int dir) { return dir == 0 || s->g.n2 <= kStoreWtMaxColN; }

// Store mode the autotuner measured fastest for this direction and shape, else
// ordinary stores.
bool pick_store_mode(int prec, int n, int dir, int other, int mode) {
    std::lock_guard<std::mutex> lk(tune_mutex());
    auto it = tune_cache().find(TuneKey{prec, n, dir, other, mode});
    return it != tune_cache().end() && it->second.wt != 0;
}

const KernelEntry* pick_entry(int prec, int n, int dir, int other, int mode) {
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        auto it = tune_cache().find(TuneKey{prec, n, dir, other, mode});
        if (it != tune_cache().end()) {
            dirac_schedule sc{it->second.radix, it->second.lines, it->second.cpt};
            if (const KernelEntry* e = find_entry(prec, n, dir, sc)) return e;
        }
    }
    return default_entry(prec, n, dir);
}

// ---------------------------------------------------------------- launches

template <typename T>
StageParams<T> stage_params(const dirac_solver* s, int dir, int e_pre, int e_post) {
    StageParams<T> p{};
    char* b = s->base;
    p.psi = reinterpret_cast<T*>(b + s->lay.psi);
    // along this direction's lines: rows read a, columns its transpose
    p.a = s->curved ? reinterpret_cast<const T*>(b + (dir == 0 ? s->lay.a : s->lay.aT)) : nullptr;
    p.E = s->curved ? reinterpret_cast<const T*>(b + s->lay.E) : nullptr;
    p.inv_s = reinterpret_cast<const T*>(b + s->lay.inv_s[dir]);     // ones without a layer
    p.K = reinterpret_cast<const cpx<T>*>(b + s->lay.K[dir]);
    p.tw = reinterpret_cast<const cpx<T>*>(b + s->lay.tw[dir]);
    p.n1 = s->g.n1;
    p.nlines = dir == 0 ? s->g.n2 : s->g.n1;
    assert(dir == 0 || e_pre == 0);                 // Step 1 belongs to the row launch
    p.e_pre = e_pre;
    p.e_post = e_post;
    p.e0u = cpx<T>{(T)s->e0u_re, (T)s->e0u_im};
    p.wt = s->store_wt[dir] ? 1 : 0;
    return p;
}

template <typename T>
BisParams<T> bis_params(const dirac_solver* s, int dir, int e_pre, int e_post) {
    BisParams<T> p{};
    char* b = s->base;
    p.s = stage_params<T>(s, dir, e_pre, e_post);
    p.da = s->lay.da != SIZE_MAX ? reinterpret_cast<const T*>(b + s->lay.da) : nullptr;
    p.D = reinterpret_cast<const T*>(b + s->lay.D[dir]);
    p.hh = (T)(0.5 * (s->g.c * s->g.dt) * (s->g.c * s->g.dt));
    p.n = (T)(dir == 0 ? s->g.n1 : s->g.n2);
    return p;
}

template <typename T>
EmParams<T> em_params(const dirac_solver* s, int dir, int e_pre, int e_post, int64_t step) {
    EmParams<T> p{};
    p.s = stage_params<T>(s, dir, e_pre, e_post);
    p.rec = reinterpret_cast<const T*>(s->base + s->lay.em);
    // Step 1 of step n (and Step 5 of step n - 1 before it) and Step 5 of step n
    // evaluate the potentials at t_{n+1/2} (resp. t_{n-1/2})
    const double dt = s->g.dt;
    double times[3] = {0, 0, 0};
    if (e_pre == 2) { times[0] = (step - 0.5) * dt; times[1] = (step + 0.5) * dt; }
    else if (e_pre == 1) { times[0] = (step + 0.5) * dt; }
    times[2] = (step + 0.5) * dt;
    for (int k = 0; k < 3; ++k) {
        p.fA[k] = envelope_at(s->env_A, times[k]);
        p.fV[k] = envelope_at(s->env_V, times[k]);
    }
    return p;
}

static constexpr size_t kMaxParams = sizeof(BisParams<double>) > sizeof(EmParams<double>) ? sizeof(BisParams<double>)
                                                                                          : sizeof(EmParams<double>);
static_assert(sizeof(EmExpParams<double>) <= kMaxParams, "parameter block");

// States whose per-point data (state + potential record, 12 reals a point) fit
// this many bytes run the potentials' exponentials as a pointwise pass of
// their own, at full occupancy, with the direction kernels in their plain form:
// the data stays in the Infinity Cache, so the extra pass is cheap, while the
// exponentials inside the direction kernels lengthen their latency-bound chains.
// Larger states keep them in the direction kernels (one HBM round trip less).
constexpr size_t kEmPassMaxBytes = size_t(128) << 20;

bool em_pass(const dirac_solver* s) {
    if (!s->has_em) return false;
    if (s->em_form != 0) return s->em_form == 2;
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    return N * 12 * (s->prec == DIRAC_FP32 ? 4 : 8) <= kEmPassMaxBytes;
}

// One stage launch description (kernel + by-value parameter block).
struct Launch {
    const void* fn;
    dim3 grid, block;
    alignas(16) unsigned char params[kMaxParams];
    size_t psize;
};

// `step` is the index of the step the launch belongs to (it fixes the time of
// the potentials; unused otherwise).
Launch make_launch(const dirac_solver* s, int dir, int e_pre, int e_post, int64_t step = 0) {
    Launch L{};
    if (em_pass(s)) {              // the exponentials run in their own pass (make_exp_launch)
        // curved x kernels always apply their E table once: solves with potentials
        // hold the identity there (their exponentials come from the record)
        e_pre = s->curved && dir == 0 ? 1 : 0;
        e_post = 0;
    } else if (s->has_em) {
        const int nlines = dir == 0 ? s->g.n2 : s->g.n1;
        const EmEntry* e = em_entry(s->prec, dir == 0 ? s->g.n1 : s->g.n2, dir);
        L.fn = e->fn;
        L.grid = dim3((nlines + e->lines - 1) / e->lines);
        L.block = dim3(e->nthreads);
        if (s->prec == DIRAC_FP64) {
            auto p = em_params<double>(s, dir, e_pre, e_post, step);
            std::memcpy(L.params, &p, sizeof p);
            L.psize = sizeof p;
        } else {
            auto p = em_params<float>(s, dir, e_pre, e_post, step);
            std::memcpy(L.params, &p, sizeof p);
            L.psize = sizeof p;
        }
        return L;
    }
    if (s->scheme.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS && (s->curved || s->pml)) {
        // second-order directional step (b = 1 everywhere makes it the plain step)
        const int nlines = dir == 0 ? s->g.n2 : s->g.n1;
        const BisEntry* e = bis_entry(s->prec, dir == 0 ? s->g.n1 : s->g.n2, dir);
        L.fn = e->fn[s->curved ? 1 : 0];
        L.grid = dim3((nlines + e->lines - 1) / e->lines);
        L.block = dim3(e->nthreads);
        if (s->prec == DIRAC_FP64) {
            auto p = bis_params<double>(s, dir, e_pre, e_post);
            std::memcpy(L.params, &p, sizeof p);
            L.psize = sizeof p;
        } else {
            auto p = bis_params<float>(s, dir, e_pre, e_post);
            std::memcpy(L.params, &p, sizeof p);
            L.psize = sizeof p;
        }
        return L;
    }
    const KernelEntry* e = s->sched[dir];
    const int nlines = dir == 0 ? s->g.n2 : s->g.n1;
    L.fn = e->stage_fn[s->curved ? 2 : (s->pml ? 1 : 0)];
    L.grid = dim3((nlines + e->lines - 1) / e->lines);
    L.block = dim3(e->nthreads);
    if (s->prec == DIRAC_FP64) {
        auto p = stage_params<double>(s, dir, e_pre, e_post);
        std::memcpy(L.params, &p, sizeof p);
        L.psize = sizeof p;
    } else {
        auto p = stage_params<float>(s, dir, e_pre, e_post);
        std::memcpy(L.params, &p, sizeof p);
        L.psize = sizeof p;
    }
    return L;
}

// The pointwise potentials pass: Step 5 of step - 1 and Step 1 of step
// (times = 2, at t_{step-1/2} and t_{step+1/2}), Step 1 alone (times = 1,
// t_{step+1/2}), or Step 5 after the last step (closing, t_{step+1/2}).
Launch make_exp_launch(const dirac_solver* s, int times, int64_t step) {
    Launch L{};
    const size_t npts = (size_t)s->g.n1 * s->g.n2;
    const double dt = s->g.dt;
    const double t[2] = {times == 2 ? (step - 0.5) * dt : (step + 0.5) * dt, (step + 0.5) * dt};
    L.fn = em_exp_fn(s->prec == DIRAC_FP64 ? 0 : 1);
    L.grid = dim3((unsigned)((npts + 255) / 256));
    L.block = dim3(256);
    auto fill = [&](auto* psi, auto* rec) {
        using T = std::remove_const_t<std::remove_pointer_t<decltype(rec)>>;
        EmExpParams<T> p{psi, psi, rec, npts, times, {0, 0}, {0, 0}};
        for (int k = 0; k < times; ++k) {
            p.fA[k] = envelope_at(s->env_A, t[k]);
            p.fV[k] = envelope_at(s->env_V, t[k]);
        }
        std::memcpy(L.params, &p, sizeof p);
        L.psize = sizeof p;
    };
    if (s->prec == DIRAC_FP64)
        fill(reinterpret_cast<double*>(s->base + s->lay.psi), reinterpret_cast<const double*>(s->base + s->lay.em));
    else
        fill(reinterpret_cast<float*>(s->base + s->lay.psi), reinterpret_cast<const float*>(s->base + s->lay.em));
    return L;
}

static hipError_t do_launch(Launch& L, hipStream_t st) {
    void* args[] = {L.params};
    return hipLaunchKernel(L.fn, L.grid, L.block, args, 0, st);
}

// The stream is synchronised first: a replay of the graph may still be in flight.
static void drop_graph(dirac_solver* s) {
    if (s->gexec) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipGraphExecDestroy(s->gexec);
        s->gexec = nullptr;
    }
    if (s->graph) { (void)hipGraphDestroy(s->graph); s->graph = nullptr; }
}

// Graph of `chunk` middle steps: [y (no Step 5), x (Step 5 + Step 1)] repeated.
static dirac_status build_graph(dirac_solver* s) {
    drop_graph(s);
    HIP_TRY(hipGraphCreate(&s->graph, 0), "hipGraphCreate");
    Launch ly = make_launch(s, 1, 0, 0);
    Launch lx = make_launch(s, 0, 2, 0);
    hipGraphNode_t prev = nullptr;
    for (int c = 0; c < s->graph_chunk; ++c) {
        for (Launch* L : {&ly, &lx}) {
            void* args[] = {L->params};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(L->fn);
            kp.gridDim = L->grid;
            kp.blockDim = L->block;
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node;
            HIP_TRY(hipGraphAddKernelNode(&node, s->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp),
                    "hipGraphAddKernelNode");
            prev = node;
        }
    }
    HIP_TRY(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return DIRAC_OK;
}

// Enqueue nsteps steps: x(E once) y, then (y, x(E twice)) pairs, then y(+E).
dirac_status enqueue_steps(dirac_solver* s, int64_t nsteps, bool allow_graph) {
    if (nsteps <= 0) return DIRAC_OK;
    hipStream_t st = s->stream;
    if (em_pass(s)) {
        // the potentials' time enters the pass's parameters: direct launches
        const int64_t n0 = s->step;
        Launch lx = make_launch(s, 0, 0, 0), ly = make_launch(s, 1, 0, 0);
        for (int64_t k = 0; k < nsteps; ++k) {
            Launch le = make_exp_launch(s, k == 0 ? 1 : 2, n0 + k);
            HIP_TRY(do_launch(le, st), "launch potentials pass");
            HIP_TRY(do_launch(lx, st), "launch x stage");
            HIP_TRY(do_launch(ly, st), "launch y stage");
        }
        Launch lc = make_exp_launch(s, 1, n0 + nsteps - 1);
        HIP_TRY(do_launch(lc, st), "launch potentials pass");
        return DIRAC_OK;
    }
    if (s->has_em) {
        // the potentials' time enters every launch's parameters: direct launches
        const int64_t n0 = s->step;
        for (int64_t k = 0; k < nsteps; ++k) {
            Launch lx = make_launch(s, 0, k == 0 ? 1 : 2, 0, n0 + k);
            Launch ly = make_launch(s, 1, 0, k == nsteps - 1 ? 1 : 0, n0 + k);
            HIP_TRY(do_launch(lx, st), "launch x stage");
            HIP_TRY(do_launch(ly, st), "launch y stage");
        }
        return DIRAC_OK;
    }
    Launch x1 = make_launch(s, 0, 1, 0);
    HIP_TRY(do_launch(x1, st), "launch x stage");
    int64_t middle = nsteps - 1;     // number of (y, x(E E)) pairs
    if (allow_graph && s->use_graph && middle >= s->graph_chunk) {
        if (!s->gexec) {
            dirac_status r = build_graph(s);
            if (r != DIRAC_OK) return r;
        }
        while (middle >= s->graph_chunk) {
            HIP_TRY(hipGraphLaunch(s->gexec, st), "hipGraphLaunch");
            middle -= s->graph_chunk;
        }
    }
    if (middle > 0) {
        Launch y0 = make_launch(s, 1, 0, 0);
        Launch x2 = make_launch(s, 0, 2, 0);
        for (int64_t k = 0; k < middle; ++k) {
            HIP_TRY(do_launch(y0, st), "launch y stage");
            HIP_TRY(do_launch(x2, st), "launch x stage");
        }
    }
    Launch y1 = make_launch(s, 1, 0, 1);
    HIP_TRY(do_launch(y1, st), "launch y stage");
    return DIRAC_OK;
}

}  // namespace dirac

using namespace dirac;

// ============================================================== C ABI

extern "C" {

const char* dirac_last_error(void) { return g_last_error.c_str(); }

size_t dirac_footprint_bytes(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec) {
    return dirac_footprint_bytes_scheme(g, m, pml, prec, nullptr);
}

size_t dirac_footprint_bytes_scheme(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec,
                                    const dirac_scheme* sc) {
    return dirac_footprint_bytes_ex(g, m, pml, prec, sc, nullptr);
}

size_t dirac_footprint_bytes_ex(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml, int32_t prec,
                                const dirac_scheme* sc, const dirac_em* em) {
    if (validate(g, m, pml, prec, sc, em) != DIRAC_OK) return 0;
    return make_layout(g, m, pml, prec, sc, em).total;
}

dirac_status dirac_create_metric(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml,
                                 int32_t prec, void* device_buffer, size_t bytes, void* hip_stream,
                                 dirac_solver** out) {
    return dirac_create_solver(g, m, pml, prec, nullptr, nullptr, device_buffer, bytes, hip_stream, out);
}

dirac_status dirac_cn_stats(const dirac_solver* s, int64_t* iterations, double* last_rel_residual) {
    if (!s || !iterations || !last_rel_residual) return fail(DIRAC_E_ARG, "null argument");
    *iterations = s->cn_iters;
    *last_rel_residual = s->cn_last_res;
    return DIRAC_OK;
}

dirac_status dirac_cn_set_limits(dirac_solver* s, int32_t max_iter, double rtol) {
    if (!s) return fail(DIRAC_E_ARG, "null solver");
    if (s->scheme.scheme != DIRAC_SCHEME_CN_GMRES) return fail(DIRAC_E_ARG, "not a Scheme I solver");
    if (max_iter < 1) return fail(DIRAC_E_ARG, "max_iter must be >= 1");
    if (!(rtol > 0) || !std::isfinite(rtol)) return fail(DIRAC_E_ARG, "rtol must be finite and > 0");
    s->scheme.gmres_max_iter = max_iter;
    s->scheme.gmres_rtol = rtol;
    return DIRAC_OK;
}

dirac_status dirac_create_solver(const dirac_grid* g, const dirac_metric* m, const dirac_pml* pml,
                                 int32_t prec, const dirac_scheme* scp, const dirac_em* em, void* device_buffer,
                                 size_t bytes, void* hip_stream, dirac_solver** out) {
    g_last_error.clear();
    if (!out) return fail(DIRAC_E_ARG, "null output handle");
    *out = nullptr;
    dirac_status st = validate(g, m, pml, prec, scp, em);
    if (st != DIRAC_OK) return st;
    if (!device_buffer) return fail(DIRAC_E_ARG, "null device buffer");
    const dirac_scheme sc = scheme_or_default(scp);
    Layout lay = make_layout(g, m, pml, prec, scp, em);
    if (bytes < lay.total)
        return fail(DIRAC_E_SIZE, "device buffer of %zu bytes < footprint %zu", bytes, lay.total);
    for (int dir = 0; dir < 2; ++dir) {
        const int n = dir == 0 ? g->n1 : g->n2;
        if (!default_entry(prec, n, dir) || !obs_entry(prec, n, dir))
            return fail(DIRAC_E_SIZE, "no compiled kernel for n = %d (precision %d, direction %d)", n, prec, dir);
    }
    // Check the pointer is device memory of the current device.
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, device_buffer) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(DIRAC_E_ARG, "device_buffer is not device memory");
    }
    dirac_solver* s = new (std::nothrow) dirac_solver();
    if (!s) return fail(DIRAC_E_NOMEM, "host allocation failed");
    s->g = *g;
    s->metric = *m;
    s->metric.phi = s->metric.psi = s->metric.dphi_dx = s->metric.dphi_dy = s->metric.dpsi_dx = s->metric.dpsi_dy = nullptr;
    s->pmlp = *pml;
    s->prec = prec;
    s->scheme = sc;
    if (em) {
        s->has_em = true;
        s->em_charge = em->charge;
        s->env_V = em->fV;
        s->env_A = em->fA;
    }
    s->stream = static_cast<hipStream_t>(hip_stream);
    const uintptr_t raw = reinterpret_cast<uintptr_t>(device_buffer);
    s->base = reinterpret_cast<char*>((raw + 255) & ~uintptr_t(255));
    s->lay = lay;
    s->curved = m->kind != DIRAC_METRIC_FLAT;
    s->pml = pml->width_pts > 0;
    const double mu = g->dt * g->m * g->c * g->c / 2.0;
    s->e0u_re = std::cos(mu);
    s->e0u_im = -std::sin(mu);
    hipGetDevice(&s->device);

    auto bail = [&](dirac_status r) { delete s; return r; };
    const size_t N = (size_t)g->n1 * g->n2;
    const bool fp32 = prec == DIRAC_FP32;
    char* b = s->base;
    if (m->kind == DIRAC_METRIC_FIELDS) {
        const double* planes[6] = {m->phi, m->psi, m->dphi_dx, m->dphi_dy, m->dpsi_dx, m->dpsi_dy};
        for (int k = 0; k < 6; ++k) {
            hipError_t e = hipMemcpyAsync(b + lay.fields + k * N * 8, planes[k], N * 8, hipMemcpyHostToDevice, s->stream);
            if (e != hipSuccess) return bail(hip_fail(e, "upload metric fields"));
        }
    }
    if (em) {
        // potential profiles staged as FP64 planes in the scratch area
        const double* planes[3] = {em->V, em->Ax, em->Ay};
        for (int k = 0; k < 3; ++k) {
            char* dst = b + lay.scratch + k * N * 8;
            hipError_t e = planes[k] ? hipMemcpyAsync(dst, planes[k], N * 8, hipMemcpyHostToDevice, s->stream)
                                     : hipMemsetAsync(dst, 0, N * 8, s->stream);
            if (e != hipSuccess) return bail(hip_fail(e, "upload potentials"));
        }
    }
    for (int ax = 0; ax < 2; ++ax) {
        SetupAxisParams ap{};
        ap.n = ax == 0 ? g->n1 : g->n2;
        ap.a = ax == 0 ? g->a1 : g->a2;
        ap.c = g->c;
        ap.dt = g->dt;
        ap.pml_width = pml->width_pts;
        ap.pml_type = pml->type;
        ap.sigma0 = pml->sigma0;
        ap.ctheta = std::cos(pml->theta);
        ap.fp32 = fp32;
        ap.k_printed = sc.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS_PRINTED;
        ap.inv_s = b + lay.inv_s[ax];
        ap.K = b + lay.K[ax];
        ap.D = b + lay.D[ax];
        ap.tw = b + lay.tw[ax];
        hipError_t e = launch_setup_axis(ap, s->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "setup axis tables"));
    }
    SetupPointParams pp{};
    pp.n1 = g->n1; pp.n2 = g->n2; pp.a1 = g->a1; pp.a2 = g->a2;
    pp.dt = g->dt; pp.c = g->c; pp.m = g->m;
    pp.kind = m->kind; pp.spin = m->spin; pp.bump_A = m->bump_A; pp.bump_s = m->bump_s;
    pp.fields = m->kind == DIRAC_METRIC_FIELDS ? reinterpret_cast<const double*>(b + lay.fields) : nullptr;
    pp.pml_width = pml->width_pts; pp.pml_type = pml->type; pp.sigma0 = pml->sigma0;
    pp.ctheta = std::cos(pml->theta);
    pp.fp32 = fp32;
    pp.a_out = s->curved ? b + lay.a : nullptr;
    pp.E_out = s->curved ? b + lay.E : nullptr;
    pp.da_out = lay.da != SIZE_MAX ? b + lay.da : nullptr;
    pp.em_planes = em ? reinterpret_cast<const double*>(b + lay.scratch) : nullptr;
    pp.charge = em ? em->charge : 0.0;
    pp.em_out = em ? b + lay.em : nullptr;
    pp.obs_em = em ? reinterpret_cast<double*>(b + lay.obs) + 5 * N : nullptr;
    pp.obs = reinterpret_cast<double*>(b + lay.obs);
    pp.partial = reinterpret_cast<double*>(b + lay.partials);
    double* fold = reinterpret_cast<double*>(b + lay.out);
    hipError_t e = launch_setup_points(pp, fold, s->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "setup point tables"));
    if (s->curved) {
        e = launch_transpose(b + lay.a, b + lay.aT, g->n1, g->n2, fp32 ? 4 : 8, s->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "transpose a"));
    }
    double host_fold[3];
    e = hipMemcpyAsync(host_fold, fold, sizeof host_fold, hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "read setup check"));
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "setup synchronise"));
    if (host_fold[2] != 0.0)
        return bail(fail(DIRAC_E_NONFINITE, "%.0f grid points have non-finite metric fields or tables", host_fold[2]));
    if (sc.scheme != DIRAC_SCHEME_CN_GMRES && (host_fold[0] < 0.0 || host_fold[1] > 1.0 + 1e-12))
        return bail(fail(DIRAC_E_UNSTABLE,
                         "blend coefficient b = a/S ranges over [%.17g, %.17g]; the directional step is "
                         "stable only for b in [0, 1]", host_fold[0], host_fold[1]));
    s->b_min = host_fold[0];
    s->b_max = host_fold[1];
    const int mode = tune_mode(s);
    s->sched[0] = pick_entry(prec, g->n1, 0, g->n2, mode);
    s->sched[1] = pick_entry(prec, g->n2, 1, g->n1, mode);
    s->store_wt[0] = store_wt_compiled(s, 0) && pick_store_mode(prec, g->n1, 0, g->n2, mode);
    s->store_wt[1] = store_wt_compiled(s, 1) && pick_store_mode(prec, g->n2, 1, g->n1, mode);
    *out = s;
    return DIRAC_OK;
}

dirac_status dirac_set_initial_spinor(dirac_solver* s, const double* psi_host) {
    if (!s || !psi_host) return fail(DIRAC_E_ARG, "null solver or spinor");
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    for (size_t i = 0; i < 4 * N; ++i)
        if (!std::isfinite(psi_host[i])) return fail(DIRAC_E_NONFINITE, "initial spinor has a non-finite value at real index %zu", i);
    char* b = s->base;
    if (s->prec == DIRAC_FP64) {
        HIP_TRY(hipMemcpyAsync(b + s->lay.psi, psi_host, N * 32, hipMemcpyHostToDevice, s->stream), "upload spinor");
    } else {
        HIP_TRY(hipMemcpyAsync(b + s->lay.scratch, psi_host, N * 32, hipMemcpyHostToDevice, s->stream), "upload spinor");
        HIP_TRY(launch_c128_to_f32(reinterpret_cast<const double*>(b + s->lay.scratch),
                                   reinterpret_cast<float*>(b + s->lay.psi), 4 * N, s->stream), "convert spinor");
    }
    HIP_TRY(hipStreamSynchronize(s->stream), "synchronise");
    s->step = 0;
    s->has_state = true;
    return DIRAC_OK;
}

dirac_status dirac_set_initial_spinor_device(dirac_solver* s, const void* psi_dev) {
    if (!s || !psi_dev) return fail(DIRAC_E_ARG, "null solver or spinor");
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    char* b = s->base;
    if (s->prec == DIRAC_FP64) {
        HIP_TRY(hipMemcpyAsync(b + s->lay.psi, psi_dev, N * 32, hipMemcpyDeviceToDevice, s->stream), "copy spinor");
    } else {
        HIP_TRY(launch_c128_to_f32(static_cast<const double*>(psi_dev), reinterpret_cast<float*>(b + s->lay.psi),
                                   4 * N, s->stream), "convert spinor");
    }
    s->step = 0;
    s->has_state = true;
    return DIRAC_OK;
}

dirac_status dirac_step_n(dirac_solver* s, int64_t nsteps) {
    if (!s) return fail(DIRAC_E_ARG, "null solver");
    if (nsteps < 0) return fail(DIRAC_E_ARG, "nsteps must be >= 0");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    if (s->scheme.scheme == DIRAC_SCHEME_CN_GMRES) return cn_step_n(s, nsteps);
    dirac_status r = enqueue_steps(s, nsteps, true);
    if (r != DIRAC_OK) return r;
    s->step += nsteps;
    return DIRAC_OK;
}

}  // extern "C"

namespace dirac {

// Observables with the reduction partials (8 doubles per workgroup of the two
// derivative passes) at `parts` and the 8 reduced sums at `dout`: the solver's
// own buffer, or the library's static scratch array.  max_parts bounds the
// workgroup count (DIRAC_E_SIZE beyond it, before anything is launched).
static dirac_status observables_into(dirac_solver* s, dirac_obs* out, double* parts, double* dout,
                                     size_t max_parts) {
    if (!s || !out) return fail(DIRAC_E_ARG, "null solver or output");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    char* b = s->base;
    ObsParams p{};
    p.psi = b + s->lay.psi;
    const double* obs = reinterpret_cast<const double*>(b + s->lay.obs);
    p.w = obs; p.ca = obs + N; p.gx = obs + 2 * N; p.gy = obs + 3 * N; p.V = obs + 4 * N;
    if (s->has_em) {
        const double t = s->step * s->g.dt;
        p.ax = obs + 5 * N; p.ay = obs + 6 * N; p.v0 = obs + 7 * N;
        p.fA = envelope_at(s->env_A, t);
        p.fV = envelope_at(s->env_V, t);
    }
    p.n1 = s->g.n1; p.n2 = s->g.n2;
    p.a1 = s->g.a1; p.a2 = s->g.a2;
    p.h1 = 2.0 * s->g.a1 / s->g.n1; p.h2 = 2.0 * s->g.a2 / s->g.n2;
    size_t need = 0;
    for (int dir = 0; dir < 2; ++dir) {
        const KernelEntry* e = obs_entry(s->prec, dir == 0 ? s->g.n1 : s->g.n2, dir);
        const int nl = dir == 0 ? s->g.n2 : s->g.n1;
        need += (size_t)((nl + e->lines - 1) / e->lines);
    }
    if (need > max_parts)
        return fail(DIRAC_E_SIZE, "observables need %zu reduction partials, more than the %zu available", need,
                    max_parts);
    int nparts = 0;
    for (int dir = 0; dir < 2; ++dir) {
        const KernelEntry* e = obs_entry(s->prec, dir == 0 ? s->g.n1 : s->g.n2, dir);
        p.nlines = dir == 0 ? s->g.n2 : s->g.n1;
        p.D = b + s->lay.D[dir];
        p.tw = b + s->lay.tw[dir];
        p.partials = parts + 8 * (size_t)nparts;
        const int nb = (p.nlines + e->lines - 1) / e->lines;
        void* args[] = {&p};
        HIP_TRY(hipLaunchKernel(e->obs_fn, dim3(nb), dim3(e->nthreads), args, 0, s->stream), "launch observables");
        nparts += nb;
    }
    HIP_TRY(launch_reduce_partials(parts, nparts, dout, s->stream), "reduce observables");
    double h[8];
    HIP_TRY(hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s->stream), "read observables");
    HIP_TRY(hipStreamSynchronize(s->stream), "synchronise");
    const double dA = (2.0 * s->g.a1 / s->g.n1) * (2.0 * s->g.a2 / s->g.n2);
    out->step = s->step;
    out->t = s->step * s->g.dt;
    out->norm_l2 = dA * h[0];
    out->norm_w = dA * h[1];
    out->x_mean = h[2] / h[0];
    out->y_mean = h[3] / h[0];
    out->energy_re = dA * h[4];
    out->energy_im = dA * h[5];
    out->finite = h[6] == 0.0 && std::isfinite(h[0]);
    out->reserved = 0;
    return DIRAC_OK;
}

// Static scratch of the allocation-free observables: the reduction partials of
// at most kObsStaticParts workgroups (one per line of each direction at the
// largest grid, 8192 x 8192) followed by the 8 reduced sums, 1 MiB in all.
// Every GPU the library runs on holds its own copy until the process ends.  In
// host code the array's name is not a device address: kernels and copies use
// the address hipGetSymbolAddress returns for the device, kept per device.
constexpr size_t kObsStaticParts = 2 * 8192;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[(kObsStaticParts + 1) * 8];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device with
// that device current.
static dirac_status static_scratch(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return fail(DIRAC_E_DEVICE, "device index %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
        if (cur != device) HIP_TRY(hipSetDevice(device), "hipSetDevice");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(DIRAC_E_DEVICE, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return DIRAC_OK;
}

}  // namespace dirac

extern "C" {

dirac_status dirac_observables(dirac_solver* s, dirac_obs* out) {
    if (!s) return fail(DIRAC_E_ARG, "null solver or output");
    char* b = s->base;
    return observables_into(s, out, reinterpret_cast<double*>(b + s->lay.partials),
                            reinterpret_cast<double*>(b + s->lay.out), SIZE_MAX);
}

dirac_status dirac_observables_static(dirac_solver* s, dirac_obs* out) {
    if (!s || !out) return fail(DIRAC_E_ARG, "null solver or output");
    double* sc = nullptr;
    dirac_status r = static_scratch(s->device, &sc);
    if (r != DIRAC_OK) return r;
    return observables_into(s, out, sc, sc + kObsStaticParts * 8, kObsStaticParts);
}

dirac_status dirac_get_spinor(dirac_solver* s, double* psi_host_out) {
    if (!s || !psi_host_out) return fail(DIRAC_E_ARG, "null solver or output");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    char* b = s->base;
    if (s->prec == DIRAC_FP64) {
        HIP_TRY(hipMemcpyAsync(psi_host_out, b + s->lay.psi, N * 32, hipMemcpyDeviceToHost, s->stream), "download spinor");
    } else {
        HIP_TRY(launch_f32_to_c128(reinterpret_cast<const float*>(b + s->lay.psi),
                                   reinterpret_cast<double*>(b + s->lay.scratch), 4 * N, s->stream), "convert spinor");
        HIP_TRY(hipMemcpyAsync(psi_host_out, b + s->lay.scratch, N * 32, hipMemcpyDeviceToHost, s->stream), "download spinor");
    }
    HIP_TRY(hipStreamSynchronize(s->stream), "synchronise");
    return DIRAC_OK;
}

dirac_status dirac_destroy(dirac_solver* s) {
    if (!s) return fail(DIRAC_E_ARG, "null solver");
    (void)hipStreamSynchronize(s->stream);      // nothing of this solve may be in flight
    drop_graph(s);
    for (auto& ev : s->events) (void)hipEventDestroy(ev);
    for (auto& ev : s->cn_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (s->cn_head) (void)hipHostFree(s->cn_head);
    delete s;
    return DIRAC_OK;
}

// ------------------------------------------------------------- schedules

int32_t dirac_schedule_count(int32_t n, int32_t prec, int32_t dir) {
    int c = 0;
    for (const auto& e : kernel_registry()) c += (e.prec == prec && e.n == n && e.dir == dir);
    return c;
}

dirac_status dirac_schedule_get(int32_t n, int32_t prec, int32_t dir, int32_t i, dirac_schedule* out) {
    if (!out) return fail(DIRAC_E_ARG, "null output");
    int c = 0;
    for (const auto& e : kernel_registry()) {
        if (e.prec == prec && e.n == n && e.dir == dir) {
            if (c == i) {
                out->radix = e.radix;
                out->lines_per_wg = e.lines;
                out->components_per_thread = e.cpt;
                return DIRAC_OK;
            }
            ++c;
        }
    }
    return fail(DIRAC_E_ARG, "no schedule %d for n = %d", i, n);
}

dirac_status dirac_get_schedule(const dirac_solver* s, int32_t dir, dirac_schedule* out) {
    if (!s || !out || dir < 0 || dir > 1) return fail(DIRAC_E_ARG, "bad arguments");
    out->radix = s->sched[dir]->radix;
    out->lines_per_wg = s->sched[dir]->lines;
    out->components_per_thread = s->sched[dir]->cpt;
    return DIRAC_OK;
}

dirac_status dirac_set_schedule(dirac_solver* s, int32_t dir, const dirac_schedule* sch) {
    if (!s || !sch || dir < 0 || dir > 1) return fail(DIRAC_E_ARG, "bad arguments");
    const KernelEntry* e = find_entry(s->prec, dir == 0 ? s->g.n1 : s->g.n2, dir, *sch);
    if (!e)
        return fail(DIRAC_E_ARG, "schedule radix %d lines %d components %d not compiled", sch->radix,
                    sch->lines_per_wg, sch->components_per_thread);
    s->sched[dir] = e;
    drop_graph(s);
    return DIRAC_OK;
}

dirac_status dirac_set_store_mode(dirac_solver* s, int32_t write_through) {
    if (!s || write_through < 0 || write_through > 3) return fail(DIRAC_E_ARG, "bad arguments");
    if (s->scheme.scheme == DIRAC_SCHEME_CN_GMRES)
        return fail(DIRAC_E_ARG, "the store mode applies to Scheme II's directional steps");
    if ((write_through & 2) && !store_wt_compiled(s, 1))
        return fail(DIRAC_E_ARG, "write-through stores of the y kernel are compiled for n2 <= %d only",
                    kStoreWtMaxColN);
    s->store_wt[0] = (write_through & 1) != 0;
    s->store_wt[1] = (write_through & 2) != 0;
    drop_graph(s);
    return DIRAC_OK;
}

dirac_status dirac_get_store_mode(const dirac_solver* s, int32_t* write_through) {
    if (!s || !write_through) return fail(DIRAC_E_ARG, "bad arguments");
    *write_through = (s->store_wt[0] ? 1 : 0) | (s->store_wt[1] ? 2 : 0);
    return DIRAC_OK;
}

dirac_status dirac_set_potential_form(dirac_solver* s, int32_t form) {
    if (!s) return fail(DIRAC_E_ARG, "null solver");
    if (!s->has_em) return fail(DIRAC_E_ARG, "the solver has no potentials");
    if (form < 0 || form > 2) return fail(DIRAC_E_ARG, "form must be 0, 1 or 2");
    (void)hipStreamSynchronize(s->stream);
    s->em_form = form;
    // the kernels of the new form with the schedules and store modes tuned for it
    const int mode = tune_mode(s);
    s->sched[0] = pick_entry(s->prec, s->g.n1, 0, s->g.n2, mode);
    s->sched[1] = pick_entry(s->prec, s->g.n2, 1, s->g.n1, mode);
    s->store_wt[0] = store_wt_compiled(s, 0) && pick_store_mode(s->prec, s->g.n1, 0, s->g.n2, mode);
    s->store_wt[1] = store_wt_compiled(s, 1) && pick_store_mode(s->prec, s->g.n2, 1, s->g.n1, mode);
    return DIRAC_OK;
}

dirac_status dirac_get_potential_form(const dirac_solver* s, int32_t* pass) {
    if (!s || !pass) return fail(DIRAC_E_ARG, "null argument");
    *pass = em_pass(s) ? 1 : 0;
    return DIRAC_OK;
}

dirac_status dirac_set_launch_mode(dirac_solver* s, int32_t use_graph, int32_t chunk) {
    if (!s || chunk < 1 || chunk > 4096) return fail(DIRAC_E_ARG, "bad arguments");
    s->use_graph = use_graph != 0;
    s->graph_chunk = chunk;
    drop_graph(s);
    return DIRAC_OK;
}

dirac_status dirac_step_n_timed(dirac_solver* s, int64_t nsteps, double* ms_out, int64_t* counts_out) {
    if (!s || !ms_out || !counts_out) return fail(DIRAC_E_ARG, "null argument");
    if (nsteps < 0) return fail(DIRAC_E_ARG, "nsteps must be >= 0");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    if (s->scheme.scheme == DIRAC_SCHEME_CN_GMRES) return fail(DIRAC_E_ARG, "per-direction timing is for Scheme II");
    ms_out[0] = ms_out[1] = 0.0;
    counts_out[0] = counts_out[1] = 0;
    if (nsteps == 0) return DIRAC_OK;
    // every launch carries its own start/stop events (hipExtLaunchKernel): the
    // timestamps are those of the kernel dispatch itself, so the durations are
    // kernel execution times in the real x, y, x, y ... order, with no extra
    // packets between the launches
    // with a separate potentials pass, the pass before a step's x kernel counts
    // toward the x class (Steps 5 and 1 belong to it) and the closing pass
    // toward the last y
    const bool pass = em_pass(s);
    const size_t nl = (size_t)nsteps * (pass ? 3 : 2) + (pass ? 1 : 0);
    while (s->events.size() < 2 * nl) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev), "hipEventCreate");
        s->events.push_back(ev);
    }
    hipStream_t st = s->stream;
    std::vector<int> cls;                   // per launch: class, +2 when it is the step's kernel (counted)
    cls.reserve(nl);
    size_t k = 0;
    auto timed = [&](Launch& L, int c) -> dirac_status {
        void* args[] = {L.params};
        HIP_TRY(hipExtLaunchKernel(L.fn, L.grid, L.block, args, 0, st, s->events[2 * k], s->events[2 * k + 1], 0),
                "launch stage");
        cls.push_back(c);
        ++k;
        return DIRAC_OK;
    };
    for (int64_t n = 0; n < nsteps; ++n) {
        dirac_status r;
        if (pass) {
            Launch le = make_exp_launch(s, n == 0 ? 1 : 2, s->step + n);
            if ((r = timed(le, 0)) != DIRAC_OK) return r;
        }
        Launch lx = make_launch(s, 0, n == 0 ? 1 : 2, 0, s->step + n);
        Launch ly = make_launch(s, 1, 0, n == nsteps - 1 ? 1 : 0, s->step + n);
        if ((r = timed(lx, 2)) != DIRAC_OK || (r = timed(ly, 3)) != DIRAC_OK) return r;
    }
    if (pass) {
        Launch lc = make_exp_launch(s, 1, s->step + nsteps - 1);
        dirac_status r = timed(lc, 1);
        if (r != DIRAC_OK) return r;
    }
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    for (size_t i = 0; i < k; ++i) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, s->events[2 * i], s->events[2 * i + 1]), "hipEventElapsedTime");
        ms_out[cls[i] & 1] += ms;
        if (cls[i] & 2) counts_out[cls[i] & 1] += 1;
    }
    s->step += nsteps;
    return DIRAC_OK;
}

dirac_status dirac_time_directions(dirac_solver* s, int32_t reps, double* us_out) {
    if (!s || !us_out || reps < 1 || reps > 100000) return fail(DIRAC_E_ARG, "bad arguments");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    if (s->scheme.scheme == DIRAC_SCHEME_CN_GMRES) return fail(DIRAC_E_ARG, "per-direction timing is for Scheme II");
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    const size_t bytes = N * 4 * (s->prec == DIRAC_FP32 ? 4 : 8);
    char* b = s->base;
    hipStream_t st = s->stream;
    HIP_TRY(hipMemcpyAsync(b + s->lay.scratch, b + s->lay.psi, bytes, hipMemcpyDeviceToDevice, st), "save state");
    hipEvent_t ev[2];
    HIP_TRY(hipEventCreate(&ev[0]), "hipEventCreate");
    if (hipEventCreate(&ev[1]) != hipSuccess) { (void)hipEventDestroy(ev[0]); return fail(DIRAC_E_DEVICE, "hipEventCreate"); }
    dirac_status result = DIRAC_OK;
    for (int dir = 0; dir < 2 && result == DIRAC_OK; ++dir) {
        // the x class includes the potentials pass (Steps 5 and 1) when it is separate
        std::vector<Launch> Ls;
        if (dir == 0 && em_pass(s)) Ls.push_back(make_exp_launch(s, 2, s->step));
        Ls.push_back(make_launch(s, dir, dir == 0 ? 2 : 0, 0, s->step));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        auto step = [&]() -> dirac_status {
            HIP_TRY(hipGraphCreate(&graph, 0), "hipGraphCreate");
            hipGraphNode_t prev = nullptr;
            for (int k = 0; k < reps; ++k) {
                for (Launch& L : Ls) {
                    void* args[] = {L.params};
                    hipKernelNodeParams kp{};
                    kp.func = const_cast<void*>(L.fn);
                    kp.gridDim = L.grid;
                    kp.blockDim = L.block;
                    kp.kernelParams = args;
                    hipGraphNode_t node;
                    HIP_TRY(hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp),
                            "hipGraphAddKernelNode");
                    prev = node;
                }
            }
            HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            HIP_TRY(hipGraphLaunch(exec, st), "hipGraphLaunch");          // warm
            HIP_TRY(hipEventRecord(ev[0], st), "hipEventRecord");
            HIP_TRY(hipGraphLaunch(exec, st), "hipGraphLaunch");
            HIP_TRY(hipEventRecord(ev[1], st), "hipEventRecord");
            HIP_TRY(hipEventSynchronize(ev[1]), "hipEventSynchronize");
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
            us_out[dir] = 1e3 * (double)ms / reps;
            return DIRAC_OK;
        };
        result = step();
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    HIP_TRY(hipMemcpyAsync(b + s->lay.psi, b + s->lay.scratch, bytes, hipMemcpyDeviceToDevice, st), "restore state");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return result;
}

dirac_status dirac_autotune(dirac_solver* s, int32_t reps) {
    if (!s || reps < 1 || reps > 4096) return fail(DIRAC_E_ARG, "bad arguments");
    if (s->scheme.scheme == DIRAC_SCHEME_CN_GMRES)
        return fail(DIRAC_E_ARG, "the autotuner applies to Scheme II's directional steps");
    // the corrected second-order step and the potential kernels have one
    // schedule each: only their store modes are searched
    const bool one_schedule = s->scheme.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS || (s->has_em && !em_pass(s));
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    const size_t N = (size_t)s->g.n1 * s->g.n2;
    const size_t bytes = N * 4 * (s->prec == DIRAC_FP32 ? 4 : 8);
    char* b = s->base;
    HIP_TRY(hipMemcpyAsync(b + s->lay.scratch, b + s->lay.psi, bytes, hipMemcpyDeviceToDevice, s->stream), "save state");
    const int64_t step0 = s->step;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    const int mode = tune_mode(s);
    dirac_status result = DIRAC_OK;
    // Candidates are timed as they run: reps + 1 steps whose middle reps (y, x)
    // pairs replay one HIP graph (direct launches of small grids would time
    // the host's launch rate, not the kernels; solves with potentials launch
    // directly anyway).  The first pass builds the graph and warms up; the
    // second is timed.
    const bool use_graph0 = s->use_graph;
    const int chunk0 = s->graph_chunk;
    s->use_graph = true;
    s->graph_chunk = std::max(1, reps);
    auto time_steps = [&](float& ms) -> dirac_status {
        drop_graph(s);
        dirac_status r = enqueue_steps(s, reps + 1, true);
        if (r != DIRAC_OK) return r;
        hipEventRecord(e0, s->stream);
        if ((r = enqueue_steps(s, reps + 1, true)) != DIRAC_OK) return r;
        hipEventRecord(e1, s->stream);
        if (hipEventSynchronize(e1) != hipSuccess) return fail(DIRAC_E_DEVICE, "autotune sync");
        ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        return DIRAC_OK;
    };
    // Coordinate search over (schedule, store mode) per direction, two sweeps
    // x, y, x, y: the choices interact (the y kernel reads what the x kernel
    // wrote, and how it was written), so each direction is re-tuned once with
    // the other's choice in place.
    s->store_wt[0] = s->store_wt[1] = false;
    double dir_ms[2] = {0, 0};
    for (int sweep = 0; sweep < 2 && result == DIRAC_OK; ++sweep) {
        for (int dir = 0; dir < 2 && result == DIRAC_OK; ++dir) {
            const int n = dir == 0 ? s->g.n1 : s->g.n2;
            const KernelEntry* best = s->sched[dir];
            bool best_wt = s->store_wt[dir];
            double best_ms = 1e300;
            for (const auto& e : kernel_registry()) {
                if (e.prec != s->prec || e.n != n || e.dir != dir) continue;
                if (one_schedule && &e != best) continue;
                for (int wt = 0; wt <= (store_wt_compiled(s, dir) ? 1 : 0) && result == DIRAC_OK; ++wt) {
                    s->sched[dir] = &e;
                    s->store_wt[dir] = wt != 0;
                    float ms = 0;
                    if ((result = time_steps(ms)) != DIRAC_OK) break;
                    if (ms < best_ms) { best_ms = ms; best = &e; best_wt = wt != 0; }
                }
                if (result != DIRAC_OK) break;
            }
            s->sched[dir] = best;
            s->store_wt[dir] = best_wt;
            dir_ms[dir] = best_ms;
        }
    }
    if (result != DIRAC_OK) s->store_wt[0] = s->store_wt[1] = false;
    if (result == DIRAC_OK) {
        std::lock_guard<std::mutex> lk(tune_mutex());
        for (int dir = 0; dir < 2; ++dir) {
            const int n = dir == 0 ? s->g.n1 : s->g.n2;
            const int other = dir == 0 ? s->g.n2 : s->g.n1;
            const KernelEntry* best = s->sched[dir];
            tune_cache()[TuneKey{s->prec, n, dir, other, mode}] =
                TuneVal{best->radix, best->lines, best->cpt, dir_ms[dir] / reps, s->store_wt[dir] ? 1 : 0};
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph(s);
    s->use_graph = use_graph0;
    s->graph_chunk = chunk0;
    HIP_TRY(hipMemcpyAsync(b + s->lay.psi, b + s->lay.scratch, bytes, hipMemcpyDeviceToDevice, s->stream), "restore state");
    HIP_TRY(hipStreamSynchronize(s->stream), "synchronise");
    s->step = step0;
    return result;
}

dirac_status dirac_tune_cache_save(const char* path) {
    if (!path) return fail(DIRAC_E_ARG, "null path");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(DIRAC_E_ARG, "cannot open %s", path);
    std::lock_guard<std::mutex> lk(tune_mutex());
    std::fprintf(f, "# prec n dir other mode radix lines components ms_per_step write_through\n");
    for (const auto& kv : tune_cache())
        std::fprintf(f, "%d %d %d %d %d %d %d %d %.6g %d\n", kv.first.prec, kv.first.n, kv.first.dir, kv.first.other,
                     kv.first.mode, kv.second.radix, kv.second.lines, kv.second.cpt, kv.second.ms, kv.second.wt);
    std::fclose(f);
    return DIRAC_OK;
}

dirac_status dirac_tune_cache_load(const char* path) {
    if (!path) return fail(DIRAC_E_ARG, "null path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(DIRAC_E_ARG, "cannot open %s", path);
    char line[256];
    std::lock_guard<std::mutex> lk(tune_mutex());
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        TuneKey k{};
        TuneVal v{};
        const int got = std::sscanf(line, "%d %d %d %d %d %d %d %d %lf %d", &k.prec, &k.n, &k.dir, &k.other,
                                    &k.mode, &v.radix, &v.lines, &v.cpt, &v.ms, &v.wt);
        if (got == 9) v.wt = 0;      // files written before the store-mode column
        if (got >= 9) tune_cache()[k] = v;
    }
    std::fclose(f);
    return DIRAC_OK;
}

}  // extern "C"
