// batch_runtime.hip -- host side of the batched multi-solve engine: slot table,
// descriptor upload (pinned, double buffered), per-run phase schedule and its
// HIP graph.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/dirac.h"
#include "batch_kernels.hpp"
#include "batch_registry.hpp"
#include "solver.hpp"

namespace dirac {

BatchKernel& batch_kernel(int prec, int dir, int logn, int sched) {
    static BatchKernel k[2][2][8][kBatchSchedules];
    return k[prec][dir][logn - 4][sched];
}

const void*& batch_multi_kernel_fn(int prec, int dir) {
    static const void* f[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    return f[prec][dir];
}

// A size group launched on its own should fill the GPU: at least this many
// 256-thread tiles (four per compute unit); the smaller groups of a phase
// share one launch of the multi-group kernel.
constexpr int kMinGroupTiles = 1024;
// timed runs per candidate schedule in dirac_batch_autotune (the fastest counts),
// and the relative margin within which the lower-numbered schedule is kept
constexpr int kBatchTuneTrials = 3;
constexpr double kBatchTuneTie = 0.01;

static size_t align256b(size_t x) { return (x + 255) & ~size_t(255); }

// Per direction: the solves' desc indices grouped by size (capacity ints) and
// the groups' tile prefixes (capacity + 8 ints: one extra entry per group).
static size_t batch_dir_ints(int capacity) { return 2 * (size_t)capacity + 8; }

static size_t batch_half_bytes(int capacity) {
    return align256b((size_t)capacity * sizeof(BatchDesc<double>)) +
           align256b(2 * batch_dir_ints(capacity) * sizeof(int));
}

}  // namespace dirac

using namespace dirac;

struct dirac_batch {
    int prec = 0;
    int capacity = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    size_t half = 0;
    int which = 0;
    std::vector<dirac_solver*> slots;
    char* host_stage[2] = {nullptr, nullptr};
    hipEvent_t stage_done[2] = {nullptr, nullptr};
    bool use_graph = true;
    // cached graph of the last run signature
    std::vector<int64_t> sig;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t graph_done = nullptr;
    int graph_half = -1;
    uint64_t version = 0;
    uint64_t graph_version = ~0ull;
    int sched[2][12] = {};          // batch schedule per (direction, log2 n)
    std::vector<hipEvent_t> events; // start/stop pairs of the timed runs
};

static dirac_status bhip(hipError_t e, const char* what) {
    return e == hipSuccess ? DIRAC_OK : fail(DIRAC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}
#define BTRY(expr, what)                              \
    do {                                              \
        dirac_status st_ = bhip((expr), (what));      \
        if (st_ != DIRAC_OK) return st_;              \
    } while (0)

static void batch_drop_graph(dirac_batch* b) {
    if (b->gexec) {
        if (b->graph_done) (void)hipEventSynchronize(b->graph_done);
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->sig.clear();
}

template <typename T>
static void fill_desc(BatchDesc<T>& d, const dirac_solver* s, int steps, const int (&sched)[2][12]) {
    char* base = s->base;
    d.psi = reinterpret_cast<T*>(base + s->lay.psi);
    d.a[0] = s->curved ? reinterpret_cast<const T*>(base + s->lay.a) : nullptr;
    d.a[1] = s->curved ? reinterpret_cast<const T*>(base + s->lay.aT) : nullptr;
    d.E = s->curved ? reinterpret_cast<const T*>(base + s->lay.E) : nullptr;
    for (int ax = 0; ax < 2; ++ax) {
        d.inv_s[ax] = reinterpret_cast<const T*>(base + s->lay.inv_s[ax]);   // ones without a layer
        d.K[ax] = reinterpret_cast<const cpx<T>*>(base + s->lay.K[ax]);
        d.tw[ax] = reinterpret_cast<const cpx<T>*>(base + s->lay.tw[ax]);
    }
    d.n1 = s->g.n1;
    d.n2 = s->g.n2;
    d.logn[0] = __builtin_ctz((unsigned)s->g.n1);
    d.logn[1] = __builtin_ctz((unsigned)s->g.n2);
    d.mode = s->curved ? 2 : (s->pml ? 1 : 0);
    d.sched[0] = sched[0][d.logn[0]];
    d.sched[1] = sched[1][d.logn[1]];
    d.steps = steps;
    d.e0u = cpx<T>{(T)s->e0u_re, (T)s->e0u_im};
}

static int tiles_of(int n_line, int n_lines, int sched) {
    const int L = bsched_lines(n_line, sched);
    return (n_lines + L - 1) / L;
}

// The solves of one direction that share a transform length, longest run first.
struct BatchGroup {
    int logn;
    std::vector<int> members;      // positions in the run's desc array
    std::vector<int> prefix;       // tile prefix, members.size() + 1 entries
    int index_off, prefix_off;     // offsets (ints) in the direction's device arrays
};

extern "C" {

size_t dirac_batch_footprint_bytes(int32_t capacity) {
    if (capacity < 1 || capacity > (1 << 20)) return 0;
    return 2 * batch_half_bytes(capacity) + 256;
}

dirac_status dirac_batch_create(int32_t prec, int32_t capacity, void* device_buffer, size_t bytes, void* hip_stream,
                                dirac_batch** out) {
    if (!out) return fail(DIRAC_E_ARG, "null output handle");
    *out = nullptr;
    if (prec != DIRAC_FP64 && prec != DIRAC_FP32) return fail(DIRAC_E_ARG, "precision must be 0 or 1");
    if (capacity < 1 || capacity > (1 << 20)) return fail(DIRAC_E_ARG, "capacity must be in [1, 2^20]");
    if (!device_buffer) return fail(DIRAC_E_ARG, "null device buffer");
    if (bytes < dirac_batch_footprint_bytes(capacity))
        return fail(DIRAC_E_SIZE, "batch buffer of %zu bytes < footprint %zu", bytes, dirac_batch_footprint_bytes(capacity));
    for (int d = 0; d < 2; ++d) {
        for (int lg = 4; lg <= 11; ++lg)
            if (!batch_kernel(prec, d, lg, 0).fn) return fail(DIRAC_E_DEVICE, "batch kernels not compiled");
        if (!batch_multi_kernel_fn(prec, d)) return fail(DIRAC_E_DEVICE, "batch kernels not compiled");
    }
    dirac_batch* b = new (std::nothrow) dirac_batch();
    if (!b) return fail(DIRAC_E_NOMEM, "host allocation failed");
    b->prec = prec;
    b->capacity = capacity;
    b->stream = static_cast<hipStream_t>(hip_stream);
    const uintptr_t raw = reinterpret_cast<uintptr_t>(device_buffer);
    b->base = reinterpret_cast<char*>((raw + 255) & ~uintptr_t(255));
    b->half = batch_half_bytes(capacity);
    b->slots.assign(capacity, nullptr);
    for (int h = 0; h < 2; ++h) {
        if (hipHostMalloc(reinterpret_cast<void**>(&b->host_stage[h]), b->half, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&b->stage_done[h], hipEventDisableTiming) != hipSuccess) {
            dirac_batch_destroy(b);
            return fail(DIRAC_E_DEVICE, "pinned staging allocation failed");
        }
    }
    if (hipEventCreateWithFlags(&b->graph_done, hipEventDisableTiming) != hipSuccess) {
        dirac_batch_destroy(b);
        return fail(DIRAC_E_DEVICE, "event creation failed");
    }
    for (int d = 0; d < 2; ++d)
        for (int lg = 4; lg <= 11; ++lg)
            for (int sc = 0; sc < kBatchSchedules; ++sc)
                if (batch_kernel(prec, d, lg, sc).fn)
                    (void)hipFuncSetAttribute(batch_kernel(prec, d, lg, sc).fn,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    for (int d = 0; d < 2; ++d)
        (void)hipFuncSetAttribute(batch_multi_kernel_fn(prec, d), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
    *out = b;
    return DIRAC_OK;
}

dirac_status dirac_batch_add(dirac_batch* b, dirac_solver* s, int32_t* slot_out) {
    if (!b || !s || !slot_out) return fail(DIRAC_E_ARG, "null argument");
    if (s->prec != b->prec) return fail(DIRAC_E_ARG, "solver precision differs from the batch");
    if (s->has_em) return fail(DIRAC_E_ARG, "batches run solves without time-dependent potentials only");
    if (s->scheme.scheme == DIRAC_SCHEME_CN_GMRES || s->scheme.scheme == DIRAC_SCHEME_EXP_SPLIT_2BIS)
        return fail(DIRAC_E_ARG, "batches run Scheme II solves with the plain or printed directional step only");
    if (s->g.n1 > 2048 || s->g.n2 > 2048) return fail(DIRAC_E_SIZE, "batched solves need n1, n2 <= 2048");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the solver's initial spinor first");
    for (auto* t : b->slots)
        if (t == s) return fail(DIRAC_E_ARG, "solver already in the batch");
    for (int i = 0; i < b->capacity; ++i) {
        if (!b->slots[i]) {
            b->slots[i] = s;
            *slot_out = i;
            ++b->version;
            return DIRAC_OK;
        }
    }
    return fail(DIRAC_E_SIZE, "batch is full (capacity %d)", b->capacity);
}

dirac_status dirac_batch_remove(dirac_batch* b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot]) return fail(DIRAC_E_ARG, "bad slot");
    b->slots[slot] = nullptr;
    ++b->version;
    return DIRAC_OK;
}

dirac_status dirac_batch_set_graph(dirac_batch* b, int32_t use_graph) {
    if (!b) return fail(DIRAC_E_ARG, "null batch");
    b->use_graph = use_graph != 0;
    batch_drop_graph(b);
    return DIRAC_OK;
}

}  // extern "C"

// Per-launch timing of a run: durations and launch counts per kernel class,
// class = direction * 9 + (log2 n - 4) for a size group's own kernel, or
// direction * 9 + 8 for the multi-group kernel.
struct BatchTiming {
    double ms[kBatchTimingClasses];
    int64_t count[kBatchTimingClasses];
    double bytes[kBatchTimingClasses];     // algorithmic bytes of the launches (whole run)
};

// Algorithmic bytes per grid point of one phase launch: state read and written
// once, plus the per-point tables read (x: E and a, y: a; curved solves only).
static double phase_bytes_per_point(const dirac_solver* s, int dir) {
    const double sz = s->prec == DIRAC_FP32 ? 4.0 : 8.0;
    return 8.0 * sz + (s->curved ? (dir == 0 ? 5.0 * sz : sz) : 0.0);
}

// launch = false (graph mode only): record and instantiate the run's graph
// without launching it, so that a later dirac_batch_run with the same step
// counts only replays it.
static dirac_status batch_run_impl(dirac_batch* b, const int64_t* steps, BatchTiming* tm, bool launch = true) {
    if (!b || !steps) return fail(DIRAC_E_ARG, "null argument");
    std::vector<int> act;
    for (int i = 0; i < b->capacity; ++i) {
        if (steps[i] < 0) return fail(DIRAC_E_ARG, "negative step count for slot %d", i);
        if (steps[i] > 0) {
            if (!b->slots[i]) return fail(DIRAC_E_ARG, "steps for free slot %d", i);
            if (steps[i] > (1ll << 30)) return fail(DIRAC_E_ARG, "step count too large for slot %d", i);
            act.push_back(i);
        }
    }
    if (act.empty()) return DIRAC_OK;
    std::stable_sort(act.begin(), act.end(), [&](int x, int y) { return steps[x] > steps[y]; });
    const int na = (int)act.size();
    std::vector<int64_t> sig;
    sig.reserve(2 * na + 1);
    sig.push_back((int64_t)b->version);
    for (int i : act) { sig.push_back(i); sig.push_back(steps[i]); }

    const bool reuse = !tm && b->use_graph && b->gexec && sig == b->sig;
    int h = reuse ? b->graph_half : b->which;
    char* dev = b->base + (size_t)h * b->half;
    const size_t desc_bytes = align256b((size_t)b->capacity * sizeof(BatchDesc<double>));
    int* dints = reinterpret_cast<int*>(dev + desc_bytes);
    const size_t dir_ints = batch_dir_ints(b->capacity);
    // size groups per direction; act is ordered longest run first, and a stable
    // grouping keeps that order inside each group
    std::vector<BatchGroup> groups[2];
    for (int d = 0; d < 2; ++d) {
        for (int lg = 4; lg <= 11; ++lg) {
            BatchGroup g{};
            g.logn = lg;
            for (int q = 0; q < na; ++q) {
                const dirac_solver* s = b->slots[act[q]];
                if (__builtin_ctz((unsigned)(d == 0 ? s->g.n1 : s->g.n2)) == lg) g.members.push_back(q);
            }
            if (g.members.empty()) continue;
            g.prefix.assign(g.members.size() + 1, 0);
            for (size_t m = 0; m < g.members.size(); ++m) {
                const dirac_solver* s = b->slots[act[g.members[m]]];
                const int nl = d == 0 ? s->g.n1 : s->g.n2;
                const int lines = d == 0 ? s->g.n2 : s->g.n1;
                g.prefix[m + 1] = g.prefix[m] + tiles_of(nl, lines, b->sched[d][lg]);
            }
            groups[d].push_back(std::move(g));
        }
        int io = 0, po = (int)b->capacity;
        for (auto& g : groups[d]) {
            g.index_off = io;
            g.prefix_off = po;
            io += (int)g.members.size();
            po += (int)g.members.size() + 1;
        }
    }
    if (!reuse) {
        batch_drop_graph(b);
        // refill the staging half (wait until its previous upload has left the host buffer)
        BTRY(hipEventSynchronize(b->stage_done[h]), "wait for staging buffer");
        char* hs = b->host_stage[h];
        for (int q = 0; q < na; ++q) {
            const dirac_solver* s = b->slots[act[q]];
            if (b->prec == DIRAC_FP64)
                fill_desc(reinterpret_cast<BatchDesc<double>*>(hs)[q], s, (int)steps[act[q]], b->sched);
            else
                fill_desc(reinterpret_cast<BatchDesc<float>*>(hs)[q], s, (int)steps[act[q]], b->sched);
        }
        int* hints = reinterpret_cast<int*>(hs + desc_bytes);
        for (int d = 0; d < 2; ++d) {
            int* di = hints + d * dir_ints;
            for (const auto& g : groups[d]) {
                std::memcpy(di + g.index_off, g.members.data(), g.members.size() * sizeof(int));
                std::memcpy(di + g.prefix_off, g.prefix.data(), g.prefix.size() * sizeof(int));
            }
        }
        BTRY(hipMemcpyAsync(dev, hs, b->half, hipMemcpyHostToDevice, b->stream), "upload batch descriptors");
        BTRY(hipEventRecord(b->stage_done[h], b->stream), "record staging event");
        b->which ^= 1;
    }

    const int64_t qmax = steps[act[0]];
    // the launches of phase (step k, direction d): one per size group with
    // work, except that the groups too small to fill the GPU alone share one
    // launch of the multi-group kernel (at most 8 sizes: n = 16 .. 2048)
    struct GroupLaunch {
        const void* fn;
        size_t smem;
        int tiles;
        bool multi;
        BatchPhase<double> ph;
        BatchMultiPhase<double> mph;
    };
    auto phase_launches = [&](int d, int64_t k, std::vector<GroupLaunch>& out) {
        out.clear();
        for (const auto& g : groups[d]) {
            int nactive = (int)g.members.size();
            while (nactive > 0 && steps[act[g.members[nactive - 1]]] <= k) --nactive;
            if (nactive == 0) continue;
            const int sc = b->sched[d][g.logn];
            GroupLaunch L{};
            L.fn = batch_kernel(b->prec, d, g.logn, sc).fn;
            L.smem = batch_kernel(b->prec, d, g.logn, sc).smem;
            L.multi = false;
            L.ph.desc = reinterpret_cast<const BatchDesc<double>*>(dev);
            L.ph.index = dints + d * dir_ints + g.index_off;
            L.ph.prefix = dints + d * dir_ints + g.prefix_off;
            L.ph.nactive = nactive;
            L.ph.total_tiles = g.prefix[nactive];
            L.ph.k = (int)k;
            L.tiles = L.ph.total_tiles;
            L.mph.logn[0] = g.logn;       // kept for the merge below
            L.mph.sched[0] = sc;
            out.push_back(L);
        }
        // groups too small to fill the GPU alone share one multi-group launch;
        // the others keep their own kernels (lower register counts)
        std::vector<GroupLaunch> small, keep;
        for (auto& L : out) (L.tiles < kMinGroupTiles ? small : keep).push_back(L);
        if (small.size() > 1) {
            GroupLaunch M{};
            M.fn = batch_multi_kernel_fn(b->prec, d);
            M.multi = true;
            M.mph.desc = reinterpret_cast<const BatchDesc<double>*>(dev);
            M.mph.ngroups = (int)small.size();
            M.mph.k = (int)k;
            M.mph.start[0] = 0;
            for (size_t g = 0; g < small.size(); ++g) {
                M.mph.index[g] = small[g].ph.index;
                M.mph.prefix[g] = small[g].ph.prefix;
                M.mph.nactive[g] = small[g].ph.nactive;
                M.mph.logn[g] = small[g].mph.logn[0];
                M.mph.sched[g] = small[g].mph.sched[0];
                M.mph.start[g + 1] = M.mph.start[g] + small[g].tiles;
                M.smem = std::max(M.smem, small[g].smem);
            }
            M.tiles = M.mph.start[small.size()];
            keep.push_back(M);
            out.swap(keep);
        }
    };
    // BatchPhase<T> / BatchMultiPhase<T> have the same layout for both T.
    static_assert(sizeof(BatchPhase<double>) == sizeof(BatchPhase<float>), "phase layout");
    static_assert(sizeof(BatchMultiPhase<double>) == sizeof(BatchMultiPhase<float>), "phase layout");

    std::vector<GroupLaunch> gl;
    // algorithmic bytes of one launch: its solves' points times the bytes per point
    auto launch_bytes = [&](int d, const GroupLaunch& L) -> double {
        double by = 0;
        auto add_group = [&](const int* idx_dev, int nactive) {
            const int* idx = reinterpret_cast<const int*>(b->host_stage[h] + desc_bytes) +
                             (idx_dev - dints);
            for (int q = 0; q < nactive; ++q) {
                const dirac_solver* s = b->slots[act[idx[q]]];
                by += (double)s->g.n1 * s->g.n2 * phase_bytes_per_point(s, d);
            }
        };
        if (L.multi)
            for (int g = 0; g < L.mph.ngroups; ++g) add_group(L.mph.index[g], L.mph.nactive[g]);
        else
            add_group(L.ph.index, L.ph.nactive);
        return by;
    };
    if (tm) {
        // one launch per group with its own start/stop events (hipExtLaunchKernel):
        // kernel execution times in the order of a real run
        std::vector<std::pair<int, double>> cls;     // class and bytes of launch i
        for (int64_t k = 0; k < qmax; ++k)
            for (int d = 0; d < 2; ++d) {
                phase_launches(d, k, gl);
                for (auto& L : gl) {
                    const size_t i = cls.size();
                    while (b->events.size() < 2 * (i + 1)) {
                        hipEvent_t ev;
                        BTRY(hipEventCreate(&ev), "hipEventCreate");
                        b->events.push_back(ev);
                    }
                    void* args[] = {L.multi ? static_cast<void*>(&L.mph) : static_cast<void*>(&L.ph)};
                    BTRY(hipExtLaunchKernel(L.fn, dim3(L.tiles), dim3(kBatchThreads), args, L.smem, b->stream,
                                            b->events[2 * i], b->events[2 * i + 1], 0), "launch batch phase");
                    cls.push_back({d * 9 + (L.multi ? 8 : L.mph.logn[0] - 4), launch_bytes(d, L)});
                }
            }
        BTRY(hipStreamSynchronize(b->stream), "synchronise batch stream");
        for (size_t i = 0; i < cls.size(); ++i) {
            float ms = 0;
            BTRY(hipEventElapsedTime(&ms, b->events[2 * i], b->events[2 * i + 1]), "hipEventElapsedTime");
            tm->ms[cls[i].first] += ms;
            tm->count[cls[i].first] += 1;
            tm->bytes[cls[i].first] += cls[i].second;
        }
    } else if (!b->use_graph) {
        for (int64_t k = 0; k < qmax; ++k) {
            for (int d = 0; d < 2; ++d) {
                phase_launches(d, k, gl);
                for (auto& L : gl) {
                    void* args[] = {L.multi ? static_cast<void*>(&L.mph) : static_cast<void*>(&L.ph)};
                    BTRY(hipLaunchKernel(L.fn, dim3(L.tiles), dim3(kBatchThreads), args, L.smem, b->stream),
                         "launch batch phase");
                }
            }
        }
    } else {
        if (!reuse) {
            BTRY(hipGraphCreate(&b->graph, 0), "hipGraphCreate");
            // one chain: the group launches of a phase follow each other (they are
            // independent, but a graph with parallel branches is not used here)
            hipGraphNode_t prev = nullptr;
            for (int64_t k = 0; k < qmax; ++k) {
                for (int d = 0; d < 2; ++d) {
                    phase_launches(d, k, gl);
                    for (auto& L : gl) {
                        void* args[] = {L.multi ? static_cast<void*>(&L.mph) : static_cast<void*>(&L.ph)};
                        hipKernelNodeParams kp{};
                        kp.func = const_cast<void*>(L.fn);
                        kp.gridDim = dim3(L.tiles);
                        kp.blockDim = dim3(kBatchThreads);
                        kp.sharedMemBytes = (unsigned)L.smem;
                        kp.kernelParams = args;
                        hipGraphNode_t node;
                        BTRY(hipGraphAddKernelNode(&node, b->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp),
                             "hipGraphAddKernelNode");
                        prev = node;
                    }
                }
            }
            BTRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            b->sig = sig;
            b->graph_half = h;
        }
        if (!launch) return DIRAC_OK;
        BTRY(hipGraphLaunch(b->gexec, b->stream), "hipGraphLaunch");
        BTRY(hipEventRecord(b->graph_done, b->stream), "record graph event");
    }
    for (int i : act) b->slots[i]->step += steps[i];
    return DIRAC_OK;
}

extern "C" {

dirac_status dirac_batch_run(dirac_batch* b, const int64_t* steps) {
    return batch_run_impl(b, steps, nullptr);
}

dirac_status dirac_batch_prepare(dirac_batch* b, const int64_t* steps) {
    if (b && !b->use_graph) return DIRAC_OK;
    return batch_run_impl(b, steps, nullptr, false);
}

dirac_status dirac_batch_run_timed(dirac_batch* b, const int64_t* steps, double* ms_out, int64_t* counts_out,
                                   double* bytes_out) {
    if (!b || !steps || !ms_out || !counts_out || !bytes_out) return fail(DIRAC_E_ARG, "null argument");
    BatchTiming tm{};
    dirac_status r = batch_run_impl(b, steps, &tm);
    if (r != DIRAC_OK) return r;
    for (int i = 0; i < kBatchTimingClasses; ++i) {
        ms_out[i] = tm.ms[i];
        counts_out[i] = tm.count[i];
        bytes_out[i] = tm.bytes[i];
    }
    return DIRAC_OK;
}

static bool bsched_valid_host(int n, int sc) {
    return sc >= 0 && sc < kBatchSchedules && bsched_valid(n, sc);
}

dirac_status dirac_batch_get_schedule(const dirac_batch* b, int32_t n, int32_t dir, dirac_schedule* out) {
    if (!b || !out || dir < 0 || dir > 1 || n < 16 || n > 2048 || (n & (n - 1))) return fail(DIRAC_E_ARG, "bad arguments");
    const int sc = b->sched[dir][__builtin_ctz((unsigned)n)];
    out->radix = bsched_radix(n, sc);
    out->lines_per_wg = bsched_lines(n, sc);
    out->components_per_thread = bsched_cpt(sc);
    return DIRAC_OK;
}

dirac_status dirac_batch_set_schedule(dirac_batch* b, int32_t n, int32_t dir, const dirac_schedule* sch) {
    if (!b || !sch || dir < 0 || dir > 1 || n < 16 || n > 2048 || (n & (n - 1))) return fail(DIRAC_E_ARG, "bad arguments");
    for (int sc = 0; sc < kBatchSchedules; ++sc) {
        if (bsched_valid_host(n, sc) && bsched_radix(n, sc) == sch->radix && bsched_cpt(sc) == sch->components_per_thread &&
            (sch->lines_per_wg == 0 || sch->lines_per_wg == bsched_lines(n, sc))) {
            b->sched[dir][__builtin_ctz((unsigned)n)] = sc;
            ++b->version;
            batch_drop_graph(b);
            return DIRAC_OK;
        }
    }
    return fail(DIRAC_E_ARG, "no batch schedule with radix %d, %d components per thread for n = %d", sch->radix,
                sch->components_per_thread, n);
}

int32_t dirac_batch_schedule_count(int32_t n) {
    if (n < 16 || n > 2048 || (n & (n - 1))) return 0;
    int c = 0;
    for (int sc = 0; sc < kBatchSchedules; ++sc) c += bsched_valid_host(n, sc) ? 1 : 0;
    return c;
}

// Coordinate search: for every (direction, n) present, time each valid
// schedule on `reps` steps of the whole batch (one launch per group and phase,
// each between its own events) and score it by the summed time of the kernels
// it can change (its size group's own kernel and the multi-group kernel of the
// direction), the best of kBatchTuneTrials runs; the lowest-numbered schedule
// within kBatchTuneTie of the fastest is kept (schedule 0 is the default), so
// that near-equal schedules do not flip from one process to the next.  States
// and step counters are restored.
dirac_status dirac_batch_autotune(dirac_batch* b, int32_t reps) {
    if (!b || reps < 1 || reps > 10000) return fail(DIRAC_E_ARG, "bad arguments");
    std::vector<int> occ;
    for (int i = 0; i < b->capacity; ++i)
        if (b->slots[i]) {
            if (!b->slots[i]->has_state) return fail(DIRAC_E_STATE, "slot %d has no state", i);
            occ.push_back(i);
        }
    if (occ.empty()) return DIRAC_OK;
    const bool graph_was = b->use_graph;
    b->use_graph = false;
    batch_drop_graph(b);
    const size_t sz = b->prec == DIRAC_FP32 ? 4 : 8;
    for (int i : occ) {
        dirac_solver* s = b->slots[i];
        const size_t bytes = (size_t)s->g.n1 * s->g.n2 * 4 * sz;
        BTRY(hipMemcpyAsync(s->base + s->lay.scratch, s->base + s->lay.psi, bytes, hipMemcpyDeviceToDevice, b->stream),
             "save state");
    }
    std::vector<int64_t> steps(b->capacity, 0);
    for (int i : occ) steps[i] = reps;
    dirac_status result = DIRAC_OK;
    // summed kernel time (ms) in one timed run of the launches a schedule of
    // (direction d, n = 2^lg) can change: that size group's own kernel and the
    // kernel shared by the small groups of the direction
    auto timed_run = [&](int d, int lg, double& ms) -> dirac_status {
        BatchTiming tm{};
        dirac_status r = batch_run_impl(b, steps.data(), &tm);
        if (r != DIRAC_OK) return r;
        ms = tm.ms[d * 9 + (lg - 4)] + tm.ms[d * 9 + 8];
        return DIRAC_OK;
    };
    double warm = 0;
    result = timed_run(0, 4, warm);
    for (int d = 0; d < 2 && result == DIRAC_OK; ++d) {
        for (int lg = 4; lg <= 11 && result == DIRAC_OK; ++lg) {
            bool present = false;
            for (int i : occ) present |= __builtin_ctz((unsigned)(d == 0 ? b->slots[i]->g.n1 : b->slots[i]->g.n2)) == lg;
            if (!present) continue;
            const int n = 1 << lg;
            const int was = b->sched[d][lg];
            double t[kBatchSchedules];
            double fastest = 1e300;
            for (int sc = 0; sc < kBatchSchedules && result == DIRAC_OK; ++sc) {
                t[sc] = 1e300;
                if (!bsched_valid_host(n, sc)) continue;
                b->sched[d][lg] = sc;
                ++b->version;
                for (int k = 0; k < kBatchTuneTrials && result == DIRAC_OK; ++k) {
                    double ms = 0;
                    result = timed_run(d, lg, ms);
                    if (result == DIRAC_OK) t[sc] = std::min(t[sc], ms);
                }
                fastest = std::min(fastest, t[sc]);
            }
            int pick = was;
            if (result == DIRAC_OK)
                for (int sc = kBatchSchedules - 1; sc >= 0; --sc)
                    if (t[sc] <= fastest * (1.0 + kBatchTuneTie)) pick = sc;
            b->sched[d][lg] = pick;
            ++b->version;
        }
    }
    for (int i : occ) {
        dirac_solver* s = b->slots[i];
        const size_t bytes = (size_t)s->g.n1 * s->g.n2 * 4 * sz;
        BTRY(hipMemcpyAsync(s->base + s->lay.psi, s->base + s->lay.scratch, bytes, hipMemcpyDeviceToDevice, b->stream),
             "restore state");
    }
    BTRY(hipStreamSynchronize(b->stream), "synchronise");
    // every timed run advanced the step counters; put them back
    int runs = 1;
    for (int d = 0; d < 2; ++d)
        for (int lg = 4; lg <= 11; ++lg) {
            bool present = false;
            for (int i : occ) present |= __builtin_ctz((unsigned)(d == 0 ? b->slots[i]->g.n1 : b->slots[i]->g.n2)) == lg;
            if (present)
                for (int sc = 0; sc < kBatchSchedules; ++sc)
                    runs += bsched_valid_host(1 << lg, sc) ? kBatchTuneTrials : 0;
        }
    if (result == DIRAC_OK)
        for (int i : occ) b->slots[i]->step -= (int64_t)runs * reps;
    b->use_graph = graph_was;
    return result;
}

dirac_status dirac_batch_sync(dirac_batch* b) {
    if (!b) return fail(DIRAC_E_ARG, "null batch");
    BTRY(hipStreamSynchronize(b->stream), "synchronise batch stream");
    return DIRAC_OK;
}

dirac_status dirac_batch_destroy(dirac_batch* b) {
    if (!b) return fail(DIRAC_E_ARG, "null batch");
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (int h = 0; h < 2; ++h) {
        if (b->host_stage[h]) (void)hipHostFree(b->host_stage[h]);
        if (b->stage_done[h]) (void)hipEventDestroy(b->stage_done[h]);
    }
    if (b->graph_done) (void)hipEventDestroy(b->graph_done);
    for (hipEvent_t ev : b->events) (void)hipEventDestroy(ev);
    delete b;
    return DIRAC_OK;
}

}  // extern "C"
