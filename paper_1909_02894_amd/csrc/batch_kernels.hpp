// batch_kernels.hpp -- one kernel per direction phase that advances many
// independent solves of mixed grid sizes at once.
//
// A phase (step k, direction d) covers every tile (L lines) of every solve that
// is still active at step k; the workgroup -> (solve, tile) map is a binary
// search in the per-direction tile prefix of the solves, which are ordered by
// their step counts (longest first), so the active solves are always a prefix.
// All batch schedules use 256-thread workgroups.  Per (direction, n) the batch
// picks one of up to four schedules (radix R in {8, 4}, both components in a
// thread or one per lane), with L = 256 / ((n / R) (2 / components)) lines per
// tile, for n up to 2048; schedule 0 (R = 4 for n <= 64, else 8, both
// components) is the default and the others are chosen by the batch autotuner.
// The per-line arithmetic is that of the single-solve direction kernel with the
// same radix, so a solve's result is the same bit for bit alone or in any mix.
#pragma once
#include "stage_kernels.hpp"

namespace dirac {

template <typename T>
struct BatchDesc {
    T* psi;
    const T* a[2];          // a(x) along rows, and transposed (along columns); null when flat
    const T* E;
    const T* inv_s[2];
    const cpx<T>* K[2];
    const cpx<T>* tw[2];
    int n1, n2;
    int logn[2];      // log2 of the transform length per direction
    int mode;         // 0 flat, 1 flat + layer, 2 curved
    int sched[2];     // batch schedule per direction
    int steps;        // steps of this solve in the current run
    cpx<T> e0u;
};

// One launch: the tiles of every active solve of one size group (one
// transform length n along the phase's direction, hence one schedule).
template <typename T>
struct BatchPhase {
    const BatchDesc<T>* desc;   // all solves of the run
    const int* index;           // the group's solves (desc indices), longest run first
    const int* prefix;          // tile prefix over the group (nactive + 1 entries used)
    int nactive;
    int total_tiles;
    int k;                      // step index within the run
};

__host__ __device__ constexpr int batch_radix(int n) { return n <= 64 ? 4 : 8; }
constexpr int kBatchThreads = 256;
constexpr int kBatchSchedules = 4;

// Schedule s for transform length n: radix and components per thread.
__host__ __device__ constexpr int bsched_radix(int n, int s) {
    return (s < 2) == (batch_radix(n) == 8) ? 8 : 4;
}
__host__ __device__ constexpr int bsched_cpt(int s) { return (s & 1) ? 1 : 2; }
__host__ __device__ constexpr int bsched_threads_per_line(int n, int s) {
    return (n / bsched_radix(n, s)) * (bsched_cpt(s) == 1 ? 2 : 1);
}
__host__ __device__ constexpr bool bsched_valid(int n, int s) {
    return s >= 0 && s < kBatchSchedules && n % bsched_radix(n, s) == 0 && n / bsched_radix(n, s) >= 2 &&
           bsched_threads_per_line(n, s) <= kBatchThreads && kBatchThreads % bsched_threads_per_line(n, s) == 0 &&
           n % (bsched_radix(n, s) * bsched_radix(n, s)) == 0;
}
__host__ __device__ constexpr int bsched_lines(int n, int s) { return kBatchThreads / bsched_threads_per_line(n, s); }
__host__ __device__ constexpr int batch_lines(int n) { return bsched_lines(n, 0); }

constexpr int kBatchMaxGroups = 8;
// kernel classes of the timed run: 2 directions x (8 group lengths + the multi-group kernel)
constexpr int kBatchTimingClasses = 18;

// One launch covering several size groups (used when some group is too small
// to fill the GPU on its own): group g owns tiles [start[g], start[g+1]).
template <typename T>
struct BatchMultiPhase {
    const BatchDesc<T>* desc;
    const int* index[kBatchMaxGroups];
    const int* prefix[kBatchMaxGroups];
    int nactive[kBatchMaxGroups];
    int logn[kBatchMaxGroups];
    int sched[kBatchMaxGroups];
    int start[kBatchMaxGroups + 1];
    int ngroups;
    int k;
};

template <typename T, bool COLS, int N, int S>
__host__ __device__ constexpr size_t batch_smem_bytes_s() {
    return (LineFFT<T, N, bsched_radix(N, S), bsched_lines(N, S), COLS, bsched_cpt(S)>::LDS_ELEMS +
            TwStage<T, N>::ELEMS) * sizeof(cpx<T>);
}
template <typename T, bool COLS, int N>
__host__ __device__ constexpr size_t batch_smem_bytes() {
    return batch_smem_bytes_s<T, COLS, N, 0>();
}

template <typename T, bool COLS, int N, int S>
__device__ __forceinline__ void batch_tile(const BatchDesc<T>& d, int tile, int k, char* smem) {
    constexpr int R = bsched_radix(N, S), L = bsched_lines(N, S), CPT = bsched_cpt(S);
    using F = LineFFT<T, N, R, L, COLS, CPT>;
    static_assert(F::NT == kBatchThreads, "batch schedules use 256-thread workgroups");
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* twl = lds + F::LDS_ELEMS;
    constexpr int dir = COLS ? 1 : 0;
    StageParams<T> p;
    p.psi = d.psi;
    p.a = d.a[dir];
    p.E = d.E;
    p.inv_s = d.inv_s[dir];
    p.K = d.K[dir];
    p.tw = d.tw[dir];
    p.n1 = d.n1;
    p.nlines = COLS ? d.n1 : d.n2;
    p.e_pre = COLS ? 0 : (k == 0 ? 1 : 2);
    p.e_post = COLS ? (k == d.steps - 1 ? 1 : 0) : 0;
    p.e0u = d.e0u;
    p.wt = 0;
    if (d.mode == 0) stage_tile<T, N, R, L, COLS, 0, CPT>(p, tile, lds, twl);
    else if (d.mode == 1) stage_tile<T, N, R, L, COLS, 1, CPT>(p, tile, lds, twl);
    else stage_tile<T, N, R, L, COLS, 2, CPT>(p, tile, lds, twl);
}

// Phase kernel of one size group: the workgroup -> (solve, tile) map is a
// binary search in the group's tile prefix.  One instantiation per (n,
// schedule) keeps each kernel's register allocation to what its own schedule
// needs (a kernel covering every size would take the largest).
template <typename T, bool COLS, int N, int S>
__global__ void __launch_bounds__(kBatchThreads) batch_group_kernel(BatchPhase<T> ph) {
    extern __shared__ __align__(16) char smem[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ph.total_tiles) return;
    int lo = 0, hi = ph.nactive;                 // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ph.prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const BatchDesc<T> d = ph.desc[ph.index[lo]];
    batch_tile<T, COLS, N, S>(d, t - ph.prefix[lo], ph.k, smem);
}

template <typename T, bool COLS, int N>
__device__ __forceinline__ void batch_tile_sched(const BatchDesc<T>& d, int tile, int k, char* smem, int s) {
    if constexpr (bsched_valid(N, 1)) { if (s == 1) { batch_tile<T, COLS, N, 1>(d, tile, k, smem); return; } }
    if constexpr (bsched_valid(N, 2)) { if (s == 2) { batch_tile<T, COLS, N, 2>(d, tile, k, smem); return; } }
    if constexpr (bsched_valid(N, 3)) { if (s == 3) { batch_tile<T, COLS, N, 3>(d, tile, k, smem); return; } }
    batch_tile<T, COLS, N, 0>(d, tile, k, smem);
}

// Phase kernel over several size groups: find the group by its tile range,
// then the solve by a binary search in the group's prefix.
template <typename T, bool COLS>
__global__ void __launch_bounds__(kBatchThreads) batch_multi_kernel(BatchMultiPhase<T> ph) {
    extern __shared__ __align__(16) char smem[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ph.start[ph.ngroups]) return;
    int g = 0;
    while (g + 1 < ph.ngroups && t >= ph.start[g + 1]) ++g;
    const int tl = t - ph.start[g];
    const int* prefix = ph.prefix[g];
    int lo = 0, hi = ph.nactive[g];
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= tl) lo = mid; else hi = mid;
    }
    const BatchDesc<T> d = ph.desc[ph.index[g][lo]];
    const int tile = tl - prefix[lo];
    const int s = ph.sched[g];
    switch (ph.logn[g]) {
        case 4: batch_tile_sched<T, COLS, 16>(d, tile, ph.k, smem, s); break;
        case 5: batch_tile_sched<T, COLS, 32>(d, tile, ph.k, smem, s); break;
        case 6: batch_tile_sched<T, COLS, 64>(d, tile, ph.k, smem, s); break;
        case 7: batch_tile_sched<T, COLS, 128>(d, tile, ph.k, smem, s); break;
        case 8: batch_tile_sched<T, COLS, 256>(d, tile, ph.k, smem, s); break;
        case 9: batch_tile_sched<T, COLS, 512>(d, tile, ph.k, smem, s); break;
        case 10: batch_tile_sched<T, COLS, 1024>(d, tile, ph.k, smem, s); break;
        default: batch_tile_sched<T, COLS, 2048>(d, tile, ph.k, smem, s); break;
    }
}

}  // namespace dirac
