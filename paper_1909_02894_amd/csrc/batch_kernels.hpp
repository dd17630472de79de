// batch_kernels.hpp -- one kernel per direction phase that advances many
// independent solves of mixed grid sizes at once.
//
// A phase (step k, direction d) covers every tile (L lines) of every solve that
// is still active at step k; the workgroup -> (solve, tile) map is a binary
// search in the per-direction tile prefix of the solves, which are ordered by
// their step counts (longest first), so the active solves are always a prefix.
// All batch schedules use 256-thread workgroups with both spinor components in
// a thread: radix R = 4 for n <= 64, else 8, and L = 256 / (n / R) lines per
// tile, for n up to 2048.  The per-line arithmetic is that of the
// single-solve direction kernel with the same radix, so a solve's result is the
// same bit for bit alone or in any mix.
#pragma once
#include "stage_kernels.hpp"

namespace dirac {

template <typename T>
struct BatchDesc {
    T* psi;
    const T* a;
    const T* E;
    const T* inv_s[2];
    const cpx<T>* K[2];
    const cpx<T>* tw[2];
    int n1, n2;
    int logn[2];      // log2 of the transform length per direction
    int mode;         // 0 flat, 1 flat + layer, 2 curved
    int steps;        // steps of this solve in the current run
    cpx<T> e0u;
};

template <typename T>
struct BatchPhase {
    const BatchDesc<T>* desc;   // ordered by steps, longest first
    const int* prefix;          // tile prefix of this direction (nactive + 1 entries used)
    int nactive;
    int total_tiles;
    int k;                      // step index within the run
};

__host__ __device__ constexpr int batch_radix(int n) { return n <= 64 ? 4 : 8; }
__host__ __device__ constexpr int batch_lines(int n) { return 256 / (n / batch_radix(n)); }
constexpr int kBatchCPT = 2;
constexpr int kBatchThreads = 256;

template <typename T, bool COLS, int N>
__host__ __device__ constexpr size_t batch_smem_bytes() {
    return (LineFFT<T, N, batch_radix(N), batch_lines(N), COLS, kBatchCPT>::LDS_ELEMS + TwStage<T, N>::ELEMS) *
           sizeof(cpx<T>);
}

template <typename T, bool COLS, int N>
__device__ __forceinline__ void batch_tile(const BatchDesc<T>& d, int tile, int k, char* smem) {
    constexpr int R = batch_radix(N), L = batch_lines(N);
    using F = LineFFT<T, N, R, L, COLS, kBatchCPT>;
    static_assert(F::NT == kBatchThreads, "batch schedules use 256-thread workgroups");
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* twl = lds + F::LDS_ELEMS;
    constexpr int dir = COLS ? 1 : 0;
    StageParams<T> p;
    p.psi = d.psi;
    p.a = d.a;
    p.E = d.E;
    p.inv_s = d.inv_s[dir];
    p.K = d.K[dir];
    p.tw = d.tw[dir];
    p.n1 = d.n1;
    p.nlines = COLS ? d.n1 : d.n2;
    p.e_pre = COLS ? 0 : (k == 0 ? 1 : 2);
    p.e_post = COLS ? (k == d.steps - 1 ? 1 : 0) : 0;
    p.e0u = d.e0u;
    if (d.mode == 0) stage_tile<T, N, R, L, COLS, 0, kBatchCPT>(p, tile, lds, twl);
    else if (d.mode == 1) stage_tile<T, N, R, L, COLS, 1, kBatchCPT>(p, tile, lds, twl);
    else stage_tile<T, N, R, L, COLS, 2, kBatchCPT>(p, tile, lds, twl);
}

template <typename T, bool COLS>
__global__ void __launch_bounds__(kBatchThreads) batch_stage_kernel(BatchPhase<T> ph) {
    extern __shared__ __align__(16) char smem[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ph.total_tiles) return;
    int lo = 0, hi = ph.nactive;                 // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ph.prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const BatchDesc<T> d = ph.desc[lo];
    const int tile = t - ph.prefix[lo];
    switch (d.logn[COLS ? 1 : 0]) {
        case 4: batch_tile<T, COLS, 16>(d, tile, ph.k, smem); break;
        case 5: batch_tile<T, COLS, 32>(d, tile, ph.k, smem); break;
        case 6: batch_tile<T, COLS, 64>(d, tile, ph.k, smem); break;
        case 7: batch_tile<T, COLS, 128>(d, tile, ph.k, smem); break;
        case 8: batch_tile<T, COLS, 256>(d, tile, ph.k, smem); break;
        case 9: batch_tile<T, COLS, 512>(d, tile, ph.k, smem); break;
        case 10: batch_tile<T, COLS, 1024>(d, tile, ph.k, smem); break;
        default: batch_tile<T, COLS, 2048>(d, tile, ph.k, smem); break;
    }
}

template <typename T, bool COLS>
constexpr size_t batch_smem_for_logn(int logn) {
    return logn == 4 ? batch_smem_bytes<T, COLS, 16>() : logn == 5 ? batch_smem_bytes<T, COLS, 32>()
         : logn == 6 ? batch_smem_bytes<T, COLS, 64>() : logn == 7 ? batch_smem_bytes<T, COLS, 128>()
         : logn == 8 ? batch_smem_bytes<T, COLS, 256>() : logn == 9 ? batch_smem_bytes<T, COLS, 512>()
         : logn == 10 ? batch_smem_bytes<T, COLS, 1024>() : batch_smem_bytes<T, COLS, 2048>();
}

}  // namespace dirac
