// stage_kernels.hpp -- fused direction kernels of one time step, and the fused
// spectral-derivative / reduction kernels of the observables.
//
// Direction kernel (one launch per direction per step), for each line:
//   [Step 1: psi <- E psi, once or twice (Step 5 of the previous step, then
//    Step 1 of this one)]                      (Scheme II Steps 1 and 5)
//   old <- psi
//   psi_hat <- F_i psi (both components)        (Sec. 5 partial DFT)
//   psi_hat <- (K_i(xi) / n) psi_hat, K_x = cos I - i sin sigma_x,
//              K_y = cos I - i sin sigma_y, angle c dt xi   (eq. (second_scheme))
//   Xi <- unnormalised inverse transform of psi_hat
//   psi <- b Xi + (1 - b) old, b = a(x) / S^i(x^i)          (eq. (second_scheme) with PML)
//   [Step 5 after the last step: psi <- E psi]
// The state is an AoS array of points (component 0, component 1), each a
// complex (re, im), so one grid point is 4 reals: rows are contiguous (x
// direction), columns are read as coalesced row segments of L points.
#pragma once
#include "fft_line.hpp"

namespace dirac {

template <typename T>
struct StageParams {
    T* psi;                      // state, 4 T per point, row pitch n1 points
    const T* a;                  // a(x) per point along this direction's lines (row-major for x,
                                 // the transposed table for y: a[line * n + pos]), or null (a = 1)
    const T* E;                  // half-step exponential per point (e0 re, im, e1 re, im), or null
    const T* inv_s;              // 1/S along the line direction (n entries; ones without a layer)
    const cpx<T>* K;             // symbol per mode, already scaled by 1/n
    const cpx<T>* tw;            // exp(-2 pi i k / n), k < n
    int n1;                      // points per row
    int nlines;                  // lines of this direction
    int e_pre;                   // Step-1 exponentials applied before the transform: 1 or 2 in
                                 // direction-x launches (which load E up front; 0 in the flat
                                 // ones behind a potentials pass); direction-y kernels ignore it
    int e_post;                  // Step-5 exponential applied after the blend (0, 1)
    cpx<T> e0u;                  // uniform e0 when E is null (flat: e^{-i dt m c^2 / 2})
    int wt;                      // 1: write-through state stores (rows; columns of n <= 1024)
};

struct ObsParams {
    const void* psi;             // state (T)
    const double* w;             // observable weight planes, each n1*n2 doubles:
    const double* ca;            //   w = e^{chi - Phi + Psi}, ca = c a,
    const double* gx;            //   gx = c a chi_x / 2, gy = c a chi_y / 2,
    const double* gy;            //   V = e^Phi m c^2
    const double* V;
    const double* ax;            // potentials, or null: e c a A_x, e c a A_y, e V planes
    const double* ay;
    const double* v0;
    double fA, fV;               //   and their envelopes at the observation time
    const void* D;               // derivative symbol xi_p / n (T), n entries
    const void* tw;              // twiddles (cpx<T>)
    double* partials;            // 8 doubles per workgroup
    int n1, n2;
    int nlines;
    double a1, a2, h1, h2;
};

// Point access with 32-bit byte offsets (every supported state is < 2 GiB), so
// addresses are formed as a scalar base plus a 32-bit vector offset.
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t elem) {
    return gld(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + elem * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}
template <typename T>
__device__ __forceinline__ const T* at(const T* base, uint32_t elem) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + elem * (uint32_t)sizeof(T));
}

// One spinor component of a point (component c at byte offset c * 2 sizeof(T)).
template <typename T>
__device__ __forceinline__ cpx<T> load_comp(const T* p, uint32_t idx, int c) {
    const char* b = reinterpret_cast<const char*>(p) + idx * (uint32_t)(4 * sizeof(T)) + c * (uint32_t)(2 * sizeof(T));
    return gld(reinterpret_cast<const cpx<T>*>(b));
}
// Both components of a point in one access (16 B for FP32) or two (FP64).
template <typename T>
__device__ __forceinline__ void load_point(const T* p, uint32_t idx, cpx<T>& u, cpx<T>& v) {
    const char* b = reinterpret_cast<const char*>(p) + idx * (uint32_t)(4 * sizeof(T));
    if constexpr (sizeof(T) == 8) {
        const d2v A = gld(reinterpret_cast<const d2v*>(b)), B = gld(reinterpret_cast<const d2v*>(b) + 1);
        u = {(T)A.x, (T)A.y};
        v = {(T)B.x, (T)B.y};
    } else {
        const f4v A = gld(reinterpret_cast<const f4v*>(b));
        u = {(T)A.x, (T)A.y};
        v = {(T)A.z, (T)A.w};
    }
}
// Longest column line whose kernel carries the write-through store path.
constexpr int kStoreWtMaxColN = 1024;

// WT: device-scope write-through stores (gst_wt16 / gst_wt8) instead of
// ordinary ones; p must be wave-uniform then (the kernel's state pointer).
template <typename T, bool WT = false>
__device__ __forceinline__ void store_point(T* p, uint32_t idx, cpx<T> u, cpx<T> v) {
    const uint32_t off = idx * (uint32_t)(4 * sizeof(T));
    char* b = reinterpret_cast<char*>(p) + off;
    if constexpr (sizeof(T) == 8) {
        const d2v a{u.re, u.im}, c{v.re, v.im};
        if constexpr (WT) {
            gst_wt16(p, off, __builtin_bit_cast(u32x4, a));
            gst_wt16(p, off + 16, __builtin_bit_cast(u32x4, c));
        } else {
            gst(reinterpret_cast<d2v*>(b), a);
            gst(reinterpret_cast<d2v*>(b) + 1, c);
        }
    } else {
        const f4v a{u.re, u.im, v.re, v.im};
        if constexpr (WT) gst_wt16(p, off, __builtin_bit_cast(u32x4, a));
        else gst(reinterpret_cast<f4v*>(b), a);
    }
}
template <typename T, bool WT = false>
__device__ __forceinline__ void store_comp(T* p, uint32_t idx, int c, cpx<T> v) {
    const uint32_t off = idx * (uint32_t)(4 * sizeof(T)) + c * (uint32_t)(2 * sizeof(T));
    char* b = reinterpret_cast<char*>(p) + off;
    if constexpr (sizeof(T) == 8) {
        const d2v a{v.re, v.im};
        if constexpr (WT) gst_wt16(p, off, __builtin_bit_cast(u32x4, a));
        else gst(reinterpret_cast<d2v*>(b), a);
    } else {
        const f2v a{v.re, v.im};
        if constexpr (WT) gst_wt8(p, off, __builtin_bit_cast(u32x2, a));
        else gst(reinterpret_cast<f2v*>(b), a);
    }
}

// Workgroup -> tile map that keeps neighbouring tiles on one XCD.  Workgroups
// are dispatched round-robin over the 8 XCDs, each with its own L2; tiles that
// share cache lines (adjacent column tiles, adjacent rows of the per-point
// tables) are given to consecutive workgroups of the same XCD.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int x = b & 7, k = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + k;
}

// Small twiddle tables are staged in LDS at kernel start (one coalesced read)
// so the per-pass twiddle reads do not sit on the critical path.
template <typename T, int N>
struct TwStage {
    static constexpr bool ON = N * sizeof(cpx<T>) <= 16384;
    static constexpr int ELEMS = ON ? N : 1;
};

// MODE 0: flat, no absorbing layer (b = 1: psi <- Xi; E uniform diagonal)
// MODE 1: flat with layer (b = 1/S along the line; E uniform diagonal)
// MODE 2: curved (b = a(x) [/S]; E from the per-point table)
// One tile (L lines) of a direction stage, executed by F::NT threads.  lds and
// twl are the workgroup's exchange buffer (F::LDS_ELEMS) and twiddle stage
// (TwStage::ELEMS).  Every per-line operation depends on (T, N, R, MODE) only:
// the 2x2 mixes are written per output component as (own, other) expressions
// that are the same whether the other component sits in the same thread
// (CPT = 2) or in the partner lane (CPT = 1), so results do not depend on L or CPT.
template <typename T, int N, int R, int L, bool COLS, int MODE, int CPT>
__device__ __forceinline__ void stage_tile(const StageParams<T>& p, int tile, cpx<T>* lds, cpx<T>* twl) {
    using F = LineFFT<T, N, R, L, COLS, CPT>;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    constexpr bool BLEND = MODE != 0;
    // prefetch symbols and blend weights before the transform when registers allow
    constexpr bool PF = sizeof(T) * R * CPT <= 64 && F::NT <= 512;
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = tile * L + c.l;
    const bool valid = line < p.nlines;
    // loads read a clamped line (always in bounds, results unused past the
    // last line) so that they carry no branches; stores are guarded
    const int lline = valid ? line : p.nlines - 1;
    const uint32_t n1 = (uint32_t)p.n1;
    auto gidx = [&](int ln, int pos) -> uint32_t {
        return COLS ? (uint32_t)pos * n1 + ln : (uint32_t)ln * n1 + pos;
    };
    // the a table is laid out along this direction's lines (transposed for columns)
    auto aidx = [&](int ln, int pos) -> uint32_t { return (uint32_t)ln * N + pos; };
    // v[cc][r] <- f(own, other, component, r) for every carried component
    auto mix = [&](cpx<T> (&a)[CPT][R], auto&& f) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (CPT == 1) {
                const cpx<T> o = a[0][r];
                a[0][r] = f(o, partner(o), c.comp, r);
            } else {
                const cpx<T> a0 = a[0][r], a1 = a[1][r];
                a[0][r] = f(a0, a1, 0, r);
                a[1][r] = f(a1, a0, 1, r);
            }
        }
    };

    // Every global load of the tile is issued in one branch-free block before
    // the first use of any of them, so the tile pays one memory latency:
    // state, Step-1 exponential, twiddles, symbols and blend weights.
    cpx<T> v[CPT][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t q = gidx(lline, c.j + r * P);
        if constexpr (CPT == 1) v[0][r] = load_comp(p.psi, q, c.comp);
        else load_point(p.psi, q, v[0][r], v[1][r]);
    }
    // Step 1 (and Step 5 of the previous step): row `comp` of
    // E = [[e0, e1], [conj e1, conj e0]]: A own + B other with A = e0, B = e1 for
    // component 0 and their conjugates for component 1.  Direction-x launches
    // always open with Step 1 (e_pre is 1 or 2), so they load E up front and
    // apply it once unconditionally.
    constexpr bool PRELOAD_E = MODE == 2 && !COLS;
    cpx<T> e0[MODE == 2 ? R : 1], e1[MODE == 2 ? R : 1];
    auto loadE = [&]() {
        if constexpr (MODE == 2) {
#pragma unroll
            for (int r = 0; r < R; ++r) load_point(p.E, gidx(lline, c.j + r * P), e0[r], e1[r]);
        }
    };
    auto applyE = [&](int times) {
        if constexpr (MODE == 2) {
            for (int t = 0; t < times; ++t)
                mix(v, [&](cpx<T> own, cpx<T> other, int comp, int r) {
                    const T sg = comp ? T(-1) : T(1);
                    return cmul(cpx<T>{e0[r].re, sg * e0[r].im}, own) + cmul(cpx<T>{e1[r].re, sg * e1[r].im}, other);
                });
        } else {
            for (int t = 0; t < times; ++t)
                mix(v, [&](cpx<T> own, cpx<T>, int comp, int) {
                    return cmul(cpx<T>{p.e0u.re, comp ? -p.e0u.im : p.e0u.im}, own);
                });
        }
    };
    if constexpr (PRELOAD_E) loadE();
    const cpx<T>* tw = p.tw;
    cpx<T> twv[TS::ON ? F::TW_ITER : 1];
    if constexpr (TS::ON) F::tw_load(twv, p.tw, threadIdx.x);
    // blend weight b = a(x) / S(x^i) (MODE 2) or 1 / S(x^i) (MODE 1); the 1/S
    // table is always present in blended modes (ones without a layer)
    cpx<T> kk[PF ? R : 1];
    T bb[BLEND ? R : 1];
    auto blend_weights = [&]() {
        if constexpr (BLEND) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T sv = gld(p.inv_s + c.j + r * P);
                // columns of 4096+ points (states beyond the Infinity Cache) read a with
                // a streaming load, which keeps it from evicting the partly written row
                // segments of neighbouring column tiles; shorter lines keep it cached
                // (curved FP64 2048² columns: 113 us cached, 133 us streamed)
                if constexpr (MODE == 2 && COLS && N >= 4096) bb[r] = ld_nt(p.a + aidx(lline, c.j + r * P)) * sv;
                else bb[r] = MODE == 2 ? ld_at(p.a, aidx(lline, c.j + r * P)) * sv : sv;
            }
        }
    };
    if constexpr (PF) {
#pragma unroll
        for (int s = 0; s < R; ++s) kk[s] = gld(p.K + c.j + s * P);
        blend_weights();
    }
    if constexpr (TS::ON) {
        F::tw_store(twv, twl, threadIdx.x);
        tw = twl;
    }
    if constexpr (PRELOAD_E) {
        applyE(1);                                 // e_pre is 1 or 2 here
        if (p.e_pre > 1) applyE(1);
    } else if constexpr (!COLS) {                  // column launches never open with Step 1
        if (p.e_pre > 0) {
            loadE();
            applyE(p.e_pre);
        }
    }
    // The blend needs the state before the transform.  Long column tiles, whose
    // registers are the tightest, read it again from memory at the blend
    // instead of holding it through both transforms (no other workgroup writes
    // these points, and this one stores them only after the blend, and column
    // launches apply no E before the transform, so the values are the same).
    constexpr bool REREAD = BLEND && COLS && N * sizeof(cpx<T>) >= 32768;
    cpx<T> old[BLEND ? CPT : 1][BLEND ? R : 1];
    if constexpr (BLEND && !REREAD) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
            for (int r = 0; r < R; ++r) old[cc][r] = v[cc][r];
    }

    F::template fft<false, TS::ON>(v, lds, c, tw);
    mix(v, [&](cpx<T> own, cpx<T> other, int comp, int s) {
        cpx<T> k;
        if constexpr (PF) k = kk[s];
        else k = gld(p.K + c.j + s * P);               // (cos, sin) / n
        if constexpr (!COLS) {                         // K_x = cos I - i sin sigma_x
            return scal(k.re, own) + mul_mi(scal(k.im, other));
        } else {                                       // K_y = [[cos, -sin], [sin, cos]]
            return scal(k.re, own) - scal(comp ? -k.im : k.im, other);
        }
    });
    F::template fft<true, TS::ON>(v, lds, c, tw);

    if constexpr (BLEND) {
        if constexpr (REREAD) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t q = gidx(lline, c.j + r * P);
                if constexpr (CPT == 1) old[0][r] = load_comp(p.psi, q, c.comp);
                else load_point(p.psi, q, old[0][r], old[1][r]);
            }
        }
        if constexpr (!PF) blend_weights();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T b = bb[r];
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) v[cc][r] = scal(b, v[cc][r]) + scal(T(1) - b, old[cc][r]);
        }
    }
    if (p.e_post) {
        loadE();
        applyE(1);
    }
    if (!valid) return;
    // write-through stores exist in every row kernel and in the column kernels
    // of n <= 1024: the extra store path perturbs the long column kernels
    // (the 4096-point one ran 16% slower with it, executed or not)
    if ((!COLS || N <= kStoreWtMaxColN) && p.wt) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t q = gidx(line, c.j + r * P);
            if constexpr (CPT == 1) store_comp<T, true>(p.psi, q, c.comp, v[0][r]);
            else store_point<T, true>(p.psi, q, v[0][r], v[1][r]);
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t q = gidx(line, c.j + r * P);
            if constexpr (CPT == 1) store_comp(p.psi, q, c.comp, v[0][r]);
            else store_point(p.psi, q, v[0][r], v[1][r]);
        }
    }
}

template <typename T, int N, int R, int L, bool COLS, int MODE, int CPT>
__global__ void __launch_bounds__((CPT == 1 ? 2 : 1) * (N / R) * L)
stage_kernel(StageParams<T> p) {
    __shared__ cpx<T> lds[LineFFT<T, N, R, L, COLS, CPT>::LDS_ELEMS];
    __shared__ cpx<T> twl[TwStage<T, N>::ELEMS];
    stage_tile<T, N, R, L, COLS, MODE, CPT>(p, xcd_tile(blockIdx.x, gridDim.x), lds, twl);
}

// Deterministic workgroup sum of NV doubles per thread into out[0..NV).
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV], double* out) {
    __shared__ double red[NT > 64 ? NT / 64 : 1][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = acc[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        acc[k] = x;
    }
    if (NT <= 64) {
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k) out[k] = acc[k];
        }
        return;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double x = 0.0;
            for (int w = 0; w < NT / 64; ++w) x += red[w][k];
            out[k] = x;
        }
    }
}

// Observable pass along one direction: Dpsi = F_i^{-1}[i xi F_i psi] / n in
// registers, then FP64 partial sums per workgroup.  Direction x (rows) also
// accumulates the density moments and the pointwise Hamiltonian terms.
// partial layout: [sum|psi|^2, sum w|psi|^2, sum x|psi|^2, sum y|psi|^2,
//                  energy re, energy im, non-finite count, 0]
template <typename T, int N, int R, int L, bool COLS, int CPT>
__global__ void __launch_bounds__((CPT == 1 ? 2 : 1) * (N / R) * L)
obs_kernel(ObsParams p) {
    using F = LineFFT<T, N, R, L, COLS, CPT>;
    static_assert(F::NT % 64 == 0, "observable kernels reduce whole waves");
    constexpr int P = F::P;
    __shared__ cpx<T> lds[F::LDS_ELEMS];
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = xcd_tile(blockIdx.x, gridDim.x) * L + c.l;
    const bool valid = line < p.nlines;
    const T* psi = static_cast<const T*>(p.psi);
    const T* D = static_cast<const T*>(p.D);
    const cpx<T>* tw = static_cast<const cpx<T>*>(p.tw);

    cpx<T> v[CPT][R], old[CPT][R];
    uint32_t idx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int pos = c.j + r * P;
        idx[r] = COLS ? (uint32_t)pos * (uint32_t)p.n1 + line : (uint32_t)line * (uint32_t)p.n1 + pos;
        if constexpr (CPT == 1) {
            v[0][r] = valid ? load_comp(psi, idx[r], c.comp) : cpx<T>{0, 0};
        } else {
            v[0][r] = v[1][r] = cpx<T>{0, 0};
            if (valid) load_point(psi, idx[r], v[0][r], v[1][r]);
        }
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) old[cc][r] = v[cc][r];
    }
    F::template fft<false>(v, lds, c, tw);
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) v[cc][s] = mul_i(scal(D[c.j + s * P], v[cc][s]));
    F::template fft<true>(v, lds, c, tw);

    // Each carried component adds its share of the sums; the other component
    // (same thread, or the partner lane) enters where the Hamiltonian mixes them.
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            cpx<T> dother, pother;
            if constexpr (CPT == 1) {
                dother = partner(v[0][r]);
                pother = partner(old[0][r]);
            } else {
                dother = v[1 - cc][r];
                pother = old[1 - cc][r];
            }
            const int comp = CPT == 1 ? c.comp : cc;
            if (!valid) continue;
            const double sgn = comp ? -1.0 : 1.0;
            const uint32_t q = idx[r];
            const double pr = old[cc][r].re, pi = old[cc][r].im;   // own component
            const double orr = pother.re, oi = pother.im;          // other component
            const double dr = dother.re, di = dother.im;           // derivative of the other component
            const double w = p.w[q], ca = p.ca[q];
            // conj(own) * D(other)
            const double sr = pr * dr + pi * di, si = pr * di - pi * dr;
            double er, ei;
            if constexpr (!COLS) {
                // -i ca (conj(p0) d1 + conj(p1) d0): this component's term -i ca conj(own) D(other)
                er = ca * si;
                ei = -ca * sr;
                // conj(own) [coef other] with coef = -i (gx - i gy) for component 0 and
                // -i (gx + i gy) for component 1, plus +-V |own|^2
                const double gx = p.gx[q], gy = p.gy[q];
                double V = sgn * p.V[q];
                double ar = -sgn * gy, ai = -gx;
                if (p.ax) {
                    // - e c a fA (A_x sigma_x + A_y sigma_y) - e A0: the other component's
                    // coefficient gains -fA (ax -+ i ay), the diagonal -fV v0
                    ar -= p.fA * p.ax[q];
                    ai += sgn * p.fA * p.ay[q];
                    V -= p.fV * p.v0[q];
                }
                const double tr = ar * orr - ai * oi, ti = ar * oi + ai * orr;
                er += pr * tr + pi * ti;
                ei += pr * ti - pi * tr;
                const double dens = pr * pr + pi * pi;
                er += V * dens;
                const int ix = COLS ? line : c.j + r * P;
                const int iy = COLS ? c.j + r * P : line;
                const double x = -p.a1 + ix * p.h1, y = -p.a2 + iy * p.h2;
                acc[0] += dens;
                acc[1] += w * dens;
                acc[2] += x * dens;
                acc[3] += y * dens;
                acc[6] += (isfinite(pr) && isfinite(pi)) ? 0.0 : 1.0;
            } else {
                // ca (-conj(p0) d1 + conj(p1) d0): this component's term -sgn ca conj(own) D(other)
                er = -sgn * ca * sr;
                ei = -sgn * ca * si;
            }
            acc[4] += w * er;
            acc[5] += w * ei;
        }
    }
    block_sum<F::NT, 8>(acc, p.partials + 8 * (size_t)blockIdx.x);
}

}  // namespace dirac
