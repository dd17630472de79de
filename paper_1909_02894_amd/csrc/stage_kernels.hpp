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
    const T* a;                  // a(x) per point, or null (a = 1)
    const T* E;                  // half-step exponential per point (e0 re, im, e1 re, im), or null
    const T* inv_s;              // 1/S along the line direction (n entries), or null (no layer)
    const cpx<T>* K;             // symbol per mode, already scaled by 1/n
    const cpx<T>* tw;            // exp(-2 pi i k / n), k < n
    int n1;                      // points per row
    int nlines;                  // lines of this direction
    int e_pre;                   // Step-1 exponentials applied before the transform (0, 1, 2)
    int e_post;                  // Step-5 exponential applied after the blend (0, 1)
    cpx<T> e0u;                  // uniform e0 when E is null (flat: e^{-i dt m c^2 / 2})
};

struct ObsParams {
    const void* psi;             // state (T)
    const double* w;             // observable weight planes, each n1*n2 doubles:
    const double* ca;            //   w = e^{chi - Phi + Psi}, ca = c a,
    const double* gx;            //   gx = c a chi_x / 2, gy = c a chi_y / 2,
    const double* gy;            //   V = e^Phi m c^2
    const double* V;
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
__device__ __forceinline__ const T* at(const T* base, uint32_t elem) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + elem * (uint32_t)sizeof(T));
}
template <typename T> struct PointIO;
template <> struct PointIO<double> {
    static __device__ __forceinline__ void load(const double* p, uint32_t idx, cpx<double>& u, cpx<double>& v) {
        const double2* q = reinterpret_cast<const double2*>(reinterpret_cast<const char*>(p) + idx * 32u);
        const double2 A = q[0], B = q[1];
        u = {A.x, A.y};
        v = {B.x, B.y};
    }
    static __device__ __forceinline__ void store(double* p, uint32_t idx, cpx<double> u, cpx<double> v) {
        double2* q = reinterpret_cast<double2*>(reinterpret_cast<char*>(p) + idx * 32u);
        q[0] = make_double2(u.re, u.im);
        q[1] = make_double2(v.re, v.im);
    }
};
template <> struct PointIO<float> {
    static __device__ __forceinline__ void load(const float* p, uint32_t idx, cpx<float>& u, cpx<float>& v) {
        const float4 A = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(p) + idx * 16u);
        u = {A.x, A.y};
        v = {A.z, A.w};
    }
    static __device__ __forceinline__ void store(float* p, uint32_t idx, cpx<float> u, cpx<float> v) {
        *reinterpret_cast<float4*>(reinterpret_cast<char*>(p) + idx * 16u) = make_float4(u.re, u.im, v.re, v.im);
    }
};

// [u; v] <- [[e0, e1], [conj e1, conj e0]] [u; v]
template <typename T>
__device__ __forceinline__ void apply_E(cpx<T>& u, cpx<T>& v, cpx<T> e0, cpx<T> e1) {
    const cpx<T> nu = cmul(e0, u) + cmul(e1, v);
    const cpx<T> nv = cmulc(u, e1) + cmulc(v, e0);
    u = nu;
    v = nv;
}
// flat: E = diag(e0, conj e0)
template <typename T>
__device__ __forceinline__ void apply_Ediag(cpx<T>& u, cpx<T>& v, cpx<T> e0) {
    u = cmul(e0, u);
    v = cmulc(v, e0);
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
// (TwStage::ELEMS).  Every per-line operation depends on (T, N, R, MODE) only.
template <typename T, int N, int R, int L, bool COLS, bool SPLIT, int MODE>
__device__ __forceinline__ void stage_tile(const StageParams<T>& p, int tile, cpx<T>* lds, cpx<T>* twl) {
    using F = LineFFT<T, N, R, L, COLS, SPLIT>;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    constexpr bool BLEND = MODE != 0;
    // prefetch symbols and blend weights before the transform when registers allow
    constexpr bool PF = sizeof(T) * R <= 32;
    const int tid = threadIdx.x;
    const int l = COLS ? tid % L : tid / P;
    const int j = COLS ? tid / L : tid % P;
    const int line = tile * L + l;
    const bool valid = line < p.nlines;
    const uint32_t n1 = (uint32_t)p.n1;
    auto gidx = [&](int pos) -> uint32_t { return COLS ? (uint32_t)pos * n1 + line : (uint32_t)line * n1 + pos; };

    cpx<T> v[2][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (valid) PointIO<T>::load(p.psi, gidx(j + r * P), v[0][r], v[1][r]);
        else v[0][r] = v[1][r] = cpx<T>{0, 0};
    }
    const cpx<T>* tw = p.tw;
    if constexpr (TS::ON) {
        for (int k = tid; k < N; k += F::NT) twl[k] = p.tw[k];
        tw = twl;
    }
    cpx<T> kk[PF ? R : 1];
    T bb[PF && BLEND ? R : 1];
    if constexpr (PF) {
#pragma unroll
        for (int s = 0; s < R; ++s) kk[s] = p.K[j + s * P];
        if constexpr (BLEND) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                T b = T(1);
                if constexpr (MODE == 2) b = valid ? *at(p.a, gidx(j + r * P)) : T(0);
                if (MODE == 1 || p.inv_s) b *= p.inv_s[j + r * P];
                bb[r] = b;
            }
        }
    }
    if (p.e_pre > 0 && valid) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MODE == 2) {
                cpx<T> e0, e1;
                PointIO<T>::load(p.E, gidx(j + r * P), e0, e1);
                apply_E(v[0][r], v[1][r], e0, e1);
                if (p.e_pre > 1) apply_E(v[0][r], v[1][r], e0, e1);
            } else {
                apply_Ediag(v[0][r], v[1][r], p.e0u);
                if (p.e_pre > 1) apply_Ediag(v[0][r], v[1][r], p.e0u);
            }
        }
    }
    cpx<T> old[BLEND ? 2 : 1][BLEND ? R : 1];
    if constexpr (BLEND) {
#pragma unroll
        for (int r = 0; r < R; ++r) { old[0][r] = v[0][r]; old[1][r] = v[1][r]; }
    }

    F::template fft<false>(v, lds, l, j, tw);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const cpx<T> k = PF ? kk[PF ? s : 0] : p.K[j + s * P];      // (cos, sin) / n
        const cpx<T> u = v[0][s], w = v[1][s];
        if constexpr (!COLS) {                // K_x = cos I - i sin sigma_x
            v[0][s] = scal(k.re, u) + mul_mi(scal(k.im, w));
            v[1][s] = scal(k.re, w) + mul_mi(scal(k.im, u));
        } else {                              // K_y = [[cos, -sin], [sin, cos]]
            v[0][s] = scal(k.re, u) - scal(k.im, w);
            v[1][s] = scal(k.re, w) + scal(k.im, u);
        }
    }
    F::template fft<true>(v, lds, l, j, tw);

    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        cpx<T> u = v[0][r], w = v[1][r];
        if constexpr (BLEND) {
            T b;
            if constexpr (PF) {
                b = bb[r];
            } else {
                b = T(1);
                if constexpr (MODE == 2) b = *at(p.a, gidx(j + r * P));
                if (MODE == 1 || p.inv_s) b *= p.inv_s[j + r * P];
            }
            const T ob = T(1) - b;
            u = scal(b, u) + scal(ob, old[0][r]);
            w = scal(b, w) + scal(ob, old[1][r]);
        }
        if (p.e_post) {
            if constexpr (MODE == 2) {
                cpx<T> e0, e1;
                PointIO<T>::load(p.E, gidx(j + r * P), e0, e1);
                apply_E(u, w, e0, e1);
            } else {
                apply_Ediag(u, w, p.e0u);
            }
        }
        PointIO<T>::store(p.psi, gidx(j + r * P), u, w);
    }
}

template <typename T, int N, int R, int L, bool COLS, bool SPLIT, int MODE>
__global__ void __launch_bounds__(N / R * L)
stage_kernel(StageParams<T> p) {
    __shared__ cpx<T> lds[LineFFT<T, N, R, L, COLS, SPLIT>::LDS_ELEMS];
    __shared__ cpx<T> twl[TwStage<T, N>::ELEMS];
    stage_tile<T, N, R, L, COLS, SPLIT, MODE>(p, xcd_tile(blockIdx.x, gridDim.x), lds, twl);
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
template <typename T, int N, int R, int L, bool COLS, bool SPLIT>
__global__ void __launch_bounds__(N / R * L)
obs_kernel(ObsParams p) {
    using F = LineFFT<T, N, R, L, COLS, SPLIT>;
    static_assert(F::NT % 64 == 0, "observable kernels reduce whole waves");
    constexpr int P = F::P;
    __shared__ cpx<T> lds[F::LDS_ELEMS];
    const int tid = threadIdx.x;
    const int l = COLS ? tid % L : tid / P;
    const int j = COLS ? tid / L : tid % P;
    const int line = xcd_tile(blockIdx.x, gridDim.x) * L + l;
    const bool valid = line < p.nlines;
    const T* psi = static_cast<const T*>(p.psi);
    const T* D = static_cast<const T*>(p.D);
    const cpx<T>* tw = static_cast<const cpx<T>*>(p.tw);

    cpx<T> v[2][R], old[2][R];
    uint32_t idx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int pos = j + r * P;
        idx[r] = COLS ? (uint32_t)pos * (uint32_t)p.n1 + line : (uint32_t)line * (uint32_t)p.n1 + pos;
        if (valid) PointIO<T>::load(psi, idx[r], v[0][r], v[1][r]);
        else v[0][r] = v[1][r] = cpx<T>{0, 0};
        old[0][r] = v[0][r];
        old[1][r] = v[1][r];
    }
    F::template fft<false>(v, lds, l, j, tw);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const T d = D[j + s * P];
        v[0][s] = mul_i(scal(d, v[0][s]));
        v[1][s] = mul_i(scal(d, v[1][s]));
    }
    F::template fft<true>(v, lds, l, j, tw);

    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t q = idx[r];
            const double p0r = old[0][r].re, p0i = old[0][r].im, p1r = old[1][r].re, p1i = old[1][r].im;
            const double d0r = v[0][r].re, d0i = v[0][r].im, d1r = v[1][r].re, d1i = v[1][r].im;
            const double w = p.w[q], ca = p.ca[q];
            double er, ei;
            if constexpr (!COLS) {
                // psi^dag (-i ca sigma_x Dpsi) = -i ca (conj(p0) d1 + conj(p1) d0)
                const double sr = p0r * d1r + p0i * d1i + p1r * d0r + p1i * d0i;
                const double si = p0r * d1i - p0i * d1r + p1r * d0i - p1i * d0r;
                er = ca * si;
                ei = -ca * sr;
                // psi^dag [-i (gx sx + gy sy) + V sz] psi
                //  = conj(p0)[-i(gx - i gy) p1 + V p0] + conj(p1)[-i(gx + i gy) p0 - V p1]
                const double gx = p.gx[q], gy = p.gy[q], V = p.V[q];
                const double ar = -gy, ai = -gx;     // -i (gx - i gy)
                const double br = gy, bi = -gx;      // -i (gx + i gy)
                const double t1r = ar * p1r - ai * p1i, t1i = ar * p1i + ai * p1r;   // (..) p1
                const double t2r = br * p0r - bi * p0i, t2i = br * p0i + bi * p0r;   // (..) p0
                er += p0r * t1r + p0i * t1i + p1r * t2r + p1i * t2i;
                ei += p0r * t1i - p0i * t1r + p1r * t2i - p1i * t2r;
                const double dens0 = p0r * p0r + p0i * p0i, dens1 = p1r * p1r + p1i * p1i;
                er += V * (dens0 - dens1);
                const double dens = dens0 + dens1;
                const int ix = COLS ? line : j + r * P;
                const int iy = COLS ? j + r * P : line;
                const double x = -p.a1 + ix * p.h1, y = -p.a2 + iy * p.h2;
                acc[0] += dens;
                acc[1] += w * dens;
                acc[2] += x * dens;
                acc[3] += y * dens;
                const bool fin = isfinite(p0r) && isfinite(p0i) && isfinite(p1r) && isfinite(p1i);
                acc[6] += fin ? 0.0 : 1.0;
            } else {
                // psi^dag (-i ca sigma_y Dpsi) = ca (-conj(p0) d1 + conj(p1) d0)
                const double sr = -(p0r * d1r + p0i * d1i) + (p1r * d0r + p1i * d0i);
                const double si = -(p0r * d1i - p0i * d1r) + (p1r * d0i - p1i * d0r);
                er = ca * sr;
                ei = ca * si;
            }
            acc[4] += w * er;
            acc[5] += w * ei;
        }
    }
    block_sum<F::NT, 8>(acc, p.partials + 8 * (size_t)blockIdx.x);
}

}  // namespace dirac
