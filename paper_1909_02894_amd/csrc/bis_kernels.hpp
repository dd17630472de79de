// bis_kernels.hpp -- direction kernels of the second-order directional step
// (Sec. 5.2, eq. (step2bis), corrected reading).  Per line, after the forward
// transform psi_hat = F_i psi:
//   psi* = b Xi + (1 - b) psi
//          + ((c dt)^2 / 2) (b (1 - b) F^-1[xi^2 psi_hat] + b b' F^-1[i xi psi_hat]),
//   Xi = F^-1[K_i psi_hat],  b = a / S^i,  b' = (d_i a) / S^i,
// i.e. the blend of eq. (second_scheme) plus the difference between the exact
// transport d_t psi = -c b sigma_i d_i psi and the blend at second order in dt.
// Three inverse transforms share the forward one; Step 1 / Step 5 are fused as
// in the plain direction kernel.  One schedule per size: radix 4, both
// components in a thread, 256-thread workgroups (n / 4 threads per line up to
// n = 2048).
#pragma once
#include "stage_kernels.hpp"

namespace dirac {

template <typename T>
struct BisParams {
    StageParams<T> s;
    const T* da;       // (d_x a, d_y a) per point (curved), or null
    const T* D;        // xi / n along the line direction
    T hh;              // (c dt)^2 / 2
    T n;               // transform length, so xi^2 / n = n D^2
};

struct BisEntry {
    int prec, n, dir, lines, nthreads;
    const void* fn[2];     // [0] flat with layer, [1] curved
};

// Radix 4; one row or two columns per workgroup (row segments of two points)
// from 64-thread lines, so that a 512-point grid gives every SIMD a wave; at
// least 64 threads per workgroup.
constexpr int kBisRadix = 4;
__host__ __device__ constexpr int bis_lines(int n, bool cols) {
    return (n / kBisRadix) >= 256 ? 1
           : (n / kBisRadix) >= 64 ? (cols ? 2 : 1)
           : (cols && 64 / (n / kBisRadix) < 2 ? 2 : 64 / (n / kBisRadix));
}
__host__ __device__ constexpr int bis_threads(int n, bool cols) { return (n / kBisRadix) * bis_lines(n, cols); }

const BisEntry* bis_entry(int prec, int n, int dir);

// MODE 1: flat with layer (b = 1/S, b' = 0, uniform diagonal E); MODE 2: curved.
template <typename T, int N, bool COLS, int MODE>
__global__ void __launch_bounds__(bis_threads(N, COLS)) bis_stage_kernel(BisParams<T> bp) {
    constexpr int R = kBisRadix, L = bis_lines(N, COLS);
    using F = LineFFT<T, N, R, L, COLS, 2>;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    constexpr int dir = COLS ? 1 : 0;
    __shared__ cpx<T> lds[F::LDS_ELEMS];
    __shared__ cpx<T> twl[TS::ELEMS];
    const StageParams<T>& p = bp.s;
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = xcd_tile(blockIdx.x, gridDim.x) * L + c.l;
    const bool valid = line < p.nlines;
    const int lline = valid ? line : p.nlines - 1;     // loads: clamped, branch-free
    const uint32_t n1 = (uint32_t)p.n1;
    auto gidx = [&](int ln, int pos) -> uint32_t {
        return COLS ? (uint32_t)pos * n1 + ln : (uint32_t)ln * n1 + pos;
    };

    // every global load of the tile goes out before the first wait
    cpx<T> v[2][R];
#pragma unroll
    for (int r = 0; r < R; ++r) load_point(p.psi, gidx(lline, c.j + r * P), v[0][r], v[1][r]);
    // Step 1 / Step 5: row comp of E = [[e0, e1], [conj e1, conj e0]];
    // direction-x launches always open with Step 1 and load E up front
    constexpr bool PRELOAD_E = MODE == 2 && !COLS;
    cpx<T> e0[MODE == 2 ? R : 1], e1[MODE == 2 ? R : 1];
    auto loadE = [&]() {
        if constexpr (MODE == 2) {
#pragma unroll
            for (int r = 0; r < R; ++r) load_point(p.E, gidx(lline, c.j + r * P), e0[r], e1[r]);
        }
    };
    if constexpr (PRELOAD_E) loadE();
    const cpx<T>* tw = p.tw;
    cpx<T> twv[TS::ON ? F::TW_ITER : 1];
    if constexpr (TS::ON) F::tw_load(twv, p.tw, threadIdx.x);
    T b[R], k2[R], k1[R], dsym[R];
    cpx<T> ksym[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int pos = c.j + r * P;
        const T s = gld(p.inv_s + pos);            // ones without a layer
        T a = T(1), da = T(0);
        if constexpr (MODE == 2) {
            const uint32_t q = gidx(lline, pos);
            a = ld_at(p.a, (uint32_t)lline * N + pos);   // a along this direction's lines
            da = ld_at(bp.da, 2 * q + dir);
        }
        b[r] = a * s;
        k2[r] = bp.hh * (b[r] * (T(1) - b[r]));
        k1[r] = bp.hh * (b[r] * (da * s));
        dsym[r] = gld(bp.D + pos);
        ksym[r] = gld(p.K + pos);
    }
    if constexpr (TS::ON) {
        F::tw_store(twv, twl, threadIdx.x);
        tw = twl;
    }
    auto applyE = [&](int times) {
        if constexpr (MODE == 2) {
            for (int t = 0; t < times; ++t) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const cpx<T> u = v[0][r], w = v[1][r];
                    v[0][r] = cmul(e0[r], u) + cmul(e1[r], w);
                    v[1][r] = cmul(cpx<T>{e0[r].re, -e0[r].im}, w) + cmul(cpx<T>{e1[r].re, -e1[r].im}, u);
                }
            }
        } else {                               // uniform diag(e0u, conj e0u)
            for (int t = 0; t < times; ++t) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    v[0][r] = cmul(p.e0u, v[0][r]);
                    v[1][r] = cmul(cpx<T>{p.e0u.re, -p.e0u.im}, v[1][r]);
                }
            }
        }
    };
    if constexpr (PRELOAD_E) {
        applyE(1);                             // e_pre is 1 or 2 here
        if (p.e_pre > 1) applyE(1);
    } else if (p.e_pre > 0) {
        loadE();
        applyE(p.e_pre);
    }
    cpx<T> old[2][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        old[0][r] = v[0][r];
        old[1][r] = v[1][r];
    }

    F::template fft<false, TS::ON>(v, lds, c, tw);
    cpx<T> acc[2][R], t[2][R];
    // b (1 - b) (c dt)^2 / 2 * F^-1[xi^2 psi_hat]
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const T d = dsym[s];
        const T w2 = bp.n * d * d;
        t[0][s] = scal(w2, v[0][s]);
        t[1][s] = scal(w2, v[1][s]);
    }
    F::template fft<true, TS::ON>(t, lds, c, tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[0][r] = scal(k2[r], t[0][r]);
        acc[1][r] = scal(k2[r], t[1][r]);
    }
    if constexpr (MODE == 2) {
        // + b b' (c dt)^2 / 2 * F^-1[i xi psi_hat]
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const T d = dsym[s];
            t[0][s] = mul_i(scal(d, v[0][s]));
            t[1][s] = mul_i(scal(d, v[1][s]));
        }
        F::template fft<true, TS::ON>(t, lds, c, tw);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[0][r] = acc[0][r] + scal(k1[r], t[0][r]);
            acc[1][r] = acc[1][r] + scal(k1[r], t[1][r]);
        }
    }
    // Xi = F^-1[K psi_hat]
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const cpx<T> k = ksym[s];
        const cpx<T> a0 = v[0][s], a1 = v[1][s];
        if constexpr (!COLS) {                 // K_x = cos I - i sin sigma_x
            v[0][s] = scal(k.re, a0) + mul_mi(scal(k.im, a1));
            v[1][s] = scal(k.re, a1) + mul_mi(scal(k.im, a0));
        } else {                               // K_y = [[cos, -sin], [sin, cos]]
            v[0][s] = scal(k.re, a0) - scal(k.im, a1);
            v[1][s] = scal(k.re, a1) + scal(k.im, a0);
        }
    }
    F::template fft<true, TS::ON>(v, lds, c, tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
            v[cc][r] = scal(b[r], v[cc][r]) + scal(T(1) - b[r], old[cc][r]) + acc[cc][r];
    }
    if (p.e_post) {
        loadE();
        applyE(1);
    }
    if (!valid) return;
    if ((!COLS || N <= kStoreWtMaxColN) && p.wt) {     // write-through (as in stage_tile)
#pragma unroll
        for (int r = 0; r < R; ++r) store_point<T, true>(p.psi, gidx(line, c.j + r * P), v[0][r], v[1][r]);
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) store_point(p.psi, gidx(line, c.j + r * P), v[0][r], v[1][r]);
    }
}

}  // namespace dirac
