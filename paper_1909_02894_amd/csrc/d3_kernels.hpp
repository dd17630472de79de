// d3_kernels.hpp -- direction kernels of the 3-D, 4-spinor step (Scheme II with
// three directions, Sec. 5.2; Dirac representation beta = diag(1, 1, -1, -1),
// alpha^i = [[0, sigma_i], [sigma_i, 0]]).
//
// State: [n3][n2][n1] points, each 4 complex components (u0, u1, w0, w1), i.e.
// 8 T per point.  A line of direction x is a row (stride 1); of direction y a
// column of one z plane (stride n1, lines ordered x-fastest); of direction z a
// column through the planes (stride n1 n2, lines ordered x-fastest), so the L
// lines of a tile are neighbours in memory for y and z.  Per line:
//   [Step 1 (and Step 5 of the previous step): psi <- E psi]
//   psi <- b F^-1[K_i F psi] + (1 - b) psi,  K_i = cos I - i sin alpha^i
//   [Step 5 after the last step]
// The two component pairs (u0, u1) and (w0, w1) are transformed one after the
// other through the same LDS exchange buffer.
// E = [[e0 I, D g.sigma], [D g.sigma, conj(e0) I]] with e0 = C - i D w, stored per
// point as (C, -D w, D g_x, D g_y, D g_z) (curved), or diag(e0u, e0u, conj, conj) (flat).
#pragma once
#include "stage_kernels.hpp"

namespace dirac {

template <typename T>
struct D3Params {
    T* psi;                 // 8 T per point
    const T* a;             // a(x) per point, or null (flat)
    const T* E;             // exponential record per point (D3_EREC T), or null (flat)
    const T* inv_s;         // 1/S along the line direction (ones without a layer)
    const cpx<T>* K;        // (cos, sin)(c dt xi) / n
    const cpx<T>* tw;       // exp(-2 pi i k / n)
    int n1, n2;
    int nlines;
    int e_pre, e_post;
    cpx<T> e0u;             // flat: e^{-i dt m c^2 / 2}
};

template <typename T>
__host__ __device__ constexpr int d3_erec() { return sizeof(T) == 8 ? 6 : 8; }
template <typename T>
__host__ __device__ constexpr int d3_radix(int n) { return (sizeof(T) == 8 || n <= 64) ? 4 : 8; }
template <typename T>
__host__ __device__ constexpr int d3_lines(int n) {
    return (n / d3_radix<T>(n)) >= 256 ? 1 : 256 / (n / d3_radix<T>(n));
}
template <typename T>
__host__ __device__ constexpr int d3_threads(int n) { return (n / d3_radix<T>(n)) * d3_lines<T>(n); }

struct D3Entry {
    int prec, n, dir, lines, nthreads;
    const void* fn[3];      // flat, flat + layer, curved
};
const D3Entry* d3_entry(int prec, int n, int dir);

template <typename T>
__device__ __forceinline__ void load_point4(const T* p, uint32_t idx, cpx<T>& u0, cpx<T>& u1, cpx<T>& w0,
                                            cpx<T>& w1) {
    const char* b = reinterpret_cast<const char*>(p) + idx * (uint32_t)(8 * sizeof(T));
    if constexpr (sizeof(T) == 8) {
        const double2* q = reinterpret_cast<const double2*>(b);
        const double2 A = q[0], B = q[1], C = q[2], D = q[3];
        u0 = {A.x, A.y}; u1 = {B.x, B.y}; w0 = {C.x, C.y}; w1 = {D.x, D.y};
    } else {
        const float4* q = reinterpret_cast<const float4*>(b);
        const float4 A = q[0], B = q[1];
        u0 = {A.x, A.y}; u1 = {A.z, A.w}; w0 = {B.x, B.y}; w1 = {B.z, B.w};
    }
}
template <typename T>
__device__ __forceinline__ void store_point4(T* p, uint32_t idx, cpx<T> u0, cpx<T> u1, cpx<T> w0, cpx<T> w1) {
    char* b = reinterpret_cast<char*>(p) + idx * (uint32_t)(8 * sizeof(T));
    if constexpr (sizeof(T) == 8) {
        d2v* q = reinterpret_cast<d2v*>(b);
        gst(q, d2v{u0.re, u0.im}); gst(q + 1, d2v{u1.re, u1.im});
        gst(q + 2, d2v{w0.re, w0.im}); gst(q + 3, d2v{w1.re, w1.im});
    } else {
        f4v* q = reinterpret_cast<f4v*>(b);
        gst(q, f4v{u0.re, u0.im, u1.re, u1.im});
        gst(q + 1, f4v{w0.re, w0.im, w1.re, w1.im});
    }
}
// (C, -D w, D g_x, D g_y, D g_z)
template <typename T>
__device__ __forceinline__ void load_erec(const T* E, uint32_t idx, T (&e)[5]) {
    const char* b = reinterpret_cast<const char*>(E) + idx * (uint32_t)(d3_erec<T>() * sizeof(T));
    if constexpr (sizeof(T) == 8) {
        const double2* q = reinterpret_cast<const double2*>(b);
        const double2 A = q[0], B = q[1], C = q[2];
        e[0] = A.x; e[1] = A.y; e[2] = B.x; e[3] = B.y; e[4] = C.x;
    } else {
        const float4* q = reinterpret_cast<const float4*>(b);
        const float4 A = q[0], B = q[1];
        e[0] = A.x; e[1] = A.y; e[2] = A.z; e[3] = A.w; e[4] = B.x;
    }
}

// DIR 0: x (rows), 1: y, 2: z.  MODE 0 flat, 1 flat + layer, 2 curved.
template <typename T, int N, int DIR, int MODE>
__global__ void __launch_bounds__(d3_threads<T>(N)) d3_stage_kernel(D3Params<T> p) {
    constexpr int R = d3_radix<T>(N), L = d3_lines<T>(N);
    constexpr bool COLS = DIR != 0;
    constexpr bool BLEND = MODE != 0;
    using F = LineFFT<T, N, R, L, COLS, 2>;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    __shared__ cpx<T> lds[F::LDS_ELEMS];
    __shared__ cpx<T> twl[TS::ELEMS];
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = xcd_tile(blockIdx.x, gridDim.x) * L + c.l;
    const bool valid = line < p.nlines;
    const uint32_t n1 = (uint32_t)p.n1, plane = (uint32_t)p.n1 * (uint32_t)p.n2;
    uint32_t base, stride;
    if constexpr (DIR == 0) { base = (uint32_t)line * n1; stride = 1; }
    else if constexpr (DIR == 1) { base = ((uint32_t)line / n1) * plane + (uint32_t)line % n1; stride = n1; }
    else { base = (uint32_t)line; stride = plane; }
    auto gidx = [&](int pos) -> uint32_t { return base + (uint32_t)pos * stride; };

    cpx<T> u[2][R], w[2][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        u[0][r] = u[1][r] = w[0][r] = w[1][r] = cpx<T>{0, 0};
        if (valid) load_point4(p.psi, gidx(c.j + r * P), u[0][r], u[1][r], w[0][r], w[1][r]);
    }
    const cpx<T>* tw = p.tw;
    if constexpr (TS::ON) {                    // unrolled: no wait between the loads
        cpx<T> twv[F::TW_ITER];
        F::tw_load(twv, p.tw, threadIdx.x);
        F::tw_store(twv, twl, threadIdx.x);
        tw = twl;
    }
    auto applyE = [&](int times) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (MODE == 2) {
                T e[5] = {T(1), T(0), T(0), T(0), T(0)};
                if (valid) load_erec(p.E, gidx(c.j + r * P), e);
                const cpx<T> e0{e[0], e[1]}, e0c{e[0], -e[1]};
                const cpx<T> pxy{e[2], -e[3]}, mxy{e[2], e[3]};     // D (g_x - i g_y), D (g_x + i g_y)
                for (int t = 0; t < times; ++t) {
                    const cpx<T> a0 = u[0][r], a1 = u[1][r], b0 = w[0][r], b1 = w[1][r];
                    // D g.sigma v = (D g_z v0 + D(g_x - i g_y) v1, D(g_x + i g_y) v0 - D g_z v1)
                    u[0][r] = cmul(e0, a0) + scal(e[4], b0) + cmul(pxy, b1);
                    u[1][r] = cmul(e0, a1) + cmul(mxy, b0) - scal(e[4], b1);
                    w[0][r] = cmul(e0c, b0) + scal(e[4], a0) + cmul(pxy, a1);
                    w[1][r] = cmul(e0c, b1) + cmul(mxy, a0) - scal(e[4], a1);
                }
            } else {
                const cpx<T> e0 = p.e0u, e0c{p.e0u.re, -p.e0u.im};
                for (int t = 0; t < times; ++t) {
                    u[0][r] = cmul(e0, u[0][r]);
                    u[1][r] = cmul(e0, u[1][r]);
                    w[0][r] = cmul(e0c, w[0][r]);
                    w[1][r] = cmul(e0c, w[1][r]);
                }
            }
        }
    };
    if (p.e_pre > 0) applyE(p.e_pre);
    cpx<T> ou[BLEND ? 2 : 1][BLEND ? R : 1], ow[BLEND ? 2 : 1][BLEND ? R : 1];
    if constexpr (BLEND) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ou[0][r] = u[0][r]; ou[1][r] = u[1][r];
            ow[0][r] = w[0][r]; ow[1][r] = w[1][r];
        }
    }
    F::template fft<false, TS::ON>(u, lds, c, tw);
    F::template fft<false, TS::ON>(w, lds, c, tw);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const cpx<T> k = p.K[c.j + s * P];
        const T cs = k.re, sn = k.im;
        const cpx<T> a0 = u[0][s], a1 = u[1][s], b0 = w[0][s], b1 = w[1][s];
        if constexpr (DIR == 0) {          // alpha_x: (u, w) -> (sigma_x w, sigma_x u)
            u[0][s] = scal(cs, a0) + mul_mi(scal(sn, b1));
            u[1][s] = scal(cs, a1) + mul_mi(scal(sn, b0));
            w[0][s] = scal(cs, b0) + mul_mi(scal(sn, a1));
            w[1][s] = scal(cs, b1) + mul_mi(scal(sn, a0));
        } else if constexpr (DIR == 1) {   // alpha_y: -i sin sigma_y v = sin (-v1, v0)
            u[0][s] = scal(cs, a0) - scal(sn, b1);
            u[1][s] = scal(cs, a1) + scal(sn, b0);
            w[0][s] = scal(cs, b0) - scal(sn, a1);
            w[1][s] = scal(cs, b1) + scal(sn, a0);
        } else {                           // alpha_z: -i sin sigma_z v = (-i sin v0, i sin v1)
            u[0][s] = scal(cs, a0) + mul_mi(scal(sn, b0));
            u[1][s] = scal(cs, a1) + mul_i(scal(sn, b1));
            w[0][s] = scal(cs, b0) + mul_mi(scal(sn, a0));
            w[1][s] = scal(cs, b1) + mul_i(scal(sn, a1));
        }
    }
    F::template fft<true, TS::ON>(u, lds, c, tw);
    F::template fft<true, TS::ON>(w, lds, c, tw);
    if constexpr (BLEND) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int pos = c.j + r * P;
            T b = gld(p.inv_s + pos);              // ones without a layer
            if constexpr (MODE == 2) b = (valid ? ld_at(p.a, gidx(pos)) : T(0)) * b;
            const T ob = T(1) - b;
            u[0][r] = scal(b, u[0][r]) + scal(ob, ou[0][r]);
            u[1][r] = scal(b, u[1][r]) + scal(ob, ou[1][r]);
            w[0][r] = scal(b, w[0][r]) + scal(ob, ow[0][r]);
            w[1][r] = scal(b, w[1][r]) + scal(ob, ow[1][r]);
        }
    }
    if (p.e_post) applyE(1);
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; ++r) store_point4(p.psi, gidx(c.j + r * P), u[0][r], u[1][r], w[0][r], w[1][r]);
}

}  // namespace dirac
