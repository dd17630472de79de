// fft_line.hpp -- register/LDS Stockham FFT of one grid line (row or column)
// for both spinor components, for gfx950 (wave64).
//
// The partial transforms F_i / F_i^{-1} of Sec. 5 (unnormalised forward sum
// psi_k exp(-2 pi i p k / n); the 1/n of the inverse is folded into the
// Fourier symbol by the caller) are computed with the iterative Stockham
// autosort decimation-in-time formulation (Govindaraju et al., SC'08): pass
// with radix Rp after Ns = product of earlier radices reads butterfly jj's
// inputs at jj + r n/Rp, multiplies input r by W_n^{r (jj mod Ns) n/(Ns Rp)},
// takes a radix-Rp DFT and writes output s at (jj / Ns) Ns Rp + jj mod Ns + s Ns.
//
// Thread layout.  A line of n points is handled by P = n / R logical threads
// per spinor component; logical thread j keeps R values in registers.  The
// first and the last pass have radix R, so on entry thread j holds positions
// j + r P and on exit it holds modes j + s P: the symbol multiply and the
// blend with the untouched input happen in registers, and only the interior
// passes go through LDS.
// Radix schedule: n = R^e * rem (rem < R), passes [R, rem, R, ..., R].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dirac {

template <typename T> struct cpx { T re, im; };

template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T> __device__ __forceinline__ cpx<T> conjc(cpx<T> a) { return {a.re, -a.im}; }
template <typename T> __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.im, a.re}; }   // * i
template <typename T> __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.im, -a.re}; }  // * -i
template <typename T> __device__ __forceinline__ cpx<T> scal(T s, cpx<T> a) { return {s * a.re, s * a.im}; }

// cos / sin of 2 pi m / 16 (m = 0..15), as double literals.
__host__ __device__ constexpr double cos16(int m) {
    return m == 0 ? 1.0 : m == 1 ? 0.92387953251128673848 : m == 2 ? 0.70710678118654752440
         : m == 3 ? 0.38268343236508977173 : m == 4 ? 0.0 : m == 5 ? -0.38268343236508977173
         : m == 6 ? -0.70710678118654752440 : m == 7 ? -0.92387953251128673848 : m == 8 ? -1.0
         : m == 9 ? -0.92387953251128673848 : m == 10 ? -0.70710678118654752440
         : m == 11 ? -0.38268343236508977173 : m == 12 ? 0.0 : m == 13 ? 0.38268343236508977173
         : m == 14 ? 0.70710678118654752440 : 0.92387953251128673848;
}
__host__ __device__ constexpr double sin16(int m) { return cos16((m + 12) % 16); }

// v * exp(-+ 2 pi i M / 16): forward sign -, inverse sign +.
template <typename T, int M, bool INV>
__device__ __forceinline__ cpx<T> rot16(cpx<T> v) {
    if constexpr (M == 0) {
        return v;
    } else if constexpr (M == 4) {
        return INV ? mul_i(v) : mul_mi(v);
    } else if constexpr (M == 8) {
        return {-v.re, -v.im};
    } else if constexpr (M == 12) {
        return INV ? mul_mi(v) : mul_i(v);
    } else {
        const T c = (T)cos16(M);
        const T s = INV ? (T)sin16(M) : (T)(-sin16(M));
        return {v.re * c - v.im * s, v.re * s + v.im * c};
    }
}

// Global-memory access through address-space-1 pointers.  Pointers that reach
// a kernel inside a descriptor table (the batch engine) are otherwise generic
// and compile to flat instructions, whose completion is tracked by the memory
// and the LDS counters together, so every LDS wait would also wait for memory.
// Only scalar and clang vector element types are loaded this way: a struct
// copy goes through a generic reference again.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T gld(const T* p) { return *(const __attribute__((address_space(1))) T*)p; }
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) { *(__attribute__((address_space(1))) T*)p = v; }
// Device-scope write-through stores (buffer_store ... sc1) of 16 or 8 bytes at
// byte offset `off` from the wave-uniform `base`: the line goes to memory at
// once instead of sitting dirty in this XCD's L2 until the end-of-dispatch
// write-back.  Full-width stores, so a wave's contiguous stores still combine
// into whole lines.  The resource's third dword is the gfx9 raw-buffer format;
// the range (2 GiB) covers every supported state.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wt_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
constexpr int kCacheSc1 = 16;      // cache-policy bit sc1 of the buffer intrinsics
__device__ __forceinline__ void gst_wt16(const void* base, uint32_t off, u32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, wt_rsrc(base), (int)off, 0, kCacheSc1);
}
__device__ __forceinline__ void gst_wt8(const void* base, uint32_t off, u32x2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(v, wt_rsrc(base), (int)off, 0, kCacheSc1);
}
__device__ __forceinline__ cpx<float> gld(const cpx<float>* p) {
    const f2v v = gld(reinterpret_cast<const f2v*>(p));
    return {v.x, v.y};
}
__device__ __forceinline__ cpx<double> gld(const cpx<double>* p) {
    const d2v v = gld(reinterpret_cast<const d2v*>(p));
    return {v.x, v.y};
}

__host__ __device__ constexpr int bitrev(int i, int R) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
    return r;
}

template <typename T, int LEN, int K, bool INV>
__device__ __forceinline__ void dft_butterflies(cpx<T>* y) {
    if constexpr (K < LEN / 2) {
        const cpx<T> u = y[K];
        const cpx<T> t = rot16<T, (16 / LEN) * K, INV>(y[K + LEN / 2]);
        y[K] = u + t;
        y[K + LEN / 2] = u - t;
        dft_butterflies<T, LEN, K + 1, INV>(y);
    }
}

template <typename T, int R, int LEN, bool INV>
__device__ __forceinline__ void dft_stages(cpx<T>* y) {
    if constexpr (LEN <= R) {
#pragma unroll
        for (int i = 0; i < R; i += LEN) dft_butterflies<T, LEN, 0, INV>(y + i);
        dft_stages<T, R, LEN * 2, INV>(y);
    }
}

// In-register DFT of size R (2, 4, 8, 16): x_s <- sum_r x_r exp(-+ 2 pi i r s / R).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T>* x) {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16, "radix");
    if constexpr (R > 1) {
        cpx<T> y[R];
#pragma unroll
        for (int i = 0; i < R; ++i) y[i] = x[bitrev(i, R)];
        dft_stages<T, R, 2, INV>(y);
#pragma unroll
        for (int i = 0; i < R; ++i) x[i] = y[i];
    }
}

__host__ __device__ constexpr int ilog(int n, int r) {  // largest e with r^e | n
    int e = 0;
    while (n % r == 0 && n > 1) { n /= r; ++e; }
    return e;
}
__host__ __device__ constexpr int ipow(int r, int e) { int v = 1; for (int i = 0; i < e; ++i) v *= r; return v; }

// Largest LDS exchange buffer (bytes) that holds both spinor components of a
// tile at once; larger tiles of threads carrying both exchange them one at a time.
#ifndef DIRAC_LDS_BOTH_MAX
#define DIRAC_LDS_BOTH_MAX (160 * 1024)
#endif
constexpr size_t kLdsBothMax = DIRAC_LDS_BOTH_MAX;

// Exchange of a 32-bit value with the partner lane (lane xor 32) of the same
// wave, with gfx950's v_permlane32_swap (upper half of the first operand <->
// lower half of the second): lanes 0..31 find the partner's value in the second
// result, lanes 32..63 in the first.
__device__ __forceinline__ uint32_t partner_u32(uint32_t x) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
}
__device__ __forceinline__ float partner(float x) {
    return __uint_as_float(partner_u32(__float_as_uint(x)));
}
__device__ __forceinline__ double partner(double x) {
    const uint64_t b = __double_as_longlong(x);
    const uint32_t lo = partner_u32((uint32_t)b), hi = partner_u32((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ cpx<T> partner(cpx<T> v) { return {partner(v.re), partner(v.im)}; }

// One line geometry: N-point transform, R values per thread per component,
// L lines per workgroup, COLS = lines are columns (line index fastest among
// threads, for coalesced row segments), CPT = spinor components per thread.
//
// CPT = 2: a thread carries both components of its R points (NT = P L threads).
// CPT = 1: a thread carries ONE component: in every wave, lanes 0..31 hold
// component 0 and lanes 32..63 component 1 of the same 32 logical threads, so
// the two components of a point sit in partner lanes (lane xor 32) and the
// 2x2 mixes (half-step exponential, directional symbol) exchange them with one
// permlane swap (NT = 2 P L threads, half the registers per thread).
// A line of N points is held by P = N / R logical threads.
template <typename T, int N, int R, int L, bool COLS, int CPT>
struct LineFFT {
    static constexpr int P = N / R;
    static constexpr int NTL = P * L;
    static constexpr int NT = (CPT == 1 ? 2 : 1) * NTL;
    static constexpr int E = ilog(N, R);
    static constexpr int REM = N / ipow(R, E);
    static constexpr int NPASS = E + (REM > 1 ? 1 : 0);
    // LDS layout, padded against bank conflicts: rows keep each (line, component)
    // run contiguous with one pad element after every R elements (the first
    // exchange writes with stride R); columns interleave the L lines of a position
    // and add COL_PAD pad elements every 16.  The first exchange of a column
    // tile writes element (R j + s) L + l from lane (j, l): with 16 / R pads per
    // 16 elements, neighbouring j land L R + L elements apart, so the lanes of
    // one access cover distinct banks (one pad suffices for a single line).
    // SEQ: when the layout of both components would not fit kLdsBothMax bytes, a
    // thread carrying both (CPT = 2) exchanges them one after the other through
    // a one-component buffer (twice the barriers, half the LDS; every value takes
    // the same path, so results are bitwise the same).
    static constexpr int ROW_STRIDE = N + N / R;
    static constexpr int COL_PAD = (L == 1 || R >= 16) ? 1 : 16 / R;
    __host__ __device__ static constexpr int lds_elems(int ncomp) {
        return (NPASS > 1) ? (COLS ? ncomp * N * L + (ncomp * N * L / 16) * COL_PAD : L * ncomp * ROW_STRIDE) : 1;
    }
    static constexpr bool SEQ = CPT == 2 && (lds_elems(2) * sizeof(cpx<T>) > kLdsBothMax ||
                                              (lds_elems(2) * sizeof(cpx<T>) > kLdsBothMax / 2 && NT <= 256));
    static constexpr int NCL = SEQ ? 1 : 2;        // components held in LDS at once
    static constexpr int LDS_ELEMS = lds_elems(NCL);
    static_assert(LDS_ELEMS * sizeof(cpx<T>) <= 160 * 1024, "exchange buffer exceeds the LDS");
    static_assert(CPT == 1 || CPT == 2, "components per thread");
    static_assert(N % R == 0, "R must divide N");
    static_assert(NPASS == 1 ? N == R : E >= 2, "schedule needs radix-R first and last passes");
    static_assert((CPT == 2 || NTL % 32 == 0) && NT <= 1024, "32 logical threads per wave, <= 1024 threads");

    __host__ __device__ static constexpr int radix_of(int p) { return (p == 1 && REM > 1) ? REM : R; }
    __host__ __device__ static constexpr int ns_of(int p) {
        int ns = 1;
        for (int q = 0; q < p; ++q) ns *= radix_of(q);
        return ns;
    }
    __device__ static __forceinline__ int lidx(int l, int comp, int pos) {
        const int cm = SEQ ? 0 : comp;
        if constexpr (COLS) {
            const int a = (cm * N + pos) * L + l;
            return a + (a / 16) * COL_PAD;
        } else {
            return (l * NCL + cm) * ROW_STRIDE + pos + pos / R;
        }
    }
    // Coordinates of physical thread t: component (CPT = 1), line within the
    // tile, and logical thread index j within the line.
    struct Coord { int comp, l, j; };
    __device__ static __forceinline__ Coord coord(int t) {
        if constexpr (CPT == 1) {
            const int comp = (t >> 5) & 1;
            const int u = ((t >> 6) << 5) | (t & 31);
            return Coord{comp, COLS ? u % L : u / P, COLS ? u / L : u % P};
        } else {
            return Coord{0, COLS ? t % L : t / P, COLS ? t / L : t % P};
        }
    }
    __device__ static __forceinline__ int slot(const Coord& c, int cc) { return CPT == 1 ? c.comp : cc; }

    // Per-pass twiddle layout (for tables staged in LDS).  Pass p >= 1 reads
    // W_N^{r k N / (Ns Rp)} for k = jj mod Ns and r = 1..Rp-1; the plain table
    // W_N^m read at m = r k N / (Ns Rp) puts the distinct k of a wave a multiple
    // of 32 banks apart (up to 8-way conflicts).  Stored per pass as
    // [k][r - 1] instead, neighbouring k sit Rp - 1 (odd) entries apart, so a
    // wave's reads fall on distinct banks.  Entry count: sum_p Ns_p (Rp - 1) < N.
    __host__ __device__ static constexpr int tw_off(int p) {
        int o = 0;
        for (int q = 1; q < p; ++q) o += ns_of(q) * (radix_of(q) - 1);
        return o;
    }
    static constexpr int TW_ENTRIES = NPASS > 1 ? tw_off(NPASS) : 1;
    static_assert(TW_ENTRIES <= N, "the per-pass layout fits an N-entry stage");
    static constexpr int TW_ITER = (TW_ENTRIES + NT - 1) / NT;
    template <int PASS>
    __device__ static __forceinline__ int tw_src(int e) {
        if constexpr (PASS >= NPASS) {
            return 0;
        } else {
            constexpr int Rp = radix_of(PASS), Ns = ns_of(PASS), off = tw_off(PASS);
            if (e < off + Ns * (Rp - 1)) {
                const int q = e - off;
                return (q % (Rp - 1) + 1) * (q / (Rp - 1)) * (N / (Ns * Rp));
            }
            return tw_src<PASS + 1>(e);
        }
    }
    // Gather the per-pass layout from the plain table tw[m] = exp(-2 pi i m / N):
    // tw_load issues the loads (thread t takes entries t + i NT), tw_store
    // writes them to LDS once they have arrived.
    __device__ static __forceinline__ void tw_load(cpx<T> (&reg)[TW_ITER], const cpx<T>* tw, int t) {
#pragma unroll
        for (int i = 0; i < TW_ITER; ++i) {
            const int e = t + i * NT;
            const int src = tw_src<1>(TW_ENTRIES % NT == 0 || e < TW_ENTRIES ? e : TW_ENTRIES - 1);
            reg[i] = gld(tw + src);
        }
    }
    __device__ static __forceinline__ void tw_store(const cpx<T> (&reg)[TW_ITER], cpx<T>* twl, int t) {
#pragma unroll
        for (int i = 0; i < TW_ITER; ++i) {
            const int e = t + i * NT;
            if (TW_ENTRIES % NT == 0 || e < TW_ENTRIES) twl[e] = reg[i];
        }
    }

    // Exchange after pass PASS-1 and compute pass PASS (PASS >= 1).  PP: tw is
    // the per-pass layout (else the plain table).
    template <bool INV, bool PP, int PASS>
    __device__ static __forceinline__ void pass(cpx<T> (&v)[CPT][R], cpx<T>* lds, const Coord& c,
                                                const cpx<T>* __restrict__ tw) {
        constexpr int Rq = radix_of(PASS - 1), Nq = ns_of(PASS - 1);
        constexpr int Rp = radix_of(PASS), Ns = ns_of(PASS);
        // components [c0, c1) through the buffer: all at once, or one at a time (SEQ)
        auto exchange = [&](int c0, int c1) {
#pragma unroll
            for (int cc = c0; cc < c1; ++cc) {
#pragma unroll
                for (int t = 0; t < R / Rq; ++t) {
                    const int jj = c.j + t * P;
                    const int base = (jj / Nq) * Nq * Rq + (jj % Nq);
#pragma unroll
                    for (int s = 0; s < Rq; ++s) lds[lidx(c.l, slot(c, cc), base + s * Nq)] = v[cc][t * Rq + s];
                }
            }
            __syncthreads();
#pragma unroll
            for (int cc = c0; cc < c1; ++cc) {
#pragma unroll
                for (int t = 0; t < R / Rp; ++t) {
                    const int jj = c.j + t * P;
#pragma unroll
                    for (int r = 0; r < Rp; ++r) v[cc][t * Rp + r] = lds[lidx(c.l, slot(c, cc), jj + r * (N / Rp))];
                }
            }
            __syncthreads();
        };
        if constexpr (SEQ) {
            exchange(0, 1);
            exchange(1, 2);
        } else {
            exchange(0, CPT);
        }
#pragma unroll
        for (int t = 0; t < R / Rp; ++t) {
            const int jj = c.j + t * P;
            const int k = jj % Ns;
#pragma unroll
            for (int r = 1; r < Rp; ++r) {
                const cpx<T> w = PP ? tw[tw_off(PASS) + k * (Rp - 1) + (r - 1)] : tw[r * k * (N / (Ns * Rp))];
#pragma unroll
                for (int cc = 0; cc < CPT; ++cc)
                    v[cc][t * Rp + r] = INV ? cmulc(v[cc][t * Rp + r], w) : cmul(v[cc][t * Rp + r], w);
            }
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) dft<T, Rp, INV>(&v[cc][t * Rp]);
        }
        if constexpr (PASS + 1 < NPASS) pass<INV, PP, PASS + 1>(v, lds, c, tw);
    }

    // Transform the components this thread carries.  Entry: v[cc][r] = position
    // j + r P.  Exit: v[cc][s] = mode (forward) / position (inverse) j + s P.
    // tw: the plain table tw[m] = exp(-2 pi i m / N) (PP = false) or its
    // per-pass layout (PP = true); the inverse uses conjugates and is unnormalised.
    template <bool INV, bool PP = false>
    __device__ static __forceinline__ void fft(cpx<T> (&v)[CPT][R], cpx<T>* lds, const Coord& c,
                                               const cpx<T>* __restrict__ tw) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) dft<T, R, INV>(v[cc]);
        if constexpr (NPASS > 1) pass<INV, PP, 1>(v, lds, c, tw);
    }
};

}  // namespace dirac
