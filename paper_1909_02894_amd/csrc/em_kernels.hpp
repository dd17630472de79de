// em_kernels.hpp -- direction kernels for solves with time-dependent
// electromagnetic potentials (Sec. 2: F(t, x) with A and A0).  The directional
// step is that of eq. (second_scheme); the Step 1 / Step 5 exponential is built
// per point inside the kernel for the time of the step instead of being read
// from a table:
//   E(t) = e^{i (dt/2) e A0} (C I + D u.sigma),  u.u = r^2,  C = cosh r,  D = sinh r / r,
//   u = (sx + i qx fA(t), sy + i qy fA(t), -i wz),
// from a per-point record (sx, sy, wz, qx, qy, q0, a, 0):
//   sx = -(dt/4) c a chi_x, sy = -(dt/4) c a chi_y, wz = (dt/2) m c^2 e^Phi,
//   qx = (dt/2) e c a A_x(x), qy = (dt/2) e c a A_y(x), q0 = (dt/2) e V(x).
// E is evaluated in FP64 and rounded to the state precision.
#pragma once
#include "stage_kernels.hpp"

namespace dirac {

template <typename T>
struct EmParams {
    StageParams<T> s;            // psi, inv_s, K, tw, n1, nlines, e_pre (x only), e_post (a, E, e0u unused)
    const T* rec;                // 8 T per point
    double fA[3], fV[3];         // envelope values: Step-1 applications in order, then Step 5
};

struct EmEntry {
    int prec, n, dir, lines, nthreads;
    const void* fn;
};

// Radix 4 in both directions (more threads per line: the row kernels are
// ALU-bound on the per-point exponentials, and radix 8 with both components per
// thread would hold the column kernels to one wave per SIMD); one row or two
// columns per workgroup (row segments of two points) up to 256-thread lines, so
// that a 512-point grid gives every SIMD a wave.  At least 64 threads per workgroup.
__host__ __device__ constexpr int em_radix(int) { return 4; }
__host__ __device__ constexpr int em_lines(int n, bool cols) {
    return (n / em_radix(n)) >= 256 ? 1
           : (n / em_radix(n)) >= 64 ? (cols ? 2 : 1)
           : (cols && 64 / (n / em_radix(n)) < 2 ? 2 : 64 / (n / em_radix(n)));
}
__host__ __device__ constexpr int em_threads(int n, bool cols) { return (n / em_radix(n)) * em_lines(n, cols); }

const EmEntry* em_entry(int prec, int n, int dir);
hipError_t launch_em_exp(const double* in, double* out, const double* rec, size_t npts, int times, const double* fA,
                         const double* fV, hipStream_t s);
// The pointwise exponential kernel (em_exp_kernel<double / float>), for launch
// descriptions built by the runtime.
const void* em_exp_fn(int prec);

struct Mat2 {
    cpx<double> m00, m01, m10, m11;
};

__device__ __forceinline__ cpx<double> cmul_d(cpx<double> a, cpx<double> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Principal square root, in the cancellation-free form.
__device__ __forceinline__ cpx<double> csqrt_d(cpx<double> z) {
    const double r = hypot(z.re, z.im);
    if (z.re >= 0) {
        const double t = sqrt(0.5 * (r + z.re));
        return {t, t > 0 ? 0.5 * z.im / t : 0.0};
    }
    const double t = sqrt(0.5 * (r - z.re));
    return {0.5 * fabs(z.im) / t, copysign(t, z.im)};
}

// C = cosh r = sum_k z^k / (2k)!, D = sinh r / r = sum_k z^k / (2k+1)!, z = r^2,
// the first K terms in Horner form with constant coefficients.
template <int K>
__device__ __forceinline__ void em_series(cpx<double> z, cpx<double>& C, cpx<double>& D) {
    cpx<double> c{1.0, 0.0}, d{1.0, 0.0};
#pragma unroll
    for (int k = K - 1; k >= 1; --k) {
        const double fc = 1.0 / ((2.0 * k - 1.0) * (2.0 * k)), fd = 1.0 / ((2.0 * k) * (2.0 * k + 1.0));
        const cpx<double> zc = cmul_d(z, c), zd = cmul_d(z, d);
        c = cpx<double>{1.0 + fc * zc.re, fc * zc.im};
        d = cpx<double>{1.0 + fd * zd.re, fd * zd.im};
    }
    C = c;
    D = d;
}

__device__ __forceinline__ Mat2 em_exponential(const double (&q)[6], double fA, double fV) {
    const cpx<double> ux{q[0], q[3] * fA}, uy{q[1], q[4] * fA}, uz{0.0, -q[2]};
    const cpx<double> s2 = cmul_d(ux, ux) + cmul_d(uy, uy) + cmul_d(uz, uz);
    cpx<double> C, D;
    const double a2 = s2.re * s2.re + s2.im * s2.im;       // |u.u|^2
    if (a2 < 1e-8) {
        em_series<4>(s2, C, D);                              // |u.u| < 1e-4: next term < 3e-21
    } else if (a2 < 0.0625) {
        em_series<9>(s2, C, D);                              // |u.u| < 1/4: next term < 1e-21
    } else {
        const cpx<double> r = csqrt_d(s2);
        double sn, cs;
        sincos(r.im, &sn, &cs);
        const double ep = exp(r.re), em = exp(-r.re);
        const cpx<double> epr{ep * cs, ep * sn}, emr{em * cs, -em * sn};   // e^{r}, e^{-r}
        C = cpx<double>{0.5 * (epr.re + emr.re), 0.5 * (epr.im + emr.im)};
        const cpx<double> sh{0.5 * (epr.re - emr.re), 0.5 * (epr.im - emr.im)};
        const double den = r.re * r.re + r.im * r.im;                    // sinh r / r
        D = cpx<double>{(sh.re * r.re + sh.im * r.im) / den, (sh.im * r.re - sh.re * r.im) / den};
    }
    double ps, pc;
    sincos(q[5] * fV, &ps, &pc);
    const cpx<double> ph{pc, ps};
    const cpx<double> Duz = cmul_d(D, uz);
    const cpx<double> a = cpx<double>{ux.re + uy.im, ux.im - uy.re};            // ux - i uy
    const cpx<double> b = cpx<double>{ux.re - uy.im, ux.im + uy.re};            // ux + i uy
    Mat2 m;
    m.m00 = cmul_d(ph, C + Duz);
    m.m01 = cmul_d(ph, cmul_d(D, a));
    m.m10 = cmul_d(ph, cmul_d(D, b));
    m.m11 = cmul_d(ph, cpx<double>{C.re - Duz.re, C.im - Duz.im});
    return m;
}

// Point record: 8 T (64 B FP64 / 32 B FP32), read with 16-byte loads.
template <typename T>
__device__ __forceinline__ void load_record(const T* rec, uint32_t idx, double (&q)[6], double& a) {
    const char* b = reinterpret_cast<const char*>(rec) + idx * (uint32_t)(8 * sizeof(T));
    if constexpr (sizeof(T) == 8) {
        const d2v* r = reinterpret_cast<const d2v*>(b);
        const d2v r0 = gld(r), r1 = gld(r + 1), r2 = gld(r + 2), r3 = gld(r + 3);
        q[0] = r0.x; q[1] = r0.y; q[2] = r1.x; q[3] = r1.y; q[4] = r2.x; q[5] = r2.y; a = r3.x;
    } else {
        const f4v* r = reinterpret_cast<const f4v*>(b);
        const f4v r0 = gld(r), r1 = gld(r + 1);
        q[0] = r0.x; q[1] = r0.y; q[2] = r0.z; q[3] = r0.w; q[4] = r1.x; q[5] = r1.y; a = r1.z;
    }
}

// The record's a alone (the column kernels, which apply no exponential before
// their transform).
template <typename T>
__device__ __forceinline__ double load_record_a(const T* rec, uint32_t idx) {
    return (double)gld(rec + (size_t)idx * 8 + 6);
}

template <typename T>
__device__ __forceinline__ void apply_mat(const Mat2& m, cpx<T>& u, cpx<T>& v) {
    const cpx<T> m00{(T)m.m00.re, (T)m.m00.im}, m01{(T)m.m01.re, (T)m.m01.im};
    const cpx<T> m10{(T)m.m10.re, (T)m.m10.im}, m11{(T)m.m11.re, (T)m.m11.im};
    const cpx<T> nu = cmul(m00, u) + cmul(m01, v);
    const cpx<T> nv = cmul(m10, u) + cmul(m11, v);
    u = nu;
    v = nv;
}

template <typename T, int N, bool COLS>
__global__ void __launch_bounds__(em_threads(N, COLS)) em_stage_kernel(EmParams<T> ep) {
    constexpr int R = em_radix(N), L = em_lines(N, COLS);
    using F = LineFFT<T, N, R, L, COLS, 2>;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    __shared__ cpx<T> lds[F::LDS_ELEMS];
    __shared__ cpx<T> twl[TS::ELEMS];
    const StageParams<T>& p = ep.s;
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = xcd_tile(blockIdx.x, gridDim.x) * L + c.l;
    const bool valid = line < p.nlines;
    const int lline = valid ? line : p.nlines - 1;     // loads: clamped, branch-free
    const uint32_t n1 = (uint32_t)p.n1;
    auto gidx = [&](int ln, int pos) -> uint32_t {
        return COLS ? (uint32_t)pos * n1 + ln : (uint32_t)ln * n1 + pos;
    };

    // every global load of the tile goes out before the first wait; the column
    // kernels (e_pre = 0) read only a from the record
    cpx<T> v[2][R], old[2][R], ksym[R];
    double q[COLS ? 1 : R][6], a[R];
    T b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t g = gidx(lline, c.j + r * P);
        load_point(p.psi, g, v[0][r], v[1][r]);
        if constexpr (COLS) a[r] = load_record_a(ep.rec, g);
        else load_record(ep.rec, g, q[r], a[r]);
    }
    const cpx<T>* tw = p.tw;
    cpx<T> twv[TS::ON ? F::TW_ITER : 1];
    if constexpr (TS::ON) F::tw_load(twv, p.tw, threadIdx.x);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        b[r] = (T)a[r] * gld(p.inv_s + c.j + r * P);       // ones without a layer
        ksym[r] = gld(p.K + c.j + r * P);
    }
    if constexpr (TS::ON) {
        F::tw_store(twv, twl, threadIdx.x);
        tw = twl;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (!COLS)
            for (int k = 0; k < p.e_pre; ++k) apply_mat(em_exponential(q[r], ep.fA[k], ep.fV[k]), v[0][r], v[1][r]);
        old[0][r] = v[0][r];
        old[1][r] = v[1][r];
    }
    F::template fft<false, TS::ON>(v, lds, c, tw);
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
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t g = gidx(line, c.j + r * P);
        cpx<T> u = scal(b[r], v[0][r]) + scal(T(1) - b[r], old[0][r]);
        cpx<T> w = scal(b[r], v[1][r]) + scal(T(1) - b[r], old[1][r]);
        if (p.e_post) {
            double qe[6], ae;
            load_record(ep.rec, g, qe, ae);
            apply_mat(em_exponential(qe, ep.fA[2], ep.fV[2]), u, w);
        }
        if ((!COLS || N <= kStoreWtMaxColN) && p.wt) store_point<T, true>(p.psi, g, u, w);   // as in stage_tile
        else store_point(p.psi, g, u, w);
    }
}

// out <- E(t_1) E(t_0) in (times = 2) or E(t_0) in (times = 1), one thread per
// point (out may be in): Steps 1 / 5 with potentials, as a pass of their own
// (Scheme I, and Scheme II on states small enough to stay in the caches, where
// the direction kernels then run in their plain form).
template <typename T>
struct EmExpParams {
    const T* in;
    T* out;
    const T* rec;
    size_t npts;
    int times;
    double fA[2], fV[2];
};

template <typename T>
__global__ void __launch_bounds__(256) em_exp_kernel(EmExpParams<T> p) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.npts) return;
    cpx<T> u, v;
    double q[6], a;
    load_point(p.in, (uint32_t)i, u, v);
    load_record(p.rec, (uint32_t)i, q, a);
    for (int k = 0; k < p.times; ++k) apply_mat(em_exponential(q, p.fA[k], p.fV[k]), u, v);
    store_point(p.out, (uint32_t)i, u, v);
}

}  // namespace dirac
