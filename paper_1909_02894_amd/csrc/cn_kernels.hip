// cn_kernels.hip -- Numerical Scheme I (Sec. 5.1): the Crank-Nicolson transport
// step G psi* = G~ psi^{n+1/2}, G = I + (dt/2) alpha(x).T, G~ = I - (dt/2) alpha(x).T,
// solved with restarted GMRES whose matrix-vector product runs on the same line
// transforms as the direction kernels (FP64).
//
// alpha(x).T psi = c (b_x sigma_x [[d_x]] psi + b_y sigma_y [[d_y]] psi), with the
// spectral derivative of eq. (trick) and b_i = a / S^i (Appendix A, with layers).
#include <hip/hip_runtime.h>

#include "cn_kernels.hpp"
#include "stage_kernels.hpp"

namespace dirac {

// Row passes: radix 4 up to 512 points (more threads per line); column passes: radix 8
// and at least two lines per workgroup (32-byte row segments of the FP64 state).
// At least 64 threads per workgroup, and as many workgroups as lines allow.
__host__ __device__ constexpr int cn_radix(int n, bool cols) { return n <= 64 ? 4 : (cols || n > 512 ? 8 : 4); }
__host__ __device__ constexpr int cn_lines(int n, bool cols) {
    return (n / cn_radix(n, cols)) >= 64 ? (cols ? 2 : 1)
                                         : (cols && 64 / (n / cn_radix(n, cols)) < 2 ? 2 : 64 / (n / cn_radix(n, cols)));
}

// out = in + s h c b_x sigma_x [[d_x]] in          (x pass, rows)
// out = out + s h c b_y sigma_y [[d_y]] in         (y pass, columns)
template <int N, bool COLS>
__global__ void __launch_bounds__((N / cn_radix(N, COLS)) * cn_lines(N, COLS)) cn_apply_kernel(CnApplyParams p) {
    using T = double;
    constexpr int R = cn_radix(N, COLS), L = cn_lines(N, COLS);
    using F = LineFFT<T, N, R, L, COLS, 2>;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    __shared__ cpx<T> lds[F::LDS_ELEMS];
    __shared__ cpx<T> twl[TS::ELEMS];
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = xcd_tile(blockIdx.x, gridDim.x) * L + c.l;
    const bool valid = line < p.nlines;
    const int lline = valid ? line : p.nlines - 1;     // loads: clamped, branch-free
    const uint32_t n1 = (uint32_t)p.n1;
    auto gidx = [&](int ln, int pos) -> uint32_t {
        return COLS ? (uint32_t)pos * n1 + ln : (uint32_t)ln * n1 + pos;
    };
    // every global load goes out before the first wait: the vector, twiddles,
    // derivative symbol, blend factors and (y pass) the x pass's output
    cpx<T> v[2][R], in[2][R], o[2][R];
    T d[R], bf[R];
#pragma unroll
    for (int r = 0; r < R; ++r) load_point(p.in, gidx(lline, c.j + r * P), v[0][r], v[1][r]);
    const cpx<T>* tw = p.tw;
    cpx<T> twv[TS::ON ? F::TW_ITER : 1];
    if constexpr (TS::ON) F::tw_load(twv, p.tw, threadIdx.x);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        d[r] = gld(p.D + c.j + r * P);
        bf[r] = gld(p.inv_s + c.j + r * P);              // ones without a layer
    }
    if (p.a) {
#pragma unroll
        for (int r = 0; r < R; ++r) bf[r] = ld_at(p.a, gidx(lline, c.j + r * P)) * bf[r];
    }
    if constexpr (COLS) {
#pragma unroll
        for (int r = 0; r < R; ++r) load_point(p.out, gidx(lline, c.j + r * P), o[0][r], o[1][r]);
    }
    if constexpr (TS::ON) {
        F::tw_store(twv, twl, threadIdx.x);
        tw = twl;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        in[0][r] = v[0][r];
        in[1][r] = v[1][r];
    }
    F::template fft<false, TS::ON>(v, lds, c, tw);
#pragma unroll
    for (int s = 0; s < R; ++s) {
        v[0][s] = mul_i(scal(d[s], v[0][s]));
        v[1][s] = mul_i(scal(d[s], v[1][s]));
    }
    F::template fft<true, TS::ON>(v, lds, c, tw);
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t q = gidx(line, c.j + r * P);
        const T f = p.scale * bf[r];               // s (dt/2) c b
        cpx<T> t0, t1;                             // sigma_i [[d_i]] psi
        if constexpr (!COLS) {
            t0 = v[1][r];
            t1 = v[0][r];
        } else {
            t0 = mul_mi(v[1][r]);
            t1 = mul_i(v[0][r]);
        }
        cpx<T> o0, o1;
        if constexpr (!COLS) {
            o0 = in[0][r];
            o1 = in[1][r];
        } else {
            o0 = o[0][r];
            o1 = o[1][r];
        }
        store_point(p.out, q, o0 + scal(f, t0), o1 + scal(f, t1));
    }
}

// psi <- E psi (times = 1 or 2), E = [[e0, e1], [conj e1, conj e0]] per point, or the
// uniform diagonal diag(e0u, conj e0u) when E is null.
__global__ void cn_exp_kernel(double* psi, const double* E, double2 e0u, size_t npts, int times) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    cpx<double> u, v, e0{e0u.x, e0u.y}, e1{0, 0};
    load_point(psi, (uint32_t)i, u, v);
    if (E) load_point(E, (uint32_t)i, e0, e1);
    for (int t = 0; t < times; ++t) {
        const cpx<double> nu = cmul(e0, u) + cmul(e1, v);
        const cpx<double> nv = cmul(cpx<double>{e0.re, -e0.im}, v) + cmul(cpx<double>{e1.re, -e1.im}, u);
        u = nu;
        v = nv;
    }
    store_point(psi, (uint32_t)i, u, v);
}

// Fixed-order workgroup sum of NS complex values per thread (a 64-lane butterfly,
// then the four waves in order); slot k of the result goes to out[2k], out[2k+1].
template <int NS>
__device__ __forceinline__ void block_sum_store(double (&ar)[NS], double (&ai)[NS], double* out) {
    static_assert(NS >= 1 && NS <= 9, "slots per launch");
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            ar[k] += __shfl_xor(ar[k], off);
            ai[k] += __shfl_xor(ai[k], off);
        }
    }
    __shared__ double sr[NS][4], si[NS][4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            sr[k][wave] = ar[k];
            si[k][wave] = ai[k];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < NS) {
        const int k = threadIdx.x;
        out[2 * k] = ((sr[k][0] + sr[k][1]) + sr[k][2]) + sr[k][3];
        out[2 * k + 1] = ((si[k][0] + si[k][1]) + si[k][2]) + si[k][3];
    }
}

// Partial sums of <V_k, w> = sum_i conj(V_k[i]) w[i] for the NK vectors k0 .. k0+NK-1
// and, with SELF, of ||w||^2 (slot k0+NK, real) over a grid-stride range of complex
// elements: partials[block][slot] (complex), fixed order.  All loads of an element
// are issued together.
template <int NK, bool SELF>
__global__ void __launch_bounds__(256) cn_dots_kernel(const double* V, size_t vstride, int k0, const double* w,
                                                      size_t ncplx, double* partials, int ldp) {
    constexpr int NS = NK + (SELF ? 1 : 0);
    double ar[NS], ai[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) ar[k] = ai[k] = 0.0;
    const double2* W = reinterpret_cast<const double2*>(w);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        const double2 x = W[i];
        double2 y[NK > 0 ? NK : 1];
#pragma unroll
        for (int k = 0; k < NK; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)(k0 + k) * vstride)[i];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            ar[k] += y[k].x * x.x + y[k].y * x.y;
            ai[k] += y[k].x * x.y - y[k].y * x.x;
        }
        if constexpr (SELF) ar[NK] += x.x * x.x + x.y * x.y;
    }
    block_sum_store<NS>(ar, ai, partials + 2 * ((size_t)blockIdx.x * ldp + k0));
}

// The first Gram-Schmidt update fused with the second pass's dots:
// w <- w - sum_{k<NK} coef_k V_k in place, and partial sums of <V_k, w> (slots 0..NK-1)
// and ||w||^2 (slot NK) of the updated w, as cn_dots_kernel writes them.
template <int NK>
__global__ void __launch_bounds__(256) cn_axpy_dots_kernel(const double* V, size_t vstride, const double* coef,
                                                           double* w, size_t ncplx, double* partials, int ldp) {
    constexpr int NS = NK + 1;
    double ar[NS], ai[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) ar[k] = ai[k] = 0.0;
    double2* W = reinterpret_cast<double2*>(w);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        double2 x = W[i];
        double2 y[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)k * vstride)[i];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const double cr = coef[2 * k], ci = coef[2 * k + 1];
            x.x -= cr * y[k].x - ci * y[k].y;
            x.y -= cr * y[k].y + ci * y[k].x;
        }
        W[i] = x;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            ar[k] += y[k].x * x.x + y[k].y * x.y;
            ai[k] += y[k].x * x.y - y[k].y * x.x;
        }
        ar[NK] += x.x * x.x + x.y * x.y;
    }
    block_sum_store<NS>(ar, ai, partials + 2 * (size_t)blockIdx.x * ldp);
}

// out <- alpha (w - sign sum_{k<nk} coef_k V_k), nk = 8 nfull + NKR, coef complex on the
// device (out may be w).  alpha = 1, or with NORM the reciprocal norm of the result:
// coef[nk] holds ||w||^2 and the V_k are orthonormal, so the result's squared norm is
// ||w||^2 - sum |coef_k|^2 (clamped at 0; alpha = 0 then); block 0 stores it to norm_out.
template <int NKR, bool NORM>
__global__ void __launch_bounds__(256) cn_axpy_kernel(const double* V, size_t vstride, int nfull, const double* coef,
                                                      const double* w, double* out, size_t ncplx, double sign,
                                                      double* norm_out) {
    double alpha = 1.0;
    if constexpr (NORM) {
        const int nk = 8 * nfull + NKR;
        double n2 = coef[2 * nk];
        for (int k = 0; k < nk; ++k) n2 -= coef[2 * k] * coef[2 * k] + coef[2 * k + 1] * coef[2 * k + 1];
        n2 = n2 > 0.0 ? n2 : 0.0;
        alpha = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) norm_out[0] = n2;
    }
    const double2* Wi = reinterpret_cast<const double2*>(w);
    double2* O = reinterpret_cast<double2*>(out);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        double2 x = Wi[i];
        for (int c8 = 0; c8 < nfull; ++c8) {
            double2 y[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)(8 * c8 + k) * vstride)[i];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double cr = coef[2 * (8 * c8 + k)], ci = coef[2 * (8 * c8 + k) + 1];
                x.x -= sign * (cr * y[k].x - ci * y[k].y);
                x.y -= sign * (cr * y[k].y + ci * y[k].x);
            }
        }
        double2 y[NKR > 0 ? NKR : 1];
#pragma unroll
        for (int k = 0; k < NKR; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)(8 * nfull + k) * vstride)[i];
#pragma unroll
        for (int k = 0; k < NKR; ++k) {
            const double cr = coef[2 * (8 * nfull + k)], ci = coef[2 * (8 * nfull + k) + 1];
            x.x -= sign * (cr * y[k].x - ci * y[k].y);
            x.y -= sign * (cr * y[k].y + ci * y[k].x);
        }
        if constexpr (NORM) {
            x.x *= alpha;
            x.y *= alpha;
        }
        O[i] = x;
    }
}

// out[k] = sum over blocks of partials[block][k] (complex), one workgroup per slot, fixed order.
__global__ void __launch_bounds__(256) cn_reduce_kernel(const double* partials, int nblocks, int ldp, double* out) {
    const int k = blockIdx.x;
    double r = 0, i = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        r += partials[2 * ((size_t)b * ldp + k)];
        i += partials[2 * ((size_t)b * ldp + k) + 1];
    }
    __shared__ double sr[256], si[256];
    sr[threadIdx.x] = r;
    si[threadIdx.x] = i;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sr[threadIdx.x] += sr[threadIdx.x + off];
            si[threadIdx.x] += si[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * k] = sr[0];
        out[2 * k + 1] = si[0];
    }
}

// y <- alpha x (alpha real), or y <- x when alpha == 1.
__global__ void cn_scale_kernel(const double* x, double* y, size_t n, double alpha) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = alpha * x[i];
}

// y <- x - y  (residual r = b - A x0 with y = A x0)
__global__ void cn_sub_kernel(const double* x, double* y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = x[i] - y[i];
}

// ---------------------------------------------------------------- launchers

template <bool COLS>
static hipError_t launch_apply_dir(int n, int nlines, const CnApplyParams& p, hipStream_t s) {
    const int L = cn_lines(n, COLS);
    const dim3 grid((nlines + L - 1) / L), block((n / cn_radix(n, COLS)) * L);
    switch (n) {
        case 16: hipLaunchKernelGGL((cn_apply_kernel<16, COLS>), grid, block, 0, s, p); break;
        case 32: hipLaunchKernelGGL((cn_apply_kernel<32, COLS>), grid, block, 0, s, p); break;
        case 64: hipLaunchKernelGGL((cn_apply_kernel<64, COLS>), grid, block, 0, s, p); break;
        case 128: hipLaunchKernelGGL((cn_apply_kernel<128, COLS>), grid, block, 0, s, p); break;
        case 256: hipLaunchKernelGGL((cn_apply_kernel<256, COLS>), grid, block, 0, s, p); break;
        case 512: hipLaunchKernelGGL((cn_apply_kernel<512, COLS>), grid, block, 0, s, p); break;
        case 1024: hipLaunchKernelGGL((cn_apply_kernel<1024, COLS>), grid, block, 0, s, p); break;
        case 2048: hipLaunchKernelGGL((cn_apply_kernel<2048, COLS>), grid, block, 0, s, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cn_apply(int dir, int n, int nlines, const CnApplyParams& p, hipStream_t s) {
    return dir == 0 ? launch_apply_dir<false>(n, nlines, p, s) : launch_apply_dir<true>(n, nlines, p, s);
}

hipError_t launch_cn_exp(double* psi, const double* E, double e0r, double e0i, size_t npts, int times, hipStream_t s) {
    hipLaunchKernelGGL(cn_exp_kernel, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, psi, E,
                       make_double2(e0r, e0i), npts, times);
    return hipGetLastError();
}

template <bool SELF>
static void launch_dots_chunk(int nk, const double* V, size_t vstride, int k0, const double* w, size_t ncplx,
                              double* partials, int nblocks, int ldp, hipStream_t s) {
#define DIRAC_CN_DOTS(NK)                                                                                    \
    case NK:                                                                                                 \
        hipLaunchKernelGGL((cn_dots_kernel<NK, SELF>), dim3(nblocks), dim3(256), 0, s, V, vstride, k0, w,   \
                           ncplx, partials, ldp);                                                           \
        break;
    if constexpr (SELF) {
        if (nk == 0) {
            hipLaunchKernelGGL((cn_dots_kernel<0, true>), dim3(nblocks), dim3(256), 0, s, V, vstride, k0, w, ncplx,
                               partials, ldp);
            return;
        }
    }
    switch (nk) {
        DIRAC_CN_DOTS(1) DIRAC_CN_DOTS(2) DIRAC_CN_DOTS(3) DIRAC_CN_DOTS(4)
        DIRAC_CN_DOTS(5) DIRAC_CN_DOTS(6) DIRAC_CN_DOTS(7) DIRAC_CN_DOTS(8)
        default: break;
    }
#undef DIRAC_CN_DOTS
}

hipError_t launch_cn_dots(const double* V, size_t vstride, int nk, bool self, const double* w, size_t ncplx,
                          double* partials, int nblocks, int ldp, double* out, hipStream_t s) {
    const int slots = nk + (self ? 1 : 0);
    if (slots < 1 || slots > ldp || nblocks < 1) return hipErrorInvalidValue;
    int k0 = 0;
    for (; nk - k0 > 8; k0 += 8) launch_dots_chunk<false>(8, V, vstride, k0, w, ncplx, partials, nblocks, ldp, s);
    if (self)
        launch_dots_chunk<true>(nk - k0, V, vstride, k0, w, ncplx, partials, nblocks, ldp, s);
    else
        launch_dots_chunk<false>(nk - k0, V, vstride, k0, w, ncplx, partials, nblocks, ldp, s);
    hipLaunchKernelGGL(cn_reduce_kernel, dim3(slots), dim3(256), 0, s, (const double*)partials, nblocks, ldp, out);
    return hipGetLastError();
}

hipError_t launch_cn_axpy_dots(const double* V, size_t vstride, int nk, const double* coef, double* w, size_t ncplx,
                               double* partials, int nblocks, int ldp, double* out, hipStream_t s) {
    if (nk < 1 || nk > kCnFusedMax || nk + 1 > ldp || nblocks < 1) return hipErrorInvalidValue;
#define DIRAC_CN_AXD(NK)                                                                                     \
    case NK:                                                                                                 \
        hipLaunchKernelGGL((cn_axpy_dots_kernel<NK>), dim3(nblocks), dim3(256), 0, s, V, vstride, coef, w,  \
                           ncplx, partials, ldp);                                                           \
        break;
    switch (nk) {
        DIRAC_CN_AXD(1) DIRAC_CN_AXD(2) DIRAC_CN_AXD(3) DIRAC_CN_AXD(4)
        DIRAC_CN_AXD(5) DIRAC_CN_AXD(6) DIRAC_CN_AXD(7) DIRAC_CN_AXD(8)
        default: break;
    }
#undef DIRAC_CN_AXD
    hipLaunchKernelGGL(cn_reduce_kernel, dim3(nk + 1), dim3(256), 0, s, (const double*)partials, nblocks, ldp, out);
    return hipGetLastError();
}

template <bool NORM>
static hipError_t launch_axpy_t(const double* V, size_t vstride, int nk, const double* coef, const double* w,
                                double* out, size_t ncplx, double sign, double* norm_out, hipStream_t s) {
    if (nk < 0 || (NORM && !norm_out)) return hipErrorInvalidValue;
    const int nfull = nk / 8;
#define DIRAC_CN_AXPY(R)                                                                                     \
    case R:                                                                                                  \
        hipLaunchKernelGGL((cn_axpy_kernel<R, NORM>), dim3(1024), dim3(256), 0, s, V, vstride, nfull, coef,  \
                           w, out, ncplx, sign, norm_out);                                                  \
        break;
    switch (nk % 8) {
        DIRAC_CN_AXPY(0) DIRAC_CN_AXPY(1) DIRAC_CN_AXPY(2) DIRAC_CN_AXPY(3)
        DIRAC_CN_AXPY(4) DIRAC_CN_AXPY(5) DIRAC_CN_AXPY(6) DIRAC_CN_AXPY(7)
        default: break;
    }
#undef DIRAC_CN_AXPY
    return hipGetLastError();
}

hipError_t launch_cn_axpy(const double* V, size_t vstride, int nk, const double* coef, const double* w, double* out,
                          size_t ncplx, double sign, hipStream_t s) {
    return launch_axpy_t<false>(V, vstride, nk, coef, w, out, ncplx, sign, nullptr, s);
}

hipError_t launch_cn_axpy_normalise(const double* V, size_t vstride, int nk, const double* coef, const double* w,
                                    double* out, size_t ncplx, double* norm2_out, hipStream_t s) {
    return launch_axpy_t<true>(V, vstride, nk, coef, w, out, ncplx, 1.0, norm2_out, s);
}

hipError_t launch_cn_scale(const double* x, double* y, size_t n, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(cn_scale_kernel, dim3(1024), dim3(256), 0, s, x, y, n, alpha);
    return hipGetLastError();
}

hipError_t launch_cn_sub(const double* x, double* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(cn_sub_kernel, dim3(1024), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace dirac
