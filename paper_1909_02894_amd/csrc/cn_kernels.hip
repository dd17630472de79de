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

__host__ __device__ constexpr int cn_radix(int n) { return n <= 64 ? 4 : 8; }
__host__ __device__ constexpr int cn_lines(int n) { return (n / cn_radix(n)) >= 256 ? 1 : 256 / (n / cn_radix(n)); }

// out = in + s h c b_x sigma_x [[d_x]] in          (x pass, rows)
// out = out + s h c b_y sigma_y [[d_y]] in         (y pass, columns)
template <int N, bool COLS>
__global__ void __launch_bounds__((N / cn_radix(N)) * cn_lines(N)) cn_apply_kernel(CnApplyParams p) {
    using T = double;
    constexpr int R = cn_radix(N), L = cn_lines(N);
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

// Partial sums of sum_i conj(V_k[i]) w[i] for k in [k0, k0 + 8) over a grid-stride
// range of complex elements; partials[block][k] (complex), fixed order.
__global__ void __launch_bounds__(256) cn_multidot_kernel(const double* V, size_t vstride, int k0, int nk,
                                                          const double* w, size_t ncplx, double* partials, int ldp) {
    double ar[8] = {0, 0, 0, 0, 0, 0, 0, 0}, ai[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        const double2 x = reinterpret_cast<const double2*>(w)[i];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < nk) {
                const double2 y = reinterpret_cast<const double2*>(V + (size_t)(k0 + k) * vstride)[i];
                ar[k] += y.x * x.x + y.y * x.y;
                ai[k] += y.x * x.y - y.y * x.x;
            }
        }
    }
    __shared__ double sr[256][8], si[256][8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { sr[threadIdx.x][k] = ar[k]; si[threadIdx.x][k] = ai[k]; }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                sr[threadIdx.x][k] += sr[threadIdx.x + off][k];
                si[threadIdx.x][k] += si[threadIdx.x + off][k];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < (unsigned)nk) {
        partials[2 * ((size_t)blockIdx.x * ldp + k0 + threadIdx.x)] = sr[0][threadIdx.x];
        partials[2 * ((size_t)blockIdx.x * ldp + k0 + threadIdx.x) + 1] = si[0][threadIdx.x];
    }
}

// out[k] = sum over blocks of partials[block][k], k < nk: one workgroup per k,
// a fixed per-thread order over the blocks and a fixed tree, so the result does
// not depend on timing.
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

// w <- w - sign sum_k coef[k] V_k (coef complex, read from device memory), k < nk.
__global__ void __launch_bounds__(256) cn_multiaxpy_kernel(const double* V, size_t vstride, int nk,
                                                           const double* coef, double* w, size_t ncplx, double sign) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        double2 x = reinterpret_cast<double2*>(w)[i];
        for (int k = 0; k < nk; ++k) {
            const double2 y = reinterpret_cast<const double2*>(V + (size_t)k * vstride)[i];
            const double cr = coef[2 * k], ci = coef[2 * k + 1];
            x.x -= sign * (cr * y.x - ci * y.y);
            x.y -= sign * (cr * y.y + ci * y.x);
        }
        reinterpret_cast<double2*>(w)[i] = x;
    }
}

// y <- alpha x (alpha real), or y <- x when alpha == 1.
__global__ void cn_scale_kernel(const double* x, double* y, size_t n, double alpha) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = alpha * x[i];
}

// y <- x / sqrt(norm2[0]): normalisation by a norm the device computed
__global__ void cn_scale_by_norm_kernel(const double* x, double* y, size_t n, const double* norm2) {
    const double alpha = 1.0 / sqrt(norm2[0]);
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
    const int L = cn_lines(n);
    const dim3 grid((nlines + L - 1) / L), block((n / cn_radix(n)) * L);
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

hipError_t launch_cn_dots(const double* V, size_t vstride, int nk, const double* w, size_t ncplx, double* partials,
                          int nblocks, int ldp, double* out, hipStream_t s) {
    for (int k0 = 0; k0 < nk; k0 += 8) {
        hipLaunchKernelGGL(cn_multidot_kernel, dim3(nblocks), dim3(256), 0, s, V, vstride, k0,
                           nk - k0 < 8 ? nk - k0 : 8, w, ncplx, partials, ldp);
    }
    hipLaunchKernelGGL(cn_reduce_kernel, dim3(nk), dim3(256), 0, s, (const double*)partials, nblocks, ldp, out);
    return hipGetLastError();
}

hipError_t launch_cn_axpy(const double* V, size_t vstride, int nk, const double* coef, double* w, size_t ncplx,
                          double sign, hipStream_t s) {
    hipLaunchKernelGGL(cn_multiaxpy_kernel, dim3(1024), dim3(256), 0, s, V, vstride, nk, coef, w, ncplx, sign);
    return hipGetLastError();
}

hipError_t launch_cn_scale(const double* x, double* y, size_t n, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(cn_scale_kernel, dim3(1024), dim3(256), 0, s, x, y, n, alpha);
    return hipGetLastError();
}

hipError_t launch_cn_scale_by_norm(const double* x, double* y, size_t n, const double* norm2, hipStream_t s) {
    hipLaunchKernelGGL(cn_scale_by_norm_kernel, dim3(1024), dim3(256), 0, s, x, y, n, norm2);
    return hipGetLastError();
}

hipError_t launch_cn_sub(const double* x, double* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(cn_sub_kernel, dim3(1024), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace dirac
