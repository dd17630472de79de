// setup_kernels.hip -- FP64 table generation on the device (once per solve),
// state conversions, and the fixed-order final reduction of the observables.
#include <hip/hip_runtime.h>
#include <math.h>
#include "setup_kernels.hpp"

namespace dirac {

// 1/S at grid index k of an axis (Sec. 3): S = 1 + cos(theta) Sigma~ (theta with
// sin(theta) = 0 only; complex stretches are rejected on the host).  The layer is
// the width grid points next to the seam x = +-a; s = |x_k| - L = -d h with
// d = min(k, n - k) whole grid steps.  Types I..VI; singular types give 0 at d = 0.
__device__ double pml_inv_s(int k, int n, double a, int width, int type, double s0, double ctheta) {
    if (width <= 0) return 1.0;
    const int d = k < n - k ? k : n - k;
    if (d > width) return 1.0;
    const double h = 2.0 * a / n;
    const double delta = width * h;
    const double s = -d * h;
    double sig;
    if (type == 1) {
        sig = s0 * (s + delta) * (s + delta);
    } else if (type == 2) {
        sig = s0 * (s + delta) * (s + delta) * (s + delta);
    } else {
        if (d == 0) return 0.0;
        if (type == 3) sig = -s0 / s;
        else if (type == 4) sig = s0 / (s * s);
        else if (type == 5) sig = -s0 / s - s0 / delta;
        else sig = s0 / (s * s) - s0 / (delta * delta);
    }
    return 1.0 / (1.0 + ctheta * sig);
}

template <typename T>
__device__ void put(void* base, size_t i, double v) { static_cast<T*>(base)[i] = (T)v; }

__global__ void setup_axis_kernel(SetupAxisParams p) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n) return;
    const int n = p.n;
    const double invs = pml_inv_s(k, n, p.a, p.pml_width, p.pml_type, p.sigma0, p.ctheta);
    const int pp = k < n / 2 ? k : k - n;               // Nyquist keeps p = -n/2
    const double xi = pp * M_PI / p.a;
    const double th = p.c * p.dt * xi;
    const double g = p.k_printed ? 1.0 - th * th : 1.0;
    const double cs = g * cos(th), sn = g * sin(th);
    double ts, tc;
    sincospi(2.0 * k / n, &ts, &tc);                    // exp(-2 pi i k / n) = (tc, -ts)
    const double inv_n = 1.0 / n;
    if (p.fp32) {
        put<float>(p.inv_s, k, invs);
        put<float>(p.K, 2 * k, cs * inv_n);
        put<float>(p.K, 2 * k + 1, sn * inv_n);
        put<float>(p.D, k, xi * inv_n);
        put<float>(p.tw, 2 * k, tc);
        put<float>(p.tw, 2 * k + 1, -ts);
    } else {
        put<double>(p.inv_s, k, invs);
        put<double>(p.K, 2 * k, cs * inv_n);
        put<double>(p.K, 2 * k + 1, sn * inv_n);
        put<double>(p.D, k, xi * inv_n);
        put<double>(p.tw, 2 * k, tc);
        put<double>(p.tw, 2 * k + 1, -ts);
    }
}

// Metric fields at (x, y): Phi, Psi, grad Phi, grad Psi.
struct Fields { double phi, psi, phix, phiy, psix, psiy; };

__device__ Fields metric_at(const SetupPointParams& p, double x, double y, size_t q) {
    Fields f{0, 0, 0, 0, 0, 0};
    const double r2 = x * x + y * y;
    if (p.kind == 2) {                 // Numerical Experiment 3
        f.phi = exp(-0.01 * r2);
        f.psi = exp(-0.005 * r2);
        f.phix = -0.02 * x * f.phi;
        f.phiy = -0.02 * y * f.phi;
        f.psix = -0.01 * x * f.psi;
        f.psiy = -0.01 * y * f.psi;
    } else if (p.kind == 1) {          // static sheet over h = A exp(-r^2/s^2)
        const double s2 = p.bump_s * p.bump_s;
        const double h = p.bump_A * exp(-r2 / s2);
        const double G = 4.0 * r2 * h * h / (s2 * s2);                 // |grad h|^2
        const double dG = 8.0 * h * h / (s2 * s2) * (1.0 - 2.0 * r2 / s2);  // grad G = dG (x, y)
        f.psi = 0.25 * log1p(G);
        f.psix = 0.25 * dG * x / (1.0 + G);
        f.psiy = 0.25 * dG * y / (1.0 + G);
    } else if (p.kind == 3) {          // caller-given planes
        const size_t N = (size_t)p.n1 * p.n2;
        f.phi = p.fields[q];
        f.psi = p.fields[N + q];
        f.phix = p.fields[2 * N + q];
        f.phiy = p.fields[3 * N + q];
        f.psix = p.fields[4 * N + q];
        f.psiy = p.fields[5 * N + q];
    }
    return f;
}

// Per point: a = e^{Phi - Psi}; the Step-1 exponential E = exp(u . sigma),
// u = (-(dt/4) c a chi_x, -(dt/4) c a chi_y, -i (dt/2) m c^2 e^Phi), in closed
// form C I + D (u . sigma) (C, D real: cosh/sinh(r)/r for u.u = r^2 >= 0,
// cos/sin(r)/r for u.u = -r^2 < 0, series for |u.u| < 1e-8); observable
// planes; and per-workgroup bounds of the blend coefficients b_x = a/S^1,
// b_y = a/S^2 plus a count of non-finite field values.
__global__ void setup_point_kernel(SetupPointParams p) {
    const size_t N = (size_t)p.n1 * p.n2;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double bmin = 1e300, bmax = -1e300, bad = 0.0;
    if (q < N) {
        const int i = (int)(q % p.n1), jy = (int)(q / p.n1);
        const double x = -p.a1 + i * (2.0 * p.a1 / p.n1);
        const double y = -p.a2 + jy * (2.0 * p.a2 / p.n2);
        const Fields f = metric_at(p, x, y, q);
        double chix = 0, chiy = 0, chi = 0;
        if (p.spin == 1) { chix = f.phix; chiy = f.phiy; chi = f.phi; }
        else if (p.spin == 2) { chix = f.phix + f.psix; chiy = f.phiy + f.psiy; chi = f.phi + f.psi; }
        const double a = exp(f.phi - f.psi);
        const double ux = -(p.dt / 4.0) * p.c * a * chix;
        const double uy = -(p.dt / 4.0) * p.c * a * chiy;
        const double wz = (p.dt / 2.0) * p.m * p.c * p.c * exp(f.phi);   // u_z = -i wz
        const double s2 = ux * ux + uy * uy - wz * wz;
        double C, D;
        if (fabs(s2) < 1e-8) {
            C = 1.0 + s2 / 2.0 + s2 * s2 / 24.0;
            D = 1.0 + s2 / 6.0 + s2 * s2 / 120.0;
        } else if (s2 >= 0) {
            const double r = sqrt(s2);
            C = cosh(r);
            D = sinh(r) / r;
        } else {
            const double r = sqrt(-s2);
            C = cos(r);
            D = sin(r) / r;
        }
        // e0 = C + D u_z = C - i D wz ; e1 = D (u_x - i u_y)
        const double e0r = C, e0i = -D * wz, e1r = D * ux, e1i = -D * uy;
        if (p.a_out) {
            if (p.fp32) put<float>(p.a_out, q, a); else put<double>(p.a_out, q, a);
        }
        double emv = 0.0, emx = 0.0, emy = 0.0;
        if (p.em_planes) {
            emv = p.em_planes[q];
            emx = p.em_planes[N + q];
            emy = p.em_planes[2 * N + q];
        }
        if (p.em_out) {
            // record for the in-kernel exponential with potentials (e = charge)
            const double rec[8] = {ux, uy, wz, (p.dt / 2.0) * p.charge * p.c * a * emx,
                                   (p.dt / 2.0) * p.charge * p.c * a * emy, (p.dt / 2.0) * p.charge * emv, a, 0.0};
            for (int k = 0; k < 8; ++k) {
                if (p.fp32) put<float>(p.em_out, 8 * q + k, rec[k]); else put<double>(p.em_out, 8 * q + k, rec[k]);
            }
        }
        if (p.obs_em) {
            p.obs_em[q] = p.charge * p.c * a * emx;
            p.obs_em[N + q] = p.charge * p.c * a * emy;
            p.obs_em[2 * N + q] = p.charge * emv;
        }
        if (p.da_out) {
            const double dax = a * (f.phix - f.psix), day = a * (f.phiy - f.psiy);
            if (p.fp32) { put<float>(p.da_out, 2 * q, dax); put<float>(p.da_out, 2 * q + 1, day); }
            else { put<double>(p.da_out, 2 * q, dax); put<double>(p.da_out, 2 * q + 1, day); }
        }
        if (p.E_out) {
            // with potentials the exponentials come from the record: the table holds
            // the identity, which the plain row kernel then applies (exactly) behind
            // a potentials pass
            const bool id = p.em_out != nullptr;
            const double t0r = id ? 1.0 : e0r, t0i = id ? 0.0 : e0i, t1r = id ? 0.0 : e1r, t1i = id ? 0.0 : e1i;
            if (p.fp32) {
                put<float>(p.E_out, 4 * q, t0r); put<float>(p.E_out, 4 * q + 1, t0i);
                put<float>(p.E_out, 4 * q + 2, t1r); put<float>(p.E_out, 4 * q + 3, t1i);
            } else {
                put<double>(p.E_out, 4 * q, t0r); put<double>(p.E_out, 4 * q + 1, t0i);
                put<double>(p.E_out, 4 * q + 2, t1r); put<double>(p.E_out, 4 * q + 3, t1i);
            }
        }
        p.obs[q] = exp(chi - f.phi + f.psi);             // weight w
        p.obs[N + q] = p.c * a;                          // c a
        p.obs[2 * N + q] = 0.5 * p.c * a * chix;         // gx
        p.obs[3 * N + q] = 0.5 * p.c * a * chiy;         // gy
        p.obs[4 * N + q] = exp(f.phi) * p.m * p.c * p.c; // V
        const double bx = a * pml_inv_s(i, p.n1, p.a1, p.pml_width, p.pml_type, p.sigma0, p.ctheta);
        const double by = a * pml_inv_s(jy, p.n2, p.a2, p.pml_width, p.pml_type, p.sigma0, p.ctheta);
        bmin = fmin(bx, by);
        bmax = fmax(bx, by);
        const bool fin = isfinite(f.phi) && isfinite(f.psi) && isfinite(f.phix) && isfinite(f.phiy)
                         && isfinite(f.psix) && isfinite(f.psiy) && isfinite(bx) && isfinite(by)
                         && isfinite(e0r) && isfinite(e0i) && isfinite(e1r) && isfinite(e1i)
                         && isfinite(emv) && isfinite(emx) && isfinite(emy);
        bad = fin ? 0.0 : 1.0;
    }
    __shared__ double smin[256], smax[256], sbad[256];
    smin[threadIdx.x] = bmin;
    smax[threadIdx.x] = bmax;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
            sbad[threadIdx.x] += sbad[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        p.partial[3 * blockIdx.x] = smin[0];
        p.partial[3 * blockIdx.x + 1] = smax[0];
        p.partial[3 * blockIdx.x + 2] = sbad[0];
    }
}

// Fold the setup partials into 3 doubles (min b, max b, bad count); one workgroup.
__global__ void setup_fold_kernel(const double* part, int nblocks, double* out) {
    __shared__ double smin[256], smax[256], sbad[256];
    double mn = 1e300, mx = -1e300, bd = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        mn = fmin(mn, part[3 * b]);
        mx = fmax(mx, part[3 * b + 1]);
        bd += part[3 * b + 2];
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bd;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
            sbad[threadIdx.x] += sbad[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = smin[0]; out[1] = smax[0]; out[2] = sbad[0]; }
}

// complex128 <-> state conversions (count = number of reals)
__global__ void c128_to_f32_kernel(const double* src, float* dst, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}
__global__ void f32_to_c128_kernel(const float* src, double* dst, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

// Fixed-order sum of nparts 8-double partial records: thread t adds records
// t, t + 256, ... in order, then a fixed tree.  One workgroup of 256 threads.
__global__ void reduce_partials_kernel(const double* part, int nparts, double* out) {
    __shared__ double red[256][8];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += 256) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += part[8 * (size_t)b + k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
#pragma unroll
            for (int k = 0; k < 8; ++k) red[threadIdx.x][k] += red[threadIdx.x + off][k];
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = red[0][threadIdx.x];
}

}  // namespace dirac

namespace dirac {

// 32 x 32 tiles through LDS (one padding column against bank conflicts):
// coalesced reads of in's rows and writes of out's rows.
template <typename T>
__global__ void transpose_kernel(const T* in, T* out, int n1, int n2) {
    __shared__ T tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int k = 0; k < 32; k += 8) {
        const int r = r0 + ty + k, c = c0 + tx;
        if (r < n2 && c < n1) tile[ty + k][tx] = in[(size_t)r * n1 + c];
    }
    __syncthreads();
    for (int k = 0; k < 32; k += 8) {
        const int c = c0 + ty + k, r = r0 + tx;
        if (c < n1 && r < n2) out[(size_t)c * n2 + r] = tile[tx][ty + k];
    }
}

hipError_t launch_transpose(const void* in, void* out, int n1, int n2, int elem, hipStream_t s) {
    const dim3 grid((unsigned)((n1 + 31) / 32), (unsigned)((n2 + 31) / 32)), block(32, 8);
    if (elem == 8)
        hipLaunchKernelGGL(transpose_kernel<double>, grid, block, 0, s, static_cast<const double*>(in),
                           static_cast<double*>(out), n1, n2);
    else if (elem == 4)
        hipLaunchKernelGGL(transpose_kernel<float>, grid, block, 0, s, static_cast<const float*>(in),
                           static_cast<float*>(out), n1, n2);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_setup_axis(const SetupAxisParams& p, hipStream_t s) {
    hipLaunchKernelGGL(setup_axis_kernel, dim3((p.n + 255) / 256), dim3(256), 0, s, p);
    return hipGetLastError();
}
hipError_t launch_setup_points(const SetupPointParams& p, double* fold_out, hipStream_t s) {
    const size_t N = (size_t)p.n1 * p.n2;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(setup_point_kernel, dim3(nb), dim3(256), 0, s, p);
    hipLaunchKernelGGL(setup_fold_kernel, dim3(1), dim3(256), 0, s, (const double*)p.partial, nb, fold_out);
    return hipGetLastError();
}
hipError_t launch_c128_to_f32(const double* src, float* dst, size_t count, hipStream_t s) {
    hipLaunchKernelGGL(c128_to_f32_kernel, dim3(1024), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}
hipError_t launch_f32_to_c128(const float* src, double* dst, size_t count, hipStream_t s) {
    hipLaunchKernelGGL(f32_to_c128_kernel, dim3(1024), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}
hipError_t launch_reduce_partials(const double* part, int nparts, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, part, nparts, out);
    return hipGetLastError();
}

}  // namespace dirac
