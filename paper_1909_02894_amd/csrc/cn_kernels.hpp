// cn_kernels.hpp -- parameters and host launchers of the Scheme I (Crank-Nicolson
// + GMRES) kernels.  All vectors are FP64 states: 4 doubles per grid point.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "fft_line.hpp"

namespace dirac {

struct CnApplyParams {
    const double* in;        // vector the transport operator acts on
    double* out;             // x pass: out = in + term; y pass: out += term
    const double* a;         // a(x) per point, or null (a = 1)
    const double* inv_s;     // 1/S along the line direction (ones without a layer)
    const double* D;         // xi / n along the line direction
    const cpx<double>* tw;   // twiddles
    int n1;                  // points per row
    int nlines;
    double scale;            // s (dt / 2) c, s = +1 for G, -1 for G~
};

constexpr int kCnDotBlocks = 512;

hipError_t launch_cn_apply(int dir, int n, int nlines, const CnApplyParams& p, hipStream_t s);
hipError_t launch_cn_exp(double* psi, const double* E, double e0r, double e0i, size_t npts, int times, hipStream_t s);
hipError_t launch_cn_dots(const double* V, size_t vstride, int nk, const double* w, size_t ncplx, double* partials,
                          int nblocks, int ldp, double* out, hipStream_t s);
hipError_t launch_cn_axpy(const double* V, size_t vstride, int nk, const double* coef, double* w, size_t ncplx,
                          double sign, hipStream_t s);
hipError_t launch_cn_scale(const double* x, double* y, size_t n, double alpha, hipStream_t s);
hipError_t launch_cn_scale_by_norm(const double* x, double* y, size_t n, const double* norm2, hipStream_t s);
hipError_t launch_cn_sub(const double* x, double* y, size_t n, hipStream_t s);

}  // namespace dirac
