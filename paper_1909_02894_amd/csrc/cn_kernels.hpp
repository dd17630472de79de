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
constexpr int kCnFusedMax = 8;      // basis vectors the fused update + dots kernel holds in registers

hipError_t launch_cn_apply(int dir, int n, int nlines, const CnApplyParams& p, hipStream_t s);
hipError_t launch_cn_exp(double* psi, const double* E, double e0r, double e0i, size_t npts, int times, hipStream_t s);
// out[k] = <V_k, w> for k < nk, and out[nk] = ||w||^2 when self (complex slots, fixed-order sums);
// partials: nblocks x ldp complex scratch.
hipError_t launch_cn_dots(const double* V, size_t vstride, int nk, bool self, const double* w, size_t ncplx,
                          double* partials, int nblocks, int ldp, double* out, hipStream_t s);
// w <- w - sum_{k<nk} coef_k V_k, then out[k] = <V_k, w> (k < nk), out[nk] = ||w||^2;
// nk <= kCnFusedMax.
hipError_t launch_cn_axpy_dots(const double* V, size_t vstride, int nk, const double* coef, double* w, size_t ncplx,
                               double* partials, int nblocks, int ldp, double* out, hipStream_t s);
// out <- w - sign sum_{k<nk} coef_k V_k (out may be w)
hipError_t launch_cn_axpy(const double* V, size_t vstride, int nk, const double* coef, const double* w, double* out,
                          size_t ncplx, double sign, hipStream_t s);
// out <- (w - sum_{k<nk} coef_k V_k) / norm with norm^2 = coef[nk] - sum |coef_k|^2 (coef[nk] = ||w||^2,
// V_k orthonormal), stored to norm2_out[0]
hipError_t launch_cn_axpy_normalise(const double* V, size_t vstride, int nk, const double* coef, const double* w,
                                    double* out, size_t ncplx, double* norm2_out, hipStream_t s);
hipError_t launch_cn_scale(const double* x, double* y, size_t n, double alpha, hipStream_t s);
hipError_t launch_cn_sub(const double* x, double* y, size_t n, hipStream_t s);

}  // namespace dirac
