// cn_kernels.hpp -- parameters and host launchers of the Scheme I (Crank-Nicolson
// + GMRES) kernels.  All vectors are FP64 states: 4 doubles per grid point.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "fft_line.hpp"

namespace dirac {

constexpr int kCnDotBlocks = 512;     // workgroups of the reduction kernels
constexpr int kCnMaxRestart = 63;     // Krylov vectors per cycle (validated on creation)
constexpr int kCnChunk = 8;           // basis vectors one reduction launch handles

// Device-resident state of the GMRES solve of one step: the Hessenberg
// least-squares problem after Givens rotations (R, cs, sn, g), the cycle's
// counters and the stopping rule.  Written by the single-workgroup finish
// kernels (and the init kernel) and read by the other kernels.
struct CnCtrl {
    // head (CnHead): the fields the host reads after a cycle
    double beta;          // norm of the current cycle's starting residual
    double bnorm;         // ||rhs||
    double tol;           // rtol ||rhs||
    double res2;          // squared norm of the last explicit residual
    double hn;            // norm of the newest Arnoldi vector before normalisation
    double hdt;           // dt / 2 (G = I + hdt A)
    double rtol;
    double pad0;
    int k;                // columns of the current cycle
    int done;             // the cycle has ended (converged estimate, breakdown, full or out of iterations)
    int used;             // iterations of this step
    int max_iter;
    int m;                // restart length
    int state;            // 0 iterating, 1 restart needed, 2 converged, 3 out of iterations
    int nonfinite;
    int pad1;
    // the least-squares problem and the rest
    unsigned pad2[4];
    double cs[kCnMaxRestart + 1];
    double sn[2 * (kCnMaxRestart + 1)];        // complex
    double g[2 * (kCnMaxRestart + 2)];         // complex
    double R[2 * (kCnMaxRestart + 1) * (kCnMaxRestart + 1)];   // complex, R(i, j) at 2 (j (m_max + 1) + i)
};

// The first 96 bytes of CnCtrl, which the host reads after a cycle.
struct CnHead {
    double beta, bnorm, tol, res2, hn, hdt, rtol, pad0;
    int k, done, used, max_iter, m, state, nonfinite, pad1;
};
static_assert(sizeof(CnHead) == 96 && offsetof(CnCtrl, pad2) == sizeof(CnHead), "CnCtrl head layout");

// Arnoldi coefficient record of iteration j: H_A(0..j, j) and the subdiagonal
// entry H_A(j + 1, j) = hn_j in slot j + 1 (kCnMaxRestart + 1 complex slots).
constexpr size_t kCnRecDoubles = 2 * (kCnMaxRestart + 1);

// out_x = base + f c b_x sigma_x [[d_x]] v    (rows)
// out_y =        f c b_y sigma_y [[d_y]] v    (columns)
// with v = in, or in / in_norm[0] when in_norm is given (the x pass then also
// stores that v to vout), and base = 0, v or (b - v) by `base`.  G v = out_x +
// out_y for base = v, f = dt/2; the A of the Arnoldi process for base = 0, f = 1.
struct CnApplyParams {
    const double* in;
    const double* in_norm;   // divide the input by in_norm[0] (0 -> zero vector), or null
    double* vout;            // x pass: the (divided) input, or null
    const double* b;         // base 2: b - v
    double* out;             // out_x (x pass) or out_y (y pass)
    const double* a;         // a(x) along this direction's lines (a[line * n + pos]), or null (a = 1)
    const double* inv_s;     // 1/S along the line direction (ones without a layer)
    const double* D;         // xi / n along the line direction
    const cpx<double>* tw;   // twiddles
    const int* gate;         // skip the launch when gate[0] == 0 (null: always run)
    int n1;                  // points per row
    int nlines;
    int base;                // 0: none, 1: v, 2: b - v (x pass only)
    double scale;            // f c
};

hipError_t launch_cn_apply(int dir, int n, int nlines, const CnApplyParams& p, hipStream_t s);
// Both directions of a square n x n grid (n <= 512) in one launch (px: x pass,
// py: y pass); the gate is px's.
hipError_t launch_cn_apply2(int n, const CnApplyParams& px, const CnApplyParams& py, hipStream_t s);
// out <- E^times in per point (E = diag(e0, conj e0) when E is null); out may be in.
hipError_t launch_cn_exp(const double* in, double* out, const double* E, double e0r, double e0i, size_t npts,
                         int times, hipStream_t s);

// The reductions below run kCnDotBlocks workgroups of 256 threads over the ncplx
// complex entries of the vectors; each workgroup writes fixed-order partial
// sums, and the workgroup that finishes last sums them in workgroup order
// (bitwise reproducible) and updates `ctrl`.

// Constants of the stopping rule and the Hessenberg matrix for the calls that follow.
hipError_t launch_cn_init(CnCtrl* ctrl, double hdt, double rtol, int max_iter, int m, hipStream_t s);
// rhs <- rx + ry; x <- 2 rhs - x; the partial sums of ||rhs||^2 (finished with
// the first residual's).
hipError_t launch_cn_rhs(const double* rx, const double* ry, double* rhs, double* x, size_t ncplx, double* partials,
                         hipStream_t s);
// The step's first residual r <- rx + ry (in ry), then with ||rhs|| (bnorm,
// tol = rtol bnorm, the step's counters reset): converged if ||r|| <= tol, else
// a new cycle from r.
hipError_t launch_cn_residual(const double* rx, double* ry, size_t ncplx, double* partials, CnCtrl* ctrl,
                              hipStream_t s);
// Arnoldi iteration j (basis V, vstride doubles apart), classical Gram-Schmidt:
// w <- wx + wy (in wx); h_k = <V_k, w> (k <= j), hn = ||w - V h||; the Givens
// update of column j.
hipError_t launch_cn_gs1(const double* V, size_t vstride, int j, double* wx, const double* wy, size_t ncplx,
                         double* partials, double* rec, CnCtrl* ctrl, hipStream_t s);
// V_{j+1} = (w - sum h_k V_k) / hn.
hipError_t launch_cn_gs_update(double* V, size_t vstride, int j, const double* w, size_t ncplx, const double* rec,
                               CnCtrl* ctrl, hipStream_t s);
// The end of a cycle (gated on ctrl->done): x += V y with R y = g solved per
// workgroup, and the residual r = rhs - G x = V (beta e_0 - H_G y) from the
// Arnoldi relation to r_out with its norm; then the outcome (converged, out of
// iterations, or a restart from r).  nk = columns queued (>= the cycle's k).
// Then the state head is written to `host` (pinned host memory), every time.
hipError_t launch_cn_update(const double* V, size_t vstride, int nk, double* x, double* r_out, size_t ncplx,
                            const double* rec, double* partials, CnCtrl* ctrl, CnHead* host, hipStream_t s);

}  // namespace dirac
