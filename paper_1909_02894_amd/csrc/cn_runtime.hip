// cn_runtime.hip -- host driver of Numerical Scheme I (Sec. 5.1, eq. (cn)):
//   psi^{n+1/2} = E psi^n                                  (Step 1)
//   G psi* = G~ psi^{n+1/2}, solved by restarted GMRES      (Step 2, Crank-Nicolson)
//   psi^{n+1} = E psi*                                      (Step 3)
// with G = I + (dt/2) A and G~ = I - (dt/2) A, A = alpha(x).T.
//
// GMRES(m) from the first-order predictor x0 = psi - dt A psi (= 2 G~ psi - psi,
// one Arnoldi iteration fewer than x0 = psi at the same tolerance).  Arnoldi runs
// on A (same Krylov space as G) with one classical Gram-Schmidt pass (A v is far
// from parallel to v, so the pass does not cancel); the least-squares problem
// of I + (dt/2) H_A,
// its Givens rotations, the back substitution and every vector operation stay
// on the device.  The host queues a cycle's iterations (as many as the last
// cycle needed) and the update, then reads the device state once.  The update
// also forms the residual b - G x = V (beta e_0 - H_G y) from the Arnoldi
// relation G V = V H_G, vector by vector (it does not assume an orthonormal
// basis, unlike the rotated estimate |g_k|); its norm decides convergence and a
// restart starts from it.  Iterations queued past convergence change nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/dirac.h"
#include "cn_kernels.hpp"
#include "em_kernels.hpp"
#include "solver.hpp"

namespace dirac {

namespace {

// Iterations queued for a solver's first cycle (later cycles: the last one's length).
constexpr int kCnFirstBatch = 4;

size_t align_up_256(size_t x) { return (x + 255) & ~size_t(255); }

struct CnCtx {
    dirac_solver* s;
    hipStream_t st;
    size_t npts, ncplx, vstride;      // vstride in doubles
    double* psi;
    double* rhs;
    double* wx;                       // x part of an operator product, then the Arnoldi vector w
    double* wy;                       // y part; the cycle's starting residual
    double* V;                        // Krylov basis, m + 1 vectors
    double* part;
    double* rec;                      // Arnoldi coefficient records, one per iteration
    CnCtrl* ctrl;

    double* vec(int k) const { return V + (size_t)k * vstride; }
    double* rec_of(int j) const { return rec + (size_t)j * kCnRecDoubles; }
};

#define CN_TRY(expr, what)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(DIRAC_E_DEVICE, "%s: %s", (what), hipGetErrorString(e_));    \
    } while (0)

// out_x / out_y of the transport operator on `in` (see CnApplyParams).
hipError_t apply(const CnCtx& c, const double* in, const double* in_norm, double* vout, int base, const double* bvec,
                 double f, const int* gate) {
    dirac_solver* s = c.s;
    char* b = s->base;
    CnApplyParams pp[2];
    for (int dir = 0; dir < 2; ++dir) {
        CnApplyParams& p = pp[dir];
        p = CnApplyParams{};
        p.in = in;
        p.in_norm = in_norm;
        p.vout = dir == 0 ? vout : nullptr;
        p.b = bvec;
        p.out = dir == 0 ? c.wx : c.wy;
        p.a = s->curved ? reinterpret_cast<const double*>(b + s->lay.a) : nullptr;
        p.inv_s = reinterpret_cast<const double*>(b + s->lay.inv_s[dir]);   // ones without a layer
        p.D = reinterpret_cast<const double*>(b + s->lay.D[dir]);
        p.tw = reinterpret_cast<const cpx<double>*>(b + s->lay.tw[dir]);
        p.gate = gate;
        p.n1 = s->g.n1;
        p.nlines = dir == 0 ? s->g.n2 : s->g.n1;
        p.base = dir == 0 ? base : 0;
        p.scale = f * s->g.c;
    }
    // square grids up to 512 points: both directions in one launch, side by side
    if (s->g.n1 == s->g.n2 && s->g.n1 <= 512) return launch_cn_apply2(s->g.n1, pp[0], pp[1], c.st);
    for (int dir = 0; dir < 2; ++dir) {
        hipError_t e = launch_cn_apply(dir, dir == 0 ? s->g.n1 : s->g.n2, pp[dir].nlines, pp[dir], c.st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Arnoldi iteration j: w = A V_j (V_0 = r / beta is formed by the x pass of
// iteration 0 from the residual in wy), Gram-Schmidt dots and the Givens update
// of column j, V_{j+1}.
hipError_t arnoldi(const CnCtx& c, int j) {
    hipError_t e;
    if (j == 0) e = apply(c, c.wy, &c.ctrl->beta, c.vec(0), 0, nullptr, 1.0, nullptr);
    else e = apply(c, c.vec(j), nullptr, nullptr, 0, nullptr, 1.0, nullptr);
    if (e != hipSuccess) return e;
    if ((e = launch_cn_gs1(c.V, c.vstride, j, c.wx, c.wy, c.ncplx, c.part, c.rec_of(j), c.ctrl, c.st)) != hipSuccess)
        return e;
    return launch_cn_gs_update(c.V, c.vstride, j, c.wx, c.ncplx, c.rec_of(j), c.ctrl, c.st);
}

// The host's copy of the solve state after a cycle.
struct CtrlHead {
    double beta, bnorm, tol, res2, hn, hdt, rtol, pad0;
    int k, done, used, max_iter, m, state, nonfinite, pad1;
};
static_assert(sizeof(CtrlHead) <= sizeof(CnCtrl), "control head");

dirac_status read_ctrl(const CnCtx& c, CtrlHead& h) {
    CN_TRY(hipMemcpyAsync(&h, c.ctrl, sizeof h, hipMemcpyDeviceToHost, c.st), "read GMRES state");
    CN_TRY(hipStreamSynchronize(c.st), "synchronise GMRES");
    return DIRAC_OK;
}

// Solve G x = rhs for the step: on entry psi holds psi^{n+1/2}; on exit the solution.
dirac_status gmres(CnCtx& c, int64_t& iters, double& rel_res) {
    dirac_solver* s = c.s;
    const int m = s->scheme.gmres_restart;
    const double hdt = 0.5 * s->g.dt;
    // rhs = G~ psi, x0 = 2 rhs - psi, r0 = rhs - G x0 (to wy), a cycle starts from it
    CN_TRY(apply(c, c.psi, nullptr, nullptr, 1, nullptr, -hdt, nullptr), "apply G~");
    CN_TRY(launch_cn_rhs(c.wx, c.wy, c.rhs, c.psi, c.ncplx, c.part, c.ctrl, c.st), "right-hand side");
    CN_TRY(apply(c, c.psi, nullptr, nullptr, 2, c.rhs, -hdt, nullptr), "residual");
    CN_TRY(launch_cn_residual(c.wx, c.wy, c.ncplx, c.part, c.ctrl, true, c.st), "residual norm");
    CtrlHead h{};
    int j = 0;
    int batch = std::min(m, std::max(1, s->cn_cycle_len > 0 ? s->cn_cycle_len : kCnFirstBatch));
    for (;;) {
        const int nb = std::min(batch, m - j);
        for (int q = 0; q < nb; ++q) CN_TRY(arnoldi(c, j + q), "Arnoldi iteration");
        j += nb;
        // gated on the cycle's end: x += V y, the residual and the verdict
        CN_TRY(launch_cn_update(c.V, c.vstride, j, c.psi, c.wy, c.ncplx, c.rec, c.part, c.ctrl, c.st),
               "solution update");
        dirac_status r = read_ctrl(c, h);
        if (r != DIRAC_OK) return r;
        rel_res = h.bnorm > 0 ? std::sqrt(h.res2) / h.bnorm : 0.0;
        if (h.nonfinite) {
            iters += h.used;
            return fail(DIRAC_E_NONFINITE, "GMRES produced a non-finite value");
        }
        if (h.state == 2) break;                                 // converged
        if (h.state == 3) {
            iters += h.used;
            return fail(DIRAC_E_NOCONV, "GMRES stopped after %d iterations at relative residual %.3g", h.used,
                        rel_res);
        }
        if (h.state == 1) {                                      // restart from the new residual
            s->cn_cycle_len = m;
            j = 0;
            batch = m;
        } else {                                                 // the cycle goes on
            if (j >= m) return fail(DIRAC_E_DEVICE, "GMRES cycle state is inconsistent");
            batch = 1;
        }
    }
    if (h.k > 0) s->cn_cycle_len = h.k;
    iters += h.used;
    return DIRAC_OK;
}

}  // namespace

dirac_status cn_step_n(dirac_solver* s, int64_t nsteps) {
    if (nsteps == 0) return DIRAC_OK;
    char* b = s->base;
    CnCtx c{};
    c.s = s;
    c.st = s->stream;
    c.npts = (size_t)s->g.n1 * s->g.n2;
    c.ncplx = 2 * c.npts;
    c.vstride = s->lay.cn_vecbytes / sizeof(double);
    c.psi = reinterpret_cast<double*>(b + s->lay.psi);
    double* vecs = reinterpret_cast<double*>(b + s->lay.cn_vec);
    c.rhs = vecs;
    c.wx = vecs + c.vstride;
    c.wy = vecs + 2 * c.vstride;
    c.V = vecs + 3 * c.vstride;
    c.part = reinterpret_cast<double*>(b + s->lay.cn_part);
    c.ctrl = reinterpret_cast<CnCtrl*>(b + s->lay.cn_coef);
    c.rec = reinterpret_cast<double*>(b + s->lay.cn_coef + align_up_256(sizeof(CnCtrl)));
    const double* E = s->curved ? reinterpret_cast<const double*>(b + s->lay.E) : nullptr;
    // Step 3 of the previous step, then Step 1 of this one (one application when
    // the step opens the call, or Step 3 alone after the last step); with
    // time-dependent potentials the two use t_{n-1/2} and t_{n+1/2}
    auto exp_steps = [&](int64_t n_abs, int times, bool closing) -> hipError_t {
        if (!s->has_em) return launch_cn_exp(c.psi, E, s->e0u_re, s->e0u_im, c.npts, times, c.st);
        const double dt = s->g.dt;
        double t[2];
        if (closing) t[0] = (n_abs + 0.5) * dt;
        else if (times == 2) { t[0] = (n_abs - 0.5) * dt; t[1] = (n_abs + 0.5) * dt; }
        else t[0] = (n_abs + 0.5) * dt;
        double fA[2] = {0, 0}, fV[2] = {0, 0};
        for (int k = 0; k < times; ++k) {
            fA[k] = envelope_at(s->env_A, t[k]);
            fV[k] = envelope_at(s->env_V, t[k]);
        }
        return launch_em_exp(c.psi, reinterpret_cast<const double*>(b + s->lay.em), c.npts, times, fA, fV, c.st);
    };
    // A failed call leaves the solver as it was: the state at entry is kept in
    // the staging area (N x 32 bytes, Scheme I is FP64) and put back, with the
    // step counter, if any step fails (its Step 1 and the closing Step 3 of the
    // earlier steps of this call would otherwise be half applied).
    const size_t state_bytes = c.npts * 32;
    char* saved = b + s->lay.scratch;
    CN_TRY(hipMemcpyAsync(saved, c.psi, state_bytes, hipMemcpyDeviceToDevice, c.st), "save state");
    CN_TRY(launch_cn_init(c.ctrl, 0.5 * s->g.dt, s->scheme.gmres_rtol, s->scheme.gmres_max_iter,
                          s->scheme.gmres_restart, c.st), "GMRES set-up");
    const int64_t step0 = s->step;
    auto steps = [&]() -> dirac_status {
        for (int64_t n = 0; n < nsteps; ++n) {
            CN_TRY(exp_steps(s->step, n == 0 ? 1 : 2, false), "Step 1");
            dirac_status r = gmres(c, s->cn_iters, s->cn_last_res);
            if (r != DIRAC_OK) return r;
            s->step += 1;
        }
        CN_TRY(exp_steps(s->step - 1, 1, true), "Step 3");
        CN_TRY(hipStreamSynchronize(c.st), "synchronise");
        return DIRAC_OK;
    };
    const dirac_status r = steps();
    if (r != DIRAC_OK) {
        const std::string msg = dirac_last_error();
        s->step = step0;
        s->cn_cycle_len = 0;
        const hipError_t e1 = hipMemcpyAsync(c.psi, saved, state_bytes, hipMemcpyDeviceToDevice, c.st);
        const hipError_t e2 = hipStreamSynchronize(c.st);
        if (e1 != hipSuccess || e2 != hipSuccess)
            return fail(r, "%s (restoring the state also failed: %s)", msg.c_str(),
                        hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return fail(r, "%s", msg.c_str());
    }
    return DIRAC_OK;
}

}  // namespace dirac
