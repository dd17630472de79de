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

// One of the two sets of solve buffers; step n of a call uses set n mod 2, so
// that step n + 1 can be queued before step n's outcome is known.
struct CnCtx {
    dirac_solver* s;
    hipStream_t st;
    size_t npts, ncplx, vstride;      // vstride in doubles
    double* psi;                      // the step's state: Step 1 output, GMRES solution
    double* rhs;
    double* wx;                       // x part of an operator product, then the Arnoldi vector w
    double* wy;                       // y part; the cycle's starting residual
    double* V;                        // Krylov basis, m + 1 vectors
    double* part;                     // reduction partials (shared by both sets: stream order)
    double* rec;                      // Arnoldi coefficient records, one per iteration
    CnCtrl* ctrl;
    CnHead* head;                     // pinned host copy of the state head (written by a kernel)
    hipEvent_t ev;                    // recorded after the kernel that writes the head
    int j;                            // columns queued in the current cycle

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
        // a along this direction's lines (the transposed table for columns)
        p.a = s->curved ? reinterpret_cast<const double*>(b + (dir == 0 ? s->lay.a : s->lay.aT)) : nullptr;
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

// The end of the queued iterations: the end-of-cycle kernels (the update is a
// no-op until the cycle has ended; the finish writes the state head to the
// pinned host copy every time) and the event the host waits for.
hipError_t close_batch(CnCtx& c) {
    hipError_t e = launch_cn_update(c.V, c.vstride, c.j, c.psi, c.wy, c.ncplx, c.rec, c.part, c.ctrl, c.head, c.st);
    if (e == hipSuccess) e = hipEventRecord(c.ev, c.st);
    return e;
}

hipError_t queue_iterations(CnCtx& c, int nb) {
    for (int q = 0; q < nb; ++q) {
        hipError_t e = arnoldi(c, c.j + q);
        if (e != hipSuccess) return e;
    }
    c.j += nb;
    return close_batch(c);
}

// Step 2 on c.psi (= psi^{n+1/2}): rhs = G~ psi, x0 = 2 rhs - psi, r0 = rhs - G x0
// (to wy), then the first `batch` iterations of a cycle from r0.
hipError_t begin_solve(CnCtx& c, int batch) {
    dirac_solver* s = c.s;
    const double hdt = 0.5 * s->g.dt;
    hipError_t e = apply(c, c.psi, nullptr, nullptr, 1, nullptr, -hdt, nullptr);
    if (e == hipSuccess) e = launch_cn_rhs(c.wx, c.wy, c.rhs, c.psi, c.ncplx, c.part, c.st);
    if (e == hipSuccess) e = apply(c, c.psi, nullptr, nullptr, 2, c.rhs, -hdt, nullptr);
    if (e == hipSuccess) e = launch_cn_residual(c.wx, c.wy, c.ncplx, c.part, c.ctrl, c.st);
    c.j = 0;
    if (e == hipSuccess) e = queue_iterations(c, std::min(batch, s->scheme.gmres_restart));
    return e;
}

// Waits for c's last head copy and acts on it: done (converged), a failure, or
// the next batch queued (a restart from the new residual, or one more
// iteration of the current cycle).
dirac_status advance(CnCtx& c, bool& done) {
    dirac_solver* s = c.s;
    const int m = s->scheme.gmres_restart;
    done = false;
    CN_TRY(hipEventSynchronize(c.ev), "synchronise GMRES");
    const CnHead h = *c.head;
    s->cn_last_res = h.bnorm > 0 ? std::sqrt(h.res2) / h.bnorm : 0.0;
    if (h.nonfinite) {
        s->cn_iters += h.used;
        return fail(DIRAC_E_NONFINITE, "GMRES produced a non-finite value");
    }
    if (h.state == 2) {                                          // converged
        if (h.k > 0) s->cn_cycle_len = h.k;
        s->cn_iters += h.used;
        done = true;
        return DIRAC_OK;
    }
    if (h.state == 3) {
        s->cn_iters += h.used;
        return fail(DIRAC_E_NOCONV, "GMRES stopped after %d iterations at relative residual %.3g", h.used,
                    s->cn_last_res);
    }
    if (h.state == 1) {                                          // restart from the new residual
        s->cn_cycle_len = m;
        c.j = 0;
        CN_TRY(queue_iterations(c, m), "GMRES restart");
    } else {                                                     // the cycle goes on
        if (c.j >= m) return fail(DIRAC_E_DEVICE, "GMRES cycle state is inconsistent");
        CN_TRY(queue_iterations(c, 1), "Arnoldi iteration");
    }
    return DIRAC_OK;
}

}  // namespace

dirac_status cn_step_n(dirac_solver* s, int64_t nsteps) {
    if (nsteps == 0) return DIRAC_OK;
    char* b = s->base;
    const int m = s->scheme.gmres_restart;
    // coherent: the finish kernel's stores reach host memory directly
    if (!s->cn_head)
        CN_TRY(hipHostMalloc(&s->cn_head, 2 * sizeof(CnHead), hipHostMallocCoherent), "allocate the GMRES state copy");
    for (int k = 0; k < 2; ++k)
        if (!s->cn_ev[k]) CN_TRY(hipEventCreateWithFlags(&s->cn_ev[k], hipEventDisableTiming), "create an event");
    const size_t vstride = s->lay.cn_vecbytes / sizeof(double);
    const size_t set_vecs = (size_t)m + 4;
    const size_t coef_set = align_up_256(sizeof(CnCtrl)) + (size_t)m * kCnRecDoubles * 8;
    double* vecs = reinterpret_cast<double*>(b + s->lay.cn_vec);
    CnCtx cx[2];
    for (int k = 0; k < 2; ++k) {
        CnCtx& c = cx[k];
        c = CnCtx{};
        c.s = s;
        c.st = s->stream;
        c.npts = (size_t)s->g.n1 * s->g.n2;
        c.ncplx = 2 * c.npts;
        c.vstride = vstride;
        double* v = vecs + (size_t)k * set_vecs * vstride;
        c.psi = k == 0 ? reinterpret_cast<double*>(b + s->lay.psi) : vecs + 2 * set_vecs * vstride;
        c.rhs = v;
        c.wx = v + vstride;
        c.wy = v + 2 * vstride;
        c.V = v + 3 * vstride;
        c.part = reinterpret_cast<double*>(b + s->lay.cn_part);
        char* coef = b + s->lay.cn_coef + k * coef_set;
        c.ctrl = reinterpret_cast<CnCtrl*>(coef);
        c.rec = reinterpret_cast<double*>(coef + align_up_256(sizeof(CnCtrl)));
        c.head = static_cast<CnHead*>(s->cn_head) + k;
        c.ev = s->cn_ev[k];
        c.j = 0;
    }
    const double* E = s->curved ? reinterpret_cast<const double*>(b + s->lay.E) : nullptr;
    // Step 3 of the previous step, then Step 1 of this one (one application when
    // the step opens the call, or Step 3 alone after the last step); with
    // time-dependent potentials the two use t_{n-1/2} and t_{n+1/2}
    const size_t npts = cx[0].npts;
    auto exp_steps = [&](int64_t n_abs, int times, bool closing, const double* in, double* out) -> hipError_t {
        if (!s->has_em) return launch_cn_exp(in, out, E, s->e0u_re, s->e0u_im, npts, times, s->stream);
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
        return launch_em_exp(in, out, reinterpret_cast<const double*>(b + s->lay.em), npts, times, fA, fV,
                             s->stream);
    };
    // A failed call leaves the solver as it was: the state at entry is kept in
    // the staging area (N x 32 bytes, Scheme I is FP64) and put back, with the
    // step counter, if any step fails (its Step 1 and the closing Step 3 of the
    // earlier steps of this call would otherwise be half applied).
    const size_t state_bytes = npts * 32;
    double* psi = cx[0].psi;
    char* saved = b + s->lay.scratch;
    CN_TRY(hipMemcpyAsync(saved, psi, state_bytes, hipMemcpyDeviceToDevice, s->stream), "save state");
    for (int k = 0; k < 2; ++k)
        CN_TRY(launch_cn_init(cx[k].ctrl, 0.5 * s->g.dt, s->scheme.gmres_rtol, s->scheme.gmres_max_iter, m,
                              s->stream), "GMRES set-up");
    const int64_t step0 = s->step;
    // Step 3 of step n - 1 and Step 1 of step n (Step 1 alone for the call's
    // first step) into set n mod 2, and the first batch of its solve.
    auto start_step = [&](int64_t n) -> dirac_status {
        CnCtx& c = cx[n & 1];
        const double* in = cx[n == 0 ? 0 : (n - 1) & 1].psi;
        CN_TRY(exp_steps(step0 + n, n == 0 ? 1 : 2, false, in, c.psi), "Step 1");
        const int batch = std::max(1, s->cn_cycle_len > 0 ? s->cn_cycle_len : kCnFirstBatch);
        CN_TRY(begin_solve(c, batch), "GMRES start");
        return DIRAC_OK;
    };
    // Step n + 1 is queued before step n's outcome is read (once a cycle length
    // is known), so the host round trip overlaps device work.  If step n needs
    // more iterations, they are queued after it and step n + 1 is queued again
    // (the first copy worked on a state that was not final, in the other set,
    // which nothing reads).
    auto steps = [&]() -> dirac_status {
        dirac_status r = start_step(0);
        if (r != DIRAC_OK) return r;
        for (int64_t n = 0; n < nsteps; ++n) {
            const bool ahead = n + 1 < nsteps && s->cn_cycle_len > 0;
            if (ahead && (r = start_step(n + 1)) != DIRAC_OK) return r;
            bool done = false, first = true;
            for (;;) {
                if ((r = advance(cx[n & 1], done)) != DIRAC_OK) return r;
                if (done) break;
                first = false;
            }
            s->step += 1;
            if (n + 1 < nsteps && (!ahead || !first) && (r = start_step(n + 1)) != DIRAC_OK) return r;
        }
        CN_TRY(exp_steps(step0 + nsteps - 1, 1, true, cx[(nsteps - 1) & 1].psi, psi), "Step 3");
        CN_TRY(hipStreamSynchronize(s->stream), "synchronise");
        return DIRAC_OK;
    };
    const dirac_status r = steps();
    if (r != DIRAC_OK) {
        const std::string msg = dirac_last_error();
        s->step = step0;
        s->cn_cycle_len = 0;
        const hipError_t e1 = hipMemcpyAsync(psi, saved, state_bytes, hipMemcpyDeviceToDevice, s->stream);
        const hipError_t e2 = hipStreamSynchronize(s->stream);
        if (e1 != hipSuccess || e2 != hipSuccess)
            return fail(r, "%s (restoring the state also failed: %s)", msg.c_str(),
                        hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return fail(r, "%s", msg.c_str());
    }
    return DIRAC_OK;
}

}  // namespace dirac
