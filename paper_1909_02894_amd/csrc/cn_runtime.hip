// cn_runtime.hip -- host driver of Numerical Scheme I (Sec. 5.1, eq. (cn)):
//   psi^{n+1/2} = E psi^n                                  (Step 1)
//   G psi* = G~ psi^{n+1/2}, solved by restarted GMRES      (Step 2, Crank-Nicolson)
//   psi^{n+1} = E psi*                                      (Step 3)
// with G = I + (dt/2) alpha.T and G~ = I - (dt/2) alpha.T.  Every vector operation
// runs on the device; the host holds only the small Hessenberg least-squares
// problem of each GMRES cycle (Givens rotations, back substitution), and reads
// its columns in batches (gmres below).
//
// GMRES(m): Arnoldi with classical Gram-Schmidt applied twice (CGS2), started
// from x0 = psi^{n+1/2}; a cycle ends when the rotated residual estimate falls
// below rtol ||G~ psi||, and the next cycle's explicit residual b - G x decides
// convergence, so the reported residual is always a true one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/dirac.h"
#include "cn_kernels.hpp"
#include "em_kernels.hpp"
#include "solver.hpp"

namespace dirac {

namespace {

using zd = std::complex<double>;

struct CnCtx {
    dirac_solver* s;
    hipStream_t st;
    size_t npts, ncplx, vstride;      // vstride in doubles
    double* psi;
    double* rhs;
    double* work;
    double* V;                        // Krylov basis, m + 1 vectors
    double* part;
    double* coef;                     // [5][64] complex: (unused), (unused), norm, update, rhs norm;
                                      // then per Arnoldi iteration j: [3][64] h pass 1, h pass 2, norm
    double h;                         // (dt / 2) c

    double* vec(int k) const { return V + (size_t)k * vstride; }
    double* coef_row(int r) const { return coef + (size_t)r * 128; }
    double* rec_row(int j, int r) const { return coef + (size_t)(5 + 3 * j + r) * 128; }
};

#define CN_TRY(expr, what)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(DIRAC_E_DEVICE, "%s: %s", (what), hipGetErrorString(e_));    \
    } while (0)

// out = in + sign (dt/2) alpha.T in: the x pass writes out, the y pass accumulates.
hipError_t apply_G(const CnCtx& c, const double* in, double* out, double sign) {
    dirac_solver* s = c.s;
    char* b = s->base;
    for (int dir = 0; dir < 2; ++dir) {
        CnApplyParams p{};
        p.in = in;
        p.out = out;
        p.a = s->curved ? reinterpret_cast<const double*>(b + s->lay.a) : nullptr;
        p.inv_s = reinterpret_cast<const double*>(b + s->lay.inv_s[dir]);   // ones without a layer
        p.D = reinterpret_cast<const double*>(b + s->lay.D[dir]);
        p.tw = reinterpret_cast<const cpx<double>*>(b + s->lay.tw[dir]);
        p.n1 = s->g.n1;
        p.nlines = dir == 0 ? s->g.n2 : s->g.n1;
        p.scale = sign * c.h;
        hipError_t e = launch_cn_apply(dir, dir == 0 ? s->g.n1 : s->g.n2, p.nlines, p, c.st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ||v||^2 into coef row `row`, slot 0 (device), fixed-order reduction.
hipError_t norm2_dev(const CnCtx& c, const double* v, int row) {
    return launch_cn_dots(nullptr, 0, 0, true, v, c.ncplx, c.part, kCnDotBlocks, 64, c.coef_row(row), c.st);
}

dirac_status read_coef(const CnCtx& c, const double* src, double* host, size_t doubles) {
    CN_TRY(hipMemcpyAsync(host, src, doubles * sizeof(double), hipMemcpyDeviceToHost, c.st), "read GMRES coefficients");
    CN_TRY(hipStreamSynchronize(c.st), "synchronise GMRES");
    return DIRAC_OK;
}

// Solve G x = rhs in place (x = psi on entry is the initial guess).  The norm
// of rhs is on the device (coef row 4) and read with the first residual.
//
// Arnoldi iterations are queued in batches without a host round trip: each
// iteration's Hessenberg column and norm go to their own coefficient rows and
// the next basis vector is normalised on the device by that norm; the host
// then reads the batch's columns at once and applies the rotations column by
// column.  A cycle that converges inside a batch uses only its first columns
// (the later ones were computed and are dropped), so the iterate is the one
// the column-by-column form gives.  The first batch of a cycle is the previous
// cycle's length (steady solves converge at the same count); later batches are
// single iterations.
dirac_status gmres(CnCtx& c, int64_t& iters, double& rel_res) {
    dirac_solver* s = c.s;
    const int m = s->scheme.gmres_restart;
    std::vector<zd> H((size_t)(m + 1) * m), g(m + 1), sn(m), y(m);
    std::vector<double> cs(m), host(5 * 128), cols((size_t)3 * 128 * m);
    std::vector<double>& upload = s->cn_host;            // outlives the async upload
    upload.assign(128, 0.0);
    auto Hat = [&](int i, int j) -> zd& { return H[(size_t)i * m + j]; };
    int64_t used = 0;
    double tol = 0.0, bnorm = 0.0;
    bool first = true;
    for (;;) {
        // explicit residual r = rhs - G x
        CN_TRY(apply_G(c, c.psi, c.work, +1.0), "apply G");
        CN_TRY(launch_cn_sub(c.rhs, c.work, 4 * c.npts, c.st), "residual");
        CN_TRY(norm2_dev(c, c.work, 2), "residual norm");
        dirac_status r = read_coef(c, c.coef, host.data(), 5 * 128);
        if (r != DIRAC_OK) return r;
        if (first) {
            bnorm = std::sqrt(host[512]);
            tol = s->scheme.gmres_rtol * bnorm;
            first = false;
        }
        const double beta = std::sqrt(host[256]);
        if (!std::isfinite(beta)) return fail(DIRAC_E_NONFINITE, "GMRES residual is not finite");
        rel_res = bnorm > 0 ? beta / bnorm : 0.0;
        if (beta <= tol) break;
        if (used >= s->scheme.gmres_max_iter)
            return fail(DIRAC_E_NOCONV, "GMRES stopped after %lld iterations at relative residual %.3g",
                        (long long)used, rel_res);
        CN_TRY(launch_cn_scale(c.work, c.vec(0), 4 * c.npts, 1.0 / beta, c.st), "normalise");
        std::fill(g.begin(), g.end(), zd(0));
        g[0] = beta;
        int k = 0, j = 0;
        bool done = false;
        int batch = std::max(1, s->cn_cycle_len);
        while (!done && j < m) {
            const int nb = (int)std::min<int64_t>({(int64_t)batch, (int64_t)(m - j),
                                                   std::max<int64_t>(1, s->scheme.gmres_max_iter - used)});
            batch = 1;
            for (int q = 0; q < nb; ++q) {
                const int jj = j + q;
                CN_TRY(apply_G(c, c.vec(jj), c.work, +1.0), "apply G");
                // classical Gram-Schmidt applied twice; the second pass's dots ride on the
                // first update, and the second update writes the next basis vector, normalised
                // by ||w1||^2 - ||h2||^2 (w1 after the first pass, V orthonormal)
                const int nk = jj + 1;
                CN_TRY(launch_cn_dots(c.V, c.vstride, nk, false, c.work, c.ncplx, c.part, kCnDotBlocks, 64,
                                      c.rec_row(jj, 0), c.st), "Gram-Schmidt dots");
                if (nk <= kCnFusedMax) {
                    CN_TRY(launch_cn_axpy_dots(c.V, c.vstride, nk, c.rec_row(jj, 0), c.work, c.ncplx, c.part,
                                               kCnDotBlocks, 64, c.rec_row(jj, 1), c.st), "Gram-Schmidt update");
                } else {
                    CN_TRY(launch_cn_axpy(c.V, c.vstride, nk, c.rec_row(jj, 0), c.work, c.work, c.ncplx, 1.0, c.st),
                           "Gram-Schmidt update");
                    CN_TRY(launch_cn_dots(c.V, c.vstride, nk, true, c.work, c.ncplx, c.part, kCnDotBlocks, 64,
                                          c.rec_row(jj, 1), c.st), "Gram-Schmidt dots");
                }
                CN_TRY(launch_cn_axpy_normalise(c.V, c.vstride, nk, c.rec_row(jj, 1), c.work, c.vec(jj + 1),
                                                c.ncplx, c.rec_row(jj, 2), c.st), "normalise");
            }
            r = read_coef(c, c.rec_row(j, 0), cols.data(), (size_t)3 * 128 * nb);
            if (r != DIRAC_OK) return r;
            for (int q = 0; q < nb && !done; ++q) {
                const int jc = j + q;
                const double* col = cols.data() + (size_t)3 * 128 * q;
                ++used;
                for (int i = 0; i <= jc; ++i)
                    Hat(i, jc) = zd(col[2 * i] + col[128 + 2 * i], col[2 * i + 1] + col[128 + 2 * i + 1]);
                const double hn = std::sqrt(col[256]);
                if (!std::isfinite(hn)) return fail(DIRAC_E_NONFINITE, "Arnoldi vector is not finite");
                // previous rotations on the new column
                for (int i = 0; i < jc; ++i) {
                    const zd a = Hat(i, jc), b2 = Hat(i + 1, jc);
                    Hat(i, jc) = cs[i] * a + sn[i] * b2;
                    Hat(i + 1, jc) = -std::conj(sn[i]) * a + cs[i] * b2;
                }
                // new rotation zeroing the subdiagonal hn (real, >= 0)
                const zd a = Hat(jc, jc);
                const double aa = std::abs(a), rr = std::hypot(aa, hn);
                if (aa == 0.0) {
                    cs[jc] = 0.0;
                    sn[jc] = 1.0;
                } else {
                    cs[jc] = aa / rr;
                    sn[jc] = (a / aa) * hn / rr;
                }
                Hat(jc, jc) = cs[jc] * a + sn[jc] * hn;
                g[jc + 1] = -std::conj(sn[jc]) * g[jc];
                g[jc] = cs[jc] * g[jc];
                k = jc + 1;
                const double est = std::abs(g[jc + 1]);
                if (hn == 0.0 || est <= tol || used >= s->scheme.gmres_max_iter) done = true;
            }
            j += nb;
        }
        s->cn_cycle_len = k;
        // back substitution H y = g and x += V y
        for (int i = k - 1; i >= 0; --i) {
            zd acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= Hat(i, l) * y[l];
            y[i] = acc / Hat(i, i);
        }
        for (int i = 0; i < k; ++i) {
            upload[2 * i] = y[i].real();
            upload[2 * i + 1] = y[i].imag();
        }
        CN_TRY(hipMemcpyAsync(c.coef_row(3), upload.data(), 2 * k * sizeof(double), hipMemcpyHostToDevice, c.st),
               "upload update");
        CN_TRY(launch_cn_axpy(c.V, c.vstride, k, c.coef_row(3), c.psi, c.psi, c.ncplx, -1.0, c.st),
               "solution update");
    }
    iters += used;
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
    c.work = vecs + c.vstride;
    c.V = vecs + 2 * c.vstride;
    c.part = reinterpret_cast<double*>(b + s->lay.cn_part);
    c.coef = reinterpret_cast<double*>(b + s->lay.cn_coef);
    c.h = 0.5 * s->g.dt * s->g.c;
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
    const int64_t step0 = s->step;
    auto steps = [&]() -> dirac_status {
        for (int64_t n = 0; n < nsteps; ++n) {
            CN_TRY(exp_steps(s->step, n == 0 ? 1 : 2, false), "Step 1");
            CN_TRY(apply_G(c, c.psi, c.rhs, -1.0), "apply G~");
            CN_TRY(norm2_dev(c, c.rhs, 4), "right-hand side norm");
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
