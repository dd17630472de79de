// cn_kernels.hip -- Numerical Scheme I (Sec. 5.1): the Crank-Nicolson transport
// step G psi* = G~ psi^{n+1/2}, G = I + (dt/2) A, G~ = I - (dt/2) A with
// A psi = alpha(x).T psi = c (b_x sigma_x [[d_x]] psi + b_y sigma_y [[d_y]] psi)
// (spectral derivative of eq. (trick), b_i = a / S^i: Appendix A with layers),
// solved by restarted GMRES (FP64).
//
// The Krylov space of G is that of A, so the Arnoldi process runs on A: A v is
// far from parallel to v (A is close to skew-adjoint), so one classical
// Gram-Schmidt pass does not cancel and keeps the basis orthonormal to rounding
// over a cycle (on G = I + (dt/2) A almost all of G v lies along v and one pass
// loses orthogonality completely).  The Hessenberg matrix of G is
// I + (dt/2) H_A.  Each reduction ends in one workgroup that sums the
// per-workgroup partials in a fixed order (bitwise reproducible) and updates the
// device-resident least-squares state (Givens rotations), so a whole GMRES cycle
// needs no host round trip.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Radix and lines per workgroup of both directions in the merged kernel: the
// column rule, one workgroup shape (radix 4 with one line per workgroup at 512
// points, twice the waves, measured 15% slower), and one spinor component per
// thread (kCn2Cpt).
__host__ __device__ constexpr int cn2_radix(int n) { return cn_radix(n, true); }
__host__ __device__ constexpr int cn2_lines(int n) { return cn_lines(n, true); }
constexpr int kCn2Cpt = 1;
// Spinor components per thread of the per-direction kernels (other grids): one
// per lane for rows (2048-point FP64 rows 161 -> 139 us), both for columns,
// which then read whole 32-byte points (one per lane: 118 -> 132 us).
constexpr int cn_cpt(bool cols) { return cols ? 2 : 1; }

// Tile shape of a pass: the row or column rule, or (M2) the merged kernel's.
template <int N, bool COLS, bool M2 = false>
struct CnTile {
    static constexpr int R = M2 ? cn2_radix(N) : cn_radix(N, COLS), L = M2 ? cn2_lines(N) : cn_lines(N, COLS);
    static constexpr int CPT = M2 ? kCn2Cpt : cn_cpt(COLS);
    using F = LineFFT<double, N, R, L, COLS, CPT>;
    static constexpr int NT = F::NT;
    static constexpr int LDS = F::LDS_ELEMS;
    static constexpr int TW = TwStage<double, N>::ELEMS;
};

// One tile of one direction of the transport operator (see CnApplyParams);
// lds / twl: the workgroup's exchange buffer and twiddle stage.  With one
// component per thread (CPT = 1), a thread transforms its component k and
// takes [[d]] v_{1-k}, which output component k needs, from its partner lane.
template <int N, bool COLS, bool M2 = false>
__device__ __forceinline__ void cn_apply_tile(const CnApplyParams& p, int tile, cpx<double>* lds, cpx<double>* twl) {
    using T = double;
    constexpr int R = CnTile<N, COLS, M2>::R, L = CnTile<N, COLS, M2>::L, CPT = CnTile<N, COLS, M2>::CPT;
    using F = typename CnTile<N, COLS, M2>::F;
    using TS = TwStage<T, N>;
    constexpr int P = F::P;
    const typename F::Coord c = F::coord(threadIdx.x);
    const int line = tile * L + c.l;
    const bool valid = line < p.nlines;
    const int lline = valid ? line : p.nlines - 1;     // loads: clamped, branch-free
    const uint32_t n1 = (uint32_t)p.n1;
    auto gidx = [&](int ln, int pos) -> uint32_t {
        return COLS ? (uint32_t)pos * n1 + ln : (uint32_t)ln * n1 + pos;
    };
    // every global load goes out before the first wait
    cpx<T> v[CPT][R], bq[COLS ? 1 : CPT][COLS ? 1 : R];
    T d[R], bf[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (CPT == 1) v[0][r] = load_comp(p.in, gidx(lline, c.j + r * P), c.comp);
        else load_point(p.in, gidx(lline, c.j + r * P), v[0][r], v[1][r]);
    }
    if constexpr (!COLS) {
        if (p.base == 2) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (CPT == 1) bq[0][r] = load_comp(p.b, gidx(lline, c.j + r * P), c.comp);
                else load_point(p.b, gidx(lline, c.j + r * P), bq[0][r], bq[1][r]);
            }
        }
    }
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
        for (int r = 0; r < R; ++r) bf[r] = ld_at(p.a, (uint32_t)lline * N + c.j + r * P) * bf[r];
    }
    T inv = 1.0;
    if (p.in_norm) {
        const T nv = p.in_norm[0];
        inv = nv > 0.0 ? 1.0 / nv : 0.0;
    }
    if constexpr (TS::ON) {
        F::tw_store(twv, twl, threadIdx.x);
        tw = twl;
    }
    if (p.in_norm) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
            for (int r = 0; r < R; ++r) v[cc][r] = scal(inv, v[cc][r]);
    }
    cpx<T> in[COLS ? 1 : CPT][COLS ? 1 : R];
    if constexpr (!COLS) {
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
            for (int r = 0; r < R; ++r) in[cc][r] = v[cc][r];
        if (p.vout && valid) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (CPT == 1) store_comp(p.vout, gidx(line, c.j + r * P), c.comp, v[0][r]);
                else store_point(p.vout, gidx(line, c.j + r * P), v[0][r], v[1][r]);
            }
        }
    }
    F::template fft<false, TS::ON>(v, lds, c, tw);
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc)
#pragma unroll
        for (int s = 0; s < R; ++s) v[cc][s] = mul_i(scal(d[s], v[cc][s]));
    F::template fft<true, TS::ON>(v, lds, c, tw);
    // sigma_i [[d_i]] v: rows (sigma_x) t0 = [[d]] v1, t1 = [[d]] v0; columns
    // (sigma_y) t0 = -i [[d]] v1, t1 = i [[d]] v0
    cpx<T> tq[CPT][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (CPT == 1) {
            const cpx<T> w = partner(v[0][r]);         // [[d]] v_{1-k}
            tq[0][r] = COLS ? (c.comp == 0 ? mul_mi(w) : mul_i(w)) : w;
        } else {
            tq[0][r] = COLS ? mul_mi(v[1][r]) : v[1][r];
            tq[1][r] = COLS ? mul_i(v[0][r]) : v[0][r];
        }
    }
    if (!valid) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t q = gidx(line, c.j + r * P);
        const T f = p.scale * bf[r];               // f c b
        cpx<T> o[CPT];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            o[cc] = scal(f, tq[cc][r]);
            if constexpr (!COLS) {
                if (p.base == 1) o[cc] = in[cc][r] + o[cc];
                else if (p.base == 2) o[cc] = (bq[cc][r] - in[cc][r]) + o[cc];
            }
        }
        if constexpr (CPT == 1) store_comp(p.out, q, c.comp, o[0]);
        else store_point(p.out, q, o[0], o[1]);
    }
}

// One direction of the transport operator.
template <int N, bool COLS>
__global__ void __launch_bounds__((CnTile<N, COLS>::NT)) cn_apply_kernel(CnApplyParams p) {
    if (p.gate && p.gate[0] == 0) return;
    __shared__ cpx<double> lds[CnTile<N, COLS>::LDS];
    __shared__ cpx<double> twl[CnTile<N, COLS>::TW];
    cn_apply_tile<N, COLS>(p, xcd_tile(blockIdx.x, gridDim.x), lds, twl);
}

// Both directions of a square grid in one launch: the first ntx tiles of the
// (XCD-aware) tile order are row tiles, the rest column tiles, with one
// workgroup shape (cn2_radix, cn2_lines).  The two write separate outputs, so
// they run side by side.
template <int N>
__global__ void __launch_bounds__((CnTile<N, true, true>::NT)) cn_apply2_kernel(CnApplyParams px, CnApplyParams py,
                                                                                int ntx) {
    using TX = CnTile<N, false, true>;
    using TY = CnTile<N, true, true>;
    static_assert(TX::NT == TY::NT, "row and column tiles need the same workgroup");
    if (px.gate && px.gate[0] == 0) return;
    constexpr int LDS = TX::LDS > TY::LDS ? TX::LDS : TY::LDS;
    __shared__ cpx<double> lds[LDS];
    __shared__ cpx<double> twl[TY::TW];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t < ntx) cn_apply_tile<N, false, true>(px, t, lds, twl);
    else cn_apply_tile<N, true, true>(py, t - ntx, lds, twl);
}

// psi <- E^times in (times = 1 or 2; psi may be in), E = [[e0, e1], [conj e1, conj e0]]
// per point, or the uniform diagonal diag(e0u, conj e0u) when E is null.
__global__ void cn_exp_kernel(const double* in, double* psi, const double* E, double2 e0u, size_t npts, int times) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    cpx<double> u, v, e0{e0u.x, e0u.y}, e1{0, 0};
    load_point(in, (uint32_t)i, u, v);
    if (E) load_point(E, (uint32_t)i, e0, e1);
    for (int t = 0; t < times; ++t) {
        const cpx<double> nu = cmul(e0, u) + cmul(e1, v);
        const cpx<double> nv = cmul(cpx<double>{e0.re, -e0.im}, v) + cmul(cpx<double>{e1.re, -e1.im}, u);
        u = nu;
        v = nv;
    }
    store_point(psi, (uint32_t)i, u, v);
}

// ------------------------------------------------------------ reductions

constexpr int kCnThreads = 256;
constexpr int kCnSlots = kCnMaxRestart + 2;      // partial slots per workgroup (complex)
static_assert(kCnDotBlocks % 32 == 0, "the final sums take 32 workgroups per lane");

// Fixed-order workgroup sum of NS complex values per thread: a 64-lane
// butterfly, then the four waves in order; slot s0 + k of this workgroup's
// partials receives value k.
template <int NS>
__device__ __forceinline__ void store_partials(double (&ar)[NS], double (&ai)[NS], double* partials, int s0) {
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
        double* o = partials + 2 * ((size_t)blockIdx.x * kCnSlots + s0 + k);
        o[0] = ((sr[k][0] + sr[k][1]) + sr[k][2]) + sr[k][3];
        o[1] = ((si[k][0] + si[k][1]) + si[k][2]) + si[k][3];
    }
}

// out[s] = sum over the kCnDotBlocks workgroups' partial slot s (complex),
// s < nslots, by one workgroup into shared memory: 32 lanes per slot each load
// the partials of workgroups lane, lane + 32, ... at once and add them in that
// order, then a fixed 32-lane butterfly (bitwise reproducible).
__device__ void final_sums(const double* partials, int nslots, double* out) {
    constexpr int PER = kCnDotBlocks / 32;
    const int lane = threadIdx.x & 31;
    for (int s0 = 0; s0 < nslots; s0 += kCnThreads / 32) {
        const int sl = s0 + (int)(threadIdx.x >> 5);
        double r = 0.0, i = 0.0;
        if (sl < nslots) {
            double2 v[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q)
                v[q] = *reinterpret_cast<const double2*>(partials + 2 * ((size_t)(lane + 32 * q) * kCnSlots + sl));
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                r += v[q].x;
                i += v[q].y;
            }
        }
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
            r += __shfl_xor(r, off, 32);
            i += __shfl_xor(i, off, 32);
        }
        if (lane == 0 && sl < nslots) {
            out[2 * sl] = r;
            out[2 * sl + 1] = i;
        }
    }
    __syncthreads();
}

// Complex arithmetic of the least-squares state.
struct zc { double re, im; };
__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zc zconj(zc a) { return {a.re, -a.im}; }
__device__ __forceinline__ zc zadd(zc a, zc b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ zc zsub(zc a, zc b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ zc zscal(double s, zc a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ double zabs(zc a) { return hypot(a.re, a.im); }
__device__ __forceinline__ zc zdiv(zc a, zc b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// The scalars of the solve state a finishing workgroup reads, loaded by every
// thread at the kernel's start together with the partial sums.
struct CtrlSnap {
    double hdt, tol, rtol;
    zc gj;                // g_j (Givens update of column j)
    int done, nonfinite, used, max_iter, m, k;
};

__device__ __forceinline__ CtrlSnap load_snap(const CnCtrl* c, int j, bool with_g) {
    CtrlSnap q;
    q.hdt = c->hdt;
    q.tol = c->tol;
    q.rtol = c->rtol;
    q.gj = with_g ? zc{c->g[2 * j], c->g[2 * j + 1]} : zc{0.0, 0.0};
    q.done = c->done;
    q.nonfinite = c->nonfinite;
    q.used = c->used;
    q.max_iter = c->max_iter;
    q.m = c->m;
    q.k = c->k;
    return q;
}

// Givens update of column j of the cycle's least-squares problem (thread 0; the
// earlier rotations cs, sn are in shared memory).  h: H_A(0..j, j) (complex,
// shared memory), hn: the norm of the new Arnoldi vector.  Column j of
// H_G = I + (dt/2) H_A is rotated by the earlier rotations, a new rotation zeroes
// its subdiagonal (dt/2) hn, and g, k, the iteration count and the end-of-cycle
// flag are updated; the rotated column goes to R by the whole workgroup.
__device__ void givens_column(CnCtrl* c, int j, const double* h, double hn, const CtrlSnap& q, const double* cs,
                              const double* sn) {
    constexpr int M1 = kCnMaxRestart + 1;
    __shared__ double col[2 * M1];
    if (q.done) return;                            // the cycle has already ended (uniform)
    const double hd = q.hdt;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        col[2 * i] = hd * h[2 * i] + (i == j ? 1.0 : 0.0);
        col[2 * i + 1] = hd * h[2 * i + 1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!isfinite(hn)) {
            c->nonfinite = 1;
            c->done = 1;
        } else {
            const double sub = hd * hn;
            for (int i = 0; i < j; ++i) {
                const zc a{col[2 * i], col[2 * i + 1]}, b{col[2 * i + 2], col[2 * i + 3]};
                const zc r{sn[2 * i], sn[2 * i + 1]};
                const zc na = zadd(zscal(cs[i], a), zmul(r, b));
                const zc nb = zadd(zscal(-1.0, zmul(zconj(r), a)), zscal(cs[i], b));
                col[2 * i] = na.re; col[2 * i + 1] = na.im;
                col[2 * i + 2] = nb.re; col[2 * i + 3] = nb.im;
            }
            const zc a{col[2 * j], col[2 * j + 1]};
            const double aa = zabs(a), rr = hypot(aa, sub);
            double cj;
            zc sj;
            if (aa == 0.0) {
                cj = 0.0;
                sj = {1.0, 0.0};
            } else {
                cj = aa / rr;
                sj = zscal(sub / rr, zscal(1.0 / aa, a));
            }
            const zc d = zadd(zscal(cj, a), zscal(sub, sj));
            col[2 * j] = d.re; col[2 * j + 1] = d.im;
            c->cs[j] = cj;
            c->sn[2 * j] = sj.re; c->sn[2 * j + 1] = sj.im;
            const zc gj = q.gj;
            const zc g1 = zscal(-1.0, zmul(zconj(sj), gj));
            c->g[2 * j + 2] = g1.re; c->g[2 * j + 3] = g1.im;
            c->g[2 * j] = cj * gj.re; c->g[2 * j + 1] = cj * gj.im;
            c->k = j + 1;
            c->used = q.used + 1;
            const double est = zabs(g1);
            if (sub == 0.0 || est <= q.tol || q.used + 1 >= q.max_iter || j + 1 >= q.m) c->done = 1;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        c->R[2 * ((size_t)j * M1 + i)] = col[2 * i];
        c->R[2 * ((size_t)j * M1 + i) + 1] = col[2 * i + 1];
    }
}

// A new cycle from the residual of norm beta (thread 0).
__device__ void start_cycle(CnCtrl* c, double beta) {
    c->beta = beta;
    c->k = 0;
    c->done = 0;
    c->state = 0;
    c->g[0] = beta;
    c->g[1] = 0.0;
}

// Solver constants for the calls that follow; clears the flags.
__global__ void cn_init_kernel(CnCtrl* c, double hdt, double rtol, int max_iter, int m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->hdt = hdt;
        c->rtol = rtol;
        c->max_iter = max_iter;
        c->m = m;
        c->nonfinite = 0;
        c->done = 0;
        c->state = 0;
        c->k = 0;
    }
}

// rhs <- rx + ry, x <- 2 rhs - x (the first-order predictor of the solution,
// psi - dt A psi), ||rhs||; the step's counters are reset.
__global__ void __launch_bounds__(kCnThreads) cn_rhs_kernel(const double* rx, const double* ry, double* rhs,
                                                             double* x, size_t ncplx, double* partials) {
    double ar[1] = {0.0}, ai[1] = {0.0};
    const double2* RX = reinterpret_cast<const double2*>(rx);
    const double2* RY = reinterpret_cast<const double2*>(ry);
    double2* B = reinterpret_cast<double2*>(rhs);
    double2* X = reinterpret_cast<double2*>(x);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        const double2 a = RX[i], b = RY[i], h = X[i];
        const double2 r = {a.x + b.x, a.y + b.y};
        B[i] = r;
        X[i] = make_double2(2.0 * r.x - h.x, 2.0 * r.y - h.y);
        ar[0] += r.x * r.x + r.y * r.y;
    }
    store_partials<1>(ar, ai, partials, 1);       // slot 1: read with the first residual's (slot 0)
}

// r <- rx + ry (in ry) and ||r||^2; see launch_cn_residual.
__global__ void __launch_bounds__(kCnThreads) cn_residual_kernel(const double* rx, double* ry, size_t ncplx,
                                                                  double* partials) {
    double ar[1] = {0.0}, ai[1] = {0.0};
    const double2* RX = reinterpret_cast<const double2*>(rx);
    double2* RY = reinterpret_cast<double2*>(ry);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        const double2 a = RX[i], b = RY[i];
        const double2 r = {a.x + b.x, a.y + b.y};
        RY[i] = r;
        ar[0] += r.x * r.x + r.y * r.y;
    }
    store_partials<1>(ar, ai, partials, 0);
}

// First Gram-Schmidt pass of Arnoldi iteration j, basis vectors k0 .. k0+NK-1 of
// this launch: dots with w (FIRST: w = wx + wy is formed and stored to wx, and
// ||w||^2 goes to slot j + 1).  The last workgroup of the last launch stores the
// coefficients and decides: a second pass, or the Givens update of column j.
template <int NK, bool FIRST>
__global__ void __launch_bounds__(kCnThreads) cn_gs1_kernel(const double* V, size_t vstride, int k0, int j,
                                                             double* wx, const double* wy, size_t ncplx,
                                                             double* partials) {
    double ar[NK], ai[NK], nr[1] = {0.0}, ni[1] = {0.0};
#pragma unroll
    for (int k = 0; k < NK; ++k) ar[k] = ai[k] = 0.0;
    double2* W = reinterpret_cast<double2*>(wx);
    const double2* WY = reinterpret_cast<const double2*>(wy);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        double2 x = W[i];
        double2 y[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)(k0 + k) * vstride)[i];
        if constexpr (FIRST) {
            if (WY) {
                const double2 b = WY[i];
                x.x += b.x;
                x.y += b.y;
                W[i] = x;
            }
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            ar[k] += y[k].x * x.x + y[k].y * x.y;
            ai[k] += y[k].x * x.y - y[k].y * x.x;
        }
        if constexpr (FIRST) nr[0] += x.x * x.x + x.y * x.y;
    }
    store_partials<NK>(ar, ai, partials, k0);
    if constexpr (FIRST) {
        __syncthreads();
        store_partials<1>(nr, ni, partials, j + 1);
    }
}

// What the finishing workgroup does with the final sums of a reduction.
// kFinStart: ||rhs||^2 in slot 1 and the first residual's norm in slot 0;
// kFinRes: the residual after a cycle; kFinGs: the Gram-Schmidt dots of an iteration.
enum CnFinish { kFinStart = 1, kFinRes = 2, kFinGs = 3 };

// One workgroup after each reduction kernel: the final sums of its partials,
// then the solve-state update of `kind` (thread 0) and, after the Gram-Schmidt
// dots of an Arnoldi iteration, the Givens update of column j.  Every load of
// the solve state is issued with the partials' loads (one memory round trip).
// After a cycle (kFinRes), the head of the state is also written to `host`
// (pinned host memory) for the host's decision.
__global__ void __launch_bounds__(kCnThreads) cn_finish_kernel(const double* partials, int nslots, int kind, int j,
                                                                double* rec, CnCtrl* c, CnHead* host) {
    constexpr int M1 = kCnMaxRestart + 1;
    __shared__ double s[2 * kCnSlots];
    __shared__ double h[2 * M1], cs[M1], sn[2 * M1];
    __shared__ double hn_s;
    const int t = threadIdx.x;
    const bool gs = kind == kFinGs;
    double pc = 0.0, pr = 0.0, pi = 0.0;
    if (gs && t < j) {
        pc = c->cs[t];
        pr = c->sn[2 * t];
        pi = c->sn[2 * t + 1];
    }
    const CtrlSnap q = load_snap(c, j, gs);
    final_sums(partials, nslots, s);
    // after a cycle's end: nothing to decide while the cycle goes on, nor when it
    // ended with no column (the first residual met the tolerance; the update
    // kernel wrote nothing)
    const bool decide = kind != kFinRes || !(q.done == 0 || (q.k == 0 && !q.nonfinite));
    if (gs && t < j) {
        cs[t] = pc;
        sn[2 * t] = pr;
        sn[2 * t + 1] = pi;
    }
    if (t == 0 && decide) {
        if (kind == kFinStart || kind == kFinRes) {
            const double r2 = s[0];
            double tol = q.tol;
            int nonfinite = q.nonfinite;
            if (kind == kFinStart) {               // the step's right-hand side: counters reset
                const double b2 = s[2];
                tol = q.rtol * sqrt(b2);
                nonfinite = isfinite(b2) ? 0 : 1;
                c->bnorm = sqrt(b2);
                c->tol = tol;
                c->used = 0;
                c->k = 0;                          // no column yet: the update leaves x as it is
            }
            c->res2 = r2;
            if (!isfinite(r2) || nonfinite) {
                c->nonfinite = 1;
                c->done = 1;
                c->state = 3;
            } else if (sqrt(r2) <= tol) {
                c->nonfinite = 0;
                c->done = 1;
                c->state = 2;
            } else if (kind == kFinRes && q.used >= q.max_iter) {
                c->state = 3;
            } else {
                c->nonfinite = 0;
                start_cycle(c, sqrt(r2));
                if (kind == kFinRes) c->state = 1;
            }
        } else {
            double* h1 = rec;                      // Gram-Schmidt coefficients, slots 0..j
            double p2 = 0.0;
            for (int k = 0; k <= j; ++k) {
                h1[2 * k] = h[2 * k] = s[2 * k];
                h1[2 * k + 1] = h[2 * k + 1] = s[2 * k + 1];
                p2 += s[2 * k] * s[2 * k] + s[2 * k + 1] * s[2 * k + 1];
            }
            const double w2 = s[2 * (j + 1)];
            const double n2 = w2 - p2;             // ||w - V h||^2 with an orthonormal basis
            hn_s = isfinite(w2) ? sqrt(n2 > 0.0 ? n2 : 0.0) : NAN;
            c->hn = hn_s;
            h1[2 * (j + 1)] = hn_s;                // the subdiagonal entry, for the residual
            h1[2 * (j + 1) + 1] = 0.0;
        }
    }
    __syncthreads();
    if (gs) givens_column(c, j, h, hn_s, q, cs, sn);
    if (host && t == 0) {                          // this thread wrote c's head above
        const CnHead* hd = reinterpret_cast<const CnHead*>(c);
        *host = *hd;
    }
}

// V_{j+1} <- (w - sum_{k<=j} h_k V_k) / ctrl->hn (0 for hn = 0), j + 1 = 8 nfull +
// NKR coefficients.
template <int NKR>
__global__ void __launch_bounds__(kCnThreads) cn_gs_update_kernel(double* V, size_t vstride, int nfull, int j,
                                                                   const double* w, size_t ncplx, const double* rec,
                                                                   const CnCtrl* c) {
    const double* coef = rec;
    const double hn = c->hn;
    const double alpha = hn > 0.0 ? 1.0 / hn : 0.0;
    double2* out = reinterpret_cast<double2*>(V + (size_t)(j + 1) * vstride);
    const double2* Wi = reinterpret_cast<const double2*>(w);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        double2 x = Wi[i];
        for (int c8 = 0; c8 < nfull; ++c8) {
            double2 y[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)(8 * c8 + k) * vstride)[i];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double cr = coef[2 * (8 * c8 + k)], ci = coef[2 * (8 * c8 + k) + 1];
                x.x -= cr * y[k].x - ci * y[k].y;
                x.y -= cr * y[k].y + ci * y[k].x;
            }
        }
        double2 y[NKR > 0 ? NKR : 1];
#pragma unroll
        for (int k = 0; k < NKR; ++k) y[k] = reinterpret_cast<const double2*>(V + (size_t)(8 * nfull + k) * vstride)[i];
#pragma unroll
        for (int k = 0; k < NKR; ++k) {
            const double cr = coef[2 * (8 * nfull + k)], ci = coef[2 * (8 * nfull + k) + 1];
            x.x -= cr * y[k].x - ci * y[k].y;
            x.y -= cr * y[k].y + ci * y[k].x;
        }
        x.x *= alpha;
        x.y *= alpha;
        out[i] = x;
    }
}

// The end of a cycle (gated on done): x += sum_{i<k} y_i V_i with R y = g (upper
// triangular, k x k, solved by each workgroup in shared memory), and the new
// residual r = rhs - G x = V_{k+1} (beta e_0 - H_G y) from the Arnoldi relation
// G V_k = V_{k+1} H_G (no operator product), written to r_out with fixed-order
// partial sums of ||r||^2.  nv = 8 nfull + NKR basis vectors are read (nv - 1 =
// the columns queued, >= k; coefficients beyond k are 0).
template <int NKR>
__global__ void __launch_bounds__(kCnThreads) cn_update_kernel(const double* V, size_t vstride, int nfull,
                                                                double* x, double* r_out, size_t ncplx,
                                                                const double* rec, double* partials,
                                                                const CnCtrl* c) {
    constexpr int M1 = kCnMaxRestart + 1;
    // the least-squares state of up to nq = nv - 1 columns, packed: R column l
    // (rows 0..l) at l (l + 1) / 2, H_A column j (rows 0..j + 1) at j (j + 3) / 2;
    // loaded with the flags in one round before the gate
    __shared__ double y[2 * M1], g[2 * M1], cr[2 * (M1 + 1)];
    __shared__ double Rp[M1 * (M1 - 1)], Hp[(M1 - 1) * (M1 + 2)];
    const int nq = 8 * nfull + NKR - 1;
    const int done = c->done, nonfinite = c->nonfinite, k = c->k;
    const double beta = c->beta, hd = c->hdt;
    for (int i = threadIdx.x; i < 2 * M1; i += blockDim.x) {
        y[i] = 0.0;
        g[i] = i < 2 * nq ? c->g[i] : 0.0;
    }
    for (int i = threadIdx.x; i < 2 * (M1 + 1); i += blockDim.x) cr[i] = 0.0;
    for (int e = threadIdx.x; e < nq * nq; e += blockDim.x) {
        const int i = e % nq, l = e / nq;
        if (i <= l) {
            const int o = l * (l + 1) / 2 + i;
            Rp[2 * o] = c->R[2 * ((size_t)l * M1 + i)];
            Rp[2 * o + 1] = c->R[2 * ((size_t)l * M1 + i) + 1];
        }
    }
    for (int e = threadIdx.x; e < nq * (nq + 1); e += blockDim.x) {
        const int i = e % (nq + 1), j = e / (nq + 1);
        if (i <= j + 1) {
            const int o = j * (j + 3) / 2 + i;
            Hp[2 * o] = rec[(size_t)j * kCnRecDoubles + 2 * i];
            Hp[2 * o + 1] = rec[(size_t)j * kCnRecDoubles + 2 * i + 1];
        }
    }
    if (done == 0 || nonfinite || k == 0) return;  // uniform; k = 0: converged before the cycle
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            zc acc{g[2 * i], g[2 * i + 1]};
            for (int l = i + 1; l < k; ++l) {
                const int o = l * (l + 1) / 2 + i;
                acc = zsub(acc, zmul(zc{Rp[2 * o], Rp[2 * o + 1]}, zc{y[2 * l], y[2 * l + 1]}));
            }
            const int o = i * (i + 1) / 2 + i;
            const zc q = zdiv(acc, zc{Rp[2 * o], Rp[2 * o + 1]});
            y[2 * i] = q.re;
            y[2 * i + 1] = q.im;
        }
        // residual coefficients: beta e_0 - H_G y, H_G(i, j) = delta_ij + hdt H_A(i, j) (i <= j),
        // H_G(j + 1, j) = hdt hn_j, with column j of H_A and hn_j from record j
        cr[0] = beta;
        for (int j = 0; j < k; ++j) {
            const double* hj = Hp + j * (j + 3);
            const zc yj{y[2 * j], y[2 * j + 1]};
            for (int i = 0; i <= j; ++i) {
                const zc h = zadd(zscal(hd, zc{hj[2 * i], hj[2 * i + 1]}), zc{i == j ? 1.0 : 0.0, 0.0});
                const zc t = zmul(h, yj);
                cr[2 * i] -= t.re;
                cr[2 * i + 1] -= t.im;
            }
            const zc t = zscal(hd * hj[2 * (j + 1)], yj);
            cr[2 * (j + 1)] -= t.re;
            cr[2 * (j + 1) + 1] -= t.im;
        }
    }
    __syncthreads();
    double rr[1] = {0.0}, ri[1] = {0.0};
    double2* X = reinterpret_cast<double2*>(x);
    double2* RO = reinterpret_cast<double2*>(r_out);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncplx; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = X[i], r = {0.0, 0.0};
        for (int c8 = 0; c8 < nfull; ++c8) {
            double2 b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) b[q] = reinterpret_cast<const double2*>(V + (size_t)(8 * c8 + q) * vstride)[i];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int l = 8 * c8 + q;
                v.x += y[2 * l] * b[q].x - y[2 * l + 1] * b[q].y;
                v.y += y[2 * l] * b[q].y + y[2 * l + 1] * b[q].x;
                r.x += cr[2 * l] * b[q].x - cr[2 * l + 1] * b[q].y;
                r.y += cr[2 * l] * b[q].y + cr[2 * l + 1] * b[q].x;
            }
        }
        double2 b[NKR > 0 ? NKR : 1];
#pragma unroll
        for (int q = 0; q < NKR; ++q) b[q] = reinterpret_cast<const double2*>(V + (size_t)(8 * nfull + q) * vstride)[i];
#pragma unroll
        for (int q = 0; q < NKR; ++q) {
            const int l = 8 * nfull + q;
            v.x += y[2 * l] * b[q].x - y[2 * l + 1] * b[q].y;
            v.y += y[2 * l] * b[q].y + y[2 * l + 1] * b[q].x;
            r.x += cr[2 * l] * b[q].x - cr[2 * l + 1] * b[q].y;
            r.y += cr[2 * l] * b[q].y + cr[2 * l + 1] * b[q].x;
        }
        X[i] = v;
        RO[i] = r;
        rr[0] += r.x * r.x + r.y * r.y;
    }
    store_partials<1>(rr, ri, partials, 0);
}

// ---------------------------------------------------------------- launchers

template <int N, bool COLS>
static void launch_apply_n(int nlines, const CnApplyParams& p, hipStream_t s) {
    using TL = CnTile<N, COLS>;
    hipLaunchKernelGGL((cn_apply_kernel<N, COLS>), dim3((nlines + TL::L - 1) / TL::L), dim3(TL::NT), 0, s, p);
}

template <bool COLS>
static hipError_t launch_apply_dir(int n, int nlines, const CnApplyParams& p, hipStream_t s) {
    switch (n) {
        case 16: launch_apply_n<16, COLS>(nlines, p, s); break;
        case 32: launch_apply_n<32, COLS>(nlines, p, s); break;
        case 64: launch_apply_n<64, COLS>(nlines, p, s); break;
        case 128: launch_apply_n<128, COLS>(nlines, p, s); break;
        case 256: launch_apply_n<256, COLS>(nlines, p, s); break;
        case 512: launch_apply_n<512, COLS>(nlines, p, s); break;
        case 1024: launch_apply_n<1024, COLS>(nlines, p, s); break;
        case 2048: launch_apply_n<2048, COLS>(nlines, p, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cn_apply(int dir, int n, int nlines, const CnApplyParams& p, hipStream_t s) {
    return dir == 0 ? launch_apply_dir<false>(n, nlines, p, s) : launch_apply_dir<true>(n, nlines, p, s);
}

hipError_t launch_cn_apply2(int n, const CnApplyParams& px, const CnApplyParams& py, hipStream_t s) {
    const int ntx = (px.nlines + cn2_lines(n) - 1) / cn2_lines(n);
    const int nty = (py.nlines + cn2_lines(n) - 1) / cn2_lines(n);
    const dim3 grid(ntx + nty);
    switch (n) {
        case 16: hipLaunchKernelGGL(cn_apply2_kernel<16>, grid, dim3(CnTile<16, true, true>::NT), 0, s, px, py, ntx); break;
        case 32: hipLaunchKernelGGL(cn_apply2_kernel<32>, grid, dim3(CnTile<32, true, true>::NT), 0, s, px, py, ntx); break;
        case 64: hipLaunchKernelGGL(cn_apply2_kernel<64>, grid, dim3(CnTile<64, true, true>::NT), 0, s, px, py, ntx); break;
        case 128: hipLaunchKernelGGL(cn_apply2_kernel<128>, grid, dim3(CnTile<128, true, true>::NT), 0, s, px, py, ntx); break;
        case 256: hipLaunchKernelGGL(cn_apply2_kernel<256>, grid, dim3(CnTile<256, true, true>::NT), 0, s, px, py, ntx); break;
        case 512: hipLaunchKernelGGL(cn_apply2_kernel<512>, grid, dim3(CnTile<512, true, true>::NT), 0, s, px, py, ntx); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cn_exp(const double* in, double* out, const double* E, double e0r, double e0i, size_t npts,
                         int times, hipStream_t s) {
    hipLaunchKernelGGL(cn_exp_kernel, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, s, in, out, E,
                       make_double2(e0r, e0i), npts, times);
    return hipGetLastError();
}

hipError_t launch_cn_init(CnCtrl* ctrl, double hdt, double rtol, int max_iter, int m, hipStream_t s) {
    hipLaunchKernelGGL(cn_init_kernel, dim3(1), dim3(64), 0, s, ctrl, hdt, rtol, max_iter, m);
    return hipGetLastError();
}

static hipError_t finish(const double* partials, int nslots, CnFinish kind, int j, double* rec, CnCtrl* ctrl,
                         hipStream_t s, CnHead* host = nullptr) {
    hipLaunchKernelGGL(cn_finish_kernel, dim3(1), dim3(kCnThreads), 0, s, partials, nslots, (int)kind, j, rec, ctrl,
                       host);
    return hipGetLastError();
}

hipError_t launch_cn_rhs(const double* rx, const double* ry, double* rhs, double* x, size_t ncplx, double* partials,
                         hipStream_t s) {
    hipLaunchKernelGGL(cn_rhs_kernel, dim3(kCnDotBlocks), dim3(kCnThreads), 0, s, rx, ry, rhs, x, ncplx, partials);
    return hipGetLastError();
}

hipError_t launch_cn_residual(const double* rx, double* ry, size_t ncplx, double* partials, CnCtrl* ctrl,
                              hipStream_t s) {
    hipLaunchKernelGGL(cn_residual_kernel, dim3(kCnDotBlocks), dim3(kCnThreads), 0, s, rx, ry, ncplx, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finish(partials, 2, kFinStart, 0, nullptr, ctrl, s);
}

// Gram-Schmidt dots of Arnoldi iteration j: with V_0 .. V_j in chunks of kCnChunk
// vectors, one launch each (the first also forms w = wx + wy and its norm),
// then the finishing workgroup.
hipError_t launch_cn_gs1(const double* V, size_t vstride, int j, double* wx, const double* wy, size_t ncplx,
                         double* partials, double* rec, CnCtrl* ctrl, hipStream_t s) {
    if (j < 0 || j >= kCnMaxRestart) return hipErrorInvalidValue;
    const int nk = j + 1;
    const int nchunks = (nk + kCnChunk - 1) / kCnChunk;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int k0 = ch * kCnChunk, cnt = std::min(kCnChunk, nk - k0);
#define DIRAC_CN_GS(NK)                                                                                          \
    case NK:                                                                                                     \
        if (ch == 0)                                                                                             \
            hipLaunchKernelGGL((cn_gs1_kernel<NK, true>), dim3(kCnDotBlocks), dim3(kCnThreads), 0, s, V, vstride,\
                               k0, j, wx, wy, ncplx, partials);                                                  \
        else                                                                                                     \
            hipLaunchKernelGGL((cn_gs1_kernel<NK, false>), dim3(kCnDotBlocks), dim3(kCnThreads), 0, s, V,        \
                               vstride, k0, j, wx, wy, ncplx, partials);                                         \
        break;
        switch (cnt) {
            DIRAC_CN_GS(1) DIRAC_CN_GS(2) DIRAC_CN_GS(3) DIRAC_CN_GS(4)
            DIRAC_CN_GS(5) DIRAC_CN_GS(6) DIRAC_CN_GS(7) DIRAC_CN_GS(8)
            default: return hipErrorInvalidValue;
        }
#undef DIRAC_CN_GS
    }
    return finish(partials, j + 2, kFinGs, j, rec, ctrl, s);
}

hipError_t launch_cn_gs_update(double* V, size_t vstride, int j, const double* w, size_t ncplx, const double* rec,
                               CnCtrl* ctrl, hipStream_t s) {
    if (j < 0 || j >= kCnMaxRestart) return hipErrorInvalidValue;
    const int nk = j + 1, nfull = nk / 8;
#define DIRAC_CN_UP(R)                                                                                           \
    case R:                                                                                                      \
        hipLaunchKernelGGL((cn_gs_update_kernel<R>), dim3(1024), dim3(kCnThreads), 0, s, V, vstride, nfull, j, w,\
                           ncplx, rec, (const CnCtrl*)ctrl);                                                     \
        break;
    switch (nk % 8) {
        DIRAC_CN_UP(0) DIRAC_CN_UP(1) DIRAC_CN_UP(2) DIRAC_CN_UP(3)
        DIRAC_CN_UP(4) DIRAC_CN_UP(5) DIRAC_CN_UP(6) DIRAC_CN_UP(7)
        default: break;
    }
#undef DIRAC_CN_UP
    return hipGetLastError();
}

hipError_t launch_cn_update(const double* V, size_t vstride, int nk, double* x, double* r_out, size_t ncplx,
                            const double* rec, double* partials, CnCtrl* ctrl, CnHead* host, hipStream_t s) {
    if (nk < 0 || nk > kCnMaxRestart) return hipErrorInvalidValue;
    const int nv = nk + 1, nfull = nv / 8;
#define DIRAC_CN_XU(R)                                                                                           \
    case R:                                                                                                      \
        hipLaunchKernelGGL((cn_update_kernel<R>), dim3(kCnDotBlocks), dim3(kCnThreads), 0, s, V, vstride, nfull, \
                           x, r_out, ncplx, rec, partials, (const CnCtrl*)ctrl);                                 \
        break;
    switch (nv % 8) {
        DIRAC_CN_XU(0) DIRAC_CN_XU(1) DIRAC_CN_XU(2) DIRAC_CN_XU(3)
        DIRAC_CN_XU(4) DIRAC_CN_XU(5) DIRAC_CN_XU(6) DIRAC_CN_XU(7)
        default: break;
    }
#undef DIRAC_CN_XU
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finish(partials, 1, kFinRes, 0, nullptr, ctrl, s, host);
}

}  // namespace dirac
