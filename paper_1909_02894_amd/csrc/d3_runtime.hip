// d3_runtime.hip -- the 3-D, 4-spinor solver: validation, device-buffer
// layout, table setup, the step launcher (direct or HIP-graph replay) and the
// observables, behind the dirac3_* C ABI.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/dirac.h"
#include "d3_kernels.hpp"
#include "setup_kernels.hpp"
#include "solver.hpp"

namespace dirac {

const D3Entry* d3_entries_f64(int* count);
const D3Entry* d3_entries_f32(int* count);

const D3Entry* d3_entry(int prec, int n, int dir) {
    int cnt = 0;
    const D3Entry* e = prec == DIRAC_FP64 ? d3_entries_f64(&cnt) : d3_entries_f32(&cnt);
    for (int i = 0; i < cnt; ++i)
        if (e[i].n == n && e[i].dir == dir) return &e[i];
    return nullptr;
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout3 {
    size_t psi, a, E, w, scratch, inv_s[3], K[3], D[3], tw[3], partials, out, total;
};

struct Setup3Params {
    int n1, n2, n3;
    double a1, a2, a3, dt, c, m;
    int kind, spin;
    const double* fields;     // FIELDS: 8 planes (phi, psi, phi_x, phi_y, phi_z, psi_x, psi_y, psi_z)
    const void* inv_s[3];     // per axis 1/S (T)
    int fp32;
    void* a_out;              // per point a (T) or null
    void* E_out;              // per point exponential record (T) or null
    double* w_out;            // per point weight e^{chi - Phi + Psi} (FP64)
    double* partial;          // 3 doubles per workgroup: min b, max b, non-finite count
};

// Per point: metric fields (FLAT, 3-D PAPER_EXP3, FIELDS), a = e^{Phi - Psi},
// the exponential record (C, -D w, D g_x, D g_y, D g_z) of
// exp(-i w beta + g . alpha), w = (dt/2) m c^2 e^Phi, g = -(dt/4) c a grad chi,
// with (-i w beta + g.alpha)^2 = (|g|^2 - w^2) I; the norm weight; and the
// blend range over the three axes.
__global__ void d3_setup_point_kernel(Setup3Params p) {
    const size_t N = (size_t)p.n1 * p.n2 * p.n3;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double bmin = 1e300, bmax = -1e300, bad = 0.0;
    if (q < N) {
        const int i = (int)(q % p.n1), j = (int)((q / p.n1) % p.n2), k = (int)(q / ((size_t)p.n1 * p.n2));
        const double x = -p.a1 + i * (2.0 * p.a1 / p.n1);
        const double y = -p.a2 + j * (2.0 * p.a2 / p.n2);
        const double z = -p.a3 + k * (2.0 * p.a3 / p.n3);
        double phi = 0, psi = 0, dphi[3] = {0, 0, 0}, dpsi[3] = {0, 0, 0};
        if (p.kind == DIRAC_METRIC_PAPER_EXP3) {
            const double r2 = x * x + y * y + z * z;
            phi = exp(-0.01 * r2);
            psi = exp(-0.005 * r2);
            const double X[3] = {x, y, z};
            for (int d = 0; d < 3; ++d) {
                dphi[d] = -0.02 * X[d] * phi;
                dpsi[d] = -0.01 * X[d] * psi;
            }
        } else if (p.kind == DIRAC_METRIC_FIELDS) {
            phi = p.fields[q];
            psi = p.fields[N + q];
            for (int d = 0; d < 3; ++d) {
                dphi[d] = p.fields[(2 + d) * N + q];
                dpsi[d] = p.fields[(5 + d) * N + q];
            }
        }
        double dchi[3] = {0, 0, 0}, chi = 0;
        if (p.spin == DIRAC_SPIN_PAPER) { for (int d = 0; d < 3; ++d) dchi[d] = dphi[d]; chi = phi; }
        else if (p.spin == DIRAC_SPIN_2P1) { for (int d = 0; d < 3; ++d) dchi[d] = dphi[d] + dpsi[d]; chi = phi + psi; }
        const double a = exp(phi - psi);
        const double w = 0.5 * p.dt * p.m * p.c * p.c * exp(phi);
        double g[3];
        for (int d = 0; d < 3; ++d) g[d] = -(p.dt / 4.0) * p.c * a * dchi[d];
        const double s2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] - w * w;
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
        const double rec[5] = {C, -D * w, D * g[0], D * g[1], D * g[2]};
        if (p.a_out) {
            if (p.fp32) static_cast<float*>(p.a_out)[q] = (float)a; else static_cast<double*>(p.a_out)[q] = a;
        }
        if (p.E_out) {
            if (p.fp32) {
                float* e = static_cast<float*>(p.E_out) + 8 * q;
                for (int t = 0; t < 5; ++t) e[t] = (float)rec[t];
                e[5] = e[6] = e[7] = 0.f;
            } else {
                double* e = static_cast<double*>(p.E_out) + 6 * q;
                for (int t = 0; t < 5; ++t) e[t] = rec[t];
                e[5] = 0.0;
            }
        }
        p.w_out[q] = exp(chi - phi + psi);
        const int idx[3] = {i, j, k};
        bool fin = isfinite(phi) && isfinite(psi) && isfinite(C) && isfinite(D);
        for (int d = 0; d < 3; ++d) {
            const double is = p.fp32 ? (double)static_cast<const float*>(p.inv_s[d])[idx[d]]
                                     : static_cast<const double*>(p.inv_s[d])[idx[d]];
            const double b = a * is;
            bmin = fmin(bmin, b);
            bmax = fmax(bmax, b);
            fin = fin && isfinite(dphi[d]) && isfinite(dpsi[d]) && isfinite(b);
        }
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

__global__ void d3_fold_kernel(const double* part, int nblocks, double* out) {
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

// Observables: per workgroup [sum |psi|^2, sum w |psi|^2, sum x|psi|^2,
// sum y|psi|^2, sum z|psi|^2, non-finite count, 0, 0] in FP64, fixed order.
template <typename T>
__global__ void __launch_bounds__(256) d3_obs_kernel(const T* psi, const double* w, int n1, int n2, size_t N,
                                                     double a1, double a2, double a3, double h1, double h2,
                                                     double h3, double* partials) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < N; q += (size_t)gridDim.x * blockDim.x) {
        cpx<T> u0, u1, w0, w1;
        load_point4(psi, (uint32_t)q, u0, u1, w0, w1);
        const double d = (double)u0.re * u0.re + (double)u0.im * u0.im + (double)u1.re * u1.re +
                         (double)u1.im * u1.im + (double)w0.re * w0.re + (double)w0.im * w0.im +
                         (double)w1.re * w1.re + (double)w1.im * w1.im;
        const int i = (int)(q % n1), j = (int)((q / n1) % n2), k = (int)(q / ((size_t)n1 * n2));
        acc[0] += d;
        acc[1] += w[q] * d;
        acc[2] += (-a1 + i * h1) * d;
        acc[3] += (-a2 + j * h2) * d;
        acc[4] += (-a3 + k * h3) * d;
        acc[5] += isfinite(d) ? 0.0 : 1.0;
    }
    __shared__ double red[4][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = 0; t < 6; ++t) {
        double x = acc[t];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[wave][t] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 0; t < 6; ++t) partials[8 * blockIdx.x + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
        partials[8 * blockIdx.x + 6] = 0.0;
        partials[8 * blockIdx.x + 7] = 0.0;
    }
}

constexpr int kObsBlocks = 512;

}  // namespace
}  // namespace dirac

using namespace dirac;

struct dirac3_solver {
    dirac3_grid g{};
    int32_t prec = 0;
    int kind = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    Layout3 lay{};
    bool curved = false, pml = false;
    double e0u_re = 1, e0u_im = 0;
    int64_t step = 0;
    bool has_state = false;
    const D3Entry* ent[3] = {nullptr, nullptr, nullptr};
    bool use_graph = true;
    int graph_chunk = 16;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<hipEvent_t> events;
};

namespace {

static bool pow2_3d(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

dirac_status validate3(const dirac3_grid* g, const dirac3_metric* m, const dirac_pml* pml, int32_t prec) {
    if (!g || !m || !pml) return fail(DIRAC_E_ARG, "null grid, metric or pml");
    if (prec != DIRAC_FP64 && prec != DIRAC_FP32) return fail(DIRAC_E_ARG, "precision must be 0 (FP64) or 1 (FP32)");
    if (!pow2_3d(g->n1) || !pow2_3d(g->n2) || !pow2_3d(g->n3))
        return fail(DIRAC_E_SIZE, "n1, n2, n3 = %d, %d, %d: each must be a power of two in [16, 1024]", g->n1, g->n2,
                    g->n3);
    const size_t N = (size_t)g->n1 * g->n2 * g->n3;
    if (N * 8 * (prec == DIRAC_FP32 ? 4 : 8) >= ((size_t)1 << 31))
        return fail(DIRAC_E_SIZE, "state of %zu points does not fit 2 GiB of 32-bit offsets", N);
    if (!(g->a1 > 0) || !(g->a2 > 0) || !(g->a3 > 0) || !std::isfinite(g->a1) || !std::isfinite(g->a2) ||
        !std::isfinite(g->a3))
        return fail(DIRAC_E_ARG, "half-widths must be finite and > 0");
    if (!(g->dt > 0) || !std::isfinite(g->dt)) return fail(DIRAC_E_ARG, "dt must be finite and > 0");
    if (!(g->c > 0) || !std::isfinite(g->c)) return fail(DIRAC_E_ARG, "c must be finite and > 0");
    if (!(g->m >= 0) || !std::isfinite(g->m)) return fail(DIRAC_E_ARG, "m must be finite and >= 0");
    if (m->kind != DIRAC_METRIC_FLAT && m->kind != DIRAC_METRIC_PAPER_EXP3 && m->kind != DIRAC_METRIC_FIELDS)
        return fail(DIRAC_E_ARG, "3-D metric kind must be FLAT, PAPER_EXP3 or FIELDS");
    if (m->spin < 0 || m->spin > 2) return fail(DIRAC_E_ARG, "unknown spin selector %d", m->spin);
    if (m->kind == DIRAC_METRIC_FIELDS &&
        (!m->phi || !m->psi || !m->dphi_dx || !m->dphi_dy || !m->dphi_dz || !m->dpsi_dx || !m->dpsi_dy || !m->dpsi_dz))
        return fail(DIRAC_E_ARG, "FIELDS metric needs all eight host arrays");
    const int nmin = std::min(g->n1, std::min(g->n2, g->n3));
    if (pml->width_pts < 0 || pml->width_pts > nmin / 2)
        return fail(DIRAC_E_ARG, "pml width %d outside [0, min(n1, n2, n3)/2]", pml->width_pts);
    if (pml->width_pts > 0) {
        if (pml->type < 1 || pml->type > 6) return fail(DIRAC_E_ARG, "pml type must be 1..6");
        if (!std::isfinite(pml->sigma0) || pml->sigma0 < 0) return fail(DIRAC_E_ARG, "pml sigma0 must be finite and >= 0");
        if (!std::isfinite(pml->theta) || (std::fabs(std::sin(pml->theta)) > 0 && pml->sigma0 > 0))
            return fail(DIRAC_E_UNSTABLE, "the directional step is stable only for a real stretch (sin theta = 0)");
    }
    for (int d = 0; d < 3; ++d) {
        const int n = d == 0 ? g->n1 : d == 1 ? g->n2 : g->n3;
        if (!d3_entry(prec, n, d)) return fail(DIRAC_E_SIZE, "no compiled 3-D kernel for n = %d", n);
    }
    return DIRAC_OK;
}

Layout3 layout3(const dirac3_grid* g, const dirac3_metric* m, int32_t prec) {
    Layout3 L{};
    const size_t N = (size_t)g->n1 * g->n2 * g->n3;
    const size_t sz = prec == DIRAC_FP32 ? 4 : 8;
    const bool curved = m->kind != DIRAC_METRIC_FLAT;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.psi = take(N * 8 * sz);
    L.a = curved ? take(N * sz) : SIZE_MAX;
    L.E = curved ? take(N * (prec == DIRAC_FP32 ? 8 : 6) * sz) : SIZE_MAX;
    L.w = take(N * 8);
    L.scratch = take(N * 64);              // complex128 staging, FIELDS staging (8 planes)
    const int ns[3] = {g->n1, g->n2, g->n3};
    for (int d = 0; d < 3; ++d) {
        L.inv_s[d] = take(ns[d] * sz);
        L.K[d] = take(ns[d] * 2 * sz);
        L.D[d] = take(ns[d] * sz);
        L.tw[d] = take(ns[d] * 2 * sz);
    }
    const size_t setup_parts = ((N + 255) / 256) * 3;
    L.partials = take(std::max(setup_parts, (size_t)kObsBlocks * 8) * 8);
    L.out = take(64 * 8);
    L.total = off + 256;
    return L;
}

template <typename T>
D3Params<T> d3_params(const dirac3_solver* s, int dir, int e_pre, int e_post) {
    D3Params<T> p{};
    char* b = s->base;
    p.psi = reinterpret_cast<T*>(b + s->lay.psi);
    p.a = s->curved ? reinterpret_cast<const T*>(b + s->lay.a) : nullptr;
    p.E = s->curved ? reinterpret_cast<const T*>(b + s->lay.E) : nullptr;
    p.inv_s = reinterpret_cast<const T*>(b + s->lay.inv_s[dir]);     // ones without a layer
    p.K = reinterpret_cast<const cpx<T>*>(b + s->lay.K[dir]);
    p.tw = reinterpret_cast<const cpx<T>*>(b + s->lay.tw[dir]);
    p.n1 = s->g.n1;
    p.n2 = s->g.n2;
    p.nlines = dir == 0 ? s->g.n2 * s->g.n3 : dir == 1 ? s->g.n1 * s->g.n3 : s->g.n1 * s->g.n2;
    p.e_pre = e_pre;
    p.e_post = e_post;
    p.e0u = cpx<T>{(T)s->e0u_re, (T)s->e0u_im};
    return p;
}

struct Launch3 {
    const void* fn;
    dim3 grid, block;
    alignas(16) unsigned char params[sizeof(D3Params<double>)];
};

Launch3 make_launch3(const dirac3_solver* s, int dir, int e_pre, int e_post) {
    Launch3 L{};
    const D3Entry* e = s->ent[dir];
    const int mode = s->curved ? 2 : (s->pml ? 1 : 0);
    L.fn = e->fn[mode];
    const int nlines = dir == 0 ? s->g.n2 * s->g.n3 : dir == 1 ? s->g.n1 * s->g.n3 : s->g.n1 * s->g.n2;
    L.grid = dim3((nlines + e->lines - 1) / e->lines);
    L.block = dim3(e->nthreads);
    if (s->prec == DIRAC_FP64) {
        auto p = d3_params<double>(s, dir, e_pre, e_post);
        std::memcpy(L.params, &p, sizeof p);
    } else {
        auto p = d3_params<float>(s, dir, e_pre, e_post);
        std::memcpy(L.params, &p, sizeof p);
    }
    return L;
}

hipError_t launch3(Launch3& L, hipStream_t st) {
    void* args[] = {L.params};
    return hipLaunchKernel(L.fn, L.grid, L.block, args, 0, st);
}

void drop_graph3(dirac3_solver* s) {
    if (s->gexec) {
        (void)hipStreamSynchronize(s->stream);   // a replay may still be in flight
        (void)hipGraphExecDestroy(s->gexec);
        s->gexec = nullptr;
    }
    if (s->graph) { (void)hipGraphDestroy(s->graph); s->graph = nullptr; }
}

#define D3_TRY(expr, what)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(DIRAC_E_DEVICE, "%s: %s", (what), hipGetErrorString(e_));    \
    } while (0)

// Graph of graph_chunk middle steps: [y, z (no Step 5), x (Step 5 + Step 1)] repeated.
dirac_status build_graph3(dirac3_solver* s) {
    drop_graph3(s);
    D3_TRY(hipGraphCreate(&s->graph, 0), "hipGraphCreate");
    Launch3 ly = make_launch3(s, 1, 0, 0), lz = make_launch3(s, 2, 0, 0), lx = make_launch3(s, 0, 2, 0);
    hipGraphNode_t prev = nullptr;
    for (int c = 0; c < s->graph_chunk; ++c) {
        for (Launch3* L : {&ly, &lz, &lx}) {
            void* args[] = {L->params};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(L->fn);
            kp.gridDim = L->grid;
            kp.blockDim = L->block;
            kp.kernelParams = args;
            hipGraphNode_t node;
            D3_TRY(hipGraphAddKernelNode(&node, s->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp),
                   "hipGraphAddKernelNode");
            prev = node;
        }
    }
    D3_TRY(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return DIRAC_OK;
}

dirac_status enqueue3(dirac3_solver* s, int64_t nsteps) {
    if (nsteps <= 0) return DIRAC_OK;
    hipStream_t st = s->stream;
    Launch3 x1 = make_launch3(s, 0, 1, 0);
    D3_TRY(launch3(x1, st), "launch x stage");
    int64_t middle = nsteps - 1;
    if (s->use_graph && middle >= s->graph_chunk) {
        if (!s->gexec) {
            dirac_status r = build_graph3(s);
            if (r != DIRAC_OK) return r;
        }
        while (middle >= s->graph_chunk) {
            D3_TRY(hipGraphLaunch(s->gexec, st), "hipGraphLaunch");
            middle -= s->graph_chunk;
        }
    }
    Launch3 ly = make_launch3(s, 1, 0, 0), lz = make_launch3(s, 2, 0, 0), lx = make_launch3(s, 0, 2, 0);
    for (int64_t k = 0; k < middle; ++k) {
        D3_TRY(launch3(ly, st), "launch y stage");
        D3_TRY(launch3(lz, st), "launch z stage");
        D3_TRY(launch3(lx, st), "launch x stage");
    }
    D3_TRY(launch3(ly, st), "launch y stage");
    Launch3 zl = make_launch3(s, 2, 0, 1);
    D3_TRY(launch3(zl, st), "launch z stage");
    return DIRAC_OK;
}

}  // namespace

extern "C" {

size_t dirac3_footprint_bytes(const dirac3_grid* g, const dirac3_metric* m, const dirac_pml* pml, int32_t prec) {
    if (validate3(g, m, pml, prec) != DIRAC_OK) return 0;
    return layout3(g, m, prec).total;
}

dirac_status dirac3_create(const dirac3_grid* g, const dirac3_metric* m, const dirac_pml* pml, int32_t prec,
                           void* device_buffer, size_t bytes, void* hip_stream, dirac3_solver** out) {
    if (!out) return fail(DIRAC_E_ARG, "null output handle");
    *out = nullptr;
    dirac_status st = validate3(g, m, pml, prec);
    if (st != DIRAC_OK) return st;
    if (!device_buffer) return fail(DIRAC_E_ARG, "null device buffer");
    Layout3 lay = layout3(g, m, prec);
    if (bytes < lay.total) return fail(DIRAC_E_SIZE, "device buffer of %zu bytes < footprint %zu", bytes, lay.total);
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, device_buffer) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(DIRAC_E_ARG, "device_buffer is not device memory");
    }
    dirac3_solver* s = new (std::nothrow) dirac3_solver();
    if (!s) return fail(DIRAC_E_NOMEM, "host allocation failed");
    auto bail = [&](dirac_status r) { delete s; return r; };
    s->g = *g;
    s->prec = prec;
    s->kind = m->kind;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(device_buffer) + 255) & ~uintptr_t(255));
    s->lay = lay;
    s->curved = m->kind != DIRAC_METRIC_FLAT;
    s->pml = pml->width_pts > 0;
    const double mu = g->dt * g->m * g->c * g->c / 2.0;
    s->e0u_re = std::cos(mu);
    s->e0u_im = -std::sin(mu);
    for (int d = 0; d < 3; ++d) s->ent[d] = d3_entry(prec, d == 0 ? g->n1 : d == 1 ? g->n2 : g->n3, d);
    const size_t N = (size_t)g->n1 * g->n2 * g->n3;
    const bool fp32 = prec == DIRAC_FP32;
    char* b = s->base;
    if (m->kind == DIRAC_METRIC_FIELDS) {
        const double* planes[8] = {m->phi, m->psi, m->dphi_dx, m->dphi_dy, m->dphi_dz, m->dpsi_dx, m->dpsi_dy, m->dpsi_dz};
        for (int k = 0; k < 8; ++k) {
            hipError_t e = hipMemcpyAsync(b + lay.scratch + k * N * 8, planes[k], N * 8, hipMemcpyHostToDevice, s->stream);
            if (e != hipSuccess) return bail(fail(DIRAC_E_DEVICE, "upload metric fields: %s", hipGetErrorString(e)));
        }
    }
    const int ns[3] = {g->n1, g->n2, g->n3};
    const double as[3] = {g->a1, g->a2, g->a3};
    for (int d = 0; d < 3; ++d) {
        SetupAxisParams ap{};
        ap.n = ns[d];
        ap.a = as[d];
        ap.c = g->c;
        ap.dt = g->dt;
        ap.pml_width = pml->width_pts;
        ap.pml_type = pml->type;
        ap.sigma0 = pml->sigma0;
        ap.ctheta = std::cos(pml->theta);
        ap.fp32 = fp32;
        ap.k_printed = 0;
        ap.inv_s = b + lay.inv_s[d];
        ap.K = b + lay.K[d];
        ap.D = b + lay.D[d];
        ap.tw = b + lay.tw[d];
        hipError_t e = launch_setup_axis(ap, s->stream);
        if (e != hipSuccess) return bail(fail(DIRAC_E_DEVICE, "setup axis tables: %s", hipGetErrorString(e)));
    }
    Setup3Params sp{};
    sp.n1 = g->n1; sp.n2 = g->n2; sp.n3 = g->n3;
    sp.a1 = g->a1; sp.a2 = g->a2; sp.a3 = g->a3;
    sp.dt = g->dt; sp.c = g->c; sp.m = g->m;
    sp.kind = m->kind; sp.spin = m->spin;
    sp.fields = m->kind == DIRAC_METRIC_FIELDS ? reinterpret_cast<const double*>(b + lay.scratch) : nullptr;
    for (int d = 0; d < 3; ++d) sp.inv_s[d] = b + lay.inv_s[d];
    sp.fp32 = fp32;
    sp.a_out = s->curved ? b + lay.a : nullptr;
    sp.E_out = s->curved ? b + lay.E : nullptr;
    sp.w_out = reinterpret_cast<double*>(b + lay.w);
    sp.partial = reinterpret_cast<double*>(b + lay.partials);
    const int nblk = (int)((N + 255) / 256);
    hipLaunchKernelGGL(d3_setup_point_kernel, dim3(nblk), dim3(256), 0, s->stream, sp);
    double* fold = reinterpret_cast<double*>(b + lay.out);
    hipLaunchKernelGGL(d3_fold_kernel, dim3(1), dim3(256), 0, s->stream, (const double*)sp.partial, nblk, fold);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bail(fail(DIRAC_E_DEVICE, "setup: %s", hipGetErrorString(e)));
    double hf[3];
    e = hipMemcpyAsync(hf, fold, sizeof hf, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(fail(DIRAC_E_DEVICE, "setup synchronise: %s", hipGetErrorString(e)));
    if (hf[2] != 0.0) return bail(fail(DIRAC_E_NONFINITE, "%.0f grid points have non-finite fields", hf[2]));
    if (hf[0] < 0.0 || hf[1] > 1.0 + 1e-12)
        return bail(fail(DIRAC_E_UNSTABLE, "blend coefficient b = a/S ranges over [%.17g, %.17g]; the directional "
                                           "step is stable only for b in [0, 1]", hf[0], hf[1]));
    *out = s;
    return DIRAC_OK;
}

dirac_status dirac3_set_initial_spinor(dirac3_solver* s, const double* psi_host) {
    if (!s || !psi_host) return fail(DIRAC_E_ARG, "null solver or spinor");
    const size_t N = (size_t)s->g.n1 * s->g.n2 * s->g.n3;
    for (size_t i = 0; i < 8 * N; ++i)
        if (!std::isfinite(psi_host[i])) return fail(DIRAC_E_NONFINITE, "initial spinor has a non-finite value");
    char* b = s->base;
    if (s->prec == DIRAC_FP64) {
        D3_TRY(hipMemcpyAsync(b + s->lay.psi, psi_host, N * 64, hipMemcpyHostToDevice, s->stream), "upload spinor");
    } else {
        D3_TRY(hipMemcpyAsync(b + s->lay.scratch, psi_host, N * 64, hipMemcpyHostToDevice, s->stream), "upload spinor");
        D3_TRY(launch_c128_to_f32(reinterpret_cast<const double*>(b + s->lay.scratch),
                                  reinterpret_cast<float*>(b + s->lay.psi), 8 * N, s->stream), "convert spinor");
    }
    D3_TRY(hipStreamSynchronize(s->stream), "synchronise");
    s->step = 0;
    s->has_state = true;
    return DIRAC_OK;
}

dirac_status dirac3_set_initial_spinor_device(dirac3_solver* s, const void* psi_dev) {
    if (!s || !psi_dev) return fail(DIRAC_E_ARG, "null solver or spinor");
    const size_t N = (size_t)s->g.n1 * s->g.n2 * s->g.n3;
    char* b = s->base;
    if (s->prec == DIRAC_FP64) {
        D3_TRY(hipMemcpyAsync(b + s->lay.psi, psi_dev, N * 64, hipMemcpyDeviceToDevice, s->stream), "copy spinor");
    } else {
        D3_TRY(launch_c128_to_f32(static_cast<const double*>(psi_dev), reinterpret_cast<float*>(b + s->lay.psi),
                                  8 * N, s->stream), "convert spinor");
    }
    s->step = 0;
    s->has_state = true;
    return DIRAC_OK;
}

dirac_status dirac3_step_n(dirac3_solver* s, int64_t nsteps) {
    if (!s) return fail(DIRAC_E_ARG, "null solver");
    if (nsteps < 0) return fail(DIRAC_E_ARG, "nsteps must be >= 0");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    dirac_status r = enqueue3(s, nsteps);
    if (r != DIRAC_OK) return r;
    s->step += nsteps;
    return DIRAC_OK;
}

dirac_status dirac3_set_launch_mode(dirac3_solver* s, int32_t use_graph, int32_t chunk) {
    if (!s || chunk < 1 || chunk > 4096) return fail(DIRAC_E_ARG, "bad arguments");
    s->use_graph = use_graph != 0;
    s->graph_chunk = chunk;
    drop_graph3(s);
    return DIRAC_OK;
}

dirac_status dirac3_step_n_timed(dirac3_solver* s, int64_t nsteps, double* ms_out, int64_t* counts_out) {
    if (!s || !ms_out || !counts_out) return fail(DIRAC_E_ARG, "null argument");
    if (nsteps < 0) return fail(DIRAC_E_ARG, "nsteps must be >= 0");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    for (int d = 0; d < 3; ++d) { ms_out[d] = 0; counts_out[d] = 0; }
    if (nsteps == 0) return DIRAC_OK;
    const size_t nl = (size_t)nsteps * 3;
    while (s->events.size() < 2 * nl) {
        hipEvent_t ev;
        D3_TRY(hipEventCreate(&ev), "hipEventCreate");
        s->events.push_back(ev);
    }
    size_t k = 0;
    for (int64_t n = 0; n < nsteps; ++n) {
        Launch3 L[3] = {make_launch3(s, 0, n == 0 ? 1 : 2, 0), make_launch3(s, 1, 0, 0),
                        make_launch3(s, 2, 0, n == nsteps - 1 ? 1 : 0)};
        for (int d = 0; d < 3; ++d) {
            void* args[] = {L[d].params};
            D3_TRY(hipExtLaunchKernel(L[d].fn, L[d].grid, L[d].block, args, 0, s->stream, s->events[2 * k],
                                      s->events[2 * k + 1], 0), "launch stage");
            ++k;
        }
    }
    D3_TRY(hipStreamSynchronize(s->stream), "synchronise");
    for (size_t i = 0; i < k; ++i) {
        float ms = 0;
        D3_TRY(hipEventElapsedTime(&ms, s->events[2 * i], s->events[2 * i + 1]), "hipEventElapsedTime");
        ms_out[i % 3] += ms;
        counts_out[i % 3] += 1;
    }
    s->step += nsteps;
    return DIRAC_OK;
}

dirac_status dirac3_observables(dirac3_solver* s, dirac3_obs* out) {
    if (!s || !out) return fail(DIRAC_E_ARG, "null solver or output");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    const size_t N = (size_t)s->g.n1 * s->g.n2 * s->g.n3;
    char* b = s->base;
    const double h1 = 2.0 * s->g.a1 / s->g.n1, h2 = 2.0 * s->g.a2 / s->g.n2, h3 = 2.0 * s->g.a3 / s->g.n3;
    double* parts = reinterpret_cast<double*>(b + s->lay.partials);
    const double* w = reinterpret_cast<const double*>(b + s->lay.w);
    if (s->prec == DIRAC_FP64)
        hipLaunchKernelGGL(d3_obs_kernel<double>, dim3(kObsBlocks), dim3(256), 0, s->stream,
                           reinterpret_cast<const double*>(b + s->lay.psi), w, s->g.n1, s->g.n2, N, s->g.a1,
                           s->g.a2, s->g.a3, h1, h2, h3, parts);
    else
        hipLaunchKernelGGL(d3_obs_kernel<float>, dim3(kObsBlocks), dim3(256), 0, s->stream,
                           reinterpret_cast<const float*>(b + s->lay.psi), w, s->g.n1, s->g.n2, N, s->g.a1,
                           s->g.a2, s->g.a3, h1, h2, h3, parts);
    D3_TRY(hipGetLastError(), "launch observables");
    double* dout = reinterpret_cast<double*>(b + s->lay.out);
    D3_TRY(launch_reduce_partials(parts, kObsBlocks, dout, s->stream), "reduce observables");
    double h[8];
    D3_TRY(hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s->stream), "read observables");
    D3_TRY(hipStreamSynchronize(s->stream), "synchronise");
    const double dV = h1 * h2 * h3;
    out->step = s->step;
    out->t = s->step * s->g.dt;
    out->norm_l2 = dV * h[0];
    out->norm_w = dV * h[1];
    out->x_mean = h[2] / h[0];
    out->y_mean = h[3] / h[0];
    out->z_mean = h[4] / h[0];
    out->finite = h[5] == 0.0 && std::isfinite(h[0]);
    out->reserved = 0;
    return DIRAC_OK;
}

dirac_status dirac3_get_spinor(dirac3_solver* s, double* psi_host_out) {
    if (!s || !psi_host_out) return fail(DIRAC_E_ARG, "null solver or output");
    if (!s->has_state) return fail(DIRAC_E_STATE, "set the initial spinor first");
    const size_t N = (size_t)s->g.n1 * s->g.n2 * s->g.n3;
    char* b = s->base;
    if (s->prec == DIRAC_FP64) {
        D3_TRY(hipMemcpyAsync(psi_host_out, b + s->lay.psi, N * 64, hipMemcpyDeviceToHost, s->stream), "download");
    } else {
        D3_TRY(launch_f32_to_c128(reinterpret_cast<const float*>(b + s->lay.psi),
                                  reinterpret_cast<double*>(b + s->lay.scratch), 8 * N, s->stream), "convert spinor");
        D3_TRY(hipMemcpyAsync(psi_host_out, b + s->lay.scratch, N * 64, hipMemcpyDeviceToHost, s->stream), "download");
    }
    D3_TRY(hipStreamSynchronize(s->stream), "synchronise");
    return DIRAC_OK;
}

dirac_status dirac3_destroy(dirac3_solver* s) {
    if (!s) return fail(DIRAC_E_ARG, "null solver");
    (void)hipStreamSynchronize(s->stream);
    drop_graph3(s);
    for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
    delete s;
    return DIRAC_OK;
}

}  // extern "C"
