// Drives the library's host logic the way the bench and the serving loop do (CPU, stub runtime).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <random>
#include "dirac.h"

#define OK(x) do { dirac_status s_ = (x); if (s_ != DIRAC_OK) { std::printf("FAIL %s: %d %s\n", #x, s_, dirac_last_error()); std::exit(1); } } while (0)

struct Buf { void* p; size_t n; Buf(size_t n) : n(n) { p = std::calloc(1, n + 4096); } ~Buf() { std::free(p); } };

static void solve2d(int n, int prec, int kind, int pml, int scheme, bool em, int steps) {
    dirac_grid g{n, n, 20.0, 20.0, 0.01, 1.0, 1.0};
    dirac_metric m{};
    m.kind = kind; m.spin = kind == DIRAC_METRIC_FLAT ? 0 : 2; m.bump_A = 1.0; m.bump_s = 3.0;
    dirac_pml p{pml, 1, 1.0, 0.0};
    dirac_scheme sc{scheme, 0, 0, 0, 0.0};
    std::vector<double> V((size_t)n * n, 0.1), Ax((size_t)n * n, 0.2);
    dirac_em e{V.data(), Ax.data(), nullptr, 1.0, {1, 0, 0, 0, 0, 0}, {0, 1, 3, 0, 0, 0}};
    size_t fb = dirac_footprint_bytes_ex(&g, &m, &p, prec, &sc, em ? &e : nullptr);
    if (!fb) { std::printf("footprint 0: %s\n", dirac_last_error()); std::exit(1); }
    Buf buf(fb);
    dirac_solver* s = nullptr;
    OK(dirac_create_solver(&g, &m, &p, prec, &sc, em ? &e : nullptr, buf.p, fb, nullptr, &s));
    std::vector<double> psi((size_t)n * n * 4, 0.0);
    OK(dirac_set_initial_spinor(s, psi.data()));
    if (scheme == 0 && !em) OK(dirac_autotune(s, 2));
    dirac_obs o{};
    if (scheme == DIRAC_SCHEME_CN_GMRES) {
        // Scheme I keeps its solve state on the device; the stub runs no kernel, so
        // the state read after the first cycle never shows convergence: the call
        // must fail cleanly and put the solver back as it was
        for (int k = 0; k < 2; ++k) {
            const dirac_status r = dirac_step_n(s, k ? steps : 5);
            if (r != DIRAC_OK && r != DIRAC_E_DEVICE) { std::printf("FAIL scheme I step: %d\n", r); std::exit(1); }
            OK(dirac_observables(s, &o));
            if (r != DIRAC_OK && o.step != 0) { std::printf("FAIL scheme I step count not restored\n"); std::exit(1); }
        }
    } else {
        OK(dirac_step_n(s, 5));
        OK(dirac_step_n(s, steps));
    }
    OK(dirac_observables(s, &o));
    OK(dirac_observables_static(s, &o));
    if (scheme != DIRAC_SCHEME_CN_GMRES) {
        double ms[2]; int64_t c[2];
        OK(dirac_step_n_timed(s, 50, ms, c));
        double us[2];
        OK(dirac_time_directions(s, 20, us));
        OK(dirac_set_launch_mode(s, 0, 8));
        OK(dirac_step_n(s, 20));
        OK(dirac_step_n_timed(s, 10, ms, c));
        if (em) {
            // both forms of the potentials' exponentials, tuned, stepped and timed
            for (int form : {1, 2, 0}) {
                OK(dirac_set_potential_form(s, form));
                OK(dirac_autotune(s, 2));
                OK(dirac_step_n(s, 7));
                OK(dirac_step_n_timed(s, 5, ms, c));
                OK(dirac_time_directions(s, 4, us));
            }
            int32_t pass = -1;
            OK(dirac_get_potential_form(s, &pass));
            if (pass != 1) { std::printf("FAIL potential form by size\n"); std::exit(1); }
            if (dirac_set_potential_form(s, 3) != DIRAC_E_ARG) { std::printf("FAIL form 3 accepted\n"); std::exit(1); }
        } else if (dirac_set_potential_form(s, 1) != DIRAC_E_ARG) {
            std::printf("FAIL potential form without potentials\n");
            std::exit(1);
        }
    }
    OK(dirac_get_spinor(s, psi.data()));
    OK(dirac_destroy(s));
}

static void solve3d(int n, int prec, int kind) {
    dirac3_grid g{n, n / 2, n, 5.0, 5.0, 5.0, 0.01, 1.0, 1.0};
    dirac3_metric m{};
    m.kind = kind; m.spin = 1;
    dirac_pml p{n / 16, 1, 1.0, 0.0};
    size_t fb = dirac3_footprint_bytes(&g, &m, &p, prec);
    if (!fb) { std::printf("3d footprint 0: %s\n", dirac_last_error()); std::exit(1); }
    Buf buf(fb);
    dirac3_solver* s = nullptr;
    OK(dirac3_create(&g, &m, &p, prec, buf.p, fb, nullptr, &s));
    std::vector<double> psi((size_t)n * (n / 2) * n * 8, 0.0);
    OK(dirac3_set_initial_spinor(s, psi.data()));
    OK(dirac3_step_n(s, 40));
    double ms[3]; int64_t c[3];
    OK(dirac3_step_n_timed(s, 10, ms, c));
    dirac3_obs o{};
    OK(dirac3_observables(s, &o));
    OK(dirac3_get_spinor(s, psi.data()));
    OK(dirac3_destroy(s));
}

struct Member { dirac_solver* s; Buf* buf; int slot; int remaining; };

static dirac_solver* make_batch_solver(int n, int prec, Buf*& buf) {
    dirac_grid g{n, n, 20.0, 20.0, 0.01, 1.0, 0.0};
    dirac_metric m{};
    m.kind = DIRAC_METRIC_GAUSS_BUMP; m.spin = 2; m.bump_A = 1.0; m.bump_s = 3.0;
    dirac_pml p{n / 16, 1, 1.0, 0.0};
    size_t fb = dirac_footprint_bytes(&g, &m, &p, prec);
    buf = new Buf(fb);
    dirac_solver* s = nullptr;
    OK(dirac_create_metric(&g, &m, &p, prec, buf->p, fb, nullptr, &s));
    std::vector<double> psi((size_t)n * n * 4, 0.0);
    OK(dirac_set_initial_spinor(s, psi.data()));
    return s;
}

static void batch_bench(int count, int prec) {
    size_t bb = dirac_batch_footprint_bytes(count);
    Buf buf(bb);
    dirac_batch* b = nullptr;
    OK(dirac_batch_create(prec, count, buf.p, bb, nullptr, &b));
    std::vector<Member> mem;
    std::mt19937 rng(4);
    const int sizes[3] = {32, 64, 128};
    for (int i = 0; i < count; ++i) {
        Member mm{};
        mm.s = make_batch_solver(sizes[rng() % 3], prec, mm.buf);
        OK(dirac_batch_add(b, mm.s, &mm.slot));
        mem.push_back(mm);
    }
    OK(dirac_batch_autotune(b, 2));
    std::vector<int64_t> steps(count, 30);
    OK(dirac_batch_prepare(b, steps.data()));
    OK(dirac_batch_run(b, steps.data()));       // replays the prepared graph
    OK(dirac_batch_run(b, steps.data()));       // graph reuse
    {
        double ms[18], byt[18];
        int64_t cnt[18];
        OK(dirac_batch_run_timed(b, steps.data(), ms, cnt, byt));
    }
    OK(dirac_batch_run(b, steps.data()));       // graph rebuilt after the timed run
    OK(dirac_batch_sync(b));
    OK(dirac_batch_set_graph(b, 0));
    OK(dirac_batch_run(b, steps.data()));
    OK(dirac_batch_set_graph(b, 1));
    for (auto& mm : mem) { OK(dirac_batch_remove(b, mm.slot)); OK(dirac_destroy(mm.s)); delete mm.buf; }
    OK(dirac_batch_destroy(b));
}

static void serve_loop(int capacity, int prec, int requests) {
    size_t bb = dirac_batch_footprint_bytes(capacity);
    Buf buf(bb);
    dirac_batch* b = nullptr;
    OK(dirac_batch_create(prec, capacity, buf.p, bb, nullptr, &b));
    std::mt19937 rng(5);
    const int sizes[5] = {16, 32, 64, 128, 256};
    std::vector<Member> running;
    int admitted = 0;
    while (admitted < requests || !running.empty()) {
        int arrivals = rng() % 4;
        for (int a = 0; a < arrivals && admitted < requests && (int)running.size() < capacity; ++a, ++admitted) {
            Member mm{};
            mm.s = make_batch_solver(sizes[rng() % 5], prec, mm.buf);
            OK(dirac_batch_add(b, mm.s, &mm.slot));
            mm.remaining = 10 + rng() % 200;
            running.push_back(mm);
        }
        if (running.empty()) continue;
        std::vector<int64_t> steps(capacity, 0);
        for (auto& mm : running) steps[mm.slot] = std::min(16, mm.remaining);
        OK(dirac_batch_run(b, steps.data()));
        OK(dirac_batch_sync(b));
        for (size_t i = 0; i < running.size();) {
            running[i].remaining -= (int)steps[running[i].slot];
            if (running[i].remaining <= 0) {
                OK(dirac_batch_remove(b, running[i].slot));
                OK(dirac_destroy(running[i].s));
                delete running[i].buf;
                running.erase(running.begin() + i);
            } else ++i;
        }
    }
    OK(dirac_batch_destroy(b));
}

int main() {
    for (int prec = 0; prec < 2; ++prec) {
        solve2d(128, prec, DIRAC_METRIC_GAUSS_BUMP, 8, 0, false, 100);
        solve2d(256, prec, DIRAC_METRIC_FLAT, 0, 0, false, 70);
        solve2d(128, prec, DIRAC_METRIC_GAUSS_BUMP, 8, DIRAC_SCHEME_EXP_SPLIT_2BIS, false, 70);
        solve2d(128, prec, DIRAC_METRIC_PAPER_EXP3, 0, DIRAC_SCHEME_EXP_SPLIT_2BIS_PRINTED, false, 70);
        solve2d(64, prec, DIRAC_METRIC_GAUSS_BUMP, 4, 0, true, 40);
        solve3d(32, prec, DIRAC_METRIC_PAPER_EXP3);
        solve3d(64, prec, DIRAC_METRIC_FLAT);
        std::printf("prec %d single solves ok\n", prec);
        fflush(stdout);
    }
    solve2d(64, 0, DIRAC_METRIC_GAUSS_BUMP, 4, DIRAC_SCHEME_CN_GMRES, false, 5);
    solve2d(64, 0, DIRAC_METRIC_GAUSS_BUMP, 4, DIRAC_SCHEME_CN_GMRES, true, 5);
    std::printf("scheme I ok\n");
    batch_bench(48, 1);
    batch_bench(20, 0);
    std::printf("batch ok\n");
    serve_loop(64, 1, 150);
    std::printf("serve ok\n");
    return 0;
}
