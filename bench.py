"""Throughput of the directional-split Dirac step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-variants] [--skip-cpu]

Workload (the curved-graphene-shaped solve): 512 x 512 periodic grid on
[-20,20)^2, static sheet over a Gaussian bump h = A exp(-r^2/s^2) with A, s
drawn from seed 1909, absorbing layer of 32 points per side (type I, sigma0 = 1,
theta = 0), massless, c = 1, dt = 0.01, Gaussian packet of width 2 at a seeded
momentum; the state starts resident in HBM.  One "step" = Step 1 + x + y +
Step 5 of the scheme over the whole grid.  The headline value is the FP64 path
(complex128 state); the FP32 path (FP64-generated tables, FP64 reductions) and
a large flat FP32 solve beyond the 256 MB Infinity Cache are reported beside it.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def bytes_per_point(kind: str, dir_: int, precision: int) -> int:
    """Algorithmic HBM bytes per grid point of one direction-kernel launch in the
    steady state (state read + written once; per-point tables read once; the
    O(n) per-axis tables are not counted).  x: psi r/w + E + a; y: psi r/w + a."""
    sz = 8 if precision == 0 else 4
    state = 2 * 4 * sz
    if kind == "flat":
        return state
    if kind == "flat_pml":
        return state
    return state + (4 * sz + sz if dir_ == 0 else sz)


def variant_roofline(npts: int, bytes_xy, us_xy, note: str):
    """HBM roofline of a variant's dominant direction kernel: algorithmic bytes
    per point (x, y) times the points of one launch over its measured duration."""
    dom = 0 if us_xy[0] >= us_xy[1] else 1
    ach = bytes_xy[dom] * npts / (us_xy[dom] * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": "xy"[dom] + "_stage", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_point": bytes_xy[dom],
            "avg_launch_us": round(us_xy[dom], 3), "note": note}


def load_traffic(name: str, instantiation: str | None = None):
    """HBM traffic per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (profiles/traffic.json), or None when absent or taken on other kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    from paper_1909_02894_amd.profiling import kernel_sources_digest
    if d.get("kernel_sources") != kernel_sources_digest():
        return None
    ent = d.get("kernels", {}).get(name)
    if ent is None:
        return None
    rec = ent.get("by_instantiation", {}).get(instantiation) if instantiation else None
    if rec is None:
        return None
    return dict(rec, instantiation=instantiation)


def time_solve(D, spec, precision, steps, warmup, timed_steps, scheme=0):
    import torch
    s = D.Solver.from_spec(spec, precision=precision, scheme=scheme)
    from paper_1909_02894_amd import workloads as W
    psi0 = torch.from_numpy(W.initial_spinor(spec).view(np.float64).copy()).cuda()
    s.set_initial_spinor_device(psi0)
    torch.cuda.synchronize()
    s.autotune(200)                  # warm-up part 1: pick the fastest schedules and store modes
    s.step_n(warmup)
    torch.cuda.synchronize()
    st = s.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    s.step_n(steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    obs = s.observables()
    # per-launch durations in the real x, y order: every launch carries its own
    # start/stop events on the solver's stream (kernel execution time)
    kms, cnt = s.step_n_timed(timed_steps)
    kus = [1e3 * kms[d] / max(1, cnt[d]) for d in (0, 1)]
    # the same kernels replayed alone (each direction's data stays in its XCD's L2)
    iso = s.time_directions(min(timed_steps, 200))
    sched = (s.schedule(0), s.schedule(1))
    wt = s.store_mode()
    s.close()
    return dict(ms=ms, wall=wall, obs=obs, kernel_us=kus, isolated_us=iso, sched=sched, write_through=wt)


def roofline_for(spec, kind, precision, r):
    N = spec.n1 * spec.n2
    avg = [r["kernel_us"][d] * 1e-3 for d in (0, 1)]           # ms per launch
    dom = 0 if avg[0] >= avg[1] else 1
    byt = bytes_per_point(kind, dom, precision) * N
    achieved = byt / (avg[dom] * 1e-3) / 1e9
    name = f"{'x' if dom == 0 else 'y'}_stage_{'f64' if precision == 0 else 'f32'}_{spec.n1}x{spec.n2}_{kind}"
    rr, ll, cc = r["sched"][dom]
    mode = {"flat": 0, "flat_pml": 1, "curved": 2}[kind]
    inst = (f"stage_kernel<{'double' if precision == 0 else 'float'}, {spec.n1 if dom == 0 else spec.n2}, {rr}, "
            f"{ll}, {'true' if dom == 1 else 'false'}, {mode}, {cc}>")
    tr = load_traffic(name, inst)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
            "kernel": name, "avg_launch_us": round(avg[dom] * 1e3, 3),
            "algorithmic_bytes_per_launch": byt,
            "x_avg_us": round(avg[0] * 1e3, 3), "y_avg_us": round(avg[1] * 1e3, 3),
            "timing": "hipExtLaunchKernel start/stop events per launch, x/y alternating as in the run",
            "isolated_us": [round(u, 3) for u in r["isolated_us"]]}


def bench_batch(D, W, count=256, steps=1000):
    """Many independent curved solves of mixed size advanced by the batch engine:
    one graph launch for the whole run (timed on its second, graph-reusing run)."""
    import torch
    specs = W.batch_mix(count, 4000, (128, 256, 512), steps)
    b = D.Batch(precision=D.FP32, capacity=count)
    solvers = []
    for sp in specs:
        s = D.Solver.from_spec(sp, precision=D.FP32, stream=b.stream)
        s.set_initial_spinor(W.initial_spinor(sp))
        b.add(s)
        solvers.append(s)
    b.autotune(5)                   # schedule per (direction, n), states restored
    sched = {str(n): [b.schedule(n, 0), b.schedule(n, 1)] for n in (128, 256, 512)}
    b.run([steps] * count)          # builds and replays the graph
    b.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.run([steps] * count)          # the same run: graph reused
    e1.record(b.stream)
    b.sync()
    ms = e0.elapsed_time(e1)
    pts = sum(sp.n1 * sp.n2 for sp in specs)
    fin = all(s.observables()["finite"] for s in solvers[:8])
    algo = 88.0 * pts * steps
    hist = {n: sum(1 for sp in specs if sp.n1 == n) for n in (128, 256, 512)}
    b.close()
    return {"value": pts * steps / (ms * 1e-3), "unit": "grid-point*steps/s", "dtype": "f32",
            "solves": count, "steps": steps, "grid_sizes": hist, "ms": ms, "finite": fin, "schedules": sched,
            "step_roofline": {"bound": "hbm", "achieved": round(algo / (ms * 1e-3) / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              "bytes_per_point_step": 88,
                              "state_bytes": pts * 16}}


def bench_cn(D, spec, steps=40):
    """Scheme I (Crank-Nicolson transport + device GMRES) on the same workload."""
    import torch
    from paper_1909_02894_amd import workloads as W
    s = D.Solver.from_spec(spec, precision=D.FP64, scheme=D.SCHEME_CN_GMRES, gmres_restart=20, gmres_rtol=1e-12)
    s.set_initial_spinor(W.initial_spinor(spec))
    s.step_n(3)
    it0, _ = s.cn_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_n(steps)                  # synchronous: the host drives the Krylov iteration
    dt = time.perf_counter() - t0
    it1, res = s.cn_stats()
    s.close()
    return {"value": spec.n1 * spec.n2 * steps / dt, "unit": "grid-point*steps/s", "dtype": "f64",
            "steps": steps, "ms_per_step": dt * 1e3 / steps, "gmres_iterations_per_step": (it1 - it0) / steps,
            "gmres_restart": 20, "gmres_rtol": 1e-12, "last_relative_residual": res}


def bench_3d(D, W, n, precision, curved, steps=40, warmup=4):
    """The 3-D, 4-spinor step on an n^3 grid (graph replay), with per-launch kernel
    times of the x, y, z kernels from dispatch-attached events.  Algorithmic bytes
    per point and launch: state read + write (8 T each way), plus the
    exponential record (6 FP64 / 8 FP32) and a in the x kernel, a in y and z."""
    import torch
    a = 10.0
    s = D.Solver3(n, n, n, a, a, a, 0.01, 1.0, 1.0, precision,
                  D.METRIC_PAPER_EXP3 if curved else D.METRIC_FLAT, D.SPIN_PAPER if curved else D.SPIN_NONE,
                  pml_width=n // 16 if curved else 0)
    psi0 = W.gaussian_packet3(n, n, n, a, a, a, (-2.0, 0.0, 1.0), (2.0, 1.0, -1.0), 2.0, (1.0, 0.5, 0.0, 0.2j))
    s.set_initial_spinor(psi0)
    del psi0
    s.step_n(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step_n(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms, cnt = s.step_n_timed(10)
    fin = s.observables()["finite"]
    s.close()
    N = n ** 3
    sz = 8 if precision == 0 else 4
    per = [16 * sz + ((6 if sz == 8 else 8) * sz + sz if curved else 0)] + [16 * sz + (sz if curved else 0)] * 2
    us = [1e3 * kms[d] / cnt[d] for d in range(3)]
    dom = max(range(3), key=lambda d: us[d])
    ach = per[dom] * N / (us[dom] * 1e-6) / 1e9
    return {"value": N * steps / (ms * 1e-3), "unit": "grid-point*steps/s", "dtype": "f64" if sz == 8 else "f32",
            "grid": [n, n, n], "metric": "paper_exp3 3-D, layer n/16" if curved else "flat",
            "ms_per_step": ms / steps, "finite": bool(fin),
            "kernel_us": {"x": round(us[0], 2), "y": round(us[1], 2), "z": round(us[2], 2)},
            "roofline": {"bound": "hbm", "kernel": "xyz"[dom] + "_stage_3d", "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "bytes_per_point": per[dom]}}


def bench_em(D, W, spec, steps=500):
    """Scheme II with time-dependent potentials (in-kernel exponential per step)."""
    import torch
    X, Y = np.meshgrid(-spec.a1 + (2 * spec.a1 / spec.n1) * np.arange(spec.n1),
                       -spec.a2 + (2 * spec.a2 / spec.n2) * np.arange(spec.n2))
    pot = {"V": 0.5 * np.exp(-(X ** 2 + Y ** 2) / 50.0), "Ax": np.zeros_like(X), "Ay": None, "charge": 1.0,
           "env_V": (1.0, 0.0, 0.0, 0.0, 0.0, 0.0), "env_A": (0.0, 0.8, 3.0, 0.0, 5.0, 2.0)}
    pot["Ax"][:] = 1.0
    s = D.Solver.from_spec(spec, precision=D.FP64, potentials=pot)
    s.set_initial_spinor(W.initial_spinor(spec))
    s.autotune(50)                   # store modes (the state and step counter are restored)
    s.step_n(10)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step_n(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms, cnt = s.step_n_timed(100)
    s.close()
    return {"value": spec.n1 * spec.n2 * steps / (ms * 1e-3), "unit": "grid-point*steps/s", "dtype": "f64",
            "ms_per_step": ms / steps, "note": "Gaussian scalar potential and a uniform laser-like vector "
            "potential pulse; exponential rebuilt per point and step", "x_avg_us": round(1e3 * kms[0] / cnt[0], 3),
            "y_avg_us": round(1e3 * kms[1] / cnt[1], 3),
            "roofline": variant_roofline(spec.n1 * spec.n2, (128, 72), [1e3 * kms[d] / cnt[d] for d in (0, 1)],
                                         "x: state r/w 64 + the 64-byte point record, y: 64 + a 8 B/pt; the x "
                                         "kernel is ALU-bound (FP64 exponential per point, twice)")}


def bench_serve(count, rate, budget, quantum=64, seed=5000):
    from paper_1909_02894_amd import serve as S
    reqs = S.make_requests(count, rate, seed=seed)
    srv = S.Server(precision=1, budget_bytes=budget, capacity=512, quantum=quantum)
    st = srv.run(reqs)
    srv.close()
    return {"requests": st.requests, "rate_per_s": round(rate, 3), "budget_bytes": budget, "quantum": quantum,
            "p50_s": round(st.p50_s, 4), "p99_s": round(st.p99_s, 4), "mean_s": round(st.mean_s, 4),
            "throughput": st.throughput, "unit": "grid-point*steps/s", "wall_s": round(st.wall_s, 3),
            "max_running": st.max_running, "quanta": st.quanta, "peak_arena_bytes": st.peak_arena_bytes}


def cpu_baseline(spec, steps):
    from oracle import dirac_oracle as O
    from paper_1909_02894_amd import workloads as W
    from tests.helpers import oracle_problem
    T = O.build_tables(oracle_problem(spec))
    psi = W.initial_spinor(spec)
    t0 = time.perf_counter()
    O.run(psi, T, steps)
    dt = time.perf_counter() - t0
    return {"value": spec.n1 * spec.n2 * steps / dt, "unit": "grid-point*steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the same {spec.n1}x{spec.n2} curved solve (NumPy complex128, "
                      f"single-threaded pocketfft); host has {os.cpu_count()} logical CPUs",
            "seconds": round(dt, 2)}


VARIANTS = {"fp32_same_workload", "fp32_flat_4096", "step2bis_corrected_fp64", "scheme1_cn_gmres",
            "em_potentials_fp64", "fp32_3d_flat_256", "fp64_3d_curved_128", "batch_256_mixed", "serve_poisson"}


def progress(msg: str):
    """One line on stderr before each GPU stage, so a failing run names its stage."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--skip-variants", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--variants", default=None,
                    help="comma-separated variant names to run (default: all; serve_poisson needs batch_256_mixed)")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB three times (counter calibration)")
    args = ap.parse_args()
    if args.variants is not None and not set(args.variants.split(",")) <= VARIANTS:
        print(f"unknown variants: {sorted(set(args.variants.split(',')) - VARIANTS)}; known: {sorted(VARIANTS)}",
              file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); a multi-GPU form of this solver is "
              "not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1909_02894_amd import dirac as D
    from paper_1909_02894_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": 1 << 30, "copies": 3}), flush=True)
        return
    spec = W.curved_bump(n=512, seed=1909, steps=args.steps)
    K = args.steps
    timed = min(K, 500)
    progress(f"headline: curved 512x512 FP64, {K} steps")
    r64 = time_solve(D, spec, D.FP64, K, args.warmup, timed)
    N = spec.n1 * spec.n2
    value = N * K / (r64["ms"] * 1e-3)
    out = {
        "metric": "grid-point*steps/s on 1 MI355X (FP32 vs FP64), % HBM peak; p50/p99 latency",
        "value": value,
        "unit": "grid-point*steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "curved bump 512x512, seed 1909, 32-point type-I layer, m=0, dt=0.01, FP64",
                   "grid": [spec.n1, spec.n2], "bump_A": round(spec.bump_A, 6), "bump_s": round(spec.bump_s, 6),
                   "k0": [round(k, 6) for k in spec.k0],
                   "schedule": {"x": r64["sched"][0], "y": r64["sched"][1], "write_through_mask": r64["write_through"]}},
        "roofline": roofline_for(spec, "curved", D.FP64, r64),
    }
    variants = {}
    # --variants a,b: only those (e.g. for counter passes); the serving runs need the batch's rate
    chosen = None if args.variants is None else set(args.variants.split(","))
    want = lambda k: not args.skip_variants and (chosen is None or k in chosen)
    if want("fp32_same_workload"):
        progress("variant: same workload FP32")
        r32 = time_solve(D, spec, D.FP32, K, args.warmup, timed)
        variants["fp32_same_workload"] = {
            "value": N * K / (r32["ms"] * 1e-3), "ms_per_step": r32["ms"] / K, "dtype": "f32",
            "roofline": roofline_for(spec, "curved", D.FP32, r32),
            "schedule": {"x": r32["sched"][0], "y": r32["sched"][1], "write_through_mask": r32["write_through"]}}
    if want("fp32_flat_4096"):
        big = W.flat_small(n=4096, steps=200)
        progress("variant: flat 4096x4096 FP32")
        rb = time_solve(D, big, D.FP32, 200, 10, 100)
        variants["fp32_flat_4096"] = {
            "value": big.n1 * big.n2 * 200 / (rb["ms"] * 1e-3), "ms_per_step": rb["ms"] / 200, "dtype": "f32",
            "note": "flat 4096x4096 packet solve, 256 MiB state (beyond the Infinity Cache)",
            "roofline": roofline_for(big, "flat", D.FP32, rb),
            "schedule": {"x": rb["sched"][0], "y": rb["sched"][1], "write_through_mask": rb["write_through"]}}
    if want("step2bis_corrected_fp64"):
        progress("variant: second-order directional step FP64")
        rc = time_solve(D, spec, D.FP64, 500, args.warmup, 100, scheme=D.SCHEME_EXP_SPLIT_2BIS)
        variants["step2bis_corrected_fp64"] = {
            "value": N * 500 / (rc["ms"] * 1e-3), "ms_per_step": rc["ms"] / 500, "dtype": "f64",
            "note": "second-order directional step (three inverse transforms per direction), same workload",
            "x_avg_us": round(rc["kernel_us"][0], 3), "y_avg_us": round(rc["kernel_us"][1], 3),
            "roofline": variant_roofline(N, (120, 88), rc["kernel_us"],
                                         "x: state r/w 64 + E 32 + a 8 + gradient pair 16 B/pt; y: 64 + 8 + 16")}
    if want("scheme1_cn_gmres"):
        progress("variant: Scheme I")
        variants["scheme1_cn_gmres"] = bench_cn(D, spec)
    if want("em_potentials_fp64"):
        progress("variant: potentials")
        variants["em_potentials_fp64"] = bench_em(D, W, spec)
    if want("fp32_3d_flat_256"):
        progress("variant: 3-D 256^3 FP32")
        variants["fp32_3d_flat_256"] = bench_3d(D, W, 256, D.FP32, False)
    if want("fp64_3d_curved_128"):
        progress("variant: 3-D 128^3 FP64")
        variants["fp64_3d_curved_128"] = bench_3d(D, W, 128, D.FP64, True)
    if want("batch_256_mixed"):
        progress("variant: batch of 256 solves")
        bt = bench_batch(D, W)
        variants["batch_256_mixed"] = bt
        if want("serve_poisson"):
            # serving at ~0.7x the measured batch capacity
            mean_work = np.mean([n * n for n in (64, 128, 256, 512, 1024)]) * (200 + 5000) / 2.0
            rate = 0.7 * bt["value"] / mean_work
            progress("variant: serving, 288 GB budget")
            variants["serve_poisson"] = bench_serve(100, rate, 288 << 30)
            progress("variant: serving, 2 GB budget")
            variants["serve_poisson_2GB"] = bench_serve(40, rate, 2 << 30, seed=5001)
            out["latency"] = {"p50_s": variants["serve_poisson"]["p50_s"],
                              "p99_s": variants["serve_poisson"]["p99_s"], "source": "serve_poisson"}
    out["variants"] = variants
    if not args.skip_cpu:
        progress("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
