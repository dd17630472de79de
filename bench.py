"""Throughput of the directional-split Dirac step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-variants] [--skip-cpu]

Headline workload (the largest single-GPU configuration): 256 independent
curved-graphene-shaped solves advanced together by the batch engine, FP32
(tables generated in FP64 and rounded once, FP64 reductions).  Solve i draws
its grid size n uniformly from {128, 256, 512} (n x n points on [-20,20)^2,
absorbing layer of n/16 points per side, type I, sigma0 = 1, theta = 0), its
bump h = A exp(-r^2/s^2) (A in [0.5, 2], s in [2, 6]) and its packet momentum
from seed 4000 + i; massless, c = 1, dt = 0.01.  ~460 MiB of state, beyond the
256 MB Infinity Cache; inputs resident in HBM when the timed region starts.
One "step" = one time step (Step 1 + x + y + Step 5) of every solve; the K
timed steps are one replay of the run's HIP graph.  Kernel durations for the
roofline come from a second pass with per-launch HIP events.

Variants beside it: the same batch in FP64, the curved 512^2 solve (FP64 and
FP32), the flat 2048^2 precision workload (FP32 and FP64, 5000 steps), flat and
curved single solves beyond the Infinity Cache, the second-order step, Scheme I,
potentials, 3-D, and Poisson serving (p50/p99 latency).

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


def time_solve(D, spec, precision, steps, warmup, timed_steps, scheme=0, keep_state=False):
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
    state = s.get_spinor() if keep_state else None
    # per-launch durations in the real x, y order: every launch carries its own
    # start/stop events on the solver's stream (kernel execution time)
    kms, cnt = s.step_n_timed(timed_steps)
    kus = [1e3 * kms[d] / max(1, cnt[d]) for d in (0, 1)]
    # the same kernels replayed alone (each direction's data stays in its XCD's L2)
    iso = s.time_directions(min(timed_steps, 200))
    sched = (s.schedule(0), s.schedule(1))
    wt = s.store_mode()
    s.close()
    return dict(ms=ms, wall=wall, obs=obs, kernel_us=kus, isolated_us=iso, sched=sched, write_through=wt,
                state=state)


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
    sz = 8 if precision == 0 else 4
    working = N * (8 * sz if kind != "curved" else 13 * sz)       # state + per-point tables
    bound = "hbm" if working > INFINITY_CACHE_BYTES else "cache-resident"
    return {"bound": bound, "working_set_bytes": working, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
            "kernel": name, "avg_launch_us": round(avg[dom] * 1e3, 3),
            "algorithmic_bytes_per_launch": byt,
            "x_avg_us": round(avg[0] * 1e3, 3), "y_avg_us": round(avg[1] * 1e3, 3),
            "timing": "hipExtLaunchKernel start/stop events per launch, x/y alternating as in the run",
            "isolated_us": [round(u, 3) for u in r["isolated_us"]]}


BATCH_SIZES = (128, 256, 512)
INFINITY_CACHE_BYTES = 256 << 20


def batch_kernel_name(precision: int, d: int, n, sched: int | None) -> str:
    t = "double" if precision == 0 else "float"
    if n == "multi":
        return f"batch_multi_kernel<{t}, {'true' if d else 'false'}>"
    return f"batch_group_kernel<{t}, {'true' if d else 'false'}, {n}, {sched}>"


def batch_schedule_index(radix: int, cpt: int, n: int) -> int:
    """The batch kernel's schedule template argument for (radix, components):
    schedules 0/1 use the default radix (4 for n <= 64, else 8), 2/3 the other;
    odd schedules carry one component per thread."""
    default = 4 if n <= 64 else 8
    return (0 if radix == default else 2) + (1 if cpt == 1 else 0)


def bench_batch(D, W, precision, steps, warmup, timed_steps, count=256, direct=False):
    """The batch workload: autotuned schedules, `warmup` untimed steps, the
    graph of the K-step run recorded and instantiated untimed, then the timed
    replay (HIP events on the batch stream).  A second pass of `timed_steps`
    steps launches every phase kernel with its own start/stop events for the
    per-kernel durations."""
    import torch
    specs = W.batch_mix(count, 4000, BATCH_SIZES, steps)
    b = D.Batch(precision=precision, capacity=count)
    if direct:
        b.set_graph(False)          # one launch per phase kernel (counter passes)
    solvers = []
    for sp in specs:
        s = D.Solver.from_spec(sp, precision=precision, stream=b.stream)
        s.set_initial_spinor(W.initial_spinor(sp))
        b.add(s)
        solvers.append(s)
    b.autotune(5)                   # schedule per (direction, n), states restored
    sched = {n: [b.schedule(n, 0), b.schedule(n, 1)] for n in BATCH_SIZES}
    if warmup > 0:
        b.run([warmup] * count)
    b.prepare([steps] * count)      # record + instantiate the K-step graph (untimed)
    b.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.run([steps] * count)          # graph replay
    e1.record(b.stream)
    b.sync()
    ms = e0.elapsed_time(e1)
    cls = b.run_timed([timed_steps] * count)
    fin = all(s.observables()["finite"] for s in solvers[::16])
    b.close()
    pts = sum(sp.n1 * sp.n2 for sp in specs)
    sz = 8 if precision == 0 else 4
    step_bytes = 22 * sz * pts                         # x 13 sz + y 9 sz per point (curved)
    classes = {}
    for (d, n), (kms, cnt, byt) in cls.items():
        avg_us = 1e3 * kms / cnt
        bpl = byt / cnt
        sc = None if n == "multi" else batch_schedule_index(sched[n][d][0], sched[n][d][2], n)
        classes[f"{'xy'[d]}_{n}"] = {
            "kernel": batch_kernel_name(precision, d, n, sc), "launches": cnt, "avg_launch_us": round(avg_us, 2),
            "algorithmic_bytes_per_launch": round(bpl), "achieved_GBs": round(bpl / (avg_us * 1e-6) / 1e9, 1),
            "frac": round(bpl / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "total_ms": round(kms, 3)}
    dom = max(classes, key=lambda k: classes[k]["total_ms"])
    dc = classes[dom]
    phase = {}
    for d in "xy":
        ks = [c for k, c in classes.items() if k.startswith(d)]
        tb = sum(c["algorithmic_bytes_per_launch"] * c["launches"] for c in ks)
        tt = sum(c["total_ms"] for c in ks) * 1e-3
        phase[d] = round(tb / tt / 1e9 / HBM_PEAK_GBS, 4)
    tr = load_batch_traffic(dc["kernel"])
    roof = {"bound": "hbm", "achieved": dc["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dc["frac"], "traffic": tr, "kernel": dc["kernel"], "avg_launch_us": dc["avg_launch_us"],
            "algorithmic_bytes_per_launch": dc["algorithmic_bytes_per_launch"],
            "bytes_per_point": {"x": 13 * sz, "y": 9 * sz},
            "timing": f"{timed_steps} steps of direct launches, each with its own hipExtLaunchKernel start/stop "
                      "events on the batch stream (x and y phases in the order of a real run)",
            "kernels": classes, "phase_frac": phase,
            "step_frac": round(step_bytes * steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "step_timing": (f"direct launches of {steps} steps (the timed region)" if direct else
                            f"one HIP graph replay of {steps} steps (the timed region)")}
    hist = {str(n): sum(1 for sp in specs if sp.n1 == n) for n in BATCH_SIZES}
    return {"value": pts * steps / (ms * 1e-3), "ms": ms, "ms_per_step": ms / steps, "dtype": "f64" if sz == 8 else "f32",
            "solves": count, "points": pts, "state_bytes": pts * 4 * sz, "grid_sizes": hist, "finite": fin,
            "schedules": {str(n): v for n, v in sched.items()}, "roofline": roof}


def measure_copy_peak(torch, nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """A plain device-to-device copy of `nbytes` (torch's copy_, which runs the
    runtime's copy kernel), best of `reps`: the streaming rate this part reaches
    for a read + write mix, next to the nominal HBM peak."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(2 * nbytes / (best * 1e-3) / 1e9, 1),
            "what": f"device-to-device copy of {nbytes >> 20} MiB (read + write), best of {reps}"}


def load_batch_traffic(kernel: str):
    """HBM bytes per launch of a batch phase kernel from rocprofv3 FETCH_SIZE /
    WRITE_SIZE (profiles/traffic.json, key batch_kernels), or None when absent or
    taken on other kernel sources."""
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
    rec = d.get("batch_kernels", {}).get(kernel)
    return None if rec is None else dict(rec, instantiation=kernel)


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


VARIANTS = {"batch_256_fp64", "curved_512_fp64", "curved_512_fp32", "flat_2048_precision", "flat_4096_fp32",
            "flat_4096_fp64", "curved_2048_fp64", "curved_4096_fp32", "step2bis_corrected_fp64", "scheme1_cn_gmres",
            "scheme1_cn_gmres_2048", "em_potentials_fp64", "fp32_3d_flat_256", "fp64_3d_curved_128", "serve_poisson"}


def progress(msg: str):
    """One line on stderr before each GPU stage, so a failing run names its stage."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def single_variant(D, spec, kind, precision, steps, warmup, timed, note, keep_state=False):
    r = time_solve(D, spec, precision, steps, warmup, timed, keep_state=keep_state)
    out = {"value": spec.n1 * spec.n2 * steps / (r["ms"] * 1e-3), "unit": "grid-point*steps/s",
           "ms_per_step": r["ms"] / steps, "steps": steps, "dtype": "f64" if precision == 0 else "f32",
           "grid": [spec.n1, spec.n2], "note": note, "roofline": roofline_for(spec, kind, precision, r),
           "schedule": {"x": r["sched"][0], "y": r["sched"][1], "write_through_mask": r["write_through"]},
           "launch_mode": "HIP graph replay of 32-step chunks (value); direct launches with per-launch events "
                          "(kernel durations)"}
    return out, r.get("state")


def _oracle_solve(job):
    """One solve of the oracle for `steps` steps in a worker process; returns its
    grid-point*steps and the monotonic start/end times of the stepping loop."""
    sp, steps = job
    from oracle import dirac_oracle as O
    from paper_1909_02894_amd import workloads as W
    from tests.helpers import oracle_problem
    T = O.build_tables(oracle_problem(sp))
    psi = W.initial_spinor(sp)
    t0 = time.perf_counter()
    O.run(psi, T, steps)
    return sp.n1 * sp.n2 * steps, t0, time.perf_counter()


def cpu_baseline_batch(W, steps, workers):
    """The oracle on a bounded sample of the batch workload: the first `workers`
    solves of the batch, `steps` steps each, one single-threaded process per
    solve over the host cores (forked before anything touches the GPU); the rate
    is their total grid-point*steps over the wall time from the first start to
    the last end of a stepping loop."""
    import multiprocessing
    specs = W.batch_mix(256, 4000, BATCH_SIZES, steps)
    sample = specs[:workers]
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_solve, [(sp, steps) for sp in sample], chunksize=1)
    work = sum(r[0] for r in res)
    secs = max(r[2] for r in res) - min(r[1] for r in res)
    sizes = {n: sum(1 for sp in sample if sp.n1 == n) for n in BATCH_SIZES}
    return {"value": work / secs, "unit": "grid-point*steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{steps} steps of each of the first {workers} solves of the 256-solve batch (seeds "
                      f"4000-{4000 + workers - 1}; " + ", ".join(f"{c} of {n}x{n}" for n, c in sizes.items()) +
                      "), one single-threaded process per solve (NumPy complex128, pocketfft); the host has "
                      f"{os.cpu_count()} logical CPUs", "seconds": round(secs, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--skip-variants", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--variants", default=None,
                    help="comma-separated variant names to run (default: all)")
    ap.add_argument("--cpu-steps", type=int, default=250)
    ap.add_argument("--batch-direct", action="store_true",
                    help="run the batch with one launch per phase kernel instead of graph replay (counter passes)")
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
    from paper_1909_02894_amd import workloads as W
    cpu = None
    if not args.skip_cpu and not args.copy_calibration:
        # the host leg first: its worker processes are forked before the GPU is initialised
        progress("oracle on the host")
        cpu = cpu_baseline_batch(W, args.cpu_steps, min(16, os.cpu_count() or 1))
    import torch
    from paper_1909_02894_amd import dirac as D

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
    K = args.steps
    timed = max(1, min(K, 50))
    progress(f"headline: batch of 256 curved solves, FP32, {K} steps")
    hb = bench_batch(D, W, D.FP32, K, args.warmup, timed, direct=args.batch_direct)
    out = {
        "metric": "grid-point*steps/s on 1 MI355X (FP32 vs FP64), % HBM peak; p50/p99 latency",
        "value": hb["value"],
        "unit": "grid-point*steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": hb["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch of 256 independent curved-bump solves (seeds 4000+i, n uniform over "
                               "{128,256,512}, n x n on [-20,20)^2, n/16-point type-I layer, m=0, dt=0.01), FP32, "
                               "one HIP graph per run",
                   "solves": hb["solves"], "grid_sizes": hb["grid_sizes"], "points": hb["points"],
                   "state_bytes": hb["state_bytes"], "schedules": hb["schedules"]},
        "roofline": hb["roofline"],
    }
    cp = measure_copy_peak(torch)
    cp["frac_of_copy"] = round(hb["roofline"]["achieved"] / cp["GBs"], 4)
    out["roofline"]["copy"] = cp
    variants = {}
    chosen = None if args.variants is None else set(args.variants.split(","))
    want = lambda k: not args.skip_variants and (chosen is None or k in chosen)
    if want("batch_256_fp64"):
        progress("variant: the same batch in FP64")
        h64 = bench_batch(D, W, D.FP64, K, args.warmup, timed)
        variants["batch_256_fp64"] = {k: h64[k] for k in ("value", "ms_per_step", "dtype", "state_bytes", "schedules",
                                                           "finite", "roofline")}
        variants["batch_256_fp64"]["fp32_speedup"] = round(hb["value"] / h64["value"], 3)
    spec512 = W.curved_bump(n=512, seed=1909, steps=2000)
    if want("curved_512_fp64"):
        progress("variant: curved 512x512 FP64, 2000 steps")
        variants["curved_512_fp64"], _ = single_variant(
            D, spec512, "curved", D.FP64, 2000, args.warmup, 500,
            "curved bump 512x512, seed 1909, 32-point type-I layer, m=0, dt=0.01 (~20 MB working set)")
    if want("curved_512_fp32"):
        progress("variant: curved 512x512 FP32, 2000 steps")
        variants["curved_512_fp32"], _ = single_variant(
            D, spec512, "curved", D.FP32, 2000, args.warmup, 500, "the same solve in FP32")
    if want("flat_2048_precision"):
        flat = W.flat_small(n=2048, steps=5000)
        progress("variant: flat 2048x2048 FP32, 5000 steps")
        v32, s32 = single_variant(D, flat, "flat", D.FP32, 5000, 0, 100,
                                  "flat 2048x2048 packet solve, 5000 steps (precision workload)", keep_state=True)
        progress("variant: flat 2048x2048 FP64, 5000 steps")
        v64, s64 = single_variant(D, flat, "flat", D.FP64, 5000, 0, 100, "the same solve in FP64", keep_state=True)
        diff = float(np.linalg.norm((s32 - s64).ravel()) / np.linalg.norm(s64.ravel()))
        mx = float(np.abs(s32 - s64).max() / np.abs(s64).max())
        del s32, s64
        variants["flat_2048_fp32"] = v32
        variants["flat_2048_fp64"] = v64
        variants["flat_2048_precision"] = {
            "fp32_speedup": round(v32["value"] / v64["value"], 3),
            "fp32_vs_fp64_gpu_rel_l2_at_5000": diff, "fp32_vs_fp64_gpu_maxabs_over_max_at_5000": mx,
            "note": "both GPU paths after the same 5000 steps; against the exact discrete propagator the tests "
                    "bound FP32 by 1e-3 and FP64 by 1e-10 at step 5000, below the scheme's own time error (~1e-3)"}
    if want("flat_4096_fp32"):
        big = W.flat_small(n=4096, steps=200)
        progress("variant: flat 4096x4096 FP32")
        variants["flat_4096_fp32"], _ = single_variant(D, big, "flat", D.FP32, 200, 10, 100,
                                                       "flat 4096x4096 packet solve, 256 MiB state")
    if want("flat_4096_fp64"):
        big = W.flat_small(n=4096, steps=100)
        progress("variant: flat 4096x4096 FP64")
        variants["flat_4096_fp64"], _ = single_variant(D, big, "flat", D.FP64, 100, 10, 50,
                                                       "flat 4096x4096 packet solve, 512 MiB state")
    if want("curved_2048_fp64"):
        cb = W.curved_bump(n=2048, seed=1909, steps=200)
        progress("variant: curved 2048x2048 FP64")
        variants["curved_2048_fp64"], _ = single_variant(
            D, cb, "curved", D.FP64, 200, 10, 100, "curved bump 2048x2048 with a 128-point layer: 128 MiB state "
            "+ 160 MiB of per-point tables")
    if want("curved_4096_fp32"):
        cb = W.curved_bump(n=4096, seed=1909, steps=100)
        progress("variant: curved 4096x4096 FP32")
        variants["curved_4096_fp32"], _ = single_variant(
            D, cb, "curved", D.FP32, 100, 10, 50, "curved bump 4096x4096 with a 256-point layer: 256 MiB state "
            "+ 320 MiB of per-point tables")
    if want("step2bis_corrected_fp64"):
        progress("variant: second-order directional step FP64")
        N = spec512.n1 * spec512.n2
        rc = time_solve(D, spec512, D.FP64, 500, args.warmup, 100, scheme=D.SCHEME_EXP_SPLIT_2BIS)
        variants["step2bis_corrected_fp64"] = {
            "value": N * 500 / (rc["ms"] * 1e-3), "ms_per_step": rc["ms"] / 500, "dtype": "f64",
            "note": "second-order directional step (three inverse transforms per direction), curved 512x512",
            "x_avg_us": round(rc["kernel_us"][0], 3), "y_avg_us": round(rc["kernel_us"][1], 3),
            "roofline": variant_roofline(N, (120, 88), rc["kernel_us"],
                                         "x: state r/w 64 + E 32 + a 8 + gradient pair 16 B/pt; y: 64 + 8 + 16")}
    if want("scheme1_cn_gmres"):
        progress("variant: Scheme I")
        variants["scheme1_cn_gmres"] = bench_cn(D, spec512)
    if want("scheme1_cn_gmres_2048"):
        progress("variant: Scheme I, 2048x2048")
        cb = W.curved_bump(n=2048, seed=1909, steps=20, m=1.0)
        variants["scheme1_cn_gmres_2048"] = dict(bench_cn(D, cb, steps=20),
                                                 note="curved bump 2048x2048 FP64 (128 MiB state), separate "
                                                      "direction launches of the operator")
    if want("em_potentials_fp64"):
        progress("variant: potentials")
        variants["em_potentials_fp64"] = bench_em(D, W, spec512)
    if want("fp32_3d_flat_256"):
        progress("variant: 3-D 256^3 FP32")
        variants["fp32_3d_flat_256"] = bench_3d(D, W, 256, D.FP32, False)
    if want("fp64_3d_curved_128"):
        progress("variant: 3-D 128^3 FP64")
        variants["fp64_3d_curved_128"] = bench_3d(D, W, 128, D.FP64, True)
    if want("serve_poisson"):
        # serving at ~0.7x the measured batch capacity
        mean_work = np.mean([n * n for n in (64, 128, 256, 512, 1024)]) * (200 + 5000) / 2.0
        rate = 0.7 * hb["value"] / mean_work
        progress("variant: serving, 288 GB budget")
        variants["serve_poisson"] = bench_serve(100, rate, 288 << 30)
        progress("variant: serving, 2 GB budget")
        variants["serve_poisson_2GB"] = bench_serve(40, rate, 2 << 30, seed=5001)
        out["latency"] = {"p50_s": variants["serve_poisson"]["p50_s"],
                          "p99_s": variants["serve_poisson"]["p99_s"], "source": "serve_poisson"}
    out["variants"] = variants
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
