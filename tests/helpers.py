"""Test-side glue: turns a workload spec into an oracle problem."""
from oracle import dirac_oracle as O


def oracle_problem(s, fields=None, step2=0, potentials=None) -> "O.Problem":
    """potentials: the dict Solver(potentials=...) takes (V, Ax, Ay, charge, env_V, env_A)."""
    em = None
    if potentials is not None:
        import numpy as np
        z = np.zeros((s.n2, s.n1))
        pv = dict(potentials)
        em = O.EMPotentials(pv.get("V") if pv.get("V") is not None else z,
                            pv.get("Ax") if pv.get("Ax") is not None else z,
                            pv.get("Ay") if pv.get("Ay") is not None else z,
                            pv.get("charge", 1.0), O.Envelope(*pv.get("env_V", (1.0, 0, 0, 0, 0, 0))),
                            O.Envelope(*pv.get("env_A", (1.0, 0, 0, 0, 0, 0))))
    return O.Problem(n1=s.n1, n2=s.n2, a1=s.a1, a2=s.a2, dt=s.dt, c=s.c, m=s.m, metric=s.metric,
                     spin=s.spin, bump_A=s.bump_A, bump_s=s.bump_s, fields=fields,
                     pml_width=s.pml_width, pml_type=s.pml_type, pml_sigma0=s.pml_sigma0,
                     pml_theta=s.pml_theta, step2=step2, em=em)


def oracle_checkpoints(spec, checkpoints, psi0=None):
    """The oracle's states of a workload spec at the given step counts (one pass)."""
    from paper_1909_02894_amd import workloads as W
    T = O.build_tables(oracle_problem(spec))
    psi = W.initial_spinor(spec) if psi0 is None else psi0
    out, done = {}, 0
    for c in sorted(set(checkpoints)):
        psi = O.run(psi, T, c - done)
        done = c
        out[c] = psi
    return out


def oracle_final_many(specs_steps, workers=6):
    """oracle_checkpoints(spec, [steps])[steps] for each (spec, steps), computed in
    separate processes (spawned: they import NumPy and the oracle only)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=max(1, min(workers, len(specs_steps))),
                             mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(oracle_checkpoints, sp, [st]) for sp, st in specs_steps]
        return [f.result()[st] for f, (_, st) in zip(futs, specs_steps)]


def max_rel(a, ref):
    """max_k |a_k - ref_k| / max_k |ref_k|."""
    import numpy as np
    return float(np.abs(a - ref).max() / np.abs(ref).max())
