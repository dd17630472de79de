"""Batched multi-solve engine: every solve in a mixed batch equals, bit for bit,
the same solve alone in a batch and the single-solve path with the batch radix;
and matches the FP64 oracle within the parity tolerances."""
import numpy as np
import pytest

from oracle import dirac_oracle as O
from paper_1909_02894_amd import workloads as W
from tests.helpers import oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_02894_amd import dirac
    return dirac


def batch_radix(n):
    return 4 if n <= 64 else 8


def mixed_specs():
    specs = []
    for i, n in enumerate((64, 128, 256, 128, 64, 512)):
        s = W.curved_bump(n=n, seed=4000 + i, steps=0, m=0.5 * (i % 3))
        specs.append(s)
    f = W.flat_small(n=128)
    specs.append(f)
    fp = W.flat_small(n=64)
    fp.pml_width = 6
    specs.append(fp)
    r = W.curved_bump(n=128, seed=77, steps=0)
    r.n2, r.a2, r.pml_width = 32, 6.0, 4                 # rectangular
    specs.append(r)
    return specs


def single_path(D, spec, prec, steps, radix=None):
    s = D.Solver.from_spec(spec, precision=prec)
    for d, n in ((0, spec.n1), (1, spec.n2)):
        r = batch_radix(n) if radix is None else radix[(n, d)]
        match = [(l, c) for (rr, l, c) in D.schedules(n, prec, d) if rr == r]
        if not match:
            return None                          # no single-solve schedule with this radix
        lines, cpt = match[0]
        s.set_schedule(d, r, lines, cpt)
    s.set_initial_spinor(W.initial_spinor(spec))
    s.step_n(steps)
    return s.get_spinor()


@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_batch_bitwise_and_oracle(D, prec):
    specs = mixed_specs()
    steps = [7, 12, 3, 12, 0, 5, 9, 12, 4]
    b = D.Batch(precision=prec, capacity=16)
    solvers, slots = [], []
    for sp in specs:
        s = D.Solver.from_spec(sp, precision=prec)
        s.set_initial_spinor(W.initial_spinor(sp))
        solvers.append(s)
        slots.append(b.add(s))
    b.run({sl: st for sl, st in zip(slots, steps)})
    b.sync()
    for sp, s, st in zip(specs, solvers, steps):
        got = s.get_spinor()
        assert s.observables()["step"] == st
        assert np.array_equal(got, single_path(D, sp, prec, st)), (sp.n1, sp.n2, st)
        ref = O.run(W.initial_spinor(sp), O.build_tables(oracle_problem(sp)), st)
        tol = 1e-11 if prec == 0 else 2e-5
        if st:
            assert O.rel_l2(got, ref) < tol, (sp.n1, sp.n2, st)
    # alone in a batch == in the mix
    alone = D.Batch(precision=prec, capacity=1)
    sp = specs[1]
    s = D.Solver.from_spec(sp, precision=prec)
    s.set_initial_spinor(W.initial_spinor(sp))
    alone.add(s)
    alone.run([steps[1]])
    alone.sync()
    assert np.array_equal(s.get_spinor(), solvers[1].get_spinor())


def test_graph_reuse_direct_mode_and_slot_changes(D):
    specs = mixed_specs()[:4]
    outs = {}
    for use_graph in (True, False):
        b = D.Batch(precision=1, capacity=8)
        b.set_graph(use_graph)
        sv = []
        for sp in specs:
            s = D.Solver.from_spec(sp, precision=1)
            s.set_initial_spinor(W.initial_spinor(sp))
            sv.append((b.add(s), s))
        for _ in range(3):                       # the same run three times: graph reused
            b.run({sl: 4 for sl, _ in sv})
        b.remove(sv[2][0])                       # drop one, add a fresh solve into its slot
        sp = specs[2]
        s_new = D.Solver.from_spec(sp, precision=1)
        s_new.set_initial_spinor(W.initial_spinor(sp))
        sl = b.add(s_new)
        b.run({sv[0][0]: 2, sv[1][0]: 5, sl: 6, sv[3][0]: 1})
        b.sync()
        outs[use_graph] = [sv[0][1].get_spinor(), sv[1][1].get_spinor(), s_new.get_spinor(), sv[3][1].get_spinor(),
                           sv[2][1].get_spinor()]
        assert sv[0][1].observables()["step"] == 14 and s_new.observables()["step"] == 6
    for a, c in zip(outs[True], outs[False]):
        assert np.array_equal(a, c)
    # segmented runs equal one long single-solve run
    assert np.array_equal(outs[True][1], single_path(D, specs[1], 1, 17))
    assert np.array_equal(outs[True][2], single_path(D, specs[2], 1, 6))


def test_batch_rejects_bad_input(D):
    b = D.Batch(precision=0, capacity=2)
    sp = W.curved_bump(n=64, steps=0)
    s32 = D.Solver.from_spec(sp, precision=1)
    s32.set_initial_spinor(W.initial_spinor(sp))
    with pytest.raises(D.DiracError):
        b.add(s32)                                # precision mismatch
    s = D.Solver.from_spec(sp, precision=0)
    with pytest.raises(D.DiracError) as ei:
        b.add(s)                                  # no initial state
    assert ei.value.status == -6
    s.set_initial_spinor(W.initial_spinor(sp))
    sl = b.add(s)
    with pytest.raises(D.DiracError):
        b.run([0, 3])                             # steps for a free slot
    with pytest.raises(D.DiracError):
        b.run([-1, 0])
    b.run([2, 0])
    b.sync()
    assert s.observables()["step"] == 2


def test_sixteen_seeded_solves_cover_every_size(D):
    # the batch workload's recipe (seeds 4000+i, n in {128, 256, 512}) on 16 solves,
    # 20 steps each, FP32 against the FP64 oracle
    specs = W.batch_mix(16, 4000, (128, 256, 512), 20)
    assert {sp.n1 for sp in specs} == {128, 256, 512}
    b = D.Batch(precision=D.FP32, capacity=16)
    solvers = []
    for sp in specs:
        s = D.Solver.from_spec(sp, precision=D.FP32, stream=b.stream)
        s.set_initial_spinor(W.initial_spinor(sp))
        b.add(s)
        solvers.append(s)
    b.run([20] * 16)
    b.sync()
    for sp, s in zip(specs, solvers):
        ref = O.run(W.initial_spinor(sp), O.build_tables(oracle_problem(sp)), 20)
        assert O.rel_l2(s.get_spinor(), ref) < 2e-5, (sp.n1, sp.seed)
    b.close()


def test_large_group_beside_merged_small_groups(D):
    # one size group big enough for its own launch (a 2048-point solve: 2048
    # tiles per phase) beside two small groups that share a multi-group launch;
    # every solve keeps the bits of the single-solve path with the batch radix
    specs = [W.curved_bump(n=2048, seed=4100, steps=0)]
    specs += [W.curved_bump(n=n, seed=4101 + i, steps=0) for i, n in enumerate((64, 128, 64))]
    steps = [3, 5, 2, 4]
    b = D.Batch(precision=D.FP32, capacity=8)
    solvers = []
    for sp in specs:
        s = D.Solver.from_spec(sp, precision=D.FP32, stream=b.stream)
        s.set_initial_spinor(W.initial_spinor(sp))
        b.add(s)
        solvers.append(s)
    b.run(steps + [0] * 4)
    b.sync()
    for sp, s, k in zip(specs, solvers, steps):
        ref = single_path(D, sp, D.FP32, k)
        assert ref is not None and np.array_equal(s.get_spinor(), ref), (sp.n1, k)
    b.close()


def test_full_batch_workload_sampled(D):
    # the full 256-solve, 1000-step FP32 batch as bench.py runs it (one graph);
    # the 128x128 solves among them are checked against the oracle at 1000 steps
    # (bound 2e-4), every solve is finite and its weighted norm stays bounded
    specs = W.batch_mix(256, 4000, (128, 256, 512), 1000)
    b = D.Batch(precision=D.FP32, capacity=256)
    solvers = []
    for sp in specs:
        s = D.Solver.from_spec(sp, precision=D.FP32, stream=b.stream)
        s.set_initial_spinor(W.initial_spinor(sp))
        b.add(s)
        solvers.append(s)
    b.run([1000] * 256)
    b.sync()
    small = [i for i, sp in enumerate(specs) if sp.n1 == 128][:3]
    for i in small:
        sp = specs[i]
        ref = O.run(W.initial_spinor(sp), O.build_tables(oracle_problem(sp)), 1000)
        assert O.rel_l2(solvers[i].get_spinor(), ref) < 2e-4, (sp.n1, sp.seed)
    for s in solvers[::17]:
        ob = s.observables()
        assert ob["finite"] == 1 and ob["step"] == 1000
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_every_batch_schedule_and_the_tuner(D, prec):
    # every valid (radix, components) schedule of every size gives the bits of
    # the single-solve kernel with that radix; the tuner restores the states
    specs = mixed_specs()
    steps = [5, 6, 3, 6, 2, 5, 4, 6, 4]
    sizes = sorted({(sp.n1, 0) for sp in specs} | {(sp.n2, 1) for sp in specs})
    for variant in range(4):
        b = D.Batch(precision=prec, capacity=16)
        radix = {}
        for n, d in sizes:
            cands = []
            for r in (8, 4):
                for c in (2, 1):
                    try:
                        b.set_schedule(n, d, r, c)
                        cands.append((r, c))
                    except D.DiracError:
                        pass
            assert len(cands) == D.lib.dirac_batch_schedule_count(n) and cands
            r, c = cands[variant % len(cands)]
            b.set_schedule(n, d, r, c)
            assert b.schedule(n, d)[0] == r and b.schedule(n, d)[2] == c
            radix[(n, d)] = r
        solvers = []
        for sp in specs:
            s = D.Solver.from_spec(sp, precision=prec, stream=b.stream)
            s.set_initial_spinor(W.initial_spinor(sp))
            b.add(s)
            solvers.append(s)
        if variant == 3:
            b.autotune(2)
            radix = {(n, d): b.schedule(n, d)[0] for n, d in sizes}
            assert all(s.observables()["step"] == 0 for s in solvers)
        b.run(steps)
        b.sync()
        for sp, s, st in zip(specs, solvers, steps):
            got, ref = s.get_spinor(), single_path(D, sp, prec, st, radix)
            if ref is not None:
                assert np.array_equal(got, ref), (variant, sp.n1, sp.n2)
            else:
                orc = O.run(W.initial_spinor(sp), O.build_tables(oracle_problem(sp)), st)
                assert O.rel_l2(got, orc) < (1e-11 if prec == 0 else 2e-5), (variant, sp.n1, sp.n2)
        b.close()
