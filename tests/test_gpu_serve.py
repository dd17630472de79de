"""Continuous-batching server: every request's result equals, bit for bit, the
same request served alone; admission respects the memory budget."""
import numpy as np
import pytest

from oracle import dirac_oracle as O
from paper_1909_02894_amd import workloads as W
from tests.helpers import oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_02894_amd import serve
    return serve


def small_requests(S, count, rate, seed=5000):
    return S.make_requests(count, rate, seed=seed, sizes=(64, 128, 256), steps_range=(20, 90))


@pytest.mark.parametrize("policy", ["share", "srpt"])
def test_served_equals_alone_and_oracle(S, policy):
    # srpt with a fill target of one 128^2 grid: most quanta leave solves waiting
    reqs = small_requests(S, 14, 400.0)
    srv = S.Server(precision=1, budget_bytes=1 << 30, capacity=8, quantum=16, keep_results=True, policy=policy,
                   fill_points=128 * 128)
    st = srv.run(reqs)
    srv.close()
    assert st.requests == len(reqs) and st.max_running > 1
    for r in reqs:
        alone = S.Server(precision=1, budget_bytes=256 << 20, capacity=1, quantum=16, keep_results=True)
        one = S.Request(r.rid, 0.0, r.spec, r.steps)
        alone.run([one])
        alone.close()
        assert np.array_equal(one.result, r.result), r.rid
    # and the FP32 results sit within the FP32 parity tolerance of the FP64 oracle
    for r in reqs[:3]:
        ref = O.run(W.initial_spinor(r.spec), O.build_tables(oracle_problem(r.spec)), r.steps)
        assert O.rel_l2(r.result, ref) < 2e-5


def test_small_budget_queues_requests(S):
    from paper_1909_02894_amd import dirac as D
    reqs = small_requests(S, 10, 2000.0, seed=7)
    big = max(D.footprint_bytes(*D.spec_structs(r.spec)[:3], D.FP32) for r in reqs)
    srv = S.Server(precision=1, budget_bytes=2 * big + 4096, capacity=16, quantum=16)
    st = srv.run(reqs)
    srv.close()
    assert st.requests == 10
    assert st.peak_arena_bytes <= 2 * big + 4096
    assert st.max_running <= 2 or st.peak_arena_bytes <= st.budget_bytes


