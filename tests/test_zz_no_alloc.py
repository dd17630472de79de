"""The allocation-free observables entry point (dirac_observables_static, for
callers that cannot allocate device memory) against dirac_observables: the same
kernels reduce into the library's static device scratch instead of the solver's
buffer, so every value must be bitwise equal.  Two calls in a row on the shared
scratch, the second on a smaller solve, then the first solve again."""
import ctypes as C

import numpy as np
import pytest

from paper_1909_02894_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_02894_amd import dirac
    return dirac


def both(D, s):
    a = D.Obs()
    b = D.Obs()
    D._check(D.lib.dirac_observables(s.h, C.byref(a)))
    D._check(D.lib.dirac_observables_static(s.h, C.byref(b)))
    return a.as_dict(), b.as_dict()


def test_static_observables_equal_buffer_observables(D):
    big = W.curved_bump(n=512, steps=10, m=0.5)
    small = W.paper_exp3(n=64, steps=5)
    sb = D.Solver.from_spec(big, precision=D.FP64)
    sb.set_initial_spinor(W.initial_spinor(big))
    sb.step_n(10)
    ss = D.Solver.from_spec(small, precision=D.FP32)
    ss.set_initial_spinor(W.initial_spinor(small))
    ss.step_n(5)
    for s in (sb, ss, sb):
        ref, got = both(D, s)
        assert ref == got, (ref, got)
        assert got["finite"] == 1 and got["norm_l2"] > 0
    # the static form leaves the state alone
    before = sb.get_spinor()
    D.observables_static(sb.h)
    assert np.array_equal(sb.get_spinor(), before)
    with pytest.raises(D.DiracError):
        D._check(D.lib.dirac_observables_static(None, C.byref(D.Obs())))
    sb.close()
    ss.close()
