"""Degenerate inputs on the GPU, for every scheme: zero steps leave the state
and the step counter exactly as they were, the zero state stays exactly zero
(every stage is linear in psi: Steps 1/5 multiply by E, the transforms and
the symbol are linear, the blend mixes two zero fields), negative step
counts are refused, and the observables of the zero state are zero and
flagged finite."""
import numpy as np
import pytest

from paper_1909_02894_amd import workloads as W
from tests.test_gpu_em import potentials

pytestmark = pytest.mark.gpu

KINDS = [("plain", 0), ("plain", 1), ("step2bis", 0), ("potentials", 0), ("scheme1", 0)]


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_02894_amd import dirac
    return dirac


def make(D, kind, prec):
    spec = W.curved_bump(n=64, seed=11, steps=0, m=0.5)
    kw = {}
    if kind == "step2bis":
        kw["scheme"] = D.SCHEME_EXP_SPLIT_2BIS
    elif kind == "potentials":
        kw["potentials"] = potentials(spec)
    elif kind == "scheme1":
        kw["scheme"] = D.SCHEME_CN_GMRES
    print(f"[edges] {kind} prec={prec} n=64", flush=True)
    return spec, D.Solver.from_spec(spec, precision=prec, **kw)


def stored(psi, prec):
    # the state as the solver holds it: FP32 solves round the upload once
    return psi if prec == 0 else psi.astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("kind,prec", KINDS)
def test_zero_steps_change_nothing(D, kind, prec):
    spec, s = make(D, kind, prec)
    psi0 = W.initial_spinor(spec)
    s.set_initial_spinor(psi0)
    s.step_n(0)
    assert np.array_equal(s.get_spinor(), stored(psi0, prec))
    assert s.observables()["step"] == 0
    s.step_n(3)
    after = s.get_spinor()
    s.step_n(0)
    assert np.array_equal(s.get_spinor(), after)
    assert s.observables()["step"] == 3
    with pytest.raises(D.DiracError):
        s.step_n(-1)
    assert np.array_equal(s.get_spinor(), after)
    s.close()


@pytest.mark.parametrize("kind,prec", KINDS)
def test_zero_state_stays_exactly_zero(D, kind, prec):
    spec, s = make(D, kind, prec)
    zero = np.zeros_like(W.initial_spinor(spec))
    s.set_initial_spinor(zero)
    s.step_n(4)
    got = s.get_spinor()
    assert np.all(got == 0)
    ob = s.observables()
    assert ob["step"] == 4 and ob["finite"] == 1
    assert ob["norm_l2"] == 0.0 and ob["norm_w"] == 0.0
    s.close()
