"""GPU parity at the largest grids (FP64 4096^2, FP32 8192^2) and for every
compiled schedule of several sizes.

At the largest sizes the reference is analytic: a superposition of a few
Fourier modes (including the Nyquist index) evolves under the flat scheme as
U(xi)^n per mode (U = A K_y K_x A, the oracle's per-mode step matrix), which the
test evaluates at a random sample of grid points without any full-size
transform.  Tolerances: FP64 1e-11, FP32 2e-5 after 20 steps (relative to the
largest value, over the sample)."""
import math

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


MODES = [((3, -2), (1.0, 0.5j)), ((-17, 40), (0.3, -0.7)), ((-1, 1), (0.2 + 0.1j, 0.4))]


def mode_field(n1, n2, a1, a2, modes, idx=None):
    x, y = O.grid_points(n1, a1), O.grid_points(n2, a2)
    if idx is None:
        X, Y = np.meshgrid(x, y)
    else:
        X, Y = x[idx[1]], y[idx[0]]
    out = np.zeros(X.shape + (2,), complex)
    for (p1, p2), c in modes:
        ph = np.exp(1j * (p1 * math.pi / a1 * X + p2 * math.pi / a2 * Y))
        out += ph[..., None] * np.asarray(c)
    return out


@pytest.mark.parametrize("prec,n", [(0, 4096), (1, 8192)])
def test_largest_grids_against_per_mode_propagator(D, prec, n):
    a, dt, m, steps = 20.0, 0.002, 1.0, 20
    modes = MODES + [((-n // 2, 7), (0.25, 0.25j))]             # the Nyquist index along x
    spec = W.flat_small(n=n, steps=steps)
    spec.dt = dt
    psi0 = mode_field(n, n, a, a, modes)
    s = D.Solver.from_spec(spec, precision=prec)
    s.set_initial_spinor(psi0)
    del psi0
    s.step_n(steps)
    g = s.get_spinor()
    rng = np.random.default_rng(n)
    idx = (rng.integers(0, n, 4096), rng.integers(0, n, 4096))
    evolved = []
    for (p1, p2), c in modes:
        U = O.flat_step_matrix(p1 * math.pi / a, p2 * math.pi / a, m, 1.0, dt)
        evolved.append(((p1, p2), np.linalg.matrix_power(U, steps) @ np.asarray(c)))
    ref = mode_field(n, n, a, a, evolved, idx)
    err = np.abs(g[idx[0], idx[1]] - ref).max() / np.abs(ref).max()
    assert err < (1e-11 if prec == 0 else 2e-5), err
    ob = s.observables()
    assert ob["finite"] == 1 and ob["step"] == steps


@pytest.mark.parametrize("prec", [0, 1])
def test_every_schedule_of_several_sizes(D, prec):
    # curved with layer, rectangular so that each direction has its own size;
    # every compiled schedule of each direction against the oracle, and bitwise
    # equal within one radix
    for n1, n2 in ((64, 1024), (256, 128)):
        spec = W.curved_bump(n=n1, steps=2, m=1.0)
        spec.n2, spec.a2, spec.pml_width = n2, 20.0, 8
        ref = O.run(W.initial_spinor(spec), O.build_tables(oracle_problem(spec)), 2)
        for d, n in ((0, n1), (1, n2)):
            by_radix = {}
            for (r, lines, cpt) in D.schedules(n, prec, d):
                s = D.Solver.from_spec(spec, precision=prec)
                s.set_schedule(d, r, lines, cpt)
                s.set_initial_spinor(W.initial_spinor(spec))
                s.step_n(2)
                out = s.get_spinor()
                assert O.rel_l2(out, ref) < (1e-11 if prec == 0 else 5e-6), (n1, n2, d, r, lines, cpt)
                if r in by_radix:
                    assert np.array_equal(out, by_radix[r]), (n1, n2, d, r, lines, cpt)
                by_radix[r] = out
                s.close()
