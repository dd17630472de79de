"""GPU parity of the 3-D, 4-spinor step (three directions, Dirac
representation) against the 3-D oracle, the flat per-mode propagator and the
2-D GPU path (z-constant data).  Tolerances as in 2-D: FP64 1e-11, FP32 2e-5."""
import numpy as np
import pytest

from oracle import dirac_oracle as O
from oracle import dirac3_oracle as O3

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 2e-5


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_02894_amd import dirac
    return dirac


def packet3(p, k=(1.5, -0.5, 1.0), x0=(0.5, 0.0, -0.5), width=1.5):
    x, y, z = O.grid_points(p.n1, p.a1), O.grid_points(p.n2, p.a2), O.grid_points(p.n3, p.a3)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    g = np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2 + (Z - x0[2]) ** 2) / (2 * width ** 2)
               + 1j * (k[0] * X + k[1] * Y + k[2] * Z))
    return np.stack([g, 0.4 * g, 0.3j * g, -0.2 * g], axis=-1)


def gpu3(D, p, psi0, steps, precision=0, split=(), graph=True):
    f = p.fields
    fields = None if f is None else (f.phi, f.psi, *f.dphi, *f.dpsi)
    s = D.Solver3(p.n1, p.n2, p.n3, p.a1, p.a2, p.a3, p.dt, p.c, p.m, precision, p.metric, p.spin, fields,
                  p.pml_width, p.pml_type, p.pml_sigma0)
    s.set_launch_mode(graph, 4)
    s.set_initial_spinor(psi0)
    done = 0
    for k in sorted(set(split) | {steps}):
        s.step_n(k - done)
        done = k
    return s, s.get_spinor()


def test_3d_flat_matches_oracle_and_per_mode_propagator(D):
    p = O3.Problem3(n1=16, n2=16, n3=32, a1=6.0, a2=6.0, a3=8.0, dt=0.05, c=1.0, m=1.0)
    psi0 = packet3(p)
    _, g = gpu3(D, p, psi0, 12, split=(1,))
    assert O.rel_l2(g, O3.run3(psi0, O3.build_tables3(p), 12)) < TOL64
    assert O.rel_l2(g, O3.flat_exact_discrete3(psi0, p, 12)) < TOL64


@pytest.mark.parametrize("spin", [O.SPIN_PAPER, O.SPIN_2P1])
def test_3d_curved_rectangular_with_layer(D, spin):
    p = O3.Problem3(n1=32, n2=16, n3=64, a1=6.0, a2=5.0, a3=8.0, dt=0.04, c=1.1, m=0.8,
                    metric=O3.METRIC_PAPER_EXP3, spin=spin, pml_width=4)
    psi0 = packet3(p)
    s, g = gpu3(D, p, psi0, 20, split=(3,))
    T = O3.build_tables3(p)
    ref = O3.run3(psi0, T, 20)
    assert O.rel_l2(g, ref) < TOL64
    ob, ro = s.observables(), O3.observables3(ref, T)
    assert ob["step"] == 20 and ob["finite"] == 1
    for k in ("norm_l2", "norm_w", "x_mean", "y_mean", "z_mean"):
        assert abs(ob[k] - getattr(ro, k)) <= 1e-10 * max(1.0, abs(getattr(ro, k))), k
    # graph replay and direct launches give the same bits
    _, g2 = gpu3(D, p, psi0, 20, split=(3,), graph=False)
    assert np.array_equal(g, g2)


def test_3d_fp32(D):
    p = O3.Problem3(n1=64, n2=32, n3=32, a1=6.0, a2=5.0, a3=5.0, dt=0.04, c=1.0, m=1.0,
                    metric=O3.METRIC_PAPER_EXP3, spin=O.SPIN_PAPER, pml_width=3)
    psi0 = packet3(p)
    _, g = gpu3(D, p, psi0, 20, precision=D.FP32)
    assert O.rel_l2(g, O3.run3(psi0, O3.build_tables3(p), 20)) < TOL32


@pytest.mark.parametrize("shape", [(1024, 16, 16), (16, 1024, 16), (16, 16, 1024)])
def test_3d_longest_lines(D, shape):
    n1, n2, n3 = shape
    p = O3.Problem3(n1=n1, n2=n2, n3=n3, a1=20.0, a2=20.0, a3=20.0, dt=0.01, c=1.0, m=0.5, pml_width=5)
    rng = np.random.default_rng(n1 + 2 * n2)
    psi0 = rng.standard_normal((n3, n2, n1, 4)) + 1j * rng.standard_normal((n3, n2, n1, 4))
    _, g = gpu3(D, p, psi0, 3)
    assert O.rel_l2(g, O3.run3(psi0, O3.build_tables3(p), 3)) < TOL64


def test_3d_z_constant_data_equals_the_2d_solve(D):
    n1, n2, n3 = 64, 32, 16
    a1, a2, a3, dt, c, m = 6.0, 5.0, 4.0, 0.03, 1.0, 0.7
    p2 = O.Problem(n1=n1, n2=n2, a1=a1, a2=a2, dt=dt, c=c, m=m, metric=O.METRIC_PAPER_EXP3, spin=O.SPIN_PAPER,
                   pml_width=4)
    f2 = O.build_tables(p2).fields
    rep = lambda v: np.broadcast_to(v[None], (n3,) + v.shape).copy()
    z = np.zeros((n3, n2, n1))
    f3 = O3.Fields3(rep(f2.phi), rep(f2.psi), (rep(f2.phi_x), rep(f2.phi_y), z), (rep(f2.psi_x), rep(f2.psi_y), z))
    p3 = O3.Problem3(n1=n1, n2=n2, n3=n3, a1=a1, a2=a2, a3=a3, dt=dt, c=c, m=m, metric=O3.METRIC_FIELDS,
                     spin=O.SPIN_PAPER, fields=f3, pml_width=4)
    rng = np.random.default_rng(12)
    X, Y = np.meshgrid(O.grid_points(n1, a1), O.grid_points(n2, a2))
    g2 = np.exp(-(X ** 2 + Y ** 2) / 3.0 + 1j * (X - 0.5 * Y))
    psi2 = np.stack([g2, (0.3 + 0.2j) * g2], axis=-1)
    psi3 = np.zeros((n3, n2, n1, 4), complex)
    psi3[..., 0] = psi2[None, ..., 0]
    psi3[..., 3] = psi2[None, ..., 1]
    _, g3 = gpu3(D, p3, psi3, 15)
    s2 = D.Solver(n1, n2, a1, a2, dt, c, m, D.FP64, D.METRIC_PAPER_EXP3, D.SPIN_PAPER, pml_width=4)
    s2.set_initial_spinor(psi2)
    s2.step_n(15)
    out2 = s2.get_spinor()
    for k in range(n3):
        assert O.rel_l2(g3[k][..., [0, 3]], out2) < 1e-12
    assert np.max(np.abs(g3[..., 1:3])) < 1e-13
