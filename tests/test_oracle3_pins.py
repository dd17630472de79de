"""Pins of the 3-D, 4-spinor oracle against closed forms, library routines and
the (separately pinned) 2-D oracle."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import dirac_oracle as O
from oracle import dirac3_oracle as O3


def test_dirac_matrices_algebra():
    mats = list(O3.ALPHA) + [O3.BETA]
    for i, A in enumerate(mats):
        assert np.allclose(A @ A, O3.ID4)
        for B in mats[i + 1:]:
            assert np.allclose(A @ B + B @ A, 0)
    # alpha^i = Pi Lambda Pi^dag with Lambda = diag(1, 1, -1, -1)
    for A in O3.ALPHA:
        assert np.allclose(np.sort(np.linalg.eigvalsh(A)), [-1, -1, 1, 1])


@pytest.mark.parametrize("spin,m", [(O.SPIN_PAPER, 1.0), (O.SPIN_2P1, 0.3), (O.SPIN_NONE, 0.0), (O.SPIN_PAPER, 0.0)])
def test_half_step_exponential3_matches_expm(spin, m):
    p = O3.Problem3(n1=6, n2=4, n3=5, a1=5.0, a2=4.0, a3=6.0, dt=0.3, c=1.2, m=m, metric=O3.METRIC_PAPER_EXP3,
                    spin=spin)
    T = O3.build_tables3(p)
    f = T.fields
    dchi, _ = O3.spin_potential3(spin, f)
    for idx in np.ndindex(f.phi.shape):
        a = math.exp(f.phi[idx] - f.psi[idx])
        F = -0.5j * p.c * a * sum(dchi[k][idx] * O3.ALPHA[k] for k in range(3))
        H = math.exp(f.phi[idx]) * p.m * p.c * p.c * O3.BETA + F
        assert np.allclose(T.E[idx], scipy.linalg.expm(-0.5j * p.dt * H), atol=1e-14, rtol=0)


def test_flat_3d_stepping_equals_per_mode_expm():
    n1, n2, n3, a1, a2, a3, c, m, dt, steps = 8, 4, 8, 3.0, 2.0, 4.0, 1.1, 0.9, 0.13, 5
    p = O3.Problem3(n1=n1, n2=n2, n3=n3, a1=a1, a2=a2, a3=a3, dt=dt, c=c, m=m)
    rng = np.random.default_rng(4)
    psi0 = rng.standard_normal((n3, n2, n1, 4)) + 1j * rng.standard_normal((n3, n2, n1, 4))
    out = O3.run3(psi0, O3.build_tables3(p), steps)
    A = scipy.linalg.expm(-0.5j * dt * m * c * c * O3.BETA)
    P = np.fft.fftn(psi0, axes=(0, 1, 2))
    ref = np.empty_like(P)
    ps = [np.array([(q if q < n // 2 else q - n) for q in range(n)]) * math.pi / a
          for n, a in ((n1, a1), (n2, a2), (n3, a3))]
    for k3 in range(n3):
        for k2 in range(n2):
            for k1 in range(n1):
                U = A
                for i, k in enumerate((k1, k2, k3)):
                    U = scipy.linalg.expm(-1j * c * dt * ps[i][k] * O3.ALPHA[i]) @ U
                U = A @ U
                ref[k3, k2, k1] = np.linalg.matrix_power(U, steps) @ P[k3, k2, k1]
    ref = np.fft.ifftn(ref, axes=(0, 1, 2))
    assert O.rel_l2(out, ref) < 1e-13
    assert O.rel_l2(O3.flat_exact_discrete3(psi0, p, steps), ref) < 1e-13


def test_z_constant_solve_reduces_to_the_2d_scheme():
    # With data and fields constant in z, (psi_0, 0, 0, psi_3) evolves under
    # beta m + alpha_x p_x + alpha_y p_y restricted to that pair, i.e. the 2-D
    # equation sigma_x p_x + sigma_y p_y + sigma_z m; K_z(0) = I and the z blend
    # is the identity, so the 3-D scheme equals the 2-D scheme.
    n1, n2, n3, a1, a2, a3 = 16, 8, 4, 5.0, 4.0, 3.0
    dt, c, m = 0.05, 1.1, 0.7
    p2 = O.Problem(n1=n1, n2=n2, a1=a1, a2=a2, dt=dt, c=c, m=m, metric=O.METRIC_PAPER_EXP3, spin=O.SPIN_PAPER,
                   pml_width=2, pml_sigma0=0.8)
    T2 = O.build_tables(p2)
    f2 = T2.fields
    rep = lambda v: np.broadcast_to(v[None], (n3,) + v.shape).copy()
    z = np.zeros((n3, n2, n1))
    f3 = O3.Fields3(rep(f2.phi), rep(f2.psi), (rep(f2.phi_x), rep(f2.phi_y), z), (rep(f2.psi_x), rep(f2.psi_y), z))
    p3 = O3.Problem3(n1=n1, n2=n2, n3=n3, a1=a1, a2=a2, a3=a3, dt=dt, c=c, m=m, metric=O3.METRIC_FIELDS,
                     spin=O.SPIN_PAPER, fields=f3, pml_width=2, pml_sigma0=0.8)
    rng = np.random.default_rng(9)
    psi2 = rng.standard_normal((n2, n1, 2)) + 1j * rng.standard_normal((n2, n1, 2))
    psi3 = np.zeros((n3, n2, n1, 4), complex)
    psi3[..., 0] = psi2[None, ..., 0]
    psi3[..., 3] = psi2[None, ..., 1]
    out2 = O.run(psi2, T2, 6)
    out3 = O3.run3(psi3, O3.build_tables3(p3), 6)
    for k in range(n3):
        assert O.rel_l2(out3[k][..., [0, 3]], out2) < 1e-13
    assert np.max(np.abs(out3[..., 1:3])) < 1e-13


def test_massless_transport_along_z_is_an_exact_shift():
    n1, n2, n3, a = 4, 4, 32, 4.0
    h = 2 * a / n3
    p = O3.Problem3(n1=n1, n2=n2, n3=n3, a1=1.0, a2=1.0, a3=a, dt=h / 4, c=1.0, m=0.0)
    rng = np.random.default_rng(2)
    f = rng.standard_normal(n3) + 1j * rng.standard_normal(n3)
    psi = np.zeros((n3, n2, n1, 4), complex)
    for comp in ((1, 0, 1, 0), (0, 1, 0, -1)):          # alpha_z eigenvalue +1
        psi[:] = 0
        for k, v in enumerate(comp):
            psi[..., k] = v * f[:, None, None]
        out = O3.run3(psi, O3.build_tables3(p), 8)
        assert np.allclose(out, np.roll(psi, 2, axis=0), atol=1e-13)
    # eigenvalue -1 moves the other way
    for comp in ((1, 0, -1, 0), (0, 1, 0, 1)):
        psi[:] = 0
        for k, v in enumerate(comp):
            psi[..., k] = v * f[:, None, None]
        out = O3.run3(psi, O3.build_tables3(p), 8)
        assert np.allclose(out, np.roll(psi, -2, axis=0), atol=1e-13)


def test_3d_norms():
    p = O3.Problem3(n1=16, n2=8, n3=8, a1=5.0, a2=4.0, a3=4.0, dt=0.05, c=1.0, m=1.0)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((8, 8, 16, 4)) + 1j * rng.standard_normal((8, 8, 16, 4))
    T = O3.build_tables3(p)
    n0 = O3.observables3(psi, T).norm_l2
    assert abs(O3.observables3(O3.run3(psi, T, 10), T).norm_l2 / n0 - 1) < 1e-13
    # curved, no spin term, with layer, smooth data: the plain norm does not increase
    # (stability proposition; with a varying b the blend's bound holds for resolved data)
    pc = O3.Problem3(n1=32, n2=16, n3=16, a1=8.0, a2=8.0, a3=8.0, dt=0.05, c=1.0, m=1.0,
                     metric=O3.METRIC_PAPER_EXP3, spin=O.SPIN_NONE, pml_width=3)
    Tc = O3.build_tables3(pc)
    Z, Y, X = np.meshgrid(Tc.axes[2], Tc.axes[1], Tc.axes[0], indexing="ij")
    g = np.exp(-((X - 1) ** 2 + Y ** 2 + Z ** 2) / 4.0 + 1j * (1.5 * X - 0.5 * Z))
    psi = np.stack([g, 0.5 * g, 0.2j * g, 0 * g], axis=-1)
    prev = O3.observables3(psi, Tc).norm_l2
    for _ in range(5):
        psi = O3.step3(psi, Tc)
        cur = O3.observables3(psi, Tc).norm_l2
        assert cur <= prev * (1 + 1e-14)
        prev = cur
