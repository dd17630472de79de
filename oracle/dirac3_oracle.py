"""Plain FP64 CPU oracle for the 3-D, 4-spinor form of the directional-split
pseudospectral step (Numerical Scheme II, Sec. 5.2, with three directions).

TEST INFRASTRUCTURE ONLY: only ``tests/`` may import this module.  It shares
no code with the HIP library.  It reuses the 2-D oracle's grid, transform and
layer helpers (``oracle.dirac_oracle``).

Array convention: a spinor field has shape ``(n3, n2, n1, 4)`` -- axis 0 is z,
axis 1 is y, axis 2 is x, axis 3 the spinor component in the Dirac
representation: beta = diag(1, 1, -1, -1), alpha^i = [[0, sigma_i], [sigma_i, 0]]
(so alpha^i = Pi^i Lambda Pi^{i,dag} with Lambda = diag(1, 1, -1, -1), Sec. 5.2).

The step (eqs. (op_split_curved), (poly_mod), (second_scheme) in 3-D):
    psi <- E psi,  E = exp(-i dt/2 [beta m c^2 e^Phi + F]),
    for i = x, y, z:  psi <- b_i F_i^{-1}[K_i F_i psi] + (1 - b_i) psi,
                      K_i = exp(-i c dt xi alpha^i) = cos I - i sin alpha^i,
                      b_i = a / S^i,
    psi <- E psi,
with a = e^{Phi - Psi} and F = -i c a (alpha . grad chi) / 2 (R5 in 3-D: the same
spin selector).  Because beta and the alpha^i anticommute and square to I, the
exponent M = -i w beta + g . alpha (w = (dt/2) m c^2 e^Phi, g = -(dt/4) c a
grad chi) has M^2 = (|g|^2 - w^2) I and E = C I + D M with the real C, D of R6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from oracle import dirac_oracle as O

S = (O.SIGMA_X, O.SIGMA_Y, O.SIGMA_Z)
Z2 = np.zeros((2, 2), dtype=np.complex128)
ALPHA = tuple(np.block([[Z2, s], [s, Z2]]) for s in S)
BETA = np.diag([1, 1, -1, -1]).astype(np.complex128)
ID4 = np.eye(4, dtype=np.complex128)

METRIC_FLAT, METRIC_PAPER_EXP3, METRIC_FIELDS = 0, 2, 3


@dataclass
class Fields3:
    phi: np.ndarray
    psi: np.ndarray
    dphi: tuple          # (d_x, d_y, d_z) Phi
    dpsi: tuple          # (d_x, d_y, d_z) Psi


@dataclass
class Problem3:
    n1: int
    n2: int
    n3: int
    a1: float
    a2: float
    a3: float
    dt: float
    c: float = 1.0
    m: float = 1.0
    metric: int = METRIC_FLAT
    spin: int = O.SPIN_NONE
    fields: Fields3 | None = None
    pml_width: int = 0
    pml_type: int = 1
    pml_sigma0: float = 1.0


@dataclass
class Tables3:
    prob: Problem3
    axes: tuple          # grid points (x, y, z)
    h: tuple
    xi: tuple            # wavenumbers per axis
    fields: Fields3
    a: np.ndarray        # (n3, n2, n1)
    b: tuple             # b_x, b_y, b_z, each (n3, n2, n1)
    E: np.ndarray        # (n3, n2, n1, 4, 4)
    K: tuple             # per axis (n_i, 4, 4)
    chi: np.ndarray


def metric_fields3(kind: int, X, Y, Z, fields: Fields3 | None = None) -> Fields3:
    """FLAT; PAPER_EXP3 in three dimensions (Phi = exp(-0.01 |x|^2),
    Psi = exp(-0.005 |x|^2), |x|^2 = x^2 + y^2 + z^2); FIELDS given."""
    z = np.zeros_like(X)
    if kind == METRIC_FLAT:
        return Fields3(z, z.copy(), (z, z, z), (z, z, z))
    if kind == METRIC_PAPER_EXP3:
        r2 = X * X + Y * Y + Z * Z
        phi = np.exp(-0.01 * r2)
        psi = np.exp(-0.005 * r2)
        return Fields3(phi, psi, (-0.02 * X * phi, -0.02 * Y * phi, -0.02 * Z * phi),
                       (-0.01 * X * psi, -0.01 * Y * psi, -0.01 * Z * psi))
    if kind == METRIC_FIELDS:
        assert fields is not None
        return fields
    raise ValueError(f"unknown 3-D metric kind {kind}")


def spin_potential3(spin: int, f: Fields3):
    if spin == O.SPIN_NONE:
        z = np.zeros_like(f.phi)
        return (z, z, z), z
    if spin == O.SPIN_PAPER:
        return f.dphi, f.phi
    if spin == O.SPIN_2P1:
        return tuple(p + q for p, q in zip(f.dphi, f.dpsi)), f.phi + f.psi
    raise ValueError(f"unknown spin selector {spin}")


def half_step_exponential3(f: Fields3, spin: int, m: float, c: float, dt: float) -> np.ndarray:
    """E = exp(M), M = -i w beta + g . alpha, closed form C I + D M (module docstring)."""
    dchi, _ = spin_potential3(spin, f)
    a = np.exp(f.phi - f.psi)
    w = 0.5 * dt * m * c * c * np.exp(f.phi)
    g = [-(dt / 4.0) * c * a * d for d in dchi]
    s2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2 - w * w
    r = np.sqrt(np.abs(s2))
    small = np.abs(s2) < 1e-8
    with np.errstate(invalid="ignore", divide="ignore"):
        C = np.where(s2 >= 0, np.cosh(r), np.cos(r))
        D = np.where(s2 >= 0, np.sinh(r) / r, np.sin(r) / r)
    C = np.where(small, 1.0 + s2 / 2.0 + s2 * s2 / 24.0, C)
    D = np.where(small, 1.0 + s2 / 6.0 + s2 * s2 / 120.0, D)
    M = (-1j * w[..., None, None] * BETA + g[0][..., None, None] * ALPHA[0]
         + g[1][..., None, None] * ALPHA[1] + g[2][..., None, None] * ALPHA[2])
    return C[..., None, None] * ID4 + D[..., None, None] * M


def directional_symbol3(xi: np.ndarray, c: float, dt: float, axis: int) -> np.ndarray:
    """Pi^i exp(-i c dt Lambda xi) Pi^{i,dag} = cos(c dt xi) I - i sin(c dt xi) alpha^i."""
    th = c * dt * xi
    return np.cos(th)[:, None, None] * ID4 - 1j * np.sin(th)[:, None, None] * ALPHA[axis]


# array axis of each spatial direction (x, y, z) in an (n3, n2, n1, 4) field
ARRAY_AXIS = (2, 1, 0)


def build_tables3(p: Problem3) -> Tables3:
    x = O.grid_points(p.n1, p.a1)
    y = O.grid_points(p.n2, p.a2)
    z = O.grid_points(p.n3, p.a3)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    f = metric_fields3(p.metric, X, Y, Z, p.fields)
    a = np.exp(f.phi - f.psi)
    inv = [O.pml_inverse_stretch(n, aa, p.pml_width, p.pml_type, p.pml_sigma0, 0.0).real
           for n, aa in ((p.n1, p.a1), (p.n2, p.a2), (p.n3, p.a3))]
    b = (a * inv[0][None, None, :], a * inv[1][None, :, None], a * inv[2][:, None, None])
    xi = (O.wavenumbers(p.n1, p.a1), O.wavenumbers(p.n2, p.a2), O.wavenumbers(p.n3, p.a3))
    _, chi = spin_potential3(p.spin, f)
    return Tables3(p, (x, y, z), (2 * p.a1 / p.n1, 2 * p.a2 / p.n2, 2 * p.a3 / p.n3), xi, f, a, b,
                   half_step_exponential3(f, p.spin, p.m, p.c, p.dt),
                   tuple(directional_symbol3(xi[i], p.c, p.dt, i) for i in range(3)), chi)


def directional_stage3(psi: np.ndarray, axis: int, K: np.ndarray, b: np.ndarray) -> np.ndarray:
    """psi* = b F_i^{-1}[K(xi) F_i psi] + (1 - b) psi along spatial axis `axis`."""
    ax = ARRAY_AXIS[axis]
    P = O.partial_dft(psi, ax)
    P = np.moveaxis(P, ax, -2)                     # (..., n_i, 4)
    P = np.einsum("qab,...qb->...qa", K, P)
    P = np.moveaxis(P, -2, ax)
    Xi = O.partial_idft(P, ax)
    return b[..., None] * Xi + (1.0 - b[..., None]) * psi


def apply_pointwise3(M: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return np.einsum("...ab,...b->...a", M, psi)


def step3(psi: np.ndarray, T: Tables3) -> np.ndarray:
    s = apply_pointwise3(T.E, psi)                 # Step 1
    for i in range(3):                             # x, y, z
        s = directional_stage3(s, i, T.K[i], T.b[i])
    return apply_pointwise3(T.E, s)                # Step 5


def run3(psi0: np.ndarray, T: Tables3, nsteps: int) -> np.ndarray:
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        psi = step3(psi, T)
    return psi


@dataclass
class Observables3:
    norm_l2: float
    norm_w: float
    x_mean: float
    y_mean: float
    z_mean: float
    finite: bool


def observables3(psi: np.ndarray, T: Tables3) -> Observables3:
    """h1 h2 h3 sum |psi|^2, the weighted norm with w = e^{chi - Phi + Psi} (the 3-D
    form of the conserved weight, same integration by parts), mean position."""
    dens = np.sum(np.abs(psi) ** 2, axis=-1)
    dV = T.h[0] * T.h[1] * T.h[2]
    w = np.exp(T.chi - T.fields.phi + T.fields.psi)
    Z, Y, X = np.meshgrid(T.axes[2], T.axes[1], T.axes[0], indexing="ij")
    tot = dens.sum()
    return Observables3(float(dV * tot), float(dV * np.sum(w * dens)), float(np.sum(X * dens) / tot),
                        float(np.sum(Y * dens) / tot), float(np.sum(Z * dens) / tot),
                        bool(np.all(np.isfinite(psi))))


def flat_exact_discrete3(psi0: np.ndarray, p: Problem3, nsteps: int) -> np.ndarray:
    """The flat 3-D scheme's output after nsteps per Fourier mode:
    U(xi) = A K_z K_y K_x A with A = exp(-i dt m c^2 beta / 2), raised to nsteps."""
    xi = (O.wavenumbers(p.n1, p.a1), O.wavenumbers(p.n2, p.a2), O.wavenumbers(p.n3, p.a3))
    mu = p.dt * p.m * p.c * p.c / 2.0
    A = np.diag(np.exp(-1j * mu * np.diag(BETA).real))
    P = np.fft.fftn(psi0, axes=(0, 1, 2))
    out = np.empty_like(P)
    for k3 in range(p.n3):
        for k2 in range(p.n2):
            for k1 in range(p.n1):
                Ks = [math.cos(p.c * p.dt * xi[i][k]) * ID4 - 1j * math.sin(p.c * p.dt * xi[i][k]) * ALPHA[i]
                      for i, k in enumerate((k1, k2, k3))]
                U = A @ Ks[2] @ Ks[1] @ Ks[0] @ A
                out[k3, k2, k1] = np.linalg.matrix_power(U, nsteps) @ P[k3, k2, k1]
    return np.fft.ifftn(out, axes=(0, 1, 2))
