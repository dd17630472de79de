"""Plain FP64 CPU oracle for the directional-split pseudospectral step (Numerical
Scheme II) of the 2-D static curved-space Dirac equation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library.

Everything here is NumPy complex128 / float64, written for a reader to check it
against the paper by eye: no blocking, fusion or reordering beyond what the
paper's definitions state.  Array convention: a spinor field has shape
``(n2, n1, 2)`` -- axis 0 is y (index j), axis 1 is x (index i), axis 2 is the
spinor component.

Paper sections followed (Antoine, Fillion-Gourdeau, Lorin, McLean,
arXiv:1909.02894):

* grid, momenta and the partial DFT pair F_i / F_i^{-1}: Sec. 5 (space
  discretisation), the definitions of D_N^(x), D_N^(xi) and the partial
  Fourier coefficients;
* spectral derivative [[d_i]]: Sec. 5, eq. (trick);
* Strang splitting with half-step exponentials: Sec. 4.2, eq.
  (op_split_curved), and Step 1 / Step 3 of Scheme I, eqs. (step1), (step3);
* closed-form exponential of a Dirac-matrix combination: Sec. 4.1, eq.
  (exp_dirac), generalised to complex coefficients (see ``half_step_exponential``);
* directional splitting with alpha(x) = a(x) alpha: Sec. 5.2, eqs.
  (alpha_form), (poly_mod);
* the exponential directional step: Sec. 5.2, eq. (second_scheme);
* PML stretch a^i -> a^i / S^i: Sec. 3, eq. (pml2) and the remark after
  eq. (poly_mod); absorbing profiles types I-VI: Sec. 3;
* 2-D static metric equation: Sec. 6, Numerical Experiment 3, and Appendix A;
* differentiation matrix: Appendix B, eq. (spectral_rep_final).

Readings of silent or garbled passages (both this oracle and the HIP path use
them):

* R1 the Fourier-space transport factor is exp(-i c dt alpha^i xi^i), i.e.
  the directional symbol of eq. (second_scheme) (the flat eq. (split) prints
  the opposite sign in the exponent);
* R2 directions are applied x then y in every step, as printed in (poly_mod);
* R3 the Nyquist index p = -n/2 keeps xi = -n pi / (2a) in every symbol;
* R4 the absorbing layer is L* <= |x| <= L with L = a and L* = a - w h
  (w = layer width in points); the distance to the periodic seam is measured
  in whole grid steps, d_k = min(k, n - k), so |x_k| - L = -d_k h; the
  singular types III-VI give 1/S := 0 at d_k = 0;
* R5 the 2-D equation of Numerical Experiment 3 with speed of light c and a
  selectable spin-connection potential chi (``spin``): the printed form uses
  chi = Phi; chi = Phi + Psi is the conformal 2+1-D connection used for the
  Gaussian-bump sheet;
* R6 the half-step exponential is exp(u . sigma) with a complex vector u whose
  square u.u is real (possibly negative), so exp = C I + D (u . sigma) with
  real C, D (cosh/sinh for u.u >= 0, cos/sin otherwise);
* R7 the initial spinor is taken as given (not normalised); the metric is
  static, so the half-step exponential is time independent (F evaluated at
  t_{n+1/2} does not depend on t here);
* R15 eq. (step2bis) is implemented as printed (STEP2BIS_PRINTED) and, because
  the printed correction has neither the sign nor the size that the Taylor
  expansion of the blend asks for, also as the second-order correction derived
  from that expansion (STEP2BIS_CORRECTED); the latter uses the gradient of
  a along the direction and holds the layer factor 1/S fixed.  Both are
  explicit (the implicit treatment the paper mentions is not specified);
* R16 electromagnetic potentials enter F(t, x) of Sec. 2 as
  -e c a (A_x sigma_x + A_y sigma_y) - e A0 (the conformal 2-D form of
  -i alpha(x).(-i e A) - e A0), each separable: A0 = V(x) fV(t),
  A_i = A_i(x) fA(t), with fV, fA of the form c0 + c1 sin(omega t + phase) g(t),
  g a Gaussian window or 1; Steps 1 and 5 of step n use F at t_{n+1/2}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIGMA_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)

METRIC_FLAT = 0
METRIC_GAUSS_BUMP = 1
METRIC_PAPER_EXP3 = 2
METRIC_FIELDS = 3

SPIN_NONE = 0
SPIN_PAPER = 1   # chi = Phi   (the printed 2-D equation, Numerical Experiment 3)
SPIN_2P1 = 2     # chi = Phi + Psi

# Directional step (Sec. 5.2): eq. (second_scheme), or eq. (step2bis) in two readings
STEP2_PLAIN = 0              # eq. (second_scheme)
STEP2BIS_PRINTED = 1         # eq. (step2bis) as printed: + b (c dt)^2 [[d^2]] Xi
STEP2BIS_CORRECTED = 2       # second-order Taylor correction of the blend (R15)


# ---------------------------------------------------------------------------
# Grid and momenta  (Sec. 5: D_N^(x), D_N^(xi), h_i = 2 a_i / N_i, xi_p = p pi / a_i)
# ---------------------------------------------------------------------------

def grid_points(n: int, a: float) -> np.ndarray:
    """x_k = -a + k h, k = 0..n-1, h = 2a/n (Sec. 5)."""
    h = 2.0 * a / n
    return -a + h * np.arange(n, dtype=np.float64)


def wavenumbers(n: int, a: float) -> np.ndarray:
    """xi at FFT index q: p = q for q < n/2 else q - n, xi = p pi / a (Sec. 5; R3)."""
    q = np.arange(n)
    p = np.where(q < n // 2, q, q - n).astype(np.float64)
    return p * math.pi / a


# ---------------------------------------------------------------------------
# Partial DFT pair and spectral derivative (Sec. 5, eq. (trick))
# ---------------------------------------------------------------------------

def partial_dft(psi: np.ndarray, axis: int) -> np.ndarray:
    """F_i: unnormalised forward transform sum_k psi_k exp(-i xi_p (x_k + a)).

    With x_k + a = k h and xi_p = p pi / a this is exp(-2 pi i p k / n), the
    numpy.fft convention (index q = p mod n)."""
    return np.fft.fft(psi, axis=axis)


def partial_idft(psi_hat: np.ndarray, axis: int) -> np.ndarray:
    """F_i^{-1}: (1/n) sum_p psi_p exp(+i xi_p (x_k + a))."""
    return np.fft.ifft(psi_hat, axis=axis)


def spectral_derivative(psi: np.ndarray, axis: int, xi: np.ndarray) -> np.ndarray:
    """[[d_i]] psi = F_i^{-1}[ i xi F_i psi ] (eq. (trick)), literal Nyquist xi (R3)."""
    shape = [1] * psi.ndim
    shape[axis] = xi.size
    return partial_idft(1j * xi.reshape(shape) * partial_dft(psi, axis), axis)


def dft_brute(v: np.ndarray) -> np.ndarray:
    """O(n^2) DFT straight from the definition (for pins only)."""
    n = v.shape[0]
    k = np.arange(n)
    w = np.exp(-2j * math.pi * np.outer(k, k) / n)
    return w @ v


def differentiation_matrix(n: int, a: float) -> np.ndarray:
    """A_{kk'} = (1/n) sum_p i xi_p exp(i xi_p (x_k - x_k'))  (Appendix B, first line
    of the definition of the differentiation matrices), summed literally."""
    x = grid_points(n, a)
    xi = wavenumbers(n, a)
    dx = x[:, None] - x[None, :]
    return (1j * xi[None, None, :] * np.exp(1j * xi[None, None, :] * dx[:, :, None])).sum(axis=2) / n


# ---------------------------------------------------------------------------
# Metric models (Sec. 6: ds^2 = e^{2 Phi} dt^2 - e^{2 Psi} dx^2)
# ---------------------------------------------------------------------------

@dataclass
class MetricFields:
    phi: np.ndarray
    psi: np.ndarray
    phi_x: np.ndarray
    phi_y: np.ndarray
    psi_x: np.ndarray
    psi_y: np.ndarray


@dataclass
class Envelope:
    """Time profile f(t) = c0 + c1 sin(omega t + phase) g(t), g(t) =
    exp(-((t - t0) / tau)^2) for tau > 0, else 1 (R16)."""
    c0: float = 1.0
    c1: float = 0.0
    omega: float = 0.0
    phase: float = 0.0
    t0: float = 0.0
    tau: float = 0.0

    def __call__(self, t: float) -> float:
        g = math.exp(-((t - self.t0) / self.tau) ** 2) if self.tau > 0 else 1.0
        return self.c0 + self.c1 * math.sin(self.omega * t + self.phase) * g


@dataclass
class EMPotentials:
    """Electromagnetic potentials of F(t, x) (Sec. 2): A0(t, x) = V(x) fV(t) and
    A_i(t, x) = A_i(x) fA(t), with charge e; arrays of shape (n2, n1)."""
    V: np.ndarray
    Ax: np.ndarray
    Ay: np.ndarray
    charge: float = 1.0
    fV: Envelope = field(default_factory=Envelope)
    fA: Envelope = field(default_factory=Envelope)


def metric_fields(kind: int, x: np.ndarray, y: np.ndarray, bump_A: float = 0.0,
                  bump_s: float = 1.0, fields: MetricFields | None = None) -> MetricFields:
    """Phi, Psi and their gradients on the grid, arrays of shape (n2, n1).

    FLAT: Phi = Psi = 0.
    PAPER_EXP3: Phi = exp(-0.01 |x|^2), Psi = exp(-0.005 |x|^2) (Numerical
      Experiment 3).
    GAUSS_BUMP: static sheet, Phi = 0, e^{2 Psi} = sqrt(1 + |grad h|^2) for the
      out-of-plane height h = A exp(-r^2/s^2): Psi = ln(1 + |grad h|^2) / 4.
    FIELDS: given arrays.
    """
    X, Y = np.meshgrid(x, y)          # shape (n2, n1): X[j, i] = x_i
    r2 = X * X + Y * Y
    z = np.zeros_like(X)
    if kind == METRIC_FLAT:
        return MetricFields(z, z.copy(), z.copy(), z.copy(), z.copy(), z.copy())
    if kind == METRIC_PAPER_EXP3:
        phi = np.exp(-0.01 * r2)
        psi = np.exp(-0.005 * r2)
        return MetricFields(phi, psi, -0.02 * X * phi, -0.02 * Y * phi,
                            -0.01 * X * psi, -0.01 * Y * psi)
    if kind == METRIC_GAUSS_BUMP:
        A, s = float(bump_A), float(bump_s)
        h = A * np.exp(-r2 / (s * s))
        # grad h = -(2/s^2) h (x, y)
        hx = -2.0 / (s * s) * h * X
        hy = -2.0 / (s * s) * h * Y
        g = hx * hx + hy * hy                      # |grad h|^2
        # d/dx |grad h|^2 = 2 (h_x h_xx + h_y h_xy), with the second derivatives of h
        hxx = h * (4.0 * X * X / s**4 - 2.0 / (s * s))
        hyy = h * (4.0 * Y * Y / s**4 - 2.0 / (s * s))
        hxy = h * (4.0 * X * Y / s**4)
        gx = 2.0 * (hx * hxx + hy * hxy)
        gy = 2.0 * (hx * hxy + hy * hyy)
        psi = 0.25 * np.log1p(g)
        return MetricFields(z, psi, z.copy(), z.copy(), 0.25 * gx / (1.0 + g), 0.25 * gy / (1.0 + g))
    if kind == METRIC_FIELDS:
        assert fields is not None
        return fields
    raise ValueError(f"unknown metric kind {kind}")


def spin_potential(spin: int, f: MetricFields):
    """chi_x, chi_y, chi for the spin connection term (1/2) d_j chi (R5)."""
    if spin == SPIN_NONE:
        z = np.zeros_like(f.phi)
        return z, z.copy(), z.copy()
    if spin == SPIN_PAPER:
        return f.phi_x, f.phi_y, f.phi
    if spin == SPIN_2P1:
        return f.phi_x + f.psi_x, f.phi_y + f.psi_y, f.phi + f.psi
    raise ValueError(f"unknown spin selector {spin}")


# ---------------------------------------------------------------------------
# Absorbing layer (Sec. 3): S^i = 1 + e^{i theta} Sigma~(x^i), types I-VI
# ---------------------------------------------------------------------------

def pml_inverse_stretch(n: int, a: float, width: int, ptype: int = 1, sigma0: float = 1.0,
                        theta: float = 0.0) -> np.ndarray:
    """1/S^i at the n grid points of one axis (R4 for the layer geometry).

    Sigma~(x) = Sigma(|x| - L) in the layer, 0 inside; Sigma(s) per type:
      I: s0 (s+d)^2   II: s0 (s+d)^3   III: -s0/s   IV: s0/s^2
      V: -s0/s - s0/d   VI: s0/s^2 - s0/d^2      (d = L - L* = width h)
    """
    inv = np.ones(n, dtype=np.complex128)
    if width <= 0:
        return inv
    h = 2.0 * a / n
    delta = width * h
    for k in range(n):
        dk = min(k, n - k)                 # whole grid steps to the seam x = +-a
        if dk > width:
            continue
        s = -dk * h                        # |x_k| - L
        if ptype == 1:
            sig = sigma0 * (s + delta) ** 2
        elif ptype == 2:
            sig = sigma0 * (s + delta) ** 3
        elif dk == 0:                      # singular types at |x| = L: 1/S := 0
            inv[k] = 0.0
            continue
        elif ptype == 3:
            sig = -sigma0 / s
        elif ptype == 4:
            sig = sigma0 / (s * s)
        elif ptype == 5:
            sig = -sigma0 / s - sigma0 / delta
        elif ptype == 6:
            sig = sigma0 / (s * s) - sigma0 / (delta * delta)
        else:
            raise ValueError(f"unknown PML type {ptype}")
        inv[k] = 1.0 / (1.0 + np.exp(1j * theta) * sig)
    return inv


# ---------------------------------------------------------------------------
# Half-step exponential (Step 1 / Step 3; eq. (exp_dirac), R6)
# ---------------------------------------------------------------------------

def half_step_exponential(f: MetricFields, spin: int, m: float, c: float, dt: float) -> np.ndarray:
    """E = exp(-i dt/2 [beta(x) m c^2 + F(x)]) per point, shape (n2, n1, 2, 2).

    For the 2-D equation of Numerical Experiment 3, beta(x) m = e^Phi m c^2 sigma_z
    and F = -i c a (chi_x sigma_x + chi_y sigma_y)/2 with a = e^{Phi - Psi}.  The
    exponent is u . sigma with
        u = (-(dt/4) c a chi_x, -(dt/4) c a chi_y, -i (dt/2) m c^2 e^Phi),
    and (u . sigma)^2 = (u . u) I with u . u real, so
        exp(u . sigma) = C I + D (u . sigma),
    C = cosh r, D = sinh r / r for u.u = r^2 >= 0, and C = cos r, D = sin r / r for
    u.u = -r^2 < 0 (eq. (exp_dirac) is the second case with real G).  Near u.u = 0
    both are the series sum (u.u)^k/(2k)! and sum (u.u)^k/(2k+1)!.
    """
    chi_x, chi_y, _ = spin_potential(spin, f)
    a = np.exp(f.phi - f.psi)
    ux = -(dt / 4.0) * c * a * chi_x
    uy = -(dt / 4.0) * c * a * chi_y
    uz = -1j * (dt / 2.0) * m * c * c * np.exp(f.phi)
    s2 = (ux * ux + uy * uy + (uz * uz).real)        # real by construction
    r = np.sqrt(np.abs(s2))
    small = np.abs(s2) < 1e-8
    with np.errstate(invalid="ignore", divide="ignore"):
        C = np.where(s2 >= 0, np.cosh(r), np.cos(r))
        D = np.where(s2 >= 0, np.sinh(r) / r, np.sin(r) / r)
    C = np.where(small, 1.0 + s2 / 2.0 + s2 * s2 / 24.0, C)
    D = np.where(small, 1.0 + s2 / 6.0 + s2 * s2 / 120.0, D)
    E = (C[..., None, None] * ID2
         + D[..., None, None] * (ux[..., None, None] * SIGMA_X + uy[..., None, None] * SIGMA_Y
                                 + uz[..., None, None] * SIGMA_Z))
    return E


def half_step_exponential_em(f: MetricFields, spin: int, m: float, c: float, dt: float,
                             em: EMPotentials, t: float) -> np.ndarray:
    """E(t) = exp(-i dt/2 [beta(x) m c^2 + F(t, x)]) with the electromagnetic part of
    F (Sec. 2): -e c a (A_x sigma_x + A_y sigma_y) - e A0 I (alpha(x) = c a alpha in
    the conformal 2-D form).  The exponent is i (dt/2) e A0 I + u . sigma with
        u = (-(dt/4) c a chi_x + i (dt/2) e c a A_x, -(dt/4) c a chi_y + i (dt/2) e c a A_y,
             -i (dt/2) m c^2 e^Phi),
    and now u . u is complex: exp(u . sigma) = C I + D u . sigma with C = cosh r,
    D = sinh r / r, r^2 = u . u (both even in r), series near u . u = 0."""
    chi_x, chi_y, _ = spin_potential(spin, f)
    a = np.exp(f.phi - f.psi)
    fa, fv = em.fA(t), em.fV(t)
    ux = -(dt / 4.0) * c * a * chi_x + 0.5j * dt * em.charge * c * a * em.Ax * fa
    uy = -(dt / 4.0) * c * a * chi_y + 0.5j * dt * em.charge * c * a * em.Ay * fa
    uz = -0.5j * dt * m * c * c * np.exp(f.phi) * np.ones_like(a)
    s2 = ux * ux + uy * uy + uz * uz
    r = np.sqrt(s2.astype(np.complex128))
    small = np.abs(s2) < 1e-8
    with np.errstate(invalid="ignore", divide="ignore"):
        C = np.cosh(r)
        D = np.sinh(r) / r
    C = np.where(small, 1.0 + s2 / 2.0 + s2 * s2 / 24.0, C)
    D = np.where(small, 1.0 + s2 / 6.0 + s2 * s2 / 120.0, D)
    phase = np.exp(0.5j * dt * em.charge * em.V * fv)
    E = (C[..., None, None] * ID2
         + D[..., None, None] * (ux[..., None, None] * SIGMA_X + uy[..., None, None] * SIGMA_Y
                                 + uz[..., None, None] * SIGMA_Z))
    return phase[..., None, None] * E


def apply_pointwise(M: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """psi_k <- M_k psi_k for 2x2 matrices M of shape (..., 2, 2)."""
    return np.einsum("...ab,...b->...a", M, psi)


# ---------------------------------------------------------------------------
# Directional symbols (eq. (second_scheme)): Pi^i exp(-i c dt Lambda xi) Pi^{i,dag}
# = exp(-i c dt xi sigma_i) = cos(c dt xi) I - i sin(c dt xi) sigma_i   (R1)
# ---------------------------------------------------------------------------

def directional_symbol(xi: np.ndarray, c: float, dt: float, sigma: np.ndarray) -> np.ndarray:
    th = c * dt * xi
    return np.cos(th)[:, None, None] * ID2 - 1j * np.sin(th)[:, None, None] * sigma


# ---------------------------------------------------------------------------
# The solve
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    n1: int
    n2: int
    a1: float
    a2: float
    dt: float
    c: float = 1.0
    m: float = 1.0
    metric: int = METRIC_FLAT
    spin: int = SPIN_NONE
    bump_A: float = 0.0
    bump_s: float = 1.0
    fields: MetricFields | None = None
    pml_width: int = 0
    pml_type: int = 1
    pml_sigma0: float = 1.0
    pml_theta: float = 0.0
    step2: int = STEP2_PLAIN
    em: EMPotentials | None = None


@dataclass
class Tables:
    prob: Problem
    x: np.ndarray
    y: np.ndarray
    h1: float
    h2: float
    xi1: np.ndarray
    xi2: np.ndarray
    fields: MetricFields
    a: np.ndarray            # e^{Phi - Psi}, (n2, n1)
    bx: np.ndarray           # a / S^1(x_i), (n2, n1)
    by: np.ndarray           # a / S^2(y_j), (n2, n1)
    E: np.ndarray            # (n2, n1, 2, 2)
    Kx: np.ndarray           # (n1, 2, 2)
    Ky: np.ndarray           # (n2, 2, 2)
    chi_x: np.ndarray = field(default=None)
    chi_y: np.ndarray = field(default=None)
    chi: np.ndarray = field(default=None)
    dbx: np.ndarray = field(default=None)     # (d_x a) / S^1, (n2, n1)
    dby: np.ndarray = field(default=None)     # (d_y a) / S^2, (n2, n1)


def build_tables(p: Problem) -> Tables:
    """Setup of one solve (Sec. 5 grid; Sec. 5.2 directional form with PML)."""
    x = grid_points(p.n1, p.a1)
    y = grid_points(p.n2, p.a2)
    f = metric_fields(p.metric, x, y, p.bump_A, p.bump_s, p.fields)
    a = np.exp(f.phi - f.psi)
    invS1 = pml_inverse_stretch(p.n1, p.a1, p.pml_width, p.pml_type, p.pml_sigma0, p.pml_theta)
    invS2 = pml_inverse_stretch(p.n2, p.a2, p.pml_width, p.pml_type, p.pml_sigma0, p.pml_theta)
    bx = a * invS1[None, :]
    by = a * invS2[:, None]
    if np.all(np.imag(bx) == 0) and np.all(np.imag(by) == 0):
        bx, by = bx.real.copy(), by.real.copy()
    E = half_step_exponential(f, p.spin, p.m, p.c, p.dt)
    xi1 = wavenumbers(p.n1, p.a1)
    xi2 = wavenumbers(p.n2, p.a2)
    chi_x, chi_y, chi = spin_potential(p.spin, f)
    # gradient of a = e^{Phi - Psi}; the layer factor 1/S is held fixed (R15)
    dbx = a * (f.phi_x - f.psi_x) * invS1[None, :].real
    dby = a * (f.phi_y - f.psi_y) * invS2[:, None].real
    return Tables(p, x, y, 2 * p.a1 / p.n1, 2 * p.a2 / p.n2, xi1, xi2, f, a, bx, by, E,
                  directional_symbol(xi1, p.c, p.dt, SIGMA_X),
                  directional_symbol(xi2, p.c, p.dt, SIGMA_Y), chi_x, chi_y, chi, dbx, dby)


def blend_is_stable(b: np.ndarray) -> bool:
    """Stability condition of the directional blend (Sec. 5.2, stability
    proposition, case C <= 1): every per-mode amplification b e^{-i phi} + (1-b)
    stays in the unit disk iff |b| + |1 - b| <= 1, i.e. b real in [0, 1]."""
    return bool(np.all(np.abs(b) + np.abs(1.0 - b) <= 1.0 + 1e-12))


def directional_stage(psi: np.ndarray, axis: int, K: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One direction of eq. (second_scheme) with PML (a^i -> a^i/S^i):
    psi* = b F_i^{-1}[K(xi) F_i psi] + (1 - b) psi."""
    P = partial_dft(psi, axis)
    if axis == 1:
        P = np.einsum("qab,jqb->jqa", K, P)
    else:
        P = np.einsum("qab,qib->qia", K, P)
    Xi = partial_idft(P, axis)
    return b[..., None] * Xi + (1.0 - b[..., None]) * psi


def directional_stage_2bis(psi: np.ndarray, axis: int, K: np.ndarray, b: np.ndarray, xi: np.ndarray,
                           c: float, dt: float, variant: int, db: np.ndarray | None = None) -> np.ndarray:
    """One direction of eq. (step2bis).

    STEP2BIS_PRINTED, the formula as printed (with the transport speed c):
        psi* = b Xi + (1 - b) psi + b (c dt)^2 [[d_i^2]] Xi,   Xi = F_i^{-1}[K F_i psi].

    STEP2BIS_CORRECTED (R15): the blend b Xi + (1 - b) psi equals, to second order
    in dt, psi - c dt b sigma_i d_i psi + ((c dt)^2 / 2) b d_i^2 psi (e^{-i theta}
    expanded with its factor 1/2), while the exact transport d_t psi = -c b sigma_i
    d_i psi gives psi - c dt b sigma_i d_i psi + ((c dt)^2 / 2) b d_i(b d_i psi)
    (sigma_i^2 = I).  Adding the difference makes the step second order:
        psi* = b Xi + (1 - b) psi
               + ((c dt)^2 / 2) (-b (1 - b) [[d_i^2]] psi + b b' [[d_i]] psi),
    with b' = (d_i a) / S^i (the layer factor held fixed) and the spectral
    derivatives of eq. (trick): [[d_i]] <-> i xi, [[d_i^2]] <-> -xi^2.
    """
    P = partial_dft(psi, axis)
    if axis == 1:
        KP = np.einsum("qab,jqb->jqa", K, P)
        shape = (1, -1, 1)
    else:
        KP = np.einsum("qab,qib->qia", K, P)
        shape = (-1, 1, 1)
    Xi = partial_idft(KP, axis)
    bb = b[..., None]
    out = bb * Xi + (1.0 - bb) * psi
    xs = xi.reshape(shape)
    if variant == STEP2BIS_PRINTED:
        d2Xi = partial_idft(-(xs ** 2) * KP, axis)
        out = out + bb * (c * dt) ** 2 * d2Xi
    elif variant == STEP2BIS_CORRECTED:
        d2psi = partial_idft(-(xs ** 2) * P, axis)
        d1psi = partial_idft(1j * xs * P, axis)
        out = out + 0.5 * (c * dt) ** 2 * (-bb * (1.0 - bb) * d2psi + bb * db[..., None] * d1psi)
    else:
        raise ValueError(f"unknown step2bis variant {variant}")
    return out


def step_exponential(T: Tables, n: int) -> np.ndarray:
    """The Step-1 / Step-5 factor of step n: F at t_{n+1/2} = (n + 1/2) dt (eq. (step1))."""
    p = T.prob
    if p.em is None:
        return T.E
    return half_step_exponential_em(T.fields, p.spin, p.m, p.c, p.dt, p.em, (n + 0.5) * p.dt)


def step_stages(psi: np.ndarray, T: Tables, n: int = 0):
    """Step n (from t_n to t_{n+1}), returning every stage boundary (after Step 1,
    after the x direction, after the y direction, after Step 5)."""
    p = T.prob
    E = step_exponential(T, n)
    s1 = apply_pointwise(E, psi)                         # Step 1
    if p.step2 == STEP2_PLAIN:
        s2 = directional_stage(s1, 1, T.Kx, T.bx)        # direction 1 (x)
        s3 = directional_stage(s2, 0, T.Ky, T.by)        # direction 2 (y)
    else:
        s2 = directional_stage_2bis(s1, 1, T.Kx, T.bx, T.xi1, p.c, p.dt, p.step2, T.dbx)
        s3 = directional_stage_2bis(s2, 0, T.Ky, T.by, T.xi2, p.c, p.dt, p.step2, T.dby)
    s4 = apply_pointwise(E, s3)                          # Step 5
    return s1, s2, s3, s4


def step(psi: np.ndarray, T: Tables, n: int = 0) -> np.ndarray:
    return step_stages(psi, T, n)[3]


def run(psi0: np.ndarray, T: Tables, nsteps: int, callback=None, start: int = 0) -> np.ndarray:
    """Steps start .. start + nsteps - 1 (the index fixes the time of F)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for n in range(start, start + nsteps):
        psi = step(psi, T, n)
        if callback is not None:
            callback(n + 1, psi)
    return psi


# ---------------------------------------------------------------------------
# Observables
# ---------------------------------------------------------------------------

def weight(T: Tables) -> np.ndarray:
    """Weight w of the norm int w |psi|^2 that the continuous 2-D equation conserves:
    w = e^{chi - Phi + Psi} (integration by parts of the 2-D equation of Sec. 6;
    it makes (w a)_j = w a chi_j)."""
    return np.exp(T.chi - T.fields.phi + T.fields.psi)


def apply_hamiltonian(psi: np.ndarray, T: Tables, t: float = 0.0) -> np.ndarray:
    """H psi = -i c a (sigma_x [[d_x]] + sigma_y [[d_y]]) psi
               - i (c a / 2)(chi_x sigma_x + chi_y sigma_y) psi + e^Phi m c^2 sigma_z psi
               [- e c a (A_x sigma_x + A_y sigma_y) psi - e A0 psi at time t]
    (2-D equation of Sec. 6 with [[d_i]] of eq. (trick); no PML stretch)."""
    p = T.prob
    dx = spectral_derivative(psi, 1, T.xi1)
    dy = spectral_derivative(psi, 0, T.xi2)
    ca = p.c * T.a
    out = -1j * ca[..., None] * (apply_pointwise(np.broadcast_to(SIGMA_X, psi.shape[:2] + (2, 2)), dx)
                                 + apply_pointwise(np.broadcast_to(SIGMA_Y, psi.shape[:2] + (2, 2)), dy))
    spin = -0.5j * ca[..., None, None] * (T.chi_x[..., None, None] * SIGMA_X + T.chi_y[..., None, None] * SIGMA_Y)
    mass = (np.exp(T.fields.phi) * p.m * p.c * p.c)[..., None, None] * SIGMA_Z
    pot = spin + mass
    if p.em is not None:
        em = p.em
        fa, fv = em.fA(t), em.fV(t)
        pot = pot - (em.charge * ca * fa)[..., None, None] * (em.Ax[..., None, None] * SIGMA_X
                                                              + em.Ay[..., None, None] * SIGMA_Y)
        pot = pot - (em.charge * em.V * fv)[..., None, None] * ID2
    return out + apply_pointwise(pot, psi)


@dataclass
class Observables:
    norm_l2: float
    norm_w: float
    energy_re: float
    energy_im: float
    x_mean: float
    y_mean: float
    finite: bool


def observables(psi: np.ndarray, T: Tables, t: float = 0.0) -> Observables:
    """Norms, weighted energy <psi, H(t) psi>_w and mean position (t enters only
    through time-dependent potentials)."""
    dens = np.sum(np.abs(psi) ** 2, axis=2)
    dA = T.h1 * T.h2
    w = weight(T)
    finite = bool(np.all(np.isfinite(psi)))
    X, Y = np.meshgrid(T.x, T.y)
    n2 = dA * dens.sum()
    en = dA * np.sum(w * np.sum(np.conj(psi) * apply_hamiltonian(psi, T, t), axis=2))
    return Observables(float(n2), float(dA * np.sum(w * dens)), float(en.real), float(en.imag),
                       float(np.sum(X * dens) / dens.sum()), float(np.sum(Y * dens) / dens.sum()), finite)


# ---------------------------------------------------------------------------
# Exact references for flat space
# ---------------------------------------------------------------------------

def flat_step_matrix(xi_x: float, xi_y: float, m: float, c: float, dt: float) -> np.ndarray:
    """Per-mode matrix of one flat step: U = A K_y K_x A, A = exp(-i dt m c^2 sigma_z / 2)."""
    mu = dt * m * c * c / 2.0
    A = np.diag([np.exp(-1j * mu), np.exp(1j * mu)])
    Kx = math.cos(c * dt * xi_x) * ID2 - 1j * math.sin(c * dt * xi_x) * SIGMA_X
    Ky = math.cos(c * dt * xi_y) * ID2 - 1j * math.sin(c * dt * xi_y) * SIGMA_Y
    return A @ Ky @ Kx @ A


def flat_exact_discrete(psi0: np.ndarray, n1: int, n2: int, a1: float, a2: float, m: float,
                        c: float, dt: float, nsteps: int) -> np.ndarray:
    """The flat scheme's own output after nsteps, without a time loop: every Fourier
    mode evolves by U(xi)^n (U in SU(2)), here by binary powering of stacked 2x2
    matrices in FP64."""
    xi1 = wavenumbers(n1, a1)
    xi2 = wavenumbers(n2, a2)
    mu = dt * m * c * c / 2.0
    A = np.diag([np.exp(-1j * mu), np.exp(1j * mu)])
    cx, sx = np.cos(c * dt * xi1), np.sin(c * dt * xi1)
    cy, sy = np.cos(c * dt * xi2), np.sin(c * dt * xi2)
    Kx = cx[None, :, None, None] * ID2 - 1j * sx[None, :, None, None] * SIGMA_X
    Ky = cy[:, None, None, None] * ID2 - 1j * sy[:, None, None, None] * SIGMA_Y
    U = A @ Ky @ Kx @ A                                  # (n2, n1, 2, 2)
    Un = np.linalg.matrix_power(U, nsteps)
    P = np.fft.fft2(psi0, axes=(0, 1))
    return np.fft.ifft2(apply_pointwise(Un, P), axes=(0, 1))


def flat_continuous(psi0: np.ndarray, n1: int, n2: int, a1: float, a2: float, m: float,
                    c: float, t: float) -> np.ndarray:
    """Exact solution of the flat 2-D Dirac equation on the periodic grid (band
    limited data): psi_hat(t) = [cos(w t) I - i sin(w t) H(xi)/w] psi_hat(0),
    H(xi) = c (xi_x sigma_x + xi_y sigma_y) + m c^2 sigma_z, w = sqrt(m^2 c^4 + c^2 |xi|^2)."""
    xi1 = wavenumbers(n1, a1)
    xi2 = wavenumbers(n2, a2)
    XI, YI = np.meshgrid(xi1, xi2)
    w = np.sqrt(m * m * c ** 4 + c * c * (XI * XI + YI * YI))
    H = (c * XI)[..., None, None] * SIGMA_X + (c * YI)[..., None, None] * SIGMA_Y + (m * c * c) * SIGMA_Z
    with np.errstate(invalid="ignore", divide="ignore"):
        sw = np.where(w > 0, np.sin(w * t) / w, t)
    U = np.cos(w * t)[..., None, None] * ID2 - 1j * sw[..., None, None] * H
    P = np.fft.fft2(psi0, axes=(0, 1))
    return np.fft.ifft2(apply_pointwise(U, P), axes=(0, 1))


def flat_discrete_frequency(xi_x: float, xi_y: float, m: float, c: float, dt: float) -> float:
    """omega with cos(omega dt) = cos(m c^2 dt) cos(c xi_x dt) cos(c xi_y dt)
    + sin(m c^2 dt) sin(c xi_x dt) sin(c xi_y dt): half the trace of A K_y K_x A."""
    mu = m * c * c * dt
    val = (math.cos(mu) * math.cos(c * xi_x * dt) * math.cos(c * xi_y * dt)
           + math.sin(mu) * math.sin(c * xi_x * dt) * math.sin(c * xi_y * dt))
    return math.acos(max(-1.0, min(1.0, val))) / dt


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


# ---------------------------------------------------------------------------
# Numerical Scheme I (Sec. 5.1): Crank-Nicolson transport step solved by GMRES
# ---------------------------------------------------------------------------

def transport_operator(psi: np.ndarray, T: Tables) -> np.ndarray:
    """alpha(x) . T psi of eq. (hamiltonian_pml) for the 2-D equation: the
    transport part c a(x) (sigma_x [[d_x]] / S^1 + sigma_y [[d_y]] / S^2) psi with the
    spectral derivative of eq. (trick); the blend coefficients b_i = a / S^i carry
    the layer (Appendix A: a / S_x, a / S_y)."""
    c = T.prob.c
    dx = spectral_derivative(psi, 1, T.xi1)
    dy = spectral_derivative(psi, 0, T.xi2)
    sx = np.stack([dx[..., 1], dx[..., 0]], axis=-1)                  # sigma_x dx
    sy = np.stack([-1j * dy[..., 1], 1j * dy[..., 0]], axis=-1)       # sigma_y dy
    return c * (T.bx[..., None] * sx + T.by[..., None] * sy)


def cn_operators(T: Tables):
    """G = I + (dt/2) alpha . T and G~ = I - (dt/2) alpha . T (Sec. 5.1, eq. (cn))."""
    h = T.prob.dt / 2.0
    G = lambda v: v + h * transport_operator(v, T)
    Gt = lambda v: v - h * transport_operator(v, T)
    return G, Gt


def cn_solve(rhs: np.ndarray, T: Tables, x0: np.ndarray | None = None, rtol: float = 1e-14,
             restart: int = 30, maxiter: int = 200) -> np.ndarray:
    """Solve G x = rhs with GMRES (the Krylov solver the paper names, through
    scipy's implementation)."""
    import scipy.sparse.linalg as spla
    shape = rhs.shape
    n = rhs.size
    G, _ = cn_operators(T)
    A = spla.LinearOperator((n, n), matvec=lambda v: G(v.reshape(shape)).ravel(), dtype=np.complex128)
    x, info = spla.gmres(A, rhs.ravel(), x0=None if x0 is None else x0.ravel(), rtol=rtol, atol=0.0,
                         restart=restart, maxiter=maxiter)
    if info != 0:
        raise RuntimeError(f"GMRES did not converge (info={info})")
    return x.reshape(shape)


def cn_step(psi: np.ndarray, T: Tables, rtol: float = 1e-14, n: int = 0) -> np.ndarray:
    """Step n of Scheme I, eq. (cn): Step 1 (E), G psi* = G~ psi^{n+1/2}, Step 3 (E)."""
    E = step_exponential(T, n)
    half = apply_pointwise(E, psi)
    _, Gt = cn_operators(T)
    star = cn_solve(Gt(half), T, x0=half, rtol=rtol)
    return apply_pointwise(E, star)


def cn_run(psi0: np.ndarray, T: Tables, nsteps: int, rtol: float = 1e-14, start: int = 0) -> np.ndarray:
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for n in range(start, start + nsteps):
        psi = cn_step(psi, T, rtol, n)
    return psi


def cn_flat_exact(psi0: np.ndarray, n1: int, n2: int, a1: float, a2: float, m: float, c: float, dt: float,
                  nsteps: int) -> np.ndarray:
    """Flat Scheme I per Fourier mode: (A C A)^n with the Cayley factor
    C = (I + (dt/2) c i sigma.xi)^{-1} (I - (dt/2) c i sigma.xi)."""
    xi1 = wavenumbers(n1, a1)
    xi2 = wavenumbers(n2, a2)
    XI, YI = np.meshgrid(xi1, xi2)
    mu = dt * m * c * c / 2.0
    A = np.diag([np.exp(-1j * mu), np.exp(1j * mu)])
    S = 1j * (dt / 2.0) * c * (XI[..., None, None] * SIGMA_X + YI[..., None, None] * SIGMA_Y)
    Cay = np.linalg.solve(ID2 + S, ID2 - S)
    U = A @ Cay @ A
    P = np.fft.fft2(psi0, axes=(0, 1))
    return np.fft.ifft2(apply_pointwise(np.linalg.matrix_power(U, nsteps), P), axes=(0, 1))
