"""The pins hold the oracle to the paper: plant one plausible mistake at a time
in a temporary copy of the oracle (never in the repository's file) and check
that the pin suite run against that copy fails, and that the unmodified copy
passes.  CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what goes wrong, the text in oracle/dirac_oracle.py, what it becomes)
MUTATIONS_2D = [
    ("sign of the directional symbol (R1)",
     "th)[:, None, None] * ID2 - 1j * np.sin", "th)[:, None, None] * ID2 + 1j * np.sin"),
    ("blend without its (1 - b) psi term (eq. (second_scheme))",
     "return b[..., None] * Xi + (1.0 - b[..., None]) * psi", "return b[..., None] * Xi"),
    ("Nyquist mode taken as +n/2 (R3)",
     "p = np.where(q < n // 2, q, q - n)", "p = np.where(q <= n // 2, q, q - n)"),
    ("directions applied y then x (R2)",
     "        s2 = directional_stage(s1, 1, T.Kx, T.bx)        # direction 1 (x)\n"
     "        s3 = directional_stage(s2, 0, T.Ky, T.by)",
     "        s2 = directional_stage(s1, 0, T.Ky, T.by)        # direction 1 (x)\n"
     "        s3 = directional_stage(s2, 1, T.Kx, T.bx)"),
    ("y blend with the x layer factor",
     "s3 = directional_stage(s2, 0, T.Ky, T.by)", "s3 = directional_stage(s2, 0, T.Ky, T.bx)"),
    ("transposed half-step exponential (eq. (exp_dirac))",
     "                                 + uz[..., None, None] * SIGMA_Z))\n    return E",
     "                                 + uz[..., None, None] * SIGMA_Z))\n    return np.swapaxes(E, -1, -2)"),
    ("sign of the mass term in E",
     "uz = -1j * (dt / 2.0) * m * c * c * np.exp(f.phi)", "uz = 1j * (dt / 2.0) * m * c * c * np.exp(f.phi)"),
    ("sign of the spin-connection term in E (R6)",
     "ux = -(dt / 4.0) * c * a * chi_x\n    uy = -(dt / 4.0) * c * a * chi_y\n",
     "ux = (dt / 4.0) * c * a * chi_x\n    uy = (dt / 4.0) * c * a * chi_y\n"),
    ("Step 5 dropped (eq. (step3))",
     "    s4 = apply_pointwise(E, s3)                          # Step 5",
     "    s4 = s3                          # Step 5"),
    ("Scheme I blend factors swapped between the axes (Appendix A)",
     "return c * (T.bx[..., None] * sx + T.by[..., None] * sy)",
     "return c * (T.by[..., None] * sx + T.bx[..., None] * sy)"),
    ("Scheme I operator without the layer factor 1/S",
     "return c * (T.bx[..., None] * sx + T.by[..., None] * sy)",
     "return c * (T.a[..., None] * sx + T.a[..., None] * sy)"),
    ("corrected second-order step: sign of its b (1 - b) term (R15)",
     "(-bb * (1.0 - bb) * d2psi + bb * db[..., None] * d1psi)",
     "(bb * (1.0 - bb) * d2psi + bb * db[..., None] * d1psi)"),
    ("corrected second-order step without its b b' term (R15)",
     "(-bb * (1.0 - bb) * d2psi + bb * db[..., None] * d1psi)", "(-bb * (1.0 - bb) * d2psi)"),
    ("printed second-order step: correction subtracted (eq. (step2bis))",
     "out = out + bb * (c * dt) ** 2 * d2Xi", "out = out - bb * (c * dt) ** 2 * d2Xi"),
    ("potentials: sign of the vector-potential coupling (R16)",
     "ux = -(dt / 4.0) * c * a * chi_x + 0.5j * dt", "ux = -(dt / 4.0) * c * a * chi_x - 0.5j * dt"),
    ("potentials: sign of the scalar-potential phase (R16)",
     "phase = np.exp(0.5j * dt * em.charge * em.V * fv)", "phase = np.exp(-0.5j * dt * em.charge * em.V * fv)"),
    ("potentials sampled at t_n instead of t_{n+1/2} (R13)",
     "(n + 0.5) * p.dt)", "n * p.dt)"),
]

# the same for oracle/dirac3_oracle.py, checked by the 3-D pins
MUTATIONS_3D = [
    ("3-D: sign of the directional symbol",
     "ID4 - 1j * np.sin(th)[:, None, None] * ALPHA[axis]", "ID4 + 1j * np.sin(th)[:, None, None] * ALPHA[axis]"),
    ("3-D: y and z directions on each other's array axes",
     "ARRAY_AXIS = (2, 1, 0)", "ARRAY_AXIS = (2, 0, 1)"),
    ("3-D: sign of the mass term in E (R17)",
     "M = (-1j * w[..., None, None] * BETA", "M = (1j * w[..., None, None] * BETA"),
    ("3-D: blend without its (1 - b) psi term",
     "return b[..., None] * Xi + (1.0 - b[..., None]) * psi", "return b[..., None] * Xi"),
    ("3-D: Step 5 dropped",
     "    return apply_pointwise3(T.E, s)                # Step 5", "    return s"),
]

CASES = ([("dirac_oracle.py", "test_oracle_pins.py") + m for m in MUTATIONS_2D] +
         [("dirac3_oracle.py", "test_oracle3_pins.py") + m for m in MUTATIONS_3D])


def run_pins(tmp_path, name, fname, text, pins):
    """Run tests/<pins> with `oracle` imported from a copy whose <fname> holds `text`."""
    d = tmp_path / name
    shutil.copytree(os.path.join(ROOT, "oracle"), d / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__"))
    (d / "oracle" / fname).write_text(text)
    env = dict(os.environ, PYTHONPATH=str(d) + os.pathsep + ROOT, PYTHONDONTWRITEBYTECODE="1")
    # --import-mode=append keeps the repository root behind the copy on sys.path
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "--import-mode=append", os.path.join(ROOT, "tests", pins)],
                       capture_output=True, text=True, env=env, cwd=str(d), timeout=600)
    return r


@pytest.mark.parametrize("fname,pins", [("dirac_oracle.py", "test_oracle_pins.py"),
                                         ("dirac3_oracle.py", "test_oracle3_pins.py")])
def test_unmodified_copy_passes(tmp_path, fname, pins):
    src = open(os.path.join(ROOT, "oracle", fname)).read()
    r = run_pins(tmp_path, "control", fname, src, pins)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("fname,pins,what,old,new", CASES, ids=[c[2] for c in CASES])
def test_planted_mistake_fails_a_pin(tmp_path, fname, pins, what, old, new):
    src = open(os.path.join(ROOT, "oracle", fname)).read()
    assert src.count(old) == 1, f"mutation site not found: {what}"
    r = run_pins(tmp_path, "mutant", fname, src.replace(old, new), pins)
    assert r.returncode == 1, (what, r.stdout[-2000:])        # 1: tests ran and one failed
    assert "FAILED" in r.stdout and "error" not in r.stdout.splitlines()[-1].lower(), r.stdout[-2000:]
