"""Python binding of libdirac (ctypes over include/dirac.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides the device buffer (a uint8 tensor) and the stream.  If the
shared library is missing, importing this module raises ImportError -- there
is no fallback path.

Module-level functions carry the C names without the ``dirac_`` prefix
(``create_metric``, ``set_initial_spinor``, ``step_n``, ``observables``,
``get_spinor``, ``destroy``, ...); :class:`Solver` bundles them with a
torch-allocated device buffer.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdirac.so")

FP64, FP32 = 0, 1
METRIC_FLAT, METRIC_GAUSS_BUMP, METRIC_PAPER_EXP3, METRIC_FIELDS = 0, 1, 2, 3
SPIN_NONE, SPIN_PAPER, SPIN_2P1 = 0, 1, 2
SCHEME_EXP_SPLIT, SCHEME_CN_GMRES, SCHEME_EXP_SPLIT_2BIS_PRINTED, SCHEME_EXP_SPLIT_2BIS = 0, 1, 2, 3

STATUS = {0: "DIRAC_OK", -1: "DIRAC_E_ARG", -2: "DIRAC_E_SIZE", -3: "DIRAC_E_UNSTABLE",
          -4: "DIRAC_E_NOMEM", -5: "DIRAC_E_DEVICE", -6: "DIRAC_E_STATE", -7: "DIRAC_E_NONFINITE",
          -8: "DIRAC_E_NOCONV"}

_dp = C.POINTER(C.c_double)


class Grid(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("a1", C.c_double), ("a2", C.c_double),
                ("dt", C.c_double), ("c", C.c_double), ("m", C.c_double)]


class Metric(C.Structure):
    _fields_ = [("kind", C.c_int32), ("spin", C.c_int32), ("bump_A", C.c_double), ("bump_s", C.c_double),
                ("phi", _dp), ("psi", _dp), ("dphi_dx", _dp), ("dphi_dy", _dp), ("dpsi_dx", _dp),
                ("dpsi_dy", _dp)]


class Pml(C.Structure):
    _fields_ = [("width_pts", C.c_int32), ("type", C.c_int32), ("sigma0", C.c_double), ("theta", C.c_double)]


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("norm_l2", C.c_double), ("norm_w", C.c_double),
                ("energy_re", C.c_double), ("energy_im", C.c_double), ("x_mean", C.c_double),
                ("y_mean", C.c_double), ("finite", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Schedule(C.Structure):
    _fields_ = [("radix", C.c_int32), ("lines_per_wg", C.c_int32), ("components_per_thread", C.c_int32)]


class Scheme(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("gmres_restart", C.c_int32), ("gmres_max_iter", C.c_int32),
                ("reserved", C.c_int32), ("gmres_rtol", C.c_double)]


class Envelope(C.Structure):
    _fields_ = [("c0", C.c_double), ("c1", C.c_double), ("omega", C.c_double), ("phase", C.c_double),
                ("t0", C.c_double), ("tau", C.c_double)]


class Em(C.Structure):
    _fields_ = [("V", _dp), ("Ax", _dp), ("Ay", _dp), ("charge", C.c_double), ("fV", Envelope), ("fA", Envelope)]


class Grid3(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32), ("a1", C.c_double), ("a2", C.c_double),
                ("a3", C.c_double), ("dt", C.c_double), ("c", C.c_double), ("m", C.c_double)]


class Metric3(C.Structure):
    _fields_ = [("kind", C.c_int32), ("spin", C.c_int32), ("phi", _dp), ("psi", _dp), ("dphi_dx", _dp),
                ("dphi_dy", _dp), ("dphi_dz", _dp), ("dpsi_dx", _dp), ("dpsi_dy", _dp), ("dpsi_dz", _dp)]


class Obs3(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("norm_l2", C.c_double), ("norm_w", C.c_double),
                ("x_mean", C.c_double), ("y_mean", C.c_double), ("z_mean", C.c_double), ("finite", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class DiracError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


# Every symbol include/dirac.h declares: name -> (restype, argtypes)
_vp = C.c_void_p
SIGNATURES = {
    "dirac_footprint_bytes": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Pml), C.c_int32]),
    "dirac_create_metric": (C.c_int32, [C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Pml), C.c_int32, _vp,
                                        C.c_size_t, _vp, C.POINTER(_vp)]),
    "dirac_footprint_bytes_scheme": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Pml), C.c_int32,
                                                   C.POINTER(Scheme)]),
    "dirac_footprint_bytes_ex": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Pml), C.c_int32,
                                               C.POINTER(Scheme), C.POINTER(Em)]),
    "dirac_create_solver": (C.c_int32, [C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Pml), C.c_int32,
                                        C.POINTER(Scheme), C.POINTER(Em), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "dirac_cn_stats": (C.c_int32, [_vp, C.POINTER(C.c_int64), _dp]),
    "dirac_cn_set_limits": (C.c_int32, [_vp, C.c_int32, C.c_double]),
    "dirac_set_initial_spinor": (C.c_int32, [_vp, _dp]),
    "dirac_set_initial_spinor_device": (C.c_int32, [_vp, _vp]),
    "dirac_step_n": (C.c_int32, [_vp, C.c_int64]),
    "dirac_observables": (C.c_int32, [_vp, C.POINTER(Obs)]),
    "dirac_observables_static": (C.c_int32, [_vp, C.POINTER(Obs)]),
    "dirac_get_spinor": (C.c_int32, [_vp, _dp]),
    "dirac_destroy": (C.c_int32, [_vp]),
    "dirac_last_error": (C.c_char_p, []),
    "dirac_schedule_count": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    "dirac_schedule_get": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Schedule)]),
    "dirac_get_schedule": (C.c_int32, [_vp, C.c_int32, C.POINTER(Schedule)]),
    "dirac_set_schedule": (C.c_int32, [_vp, C.c_int32, C.POINTER(Schedule)]),
    "dirac_set_launch_mode": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
    "dirac_set_potential_form": (C.c_int32, [_vp, C.c_int32]),
    "dirac_get_potential_form": (C.c_int32, [_vp, C.POINTER(C.c_int32)]),
    "dirac_set_store_mode": (C.c_int32, [_vp, C.c_int32]),
    "dirac_get_store_mode": (C.c_int32, [_vp, C.POINTER(C.c_int32)]),
    "dirac_step_n_timed": (C.c_int32, [_vp, C.c_int64, _dp, C.POINTER(C.c_int64)]),
    "dirac_autotune": (C.c_int32, [_vp, C.c_int32]),
    "dirac_time_directions": (C.c_int32, [_vp, C.c_int32, _dp]),
    "dirac_tune_cache_save": (C.c_int32, [C.c_char_p]),
    "dirac_tune_cache_load": (C.c_int32, [C.c_char_p]),
    "dirac_batch_footprint_bytes": (C.c_size_t, [C.c_int32]),
    "dirac_batch_create": (C.c_int32, [C.c_int32, C.c_int32, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "dirac_batch_add": (C.c_int32, [_vp, _vp, C.POINTER(C.c_int32)]),
    "dirac_batch_remove": (C.c_int32, [_vp, C.c_int32]),
    "dirac_batch_run": (C.c_int32, [_vp, C.POINTER(C.c_int64)]),
    "dirac_batch_prepare": (C.c_int32, [_vp, C.POINTER(C.c_int64)]),
    "dirac_batch_run_timed": (C.c_int32, [_vp, C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int64), _dp]),
    "dirac_batch_sync": (C.c_int32, [_vp]),
    "dirac_batch_set_graph": (C.c_int32, [_vp, C.c_int32]),
    "dirac_batch_destroy": (C.c_int32, [_vp]),
    "dirac_batch_schedule_count": (C.c_int32, [C.c_int32]),
    "dirac_batch_get_schedule": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.POINTER(Schedule)]),
    "dirac_batch_set_schedule": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.POINTER(Schedule)]),
    "dirac_batch_autotune": (C.c_int32, [_vp, C.c_int32]),
    "dirac3_footprint_bytes": (C.c_size_t, [C.POINTER(Grid3), C.POINTER(Metric3), C.POINTER(Pml), C.c_int32]),
    "dirac3_create": (C.c_int32, [C.POINTER(Grid3), C.POINTER(Metric3), C.POINTER(Pml), C.c_int32, _vp,
                                  C.c_size_t, _vp, C.POINTER(_vp)]),
    "dirac3_set_initial_spinor": (C.c_int32, [_vp, _dp]),
    "dirac3_set_initial_spinor_device": (C.c_int32, [_vp, _vp]),
    "dirac3_step_n": (C.c_int32, [_vp, C.c_int64]),
    "dirac3_set_launch_mode": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
    "dirac3_step_n_timed": (C.c_int32, [_vp, C.c_int64, _dp, C.POINTER(C.c_int64)]),
    "dirac3_observables": (C.c_int32, [_vp, C.POINTER(Obs3)]),
    "dirac3_get_spinor": (C.c_int32, [_vp, _dp]),
    "dirac3_destroy": (C.c_int32, [_vp]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1909_02894_amd.build` "
                          "(there is no non-HIP fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.dirac_last_error().decode()


def _check(status):
    if status != 0:
        raise DiracError(status, last_error())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def make_structs(n1, n2, a1, a2, dt, c, m, metric=METRIC_FLAT, spin=SPIN_NONE, bump_A=0.0, bump_s=1.0,
                 fields=None, pml_width=0, pml_type=1, pml_sigma0=1.0, pml_theta=0.0):
    g = Grid(n1, n2, a1, a2, dt, c, m)
    mt = Metric(kind=metric, spin=spin, bump_A=bump_A, bump_s=bump_s)
    keep = []
    if fields is not None:
        names = ("phi", "psi", "dphi_dx", "dphi_dy", "dpsi_dx", "dpsi_dy")
        for nm, arr in zip(names, fields):
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            assert arr.shape == (n2, n1)
            keep.append(arr)
            setattr(mt, nm, _ptr(arr))
    p = Pml(pml_width, pml_type, pml_sigma0, pml_theta)
    return g, mt, p, keep


def spec_structs(spec, fields=None):
    """Structs for a workloads.SolveSpec."""
    return make_structs(spec.n1, spec.n2, spec.a1, spec.a2, spec.dt, spec.c, spec.m, spec.metric, spec.spin,
                        spec.bump_A, spec.bump_s, fields, spec.pml_width, spec.pml_type, spec.pml_sigma0,
                        spec.pml_theta)


# ---- C-named wrappers ---------------------------------------------------------

def footprint_bytes(grid: Grid, metric: Metric, pml: Pml, precision: int) -> int:
    return int(lib.dirac_footprint_bytes(C.byref(grid), C.byref(metric), C.byref(pml), precision))


def create_metric(grid, metric, pml, precision, device_ptr: int, nbytes: int, stream_ptr: int | None):
    h = _vp()
    _check(lib.dirac_create_metric(C.byref(grid), C.byref(metric), C.byref(pml), precision, _vp(device_ptr),
                                   nbytes, _vp(stream_ptr or 0), C.byref(h)))
    return h


def footprint_bytes_scheme(grid: Grid, metric: Metric, pml: Pml, precision: int, scheme: Scheme | None) -> int:
    return int(lib.dirac_footprint_bytes_scheme(C.byref(grid), C.byref(metric), C.byref(pml), precision,
                                                C.byref(scheme) if scheme is not None else None))


def footprint_bytes_ex(grid: Grid, metric: Metric, pml: Pml, precision: int, scheme: Scheme | None,
                       em: Em | None) -> int:
    return int(lib.dirac_footprint_bytes_ex(C.byref(grid), C.byref(metric), C.byref(pml), precision,
                                            C.byref(scheme) if scheme is not None else None,
                                            C.byref(em) if em is not None else None))


def create_solver(grid, metric, pml, precision, scheme: Scheme | None, em: Em | None, device_ptr: int,
                  nbytes: int, stream_ptr: int | None):
    h = _vp()
    _check(lib.dirac_create_solver(C.byref(grid), C.byref(metric), C.byref(pml), precision,
                                   C.byref(scheme) if scheme is not None else None,
                                   C.byref(em) if em is not None else None, _vp(device_ptr), nbytes,
                                   _vp(stream_ptr or 0), C.byref(h)))
    return h


def make_em(n1, n2, V=None, Ax=None, Ay=None, charge=1.0, env_V=(1.0, 0, 0, 0, 0, 0), env_A=(1.0, 0, 0, 0, 0, 0)):
    """An Em struct and the arrays it points to (keep both alive until creation)."""
    keep = []

    def plane(a):
        if a is None:
            return None
        arr = np.ascontiguousarray(a, dtype=np.float64)
        assert arr.shape == (n2, n1)
        keep.append(arr)
        return arr.ctypes.data_as(_dp)
    em = Em(plane(V), plane(Ax), plane(Ay), charge, Envelope(*env_V), Envelope(*env_A))
    return em, keep


def cn_stats(h):
    it = C.c_int64()
    res = C.c_double()
    _check(lib.dirac_cn_stats(h, C.byref(it), C.byref(res)))
    return int(it.value), float(res.value)


def cn_set_limits(h, max_iter: int, rtol: float):
    _check(lib.dirac_cn_set_limits(h, int(max_iter), float(rtol)))


def set_initial_spinor(h, psi: np.ndarray):
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    _check(lib.dirac_set_initial_spinor(h, psi.view(np.float64).ctypes.data_as(_dp)))


def set_initial_spinor_device(h, dev_ptr: int):
    _check(lib.dirac_set_initial_spinor_device(h, _vp(dev_ptr)))


def step_n(h, nsteps: int):
    _check(lib.dirac_step_n(h, int(nsteps)))


def observables(h) -> dict:
    o = Obs()
    _check(lib.dirac_observables(h, C.byref(o)))
    return o.as_dict()


def observables_static(h) -> dict:
    """dirac_observables_static: the same values, reduced in the library's static
    device scratch (no allocation)."""
    o = Obs()
    _check(lib.dirac_observables_static(h, C.byref(o)))
    return o.as_dict()


def get_spinor(h, n1: int, n2: int) -> np.ndarray:
    out = np.empty((n2, n1, 2), dtype=np.complex128)
    _check(lib.dirac_get_spinor(h, out.view(np.float64).ctypes.data_as(_dp)))
    return out


def destroy(h):
    _check(lib.dirac_destroy(h))


def schedules(n: int, precision: int, direction: int):
    out = []
    for i in range(lib.dirac_schedule_count(n, precision, direction)):
        s = Schedule()
        _check(lib.dirac_schedule_get(n, precision, direction, i, C.byref(s)))
        out.append((s.radix, s.lines_per_wg, s.components_per_thread))
    return out


def tune_cache_save(path: str):
    _check(lib.dirac_tune_cache_save(path.encode()))


def tune_cache_load(path: str):
    _check(lib.dirac_tune_cache_load(path.encode()))


# ---- convenience object ----------------------------------------------------------

class Solver:
    """One solve on a torch-allocated device buffer and torch's current stream."""

    def __init__(self, n1, n2, a1, a2, dt, c=1.0, m=1.0, precision=FP64, metric=METRIC_FLAT, spin=SPIN_NONE,
                 bump_A=0.0, bump_s=1.0, fields=None, pml_width=0, pml_type=1, pml_sigma0=1.0, pml_theta=0.0,
                 device=None, stream=None, scheme=SCHEME_EXP_SPLIT, gmres_restart=0, gmres_max_iter=0,
                 gmres_rtol=0.0, potentials=None):
        """potentials: None, or a dict with keys V, Ax, Ay (arrays [n2][n1] or None),
        charge, env_V, env_A ((c0, c1, omega, phase, t0, tau) tuples)."""
        import torch
        self.n1, self.n2, self.precision = n1, n2, precision
        self.grid, self.metric, self.pml, keep = make_structs(n1, n2, a1, a2, dt, c, m, metric, spin, bump_A,
                                                              bump_s, fields, pml_width, pml_type, pml_sigma0,
                                                              pml_theta)
        self.scheme = Scheme(scheme, gmres_restart, gmres_max_iter, 0, gmres_rtol)
        self.em, keep_em = (None, None) if potentials is None else make_em(n1, n2, **potentials)
        self.nbytes = footprint_bytes_ex(self.grid, self.metric, self.pml, precision, self.scheme, self.em)
        if self.nbytes == 0:
            raise DiracError(-1, last_error())
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(device)
        self.buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.h = None
        self.h = create_solver(self.grid, self.metric, self.pml, precision, self.scheme, self.em,
                               self.buffer.data_ptr(), self.nbytes, self.stream.cuda_stream)
        del keep_em
        del keep

    @classmethod
    def from_spec(cls, spec, precision=FP64, fields=None, **kw):
        return cls(spec.n1, spec.n2, spec.a1, spec.a2, spec.dt, spec.c, spec.m, precision, spec.metric, spec.spin,
                   spec.bump_A, spec.bump_s, fields, spec.pml_width, spec.pml_type, spec.pml_sigma0,
                   spec.pml_theta, **kw)

    def set_initial_spinor(self, psi):
        set_initial_spinor(self.h, psi)

    def set_initial_spinor_device(self, tensor):
        assert tensor.is_contiguous() and tensor.numel() * tensor.element_size() == self.n1 * self.n2 * 32
        set_initial_spinor_device(self.h, tensor.data_ptr())

    def step_n(self, n):
        step_n(self.h, n)

    def observables(self):
        return observables(self.h)

    def get_spinor(self):
        return get_spinor(self.h, self.n1, self.n2)

    def schedule(self, direction):
        s = Schedule()
        _check(lib.dirac_get_schedule(self.h, direction, C.byref(s)))
        return (s.radix, s.lines_per_wg, s.components_per_thread)

    def set_schedule(self, direction, radix, lines, components=2):
        s = Schedule(radix, lines, components)
        _check(lib.dirac_set_schedule(self.h, direction, C.byref(s)))

    def set_launch_mode(self, use_graph: bool, chunk: int = 32):
        _check(lib.dirac_set_launch_mode(self.h, int(use_graph), chunk))

    def set_potential_form(self, form: int):
        """Potentials: 0 by size, 1 exponentials inside the direction kernels, 2 a pointwise pass."""
        _check(lib.dirac_set_potential_form(self.h, int(form)))

    def potential_pass(self) -> bool:
        v = C.c_int32()
        _check(lib.dirac_get_potential_form(self.h, C.byref(v)))
        return bool(v.value)

    def store_mode(self) -> int:
        """Write-through mask of the direction kernels' state stores: bit 0 x, bit 1 y."""
        v = C.c_int32()
        _check(lib.dirac_get_store_mode(self.h, C.byref(v)))
        return v.value

    def set_store_mode(self, mask: int):
        _check(lib.dirac_set_store_mode(self.h, int(mask)))

    def step_n_timed(self, n):
        ms = (C.c_double * 2)()
        cnt = (C.c_int64 * 2)()
        _check(lib.dirac_step_n_timed(self.h, int(n), ms, cnt))
        return [ms[0], ms[1]], [cnt[0], cnt[1]]

    def autotune(self, reps=20):
        _check(lib.dirac_autotune(self.h, reps))

    def time_directions(self, reps=200):
        """Microseconds per launch of the x and y kernels (each replayed alone)."""
        us = (C.c_double * 2)()
        _check(lib.dirac_time_directions(self.h, reps, us))
        return [us[0], us[1]]

    def cn_set_limits(self, max_iter: int, rtol: float):
        cn_set_limits(self.h, max_iter, rtol)

    def cn_stats(self):
        """(total GMRES iterations, last relative residual) of a Scheme I solver."""
        return cn_stats(self.h)

    def close(self):
        if self.h is not None:
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_structs3(n1, n2, n3, a1, a2, a3, dt, c, m, metric=METRIC_FLAT, spin=SPIN_NONE, fields=None,
                  pml_width=0, pml_type=1, pml_sigma0=1.0, pml_theta=0.0):
    """Grid3, Metric3, Pml and the arrays the metric points to (FIELDS: eight
    planes phi, psi, dphi_dx, dphi_dy, dphi_dz, dpsi_dx, dpsi_dy, dpsi_dz)."""
    keep = []
    ptrs = [None] * 8
    if fields is not None:
        for k, f in enumerate(fields):
            arr = np.ascontiguousarray(f, dtype=np.float64)
            assert arr.shape == (n3, n2, n1)
            keep.append(arr)
            ptrs[k] = arr.ctypes.data_as(_dp)
    return (Grid3(n1, n2, n3, a1, a2, a3, dt, c, m), Metric3(metric, spin, *ptrs),
            Pml(pml_width, pml_type, pml_sigma0, pml_theta), keep)


class Solver3:
    """One 3-D, 4-spinor solve on a torch-allocated device buffer and torch's current stream."""

    def __init__(self, n1, n2, n3, a1, a2, a3, dt, c=1.0, m=1.0, precision=FP64, metric=METRIC_FLAT,
                 spin=SPIN_NONE, fields=None, pml_width=0, pml_type=1, pml_sigma0=1.0, pml_theta=0.0,
                 device=None, stream=None):
        import torch
        self.shape = (n3, n2, n1)
        self.precision = precision
        self.grid, self.metric, self.pml, keep = make_structs3(n1, n2, n3, a1, a2, a3, dt, c, m, metric, spin,
                                                               fields, pml_width, pml_type, pml_sigma0, pml_theta)
        self.nbytes = int(lib.dirac3_footprint_bytes(C.byref(self.grid), C.byref(self.metric), C.byref(self.pml),
                                                     precision))
        if self.nbytes == 0:
            raise DiracError(-1, last_error())
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(device)
        self.buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.h = None
        h = _vp()
        _check(lib.dirac3_create(C.byref(self.grid), C.byref(self.metric), C.byref(self.pml), precision,
                                 _vp(self.buffer.data_ptr()), self.nbytes, _vp(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        del keep

    def set_initial_spinor(self, psi):
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        assert psi.shape == self.shape + (4,)
        _check(lib.dirac3_set_initial_spinor(self.h, psi.view(np.float64).ctypes.data_as(_dp)))

    def set_initial_spinor_device(self, tensor):
        n3, n2, n1 = self.shape
        assert tensor.is_contiguous() and tensor.numel() * tensor.element_size() == n1 * n2 * n3 * 64
        _check(lib.dirac3_set_initial_spinor_device(self.h, _vp(tensor.data_ptr())))

    def step_n(self, n):
        _check(lib.dirac3_step_n(self.h, int(n)))

    def set_launch_mode(self, use_graph: bool, chunk: int = 16):
        _check(lib.dirac3_set_launch_mode(self.h, int(use_graph), chunk))

    def step_n_timed(self, n):
        ms = (C.c_double * 3)()
        cnt = (C.c_int64 * 3)()
        _check(lib.dirac3_step_n_timed(self.h, int(n), ms, cnt))
        return list(ms), list(cnt)

    def observables(self):
        o = Obs3()
        _check(lib.dirac3_observables(self.h, C.byref(o)))
        return o.as_dict()

    def get_spinor(self):
        out = np.empty(self.shape + (4,), dtype=np.complex128)
        _check(lib.dirac3_get_spinor(self.h, out.view(np.float64).ctypes.data_as(_dp)))
        return out

    def close(self):
        if self.h is not None:
            _check(lib.dirac3_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many solves advanced together by the batch engine (one graph launch per run)."""

    def __init__(self, precision=FP32, capacity=256, device=None, stream=None):
        import torch
        self.precision, self.capacity = precision, capacity
        self.nbytes = int(lib.dirac_batch_footprint_bytes(capacity))
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(device)
        self.buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.h = _vp()
        _check(lib.dirac_batch_create(precision, capacity, _vp(self.buffer.data_ptr()), self.nbytes,
                                      _vp(self.stream.cuda_stream), C.byref(self.h)))
        self.members = {}

    def add(self, solver: "Solver") -> int:
        slot = C.c_int32()
        _check(lib.dirac_batch_add(self.h, solver.h, C.byref(slot)))
        self.members[slot.value] = solver
        return slot.value

    def remove(self, slot: int):
        _check(lib.dirac_batch_remove(self.h, slot))
        self.members.pop(slot, None)

    def run(self, steps):
        """steps: dict slot -> n, or a sequence of capacity entries."""
        _check(lib.dirac_batch_run(self.h, self._steps_array(steps)))

    def _steps_array(self, steps):
        arr = (C.c_int64 * self.capacity)()
        if isinstance(steps, dict):
            for k, v in steps.items():
                arr[k] = int(v)
        else:
            for k, v in enumerate(steps):
                arr[k] = int(v)
        return arr

    def prepare(self, steps):
        """Record and instantiate the graph of run(steps) without launching it."""
        _check(lib.dirac_batch_prepare(self.h, self._steps_array(steps)))

    def run_timed(self, steps):
        """Run with per-launch events (synchronises).  Returns {(direction, n or
        'multi'): (ms summed, launches, algorithmic bytes)} for the kernel classes
        that ran."""
        ms = (C.c_double * 18)()
        cnt = (C.c_int64 * 18)()
        byt = (C.c_double * 18)()
        _check(lib.dirac_batch_run_timed(self.h, self._steps_array(steps), ms, cnt, byt))
        out = {}
        for c in range(18):
            if cnt[c]:
                d, k = divmod(c, 9)
                out[(d, "multi" if k == 8 else 1 << (k + 4))] = (ms[c], int(cnt[c]), byt[c])
        return out

    def sync(self):
        _check(lib.dirac_batch_sync(self.h))

    def set_graph(self, use_graph: bool):
        _check(lib.dirac_batch_set_graph(self.h, int(use_graph)))

    def schedule(self, n: int, direction: int):
        s = Schedule()
        _check(lib.dirac_batch_get_schedule(self.h, n, direction, C.byref(s)))
        return (s.radix, s.lines_per_wg, s.components_per_thread)

    def set_schedule(self, n: int, direction: int, radix: int, components: int, lines: int = 0):
        s = Schedule(radix, lines, components)
        _check(lib.dirac_batch_set_schedule(self.h, n, direction, C.byref(s)))

    def autotune(self, reps: int = 5):
        _check(lib.dirac_batch_autotune(self.h, reps))

    def close(self):
        if self.h is not None and self.h.value:
            _check(lib.dirac_batch_destroy(self.h))
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
