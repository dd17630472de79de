"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/dirac.h declares, sizes footprints and rejects invalid
arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "dirac.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dirac_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("dirac_create_metric", "dirac_set_initial_spinor", "dirac_step_n", "dirac_observables",
                     "dirac_get_spinor", "dirac_destroy", "dirac_footprint_bytes", "dirac_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1909_02894_amd import dirac as D
    lib = ctypes.CDLL(D.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
        assert name in D.SIGNATURES, f"binding lacks {name}"


def test_footprint_and_validation():
    from paper_1909_02894_amd import dirac as D
    g, m, p, _ = D.make_structs(512, 512, 20.0, 20.0, 0.01, 1.0, 0.0, metric=D.METRIC_GAUSS_BUMP,
                                spin=D.SPIN_2P1, bump_A=1.0, bump_s=3.0, pml_width=32)
    f64 = D.footprint_bytes(g, m, p, D.FP64)
    f32 = D.footprint_bytes(g, m, p, D.FP32)
    N = 512 * 512
    # state + a + E (T) + 5 FP64 observable planes + 32-byte staging per point
    assert f64 >= N * (32 + 8 + 32 + 40 + 32) and f32 >= N * (16 + 4 + 16 + 40 + 32)
    assert f32 < f64
    gf, mf, pf, _ = D.make_structs(64, 64, 20.0, 20.0, 0.01, 1.0, 1.0)
    assert D.footprint_bytes(gf, mf, pf, D.FP64) < D.footprint_bytes(*D.make_structs(64, 64, 20.0, 20.0, 0.01, 1.0, 1.0, metric=D.METRIC_PAPER_EXP3)[:3], D.FP64)

    def create_status(**kw):
        args = dict(n1=64, n2=64, a1=5.0, a2=5.0, dt=0.01, c=1.0, m=1.0)
        args.update(kw)
        g, m, p, keep = D.make_structs(**args)
        h = ctypes.c_void_p()
        return D.lib.dirac_create_metric(ctypes.byref(g), ctypes.byref(m), ctypes.byref(p), 0, None, 0, None,
                                         ctypes.byref(h))

    assert create_status(n1=48) == -2                 # not a power of two
    assert create_status(n2=8) == -2                  # below 16
    assert create_status(n1=16384) == -2              # above 8192
    assert create_status(dt=0.0) == -1
    assert create_status(c=-1.0) == -1
    assert create_status(metric=7) == -1
    assert create_status(metric=D.METRIC_FIELDS) == -1            # arrays missing
    assert create_status(pml_width=40) == -1                      # wider than half the grid
    assert create_status(pml_width=8, pml_type=9) == -1
    assert create_status(pml_width=8, pml_theta=0.3) == -3        # complex stretch: unstable
    assert "stable only for real b" in D.last_error()
    assert create_status() == -1                                  # valid grid, null device buffer
    assert "null device buffer" in D.last_error()


def test_null_handles_are_rejected():
    from paper_1909_02894_amd import dirac as D
    assert D.lib.dirac_step_n(None, 1) == -1
    assert D.lib.dirac_observables(None, None) == -1
    assert D.lib.dirac_destroy(None) == -1
    assert D.lib.dirac_set_store_mode(None, 1) == -1
    assert D.lib.dirac_get_store_mode(None, None) == -1


def test_every_size_and_precision_has_kernels():
    from paper_1909_02894_amd import dirac as D
    for prec in (D.FP64, D.FP32):
        for d in (0, 1):
            for k in range(4, 13):
                n = 1 << k
                if prec == D.FP64 and n > 4096:
                    continue
                sch = D.schedules(n, prec, d)
                assert sch, (prec, d, n)
                for r, lines, cpt in sch:
                    # cpt = 1: 2 (n / r) lines threads, 32 logical threads per wave
                    nt = (n // r) * lines * (2 if cpt == 1 else 1)
                    assert n % r == 0 and nt <= 1024 and (cpt == 2 or (n // r) * lines % 32 == 0)


def test_scheme_selection_is_validated():
    from paper_1909_02894_amd import dirac as D
    g, m, p, _ = D.make_structs(256, 128, 10.0, 10.0, 0.01, 1.0, 1.0, pml_width=16)
    split = D.footprint_bytes(g, m, p, D.FP64)
    assert D.footprint_bytes_scheme(g, m, p, D.FP64, None) == split
    assert D.footprint_bytes_scheme(g, m, p, D.FP64, D.Scheme(D.SCHEME_EXP_SPLIT, 0, 0, 0, 0.0)) == split
    cn = D.footprint_bytes_scheme(g, m, p, D.FP64, D.Scheme(D.SCHEME_CN_GMRES, 10, 0, 0, 0.0))
    # GMRES(10): rhs, work and 11 Krylov vectors of 32 bytes per point
    assert cn >= split + 13 * 256 * 128 * 32
    assert D.footprint_bytes_scheme(g, m, p, D.FP64, D.Scheme(D.SCHEME_CN_GMRES, 20, 0, 0, 0.0)) > cn

    def create_status(scheme, prec=D.FP64, **kw):
        args = dict(n1=64, n2=64, a1=5.0, a2=5.0, dt=0.01, c=1.0, m=1.0)
        args.update(kw)
        g, m, p, keep = D.make_structs(**args)
        h = ctypes.c_void_p()
        return D.lib.dirac_create_solver(ctypes.byref(g), ctypes.byref(m), ctypes.byref(p), prec,
                                         ctypes.byref(scheme), None, None, 0, None, ctypes.byref(h))

    CN = D.SCHEME_CN_GMRES
    assert create_status(D.Scheme(5, 0, 0, 0, 0.0)) == -1                     # unknown scheme
    assert create_status(D.Scheme(CN, 0, 0, 0, 0.0), prec=D.FP32) == -1       # FP64 only
    assert "FP64" in D.last_error()
    assert create_status(D.Scheme(CN, 0, 0, 0, 0.0), n1=4096) == -2           # n <= 2048
    assert create_status(D.Scheme(CN, 1, 0, 0, 0.0)) == -1                    # restart below 2
    assert create_status(D.Scheme(CN, 64, 0, 0, 0.0)) == -1                   # restart above 63
    assert create_status(D.Scheme(CN, 0, -3, 0, 0.0)) == -1
    assert create_status(D.Scheme(CN, 0, 0, 0, -1e-9)) == -1
    assert create_status(D.Scheme(CN, 0, 0, 0, float("nan"))) == -1
    assert create_status(D.Scheme(CN, 0, 0, 0, 0.0), pml_width=8, pml_theta=0.3) == -1
    assert "real stretch" in D.last_error()
    assert create_status(D.Scheme(CN, 0, 0, 0, 0.0)) == -1                    # valid; null device buffer
    assert "null device buffer" in D.last_error()
    assert D.lib.dirac_cn_stats(None, None, None) == -1


def test_step2bis_scheme_validation():
    from paper_1909_02894_amd import dirac as D
    g, m, p, _ = D.make_structs(256, 128, 20.0, 20.0, 0.01, 1.0, 0.0, metric=D.METRIC_GAUSS_BUMP,
                                spin=D.SPIN_2P1, bump_A=1.0, bump_s=3.0, pml_width=16)
    plain = D.footprint_bytes(g, m, p, D.FP64)
    printed = D.footprint_bytes_scheme(g, m, p, D.FP64, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS_PRINTED, 0, 0, 0, 0.0))
    corr = D.footprint_bytes_scheme(g, m, p, D.FP64, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS, 0, 0, 0, 0.0))
    assert printed == plain
    assert corr >= plain + 256 * 128 * 16                  # (d_x a, d_y a) per point
    # flat solves carry no gradient table
    gf, mf, pf, _ = D.make_structs(64, 64, 5.0, 5.0, 0.01, 1.0, 1.0, pml_width=4)
    assert (D.footprint_bytes_scheme(gf, mf, pf, D.FP32, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS, 0, 0, 0, 0.0))
            == D.footprint_bytes(gf, mf, pf, D.FP32))
    # printed form: c dt max|xi| = 0.05 pi 256 / 5 > sqrt(2)
    gb, mb, pb, _ = D.make_structs(512, 512, 5.0, 5.0, 0.05, 1.0, 1.0)
    assert D.footprint_bytes_scheme(gb, mb, pb, D.FP64, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS_PRINTED, 0, 0, 0, 0.0)) == 0
    assert "sqrt(2)" in D.last_error()
    assert D.footprint_bytes_scheme(gb, mb, pb, D.FP64, None) > 0
    g4, m4, p4, _ = D.make_structs(4096, 64, 5.0, 5.0, 1e-4, 1.0, 1.0)
    assert D.footprint_bytes_scheme(g4, m4, p4, D.FP32, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS, 0, 0, 0, 0.0)) == 0
    assert D.footprint_bytes_scheme(g4, m4, p4, D.FP32, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS_PRINTED, 0, 0, 0, 0.0)) > 0
    assert D.footprint_bytes_scheme(g4, m4, p4, D.FP32, D.Scheme(7, 0, 0, 0, 0.0)) == 0


def test_potentials_validation_and_footprint():
    import numpy as np
    from paper_1909_02894_amd import dirac as D
    g, m, p, _ = D.make_structs(128, 64, 10.0, 10.0, 0.01, 1.0, 1.0)
    base = D.footprint_bytes(g, m, p, D.FP64)
    V = np.zeros((64, 128))
    em, keep = D.make_em(128, 64, V=V, charge=0.5, env_A=(0.0, 1.0, 3.0, 0.0, 0.2, 0.1))
    with_em = D.footprint_bytes_ex(g, m, p, D.FP64, None, em)
    # 8 FP64 per point for the exponential record, 3 more observable planes
    assert with_em >= base + 128 * 64 * (64 + 24)
    assert D.footprint_bytes_ex(g, m, p, D.FP64, None, None) == base
    assert D.footprint_bytes_ex(g, m, p, D.FP64, D.Scheme(D.SCHEME_CN_GMRES, 0, 0, 0, 0.0), em) > 0
    assert D.footprint_bytes_ex(g, m, p, D.FP32, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS_PRINTED, 0, 0, 0, 0.0), em) > 0
    assert D.footprint_bytes_ex(g, m, p, D.FP64, D.Scheme(D.SCHEME_EXP_SPLIT_2BIS, 0, 0, 0, 0.0), em) == 0
    bad, keep2 = D.make_em(128, 64, V=V, env_V=(1.0, 0.0, 0.0, 0.0, 0.0, -1.0))
    assert D.footprint_bytes_ex(g, m, p, D.FP64, None, bad) == 0 and "tau" in D.last_error()
    bad, keep3 = D.make_em(128, 64, charge=float("inf"))
    assert D.footprint_bytes_ex(g, m, p, D.FP64, None, bad) == 0
    g4, m4, p4, _ = D.make_structs(4096, 64, 10.0, 10.0, 0.001, 1.0, 1.0)
    em4, keep4 = D.make_em(4096, 64)
    assert D.footprint_bytes_ex(g4, m4, p4, D.FP32, None, em4) == 0 and "2048" in D.last_error()


def test_3d_footprint_and_validation():
    from paper_1909_02894_amd import dirac as D
    g, m, p, _ = D.make_structs3(64, 32, 16, 5.0, 4.0, 3.0, 0.01, 1.0, 1.0, metric=D.METRIC_PAPER_EXP3,
                                 spin=D.SPIN_PAPER, pml_width=4)
    N = 64 * 32 * 16
    f64 = D.lib.dirac3_footprint_bytes(ctypes.byref(g), ctypes.byref(m), ctypes.byref(p), D.FP64)
    f32 = D.lib.dirac3_footprint_bytes(ctypes.byref(g), ctypes.byref(m), ctypes.byref(p), D.FP32)
    # state 8 T, a, E record (6 FP64 / 8 FP32), weight, 64-byte staging per point
    assert f64 >= N * (64 + 8 + 48 + 8 + 64) and f32 >= N * (32 + 4 + 32 + 8 + 64) and f32 < f64

    def status(**kw):
        args = dict(n1=32, n2=32, n3=32, a1=5.0, a2=5.0, a3=5.0, dt=0.01, c=1.0, m=1.0)
        args.update(kw)
        g, m, p, keep = D.make_structs3(**args)
        h = ctypes.c_void_p()
        return D.lib.dirac3_create(ctypes.byref(g), ctypes.byref(m), ctypes.byref(p), 0, None, 0, None,
                                   ctypes.byref(h))
    assert status(n3=48) == -2
    assert status(n1=2048) == -2
    assert status(n1=1024, n2=1024, n3=256) == -2            # state beyond 2 GiB
    assert status(metric=D.METRIC_GAUSS_BUMP) == -1
    assert status(metric=D.METRIC_FIELDS) == -1
    assert status(pml_width=20) == -1
    assert status(pml_width=4, pml_theta=0.5) == -3
    assert status(dt=-1.0) == -1
    assert status() == -1 and "null device buffer" in D.last_error()
    assert D.lib.dirac3_step_n(None, 1) == -1


def test_tune_cache_round_trip(tmp_path):
    # the cache file keeps schedules and the store mode; files written before
    # the store-mode column load with ordinary stores
    from paper_1909_02894_amd import dirac as D
    src = tmp_path / "in.txt"
    src.write_text("# prec n dir other mode radix lines components ms_per_step write_through\n"
                   "0 512 0 512 3 8 1 2 0.0121 1\n"
                   "0 512 1 512 3 8 2 1 0.0123 1\n"
                   "1 256 0 256 2 4 1 1 0.005\n")
    D.tune_cache_load(str(src))
    out = tmp_path / "out.txt"
    D.tune_cache_save(str(out))
    rows = {tuple(l.split()[:5]): l.split()[5:] for l in out.read_text().splitlines() if not l.startswith("#")}
    assert rows[("0", "512", "0", "512", "3")][:3] == ["8", "1", "2"] and rows[("0", "512", "0", "512", "3")][-1] == "1"
    assert rows[("0", "512", "1", "512", "3")][-1] == "1"
    assert rows[("1", "256", "0", "256", "2")][:3] == ["4", "1", "1"] and rows[("1", "256", "0", "256", "2")][-1] == "0"
    with pytest.raises(D.DiracError):
        D.tune_cache_load(str(tmp_path / "missing.txt"))
