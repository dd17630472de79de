"""Host logic of the serving loop that needs no GPU: the first-fit arena."""
import pytest

torch = pytest.importorskip("torch")


def test_arena_first_fit_and_merge():
    from paper_1909_02894_amd.serve import Arena
    a = Arena(10 * 256, torch.device("cpu"))
    x = a.alloc(300)            # 2 granules
    y = a.alloc(256)
    z = a.alloc(5 * 256)
    assert x == (0, 512) and y == (512, 256) and z == (768, 1280)
    assert a.alloc(1024) is None and a.used == 2048
    a.release(*y)
    t = a.alloc(512)
    assert t == (2048, 512)               # the 1-granule hole is skipped (first fit)
    assert a.alloc(512) is None
    a.release(*x)
    assert a.free[0] == (0, 768)          # merged with the released neighbour
    w = a.alloc(700)
    assert w == (0, 768)
    for blk in (w, z, t):
        a.release(*blk)
    assert a.free == [(0, 2560)] and a.used == 0


def test_quantum_plans():
    # share: every running solve advances min(quantum, remaining); srpt: least
    # remaining work (points x steps) first, until the grid points reach the target
    from types import SimpleNamespace as NS
    from paper_1909_02894_amd import serve as S
    from paper_1909_02894_amd import workloads as W

    def run(rid, n, remaining):
        spec = W.flat_small(n=n, steps=remaining)
        return S._Running(S.Request(rid, 0.0, spec, remaining), None, rid, 0, 0, remaining)

    running = {0: run(0, 256, 100), 1: run(1, 64, 30), 2: run(2, 128, 500), 3: run(3, 64, 1000)}
    share = NS(policy="share", quantum=64, fill_points=0)
    assert S.Server._plan(share, running) == {0: 64, 1: 30, 2: 64, 3: 64}
    # work: 1 -> 64*64*30 = 122880, 3 -> 4096000, 0 -> 6553600, 2 -> 8192000
    srpt = NS(policy="srpt", quantum=64, fill_points=64 * 64 * 2)
    assert S.Server._plan(srpt, running) == {1: 30, 3: 64}
    srpt.fill_points = 1
    assert S.Server._plan(srpt, running) == {1: 30}
    srpt.fill_points = 1 << 30
    assert S.Server._plan(srpt, running) == {1: 30, 3: 64, 0: 64, 2: 64}
