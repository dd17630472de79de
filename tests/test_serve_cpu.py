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
