"""Tile plans of the step kernel, checked on the host through lbm_tile_plan
(no device call): every node of the domain belongs to exactly one tile, the
strips are cut as described (column-edge chunks, 3-row head and tail,
near-equal chunks between), the launch order is row-major, and the
automatic height is the shortest that fits the SIMDs at once."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def L():
    from paper_2009_05264_amd import build_lib
    from paper_2009_05264_amd import lbmflow

    if build_lib.stale():
        build_lib.build()
    return lbmflow


def covers_once(nx, ny, tiles):
    cnt = np.zeros((ny, nx), np.int32)
    for x0, y0, y1 in tiles:
        cnt[y0:y1, x0:min(x0 + 60, nx)] += 1
    return bool((cnt == 1).all())


def column_edge(x0, nx):
    return not (x0 >= 3 and x0 + 62 < nx)


def test_every_node_in_exactly_one_tile(L):
    rng = np.random.default_rng(11)
    shapes = [(3, 3), (60, 5), (61, 7), (63, 64), (64, 9), (125, 37), (253, 37), (1600, 200), (8192, 40)]
    shapes += [(int(rng.integers(3, 700)), int(rng.integers(3, 300))) for _ in range(40)]
    for nx, ny in shapes:
        for rows in (0, 2, 3, 4, 5, 7, 8, 11, 16, 64):
            r, tiles = L.tile_plan(nx, ny, rows=rows)
            assert r >= 2 and all(0 <= y0 < y1 <= ny for _, y0, y1 in tiles), (nx, ny, rows)
            assert covers_once(nx, ny, tiles), (nx, ny, rows)


def test_strip_cuts(L):
    for nx, ny, rows in ((1600, 200, 7), (1600, 200, 8), (253, 37, 11), (400, 100, 4), (700, 90, 15)):
        r, tiles = L.tile_plan(nx, ny, rows=rows)
        assert r == rows
        strips = {}
        for x0, y0, y1 in tiles:
            strips.setdefault(x0, []).append((y0, y1))
        for x0, seg in strips.items():
            seg.sort()
            h = [y1 - y0 for y0, y1 in seg]
            if column_edge(x0, nx):
                re_ = max(1, (rows + 1) // 4)
                assert all(v == re_ for v in h[:-1]) and 1 <= h[-1] <= re_, (x0, h)
            else:
                # 3-row head and tail (the rows within two of a wall), near-equal chunks between
                assert h[0] == 3 and h[-1] == 3, (x0, h)
                mid = h[1:-1]
                assert max(mid) <= rows and max(mid) - min(mid) <= 1, (x0, mid)


def test_launch_order_is_row_major(L):
    _, tiles = L.tile_plan(1600, 200)
    keys = [(y0, x0) for x0, y0, _ in tiles]
    assert keys == sorted(keys)


def test_automatic_heights(L):
    # the figures quoted for the benchmark channel and the size sweep
    assert L.tile_plan(1600, 200)[0] == 7 and len(L.tile_plan(1600, 200)[1]) == 950
    assert len(L.tile_plan(1600, 200, rows=8)[1]) == 875
    assert L.tile_plan(200, 50)[0] == 4 and L.tile_plan(800, 200)[0] == 5
    # several rounds of waves: 7 rows with FP32 storage, 8 with 16-bit storage
    assert L.tile_plan(8192, 1024)[0] == 7
    # 16-bit storage: 8 rows while the state fits the Infinity Cache, 12 once
    # it streams from HBM (A/B state above 224 MiB)
    assert L.tile_plan(1600, 400, storage=L.STORE_F16_DEV)[0] == 8
    assert L.tile_plan(3200, 800, storage=L.STORE_F16_DEV)[0] == 8
    assert L.tile_plan(8192, 1024, storage=L.STORE_F16_DEV)[0] == 12
    assert L.tile_plan(8192, 1024, storage=L.STORE_BF16_DEV)[0] == 12
    # shortest height whose tiles and 16 finalizer waves fit the SIMDs at once
    for nx, ny, simds in ((1600, 200, 1024), (800, 200, 1024), (1200, 200, 1024), (1600, 200, 2048),
                          (400, 100, 256), (3000, 300, 4096)):
        r, tiles = L.tile_plan(nx, ny, simds=simds)
        if r < 7:
            assert len(tiles) + 16 <= simds, (nx, ny, r)
        if r <= 7:
            for q in range(4, r):
                assert len(L.tile_plan(nx, ny, rows=q)[1]) + 16 > simds, (nx, ny, q)
    # a larger device takes shorter tiles for the same channel
    assert L.tile_plan(1600, 200, simds=2048)[0] < L.tile_plan(1600, 200)[0]


def test_bad_arguments(L):
    for kw in (dict(nx=2, ny=10), dict(nx=10, ny=2), dict(nx=10, ny=10, rows=-1),
               dict(nx=10, ny=10, storage=9)):
        with pytest.raises(L.LbmError) as e:
            L.tile_plan(**kw)
        assert e.value.code == L.LBM_E_INVALID
