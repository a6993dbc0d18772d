"""dmk_tree_bin on the GPU against the CPU statement of the binning:
bit-identical keys, permutation, box starts, sorted wrapped coordinates and
axis tables; structural checks of the target tiles."""
import numpy as np
import pytest

from binning_spec import axis_tables_spec, bin_spec, heavy_count_spec, tiles_spec
from gpu_util import HAVE_GPU, dev, host, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_2606_27134_amd import residual as R
    from paper_2606_27134_amd import _lib as L


HEAVY_LOG = 16  # tiles of cost 2^16 - 1 or more run with the larger workgroup


def _points(seed, N, Lv, D, kind):
    rng = np.random.default_rng(seed)
    x = rng.random((N, 3)) * np.asarray(Lv)
    if kind == "faces":
        h = np.asarray(Lv) / 8
        k = rng.integers(0, 9, size=(N, 3))
        on = rng.random((N, 3)) < 0.5
        x = np.where(on, k * h, x)
        # free axes must stay inside [0, L)
        for ax in range(D, 3):
            x[:, ax] = np.where(x[:, ax] >= Lv[ax], np.nextafter(Lv[ax], 0.0), x[:, ax])
        x[:5, :] = np.nextafter(np.asarray(Lv), 0.0)
    elif kind == "outside":
        for ax in range(D):
            x[:, ax] += rng.integers(-3, 4, size=N) * Lv[ax]
        x[:3, 0] = -1e-300 if D > 0 else x[:3, 0]
        x[3:6, 0] = -0.0 if D > 0 else x[3:6, 0]
    return x


CASES = [
    ((1.0, 1.0, 1.0), 3, (8, 8, 8), "uniform"),
    ((1.0, 1.0, 1.0), 3, (8, 8, 8), "faces"),
    ((1.0, 1.0, 4.0), 2, (5, 3, 17), "outside"),
    ((32.0, 1.0, 1.0), 1, (64, 2, 2), "outside"),
    ((0.7, 1.3, 0.9), 0, (3, 7, 5), "faces"),
    ((1.0, 1.0, 1.0), 3, (1, 2, 1), "uniform"),
    ((0.1, 0.3, 0.2), 3, (1, 1, 1), "outside"),
]

# larger cases: the radix histograms span several chunks of the device scan
# (N = 200,000 -> 25,088 counters); the 10^6-point tiling; columns taller than the 2048 boxes the
# tile walk stages in LDS, periodic and free in z
BIG = [
    ((1.0, 1.0, 1.0), 3, (32, 32, 32), 200_000),
    ((1.0, 1.0, 8.0), 3, (2, 3, 2100), 30_000),
    ((1.0, 1.0, 8.0), 2, (2, 2, 2500), 30_000),
    ((1.0, 1.0, 1.0), 3, (64, 64, 64), 1_000_000),  # the Laplace 10^6-point workload's tiling
    ((32.0, 1.0, 1.0), 1, (256, 80, 2), 100_000),   # 20,480 columns: the column scan in blocks
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_binning_bit_exact(case):
    Lv, D, n, kind = CASES[case]
    N = 5000 + 37 * case
    x = _points(100 + case, N, Lv, D, kind)
    print("binning case", case, Lv, D, n, kind, flush=True)
    ref = bin_spec(x, Lv, D, n)
    assert ref["ok"]
    b = R.tree_bin(Lv, D, n, dev(x))
    np.testing.assert_array_equal(host(b.key()), ref["key"])
    np.testing.assert_array_equal(host(b.perm()), ref["perm"])
    np.testing.assert_array_equal(host(b.skey()), ref["skey"])
    np.testing.assert_array_equal(host(b.box_start()), ref["box_start"])
    ys = host(b.ys())
    assert ys.tobytes() == ref["ys"].tobytes()
    nbr, img = b.axis_tables()
    rn, ri = axis_tables_spec(D, n)
    np.testing.assert_array_equal(host(nbr), rn)
    np.testing.assert_array_equal(host(img), ri)
    _check_tiles(b, n, ref, D)


@pytest.mark.parametrize("case", range(len(BIG)))
def test_binning_bit_exact_large(case):
    Lv, D, n, N = BIG[case]
    x = _points(300 + case, N, Lv, D, "uniform")
    print("binning large case", case, Lv, D, n, N, flush=True)
    ref = bin_spec(x, Lv, D, n)
    b = R.tree_bin(Lv, D, n, dev(x))
    np.testing.assert_array_equal(host(b.perm()), ref["perm"])
    np.testing.assert_array_equal(host(b.box_start()), ref["box_start"])
    assert host(b.ys()).tobytes() == ref["ys"].tobytes()
    _check_tiles(b, n, ref, D)


def _check_tiles(b, n, ref, D):
    tiles = host(b.tiles())
    bs = ref["box_start"]
    covered = np.zeros(b.N, dtype=np.int64)
    n2 = n[2]
    for col, z0, z1, t0 in tiles:
        if z1 < 0:
            z = z0
            assert -(z + 1) == z1
            end = bs[col * n2 + z + 1]
            cnt = min(64, end - t0)
            assert cnt > 0 and t0 >= bs[col * n2 + z]
        else:
            assert 0 <= z0 <= z1 < n2 and z1 - z0 + 1 <= 62
            assert t0 == bs[col * n2 + z0]
            cnt = bs[col * n2 + z1 + 1] - t0
            assert 0 < cnt <= 64
        covered[t0:t0 + cnt] += 1
    assert (covered == 1).all(), "every target in exactly one tile"
    np.testing.assert_array_equal(tiles.reshape(-1, 4), tiles_spec(bs, D, n))
    assert b.nheavy == heavy_count_spec(bs, D, n, HEAVY_LOG)


def test_binning_rejects_bad_points():
    x = np.random.default_rng(5).random((100, 3))
    x[17, 2] = 1.0  # free axis: must be < L
    with pytest.raises(L.DmkError) as e:
        R.tree_bin((1, 1, 1), 2, (4, 4, 4), dev(x))
    assert e.value.code == L.DMK_EDOMAIN
    x[17, 2] = 0.5
    x[3, 0] = np.nan
    with pytest.raises(L.DmkError) as e:
        R.tree_bin((1, 1, 1), 3, (4, 4, 4), dev(x))
    assert e.value.code == L.DMK_EDOMAIN


def test_binning_dense_and_empty():
    # all points in one box, most boxes empty; many dense tiles
    rng = np.random.default_rng(9)
    x = 0.3 + 0.01 * rng.random((3000, 3))
    ref = bin_spec(x, (1, 1, 1), 3, (6, 6, 6))
    b = R.tree_bin((1, 1, 1), 3, (6, 6, 6), dev(x))
    np.testing.assert_array_equal(host(b.perm()), ref["perm"])
    np.testing.assert_array_equal(host(b.box_start()), ref["box_start"])
    assert b.ntiles == (3000 + 63) // 64
    # 46 tiles of 64 targets x 3000 sources, and one of 56 x 3000
    assert b.nheavy == b.ntiles
    _check_tiles(b, (6, 6, 6), ref, 3)


def test_binning_dense_short_last_tile():
    # a box of 65 targets among sparse ones: two dense tiles of 64 and 1
    # targets, whose costs (64 and 1 times the same neighbourhood) fall in
    # different power-of-two cost classes, so the short tile is ranked in a
    # class of its own
    rng = np.random.default_rng(11)
    x = np.concatenate([0.41 + 0.02 * rng.random((65, 3)), rng.random((400, 3))])
    print("binning dense short last tile", flush=True)
    ref = bin_spec(x, (1, 1, 1), 3, (8, 8, 8))
    b = R.tree_bin((1, 1, 1), 3, (8, 8, 8), dev(x))
    np.testing.assert_array_equal(host(b.perm()), ref["perm"])
    np.testing.assert_array_equal(host(b.box_start()), ref["box_start"])
    dense = [t for t in host(b.tiles()) if t[2] < 0]
    assert len(dense) == 2
    _check_tiles(b, (8, 8, 8), ref, 3)


def test_binning_deterministic():
    x = _points(3, 20000, (1, 1, 1), 3, "uniform")
    b1 = R.tree_bin((1, 1, 1), 3, (16, 16, 16), dev(x))
    b2 = R.tree_bin((1, 1, 1), 3, (16, 16, 16), dev(x))
    assert host(b1.perm()).tobytes() == host(b2.perm()).tobytes()
    assert host(b1.tiles()).tobytes() == host(b2.tiles()).tobytes()


def test_binning_long_runs():
    # boxes of 32, 33, a few hundred and 9000 points among sparse boxes, the
    # points in random order: keys, order, box starts and sorted coordinates
    # bit-exact, and bit-identical when binned twice
    rng = np.random.default_rng(13)
    n = (8, 8, 8)
    h = 1.0 / 8
    dense = {(1, 1, 1): 32, (2, 1, 1): 33, (3, 3, 3): 300, (5, 2, 6): 700, (6, 6, 6): 9000}
    u = rng.random((3000, 3))
    bu = np.floor(u / h).astype(int)
    keep = np.ones(len(u), dtype=bool)
    for c in dense:
        keep &= ~(bu == np.asarray(c)).all(axis=1)
    parts = [u[keep]]
    for c, m in dense.items():
        parts.append((np.asarray(c) + 0.05 + 0.9 * rng.random((m, 3))) * h)
    x = np.concatenate(parts)
    x = x[rng.permutation(len(x))]
    print("binning long runs", len(x), flush=True)
    ref = bin_spec(x, (1, 1, 1), 3, n)
    counts = np.diff(ref["box_start"])
    assert sorted(counts[counts >= 32].tolist()) == [32, 33, 300, 700, 9000]
    b1 = R.tree_bin((1, 1, 1), 3, n, dev(x))
    np.testing.assert_array_equal(host(b1.perm()), ref["perm"])
    np.testing.assert_array_equal(host(b1.skey()), ref["skey"])
    np.testing.assert_array_equal(host(b1.box_start()), ref["box_start"])
    assert host(b1.ys()).tobytes() == ref["ys"].tobytes()
    _check_tiles(b1, n, ref, 3)
    b2 = R.tree_bin((1, 1, 1), 3, n, dev(x))
    assert host(b2.perm()).tobytes() == host(b1.perm()).tobytes()
    assert host(b2.ys()).tobytes() == host(b1.ys()).tobytes()


@pytest.mark.parametrize("m", list(range(1, 13)))
def test_gather_sorted_every_width(m):
    # dst[c][j] = src[perm[j]][c] for every record width the ABI takes, on a
    # point count that leaves the last 256-point workgroup partly filled
    N = 3 * 256 + 77
    x = _points(400 + m, N, (1.0, 1.0, 1.0), 3, "uniform")
    b = R.tree_bin((1.0, 1.0, 1.0), 3, (4, 4, 4), dev(x))
    src = np.random.default_rng(500 + m).standard_normal((N, m))
    print("gather_sorted m", m, flush=True)
    got = host(R.gather_sorted(b, dev(src)))
    perm = host(b.perm())
    assert got.tobytes() == np.ascontiguousarray(src[perm].T).tobytes()
