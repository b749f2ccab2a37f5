"""Pins of the FP64 surrogate reference (CPU): the convolution against a plain
loop, the analytic gradient against central finite differences."""
import numpy as np
import pytest

from oracle import surrogate as S


def test_layout_has_310465_parameters():
    assert S.NUM_PARAMS == 310465


def test_conv_matches_plain_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 8, 8, 3))
    W = rng.normal(size=(4, 9, 3))
    b = rng.normal(size=4)
    got = S.conv_fwd(x, W, b)
    ref = np.zeros((2, 4, 4, 4))
    for n in range(2):
        for oy in range(4):
            for ox in range(4):
                for co in range(4):
                    s = b[co]
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = 2 * oy + ky - 1, 2 * ox + kx - 1
                            if 0 <= iy < 8 and 0 <= ix < 8:
                                s += np.dot(W[co, 3 * ky + kx], x[n, iy, ix])
                    ref[n, oy, ox, co] = s
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_patch_reads_cells_around_the_pose_and_half_outside():
    """A pose on a cell corner: every pixel is one cell, (floor(x) - 64 + ix,
    floor(y) - 64 + iy), and 0.5 off the map."""
    grid = np.arange(300 * 200, dtype=np.float32).reshape(200, 300) / 1e5
    p = S.patches(grid, [[10.0, 150.0, 1.0, 0.0]])[0, ..., 0]
    assert p[0, 0] == 0.5                                  # x = -54: outside
    assert p[0, 54] == grid[86, 0]
    assert p[63, 127] == grid[149, 73]
    assert np.all(p[114:, 60] == 0.5)                      # y >= 200: outside


def test_patch_is_bilinear_resampling_at_the_pose():
    """Against scipy's linear interpolation of the map padded with 0.5 (block k
    centred at index k), at the pixel centres u - 64 + ix, v - 64 + iy; on a
    ragged map with poses near its edges, at strides 1 and 4."""
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(5)
    grid = rng.uniform(0, 1, (150, 203))
    poses = [[0.3, 0.9, 1, 0], [202.7, 149.1, 1, 0], [100.25, 60.5, 1, 0], [7.99, 140.01, 1, 0]]
    for stride in (1, 4):
        src = grid if stride == 1 else S.block_means(grid, stride)
        got = S.patches(grid, poses, stride=stride)
        for b, (x, y, _, _) in enumerate(poses):
            u, v = x / stride, y / stride
            iy, ix = np.meshgrid(np.arange(128), np.arange(128), indexing="ij")
            ref = map_coordinates(src, [v - 64 + iy, u - 64 + ix], order=1,
                                  mode="grid-constant", cval=0.5)
            assert np.allclose(got[b, ..., 0], ref, rtol=0, atol=1e-12), (stride, b)


def test_patch_moves_continuously_with_the_pose():
    """Half a cell to the right, a pixel is the mean of its two cells; a pose
    an epsilon short of the next cell is an epsilon from that cell's patch."""
    rng = np.random.default_rng(6)
    grid = rng.uniform(0, 1, (300, 300))
    a = S.patches(grid, [[150.0, 150.0, 1, 0]])[0, ..., 0]
    h = S.patches(grid, [[150.5, 150.0, 1, 0]])[0, ..., 0]
    assert np.allclose(h[:, :-1], 0.5 * (a[:, :-1] + a[:, 1:]), atol=1e-15)
    e = S.patches(grid, [[151.0 - 1e-9, 150.0, 1, 0]])[0, ..., 0]
    n = S.patches(grid, [[151.0, 150.0, 1, 0]])[0, ..., 0]
    assert np.max(np.abs(e - n)) < 1e-8


def test_block_means_match_plain_loops_on_a_ragged_map():
    rng = np.random.default_rng(3)
    grid = rng.uniform(0, 1, (10, 13))
    got = S.block_means(grid, 4)
    assert got.shape == (3, 4)
    for v in range(3):
        for u in range(4):
            cells = [grid[y, x] for y in range(4 * v, min(4 * v + 4, 10))
                     for x in range(4 * u, min(4 * u + 4, 13))]
            assert np.isclose(got[v, u], sum(cells) / len(cells), rtol=1e-15)


def test_strided_patch_is_centred_on_the_block_of_the_pose():
    grid = np.arange(42 * 38, dtype=np.float64).reshape(38, 42) / 1e3
    bm = S.block_means(grid, 4)                                 # 10 x 11 blocks
    assert bm.shape == (10, 11)
    assert np.isclose(bm[9, 10], grid[36:38, 40:42].mean())     # cut by both edges
    # a pose on a block corner: pose cell (4, 12) -> block (1, 3) at pixel (64, 64)
    p = S.patches(grid, [[4.0, 12.0, 1.0, 0.0]], stride=4)[0, ..., 0]
    assert p[64, 64] == bm[3, 1]
    assert p[64, 62] == 0.5                                     # block x = -1: outside
    assert p[70, 73] == bm[9, 10]                               # the last block
    assert p[71, 64] == 0.5 and p[64, 74] == 0.5                # past the last block
    assert np.array_equal(S.patches(grid, [[3.5, 13.2, 1, 0]], stride=1),
                          S.patches(grid, [[3.5, 13.2, 1, 0]]))


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    flat = np.zeros(S.NUM_PARAMS)
    for name, o, shape in S.layout():
        fan = {1: 1, 2: 9, 3: 9}.get(len(shape), 1)
        if name.startswith("W"):
            fan = 9 * shape[2]
        elif name == "F1":
            fan = shape[1]
        elif name == "F2":
            fan = shape[0]
        k = int(np.prod(shape))
        flat[o:o + k] = rng.uniform(-1, 1, k) * np.sqrt(6.0 / fan) * (0.2 if name.startswith(("b", "c")) else 1.0)
    x = rng.uniform(0, 1, (2, 128, 128, 1))
    labels = rng.normal(size=2)
    L, grad = S.loss_and_grads(flat, x, labels, stats=(0.1, 2.0, 0.7, 1.3))
    # probe a few parameters of every tensor
    h = 1e-6
    for name, o, shape in S.layout():
        k = int(np.prod(shape))
        for idx in rng.choice(k, size=min(3, k), replace=False):
            e = np.zeros_like(flat)
            e[o + idx] = h
            lp, _ = S.loss_and_grads(flat + e, x, labels, (0.1, 2.0, 0.7, 1.3))
            lm, _ = S.loss_and_grads(flat - e, x, labels, (0.1, 2.0, 0.7, 1.3))
            fd = (lp - lm) / (2 * h)
            g = grad[o + idx]
            assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-3) + 1e-9, (name, idx, g, fd)


def test_target_and_prediction_are_inverse_and_monotone():
    rng = np.random.default_rng(8)
    lab = rng.normal(5.0, 0.7, 1000)
    st = S.label_stats(lab)
    assert np.isclose(st[0], lab.mean()) and np.isclose(st[1], lab.std())
    e = np.exp((lab - lab.mean()) / lab.std())
    assert np.isclose(st[2], e.mean()) and np.isclose(st[3], e.std())
    t = S.target(lab, st)
    assert np.isclose(t.mean(), 0.0, atol=1e-12) and np.isclose(t.std(), 1.0)
    assert np.all(np.diff(t[np.argsort(lab)]) >= 0)              # monotone
    assert np.allclose(S.prediction_nats(t, st), lab, rtol=1e-12)
    # below the exponential's range the prediction is clamped, not NaN
    assert np.isfinite(S.prediction_nats(np.array([-1e3]), st)).all()
