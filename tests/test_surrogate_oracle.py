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
    grid = np.arange(300 * 200, dtype=np.float32).reshape(200, 300) / 1e5
    p = S.patches(grid, [[10.7, 150.2, 1.0, 0.0]])[0, ..., 0]
    # pixel (iy, ix) = cell (10 - 64 + ix, 150 - 64 + iy)
    assert p[0, 0] == 0.5                                  # x = -54: outside
    assert np.isclose(p[0, 54], grid[86, 0])
    assert np.isclose(p[63, 127], grid[149, 73])
    assert np.all(p[114:, 60] == 0.5)                      # y >= 200: outside


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
    p = S.patches(grid, [[3.5, 13.2, 1.0, 0.0]], stride=4)[0, ..., 0]
    # pose cell (3, 13) -> block (0, 3): pixel (64, 64) holds block (0, 3)
    assert np.isclose(p[64, 64], bm[3, 0])
    assert p[64, 63] == 0.5                                     # block x = -1: outside
    assert np.isclose(p[70, 74], bm[9, 10])                     # the last block
    assert p[71, 64] == 0.5 and p[64, 75] == 0.5                # past the last block
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
    L, grad = S.loss_and_grads(flat, x, labels, mean=0.1, scale=2.0)
    # probe a few parameters of every tensor
    h = 1e-6
    for name, o, shape in S.layout():
        k = int(np.prod(shape))
        for idx in rng.choice(k, size=min(3, k), replace=False):
            e = np.zeros_like(flat)
            e[o + idx] = h
            lp, _ = S.loss_and_grads(flat + e, x, labels, 0.1, 2.0)
            lm, _ = S.loss_and_grads(flat - e, x, labels, 0.1, 2.0)
            fd = (lp - lm) / (2 * h)
            g = grad[o + idx]
            assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-3) + 1e-9, (name, idx, g, fd)
