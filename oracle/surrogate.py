"""FP64 reference of the learned surrogate -- TEST INFRASTRUCTURE ONLY.

Only the tests and the benchmark's baseline leg use this module.  It shares no
code with the HIP kernels.  The network (not from the paper; it ranks candidate
poses before exact FSMI re-scores the best ones):

  patch 128 x 128 of o around the pose (cells, or s x s block means, 0.5
  outside the map), bilinearly resampled at the pose's continuous position
  -> 5 x [3x3 conv, stride 2, zero padding 1, ReLU], channels 1-32-64-64-128-128
  -> global average pool -> FC 128->256 -> ReLU -> FC 256->1.

Parameters are one flat FP64 vector in the order
W1 b1 W2 b2 ... W5 b5 F1 c1 F2 c2, conv weights [co][tap = 3 ky + kx][ci],
F1 [256][128].  Loss: mean over the batch of (y - target(label))^2 with
target = (exp((label - mean)/scale) - emean)/escale (label_stats); a
prediction y reads mean + scale ln(y escale + emean) nats.

`q` (identity unless given) is applied to every tensor a reduced-precision
implementation stores between steps: the input patch, the conv weights, each
post-ReLU activation and each masked input-gradient.  Passing a rounding
function lets a test hold such an implementation to the same ReLU masks; the
arithmetic between the stored tensors stays FP64.
"""
import numpy as np

LAYERS = [(1, 32, 128), (32, 64, 64), (64, 64, 32), (64, 128, 16), (128, 128, 8)]
FEAT, HID, PATCH = 128, 256, 128


def layout():
    """[(name, offset, shape)] of the flat parameter vector."""
    out, o = [], 0
    for l, (ci, co, _) in enumerate(LAYERS):
        out.append((f"W{l + 1}", o, (co, 9, ci)))
        o += co * 9 * ci
        out.append((f"b{l + 1}", o, (co,)))
        o += co
    for name, shape in (("F1", (HID, FEAT)), ("c1", (HID,)), ("F2", (HID,)), ("c2", (1,))):
        out.append((name, o, shape))
        o += int(np.prod(shape))
    return out


NUM_PARAMS = sum(int(np.prod(s)) for _, _, s in layout())


def unpack(flat):
    flat = np.asarray(flat, np.float64)
    return {n: flat[o:o + int(np.prod(s))].reshape(s) for n, o, s in layout()}


def pack(d):
    return np.concatenate([np.asarray(d[n], np.float64).reshape(-1) for n, _, _ in layout()])


def block_means(grid, s):
    """Map of s x s block means: block (v, u) averages the cells
    x in [s u, s u + s), y in [s v, s v + s) that lie inside the map."""
    grid = np.asarray(grid, np.float64)
    Y, X = grid.shape
    Yc, Xc = -(-Y // s), -(-X // s)
    pad = np.full((Yc * s, Xc * s), np.nan)
    pad[:Y, :X] = grid
    return np.nanmean(pad.reshape(Yc, s, Xc, s), axis=(1, 3))


def patches(grid, poses, stride=1):
    """[B][128][128][1] patches, resampled at the pose's continuous position.
    With cell stride s the map is taken as its s x s block means (s = 1: the
    cells themselves), block k centred at k + 1/2 in block units, 0.5 outside
    the map.  With (u, v) = (x / s, y / s) the pose in block units, pixel
    (iy, ix) is the bilinear interpolation of the blocks at
    (u - 64 + ix + 1/2, v - 64 + iy + 1/2): blocks bx - 64 + ix + {0, 1},
    by - 64 + iy + {0, 1}, (bx, by) = (floor(floor(x) / s), floor(floor(y) / s))
    the block holding the pose's cell, weighted by fx = u - bx, fy = v - by."""
    src = np.asarray(grid, np.float64) if stride == 1 else block_means(grid, stride)
    Y, X = src.shape
    out = np.empty((len(poses), PATCH, PATCH, 1))
    for b, p in enumerate(poses):
        bx = int(np.floor(p[0])) // stride
        by = int(np.floor(p[1])) // stride
        fx = p[0] / stride - bx
        fy = p[1] / stride - by
        ys = np.arange(by - PATCH // 2, by - PATCH // 2 + PATCH + 1)
        xs = np.arange(bx - PATCH // 2, bx - PATCH // 2 + PATCH + 1)
        vy = (ys >= 0) & (ys < Y)
        vx = (xs >= 0) & (xs < X)
        win = np.full((PATCH + 1, PATCH + 1), 0.5)      # blocks, one more row and column
        win[np.ix_(vy, vx)] = src[np.ix_(ys[vy], xs[vx])]
        top = (1.0 - fx) * win[:-1, :-1] + fx * win[:-1, 1:]
        bot = (1.0 - fx) * win[1:, :-1] + fx * win[1:, 1:]
        out[b, ..., 0] = (1.0 - fy) * top + fy * bot
    return out


def conv_fwd(x, W, b):
    """x [B][H][H][ci], W [co][9][ci] -> pre-activation [B][H/2][H/2][co]
    (3x3 taps, stride 2, zero padding 1)."""
    B, H, _, ci = x.shape
    Ho = H // 2
    xp = np.zeros((B, H + 2, H + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((B, Ho, Ho, W.shape[0])) + b
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        xs = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Ho:2, :]
        out += np.einsum("bhwc,oc->bhwo", xs, W[:, tap, :])
    return out


def conv_bwd(x, W, dpre):
    """Gradients of conv_fwd: (dx, dW, db)."""
    B, H, _, ci = x.shape
    Ho = H // 2
    xp = np.zeros((B, H + 2, H + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for tap in range(9):
        ky, kx = divmod(tap, 3)
        xs = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Ho:2, :]
        dW[:, tap, :] = np.einsum("bhwo,bhwc->oc", dpre, xs)
        dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Ho:2, :] += np.einsum("bhwo,oc->bhwc", dpre, W[:, tap, :])
    return dxp[:, 1:-1, 1:-1], dW, dpre.sum(axis=(0, 1, 2))


def _ident(a):
    return a


def forward(flat, x, q=_ident):
    """x: patches [B][128][128][1].  Returns (y [B], cache)."""
    P = unpack(flat)
    acts = [q(x)]
    for l in range(5):
        pre = conv_fwd(acts[-1], q(P[f"W{l + 1}"]), P[f"b{l + 1}"])
        acts.append(q(np.maximum(pre, 0.0)))
    g = acts[-1].mean(axis=(1, 2))                       # [B][128]
    h = np.maximum(g @ P["F1"].T + P["c1"], 0.0)         # [B][256]
    y = h @ P["F2"] + P["c2"][0]
    return y, (acts, g, h)


def label_stats(labels):
    """(mean, scale, emean, escale): the labels' mean and standard deviation,
    then those of e = exp((label - mean) / scale)."""
    lab = np.asarray(labels, np.float64)
    mean = lab.mean()
    scale = lab.std() or 1.0
    e = np.exp((lab - mean) / scale)
    return mean, scale, e.mean(), (e.std() or 1.0)


def target(labels, stats=(0.0, 1.0, 0.0, 1.0)):
    """Regression target of labels (nats): exp of the standardised label,
    standardised again."""
    mean, scale, emean, escale = stats
    return (np.exp((np.asarray(labels, np.float64) - mean) / scale) - emean) / escale


def prediction_nats(y, stats=(0.0, 1.0, 0.0, 1.0)):
    """The target's inverse: mean + scale ln(y escale + emean), the logarithm's
    argument clamped to 1e-6 from below."""
    mean, scale, emean, escale = stats
    e = np.asarray(y, np.float64) * escale + emean
    return mean + scale * np.log(np.maximum(e, 1e-6))


def loss_and_grads(flat, x, labels, stats=(0.0, 1.0, 0.0, 1.0), q=_ident):
    """Batch-mean squared error against the labels' targets and its gradient."""
    P = unpack(flat)
    y, (acts, g, h) = forward(flat, x, q)
    t = target(labels, stats)
    n = len(y)
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n
    G = {}
    G["F2"] = h.T @ dy
    G["c2"] = np.array([dy.sum()])
    dh = np.outer(dy, P["F2"]) * (h > 0)
    G["F1"] = dh.T @ g
    G["c1"] = dh.sum(0)
    dg = dh @ P["F1"]                                    # [B][128]
    a5 = acts[5]
    d = np.repeat(np.repeat(dg[:, None, None, :], a5.shape[1], 1), a5.shape[2], 2) / (a5.shape[1] * a5.shape[2])
    d = q(d * (a5 > 0))
    for l in range(4, -1, -1):
        dx, dW, db = conv_bwd(acts[l], q(P[f"W{l + 1}"]), d)
        G[f"W{l + 1}"], G[f"b{l + 1}"] = dW, db
        if l > 0:
            d = q(dx * (acts[l] > 0))
    return L, pack(G)
