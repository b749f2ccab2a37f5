"""The learned surrogate on the GPU: matrix-core layout, forward and gradients
against the FP64 reference, deterministic training, checkpoints, and what the
network gains in the exact-rescore ranking path."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import surrogate as S
from paper_1905_02238_amd import fsmi as F
from paper_1905_02238_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] surrogate tests: context on cuda:0", flush=True)
    return F.context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_mfma_operand_layout(ctx):
    rng = np.random.default_rng(0)
    A = torch.from_numpy(rng.normal(size=(16, 32)).astype(np.float32)).to(torch.bfloat16).cuda()
    B = torch.from_numpy(rng.normal(size=(32, 16)).astype(np.float32)).to(torch.bfloat16).cuda()
    D = ctx.fsmi_probe_mfma(A.contiguous(), B.contiguous())
    torch.cuda.synchronize()
    ref = A.double().cpu() @ B.double().cpu()
    assert torch.allclose(D.double().cpu(), ref, rtol=1e-5, atol=1e-5)


def _poses_near_and_inside(lab, n, seed):
    ps = W.poses_in_free_space_2d(lab, n, seed)
    ps[0, :2] = [3.5, 3.5]                     # the patch hangs over the map edge
    return ps


def _bf16(a):
    """Round to BF16 (nearest even) and back to FP64."""
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).double().numpy()


def _per_tensor(g_gpu, g_ref):
    out = {}
    for name, o, shape in S.layout():
        k = int(np.prod(shape))
        a, b = g_gpu[o:o + k], g_ref[o:o + k]
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        rel = float(np.max(np.abs(a - b)) / (np.max(np.abs(b)) + 1e-300))
        out[name] = (cos, rel)
    return out


# Batch 67 (odd) leaves a ragged last stage in the weight-gradient kernels of
# the last layer (67 x 16 output pixels) and spreads the first two layers'
# weight-gradient partials over more than one run of the fixed-order sum.
# Stride 1 puts most patch windows inside the 200 x 200 map (the gathers'
# in-map path) and stride 4 most outside it (the bounds-checked path); stride
# 2, the benchmark's, mixes the two within a patch.
@pytest.mark.parametrize("stride,batch", [(1, 32), (2, 32), (4, 32), (1, 67)])
def test_forward_and_gradients_match_fp64_reference(ctx, stride, batch):
    wl = W.grid_small()
    grid, lab = wl["grid"], wl["labels"]
    poses = _poses_near_and_inside(lab, batch, 5)
    net = F.Surrogate(ctx, seed=7, max_batch=batch, patch_stride=stride)
    # the output bias lifted so every output is positive: with the label
    # statistics at (0, 1) a prediction is ln y nats, so exp gives y back
    c2 = [o for name, o, _ in S.layout() if name == "c2"][0]
    flat = net.params().double().cpu().numpy()
    flat[c2] = 3.0
    net.set_params(torch.from_numpy(flat.astype(np.float32)).cuda())
    x = S.patches(grid, poses, stride=stride)
    y_ref, _ = S.forward(flat, x)
    y_bf, _ = S.forward(flat, x, q=_bf16)
    assert np.min(y_ref) > 0.1
    pred = net.forward(dev(grid), dev(poses))
    torch.cuda.synchronize()
    y = np.exp(pred.double().cpu().numpy())
    # FP32 vs FP64 summation order can move a stored BF16 value by one ulp
    # (2^-8 relative) wherever it sits near a rounding boundary.  How far that
    # moves the output depends on the inputs, so the bar is the reference's
    # own spread: the same BF16 reference with every stored tensor perturbed
    # by up to 1e-7 relative (FP32 rounding) before it is rounded.
    spread = 0.0
    for sd in (1, 2):
        rr = np.random.default_rng(sd)
        y_p, _ = S.forward(flat, x, q=lambda a: _bf16(np.asarray(a) * (1 + rr.uniform(-1e-7, 1e-7, np.shape(a)))))
        spread = max(spread, float(np.max(np.abs(y_p - y_bf))))
    assert np.max(np.abs(y - y_bf)) <= 2.0 * spread + 1e-4 * np.max(np.abs(y_bf)) + 1e-6
    assert np.max(np.abs(y - y_ref)) <= 2e-2 * np.max(np.abs(y_ref)) + 1e-6
    labels = np.random.default_rng(1).normal(size=batch)
    loss = net.backward(dev(grid), dev(poses), dev(labels))
    g = net.grads().double().cpu().numpy()
    torch.cuda.synchronize()
    # Held to the reference that rounds to BF16 where the kernels store BF16
    # (patch, weights, activations, masked input-gradients), so both take the
    # same ReLU masks: what is left is FP32-vs-FP64 summation order.
    L_bf, g_bf = S.loss_and_grads(flat, x, labels, q=_bf16)
    assert abs(float(loss[0]) - L_bf) <= 1e-4 * abs(L_bf)
    for name, (cos, rel) in _per_tensor(g, g_bf).items():
        assert cos >= 0.99999 and rel <= 5e-3, (name, cos, rel)
    # Against plain FP64 the BF16 storage flips a few ReLU masks near zero,
    # which moves single entries by up to tens of percent; directions agree.
    L_ref, g_ref = S.loss_and_grads(flat, x, labels)
    assert abs(float(loss[0]) - L_ref) <= 2e-2 * abs(L_ref)
    for name, (cos, rel) in _per_tensor(g, g_ref).items():
        assert cos >= 0.98, (name, cos, rel)


def test_forward_at_block_boundaries(ctx):
    """Poses on and next to the edges of the s x s blocks (s = 3) and of the
    cells: the patch origin (the block holding the pose's cell, an FP64 floor
    division) and the fraction inside it must match the FP64 reference's, so
    a pose a hair below a block edge samples the block before it at fraction
    ~1 and a pose on the edge the next block at fraction 0."""
    wl = W.grid_small()
    grid = wl["grid"]
    xs = [96.0, 96.0 - 1e-9, 95.0, 95.5, 97.0, 98.999999, 99.0, 100.25]
    ys = [60.0, 60.0 - 1e-9, 61.0, 62.5, 63.0, 59.999999, 57.0, 120.75]
    poses = np.array([[x, y, 1.0, 0.0] for x in xs for y in ys[:4]] +
                     [[x, y, 1.0, 0.0] for x in xs[:4] for y in ys[4:]])
    net = F.Surrogate(ctx, seed=11, max_batch=len(poses), patch_stride=3)
    c2 = [o for name, o, _ in S.layout() if name == "c2"][0]
    flat = net.params().double().cpu().numpy()
    flat[c2] = 3.0
    net.set_params(torch.from_numpy(flat.astype(np.float32)).cuda())
    x = S.patches(grid, poses, stride=3)
    y_bf, _ = S.forward(flat, x, q=_bf16)
    pred = net.forward(dev(grid), dev(poses))
    torch.cuda.synchronize()
    y = np.exp(pred.double().cpu().numpy())
    spread = 0.0
    for sd in (1, 2):
        rr = np.random.default_rng(sd)
        y_p, _ = S.forward(flat, x, q=lambda a: _bf16(np.asarray(a) * (1 + rr.uniform(-1e-7, 1e-7, np.shape(a)))))
        spread = max(spread, float(np.max(np.abs(y_p - y_bf))))
    assert np.max(np.abs(y - y_bf)) <= 2.0 * spread + 1e-4 * np.max(np.abs(y_bf)) + 1e-6


def test_gradients_do_not_depend_on_max_batch(ctx):
    """One batch gives bit-identical loss and gradients whether the network was
    sized for exactly that batch or for a larger one.  conv1's weight gradient
    runs in a grid of one resident round of workgroups, and the number of
    partial sums it writes is not monotone in the batch (a batch of n tiles
    can write more than a larger batch would), so the partial buffer sized at
    max_batch must still hold what a smaller batch writes."""
    wl = W.grid_small()
    grid, lab = wl["grid"], wl["labels"]
    poses = _poses_near_and_inside(lab, 64, 9)
    labels = np.random.default_rng(2).normal(size=64)
    out = []
    for mb in (64, 67, 130):
        print(f"[gpu] max_batch {mb}, batch 64", flush=True)
        net = F.Surrogate(ctx, seed=7, max_batch=mb)
        loss = net.backward(dev(grid), dev(poses), dev(labels))
        out.append((float(loss[0]), net.grads().clone()))
        net.close()
    for loss, g in out[1:]:
        assert loss == out[0][0]
        assert torch.equal(g, out[0][1])


def _labelled(ctx, seeds, n_poses, size=1024):
    """Exact per-pose FSMI labels on rooms maps (360 beams, R = 400, sigma = 3)."""
    out = []
    bd = dev(W.beam_dirs_2d(360))
    for s in seeds:
        grid, lab = W.room_grid(size, s, split_extent=160, unknown_frac=0.30)
        poses = W.poses_in_free_space_2d(lab, n_poses, s)
        g, p = dev(grid), dev(poses)
        mi, _ = ctx.fsmi_eval_poses(F.params(), g, p, bd, 3.0, 400.0)
        out.append((g, p, mi))
    return out


def _train(ctx, data, seed, steps, batch=128, lr=1e-3, stride=1, cosine=False):
    net = F.Surrogate(ctx, seed=seed, max_batch=max(batch, 8192) if cosine else batch,
                      patch_stride=stride)
    net.fit_label_stats(torch.cat([d[2] for d in data]))
    losses = []
    rng = np.random.default_rng(seed)
    for it in range(steps):
        g, p, mi = data[it % len(data)]
        sel = torch.from_numpy(rng.choice(p.shape[0], batch, replace=False)).cuda()
        pb, lb = p[sel].contiguous(), mi[sel].contiguous()
        loss = net.backward(g, pb, lb)
        net.adam_step(float(lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))) if cosine else lr)
        losses.append(loss)
    torch.cuda.synchronize()
    return net, [float(l[0]) for l in losses]


def test_training_is_deterministic_and_learns(ctx):
    data = _labelled(ctx, [W.SEED_BASE + 100, W.SEED_BASE + 101], 1024)
    a, la = _train(ctx, data, seed=11, steps=40)
    b, lb = _train(ctx, data, seed=11, steps=40)
    assert la == lb
    assert torch.equal(a.params(), b.params())
    assert np.mean(la[-10:]) < np.mean(la[:10])


def test_checkpoint_resume_is_exact(ctx, tmp_path):
    data = _labelled(ctx, [W.SEED_BASE + 102], 512)
    net, _ = _train(ctx, data, seed=5, steps=6)
    path = tmp_path / "sur.ckpt"
    net.save(path)
    other = F.Surrogate(ctx, seed=99, max_batch=128)
    other.load(path)
    assert torch.equal(net.params(), other.params())
    g, p, mi = data[0]
    for _ in range(3):
        l1 = net.backward(g, p[:128].contiguous(), mi[:128].contiguous())
        net.adam_step(1e-3)
        l2 = other.backward(g, p[:128].contiguous(), mi[:128].contiguous())
        other.adam_step(1e-3)
        assert float(l1[0]) == float(l2[0])
    assert torch.equal(net.params(), other.params())


def test_surrogate_gain_over_random_candidates(ctx):
    """The benchmark's recipe (1M labels: 64 maps x 16 384 poses, patch stride
    2, 16 000 Adam steps of 128 with a cosine learning rate, seed 3) and its
    four held-out maps of 65 536 candidates (the timed map and three more):
    on each, the network ranks the candidates with a clearly positive rank
    correlation and its top prediction loses less MI to the true best pose
    than a random candidate; over the four maps, its top 1 % (the k largest
    predictions, re-scored exactly) loses less than a random 1 % re-scored the
    same way (the ablation, mean of 200 draws per map).  One map's top-1 %
    regret hinges on a single pick: over eight training seeds the surrogate
    beat the random 1 % on 2 to 4 of the four maps, with the mean below the
    random mean for every seed (the benchmark's seed study), so the mean is
    what is asserted.  Training is deterministic, so these are the
    benchmark's own figures for seed 3."""
    print("[gpu] surrogate gain test", flush=True)
    train = _labelled(ctx, [W.SEED_BASE + 100 + i for i in range(64)], 16384, size=2048)
    net, losses = _train(ctx, train, seed=3, steps=16000, batch=128, stride=2, cosine=True)
    del train
    from scipy.stats import spearmanr
    bd = dev(W.beam_dirs_2d(360))
    n = 65536
    k = n // 100 + 1
    wl = W.grid_large(n_poses=n, yaw="zero")
    g0, p0 = dev(wl["grid"]), dev(wl["poses"])
    mi0, _ = ctx.fsmi_eval_poses(F.params(), g0, p0, bd, 3.0, 400.0)
    held = [(g0, p0, mi0)] + _labelled(ctx, [W.SEED_BASE + 200 + i for i in range(3)], n,
                                       size=2048)
    ours, rand = [], []
    for (g, p, mi) in held:
        idx, mi_top, pred = ctx.fsmi_rank_poses(F.params(), net, g, p, bd, 3.0, 400.0, k,
                                                want_pred=True)
        torch.cuda.synchronize()
        true = mi.cpu().numpy()
        idx = idx.cpu().numpy()
        assert len(set(idx.tolist())) == k
        assert np.allclose(mi_top.cpu().numpy(), true[idx], rtol=1e-12)   # exact re-score
        # the top-k really are the k largest predictions
        pr = pred.cpu().numpy()
        assert np.min(pr[idx]) >= np.sort(pr)[-k]
        best = true.max()
        top1 = 1.0 - true[int(np.argmax(pr))] / best
        rand1 = float(np.mean(1.0 - true / best))          # a random single candidate
        ours_k = 1.0 - true[idx].max() / best
        rng = np.random.default_rng(0)
        rand_k = np.mean([1.0 - true[rng.choice(len(true), k, replace=False)].max() / best
                          for _ in range(200)])
        rho = spearmanr(pr, true).correlation
        recall = len(set(np.argsort(-true)[:k].tolist()) & set(idx.tolist())) / k
        print(f"[gpu] top-1 regret {top1:.4f} (random {rand1:.4f}); top-1% regret {ours_k:.4f} "
              f"(random {rand_k:.4f}); recall@1% {recall:.2f} spearman {rho:.3f} "
              f"final loss {np.mean(losses[-100:]):.3f}", flush=True)
        assert rho > 0.4
        assert top1 < rand1
        ours.append(ours_k)
        rand.append(rand_k)
    assert np.mean(ours) < np.mean(rand)
