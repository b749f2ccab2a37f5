"""The CSQMI comparator (Sec. 2.3; Approx-CSQMI truncated at Delta) on the GPU
against the FP64 oracle: explicit-boundary and unit-cell beam batches (wave-
and tile-per-beam), the fused 2D pose path, planned launches, and the paths
that reject it.

Bar: the value is a difference of three logarithms, log sum u + log C'' -
2 log A'', so the rounding of the sums shows up as an absolute error of I, not
one relative to I (a beam resolved in its first cells has a small I).  Each
sum's relative error is bounded by its terms' count times the unit roundoff
of its accumulation: in FP32 mode chains of at most eight FP32 products
(8 x 6e-8 = 5e-7) added in FP64, in FP64 mode plain FP64 sums of up to a few
thousand terms (about 4e-13 at n = 4000), four such errors in all.  Bars:
FP32 |d| <= 1e-5 |I| + 2e-6; FP64 |d| <= 1e-12 |I| + 2e-12.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1905_02238_amd import fsmi as F
from paper_1905_02238_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] csqmi: creating libfsmi context on cuda:0", flush=True)
    return F.context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(got, ref, prec):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(ref))
    d = np.abs(got - ref)
    if prec == F.FSMI_FP64:
        bad = d > 1e-12 * np.abs(ref) + 2e-12
    else:
        bad = d > 1e-5 * np.abs(ref) + 2e-6
    rel = d / np.maximum(np.abs(ref), 1e-300)
    print(f"[gpu]   max abs {d.max():.2e}, max rel {rel.max():.2e} over {len(ref)}", flush=True)
    assert not np.any(bad), (int(np.argmax(d)), float(d.max()))


LENS = [0, 1, 2, 3, 5, 63, 64, 65, 127, 200, 255, 256, 257, 511, 512, 513, 700, 33, 7, 1100]


def _batch(seed, widths):
    rng = np.random.default_rng(seed)
    lens = np.asarray(LENS, np.int64)
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    occ = rng.uniform(0.0, 1.0, int(off[-1])).astype(np.float32)
    k = rng.integers(0, int(off[-1]), int(off[-1]) // 20)
    occ[k] = rng.choice(np.array([0.0, 1.0, 0.5], np.float32), len(k))
    sigma = rng.uniform(0.3, 5.0, len(lens)).astype(np.float32)
    bound = None
    if widths:
        bound = np.zeros(int(off[-1]) + len(lens))
        for b in range(len(lens)):
            n = int(lens[b])
            bound[off[b] + b: off[b] + b + n + 1] = np.concatenate(
                [[0.0], np.cumsum(rng.uniform(0.01, 1.5, n))])
    return off, occ, bound, sigma


@pytest.mark.parametrize("Delta", [0, 3, 9, 5000])
@pytest.mark.parametrize("widths", [True, False])
@pytest.mark.parametrize("prec", [F.FSMI_FP32, F.FSMI_FP64])
def test_csqmi_eval_beams_parity(ctx, Delta, widths, prec):
    print(f"[gpu] csqmi eval_beams Delta={Delta} widths={widths} prec={prec}", flush=True)
    off, occ, bound, sigma = _batch(70 + Delta, widths)
    prm = F.params(variant=F.FSMI_CSQMI, trunc_delta=Delta, precision=prec)
    mi = ctx.fsmi_eval_beams(prm, dev(off), dev(occ), dev(sigma), None if bound is None else dev(bound))
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    ref = O.eval_beams(O.CSQMI, off, occ, sigma, bound=bound, Delta=Delta)
    got = mi.cpu().numpy()
    assert got[0] == 0.0 and ref[0] == 0.0
    check(got[1:], ref[1:], prec)


def test_csqmi_paper_beam_batch_and_plan(ctx):
    """The paper's single-beam setting (Sec. 5.1: 100 cells of 0.1 m, o ~ U(0, 1),
    sigma = 0.05 m = 0.5 cells, Delta = 3) as a batch of 20 000 unit-cell beams,
    eagerly and through a graph-captured plan."""
    print("[gpu] csqmi paper-shaped batch", flush=True)
    rng = np.random.default_rng(5)
    nb, n = 20000, 100
    off = np.arange(nb + 1, dtype=np.int64) * n
    occ = rng.uniform(0.0, 1.0, nb * n).astype(np.float32)
    sigma = np.full(nb, 0.5, np.float32)
    prm = F.params(variant=F.FSMI_CSQMI, trunc_delta=3)
    d_off, d_occ, d_sig = dev(off), dev(occ), dev(sigma)
    eager = ctx.fsmi_eval_beams(prm, d_off, d_occ, d_sig)
    plan = F.Plan(ctx, prm, d_off, d_occ, d_sig, graph=True)
    planned = plan.launch().clone()
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    plan.close()
    e = eager.cpu().numpy()
    assert np.array_equal(planned.cpu().numpy(), e)
    sel = np.arange(0, nb, 50)
    ref = O.eval_beams(O.CSQMI, off[: sel[-1] + 2], occ, sigma[: sel[-1] + 1], Delta=3)
    check(e[sel], ref[sel], F.FSMI_FP32)


@pytest.mark.parametrize("prec", [F.FSMI_FP32, F.FSMI_FP64])
@pytest.mark.parametrize("Delta", [3, 9])
def test_csqmi_poses_2d_parity(ctx, prec, Delta):
    """The fused 2D path on the 2048 x 2048 rooms (turned poses, R = 400,
    sigma = 3 cells): four poses beam by beam and pose by pose."""
    print(f"[gpu] csqmi poses 2D prec={prec} Delta={Delta}", flush=True)
    wl = W.grid_large(n_poses=4)
    prm = F.params(variant=F.FSMI_CSQMI, trunc_delta=Delta, precision=prec)
    mp, mb = ctx.fsmi_eval_poses(prm, dev(wl["grid"]), dev(wl["poses"]), dev(wl["beam_dir"]),
                                 wl["sigma"], wl["R"], want_beams=True)
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    rp, rb = O.eval_poses_2d(O.CSQMI, wl["grid"], wl["poses"], wl["beam_dir"], wl["sigma"],
                             wl["R"], Delta=Delta)
    check(mb.cpu().numpy().ravel(), rb.ravel(), prec)
    mp = mp.cpu().numpy()
    assert np.allclose(mp, mb.cpu().numpy().sum(1), rtol=1e-12, atol=0)
    check(mp, rp, prec)


def test_csqmi_rejected_on_runs_and_voxels(ctx):
    prm = F.params(variant=F.FSMI_CSQMI, trunc_delta=3)
    off, ro, rl, sp = W.rle_beams(4, 1, 1, 4, 1, 5)
    with pytest.raises(F.FsmiError) as e:
        ctx.fsmi_rle_eval_beams(prm, dev(off), dev(ro), dev(rl), dev(sp))
    assert e.value.status == F.FSMI_E_INVAL
    vox = np.full((8, 16, 16), 0.3, np.float32)
    poses = np.array([[8.5, 8.5, 4.5, 1.0, 0.0]])
    with pytest.raises(F.FsmiError):
        ctx.fsmi_eval_poses(prm, dev(vox), dev(poses), dev(W.beam_dirs_3d(2, 4)), 2.0, 10.0, 1.0)
    with pytest.raises(F.FsmiError):
        ctx.fsmi_eval_poses(F.params(variant=F.FSMI_CSQMI, trunc_delta=-1), dev(np.full((8, 8), 0.3, np.float32)),
                            dev(np.array([[4.5, 4.5, 1.0, 0.0]])), dev(W.beam_dirs_2d(4)), 1.0, 5.0)
    with pytest.raises(F.FsmiError):
        ctx.fsmi_eval_poses(F.params(variant=F.FSMI_CSQMI, flags=F.FSMI_F_SKIP_ZERO),
                            dev(np.full((8, 8), 0.3, np.float32)),
                            dev(np.array([[4.5, 4.5, 1.0, 0.0]])), dev(W.beam_dirs_2d(4)), 1.0, 5.0)
