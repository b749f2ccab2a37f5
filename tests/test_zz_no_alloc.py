"""fsmi_eval_poses_noalloc (the entry point for callers that cannot allocate)
against fsmi_eval_poses, through the C-ABI: the same kernels, so per-pose and
per-beam results must be bit-identical; two calls in a row, the second smaller,
so a call after a larger one sees none of its leftovers in the shared static
scratch; the size limit of that scratch, at and one past the maximum."""
import numpy as np
import pytest
import torch

from paper_1905_02238_amd import fsmi as F
from paper_1905_02238_amd import workloads as W

pytestmark = pytest.mark.gpu

MAX_ITEMS = 1 << 21


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] noalloc: creating libfsmi context on cuda:0", flush=True)
    return F.context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def rooms():
    occ, lab = W.room_grid(512, W.SEED_BASE + 61, split_extent=80, unknown_frac=0.3)
    return occ, lab


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX, F.FSMI_UNIFORM])
def test_noalloc_2d_matches_eval_poses_twice(ctx, rooms, variant):
    occ, lab = rooms
    g = dev(occ)
    prm = F.params(variant=variant, trunc_delta=9, uniform_h=6)
    for n_poses, n_beams, seed in ((600, 360, 1), (37, 90, 2)):   # the second call is smaller
        print(f"[gpu] noalloc 2D variant={variant} {n_poses}x{n_beams}", flush=True)
        p = dev(W.poses_in_free_space_2d(lab, n_poses, seed, yaw="uniform"))
        bd = dev(W.beam_dirs_2d(n_beams))
        ref_p, ref_b = ctx.fsmi_eval_poses(prm, g, p, bd, 3.0, 200.0, want_beams=True)
        got_p, _ = ctx.fsmi_eval_poses_noalloc(prm, g, p, bd, 3.0, 200.0)
        got_p2, got_b2 = ctx.fsmi_eval_poses_noalloc(prm, g, p, bd, 3.0, 200.0, want_beams=True)
        torch.cuda.synchronize()
        ctx.fsmi_sync()
        r = ref_p.cpu().numpy()
        assert np.all(np.isfinite(r)) and np.all(r > 0.0)
        assert np.array_equal(got_p.cpu().numpy(), r)
        assert np.array_equal(got_p2.cpu().numpy(), r)
        assert np.array_equal(got_b2.cpu().numpy(), ref_b.cpu().numpy())


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX])
def test_noalloc_3d_matches_eval_poses_twice(ctx, variant):
    vox, lab = W.voxel_map(96, 96, 48, seed=21, n_boxes=20, n_pillars=10, block=16, unknown_frac=0.1)
    g = dev(vox)
    prm = F.params(variant=variant, trunc_delta=6)
    for n_poses, rows, cols, seed in ((24, 32, 64, 1), (5, 8, 16, 2)):
        print(f"[gpu] noalloc 3D variant={variant} {n_poses}x{rows * cols}", flush=True)
        p = dev(W.poses_in_free_space_3d(lab, n_poses, seed))
        bd = dev(W.beam_dirs_3d(rows, cols))
        ref_p, ref_b = ctx.fsmi_eval_poses(prm, g, p, bd, 2.0, 90.0, 1.0, want_beams=True)
        got_p, _ = ctx.fsmi_eval_poses_noalloc(prm, g, p, bd, 2.0, 90.0, 1.0)
        torch.cuda.synchronize()
        ctx.fsmi_sync()
        r = ref_p.cpu().numpy()
        assert np.all(np.isfinite(r))
        assert np.array_equal(got_p.cpu().numpy(), r)


def test_noalloc_at_and_past_its_scratch_limit(ctx, rooms):
    occ, lab = rooms
    g = dev(occ)
    prm = F.params(variant=F.FSMI_UNIFORM, uniform_h=6)
    n_beams = 360
    n_poses = MAX_ITEMS // n_beams                      # 5825 x 360 <= 2^21
    print(f"[gpu] noalloc at the limit: {n_poses}x{n_beams}", flush=True)
    p = dev(W.poses_in_free_space_2d(lab, n_poses, 3, yaw="uniform"))
    bd = dev(W.beam_dirs_2d(n_beams))
    ref_p, _ = ctx.fsmi_eval_poses(prm, g, p, bd, 3.0, 200.0)
    got_p, _ = ctx.fsmi_eval_poses_noalloc(prm, g, p, bd, 3.0, 200.0)
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    assert np.array_equal(got_p.cpu().numpy(), ref_p.cpu().numpy())
    # one item past the limit: refused before any launch (host check) ...
    bd1 = dev(W.beam_dirs_2d(MAX_ITEMS // (n_poses + 1) + 1))
    p1 = dev(W.poses_in_free_space_2d(lab, n_poses + 1, 4))
    assert (n_poses + 1) * bd1.shape[0] > MAX_ITEMS
    with pytest.raises(F.FsmiError) as ei:
        ctx.fsmi_eval_poses_noalloc(prm, g, p1, bd1, 3.0, 200.0)
    assert ei.value.status == F.FSMI_E_CAPACITY
    # ... and accepted with caller-provided per-beam outputs
    got_p1, got_b1 = ctx.fsmi_eval_poses_noalloc(prm, g, p1, bd1, 3.0, 200.0, want_beams=True)
    ref_p1, ref_b1 = ctx.fsmi_eval_poses(prm, g, p1, bd1, 3.0, 200.0, want_beams=True)
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    assert np.array_equal(got_p1.cpu().numpy(), ref_p1.cpu().numpy())
    assert np.array_equal(got_b1.cpu().numpy(), ref_b1.cpu().numpy())
