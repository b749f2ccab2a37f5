"""The run-domain engine of FSMI-RLE (Thm 5) and Approx-FSMI-RLE (Thm 6) on the
GPU (forced with FSMI_F_RLE_RUNS) against the FP64 oracle's expanded route and
its block routes (Thm 5 with block sums by definition, Thm 6 with the cropped
rectangles): beams of 1 to 65 runs (the engine holds 64), run lengths from 2 to
40, both kernels, FP32 (1e-5 relative) and FP64 (1e-12), through
fsmi_rle_eval_beams and the fused 3D pose path; and the default switch and the
forced expanded engine giving the same values."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1905_02238_amd import fsmi as F
from paper_1905_02238_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] rle engine: creating libfsmi context on cuda:0", flush=True)
    return F.context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_err(got, ref):
    """max |got - ref| / max(|ref|, 1e-30): a result below 1e-30 nats (an
    FP32 P(e_j) underflows there) counts by its absolute error; an exact zero
    of the oracle must stay zero."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)))


def switch_beams(seed):
    """Beams of runs around the engine's switch: run counts 1 .. 65, mean run
    lengths from 2 to 40, some exactly 4, occupancies with repeats (adjacent
    runs of equal value) and known cells."""
    rng = np.random.default_rng(seed)
    specs = [(1, 30), (2, 4), (5, 4), (8, 3), (10, 12), (20, 16), (33, 8), (40, 4), (63, 5),
             (64, 4), (64, 9), (65, 6), (64, 3), (12, 40), (3, 2), (50, 6)]
    runs_o, runs_l, off = [], [], [0]
    for nr, mean in specs:
        lens = np.maximum(1, rng.poisson(mean - 1, nr) + 1)
        if mean == 4:
            lens = np.full(nr, 4)                 # exactly at the switch
        o = rng.uniform(0.02, 0.98, nr)
        o[rng.random(nr) < 0.1] = rng.choice([0.0, 1.0, 0.5])
        if nr > 2:
            o[1] = o[0]                           # two adjacent runs of one value
        runs_o.append(o.astype(np.float32))
        runs_l.append(lens.astype(np.int32))
        off.append(off[-1] + nr)
    return (np.array(off, np.int64), np.concatenate(runs_o), np.concatenate(runs_l),
            rng.uniform(0.7, 3.5, len(specs)).astype(np.float32))


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX])
@pytest.mark.parametrize("kernel", [F.FSMI_KERNEL_ERF, F.FSMI_KERNEL_DENSITY])
@pytest.mark.parametrize("prec,tol", [(F.FSMI_FP32, 1e-5), (F.FSMI_FP64, 1e-12)])
def test_rle_engine_parity_around_the_switch(ctx, variant, kernel, prec, tol):
    print(f"[gpu] rle engine variant={variant} kernel={kernel} prec={prec}", flush=True)
    off, ro, rl, sp = switch_beams(31 + variant + 2 * kernel)
    Delta = 5
    prm = F.params(variant=variant, trunc_delta=Delta, kernel=kernel, precision=prec,
                   flags=F.FSMI_F_RLE_RUNS)
    mi = ctx.fsmi_rle_eval_beams(prm, dev(off), dev(ro), dev(rl), dev(sp))
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    got = mi.cpu().numpy()
    exact = variant == F.FSMI_EXACT
    ref = O.rle_eval_beams(exact, off, ro, rl, sp, kind=kernel, Delta=Delta)
    assert rel_err(got, ref) <= tol
    # the block routes of Thm 5 / Thm 6 on the same runs
    for b in range(len(sp)):
        r0, r1 = off[b], off[b + 1]
        if exact:
            blk = O.rle_thm5(ro[r0:r1], rl[r0:r1], np.float32(sp[b]), kind=kernel)
        else:
            blk = O.rle_thm6(ro[r0:r1], rl[r0:r1], np.float32(sp[b]), Delta, kind=kernel)
        assert abs(got[b] - blk) <= max(tol, 1e-13) * max(abs(blk), 1e-30), b


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX])
def test_rle_engine_long_runs_and_sigma(ctx, variant):
    """Long beams of long runs (the reach of the kernel spans several runs) and
    sigma' from 0.3 to 12 virtual cells."""
    print(f"[gpu] rle engine long runs variant={variant}", flush=True)
    off, ro, rl, _ = W.rle_beams(48, seed=8, run_lo=8, run_hi=90, n_runs_lo=1, n_runs_hi=40)
    sp = np.geomspace(0.3, 12.0, 48).astype(np.float32)
    ref = O.rle_eval_beams(variant == F.FSMI_EXACT, off, ro, rl, sp, Delta=9)
    for flags in (F.FSMI_F_RLE_RUNS, F.FSMI_F_RLE_CELLS, 0):
        prm = F.params(variant=variant, trunc_delta=9, flags=flags)
        mi = ctx.fsmi_rle_eval_beams(prm, dev(off), dev(ro), dev(rl), dev(sp))
        torch.cuda.synchronize()
        ctx.fsmi_sync()
        assert rel_err(mi.cpu().numpy(), ref) <= 1e-5, flags


def test_rle_engine_3d_poses_match_the_oracle(ctx):
    """The fused 3D path on a voxel map with block-constant free space (runs of
    4 to 32 cells): exact and Approx beams against the oracle."""
    print("[gpu] rle engine 3D", flush=True)
    vox, lab = W.voxel_map(96, 96, 48, seed=23, n_boxes=14, n_pillars=8, block=16,
                           unknown_frac=0.1)
    poses = W.poses_in_free_space_3d(lab, 4, seed=23)
    bd = W.beam_dirs_3d(16, 32)
    for variant in (F.FSMI_EXACT, F.FSMI_APPROX):
        rp, rb = O.eval_poses_3d(variant == F.FSMI_EXACT, vox, poses, bd, 2.0, 120.0, 1.0, Delta=6)
        for flags in (F.FSMI_F_RLE_RUNS, F.FSMI_F_RLE_CELLS, 0):
            prm = F.params(variant=variant, trunc_delta=6, flags=flags)
            mp, mb = ctx.fsmi_eval_poses(prm, dev(vox), dev(poses), dev(bd), 2.0, 120.0, 1.0,
                                         want_beams=True)
            torch.cuda.synchronize()
            ctx.fsmi_sync()
            assert rel_err(mb.cpu().numpy(), rb) <= 1e-5, flags
            assert rel_err(mp.cpu().numpy(), rp) <= 1e-5, flags


def test_rle_engine_bad_runs_latch(ctx):
    off = np.array([0, 2, 4], np.int64)
    ro = np.array([0.3, 1.5, 0.2, 0.4], np.float32)       # 1.5 is no occupancy
    rl = np.array([8, 9, 10, 12], np.int32)
    sp = np.array([2.0, 2.0], np.float32)
    mi = ctx.fsmi_rle_eval_beams(F.params(flags=F.FSMI_F_RLE_RUNS), dev(off), dev(ro), dev(rl),
                                 dev(sp))
    torch.cuda.synchronize()
    with pytest.raises(F.FsmiError):
        ctx.fsmi_sync()
    got = mi.cpu().numpy()
    assert np.isnan(got[0]) and np.isfinite(got[1]) and got[1] > 0
    # the engine flags go alone, and not with the uniform kernel or on 2D paths
    for prm in (F.params(flags=F.FSMI_F_RLE_RUNS | F.FSMI_F_RLE_CELLS),
                F.params(variant=F.FSMI_UNIFORM, flags=F.FSMI_F_RLE_RUNS)):
        with pytest.raises(F.FsmiError):
            ctx.fsmi_rle_eval_beams(prm, dev(off), dev(ro), dev(rl), dev(sp))
    with pytest.raises(F.FsmiError):
        ctx.fsmi_eval_beams(F.params(flags=F.FSMI_F_RLE_RUNS), dev(off), dev(ro), dev(sp))
