"""The look-up-table mode (FSMI_F_LUT, Sec. 3.3) of 2D fsmi_eval_poses against
the FP64 oracle's exact FSMI and Approx-FSMI, within the error its tables
allow.  Per beam,
    |I_lut - I| <= eps_E sum_j P(e_j) sum_k |C_k| + eps_f n + 1e-5 |I|,
eps_E = 6e-6 bounding the linear interpolation of erfc at the table's step
(each weight G_{k,j} is half a difference of two tail values), eps_f = 5e-7
bounding that of f (C_k sums up to n of them, and a row's weights sum to at
most 1), and 1e-5 the FP32 mode's own bar.  P(e_j) and C_k come from the
oracle on the oracle's own ray walk.  The mode must really read the tables
(its values differ from the analytic FP32 path's), and every other path
rejects the flag."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1905_02238_amd import fsmi as F
from paper_1905_02238_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS_E = 6e-6
EPS_F = 5e-7


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] lut: creating libfsmi context on cuda:0", flush=True)
    return F.context(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def world_dirs(pose, bd):
    c, s = pose[2], pose[3]
    m1, m2, m3, m4 = c * bd[:, 0], s * bd[:, 1], s * bd[:, 0], c * bd[:, 1]
    return np.stack([m1 - m2, m3 + m4], 1)


def beam_bounds(grid, poses, bd, R):
    """The per-beam error allowance's table part, from the oracle's walk."""
    out = np.zeros((len(poses), len(bd)))
    for p, pose in enumerate(poses):
        for b, d in enumerate(world_dirs(pose, bd)):
            _, _, occ = O.raycast2d(grid, pose[:2], d, R)
            if len(occ) == 0:
                continue
            P = O.first_hit(occ)[1:]
            C = O.info_gain(occ)
            out[p, b] = EPS_E * P.sum() * np.abs(C).sum() + EPS_F * len(occ)
    return out


def check(ctx, wl, poses, variant):
    prm = F.params(variant=variant, trunc_delta=wl["Delta"], flags=F.FSMI_F_LUT)
    g, p, bd = dev(wl["grid"]), dev(poses), dev(wl["beam_dir"])
    mp, mb = ctx.fsmi_eval_poses(prm, g, p, bd, wl["sigma"], wl["R"], want_beams=True)
    _, ma = ctx.fsmi_eval_poses(F.params(variant=variant, trunc_delta=wl["Delta"]), g, p, bd,
                                wl["sigma"], wl["R"], want_beams=True)
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    mb, ma, mp = mb.cpu().numpy(), ma.cpu().numpy(), mp.cpu().numpy()
    rp, rb = O.eval_poses_2d(variant, wl["grid"], poses, wl["beam_dir"], wl["sigma"], wl["R"],
                             Delta=wl["Delta"])
    allow = beam_bounds(wl["grid"], poses, wl["beam_dir"], wl["R"]) + 1e-5 * np.abs(rb)
    err = np.abs(mb - rb)
    worst = float(np.max(err / allow))
    rel = float(np.max(err / np.maximum(np.abs(rb), 1e-30)))
    print(f"[gpu] lut variant={variant}: worst error / allowance {worst:.3f}, "
          f"max rel err {rel:.2e}", flush=True)
    assert np.all(err <= allow)
    assert np.allclose(mp, mb.sum(axis=1), rtol=1e-12, atol=0.0)
    assert not np.array_equal(mb, ma)          # the tables were used
    return rel


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX])
def test_lut_grid_small(ctx, variant):
    """200 x 200 rooms, 60 beams, R = 150, sigma = 2."""
    wl = dict(W.grid_small())
    wl["Delta"] = 6
    check(ctx, wl, wl["poses"], variant)


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX])
def test_lut_grid_large_two_poses(ctx, variant):
    """Two poses of the timed 2D workload (2048 x 2048 rooms, 360 beams,
    R = 400, sigma = 3, Delta = 9)."""
    wl = W.grid_large(n_poses=4096)
    check(ctx, wl, wl["poses"][[5, 3001]], variant)


def test_lut_rejected_elsewhere(ctx):
    wl = W.grid_small()
    g, p, bd = dev(wl["grid"]), dev(wl["poses"]), dev(wl["beam_dir"])
    for prm in (F.params(flags=F.FSMI_F_LUT, precision=F.FSMI_FP64),
                F.params(variant=F.FSMI_UNIFORM, flags=F.FSMI_F_LUT),
                F.params(variant=F.FSMI_CSQMI, trunc_delta=3, flags=F.FSMI_F_LUT),
                F.params(flags=F.FSMI_F_LUT | F.FSMI_F_SKIP_ZERO),
                F.params(flags=F.FSMI_F_LUT, sigma_slope=0.01)):
        with pytest.raises(F.FsmiError) as e:
            ctx.fsmi_eval_poses(prm, g, p, bd, wl["sigma"], wl["R"])
        assert e.value.status == 1
    off = dev(np.array([0, 3], np.int64))
    occ = dev(np.array([0.2, 0.5, 0.7], np.float32))
    sg = dev(np.array([1.0], np.float32))
    with pytest.raises(F.FsmiError) as e:
        ctx.fsmi_eval_beams(F.params(flags=F.FSMI_F_LUT), off, occ, sg)
    assert e.value.status == 6
    run_off = dev(np.array([0, 1], np.int64))
    rl = dev(np.array([3], np.int32))
    with pytest.raises(F.FsmiError) as e:
        ctx.fsmi_rle_eval_beams(F.params(flags=F.FSMI_F_LUT), run_off, occ[:1].contiguous(), rl, sg)
    assert e.value.status == 6
