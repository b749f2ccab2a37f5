"""Planned beam batches (fsmi_plan_*): one schedule, autotuned wave/tile
threshold, HIP-graph replays that follow new inputs, against the eager call and
the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1905_02238_amd import fsmi as F
from paper_1905_02238_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12


@pytest.fixture(scope="module")
def ctx():
    """A context of its own, so no autotuned threshold leaks in or out."""
    print("[gpu] plan tests: fresh context on cuda:0", flush=True)
    c = F.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_err(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0)
    nz = ~zero
    return float(np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz]))) if np.any(nz) else 0.0


def test_plan_schedule_and_eager_agree(ctx):
    print("[gpu] plan vs eager", flush=True)
    off, occ, sigma = W.uneven_beams(600, seed=81, n_max=1500)
    lens = np.diff(off)
    prm = F.params()
    o_, oc, sg = dev(off), dev(occ), dev(sigma)
    ref = O.eval_beams(O.EXACT, off, occ, sigma)
    for wm in (96, 512):
        plan = F.Plan(ctx, prm, o_, oc, sg, wave_max=wm)
        info = plan.info()
        assert info["wave_max"] == wm and info["max_len"] == int(lens.max())
        assert info["n_tile"] == int(np.sum(lens > wm)) and info["n_wave"] == int(np.sum(lens <= wm))
        assert not info["graph"] and info["tried"] == []
        mi = plan.launch().clone()
        torch.cuda.synchronize()
        ctx.fsmi_sync()
        assert rel_err(mi.cpu().numpy(), ref) <= TOL32
        if wm == 512:   # the eager call's default threshold: the same kernels, bit for bit
            eager = ctx.fsmi_eval_beams(prm, o_, oc, sg)
            torch.cuda.synchronize()
            assert torch.equal(mi, eager)
        plan.close()


def test_plan_graph_replays_follow_new_inputs(ctx):
    print("[gpu] plan graph replays", flush=True)
    off, occ, sigma = W.uneven_beams(500, seed=82, n_max=1200)
    prm = F.params()
    o_, oc, sg = dev(off), dev(occ), dev(sigma)
    plan = F.Plan(ctx, prm, o_, oc, sg, wave_max=512, graph=True)
    assert plan.info()["graph"]
    rng = np.random.default_rng(5)
    for r in range(4):
        occ_r = occ if r == 0 else rng.uniform(0.0, 1.0, occ.size).astype(np.float32)
        sig_r = sigma if r == 0 else rng.uniform(1.0, 6.0, sigma.size).astype(np.float32)
        oc.copy_(torch.from_numpy(occ_r))          # eager work between the replays
        sg.copy_(torch.from_numpy(sig_r))
        got = plan.launch().clone()
        eager = ctx.fsmi_eval_beams(prm, o_, oc, sg)
        torch.cuda.synchronize()
        ctx.fsmi_sync()
        assert torch.equal(got, eager), r
        if r < 2:
            assert rel_err(got.cpu().numpy(), O.eval_beams(O.EXACT, off, occ_r, sig_r)) <= TOL32
    plan.close()


def _bounded_batch(seed, n_beams, n_max):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, n_max + 1, n_beams)
    off = np.zeros(n_beams + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    occ = rng.uniform(0.0, 1.0, int(off[-1])).astype(np.float32)
    sigma = rng.uniform(0.3, 5.0, n_beams).astype(np.float32)
    bound = np.zeros(int(off[-1]) + n_beams)
    for b in range(n_beams):
        w = rng.uniform(0.05, 1.5, int(lens[b]))
        bound[off[b] + b: off[b] + b + lens[b] + 1] = np.concatenate([[0.0], np.cumsum(w)])
    return off, occ, bound, sigma


@pytest.mark.parametrize("variant", [F.FSMI_EXACT, F.FSMI_APPROX, F.FSMI_UNIFORM])
@pytest.mark.parametrize("prec", [F.FSMI_FP32, F.FSMI_FP64])
def test_plan_graph_variants_and_boundaries(ctx, variant, prec):
    print(f"[gpu] plan graph variant {variant} precision {prec}", flush=True)
    off, occ, bound, sigma = _bounded_batch(90 + variant, 160, 700)
    prm = F.params(variant=variant, trunc_delta=4, uniform_h=3, precision=prec)
    plan = F.Plan(ctx, prm, dev(off), dev(occ), dev(sigma), bound=dev(bound), wave_max=200,
                  graph=True)
    mi = plan.launch()
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    ov = {F.FSMI_EXACT: O.EXACT, F.FSMI_APPROX: O.APPROX, F.FSMI_UNIFORM: O.UNIFORM}[variant]
    ref = O.eval_beams(ov, off, occ, sigma, bound=bound, Delta=4, H=3)
    assert rel_err(mi.cpu().numpy(), ref) <= (TOL64 if prec == F.FSMI_FP64 else TOL32)
    plan.close()


def test_plan_autotune_keeps_the_fastest(ctx):
    print("[gpu] plan autotune", flush=True)
    off, occ, sigma = W.uneven_beams(20000, seed=83)
    prm = F.params()
    o_, oc, sg = dev(off), dev(occ), dev(sigma)
    plan = F.Plan(ctx, prm, o_, oc, sg, autotune=True, graph=True)
    info = plan.info()
    ws = [w for w, _ in info["tried"]]
    ms = [m for _, m in info["tried"]]
    assert len(ws) >= 3 and all(m > 0 for m in ms)
    assert info["wave_max"] == ws[int(np.argmin(ms))]
    assert info["graph"]
    mi = plan.launch().clone()
    eager = ctx.fsmi_eval_beams(prm, o_, oc, sg)    # takes the tuned threshold now
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    assert torch.equal(mi, eager)
    nb = 400
    ref = O.eval_beams(O.EXACT, off[:nb + 1], occ[:off[nb]], sigma[:nb])
    assert rel_err(mi[:nb].cpu().numpy(), ref) <= TOL32
    plan.close()


def test_plan_rejects_what_does_not_fit(ctx):
    off = np.array([0, 9000], np.int64)        # one beam longer than a workgroup's LDS holds
    occ = np.full(9000, 0.3, np.float32)
    sigma = np.array([2.0], np.float32)
    with pytest.raises(F.FsmiError) as e:
        F.Plan(ctx, F.params(), dev(off), dev(occ), dev(sigma))
    assert e.value.status == F.FSMI_E_CAPACITY
    with pytest.raises(F.FsmiError) as e:
        F.Plan(ctx, F.params(), dev(np.array([0], np.int64)), dev(occ[:1]), dev(sigma))
    assert e.value.status == F.FSMI_E_INVAL
    ctx.fsmi_sync()
