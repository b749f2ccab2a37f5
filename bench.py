"""Benchmark: beams/s of exact FSMI on one MI355X, with its roofline and the
FP64 oracle timed on the host's cores beside it.

Timed step (the metric's workload): exact FSMI (Thm 1) for 4096 candidate
poses x 360 beams on a 2048 x 2048 room grid with 30 % unknown frontier blobs,
max range 400 cells, sigma = 3 cells, FP32 with compensated sums; one step =
one fsmi_eval_poses call (grid walk, gather, P(e_j), C_k, the double sum, the
per-pose FP64 sum).  Inputs are resident in HBM before timing starts.

Other variants and workloads are measured once each and reported as extra
fields (Approx-FSMI, Uniform-FSMI on the same poses; the uneven 100k-beam
batch; 3D FSMI-RLE / Approx-FSMI-RLE on the voxel map; the 200 x 200 FP64 and
FP32 single-pose latency).  ``--quick`` skips those extras and shrinks the
CPU baseline sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic main-VALU instructions per (row j, boundary) pair of the exact
# sum, one issue slot each: l - mu (FP64 add) 1, |.| * c (FP64 mul) 1, convert 1;
# erfc = t 2^(P2(t) - x^2), t = 1/(1 + x / (2 sqrt(log2 e))): fma 1, 9-term
# Horner 9, exponent fma 1, product 1; |E_b - E_{b-1}| 1, C_k G fma 1; the
# compensated sum's share (4 ops per 4 pairs) 1.  The reciprocal and 2^x run on
# the transcendental unit, which issues alongside the main VALU on gfx950 (the
# measured rate with them counted exceeds the single-issue figure), so they are
# not charged.
SLOTS_PER_PAIR = 19
# ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s
# (one non-packed FP32 or FP64 VALU instruction per lane per clock).
ALU_PEAK_TSLOT = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--poses", type=int, default=4096)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-step", action="store_true",
                    help="for counter runs: one plain 256 MiB device copy (the traffic "
                         "calibration), then exactly one timed-workload step, nothing else")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU; runs on more than one GPU are not "
              "supported (the path shards by poses, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_02238_amd import fsmi as F
    from paper_1905_02238_amd import workloads as W

    dev = torch.device("cuda:0")
    ctx = F.context(0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    log(f"[bench] generating the 2048^2 room grid and {args.poses} poses")
    wl = W.grid_large(n_poses=args.poses)
    grid, poses, bdir = t(wl["grid"]), t(wl["poses"]), t(wl["beam_dir"])
    sigma, R = wl["sigma"], wl["R"]
    n_poses, n_beams = poses.shape[0], bdir.shape[0]
    n_total = n_poses * n_beams
    prm = F.params(variant=F.FSMI_EXACT)

    if args.profile_step:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                      # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        ctx.fsmi_eval_poses(prm, grid, poses, bdir, sigma, R)
        torch.cuda.synchronize()
        ctx.fsmi_sync()
        log("[bench] profile step done")
        return

    # cells per beam (count-only walk) -> algorithmic pairs per step
    c, s_ = poses[:, 2:3], poses[:, 3:4]
    wdir = torch.stack([c * bdir[None, :, 0] - s_ * bdir[None, :, 1],
                        s_ * bdir[None, :, 0] + c * bdir[None, :, 1]], -1).reshape(-1, 2).contiguous()
    org = poses[:, None, :2].expand(n_poses, n_beams, 2).reshape(-1, 2).contiguous()
    cnt = torch.empty(n_total, dtype=torch.int32, device=dev)
    mc = int(math.floor(math.sqrt(2.0) * R)) + 3
    import ctypes as C
    m = F._map(grid)
    ctx._stream()
    ctx._check(F.load().fsmi_raycast(ctx.handle, C.byref(m), F.FSMI_RAY_DDA, n_total,
                                     C.c_void_p(org.data_ptr()), C.c_void_p(wdir.data_ptr()),
                                     float(R), 1.0, mc, C.c_void_p(cnt.data_ptr()), None, None,
                                     None, None))
    torch.cuda.synchronize()
    n64 = cnt.to(torch.float64)
    pairs = float((n64 * (n64 + 1)).sum())
    mean_n = float(n64.mean())
    log(f"[bench] {n_total} beams, mean {mean_n:.1f} cells, {pairs:.3e} (row, boundary) pairs per step")

    # ---- timed region ----
    for _ in range(args.warmup):
        ctx.fsmi_eval_poses(prm, grid, poses, bdir, sigma, R)
    torch.cuda.synchronize()
    ctx.fsmi_sync()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev0[i].record()
        mp, _ = ctx.fsmi_eval_poses(prm, grid, poses, bdir, sigma, R)
        ev1[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.fsmi_sync()
    ev_ms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    ms_step = wall / args.steps * 1e3
    value = n_total / (wall / args.steps)
    kern_ms = float(np.mean(ev_ms))
    achieved = pairs * SLOTS_PER_PAIR / (kern_ms * 1e-3) / 1e12
    log(f"[bench] exact: {ms_step:.2f} ms/step (events {kern_ms:.2f} ms), {value/1e6:.3f} M beams/s")

    out = {
        "metric": "beams/s exact FSMI (<=1e-5 rel vs FP64)",
        "value": value,
        "unit": "beams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded room grid, frontier blobs, poses in free space)",
        "config": {"workload": "2D exact FSMI: 2048x2048 rooms + 30% unknown blobs, "
                               f"{n_poses} poses x {n_beams} beams, R=400, sigma=3",
                   "poses": n_poses, "beams_per_pose": n_beams, "max_range": R, "sigma": sigma,
                   "mean_cells_per_beam": mean_n, "pairs_per_step": pairs},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TSLOT,
                     "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TSLOT, "traffic": None,
                     "kernel": "k_poses2d<float>", "kernel_ms": kern_ms,
                     "work": f"{SLOTS_PER_PAIR} VALU slots per (row, boundary) pair"},
    }

    # ---- accuracy of the timed result on a sample of poses (oracle) ----
    import oracle as O
    sample = min(2, n_poses)
    rp, _ = O.eval_poses_2d(O.EXACT, wl["grid"], wl["poses"][:sample], wl["beam_dir"], sigma, R,
                            want_beams=False)
    got = mp[:sample].cpu().numpy()
    out["max_rel_err_vs_oracle"] = float(np.max(np.abs(got - rp) / np.abs(rp)))

    # ---- CPU baseline: the oracle as it stands, bounded sample ----
    if not args.no_cpu:
        thr = O.max_threads()
        t1 = time.perf_counter()
        O.eval_poses_2d(O.EXACT, wl["grid"], wl["poses"][:1], wl["beam_dir"], sigma, R,
                        threads=thr, want_beams=False)
        one = time.perf_counter() - t1
        budget = 3.0 if args.quick else args.cpu_seconds
        k = int(max(1, min(64, round(budget / max(one, 1e-3)))))
        t1 = time.perf_counter()
        O.eval_poses_2d(O.EXACT, wl["grid"], wl["poses"][:k], wl["beam_dir"], sigma, R,
                        threads=thr, want_beams=False)
        cs = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": k * n_beams / cs, "unit": "beams/s", "cores": thr,
                               "kind": "oracle",
                               "sample": f"first {k} poses x {n_beams} beams of the timed workload, "
                                         f"{cs:.1f} s, FP64, OpenMP over beams"}
        log(f"[bench] cpu oracle: {k} poses in {cs:.1f} s on {thr} threads")

    # ---- extras: other variants and workloads, one timed run each ----
    if not args.quick:
        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t1) / reps
        extras = {}
        for name, p in (("approx_delta9", F.params(variant=F.FSMI_APPROX, trunc_delta=9)),
                        ("uniform_h6", F.params(variant=F.FSMI_UNIFORM, uniform_h=6))):
            dt = timed(lambda: ctx.fsmi_eval_poses(p, grid, poses, bdir, sigma, R))
            extras[name] = {"beams_per_s": n_total / dt, "ms": dt * 1e3}
            log(f"[bench] {name}: {n_total/dt/1e6:.2f} M beams/s")
        off, occ, sg = W.uneven_beams(100000, seed=W.SEED_BASE + 3)
        o_, oc, s2 = t(off), t(occ), t(sg)
        dt = timed(lambda: ctx.fsmi_eval_beams(prm, o_, oc, s2))
        lens = np.diff(off).astype(np.float64)
        extras["uneven_100k_exact"] = {"beams_per_s": 1e5 / dt, "ms": dt * 1e3,
                                       "pairs": float(np.sum(lens * lens))}
        log(f"[bench] uneven 100k exact: {1e5/dt/1e6:.2f} M beams/s")
        small = W.grid_small()
        gs, ps, bs = t(small["grid"]), t(small["poses"]), t(small["beam_dir"])
        for name, pr in (("grid_small_fp64_us", F.FSMI_FP64), ("grid_small_fp32_us", F.FSMI_FP32)):
            pp = F.params(precision=pr)
            dt = timed(lambda: ctx.fsmi_eval_poses(pp, gs, ps, bs, small["sigma"], small["R"]), reps=10)
            extras[name] = dt * 1e6
        log("[bench] generating the 512x512x128 voxel map")
        vw = W.voxels_large(n_poses=256)
        vx, vp, vb = t(vw["vox"]), t(vw["poses"]), t(vw["beam_dir"])
        nv = vp.shape[0] * vb.shape[0]
        for name, p in (("rle_exact_3d", F.params(variant=F.FSMI_EXACT)),
                        ("rle_approx_delta6_3d", F.params(variant=F.FSMI_APPROX, trunc_delta=6))):
            dt = timed(lambda: ctx.fsmi_eval_poses(p, vx, vp, vb, vw["sigma"], vw["R"], vw["w"]), reps=2)
            extras[name] = {"beams_per_s": nv / dt, "ms": dt * 1e3, "poses": vp.shape[0]}
            log(f"[bench] {name}: {nv/dt/1e6:.2f} M beams/s")
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
