"""Seeded synthetic workloads shaped like the paper's maps and beams.

This module only draws inputs: occupancy grids, poses, sensor directions and
batches of beams.  It holds none of the mutual-information arithmetic, and is
the one module that both the HIP path's callers and the oracle's tests use to
make identical inputs.

Recipes (the paper uses its own robot logs and OctoMaps, which are not
available; these stand in for them):

* 2D room grids (the paper's simulated 18 m x 18 m world and its 8 m x 8 m lab,
  Sec. 5.2-5.3): a 2-cell wall border; a recursive binary space partition that
  splits the longer side at U(0.35, 0.65) while it exceeds ``split_extent``
  cells; 2-cell walls with one door gap of U{8..16} cells; each leaf room left
  unexplored (o = 0.5) with probability 0.25.  Free o ~ U(0.05, 0.3), wall
  o ~ U(0.8, 0.95), drawn per cell.  Optional frontier blobs (discs of radius
  U(20, 120) set to o = 0.5) are added until a target fraction of cells is
  unknown.
* 3D voxel maps (the paper's OctoMap scenes, Sec. 5.5): a 2-voxel ground slab,
  boxes and pillars whose voxels share one o ~ U(0.8, 0.95) per object, free
  space with one o ~ U(0.05, 0.3) per aligned ``block``^3 block (the way an
  OctoMap stores pruned free leaves), and unknown spheres at o = 0.5.
* Uneven beam batches: lengths log-uniform in [8, 2000] cells, each cell's o
  from a three-component mixture around 0.1 / 0.5 / 0.9 (+- 0.05), sigma per
  beam U(1, 6) cells.

Seeds: workload c uses ``SEED_BASE + c``.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1905022380

FREE, WALL, UNKNOWN = 0, 1, 2


# ---------------------------------------------------------------------------
# 2D room grids
# ---------------------------------------------------------------------------
def _bsp(lab, x0, y0, x1, y1, rng, split_extent, rooms):
    w, h = x1 - x0, y1 - y0
    if max(w, h) <= split_extent or min(w, h) < 8:
        rooms.append((x0, y0, x1, y1))
        return
    if w >= h:
        s = x0 + int(round(w * rng.uniform(0.35, 0.65)))
        lab[y0:y1, s:s + 2] = WALL
        gl = min(int(rng.integers(8, 17)), h)
        gy = y0 + int(rng.integers(0, h - gl + 1))
        lab[gy:gy + gl, s:s + 2] = FREE
        _bsp(lab, x0, y0, s, y1, rng, split_extent, rooms)
        _bsp(lab, s + 2, y0, x1, y1, rng, split_extent, rooms)
    else:
        s = y0 + int(round(h * rng.uniform(0.35, 0.65)))
        lab[s:s + 2, x0:x1] = WALL
        gl = min(int(rng.integers(8, 17)), w)
        gx = x0 + int(rng.integers(0, w - gl + 1))
        lab[s:s + 2, gx:gx + gl] = FREE
        _bsp(lab, x0, y0, x1, s, rng, split_extent, rooms)
        _bsp(lab, x0, s + 2, x1, y1, rng, split_extent, rooms)


def room_labels(size: int, seed: int, split_extent: int, unknown_frac: float = 0.0):
    """Label grid [Y][X] (uint8: FREE / WALL / UNKNOWN)."""
    rng = np.random.default_rng(seed)
    lab = np.full((size, size), FREE, np.uint8)
    lab[:2, :] = WALL
    lab[-2:, :] = WALL
    lab[:, :2] = WALL
    lab[:, -2:] = WALL
    rooms = []
    _bsp(lab, 2, 2, size - 2, size - 2, rng, split_extent, rooms)
    for (x0, y0, x1, y1) in rooms:
        if rng.uniform() < 0.25:
            sub = lab[y0:y1, x0:x1]
            sub[sub == FREE] = UNKNOWN
    if unknown_frac > 0.0:
        yy, xx = np.mgrid[0:size, 0:size]
        while np.count_nonzero(lab == UNKNOWN) < unknown_frac * size * size:
            cx, cy = rng.uniform(0, size, 2)
            r = rng.uniform(20.0, 120.0)
            x0, x1 = max(0, int(cx - r)), min(size, int(cx + r) + 1)
            y0, y1 = max(0, int(cy - r)), min(size, int(cy + r) + 1)
            m = (xx[y0:y1, x0:x1] - cx) ** 2 + (yy[y0:y1, x0:x1] - cy) ** 2 <= r * r
            lab[y0:y1, x0:x1][m] = UNKNOWN
    return lab


def occupancy_from_labels(lab, seed: int):
    rng = np.random.default_rng(seed + 7)
    o = np.empty(lab.shape, np.float32)
    free = lab == FREE
    wall = lab == WALL
    o[free] = rng.uniform(0.05, 0.3, np.count_nonzero(free)).astype(np.float32)
    o[wall] = rng.uniform(0.8, 0.95, np.count_nonzero(wall)).astype(np.float32)
    o[lab == UNKNOWN] = np.float32(0.5)
    return o


def room_grid(size: int, seed: int, split_extent: int, unknown_frac: float = 0.0):
    """(occupancy float32 [Y][X], labels uint8 [Y][X])."""
    lab = room_labels(size, seed, split_extent, unknown_frac)
    return occupancy_from_labels(lab, seed), lab


def poses_in_free_space_2d(lab, n: int, seed: int, yaw: str = "zero"):
    """n poses [x, y, cos(yaw), sin(yaw)] uniform over FREE cells (continuous in
    the cell); yaw 0 (``yaw="zero"``) or U[0, 2 pi) (``yaw="uniform"``, drawn
    after the positions, so the positions do not depend on it)."""
    rng = np.random.default_rng(seed + 11)
    ys, xs = np.nonzero(lab == FREE)
    pick = rng.integers(0, len(xs), n)
    out = np.zeros((n, 4), np.float64)
    out[:, 0] = xs[pick] + rng.uniform(0.0, 1.0, n)
    out[:, 1] = ys[pick] + rng.uniform(0.0, 1.0, n)
    if yaw == "uniform":
        a = rng.uniform(0.0, 2.0 * math.pi, n)
        out[:, 2] = np.cos(a)
        out[:, 3] = np.sin(a)
    elif yaw == "zero":
        out[:, 2] = 1.0
        out[:, 3] = 0.0
    else:
        raise ValueError(f"unknown yaw mode {yaw!r}")
    return out


def walks_2d(lab, n_traj: int, steps: int, seed: int, step_len: float = 4.0):
    """Candidate trajectories for the planner-level sum (Sec. 2.4): n_traj walks
    of `steps` states through FREE cells, each starting at a random free cell
    (continuous within it) with a random heading, stepping step_len cells along
    the heading and turning to a fresh random heading whenever the next state
    would leave free space.  Returns (traj_off int64 [n_traj + 1], states
    float64 [n_traj * steps][4] = x, y, cos(yaw), sin(yaw)), the yaw being the
    heading of travel."""
    rng = np.random.default_rng(seed + 17)
    ys, xs = np.nonzero(lab == FREE)
    H, Wd = lab.shape
    states, off = [], [0]
    for _ in range(n_traj):
        i = rng.integers(0, len(xs))
        x, y = xs[i] + rng.uniform(0.1, 0.9), ys[i] + rng.uniform(0.1, 0.9)
        a = rng.uniform(0.0, 2.0 * math.pi)
        for _ in range(steps):
            states.append([x, y, math.cos(a), math.sin(a)])
            for _ in range(30):
                nx, ny = x + step_len * math.cos(a), y + step_len * math.sin(a)
                if 0 <= nx < Wd and 0 <= ny < H and lab[int(ny), int(nx)] == FREE:
                    x, y = nx, ny
                    break
                a = rng.uniform(0.0, 2.0 * math.pi)
        off.append(len(states))
    return np.array(off, np.int64), np.array(states, np.float64)


def beam_dirs_2d(n_beams: int):
    """Sensor-frame unit vectors, angle 2*pi*b/B from +x (host libm)."""
    th = 2.0 * math.pi * np.arange(n_beams, dtype=np.float64) / n_beams
    return np.stack([np.cos(th), np.sin(th)], axis=1)


# ---------------------------------------------------------------------------
# 3D voxel maps
# ---------------------------------------------------------------------------
def voxel_map(X: int, Y: int, Z: int, seed: int, n_boxes: int = 160, n_pillars: int = 120,
              block: int = 32, unknown_frac: float = 0.15):
    """(occupancy float32 [Z][Y][X], labels uint8 [Z][Y][X])."""
    rng = np.random.default_rng(seed)
    lab = np.full((Z, Y, X), FREE, np.uint8)
    occ = np.empty((Z, Y, X), np.float32)
    # free space: one value per aligned block^3 block
    bz, by, bx = -(-Z // block), -(-Y // block), -(-X // block)
    bv = rng.uniform(0.05, 0.3, (bz, by, bx)).astype(np.float32)
    occ[...] = np.repeat(np.repeat(np.repeat(bv, block, 0), block, 1), block, 2)[:Z, :Y, :X]
    # unknown spheres
    target = unknown_frac * X * Y * Z
    count = 0
    while count < target:
        c = rng.uniform([0, 0, 0], [X, Y, Z])
        r = rng.uniform(10.0, 40.0)
        x0, x1 = max(0, int(c[0] - r)), min(X, int(c[0] + r) + 1)
        y0, y1 = max(0, int(c[1] - r)), min(Y, int(c[1] + r) + 1)
        z0, z1 = max(0, int(c[2] - r)), min(Z, int(c[2] + r) + 1)
        zz, yy, xx = np.ogrid[z0:z1, y0:y1, x0:x1]
        m = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= r * r
        sub = lab[z0:z1, y0:y1, x0:x1]
        count += int(np.count_nonzero(m & (sub != UNKNOWN)))
        sub[m] = UNKNOWN
        occ[z0:z1, y0:y1, x0:x1][m] = np.float32(0.5)
    # ground slab
    g = np.float32(rng.uniform(0.8, 0.95))
    lab[:2] = WALL
    occ[:2] = g
    # boxes
    for _ in range(n_boxes):
        sx, sy = rng.uniform(5, 40, 2)
        hz = rng.uniform(5, 60)
        x0 = int(rng.uniform(0, X - sx))
        y0 = int(rng.uniform(0, Y - sy))
        x1, y1, z1 = x0 + int(sx), y0 + int(sy), min(Z, 2 + int(hz))
        v = np.float32(rng.uniform(0.8, 0.95))
        lab[2:z1, y0:y1, x0:x1] = WALL
        occ[2:z1, y0:y1, x0:x1] = v
    # pillars
    yy2, xx2 = np.mgrid[0:Y, 0:X]
    for _ in range(n_pillars):
        r = rng.uniform(2, 6)
        cx, cy = rng.uniform(0, X), rng.uniform(0, Y)
        x0, x1 = max(0, int(cx - r)), min(X, int(cx + r) + 1)
        y0, y1 = max(0, int(cy - r)), min(Y, int(cy + r) + 1)
        m = (xx2[y0:y1, x0:x1] - cx) ** 2 + (yy2[y0:y1, x0:x1] - cy) ** 2 <= r * r
        v = np.float32(rng.uniform(0.8, 0.95))
        lab[:, y0:y1, x0:x1][:, m] = WALL
        occ[:, y0:y1, x0:x1][:, m] = v
    return occ, lab


def poses_in_free_space_3d(lab, n: int, seed: int, z_max: int | None = None):
    """n poses [x, y, z, cos(yaw), sin(yaw)] uniform over FREE voxels, yaw U[0, 2pi)."""
    rng = np.random.default_rng(seed + 13)
    sub = lab if z_max is None else lab[:z_max]
    zs, ys, xs = np.nonzero(sub == FREE)
    pick = rng.integers(0, len(xs), n)
    yaw = rng.uniform(0.0, 2.0 * math.pi, n)
    out = np.zeros((n, 5), np.float64)
    out[:, 0] = xs[pick] + rng.uniform(0.0, 1.0, n)
    out[:, 1] = ys[pick] + rng.uniform(0.0, 1.0, n)
    out[:, 2] = zs[pick] + rng.uniform(0.0, 1.0, n)
    out[:, 3] = np.cos(yaw)
    out[:, 4] = np.sin(yaw)
    return out


def beam_dirs_3d(rows: int = 64, cols: int = 256, fov_h_deg: float = 90.0,
                 fov_v_deg: float = 60.0):
    """Depth-camera pixel directions: equiangular pixel centres,
    az = -fov_h/2 + fov_h (c + 1/2)/cols, el = -fov_v/2 + fov_v (r + 1/2)/rows,
    d = (cos el cos az, cos el sin az, sin el).  Row-major [rows*cols][3]."""
    c = np.arange(cols, dtype=np.float64)
    r = np.arange(rows, dtype=np.float64)
    az = np.deg2rad(-fov_h_deg / 2 + fov_h_deg * (c + 0.5) / cols)
    el = np.deg2rad(-fov_v_deg / 2 + fov_v_deg * (r + 0.5) / rows)
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1)
    return d.reshape(-1, 3)


# ---------------------------------------------------------------------------
# Beam batches
# ---------------------------------------------------------------------------
def uneven_beams(n_beams: int, seed: int, n_min: int = 8, n_max: int = 2000,
                 sigma_lo: float = 1.0, sigma_hi: float = 6.0):
    """CSR batch: (off int64 [n+1], occ float32 [off[-1]], sigma float32 [n])."""
    rng = np.random.default_rng(seed)
    lens = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_beams))).astype(np.int64)
    off = np.zeros(n_beams + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    tot = int(off[-1])
    comp = rng.integers(0, 3, tot)
    centre = np.array([0.1, 0.5, 0.9])[comp]
    occ = (centre + rng.uniform(-0.05, 0.05, tot)).astype(np.float32)
    sigma = rng.uniform(sigma_lo, sigma_hi, n_beams).astype(np.float32)
    return off, occ, sigma


def random_beams(n_beams: int, seed: int, n_lo: int, n_hi: int, o_lo=0.0, o_hi=1.0,
                 widths=True, sigma_lo=0.5, sigma_hi=4.0):
    """Generic CSR batch with optional random cell boundaries.
    Returns off, occ, bound (float64 [off[-1] + n] or None), sigma."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(n_lo, n_hi + 1, n_beams).astype(np.int64)
    off = np.zeros(n_beams + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    occ = rng.uniform(o_lo, o_hi, int(off[-1])).astype(np.float32)
    sigma = rng.uniform(sigma_lo, sigma_hi, n_beams).astype(np.float32)
    bound = None
    if widths:
        bound = np.zeros(int(off[-1]) + n_beams, np.float64)
        for b in range(n_beams):
            n = int(lens[b])
            w = rng.uniform(0.02, 1.5, n)
            bound[off[b] + b: off[b] + b + n + 1] = np.concatenate([[0.0], np.cumsum(w)])
    return off, occ, bound, sigma


def rle_beams(n_beams: int, seed: int, run_lo: int, run_hi: int, n_runs_lo: int, n_runs_hi: int,
              sigma_lo=1.0, sigma_hi=3.0):
    """CSR batch of runs: (run_off int64, run_occ float32, run_len int32, sigma_p float32)."""
    rng = np.random.default_rng(seed)
    nr = rng.integers(n_runs_lo, n_runs_hi + 1, n_beams).astype(np.int64)
    off = np.zeros(n_beams + 1, np.int64)
    np.cumsum(nr, out=off[1:])
    tot = int(off[-1])
    occ = rng.uniform(0.02, 0.98, tot).astype(np.float32)
    ln = rng.integers(run_lo, run_hi + 1, tot).astype(np.int32)
    sig = rng.uniform(sigma_lo, sigma_hi, n_beams).astype(np.float32)
    return off, occ, ln, sig


def grouped_beams(n_beams: int, n_cells: int, L: int, seed: int):
    """Beams of n_cells equal-width cells in groups of L with one occupancy per
    group, o ~ U(0, 1) (the synthetic beams of the paper's run-length
    experiment, Sec. 5.4).  Returns the runs (run_off int64, run_occ float32,
    run_len int32) and the same beams expanded (off int64, occ float32)."""
    assert n_cells % L == 0
    rng = np.random.default_rng(seed)
    nr = n_cells // L
    run_off = np.arange(n_beams + 1, dtype=np.int64) * nr
    run_occ = rng.uniform(0.0, 1.0, n_beams * nr).astype(np.float32)
    run_len = np.full(n_beams * nr, L, np.int32)
    off = np.arange(n_beams + 1, dtype=np.int64) * n_cells
    occ = np.repeat(run_occ, L)
    return run_off, run_occ, run_len, off, occ


# ---------------------------------------------------------------------------
# The workloads by name
# ---------------------------------------------------------------------------
def grid_small(seed=SEED_BASE + 0):
    """200 x 200 rooms (cell 0.05 m), one pose at the grid centre (a cell vertex),
    60 beams over 360 deg, R = 150, sigma = 2."""
    occ, lab = room_grid(200, seed, split_extent=60)
    poses = np.array([[100.0, 100.0, 1.0, 0.0]])
    return dict(grid=occ, labels=lab, poses=poses, beam_dir=beam_dirs_2d(60), R=150.0,
                sigma=2.0)


def grid_large(n_poses=4096, seed=SEED_BASE + 1, yaw="uniform"):
    """2048 x 2048 rooms + 30 % unknown frontier blobs, poses uniform in free space
    with yaw U[0, 2 pi) (or 0 with ``yaw="zero"``), 360 beams at 1 deg, R = 400,
    sigma = 3 (Delta = 9, H = 6)."""
    occ, lab = room_grid(2048, seed, split_extent=160, unknown_frac=0.30)
    poses = poses_in_free_space_2d(lab, n_poses, seed, yaw=yaw)
    return dict(grid=occ, labels=lab, poses=poses, beam_dir=beam_dirs_2d(360), R=400.0,
                sigma=3.0, Delta=9, H=6)


def voxels_large(n_poses=1024, seed=SEED_BASE + 2, X=512, Y=512, Z=128):
    """512 x 512 x 128 voxels (0.1 m), 64 x 256 camera beams over 90 x 60 deg,
    R = 300, sigma = 2, w = 1 (Delta = 6)."""
    occ, lab = voxel_map(X, Y, Z, seed)
    poses = poses_in_free_space_3d(lab, n_poses, seed)
    return dict(vox=occ, labels=lab, poses=poses, beam_dir=beam_dirs_3d(), R=300.0, sigma=2.0,
                w=1.0, Delta=6)
