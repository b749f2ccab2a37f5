"""FP64 CPU oracle for FSMI (arXiv 1905.02238) -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP product path never calls it and
shares no code with it.  The arithmetic lives in ``fsmi_oracle.c`` (plain FP64
loops in the paper's order); this module only marshals numpy arrays.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        d, i, i64, p = C.c_double, C.c_int, C.c_int64, C.c_void_p
        sig = {
            "ora_f": (d, [d, d]),
            "ora_f_odds": (d, [d, d]),
            "ora_first_hit": (None, [i, p, p]),
            "ora_info_gain": (None, [i, p, d, p]),
            "ora_G": (d, [d, d, d, d]),
            "ora_fsmi_exact": (d, [i, p, p, d, d]),
            "ora_fsmi_exact_ext": (d, [i, p, p, d, d, i, d]),
            "ora_fsmi_approx": (d, [i, p, p, d, d, i]),
            "ora_fsmi_uniform": (d, [i, p, d, i]),
            "ora_kernel_weight": (d, [i, d, i, i]),
            "ora_fsmi_eqwidth": (d, [i, p, d, d, i, i, i]),
            "ora_rle_expanded": (d, [i, p, p, d, d, i, i, i]),
            "ora_rle_thm5": (d, [i, p, p, d, d, i, i, i]),
            "ora_rle_thm6": (d, [i, p, p, d, d, i, i, i]),
            "ora_rle_alpha_route": (d, [i, p, p, d, d]),
            "ora_rle_table": (d, [i, p, p, d, d, i, i]),
            "ora_tab_definition": (None, [d, d, i, i, p, p, p, p]),
            "ora_tab_recurrence": (None, [d, d, i, i, p, p, p, p]),
            "ora_raycast2d": (i, [p, i64, i64, d, d, d, d, d, i, p, p, p]),
            "ora_virtual3d": (i, [p, i64, i64, i64, p, p, d, d, i, p, p]),
            "ora_rle_runs": (i, [i, p, p, p]),
            "ora_eval_beams": (i, [i, i, i, d, d, i, i64, p, p, p, p, p, i]),
            "ora_rle_eval_beams": (i, [i, i, i, i, d, i64, p, p, p, p, p, i]),
            "ora_eval_poses_2d": (i, [i, i, i, d, d, i, p, i64, i64, i64, p, i64, p, d, d, p, p,
                                      i]),
            "ora_eval_poses_3d": (i, [i, i, i, i, d, p, i64, i64, i64, i64, p, i64, p, d, d, d,
                                      p, p, i]),
            "ora_max_threads": (i, []),
            "ora_csqmi": (d, [i, p, p, d, i]),
            "ora_fsmi_counted": (d, [i, i, p, p, d, d, i, i, p]),
            "ora_eval_trajectories_2d": (i, [i, i, i, d, p, i64, i64, i64, p, p, i64, p, d, d, p,
                                             p, p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


EXACT, APPROX, UNIFORM, CSQMI = 0, 1, 2, 3
K_ERF, K_DENSITY, K_UNIFORM = 0, 1, 2


def _pd(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def f(delta, o):
    return lib().ora_f(float(delta), float(o))


def f_odds(delta, r):
    return lib().ora_f_odds(float(delta), float(r))


def first_hit(o):
    o = _f64(o)
    P = np.zeros(len(o) + 1)
    lib().ora_first_hit(len(o), _pd(o), _pd(P))
    return P


def info_gain(o, delta_occ=1.5):
    o = _f64(o)
    Cc = np.zeros(len(o))
    lib().ora_info_gain(len(o), _pd(o), float(delta_occ), _pd(Cc))
    return Cc


def G(lk, lk1, mu, sigma):
    return lib().ora_G(float(lk), float(lk1), float(mu), float(sigma))


def fsmi_exact(o, l, sigma, delta_occ=1.5):
    o, l = _f64(o), _f64(l)
    assert len(l) == len(o) + 1
    return lib().ora_fsmi_exact(len(o), _pd(o), _pd(l), float(sigma), float(delta_occ))


def fsmi_exact_ext(o, l, sigma, slope=0.0, tail=False, delta_occ=1.5):
    """Thm 1 with range-dependent noise sigma_j = sigma + slope mu_j and, with
    tail, the max-range return term (ora_fsmi_exact_ext)."""
    o, l = _f64(o), _f64(l)
    assert len(l) == len(o) + 1
    return lib().ora_fsmi_exact_ext(len(o), _pd(o), _pd(l), float(sigma), float(slope),
                                    int(bool(tail)), float(delta_occ))


def fsmi_approx(o, l, sigma, Delta, delta_occ=1.5):
    o, l = _f64(o), _f64(l)
    assert len(l) == len(o) + 1
    return lib().ora_fsmi_approx(len(o), _pd(o), _pd(l), float(sigma), float(delta_occ),
                                 int(Delta))


def fsmi_uniform(o, H, delta_occ=1.5):
    o = _f64(o)
    return lib().ora_fsmi_uniform(len(o), _pd(o), float(delta_occ), int(H))


def kernel_weight(kind, sigma_p, d, H=0):
    return lib().ora_kernel_weight(int(kind), float(sigma_p), int(H), int(d))


def fsmi_eqwidth(o, sigma_p, kind=K_ERF, trunc=-1, H=0, delta_occ=1.5):
    o = _f64(o)
    return lib().ora_fsmi_eqwidth(len(o), _pd(o), float(sigma_p), float(delta_occ), int(kind),
                                  int(trunc), int(H))


def _runs(ro, L):
    ro = _f64(ro)
    L = np.ascontiguousarray(L, dtype=np.int32)
    assert len(ro) == len(L)
    return ro, L


def rle_expanded(ro, L, sigma_p, kind=K_ERF, trunc=-1, H=0, delta_occ=1.5):
    ro, L = _runs(ro, L)
    return lib().ora_rle_expanded(len(ro), _pd(ro), _pd(L), float(sigma_p), float(delta_occ),
                                  int(kind), int(trunc), int(H))


def rle_thm5(ro, L, sigma_p, kind=K_ERF, trunc=-1, H=0, delta_occ=1.5):
    ro, L = _runs(ro, L)
    return lib().ora_rle_thm5(len(ro), _pd(ro), _pd(L), float(sigma_p), float(delta_occ),
                              int(kind), int(trunc), int(H))


def rle_thm6(ro, L, sigma_p, Delta, kind=K_ERF, H=0, delta_occ=1.5):
    ro, L = _runs(ro, L)
    return lib().ora_rle_thm6(len(ro), _pd(ro), _pd(L), float(sigma_p), float(delta_occ),
                              int(kind), int(Delta), int(H))


def rle_alpha_route(ro, L, sigma_p, delta_occ=1.5):
    ro, L = _runs(ro, L)
    return lib().ora_rle_alpha_route(len(ro), _pd(ro), _pd(L), float(sigma_p), float(delta_occ))


def rle_table(ro, L, sigma_p, Delta, levels, delta_occ=1.5):
    """Table mode of Approx-FSMI-RLE: tables at 1 - o quantised to i / levels."""
    ro, L = _runs(ro, L)
    return lib().ora_rle_table(len(ro), _pd(ro), _pd(L), float(sigma_p), float(delta_occ),
                               int(Delta), int(levels))


def tables(x, sigma_p, Lb, Lmax, route="definition"):
    a = np.zeros((Lb + 1) * (Lb + 1))
    b = np.zeros((Lb + 1) * (Lb + 1))
    t = np.zeros(Lmax + 1)
    g = np.zeros(Lmax + 1)
    fn = lib().ora_tab_definition if route == "definition" else lib().ora_tab_recurrence
    fn(float(x), float(sigma_p), int(Lb), int(Lmax), _pd(a), _pd(b), _pd(t), _pd(g))
    return a.reshape(Lb + 1, Lb + 1), b.reshape(Lb + 1, Lb + 1), t, g


def raycast2d(grid, origin, direction, R, max_cells=None):
    """grid: float32 [Y][X]. Returns (cells int32, entries float64 [n+1], occ float32)."""
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    Y, X = grid.shape
    if max_cells is None:
        max_cells = int(np.floor(np.sqrt(2.0) * R)) + 3
    cell = np.zeros(max_cells, np.int32)
    entry = np.zeros(max_cells + 1, np.float64)
    occ = np.zeros(max_cells, np.float32)
    n = lib().ora_raycast2d(_pd(grid), X, Y, float(origin[0]), float(origin[1]),
                            float(direction[0]), float(direction[1]), float(R), int(max_cells),
                            _pd(cell), _pd(entry), _pd(occ))
    if n < 0:
        raise ValueError(f"raycast2d failed with code {n}")
    return cell[:n].copy(), entry[: n + 1].copy(), occ[:n].copy()


def virtual3d(vox, origin, direction, R, w=1.0):
    """vox: float32 [Z][Y][X]. Returns (cells int32, occ float32)."""
    vox = np.ascontiguousarray(vox, dtype=np.float32)
    Z, Y, X = vox.shape
    max_cells = int(np.floor(R / w)) + 1
    cell = np.zeros(max_cells, np.int32)
    occ = np.zeros(max_cells, np.float32)
    p = _f64(origin)
    d = _f64(direction)
    n = lib().ora_virtual3d(_pd(vox), X, Y, Z, _pd(p), _pd(d), float(R), float(w), max_cells,
                            _pd(cell), _pd(occ))
    if n < 0:
        raise ValueError(f"virtual3d failed with code {n}")
    return cell[:n].copy(), occ[:n].copy()


def rle_runs(occ):
    occ = np.ascontiguousarray(occ, dtype=np.float32)
    ro = np.zeros(max(len(occ), 1), np.float32)
    rl = np.zeros(max(len(occ), 1), np.int32)
    nr = lib().ora_rle_runs(len(occ), _pd(occ), _pd(ro), _pd(rl))
    return ro[:nr].copy(), rl[:nr].copy()


def eval_beams(variant, off, occ, sigma, bound=None, Delta=0, H=0, delta_occ=1.5, threads=0,
               slope=0.0, tail=False):
    off = np.ascontiguousarray(off, dtype=np.int64)
    occ = np.ascontiguousarray(occ, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    nb = len(off) - 1
    mi = np.zeros(nb)
    bnd = None if bound is None else _f64(bound)
    bp = None if bnd is None else _pd(bnd)
    lib().ora_eval_beams(int(variant), int(Delta), int(H), float(delta_occ), float(slope),
                         int(bool(tail)), nb, _pd(off), _pd(occ), bp, _pd(sigma), _pd(mi),
                         int(threads))
    return mi


def rle_eval_beams(exact, run_off, run_occ, run_len, sigma_p, kind=K_ERF, Delta=0, H=0,
                   delta_occ=1.5, threads=0):
    run_off = np.ascontiguousarray(run_off, dtype=np.int64)
    run_occ = np.ascontiguousarray(run_occ, dtype=np.float32)
    run_len = np.ascontiguousarray(run_len, dtype=np.int32)
    sigma_p = np.ascontiguousarray(sigma_p, dtype=np.float32)
    nb = len(run_off) - 1
    mi = np.zeros(nb)
    lib().ora_rle_eval_beams(int(bool(exact)), int(kind), int(Delta), int(H), float(delta_occ),
                             nb, _pd(run_off), _pd(run_occ), _pd(run_len), _pd(sigma_p), _pd(mi),
                             int(threads))
    return mi


def eval_poses_2d(variant, grid, poses, beam_dir, sigma, R, Delta=0, H=0, delta_occ=1.5,
                  threads=0, want_beams=True, slope=0.0, tail=False):
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    Y, X = grid.shape
    poses = _f64(poses).reshape(-1, 4)
    beam_dir = _f64(beam_dir).reshape(-1, 2)
    npo, nb = poses.shape[0], beam_dir.shape[0]
    mp = np.zeros(npo)
    mb = np.zeros((npo, nb)) if want_beams else None
    rc = lib().ora_eval_poses_2d(int(variant), int(Delta), int(H), float(delta_occ), float(slope),
                                 int(bool(tail)), _pd(grid), X, Y, npo, _pd(poses), nb,
                                 _pd(beam_dir), float(sigma), float(R), _pd(mp),
                                 None if mb is None else _pd(mb), int(threads))
    if rc != 0:
        raise ValueError("eval_poses_2d: a pose lies outside the map")
    return mp, mb


def eval_poses_3d(exact, vox, poses, beam_dir, sigma, R, w=1.0, kind=K_ERF, Delta=0, H=0,
                  delta_occ=1.5, threads=0, want_beams=True):
    vox = np.ascontiguousarray(vox, dtype=np.float32)
    Z, Y, X = vox.shape
    poses = _f64(poses).reshape(-1, 5)
    beam_dir = _f64(beam_dir).reshape(-1, 3)
    npo, nb = poses.shape[0], beam_dir.shape[0]
    mp = np.zeros(npo)
    mb = np.zeros((npo, nb)) if want_beams else None
    rc = lib().ora_eval_poses_3d(int(bool(exact)), int(kind), int(Delta), int(H),
                                 float(delta_occ), _pd(vox), X, Y, Z, npo, _pd(poses), nb,
                                 _pd(beam_dir), float(sigma), float(R), float(w), _pd(mp),
                                 None if mb is None else _pd(mb), int(threads))
    if rc != 0:
        raise ValueError("eval_poses_3d: a pose lies outside the map")
    return mp, mb


def max_threads():
    return lib().ora_max_threads()


def csqmi(o, l, sigma, Delta=-1):
    """Eq. csqmi_exact (Sec. 2.3) on one beam; Delta >= 0 truncates both double
    sums to |l - j| <= Delta (Approx-CSQMI), Delta < 0 is the exact metric."""
    o, l = _f64(o), _f64(l)
    assert len(l) == len(o) + 1
    return lib().ora_csqmi(len(o), _pd(o), _pd(l), float(sigma), int(Delta))


def fsmi_counted(variant, o, l, sigma, counted, Delta=0, H=0, delta_occ=1.5):
    """One beam's MI over the cells with counted[i] true only (cell marking, Sec. 2.4)."""
    o, l = _f64(o), _f64(l)
    assert len(l) == len(o) + 1 and len(counted) == len(o)
    m = np.ascontiguousarray(counted, dtype=np.uint8)
    return lib().ora_fsmi_counted(int(variant), len(o), _pd(o), _pd(l), float(sigma),
                                  float(delta_occ), int(Delta), int(H), _pd(m))


def eval_trajectories_2d(variant, grid, traj_off, poses, beam_dir, sigma, R, Delta=0, H=0,
                         delta_occ=1.5, want_beams=True):
    """Trajectory MI with cell marking (Sec. 2.4): (mi_traj, mi_state, mi_beam)."""
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    Y, X = grid.shape
    traj_off = np.ascontiguousarray(traj_off, dtype=np.int64)
    poses = _f64(poses).reshape(-1, 4)
    beam_dir = _f64(beam_dir).reshape(-1, 2)
    nt, ns, nb = len(traj_off) - 1, poses.shape[0], beam_dir.shape[0]
    assert traj_off[0] == 0 and traj_off[-1] == ns
    mt, ms = np.zeros(nt), np.zeros(ns)
    mb = np.zeros((ns, nb)) if want_beams else None
    rc = lib().ora_eval_trajectories_2d(int(variant), int(Delta), int(H), float(delta_occ),
                                        _pd(grid), X, Y, nt, _pd(traj_off), _pd(poses), nb,
                                        _pd(beam_dir), float(sigma), float(R), _pd(mt), _pd(ms),
                                        None if mb is None else _pd(mb))
    if rc != 0:
        raise ValueError("eval_trajectories_2d: a state lies outside the map")
    return mt, ms, mb
