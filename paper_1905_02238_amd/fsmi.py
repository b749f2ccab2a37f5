"""ctypes binding of libfsmi (include/libfsmi.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors are torch CUDA tensors (device memory owned by the caller);
the binding checks dtype / device / contiguity, allocates outputs with torch
when the caller does not pass them, and enqueues on torch's current stream.
If ``libfsmi.so`` has not been built the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsmi.so")

FSMI_OK, FSMI_E_INVAL, FSMI_E_DEVICE, FSMI_E_NOMEM, FSMI_E_CAPACITY, FSMI_E_NUMERIC, \
    FSMI_E_UNSUPPORTED = range(7)
FSMI_EXACT, FSMI_APPROX, FSMI_UNIFORM, FSMI_CSQMI = 0, 1, 2, 3
FSMI_KERNEL_ERF, FSMI_KERNEL_DENSITY = 0, 1
FSMI_FP32, FSMI_FP64 = 0, 1
FSMI_RAY_DDA, FSMI_RAY_VIRTUAL, FSMI_RAY_RLE = 0, 1, 2
FSMI_PLAN_AUTOTUNE, FSMI_PLAN_GRAPH = 1, 2
FSMI_F_SKIP_ZERO = 1
FSMI_F_MAX_RANGE = 2
FSMI_F_RLE_RUNS, FSMI_F_RLE_CELLS = 4, 8
FSMI_F_LUT = 16
FSMI_PEAK_COPY, FSMI_PEAK_FMA, FSMI_PEAK_PAIR, FSMI_PEAK_MFMA_BF16 = 0, 1, 2, 3

EXPORTS = ("fsmi_create", "fsmi_destroy", "fsmi_set_stream", "fsmi_sync", "fsmi_last_error",
           "fsmi_status_string", "fsmi_default_params", "fsmi_raycast", "fsmi_eval_beams",
           "fsmi_rle_eval_beams", "fsmi_rle_table_eval_beams", "fsmi_eval_poses",
           "fsmi_eval_poses_noalloc", "fsmi_eval_trajectories", "fsmi_probe_erfc", "fsmi_probe_f", "fsmi_probe_mfma", "fsmi_peak",
           "fsmi_sur_num_params", "fsmi_sur_create", "fsmi_sur_destroy",
           "fsmi_sur_fit_label_stats", "fsmi_sur_get_label_stats", "fsmi_sur_forward",
           "fsmi_sur_backward", "fsmi_sur_adam_step", "fsmi_sur_get_params",
           "fsmi_sur_set_params", "fsmi_sur_get_grads", "fsmi_sur_save", "fsmi_sur_load",
           "fsmi_rank_poses", "fsmi_plan_eval_beams", "fsmi_plan_launch", "fsmi_plan_get_info",
           "fsmi_plan_destroy")


class FsmiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfsmi status {status}: {msg}")
        self.status = status


class fsmi_params(C.Structure):
    _fields_ = [("delta_occ", C.c_double), ("variant", C.c_int32), ("trunc_delta", C.c_int32),
                ("uniform_h", C.c_int32), ("kernel", C.c_int32), ("precision", C.c_int32),
                ("flags", C.c_uint32), ("sigma_slope", C.c_double)]


class fsmi_map(C.Structure):
    _fields_ = [("occ", C.c_void_p), ("ndim", C.c_int32), ("dims", C.c_int64 * 3)]


class fsmi_plan_info(C.Structure):
    _fields_ = [("wave_max", C.c_int32), ("max_len", C.c_int32), ("n_tile", C.c_int64),
                ("n_wave", C.c_int64), ("graph", C.c_int32), ("n_tried", C.c_int32),
                ("tried_wave_max", C.c_int32 * 16), ("tried_ms", C.c_float * 16)]


_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH):
    """Loads libfsmi.so (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(f"libfsmi.so not found at {path}: build it with "
                                   "`python -m paper_1905_02238_amd.build` (or __graft_entry__.build())")
            L = C.CDLL(path)
            p, i32, i64, d, st = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int
            L.fsmi_create.argtypes = [C.POINTER(p), C.c_int, p]
            L.fsmi_destroy.argtypes = [p]
            L.fsmi_destroy.restype = None
            L.fsmi_set_stream.argtypes = [p, p]
            L.fsmi_sync.argtypes = [p]
            L.fsmi_last_error.argtypes = [p]
            L.fsmi_last_error.restype = C.c_char_p
            L.fsmi_status_string.argtypes = [st]
            L.fsmi_status_string.restype = C.c_char_p
            L.fsmi_default_params.argtypes = [C.POINTER(fsmi_params)]
            L.fsmi_default_params.restype = None
            L.fsmi_raycast.argtypes = [p, C.POINTER(fsmi_map), i32, i64, p, p, d, d, i32, p, p, p, p, p]
            L.fsmi_eval_beams.argtypes = [p, C.POINTER(fsmi_params), i64, p, p, p, p, p]
            L.fsmi_rle_eval_beams.argtypes = [p, C.POINTER(fsmi_params), i64, p, p, p, p, p]
            L.fsmi_rle_table_eval_beams.argtypes = [p, C.POINTER(fsmi_params), i64, p, p, p, d, i32, p]
            L.fsmi_eval_poses.argtypes = [p, C.POINTER(fsmi_params), C.POINTER(fsmi_map), i64, p,
                                          i64, p, d, d, d, p, p]
            L.fsmi_eval_poses_noalloc.argtypes = L.fsmi_eval_poses.argtypes
            L.fsmi_eval_trajectories.argtypes = [p, C.POINTER(fsmi_params), C.POINTER(fsmi_map),
                                                 i64, p, i64, p, i64, p, d, d, p, p, p]
            L.fsmi_probe_erfc.argtypes = [p, i64, p, p]
            L.fsmi_probe_f.argtypes = [p, d, i64, p, p]
            L.fsmi_peak.argtypes = [p, i32, C.POINTER(d), C.POINTER(d)]
            L.fsmi_probe_mfma.argtypes = [p, p, p, p]
            L.fsmi_sur_num_params.argtypes = []
            L.fsmi_sur_num_params.restype = i64
            L.fsmi_sur_create.argtypes = [p, C.POINTER(p), C.c_uint64, i32, i32]
            L.fsmi_sur_destroy.argtypes = [p]
            L.fsmi_sur_destroy.restype = None
            L.fsmi_sur_fit_label_stats.argtypes = [p, i64, p]
            L.fsmi_sur_get_label_stats.argtypes = [p, p]
            L.fsmi_sur_forward.argtypes = [p, C.POINTER(fsmi_map), i64, p, p]
            L.fsmi_sur_backward.argtypes = [p, C.POINTER(fsmi_map), i64, p, p, p]
            L.fsmi_sur_adam_step.argtypes = [p, C.c_float, C.c_float, C.c_float, C.c_float]
            L.fsmi_sur_get_params.argtypes = [p, p]
            L.fsmi_sur_set_params.argtypes = [p, p]
            L.fsmi_sur_get_grads.argtypes = [p, p]
            L.fsmi_sur_save.argtypes = [p, C.c_char_p]
            L.fsmi_sur_load.argtypes = [p, C.c_char_p]
            L.fsmi_rank_poses.argtypes = [p, C.POINTER(fsmi_params), p, C.POINTER(fsmi_map), i64, p,
                                          i64, p, d, d, i32, p, p, p]
            L.fsmi_plan_eval_beams.argtypes = [p, C.POINTER(fsmi_params), i64, p, p, p, p, p, i32,
                                               C.c_uint32, C.POINTER(p)]
            L.fsmi_plan_launch.argtypes = [p]
            L.fsmi_plan_get_info.argtypes = [p, C.POINTER(fsmi_plan_info)]
            L.fsmi_plan_destroy.argtypes = [p]
            L.fsmi_plan_destroy.restype = None
            for n in ("fsmi_create", "fsmi_set_stream", "fsmi_sync", "fsmi_raycast",
                      "fsmi_eval_beams", "fsmi_rle_eval_beams", "fsmi_rle_table_eval_beams",
                      "fsmi_eval_poses", "fsmi_eval_poses_noalloc",
                      "fsmi_eval_trajectories", "fsmi_probe_erfc", "fsmi_probe_f", "fsmi_probe_mfma", "fsmi_peak", "fsmi_sur_create",
                      "fsmi_sur_fit_label_stats", "fsmi_sur_get_label_stats", "fsmi_sur_forward",
                      "fsmi_sur_backward", "fsmi_sur_adam_step", "fsmi_sur_get_params",
                      "fsmi_sur_set_params", "fsmi_sur_get_grads", "fsmi_sur_save",
                      "fsmi_sur_load", "fsmi_rank_poses", "fsmi_plan_eval_beams",
                      "fsmi_plan_launch", "fsmi_plan_get_info"):
                getattr(L, n).restype = st
            _lib = L
    return _lib


def params(variant=FSMI_EXACT, delta_occ=1.5, trunc_delta=3, uniform_h=0, kernel=FSMI_KERNEL_ERF,
           precision=FSMI_FP32, flags=0, sigma_slope=0.0) -> fsmi_params:
    p = fsmi_params()
    load().fsmi_default_params(C.byref(p))
    p.delta_occ, p.variant, p.trunc_delta, p.uniform_h = delta_occ, variant, trunc_delta, uniform_h
    p.kernel, p.precision, p.flags = kernel, precision, flags
    p.sigma_slope = sigma_slope
    return p


def _ptr(t, dtype, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _map(occ: torch.Tensor) -> fsmi_map:
    m = fsmi_map()
    m.occ = _ptr(occ, torch.float32, "map").value
    if occ.dim() == 2:
        m.ndim = 2
        m.dims[0], m.dims[1], m.dims[2] = occ.shape[1], occ.shape[0], 1
    elif occ.dim() == 3:
        m.ndim = 3
        m.dims[0], m.dims[1], m.dims[2] = occ.shape[2], occ.shape[1], occ.shape[0]
    else:
        raise ValueError("map must be [Y][X] or [Z][Y][X]")
    return m


class Context:
    """An fsmi_ctx bound to one device; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = device
        self._lib = load()
        h = C.c_void_p()
        with torch.cuda.device(device):
            s = torch.cuda.current_stream(device).cuda_stream
            self._check(self._lib.fsmi_create(C.byref(h), device, C.c_void_p(s)), None)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self._lib.fsmi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, h=None):
        if st != FSMI_OK:
            L = self._lib
            msg = L.fsmi_last_error(h or self.handle).decode() if (h or getattr(self, "handle", None)) \
                else L.fsmi_status_string(st).decode()
            raise FsmiError(st, msg or L.fsmi_status_string(st).decode())

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._check(self._lib.fsmi_set_stream(self.handle, C.c_void_p(s)))

    # --- C-ABI entry points -------------------------------------------------
    def fsmi_sync(self):
        self._check(self._lib.fsmi_sync(self.handle))

    def fsmi_raycast(self, map_occ, mode, origin, direction, max_range, w=1.0, max_cells=None,
                     count=None, cell=None, entry=None, occ_out=None, run_len=None):
        n = origin.shape[0]
        dev = map_occ.device
        if max_cells is None:
            if mode == FSMI_RAY_DDA:
                max_cells = int(1.4142135623730951 * max_range) + 3
            else:
                max_cells = int(max_range / w)
        count = torch.empty(n, dtype=torch.int32, device=dev) if count is None else count
        cell = torch.empty((n, max_cells), dtype=torch.int32, device=dev) if cell is None else cell
        if mode == FSMI_RAY_DDA and entry is None:
            entry = torch.empty((n, max_cells + 1), dtype=torch.float64, device=dev)
        occ_out = torch.empty((n, max_cells), dtype=torch.float32, device=dev) if occ_out is None else occ_out
        if mode == FSMI_RAY_RLE and run_len is None:
            run_len = torch.empty((n, max_cells), dtype=torch.int32, device=dev)
        m = _map(map_occ)
        self._stream()
        self._check(self._lib.fsmi_raycast(
            self.handle, C.byref(m), mode, n, _ptr(origin, torch.float64, "origin"),
            _ptr(direction, torch.float64, "dir"), float(max_range), float(w), int(max_cells),
            _ptr(count, torch.int32, "count"), _ptr(cell, torch.int32, "cell"),
            _ptr(entry, torch.float64, "entry", True), _ptr(occ_out, torch.float32, "occ_out", True),
            _ptr(run_len, torch.int32, "run_len", True)))
        return dict(count=count, cell=cell, entry=entry, occ=occ_out, run_len=run_len)

    def fsmi_eval_beams(self, prm: fsmi_params, off, occ, sigma, bound=None, mi=None):
        n = off.shape[0] - 1
        mi = torch.empty(n, dtype=torch.float64, device=occ.device) if mi is None else mi
        self._stream()
        self._check(self._lib.fsmi_eval_beams(
            self.handle, C.byref(prm), n, _ptr(off, torch.int64, "off"),
            _ptr(occ, torch.float32, "occ"), _ptr(bound, torch.float64, "bound", True),
            _ptr(sigma, torch.float32, "sigma"), _ptr(mi, torch.float64, "mi")))
        return mi

    def fsmi_rle_eval_beams(self, prm: fsmi_params, run_off, run_occ, run_len, sigma_prime, mi=None):
        n = run_off.shape[0] - 1
        mi = torch.empty(n, dtype=torch.float64, device=run_occ.device) if mi is None else mi
        self._stream()
        self._check(self._lib.fsmi_rle_eval_beams(
            self.handle, C.byref(prm), n, _ptr(run_off, torch.int64, "run_off"),
            _ptr(run_occ, torch.float32, "run_occ"), _ptr(run_len, torch.int32, "run_len"),
            _ptr(sigma_prime, torch.float32, "sigma_prime"), _ptr(mi, torch.float64, "mi")))
        return mi

    def fsmi_rle_table_eval_beams(self, prm: fsmi_params, run_off, run_occ, run_len, sigma_prime,
                                  levels, mi=None):
        n = run_off.shape[0] - 1
        mi = torch.empty(n, dtype=torch.float64, device=run_occ.device) if mi is None else mi
        self._stream()
        self._check(self._lib.fsmi_rle_table_eval_beams(
            self.handle, C.byref(prm), n, _ptr(run_off, torch.int64, "run_off"),
            _ptr(run_occ, torch.float32, "run_occ"), _ptr(run_len, torch.int32, "run_len"),
            float(sigma_prime), int(levels), _ptr(mi, torch.float64, "mi")))
        return mi

    def fsmi_eval_poses(self, prm: fsmi_params, map_occ, poses, beam_dir, sigma, max_range, w=1.0,
                        mi_pose=None, mi_beam=None, want_beams=False, _entry="fsmi_eval_poses"):
        npo, nb = poses.shape[0], beam_dir.shape[0]
        dev = map_occ.device
        mi_pose = torch.empty(npo, dtype=torch.float64, device=dev) if mi_pose is None else mi_pose
        if want_beams and mi_beam is None:
            mi_beam = torch.empty((npo, nb), dtype=torch.float64, device=dev)
        m = _map(map_occ)
        self._stream()
        self._check(getattr(self._lib, _entry)(
            self.handle, C.byref(prm), C.byref(m), npo, _ptr(poses, torch.float64, "poses"), nb,
            _ptr(beam_dir, torch.float64, "beam_dir"), float(sigma), float(max_range), float(w),
            _ptr(mi_pose, torch.float64, "mi_pose"), _ptr(mi_beam, torch.float64, "mi_beam", True)))
        return mi_pose, mi_beam

    def fsmi_eval_poses_noalloc(self, prm: fsmi_params, map_occ, poses, beam_dir, sigma,
                                max_range, w=1.0, mi_pose=None, mi_beam=None, want_beams=False):
        """fsmi_eval_poses with the library's static scratch: no device allocation
        by the call (outputs are still the caller's; pass them to allocate nothing here)."""
        return self.fsmi_eval_poses(prm, map_occ, poses, beam_dir, sigma, max_range, w, mi_pose,
                                    mi_beam, want_beams, _entry="fsmi_eval_poses_noalloc")

    def fsmi_eval_trajectories(self, prm: fsmi_params, map_occ, traj_off, poses, beam_dir, sigma,
                               max_range, want_states=True, want_beams=False):
        """Trajectory MI with cell marking: (mi_traj, mi_state or None, mi_beam or None)."""
        nt, ns, nb = traj_off.shape[0] - 1, poses.shape[0], beam_dir.shape[0]
        dev = map_occ.device
        mt = torch.empty(nt, dtype=torch.float64, device=dev)
        ms = torch.empty(ns, dtype=torch.float64, device=dev) if want_states else None
        mb = torch.empty((ns, nb), dtype=torch.float64, device=dev) if want_beams else None
        m = _map(map_occ)
        self._stream()
        self._check(self._lib.fsmi_eval_trajectories(
            self.handle, C.byref(prm), C.byref(m), nt, _ptr(traj_off, torch.int64, "traj_off"), ns,
            _ptr(poses, torch.float64, "poses"), nb, _ptr(beam_dir, torch.float64, "beam_dir"),
            float(sigma), float(max_range), _ptr(mt, torch.float64, "mi_traj"),
            _ptr(ms, torch.float64, "mi_state", True), _ptr(mb, torch.float64, "mi_beam", True)))
        return mt, ms, mb

    def fsmi_probe_erfc(self, z, out=None):
        out = torch.empty_like(z) if out is None else out
        self._stream()
        self._check(self._lib.fsmi_probe_erfc(self.handle, z.numel(), _ptr(z, torch.float32, "z"),
                                              _ptr(out, torch.float32, "out")))
        return out

    def fsmi_probe_f(self, delta, o):
        out = torch.empty(o.shape, dtype=torch.float64, device=o.device)
        self._stream()
        self._check(self._lib.fsmi_probe_f(self.handle, float(delta), o.numel(),
                                           _ptr(o, torch.float32, "o"),
                                           _ptr(out, torch.float64, "out")))
        return out

    def fsmi_peak(self, kind, with_clock=False):
        r, mhz = C.c_double(0.0), C.c_double(0.0)
        self._stream()
        self._check(self._lib.fsmi_peak(self.handle, int(kind), C.byref(r), C.byref(mhz)))
        return (r.value, mhz.value) if with_clock else r.value

    def fsmi_probe_mfma(self, A, B):
        D = torch.empty((16, 16), dtype=torch.float32, device=A.device)
        self._stream()
        self._check(self._lib.fsmi_probe_mfma(self.handle, _ptr(A, torch.bfloat16, "A"),
                                              _ptr(B, torch.bfloat16, "B"),
                                              _ptr(D, torch.float32, "D")))
        return D

    def fsmi_rank_poses(self, prm: fsmi_params, net: "Surrogate", map_occ, poses, beam_dir, sigma,
                        max_range, k, want_pred=False):
        dev = map_occ.device
        idx = torch.empty(k, dtype=torch.int32, device=dev)
        mi = torch.empty(k, dtype=torch.float64, device=dev)
        pred = torch.empty(poses.shape[0], dtype=torch.float32, device=dev) if want_pred else None
        m = _map(map_occ)
        self._stream()
        self._check(self._lib.fsmi_rank_poses(
            self.handle, C.byref(prm), net.handle, C.byref(m), poses.shape[0],
            _ptr(poses, torch.float64, "poses"), beam_dir.shape[0],
            _ptr(beam_dir, torch.float64, "beam_dir"), float(sigma), float(max_range), int(k),
            _ptr(idx, torch.int32, "idx"), _ptr(mi, torch.float64, "mi"),
            _ptr(pred, torch.float32, "pred", True)))
        return idx, mi, pred


class Plan:
    """fsmi_plan: a beam batch bound to its buffers, scheduled once (optionally
    autotuned and captured into a HIP graph); launch() enqueues one evaluation
    that re-reads occ / bound / sigma and rewrites mi."""

    def __init__(self, ctx: Context, prm: fsmi_params, off, occ, sigma, bound=None, mi=None,
                 wave_max=0, autotune=False, graph=False):
        self.ctx = ctx
        self._lib = ctx._lib
        n = off.shape[0] - 1
        self.mi = torch.empty(n, dtype=torch.float64, device=occ.device) if mi is None else mi
        # keep the bound tensors alive for the plan's lifetime
        self._keep = (off, occ, sigma, bound, self.mi)
        flags = (FSMI_PLAN_AUTOTUNE if autotune else 0) | (FSMI_PLAN_GRAPH if graph else 0)
        h = C.c_void_p()
        ctx._stream()
        ctx._check(self._lib.fsmi_plan_eval_beams(
            ctx.handle, C.byref(prm), n, _ptr(off, torch.int64, "off"),
            _ptr(occ, torch.float32, "occ"), _ptr(bound, torch.float64, "bound", True),
            _ptr(sigma, torch.float32, "sigma"), _ptr(self.mi, torch.float64, "mi"),
            int(wave_max), flags, C.byref(h)))
        self.handle = h

    def launch(self):
        self.ctx._stream()
        self.ctx._check(self._lib.fsmi_plan_launch(self.handle))
        return self.mi

    def info(self) -> dict:
        i = fsmi_plan_info()
        self.ctx._check(self._lib.fsmi_plan_get_info(self.handle, C.byref(i)))
        return {"wave_max": i.wave_max, "max_len": i.max_len, "n_tile": i.n_tile,
                "n_wave": i.n_wave, "graph": bool(i.graph),
                "tried": [(i.tried_wave_max[k], i.tried_ms[k]) for k in range(i.n_tried)]}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.fsmi_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """fsmi_sur: the conv-net surrogate (created on a Context's device and stream)."""

    def __init__(self, ctx: Context, seed: int = 0, max_batch: int = 256, patch_stride: int = 1):
        self.ctx = ctx
        self._lib = ctx._lib
        h = C.c_void_p()
        ctx._stream()
        ctx._check(self._lib.fsmi_sur_create(ctx.handle, C.byref(h), C.c_uint64(seed),
                                             int(max_batch), int(patch_stride)))
        self.handle = h
        self.max_batch = max_batch
        self.num_params = int(self._lib.fsmi_sur_num_params())

    def close(self):
        if getattr(self, "handle", None):
            self._lib.fsmi_sur_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != FSMI_OK:
            raise FsmiError(st, self._lib.fsmi_status_string(st).decode())

    def fit_label_stats(self, labels):
        self.ctx._stream()
        self._chk(self._lib.fsmi_sur_fit_label_stats(self.handle, labels.numel(),
                                                     _ptr(labels, torch.float64, "labels")))

    def label_stats(self):
        """(mean, scale, emean, escale) of the fitted labels."""
        out = (C.c_double * 4)()
        self._chk(self._lib.fsmi_sur_get_label_stats(self.handle, C.cast(out, C.c_void_p)))
        return tuple(float(v) for v in out)

    def forward(self, map_occ, poses, pred=None):
        self.ctx._stream()
        pred = torch.empty(poses.shape[0], dtype=torch.float32, device=poses.device) if pred is None else pred
        m = _map(map_occ)
        self._chk(self._lib.fsmi_sur_forward(self.handle, C.byref(m), poses.shape[0],
                                             _ptr(poses, torch.float64, "poses"),
                                             _ptr(pred, torch.float32, "pred")))
        return pred

    def backward(self, map_occ, poses, labels, loss=None):
        self.ctx._stream()
        loss = torch.empty(1, dtype=torch.float32, device=poses.device) if loss is None else loss
        m = _map(map_occ)
        self._chk(self._lib.fsmi_sur_backward(self.handle, C.byref(m), poses.shape[0],
                                              _ptr(poses, torch.float64, "poses"),
                                              _ptr(labels, torch.float64, "labels"),
                                              _ptr(loss, torch.float32, "loss")))
        return loss

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.ctx._stream()
        self._chk(self._lib.fsmi_sur_adam_step(self.handle, lr, b1, b2, eps))

    def params(self):
        self.ctx._stream()
        out = torch.empty(self.num_params, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        self._chk(self._lib.fsmi_sur_get_params(self.handle, _ptr(out, torch.float32, "params")))
        return out

    def set_params(self, p):
        self.ctx._stream()
        self._chk(self._lib.fsmi_sur_set_params(self.handle, _ptr(p, torch.float32, "params")))

    def grads(self):
        self.ctx._stream()
        out = torch.empty(self.num_params, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        self._chk(self._lib.fsmi_sur_get_grads(self.handle, _ptr(out, torch.float32, "grads")))
        return out

    def save(self, path):
        self.ctx._stream()
        self._chk(self._lib.fsmi_sur_save(self.handle, str(path).encode()))

    def load(self, path):
        self.ctx._stream()
        self._chk(self._lib.fsmi_sur_load(self.handle, str(path).encode()))


_ctx = {}


def context(device: int = 0) -> Context:
    """A cached Context per device."""
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]
