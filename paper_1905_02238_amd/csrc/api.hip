// api.hip -- the C-ABI of libfsmi (include/libfsmi.h): contexts, argument
// validation, error latching, and dispatch to the kernel launchers.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "fsmi_dev.h"
#include "fsmi_internal.h"

using namespace fsmi;

namespace fsmi {

fsmi_status fail(fsmi_ctx ctx, fsmi_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

fsmi_status from_hip(fsmi_ctx ctx, hipError_t e, const char* where) {
  if (e == hipSuccess) return FSMI_OK;
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory) return fail(ctx, FSMI_E_NOMEM, m);
  if (e == hipErrorInvalidValue) return fail(ctx, FSMI_E_CAPACITY, m + " (launch does not fit)");
  return fail(ctx, FSMI_E_DEVICE, m);
}

bool check_params(fsmi_ctx ctx, const fsmi_params* p, fsmi_status* st) {
  if (!p) {
    *st = fail(ctx, FSMI_E_INVAL, "params is NULL");
    return false;
  }
  if (!(p->delta_occ > 1.0) || !std::isfinite(p->delta_occ)) {
    *st = fail(ctx, FSMI_E_INVAL, "delta_occ must be finite and > 1");
    return false;
  }
  if (p->variant < FSMI_EXACT || p->variant > FSMI_CSQMI) {
    *st = fail(ctx, FSMI_E_INVAL, "unknown variant");
    return false;
  }
  if ((p->variant == FSMI_APPROX || p->variant == FSMI_CSQMI) && p->trunc_delta < 0) {
    *st = fail(ctx, FSMI_E_INVAL, "trunc_delta must be >= 0");
    return false;
  }
  if (p->variant == FSMI_UNIFORM && p->uniform_h < 0) {
    *st = fail(ctx, FSMI_E_INVAL, "uniform_h must be >= 0");
    return false;
  }
  if (p->kernel != FSMI_KERNEL_ERF && p->kernel != FSMI_KERNEL_DENSITY) {
    *st = fail(ctx, FSMI_E_INVAL, "unknown kernel");
    return false;
  }
  if (p->precision != FSMI_FP32 && p->precision != FSMI_FP64) {
    *st = fail(ctx, FSMI_E_INVAL, "unknown precision");
    return false;
  }
  if (p->flags & ~(uint32_t)(FSMI_F_SKIP_ZERO | FSMI_F_MAX_RANGE | FSMI_F_RLE_RUNS | FSMI_F_RLE_CELLS |
                             FSMI_F_LUT)) {
    *st = fail(ctx, FSMI_E_INVAL, "unknown flags");
    return false;
  }
  if ((p->flags & FSMI_F_LUT) &&
      (p->flags != FSMI_F_LUT || p->precision != FSMI_FP32 || p->sigma_slope != 0.0 ||
       (p->variant != FSMI_EXACT && p->variant != FSMI_APPROX))) {
    *st = fail(ctx, FSMI_E_INVAL, "FSMI_F_LUT goes alone, with FP32 EXACT or APPROX and one sigma");
    return false;
  }
  if ((p->flags & (FSMI_F_RLE_RUNS | FSMI_F_RLE_CELLS)) &&
      (p->flags != FSMI_F_RLE_RUNS && p->flags != FSMI_F_RLE_CELLS)) {
    *st = fail(ctx, FSMI_E_INVAL, "FSMI_F_RLE_RUNS and FSMI_F_RLE_CELLS go alone");
    return false;
  }
  if (!(p->sigma_slope >= 0.0) || !std::isfinite(p->sigma_slope)) {
    *st = fail(ctx, FSMI_E_INVAL, "sigma_slope must be finite and >= 0");
    return false;
  }
  if ((p->sigma_slope != 0.0 || (p->flags & FSMI_F_MAX_RANGE)) &&
      (p->variant != FSMI_EXACT || (p->flags & FSMI_F_SKIP_ZERO))) {
    *st = fail(ctx, FSMI_E_INVAL, "sigma_slope and FSMI_F_MAX_RANGE are EXACT (not skip-zero) modes");
    return false;
  }
  if (p->variant == FSMI_CSQMI && (p->flags != 0 || p->sigma_slope != 0.0)) {
    *st = fail(ctx, FSMI_E_INVAL, "FSMI_CSQMI takes no flags and no sigma_slope");
    return false;
  }
  if ((p->flags & (FSMI_F_RLE_RUNS | FSMI_F_RLE_CELLS)) && p->variant == FSMI_UNIFORM) {
    *st = fail(ctx, FSMI_E_INVAL, "Uniform-FSMI-RLE has one engine (the expanded cells)");
    return false;
  }
  if ((p->flags & FSMI_F_SKIP_ZERO) && (p->variant != FSMI_EXACT || p->precision != FSMI_FP32)) {
    *st = fail(ctx, FSMI_E_INVAL, "FSMI_F_SKIP_ZERO is an EXACT, FP32 mode");
    return false;
  }
  return true;
}

bool ext_mode(const fsmi_params* p) {
  return p->sigma_slope != 0.0 || (p->flags & FSMI_F_MAX_RANGE);
}

EvalConst to_const(const fsmi_params* p) {
  EvalConst ec;
  ec.variant = p->variant;
  ec.Delta = p->trunc_delta;
  ec.H = p->uniform_h;
  ec.kernel = p->kernel;
  ec.precision = p->precision;
  ec.flags = p->flags;
  ec.delta_occ = p->delta_occ;
  ec.slope = p->sigma_slope;
  return ec;
}

bool check_map(fsmi_ctx ctx, const fsmi_map* m, fsmi_status* st) {
  if (!m || !m->occ) {
    *st = fail(ctx, FSMI_E_INVAL, "map or map->occ is NULL");
    return false;
  }
  if (m->ndim != 2 && m->ndim != 3) {
    *st = fail(ctx, FSMI_E_INVAL, "map ndim must be 2 or 3");
    return false;
  }
  int64_t cells = 1;
  for (int i = 0; i < m->ndim; ++i) {
    if (m->dims[i] <= 0) {
      *st = fail(ctx, FSMI_E_INVAL, "map dims must be positive");
      return false;
    }
    cells *= m->dims[i];
    if (cells >= (int64_t)1 << 31) {
      *st = fail(ctx, FSMI_E_CAPACITY, "map has 2^31 cells or more");
      return false;
    }
  }
  return true;
}

int ctx_wave_max(fsmi_ctx ctx, const fsmi_params* p, bool has_bound) {
  const int t = ctx->tuned_wave_max[p->precision == FSMI_FP64][p->variant][has_bound ? 1 : 0];
  return t > 0 ? t : beam_default_wave_max(p->precision);
}

hipError_t ensure_work(fsmi_ctx ctx, size_t bytes) {
  if (bytes <= ctx->work_bytes) return hipSuccess;
  if (ctx->d_work) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    (void)hipFree(ctx->d_work);
    ctx->d_work = nullptr;
    ctx->work_bytes = 0;
  }
  size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes + bytes / 4;
  hipError_t e = hipMalloc(&ctx->d_work, want);
  if (e != hipSuccess) return e;
  ctx->work_bytes = want;
  return hipSuccess;
}
}  // namespace fsmi

extern "C" {

const char* fsmi_status_string(fsmi_status s) {
  switch (s) {
    case FSMI_OK: return "ok";
    case FSMI_E_INVAL: return "invalid argument";
    case FSMI_E_DEVICE: return "device error";
    case FSMI_E_NOMEM: return "out of device memory";
    case FSMI_E_CAPACITY: return "capacity exceeded";
    case FSMI_E_NUMERIC: return "invalid data found on the device";
    case FSMI_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

void fsmi_default_params(fsmi_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->delta_occ = 1.5;
  p->variant = FSMI_EXACT;
  p->trunc_delta = 3;
  p->uniform_h = 0;
  p->kernel = FSMI_KERNEL_ERF;
  p->precision = FSMI_FP32;
  p->flags = 0;
  p->sigma_slope = 0.0;
}

fsmi_status fsmi_create(fsmi_ctx* out, int device, void* hip_stream) {
  if (!out) return FSMI_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FSMI_E_DEVICE;
  if (device < 0 || device >= ndev) return FSMI_E_INVAL;
  fsmi_ctx c = new (std::nothrow) fsmi_ctx_s();
  if (!c) return FSMI_E_NOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return FSMI_E_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cu = prop.multiProcessorCount;
  c->stream = (hipStream_t)hip_stream;   // NULL: the device's default stream
  // the device address of fsmi_eval_poses_noalloc's static scratch on this device
  if (noalloc_scratch_init(device) != hipSuccess) {
    delete c;
    return FSMI_E_DEVICE;
  }
  if (hipMalloc(&c->d_status, 256) != hipSuccess || hipMalloc(&c->d_counters, 64 * 4) != hipSuccess ||
      hipMalloc(&c->d_lut, lut_bytes()) != hipSuccess) {
    if (c->d_status) (void)hipFree(c->d_status);
    if (c->d_counters) (void)hipFree(c->d_counters);
    delete c;
    return FSMI_E_NOMEM;
  }
  if (hipEventCreateWithFlags(&c->handoff, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(c->d_status);
    (void)hipFree(c->d_counters);
    (void)hipFree(c->d_lut);
    delete c;
    return FSMI_E_DEVICE;
  }
  (void)hipMemset(c->d_status, 0, 256);
  (void)hipMemset(c->d_counters, 0, 64 * 4);
  (void)hipDeviceSynchronize();
  *out = c;
  return FSMI_OK;
}

void fsmi_destroy(fsmi_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->d_work) (void)hipFree(ctx->d_work);
  if (ctx->d_lut) (void)hipFree(ctx->d_lut);
  if (ctx->d_status) (void)hipFree(ctx->d_status);
  if (ctx->d_counters) (void)hipFree(ctx->d_counters);
  if (ctx->handoff) (void)hipEventDestroy(ctx->handoff);
  delete ctx;
}

fsmi_status fsmi_set_stream(fsmi_ctx ctx, void* hip_stream) {
  if (!ctx) return FSMI_E_INVAL;
  const hipStream_t s = (hipStream_t)hip_stream;   // NULL: the device's default stream
  if (s == ctx->stream) return FSMI_OK;
  // the new stream waits for everything enqueued so far on the old one, so
  // calls on the two streams never share the context's scratch at once
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipEventRecord(ctx->handoff, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->handoff, 0);
  if (e != hipSuccess) return from_hip(ctx, e, "fsmi_set_stream");
  ctx->stream = s;
  return FSMI_OK;
}

fsmi_status fsmi_sync(fsmi_ctx ctx) {
  if (!ctx) return FSMI_E_INVAL;
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return from_hip(ctx, e, "fsmi_sync");
  uint32_t st = 0;
  e = hipMemcpy(&st, ctx->d_status, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return from_hip(ctx, e, "fsmi_sync status read");
  if (st) {
    uint32_t zero = 0;
    (void)hipMemcpy(ctx->d_status, &zero, 4, hipMemcpyHostToDevice);
    std::string m = "device data error:";
    if (st & kErrOcc) m += " occupancy outside [0,1] or NaN, or bad sigma/boundaries;";
    if (st & kErrLen) m += " bad beam/run length;";
    if (st & kErrPose) m += " pose or origin outside the map;";
    if (st & kErrCap) m += " beam longer than the launch capacity;";
    if (st & kErrBound) m += " decreasing boundaries;";
    return fail(ctx, (st & kErrCap) ? FSMI_E_CAPACITY : FSMI_E_NUMERIC, m);
  }
  return FSMI_OK;
}

const char* fsmi_last_error(fsmi_ctx ctx) {
  if (!ctx) return "no context";
  return ctx->last_error.c_str();
}

fsmi_status fsmi_raycast(fsmi_ctx ctx, const fsmi_map* map, int32_t mode, int64_t n_rays,
                         const double* origin, const double* dir, double max_range, double w,
                         int32_t max_cells, int32_t* count, int32_t* cell, double* entry,
                         float* occ_out, int32_t* run_len) {
  if (!ctx) return FSMI_E_INVAL;
  fsmi_status st;
  if (!check_map(ctx, map, &st)) return st;
  if (n_rays < 0) return fail(ctx, FSMI_E_INVAL, "n_rays < 0");
  if (n_rays == 0) return FSMI_OK;
  if (!origin || !dir || !count) return fail(ctx, FSMI_E_INVAL, "origin, dir and count are required");
  if (!(max_range > 0.0) || !std::isfinite(max_range))
    return fail(ctx, FSMI_E_INVAL, "max_range must be finite and > 0");
  (void)hipSetDevice(ctx->device);
  if (mode == FSMI_RAY_DDA) {
    if (map->ndim != 2) return fail(ctx, FSMI_E_INVAL, "FSMI_RAY_DDA needs a 2D map");
    if ((cell == nullptr) != (entry == nullptr))
      return fail(ctx, FSMI_E_INVAL, "cell and entry are both given or both NULL (count only)");
    const double bound = floor(1.4142135623730951 * max_range) + 3;
    if ((double)max_cells < bound)
      return fail(ctx, FSMI_E_CAPACITY, "max_cells < floor(sqrt(2) * max_range) + 3");
    if (max_range > 8000.0) return fail(ctx, FSMI_E_CAPACITY, "max_range above 8000 cells");
    return from_hip(ctx,
                    launch_raycast2d(ctx, map->occ, map->dims[0], map->dims[1], n_rays, origin, dir,
                                     max_range, max_cells, count, cell, entry, occ_out),
                    "raycast2d");
  }
  if (mode == FSMI_RAY_VIRTUAL || mode == FSMI_RAY_RLE) {
    if (map->ndim != 3) return fail(ctx, FSMI_E_INVAL, "virtual cells need a 3D map");
    if (!(w > 0.0) || !std::isfinite(w)) return fail(ctx, FSMI_E_INVAL, "w must be finite and > 0");
    if ((double)max_cells < floor(max_range / w))
      return fail(ctx, FSMI_E_CAPACITY, "max_cells < floor(max_range / w)");
    if (max_cells > 7000) return fail(ctx, FSMI_E_CAPACITY, "more than 7000 virtual cells per ray");
    if (mode == FSMI_RAY_RLE && !run_len) return fail(ctx, FSMI_E_INVAL, "run_len is required");
    return from_hip(ctx,
                    launch_virtual3d(ctx, map->occ, map->dims[0], map->dims[1], map->dims[2], n_rays,
                                     origin, dir, max_range, w, max_cells, mode == FSMI_RAY_RLE,
                                     count, cell, occ_out, run_len),
                    "virtual3d");
  }
  return fail(ctx, FSMI_E_INVAL, "unknown ray mode");
}

fsmi_status fsmi_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                            const int64_t* off, const float* occ, const double* bound,
                            const float* sigma, double* mi) {
  if (!ctx) return FSMI_E_INVAL;
  fsmi_status st;
  if (!check_params(ctx, params, &st)) return st;
  if (n_beams < 0) return fail(ctx, FSMI_E_INVAL, "n_beams < 0");
  if (n_beams == 0) return FSMI_OK;
  if (n_beams >= ((int64_t)1 << 31)) return fail(ctx, FSMI_E_CAPACITY, "n_beams >= 2^31");
  if (!off || !occ || !sigma || !mi) return fail(ctx, FSMI_E_INVAL, "off, occ, sigma, mi are required");
  if ((params->flags & FSMI_F_SKIP_ZERO) && !bound)
    return fail(ctx, FSMI_E_INVAL, "FSMI_F_SKIP_ZERO needs explicit boundaries");
  if (params->flags & (FSMI_F_RLE_RUNS | FSMI_F_RLE_CELLS))
    return fail(ctx, FSMI_E_INVAL, "FSMI_F_RLE_* select the engine of the RLE paths");
  if (params->flags & FSMI_F_LUT)
    return fail(ctx, FSMI_E_UNSUPPORTED, "FSMI_F_LUT is implemented on 2D fsmi_eval_poses");
  if (ext_mode(params) && !bound)
    return fail(ctx, FSMI_E_INVAL, "sigma_slope and FSMI_F_MAX_RANGE need explicit boundaries");
  (void)hipSetDevice(ctx->device);
  int max_len = 0;
  hipError_t e = launch_max_len(ctx, off, n_beams, &max_len);
  if (e != hipSuccess) return from_hip(ctx, e, "eval_beams max length");
  const int wave_max = ctx_wave_max(ctx, params, bound != nullptr);
  if (!beam_fits(params->precision, wave_max, max_len))
    return fail(ctx, FSMI_E_CAPACITY, "a beam is longer than one workgroup's LDS holds");
  return from_hip(ctx,
                  launch_eval_beams(ctx, to_const(params), n_beams, off, occ, bound, sigma, mi,
                                    max_len, wave_max),
                  "eval_beams");
}

fsmi_status fsmi_rle_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                                const int64_t* run_off, const float* run_occ,
                                const int32_t* run_len, const float* sigma_prime, double* mi) {
  if (!ctx) return FSMI_E_INVAL;
  fsmi_status st;
  if (!check_params(ctx, params, &st)) return st;
  if (n_beams < 0) return fail(ctx, FSMI_E_INVAL, "n_beams < 0");
  if (n_beams == 0) return FSMI_OK;
  if (!run_off || !run_occ || !run_len || !sigma_prime || !mi)
    return fail(ctx, FSMI_E_INVAL, "run_off, run_occ, run_len, sigma_prime, mi are required");
  if (params->flags & FSMI_F_SKIP_ZERO)
    return fail(ctx, FSMI_E_INVAL, "FSMI_F_SKIP_ZERO needs explicit boundaries");
  if (ext_mode(params))
    return fail(ctx, FSMI_E_INVAL, "sigma_slope and FSMI_F_MAX_RANGE need explicit boundaries");
  if (params->variant == FSMI_CSQMI)
    return fail(ctx, FSMI_E_INVAL, "FSMI_CSQMI is a 2D path (fsmi_eval_beams, 2D poses)");
  if (params->flags & FSMI_F_LUT)
    return fail(ctx, FSMI_E_UNSUPPORTED, "FSMI_F_LUT is implemented on 2D fsmi_eval_poses");
  (void)hipSetDevice(ctx->device);
  return from_hip(ctx,
                  launch_rle_eval_beams(ctx, to_const(params), n_beams, run_off, run_occ, run_len,
                                        sigma_prime, mi, 0),
                  "rle_eval_beams");
}

fsmi_status fsmi_rle_table_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                                      const int64_t* run_off, const float* run_occ,
                                      const int32_t* run_len, double sigma_prime,
                                      int32_t levels, double* mi) {
  if (!ctx) return FSMI_E_INVAL;
  fsmi_status st;
  if (!check_params(ctx, params, &st)) return st;
  if (params->variant != FSMI_APPROX)
    return fail(ctx, FSMI_E_INVAL, "the table route is Approx-FSMI-RLE: variant FSMI_APPROX");
  if (params->precision != FSMI_FP64) return fail(ctx, FSMI_E_INVAL, "the table route runs in FP64");
  if (params->flags != 0 || ext_mode(params))
    return fail(ctx, FSMI_E_INVAL, "the table route takes no flags and no sigma_slope");
  if (params->trunc_delta < 0 || params->trunc_delta > 8)
    return fail(ctx, FSMI_E_INVAL, "the table route needs 0 <= trunc_delta <= 8");
  if (levels < 1 || levels > 1024 || (levels & (levels - 1)) != 0)
    return fail(ctx, FSMI_E_INVAL, "levels must be a power of two in [1, 1024]");
  if (!(sigma_prime > 0.0) || !std::isfinite(sigma_prime))
    return fail(ctx, FSMI_E_INVAL, "sigma_prime must be finite and > 0");
  if (n_beams < 0) return fail(ctx, FSMI_E_INVAL, "n_beams < 0");
  if (n_beams == 0) return FSMI_OK;
  if (!run_off || !run_occ || !run_len || !mi)
    return fail(ctx, FSMI_E_INVAL, "run_off, run_occ, run_len, mi are required");
  (void)hipSetDevice(ctx->device);
  return from_hip(ctx,
                  launch_rle_table(ctx, params->delta_occ, params->trunc_delta, levels, sigma_prime,
                                   n_beams, run_off, run_occ, run_len, mi),
                  "rle_table_eval_beams");
}

fsmi_status fsmi_eval_poses(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                            int64_t n_poses, const double* poses, int64_t n_beams,
                            const double* beam_dir, double sigma, double max_range, double w,
                            double* mi_pose, double* mi_beam) {
  return eval_poses_checked(ctx, params, map, n_poses, poses, n_beams, beam_dir, sigma, max_range,
                            w, mi_pose, mi_beam, nullptr);
}

}  // extern "C"

namespace fsmi {
fsmi_status eval_poses_checked(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                               int64_t n_poses, const double* poses, int64_t n_beams,
                               const double* beam_dir, double sigma, double max_range, double w,
                               double* mi_pose, double* mi_beam, const PoseScratch* ws) {
  if (!ctx) return FSMI_E_INVAL;
  fsmi_status st;
  if (!check_params(ctx, params, &st)) return st;
  if (!check_map(ctx, map, &st)) return st;
  if (n_poses < 0 || n_beams < 0) return fail(ctx, FSMI_E_INVAL, "negative count");
  if (n_poses == 0 || n_beams == 0) {
    if (n_poses > 0 && mi_pose) {
      (void)hipSetDevice(ctx->device);
      return from_hip(ctx, launch_fill_f64(ctx->stream, n_poses, 0.0, mi_pose), "zero poses");
    }
    return FSMI_OK;
  }
  if (!poses || !beam_dir || !mi_pose) return fail(ctx, FSMI_E_INVAL, "poses, beam_dir, mi_pose are required");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(ctx, FSMI_E_INVAL, "sigma must be finite and > 0");
  if (!(max_range > 0.0) || !std::isfinite(max_range))
    return fail(ctx, FSMI_E_INVAL, "max_range must be finite and > 0");
  if (n_poses > ((int64_t)1 << 40) / std::max<int64_t>(n_beams, 1))
    return fail(ctx, FSMI_E_CAPACITY, "too many items");
  (void)hipSetDevice(ctx->device);
  if (map->ndim == 2) {
    // one wave holds a beam's walk, boundaries and occupancies in LDS
    if (max_range > 4000.0) return fail(ctx, FSMI_E_CAPACITY, "max_range above 4000 cells");
    if (params->precision == FSMI_FP64 && max_range >= 3873.0)
      return fail(ctx, FSMI_E_CAPACITY, "max_range above 3872 cells in FP64");
    if (params->flags & (FSMI_F_RLE_RUNS | FSMI_F_RLE_CELLS))
      return fail(ctx, FSMI_E_INVAL, "FSMI_F_RLE_* select the engine of the RLE paths (3D maps)");
    return from_hip(ctx,
                    launch_eval_poses_2d(ctx, to_const(params), map->occ, map->dims[0], map->dims[1],
                                         n_poses, poses, n_beams, beam_dir, sigma, max_range,
                                         mi_pose, mi_beam, ws),
                    "eval_poses_2d");
  }
  if (params->flags & FSMI_F_SKIP_ZERO)
    return fail(ctx, FSMI_E_INVAL, "FSMI_F_SKIP_ZERO needs explicit boundaries (2D maps)");
  if (ext_mode(params))
    return fail(ctx, FSMI_E_INVAL, "sigma_slope and FSMI_F_MAX_RANGE need explicit boundaries (2D maps)");
  if (params->variant == FSMI_CSQMI)
    return fail(ctx, FSMI_E_INVAL, "FSMI_CSQMI is a 2D path (fsmi_eval_beams, 2D poses)");
  if (params->flags & FSMI_F_LUT)
    return fail(ctx, FSMI_E_UNSUPPORTED, "FSMI_F_LUT is implemented on 2D fsmi_eval_poses");
  if (!(w > 0.0) || !std::isfinite(w)) return fail(ctx, FSMI_E_INVAL, "w must be finite and > 0");
  if (floor(max_range / w) > 4000.0) return fail(ctx, FSMI_E_CAPACITY, "more than 4000 virtual cells per beam");
  return from_hip(ctx,
                  launch_eval_poses_3d(ctx, to_const(params), map->occ, map->dims[0], map->dims[1],
                                       map->dims[2], n_poses, poses, n_beams, beam_dir, sigma,
                                       max_range, w, mi_pose, mi_beam, ws),
                  "eval_poses_3d");
}
}  // namespace fsmi

extern "C" {

fsmi_status fsmi_eval_trajectories(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                                   int64_t n_traj, const int64_t* traj_off, int64_t n_states,
                                   const double* poses, int64_t n_beams, const double* beam_dir,
                                   double sigma, double max_range, double* mi_traj,
                                   double* mi_state, double* mi_beam) {
  if (!ctx) return FSMI_E_INVAL;
  fsmi_status st;
  if (!check_params(ctx, params, &st)) return st;
  if (!check_map(ctx, map, &st)) return st;
  if (map->ndim != 2) return fail(ctx, FSMI_E_INVAL, "trajectories are evaluated on 2D maps");
  if (params->variant == FSMI_CSQMI)
    return fail(ctx, FSMI_E_INVAL, "cell marking sums Shannon MI per cell: EXACT, APPROX or UNIFORM");
  if (params->flags != 0 || params->sigma_slope != 0.0)
    return fail(ctx, FSMI_E_INVAL, "trajectories take no flags and no sigma_slope");
  if (n_traj < 0 || n_states < 0 || n_beams < 0) return fail(ctx, FSMI_E_INVAL, "negative count");
  if (n_traj == 0) return FSMI_OK;
  if (!traj_off || !mi_traj) return fail(ctx, FSMI_E_INVAL, "traj_off and mi_traj are required");
  if (n_traj >= ((int64_t)1 << 31)) return fail(ctx, FSMI_E_CAPACITY, "n_traj >= 2^31");
  if (n_states > 0 && n_beams > 0 && (!poses || !beam_dir))
    return fail(ctx, FSMI_E_INVAL, "poses and beam_dir are required");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(ctx, FSMI_E_INVAL, "sigma must be finite and > 0");
  if (!(max_range > 0.0) || !std::isfinite(max_range))
    return fail(ctx, FSMI_E_INVAL, "max_range must be finite and > 0");
  if (max_range > 4000.0) return fail(ctx, FSMI_E_CAPACITY, "max_range above 4000 cells");
  if (params->precision == FSMI_FP64 && max_range >= 3873.0)
    return fail(ctx, FSMI_E_CAPACITY, "max_range above 3872 cells in FP64");
  if (n_beams > 0 && n_states > ((int64_t)1 << 40) / n_beams)
    return fail(ctx, FSMI_E_CAPACITY, "too many items");
  (void)hipSetDevice(ctx->device);
  return from_hip(ctx,
                  launch_eval_trajectories_2d(ctx, to_const(params), map->occ, map->dims[0],
                                              map->dims[1], n_traj, traj_off, n_states, poses,
                                              n_beams, beam_dir, sigma, max_range, mi_traj,
                                              mi_state, mi_beam),
                  "eval_trajectories");
}

fsmi_status fsmi_probe_erfc(fsmi_ctx ctx, int64_t n, const float* z, float* out) {
  if (!ctx) return FSMI_E_INVAL;
  if (n < 0 || (n > 0 && (!z || !out))) return fail(ctx, FSMI_E_INVAL, "bad probe arguments");
  (void)hipSetDevice(ctx->device);
  return from_hip(ctx, launch_erfc_probe(ctx, n, z, out), "probe_erfc");
}

fsmi_status fsmi_peak(fsmi_ctx ctx, int32_t kind, double* rate, double* clock_mhz) {
  if (!ctx) return FSMI_E_INVAL;
  if (!rate || kind < FSMI_PEAK_COPY || kind > FSMI_PEAK_MFMA_BF16)
    return fail(ctx, FSMI_E_INVAL, "bad peak kind or NULL rate");
  (void)hipSetDevice(ctx->device);
  const hipError_t e = run_peak(ctx, kind, rate, clock_mhz);
  if (e == hipErrorOutOfMemory) return fail(ctx, FSMI_E_NOMEM, "peak: out of device memory");
  return from_hip(ctx, e, "peak");
}

fsmi_status fsmi_probe_f(fsmi_ctx ctx, double delta, int64_t n, const float* o, double* out) {
  if (!ctx) return FSMI_E_INVAL;
  if (!(delta > 0.0) || !(delta < 1e300) || n < 0 || (n > 0 && (!o || !out)))
    return fail(ctx, FSMI_E_INVAL, "bad probe arguments");
  (void)hipSetDevice(ctx->device);
  return from_hip(ctx, launch_f_probe(ctx, delta, n, o, out), "probe_f");
}

}  // extern "C"
