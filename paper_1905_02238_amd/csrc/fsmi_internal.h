// fsmi_internal.h -- host-side declarations shared by the C-ABI layer and the
// kernel launchers of libfsmi.  Not installed; callers use include/libfsmi.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "libfsmi.h"

struct fsmi_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream; nullptr = the default stream
  // Orders work across a change of stream: the context's scratch (status word,
  // queue heads, work area) is shared by every call, so a call on a new stream
  // must not start before the calls enqueued on the old one have finished.
  hipEvent_t handoff = nullptr;
  uint32_t* d_status = nullptr;   // latched device error bits
  int32_t* d_counters = nullptr;  // work-queue heads, 64 entries
  void* d_work = nullptr;         // grow-only scratch for schedules / partial results
  void* d_lut = nullptr;          // the look-up tables of FSMI_F_LUT (built per call)
  size_t work_bytes = 0;
  int num_cu = 256;
  std::string last_error;
  // Autotuned wave/tile threshold of the beam-batch schedule, per
  // [precision][variant][explicit boundaries]; 0 = not tuned (use the default).
  int tuned_wave_max[2][4][2] = {};
};

namespace fsmi {

// Scalars of one evaluation, shared by every kernel family.
struct EvalConst {
  int variant;       // FSMI_EXACT / FSMI_APPROX / FSMI_UNIFORM / FSMI_CSQMI
  int Delta;         // truncation width (cells), APPROX and CSQMI
  int H;             // uniform half-width (cells), UNIFORM
  int kernel;        // FSMI_KERNEL_ERF / FSMI_KERNEL_DENSITY (equal-width engines)
  int precision;     // FSMI_FP32 / FSMI_FP64
  uint32_t flags;
  double delta_occ;  // > 1
  double slope;      // sigma_j = sigma + slope mu_j (EXACT on explicit boundaries); 0 = one sigma
};

// The table route of Approx-FSMI-RLE (k_rle_table.hip), FP64.
hipError_t launch_rle_table(fsmi_ctx ctx, double delta_occ, int Delta, int levels,
                            double sigma_p, int64_t n_beams, const int64_t* run_off,
                            const float* run_occ, const int32_t* run_len, double* mi);

// Grow-only device scratch owned by the context.
hipError_t ensure_work(fsmi_ctx ctx, size_t bytes);

// ---- argument checks and error reporting of the C-ABI (api.hip) ----
fsmi_status fail(fsmi_ctx ctx, fsmi_status s, const std::string& msg);
fsmi_status from_hip(fsmi_ctx ctx, hipError_t e, const char* where);
bool check_params(fsmi_ctx ctx, const fsmi_params* p, fsmi_status* st);
bool check_map(fsmi_ctx ctx, const fsmi_map* m, fsmi_status* st);
EvalConst to_const(const fsmi_params* p);
// sigma_slope != 0 or FSMI_F_MAX_RANGE: the extensions that need explicit boundaries
bool ext_mode(const fsmi_params* p);
// The wave/tile threshold for a beam batch: the autotuned one if any, else the default.
int ctx_wave_max(fsmi_ctx ctx, const fsmi_params* p, bool has_bound);

// ---- launchers (k_beam.hip) ----
// Beam batches: beams longer than wave_max cells are tile-per-beam (a workgroup
// each), the rest wave-per-beam.  A schedule buffer holds beam_sched_ints(n)
// int32: the beam order (longest bins first), the bin histogram and the queue
// counters.
int beam_default_wave_max(int precision);
int beam_bytes_per_cell(int precision);
bool beam_fits(int precision, int wave_max, int max_len);
size_t beam_sched_ints(int64_t n_beams);
int64_t beam_sched_n_long_index(int64_t n_beams);   // where the schedule leaves the tile-beam count
hipError_t launch_max_len(fsmi_ctx ctx, const int64_t* off, int64_t n_beams, int* host_out);
hipError_t launch_beam_schedule(hipStream_t st, const int64_t* off, int64_t n_beams, int wave_max,
                                int32_t* sched);
hipError_t launch_beam_kernels(hipStream_t st, int num_cu, const EvalConst& ec, int64_t n_beams,
                               const int64_t* off, const float* occ, const double* bound,
                               const float* sigma, double* mi, const int32_t* sched,
                               uint32_t* status, int wave_max, int max_len);
hipError_t launch_build_lut(hipStream_t st, double delta_occ, void* out);   // kLutBytes at out
size_t lut_bytes();
hipError_t launch_eval_beams(fsmi_ctx ctx, const EvalConst& ec, int64_t n_beams, const int64_t* off,
                             const float* occ, const double* bound, const float* sigma,
                             double* mi, int max_len, int wave_max);
hipError_t launch_fill_f64(hipStream_t st, int64_t n, double v, double* p);

// ---- launchers (k_ray.hip) ----
hipError_t launch_raycast2d(fsmi_ctx ctx, const float* map, int64_t X, int64_t Y, int64_t n_rays,
                            const double* origin, const double* dir, double R, int max_cells,
                            int32_t* count, int32_t* cell, double* entry, float* occ_out);
hipError_t launch_virtual3d(fsmi_ctx ctx, const float* map, int64_t X, int64_t Y, int64_t Z,
                            int64_t n_rays, const double* origin, const double* dir, double R,
                            double w, int max_cells, int rle, int32_t* count, int32_t* cell,
                            float* occ_out, int32_t* run_len);

// Caller-provided scratch of the pose launchers (fsmi_eval_poses_noalloc): the
// per-beam partial results (used when mi_beam is NULL) and the 64-bit queue
// head.  nullptr: the context's work area and counters.
struct PoseScratch {
  double* beams;
  int32_t* counter;
};

// ---- launchers (k_pose.hip) ----
hipError_t launch_eval_poses_2d(fsmi_ctx ctx, const EvalConst& ec, const float* map, int64_t X,
                                int64_t Y, int64_t n_poses, const double* poses, int64_t n_beams,
                                const double* beam_dir, double sigma, double R, double* mi_pose,
                                double* mi_beam, const PoseScratch* ws = nullptr);

// ---- launchers (k_traj.hip) ----
hipError_t launch_eval_trajectories_2d(fsmi_ctx ctx, const EvalConst& ec, const float* map,
                                       int64_t X, int64_t Y, int64_t n_traj,
                                       const int64_t* traj_off, int64_t n_states,
                                       const double* poses, int64_t n_beams,
                                       const double* beam_dir, double sigma, double R,
                                       double* mi_traj, double* mi_state, double* mi_beam);

// ---- launchers (k_rle.hip) ----
hipError_t launch_rle_eval_beams(fsmi_ctx ctx, const EvalConst& ec, int64_t n_beams,
                                 const int64_t* run_off, const float* run_occ,
                                 const int32_t* run_len, const float* sigma_p, double* mi,
                                 int max_cells);
hipError_t launch_eval_poses_3d(fsmi_ctx ctx, const EvalConst& ec, const float* map, int64_t X,
                                int64_t Y, int64_t Z, int64_t n_poses, const double* poses,
                                int64_t n_beams, const double* beam_dir, double sigma, double R,
                                double w, double* mi_pose, double* mi_beam,
                                const PoseScratch* ws = nullptr);

// fsmi_eval_poses after its argument checks (api.hip), with the scratch the
// call uses: ws == nullptr takes the context's work area and counters.
fsmi_status eval_poses_checked(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                               int64_t n_poses, const double* poses, int64_t n_beams,
                               const double* beam_dir, double sigma, double max_range, double w,
                               double* mi_pose, double* mi_beam, const PoseScratch* ws);

// ---- fsmi_eval_poses_noalloc (noalloc.hip) ----
// Resolves, once per device and with that device current, the device address
// of the library's static scratch array; called by fsmi_create.
hipError_t noalloc_scratch_init(int device);

// ---- machine ceilings (k_peak.hip) ----
hipError_t run_peak(fsmi_ctx ctx, int kind, double* rate, double* clock_mhz);

// ---- diagnostics (k_beam.hip) ----
hipError_t launch_erfc_probe(fsmi_ctx ctx, int64_t n, const float* z, float* out);
hipError_t launch_f_probe(fsmi_ctx ctx, double delta, int64_t n, const float* o, double* out);

}  // namespace fsmi
