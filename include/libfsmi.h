/*
 * libfsmi.h -- C-ABI of libfsmi, an MI355X (gfx950) implementation of FSMI:
 * fast Shannon mutual information between an occupancy map and range beams
 * (Zhang, Henderson, Tzoumas, Karaman, Sze; arXiv 1905.02238).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments are DEVICE pointers owned by the caller.  The library
 *   never frees them and keeps them past the call only where a call says so
 *   (a plan of fsmi_plan_eval_beams keeps its batch's addresses until
 *   fsmi_plan_destroy).  Scalars and the small structs below are passed on
 *   the host.
 * - Calls are asynchronous: they enqueue kernels on the context's stream and
 *   return.  Results are ready after fsmi_sync() or any later operation on
 *   that stream.  The calls that say so wait for the device (fsmi_eval_beams
 *   once, to size its launch; plan creation; surrogate creation, checkpoint
 *   save and load).
 * - Map coordinates are in cell units.  2D cell (x, y) covers
 *   [x, x+1) x [y, y+1); 3D voxel (x, y, z) likewise.  A map is stored x
 *   fastest: linear index = x + X*(y + Y*z), held in int32, so a map has
 *   fewer than 2^31 cells.
 * - Occupancy o is P(M_i = 1) in [0, 1] (Sec. 2.1).  The inverse sensor
 *   model uses delta_occ > 1 and delta_emp = 1/delta_occ (Sec. 3.3).
 * - Mutual information is returned in nats (natural log).
 * - Errors: every call returns fsmi_status.  Bad scalars, shapes and sizes are
 *   reported at once and nothing is launched.  Bad data seen on the device
 *   (an occupancy outside [0,1] or NaN, a run length <= 0, decreasing
 *   boundaries, a pose outside the map) makes that result NaN and latches an
 *   error that the next fsmi_sync() returns (FSMI_E_NUMERIC) and clears.
 * - A context is not thread-safe; separate contexts are independent.
 *
 * Readings of the paper used throughout: the event "no cell is hit" carries
 * its reading beyond the last cell, outside the integration range
 * [0, l_{n+1}), so it contributes nothing (Alg 1 loops j from 0, but no cell
 * centre mu_0 exists); sigma is one constant per beam (Sec. 2.1, Sec. 3.3).
 */
#ifndef LIBFSMI_H
#define LIBFSMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsmi_ctx_s* fsmi_ctx;

typedef enum {
  FSMI_OK = 0,
  FSMI_E_INVAL = 1,       /* bad argument (NULL pointer, sigma <= 0, ...) */
  FSMI_E_DEVICE = 2,      /* HIP runtime error */
  FSMI_E_NOMEM = 3,       /* device allocation failed */
  FSMI_E_CAPACITY = 4,    /* an output buffer or a beam is larger than allowed */
  FSMI_E_NUMERIC = 5,     /* latched device data error (see above) */
  FSMI_E_UNSUPPORTED = 6  /* valid request the library does not implement */
} fsmi_status;

/* Variants (Table 1 of the paper). */
enum {
  FSMI_EXACT = 0,   /* Thm 1, Eq. fast_exact_mi: full double sum over (j, k) */
  FSMI_APPROX = 1,  /* Eq. fsmi_approx: k restricted to |k - j| <= Delta, no renormalisation */
  FSMI_UNIFORM = 2, /* Thm 4 / Alg 4: uniform noise of half-width H cells */
  /* The comparison metric of Sec. 2.3, not Shannon MI: Approx-CSQMI, Eq.
     csqmi_exact with both double sums truncated to |l - j| <= Delta
     (trunc_delta >= 0; trunc_delta >= n - 1 gives the exact CSQMI), in the
     printed form log B + log C - 2 log A (twice the -1/2 log of the
     Cauchy-Schwarz divergence's definition).  The weight of a first hit at l
     is w_l = P(e_l)^2 prod_{i>l} (o_i^2 + (1-o_i)^2), the sum of P(m)^2 over
     the maps whose first occupied cell is l; the all-free event reads beyond
     the beam.  Gaussian noise sigma per beam on the cell centres.  2D paths
     only (fsmi_eval_beams, plans, 2D fsmi_eval_poses); kernel, flags and
     sigma_slope must be the defaults. */
  FSMI_CSQMI = 3
};
/* Weight between hit cell j and reading cell k on equal-width cells. */
enum {
  FSMI_KERNEL_ERF = 0,    /* Phi((d+1/2)/sigma') - Phi((d-1/2)/sigma') (Eq. G_jk) */
  FSMI_KERNEL_DENSITY = 1 /* exp(-d^2/(2 sigma'^2))/(sqrt(2 pi) sigma') (proof of Thm 5) */
};
enum { FSMI_FP32 = 0, FSMI_FP64 = 1 };
enum {
  /* Skip-zero exact mode (EXACT, FP32, explicit boundaries: fsmi_eval_beams
     with bound, fsmi_plan_eval_beams with bound, 2D fsmi_eval_poses): each row
     j keeps only the boundaries within 9.3 sigma sqrt(2) of mu_j (plus the
     cells straddling that band's edges); every pair left out has an FP32 weight
     below the smallest normal float, so the result is the dense sum up to
     rounding order.  A separate mode with its own work count; any other
     combination gives FSMI_E_INVAL. */
  FSMI_F_SKIP_ZERO = 1u,
  /* Max-range returns (EXACT, explicit boundaries, FP32 or FP64): a reading at
     or past l_{n+1} is reported as max range and updates every cell of the
     beam as empty, so the term
       q_n [sum_j P(e_j) (1 - Phi((l_{n+1} - mu_j)/sigma_j)) + P(e_0)],
     q_n = sum_{i=1}^{n} f(delta_emp, r_i), is added to Thm 1 (the paper's
     Thm 1 integrates the reading over [0, l_{n+1}) only, Sec. 3.1).  Not with
     FSMI_F_SKIP_ZERO. */
  FSMI_F_MAX_RANGE = 2u,
  /* Engine of FSMI-RLE / Approx-FSMI-RLE (fsmi_rle_eval_beams, 3D
     fsmi_eval_poses; not with UNIFORM).  The run engine sums each row over the
     runs within the kernel's reach from tail tables of the kernel, O(n x runs);
     the expanded engine takes the double sum over the cells.  They give the
     same value up to rounding.  By default fsmi_rle_eval_beams takes the run
     engine for an EXACT beam of at most 64 runs averaging at least 32 cells and
     the expanded engine otherwise (the paper switches at runs of 4 cells, Sec.
     5.4; 32 is the measured crossover of these kernels, and Approx's expanded
     sum of 2 Delta + 1 terms a row stays cheaper); the fused 3D fsmi_eval_poses
     evaluates every beam on its cells by default (the sampled beams' runs fall
     below the crossover, and the fused kernel would carry the run engine's
     registers).  FSMI_F_RLE_RUNS takes the run engine for every beam of at most
     64 runs, FSMI_F_RLE_CELLS the expanded engine for every beam.  At most one
     of them; no other flag with them. */
  FSMI_F_RLE_RUNS = 4u,
  FSMI_F_RLE_CELLS = 8u,
  /* Look-up-table mode (Sec. 3.3, opt-in; 2D fsmi_eval_poses and
     fsmi_eval_poses_noalloc, FP32, EXACT or APPROX, one sigma): the tail of the
     normal distribution (the Phi differences of Eq. G_jk) and f(delta_occ, .)
     are read from tables with linear interpolation instead of being evaluated:
     1536 tail entries at 1/128 of the FP32 mode's scaled argument
     |l - mu| sqrt(log2 e) / (sigma sqrt 2), within 6e-6 of erfc, and 512 f
     entries over o in [0, 1]; f(delta_emp, o) = f(delta_occ, 1 - o).  The
     tables are built on the device at each call (16 KiB, held by the context)
     and staged into LDS.  An approximation with its own error (not the 1e-5
     bar of the analytic FP32 mode).  Alone: no other flag, no sigma_slope.
     Other entry points return FSMI_E_UNSUPPORTED. */
  FSMI_F_LUT = 16u
};

typedef struct {
  double delta_occ;   /* > 1; the paper uses 1.5 (Sec. 5.1) */
  int32_t variant;    /* FSMI_EXACT | FSMI_APPROX | FSMI_UNIFORM */
  int32_t trunc_delta;/* Delta >= 0, cells (APPROX) */
  int32_t uniform_h;  /* H >= 0, cells (UNIFORM) */
  int32_t kernel;     /* FSMI_KERNEL_* (equal-width cells and RLE only) */
  int32_t precision;  /* FSMI_FP32 (default) | FSMI_FP64 */
  uint32_t flags;     /* 0, FSMI_F_SKIP_ZERO, FSMI_F_MAX_RANGE, an FSMI_F_RLE_* engine or FSMI_F_LUT */
  /* Range-dependent noise: the reading of event e_j is N(mu_j, sigma_j^2) with
     sigma_j = sigma + sigma_slope * mu_j (Alg 1 writes sigma per event; the
     paper's experiments use one sigma).  >= 0; 0 (default) is one sigma per
     beam.  Any other value needs EXACT on explicit boundaries (fsmi_eval_beams
     and fsmi_plan_eval_beams with bound, 2D fsmi_eval_poses), not
     FSMI_F_SKIP_ZERO. */
  double sigma_slope;
} fsmi_params;

typedef struct {
  const float* occ;   /* device, o per cell, x fastest */
  int32_t ndim;       /* 2 or 3 */
  int64_t dims[3];    /* X, Y, Z (Z ignored for 2D) */
} fsmi_map;

/* ---- context ---- */
/* Opens a context on HIP device `device`.  hip_stream is the hipStream_t to
   enqueue on (NULL: the device's default stream).  The context allocates a
   status word, queue counters and a grow-only work area on the device. */
fsmi_status fsmi_create(fsmi_ctx* out, int device, void* hip_stream);
void fsmi_destroy(fsmi_ctx ctx);
/* Changes the stream later calls enqueue on (NULL: the default stream).  The
   context's scratch (status word, queue heads, work area) serves every call,
   so the new stream is first made to wait for all work enqueued so far on the
   old one (an event recorded there): calls of one context stay ordered across
   stream changes.  Calls of separate contexts are independent. */
fsmi_status fsmi_set_stream(fsmi_ctx ctx, void* hip_stream);
/* Waits for the stream; returns the latched device error (and clears it). */
fsmi_status fsmi_sync(fsmi_ctx ctx);
/* Text of the last error on this context (never NULL). */
const char* fsmi_last_error(fsmi_ctx ctx);
const char* fsmi_status_string(fsmi_status s);
/* Defaults: delta_occ 1.5, EXACT, Delta 3, H 0, ERF kernel, FP32, no flags. */
void fsmi_default_params(fsmi_params* p);

/* ---- a1 / a2: ray traversal ----
   The beam's cells in ascending distance (Sec. 2.2, Sec. 3.1), per ray.
   mode FSMI_RAY_DDA (2D map): every grid cell the ray crosses.  Face distance
     t = (face - p)*(1/d) with two roundings and no FMA, recomputed from the
     integer face after each step; an exact tie of axes is one diagonal step;
     a cell is listed only if its [entry, exit) is non-empty; the last cell is
     cut at max_range; the walk ends where the ray leaves the map.
     Outputs per ray r: count[r] = n, cell[r*max_cells + i] (linear index),
     entry[r*(max_cells+1) + i] = l_{i+1} for i = 0..n (l_1 = 0, l_{n+1} the end),
     occ_out[r*max_cells + i] = o of the cell (may be NULL).  cell and entry
     may both be NULL: then only count[] is written.
     max_cells >= floor(sqrt(2)*max_range) + 3, else FSMI_E_CAPACITY.
   mode FSMI_RAY_VIRTUAL (3D map): the beam projected onto equal virtual cells
     of width w (Sec. 4): cell i = 1..floor(R/w) takes the voxel holding its
     midpoint p + (i - 1/2) w d (per axis, no FMA); the beam ends at the first
     midpoint outside the map.  cell/occ_out as above; entry unused (NULL).
     max_cells >= floor(max_range/w), else FSMI_E_CAPACITY.
   mode FSMI_RAY_RLE (3D map): as VIRTUAL, then maximal runs of bit-identical
     o (Eq. occup_rle): count[r] = n_r, occ_out = run value, run_len = L_u.
   origin [n_rays][ndim] must lie inside the map (else that ray reports
   count -1 and the call latches FSMI_E_NUMERIC); dir [n_rays][ndim] FP64,
   not both zero (directions come from host libm, so both sides agree). */
enum { FSMI_RAY_DDA = 0, FSMI_RAY_VIRTUAL = 1, FSMI_RAY_RLE = 2 };
fsmi_status fsmi_raycast(fsmi_ctx ctx, const fsmi_map* map, int32_t mode, int64_t n_rays,
                         const double* origin, const double* dir, double max_range, double w,
                         int32_t max_cells, int32_t* count, int32_t* cell, double* entry,
                         float* occ_out, int32_t* run_len);

/* ---- a3..a9, a13, a14: batches of beams in CSR form ----
   Beam b has cells off[b] .. off[b+1]-1 of occ (float, [0,1]) and, when bound
   is not NULL, boundaries bound[off[b] + b + i] = l_{i+1}, i = 0..n_b
   (n_b + 1 increasing values per beam); bound == NULL means unit cells
   l_i = i - 1.  sigma[b] > 0 is the beam's range noise in the same length
   unit as the boundaries.  mi[b] receives I(M'; Z) (FP64) per the variant:
   EXACT (Thm 1), APPROX with Delta (Eq. fsmi_approx), UNIFORM with H (Alg 4 on
   cell-index windows).  Computation in FP32 with compensated sums and an
   FP64 prefix product, or entirely in FP64 with precision = FSMI_FP64.
   Beams of uneven length are scheduled longest-first on persistent workers:
   a beam longer than the wave threshold is shared by a whole workgroup.  The
   threshold is 512 cells (FP32) or 256 (FP64), or the one the autotuner of
   fsmi_plan_eval_beams chose on this context for the same precision, variant
   and boundary kind.  Waits once for the device (the longest beam sizes the
   workgroup's LDS); fsmi_plan_eval_beams avoids that wait.  A beam holds at
   most 7679 cells (FP32) or 5485 (FP64), else FSMI_E_CAPACITY. */
fsmi_status fsmi_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                            const int64_t* off, const float* occ, const double* bound,
                            const float* sigma, double* mi);

/* ---- a13: a planned beam batch, autotuned and replayed from a HIP graph ----
   fsmi_plan_eval_beams binds the arguments of fsmi_eval_beams to a plan: it
   finds the longest beam, sorts the beams into length bins once (its own
   device buffers, n_beams + 48 int32), and, with FSMI_PLAN_AUTOTUNE, times the
   launch at each candidate wave threshold on these very inputs and keeps the
   fastest (mi is written while tuning); the choice is also kept on the context
   for later fsmi_eval_beams calls of the same kind.  With FSMI_PLAN_GRAPH the
   launch (queue reset, tile-per-beam and wave-per-beam kernels) is captured
   once into a HIP graph.  wave_max > 0 fixes the threshold (cells); 0 takes the
   context's tuned value or the default.  Synchronous.
   fsmi_plan_launch enqueues one evaluation on the context's current stream and
   returns at once: it re-reads occ, bound and sigma and rewrites mi, so their
   contents may change between launches; off, n_beams and the buffer addresses
   are fixed.  Launches of one plan must not overlap (they share the queue
   counters).  Errors as fsmi_eval_beams; FSMI_E_CAPACITY at plan time when the
   longest beam does not fit a workgroup's LDS. */
typedef struct fsmi_plan_s* fsmi_plan;
enum { FSMI_PLAN_AUTOTUNE = 1u, FSMI_PLAN_GRAPH = 2u };
typedef struct {
  int32_t wave_max;          /* beams longer than this many cells are tile-per-beam */
  int32_t max_len;           /* longest beam, cells */
  int64_t n_tile;            /* beams taken by a whole workgroup */
  int64_t n_wave;            /* beams taken by a single wave */
  int32_t graph;             /* 1: launches replay a captured HIP graph */
  int32_t n_tried;           /* candidates the autotuner timed (0 without it) */
  int32_t tried_wave_max[16];
  float tried_ms[16];        /* mean launch time of each candidate, ms */
} fsmi_plan_info;
fsmi_status fsmi_plan_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                                 const int64_t* off, const float* occ, const double* bound,
                                 const float* sigma, double* mi, int32_t wave_max,
                                 uint32_t plan_flags, fsmi_plan* out);
fsmi_status fsmi_plan_launch(fsmi_plan plan);
fsmi_status fsmi_plan_get_info(fsmi_plan plan, fsmi_plan_info* info /* host */);
/* Waits for the context's stream, then frees the plan's buffers and graph. */
void fsmi_plan_destroy(fsmi_plan plan);

/* ---- a10, a11: run-length-encoded beams on equal-width virtual cells ----
   Beam b has runs run_off[b] .. run_off[b+1]-1 with value run_occ[u] and
   length run_len[u] >= 1 (Eq. occup_rle); sigma_prime[b] = sigma / w in
   virtual cells.  EXACT gives FSMI-RLE (Thm 5), APPROX gives Approx-FSMI-RLE
   (Thm 6) with the kernel truncated at |d| <= Delta, UNIFORM gives
   Uniform-FSMI-RLE (uniform noise of half-width H cells, the Thm 5 structure
   with the uniform kernel; params.kernel is ignored); the value equals the
   plain algorithm on the expanded beam with the chosen kernel. */
fsmi_status fsmi_rle_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                                const int64_t* run_off, const float* run_occ,
                                const int32_t* run_len, const float* sigma_prime, double* mi);

/* ---- the paper's table route for Approx-FSMI-RLE (Alg 8 with the tables of
   Alg 9 and 10), kept to compare against the run engine above ----
   Same runs as fsmi_rle_eval_beams, one sigma_prime (> 0) for the batch.  The
   alpha/beta/theta/gamma tables are built on the device for x = i / levels,
   i = 0 .. levels, with the Gaussian exp(-d^2 / (2 sigma'^2)) truncated at
   |d| <= Delta (params.trunc_delta); every table read takes x = 1 - o_u
   rounded to that grid, i = floor(levels (1 - o_u) + 1/2), while P_E, D_E and
   the crop factor (1 - o_u)^(s'_u - s_u) use o itself.  Blocks of a run u
   with an earlier run v use x^{-t} (alpha[t + L'_u, L'_v] - alpha[t, L'_v]),
   the route Sec. 4.1 calls unstable: with o on the grid the value is
   Approx-FSMI-RLE's (density kernel) up to a cancellation that grows like
   x^{-Delta}, about 1e-12 relative at x = 1/64, Delta = 3 and 1e-6 at
   Delta = 6 in FP64.  Requires variant FSMI_APPROX, precision FSMI_FP64,
   flags 0, sigma_slope 0, 0 <= trunc_delta <= 8, levels a power of two in
   [1, 1024]; else FSMI_E_INVAL.  A beam of more than 1024 runs or a run
   longer than 4096 cells latches FSMI_E_CAPACITY (result NaN); bad runs latch
   as in fsmi_rle_eval_beams.  Uses the context's work area for the tables,
   and waits for the stream once to size them by the batch's longest run.
   mi [n_beams] FP64, device. */
fsmi_status fsmi_rle_table_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                                      const int64_t* run_off, const float* run_occ,
                                      const int32_t* run_len, double sigma_prime,
                                      int32_t levels, double* mi);

/* ---- a12 + fused a1..a11: many poses x many beams ----
   2D map: poses [n_poses][4] = {x, y, cos(yaw), sin(yaw)}; beam_dir [n_beams][2]
   sensor-frame unit vectors.  World direction (c*bx - s*by, s*bx + c*by), each
   product rounded on its own.  Each beam is walked as FSMI_RAY_DDA to
   max_range and evaluated with sigma and the variant.
   3D map: poses [n_poses][5] = {x, y, z, cos(yaw), sin(yaw)}; beam_dir
   [n_beams][3]; world direction (c*bx - s*by, s*bx + c*by, bz).  Each beam is
   sampled onto virtual cells of width w as FSMI_RAY_VIRTUAL, and evaluated
   with sigma' = sigma / w as FSMI-RLE (EXACT), Approx-FSMI-RLE (APPROX) or
   Uniform-FSMI-RLE (UNIFORM, half-width H virtual cells): on its expanded
   cells by default, or in the run domain over its maximal runs of
   bit-identical o with FSMI_F_RLE_RUNS (see the flag); the value is the same.
   mi_pose[p] = sum over the pose's beams (Sec. 2.4; FP64, fixed order).
   mi_beam [n_poses][n_beams] (FP64) may be NULL.  One wave keeps a beam in
   LDS: 2D max_range <= 4000 cells (FP32) or < 3873 (FP64), 3D
   floor(max_range / w) <= 4000, else FSMI_E_CAPACITY. */
fsmi_status fsmi_eval_poses(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                            int64_t n_poses, const double* poses, int64_t n_beams,
                            const double* beam_dir, double sigma, double max_range, double w,
                            double* mi_pose, double* mi_beam);

/* ---- trajectory MI with cell marking (Sec. 2.4), 2D maps ----
   Candidate trajectories in CSR form: trajectory k has the states traj_off[k]
   .. traj_off[k+1]-1 (device int64 [n_traj + 1], non-decreasing, within
   [0, n_states]) of poses [n_states][4] = {x, y, cos(yaw), sin(yaw)}, in
   travel order.  A state's scan MI is the sum over its beams as in
   fsmi_eval_poses, except that a cell's information counts only at the first
   state of the trajectory whose beams cross it, and there at every beam of
   that state crossing it (cells that have contributed are marked and not
   counted again).  Marked cells still shape the measurement: their f terms
   leave C_k while P(e_j) uses every cell.  mi_traj[k] = the sum over its
   states; mi_state [n_states] and mi_beam [n_states][n_beams] (FP64, device)
   may be NULL.  EXACT, APPROX or UNIFORM, FP32 or FP64, no flags, no
   sigma_slope (FSMI_E_INVAL otherwise).  The call reads traj_off back to the
   host once (it waits for the work before it on the stream) and evaluates the
   trajectories in groups of up to 64, one stamp map of 8 bytes per map cell
   each, within 1 GiB (at least one map); the context's work area holds those
   maps plus the per-beam and per-state sums not kept by the caller.  A
   trajectory whose offsets are invalid gives NaN and the call latches
   FSMI_E_NUMERIC (states that no valid trajectory covers keep MI 0); a state
   outside the map as in fsmi_eval_poses.  Range limits as fsmi_eval_poses on
   2D maps. */
fsmi_status fsmi_eval_trajectories(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                                   int64_t n_traj, const int64_t* traj_off, int64_t n_states,
                                   const double* poses, int64_t n_beams, const double* beam_dir,
                                   double sigma, double max_range, double* mi_traj,
                                   double* mi_state, double* mi_beam);

/* ---- fsmi_eval_poses without device allocation ----
   For callers that cannot allocate device memory during the call: code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
   Same arguments, results and errors as fsmi_eval_poses (the same kernels,
   bit-identical results), but its scratch -- the per-beam partial results
   (when mi_beam is NULL) and the work-queue head -- lives in a static device
   array of the library, 16 MiB + 256 bytes, that each device the library runs
   on holds until the process ends (its address is resolved per device by
   fsmi_create).  The call itself allocates nothing (no hipMalloc, hipFree or
   allocating library routine); the caller passes inputs and outputs.  With
   mi_beam == NULL, n_poses * n_beams must not exceed 2^21 (2 097 152), else
   FSMI_E_CAPACITY and nothing is launched; with mi_beam given there is no
   such limit.  Every call on a device shares that device's array, which keeps
   the last call's contents (the queue head is cleared by a kernel at the
   start of each call): calls that overlap on one device, from any context or
   stream, race and give wrong results -- order them. */
fsmi_status fsmi_eval_poses_noalloc(fsmi_ctx ctx, const fsmi_params* params, const fsmi_map* map,
                                    int64_t n_poses, const double* poses, int64_t n_beams,
                                    const double* beam_dir, double sigma, double max_range,
                                    double w, double* mi_pose, double* mi_beam);

/* ---- a15..a17: learned surrogate, trained on FSMI's own labels ----
   A small conv net predicts a pose's scan MI from a 128 x 128 patch of o
   around the pose, resampled at the pose's continuous position: with cell
   stride s the map is taken as its s x s block means (blocks cut by the map
   edge average their inside cells; blocks outside the map read 0.5; s = 1 is
   the cells themselves), and with (u, v) = (x / s, y / s) the pose in block
   units, patch pixel (iy, ix) is the bilinear interpolation of the blocks at
   (u - 64 + ix + 1/2, v - 64 + iy + 1/2), block k centred at k + 1/2: blocks
   bx - 64 + ix + {0, 1}, by - 64 + iy + {0, 1} with (bx, by) = (floor(floor(x)
   / s), floor(floor(y) / s)) weighted by (u - bx, v - by), bx and by held
   within +-(2^31 - 2^10).  Five 3x3 convs,
   stride 2, padding 1, ReLU (1-32-64-64-128-128 channels), global average pool,
   FC 128->256, ReLU, FC 256->1, 310465 parameters.  BF16 activations and
   weights on the matrix cores with FP32 accumulation, FP32 master weights and
   Adam moments.  Labels become regression targets through
   fsmi_sur_fit_label_stats and the loss is the batch-mean squared error.  Surrogate calls take 2D maps and 2D
   poses ([n][4]); they enqueue on the stream of the context the net was created
   with.  The network is not in the paper: it ranks candidate poses cheaply, and
   fsmi_rank_poses always re-scores its top k with exact FSMI (Thm 1). */
typedef struct fsmi_sur_s* fsmi_sur;
int64_t fsmi_sur_num_params(void);
/* Allocates parameters, optimiser state and activations for batches of up to
   max_batch poses (<= 65536); Kaiming-uniform weights from a counter-based
   generator seeded by `seed`, zero biases; patch cell stride 1..64. */
fsmi_status fsmi_sur_create(fsmi_ctx ctx, fsmi_sur* out, uint64_t seed, int32_t max_batch,
                            int32_t patch_stride);
void fsmi_sur_destroy(fsmi_sur net);
/* Statistics of n device FP64 labels (nats), kept in the net: their mean and
   standard deviation, then the mean and standard deviation of
   e = exp((label - mean) / scale).  A label's regression target is
   (e - emean) / escale: monotone in the label, with the squared error weighting
   the upper tail, where a ranking keeps its candidates.  A prediction y reads
   mean + scale ln(max(y escale + emean, 1e-6)) nats.  A new net holds
   {0, 1, 0, 1}. */
fsmi_status fsmi_sur_fit_label_stats(fsmi_sur net, int64_t n, const double* labels);
fsmi_status fsmi_sur_get_label_stats(fsmi_sur net,
                                     double* host_stats /* [4] host: mean, scale, emean, escale */);
/* pred[n] (device FP32) = predicted MI in nats; any n (processed in batches). */
fsmi_status fsmi_sur_forward(fsmi_sur net, const fsmi_map* map, int64_t n, const double* poses,
                             float* pred);
/* Forward and backward of one batch (n <= max_batch) against labels[n] (device
   FP64, nats): gradients are kept in the net; *loss (device FP32, or NULL) gets
   the MSE against the targets.  Deterministic (fixed-order reductions). */
fsmi_status fsmi_sur_backward(fsmi_sur net, const fsmi_map* map, int64_t n, const double* poses,
                              const double* labels, float* loss);
fsmi_status fsmi_sur_adam_step(fsmi_sur net, float lr, float beta1, float beta2, float eps);
/* Device FP32 [fsmi_sur_num_params()] copies of the master weights / gradients. */
fsmi_status fsmi_sur_get_params(fsmi_sur net, float* dst);
fsmi_status fsmi_sur_set_params(fsmi_sur net, const float* src);
fsmi_status fsmi_sur_get_grads(fsmi_sur net, float* dst);
/* Checkpoint (host file): step, patch stride, label statistics, weights, Adam
   moments; load adopts the file's patch stride. */
fsmi_status fsmi_sur_save(fsmi_sur net, const char* path);
fsmi_status fsmi_sur_load(fsmi_sur net, const char* path);
/* Ranks n_poses 2D candidates by the surrogate, keeps the top k (ties by index),
   and re-scores them with exact FSMI (params, beams, sigma, max_range as in
   fsmi_eval_poses).  idx_out[k] (device int32): candidate indices in the
   surrogate's order; mi_out[k] (device FP64): their exact scan MI; pred_out
   (device FP32 [n_poses] or NULL): the surrogate's predictions.  `net` must have
   been created on `ctx` (FSMI_E_INVAL otherwise): everything runs on its stream. */
fsmi_status fsmi_rank_poses(fsmi_ctx ctx, const fsmi_params* params, fsmi_sur net,
                            const fsmi_map* map, int64_t n_poses, const double* poses,
                            int64_t n_beams, const double* beam_dir, double sigma,
                            double max_range, int32_t k, int32_t* idx_out, double* mi_out,
                            float* pred_out);

/* ---- diagnostics ----
   out[i] = the library's FP32 erfc at z[i] >= 0 (the function every Gaussian
   weight G_{k,j} is built from), so its error can be measured against FP64. */
fsmi_status fsmi_probe_erfc(fsmi_ctx ctx, int64_t n, const float* z, float* out);
/* out[i] (device FP64) = f(delta, o[i]) of Sec. 2.2 (the log-odds update of a
   cell of occupancy o[i] for the odds ratio delta), as the FP32 mode evaluates
   it.  o (device FP32) in [0, 1]; delta > 0 and finite (the FP32 mode calls it
   with delta_occ and with 1/delta_occ). */
fsmi_status fsmi_probe_f(fsmi_ctx ctx, double delta, int64_t n, const float* o, double* out);
/* D (device FP32 16x16, row-major) = A (BF16 16x32) * B (BF16 32x16) through one
   matrix-core instruction, so its operand layout can be checked. */
fsmi_status fsmi_probe_mfma(fsmi_ctx ctx, const void* A, const void* B, float* D);

/* ---- machine ceilings ----
   Runs one of the library's own microbenchmarks on ctx's device, on ctx's
   stream, and returns the measured rate in *rate and, if clock_mhz is not
   NULL, the shader clock its waves ran at (their cycle counts over the
   constant-rate wall clock), in MHz.  Waits for the device.
   Allocates and frees its own buffers: 2 GiB for the copy, a few MiB for the
   others.  FSMI_E_INVAL for another kind.
     FSMI_PEAK_COPY       bytes/s moved by a plain device-to-device copy of
                          1 GiB, bytes read plus bytes written (the HBM roof);
     FSMI_PEAK_FMA        FP32 FLOP/s of independent scalar FMA chains, 2 FLOP
                          per FMA (this library does not use packed FP32);
     FSMI_PEAK_PAIR       pairs/s of one FP32 erfc of the library plus one FMA
                          per pair, operands in registers: the Phi-pair
                          ceiling of the exact double sum (Thm 1 with the
                          weights of Eq. G_jk, one erfc per (row, boundary));
     FSMI_PEAK_MFMA_BF16  FLOP/s of dense BF16 matrix-core products
                          (16x16x32, FP32 accumulate). */
enum { FSMI_PEAK_COPY = 0, FSMI_PEAK_FMA = 1, FSMI_PEAK_PAIR = 2, FSMI_PEAK_MFMA_BF16 = 3 };
fsmi_status fsmi_peak(fsmi_ctx ctx, int32_t kind, double* rate, double* clock_mhz);

#ifdef __cplusplus
}
#endif
#endif /* LIBFSMI_H */
