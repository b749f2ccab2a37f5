// k_rle.hip -- FSMI on run-length-encoded beams (fsmi_rle_eval_beams) and the
// fused 3D pose path (fsmi_eval_poses on voxel maps).
//
// FSMI-RLE (Thm 5) and Approx-FSMI-RLE (Thm 6) are evaluated per beam by one
// of two engines, chosen as the paper chooses (Sec. 5.4: decompress when runs
// are shorter than 4 cells on average):
//   - the run engine (rle_dev.h): per-run f and D_E, each row's sum over the
//     runs within the kernel's reach from two tail tables, O(n x runs in reach),
//     for beams of at most kRunCap runs with a mean run length of at least 4;
//   - the expanded engine: the runs expanded to their cells and the plain
//     double sum with the per-beam kernel table (beam_dev.h), which equals
//     the RLE formulas by the proofs of Thm 5 and Thm 6 (with the kernel
//     truncated inside the blocks too).
// Uniform-FSMI-RLE always takes the expanded engine: Alg 4 on the cells is
// already O(n).
#include <math.h>

#include <algorithm>

#include "beam_dev.h"
#include "fsmi_internal.h"
#include "ray_dev.h"
#include "rle_dev.h"

namespace fsmi {
hipError_t launch_pose_reduce(fsmi_ctx ctx, const double* mi_beam, int64_t n_poses,
                              int64_t n_beams, double* mi_pose);
namespace {

struct RleArgs {
  EvalConst ec;
  int64_t n_beams;
  const int64_t* run_off;
  const float* run_occ;
  const int32_t* run_len;
  const float* sigma_p;
  double* mi;
  int cap;             // expanded cells per beam
  int32_t* counter;    // 64-bit queue head
  uint32_t* status;
};

// LDS of one wave: A, C, P of the expanded engine and the occupancies, then the
// run region (rle_dev.h); in the run engine C's slots hold the run of each cell.
template <typename T>
__host__ __device__ inline size_t rle_lds(int cap, bool with_runs = true) {
  return (size_t)core_bytes_per_cell<T>() * cap + 8 + 4 * (size_t)cap + 16 +
         (with_runs ? run_region_bytes<T>(cap) : 0);
}

// The run region starts on the first 16-byte boundary after the occupancies
// (rle_lds leaves 16 bytes for it).
FSMI_DEV char* run_region(float* so, int cap) {
  return reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(so + cap) + 15) & ~(uintptr_t)15);
}

// The engine of a beam of nr runs over n cells.  The paper decompresses when
// runs are shorter than 4 cells (Sec. 5.4); on this chip the measured crossover
// (256-cell beams in runs of L, sigma' = 2) lies at about 32 cells for FSMI-RLE
// and beyond 128 for Approx-FSMI-RLE, whose expanded sum is only 2 Delta + 1
// terms a row: the run engine takes EXACT beams of at most kRunCap runs
// averaging 32 cells or more.  FSMI_F_RLE_RUNS / FSMI_F_RLE_CELLS force one.
constexpr int kRunEngineMeanLen = 32;
FSMI_DEV bool use_run_engine(const EvalConst& ec, int n, int nr) {
  if (ec.variant == FSMI_UNIFORM || nr > kRunCap || (ec.flags & FSMI_F_RLE_CELLS)) return false;
  if (ec.flags & FSMI_F_RLE_RUNS) return true;
  return ec.variant == FSMI_EXACT && n >= kRunEngineMeanLen * nr;
}

template <typename T>
FSMI_DEV CoreLds carve_rle(char* p, int cap, float** so) {
  CoreLds L;
  L.A = reinterpret_cast<double*>(p);
  L.C = p + 8 * (size_t)(cap + 1);
  L.P = reinterpret_cast<char*>(L.C) + sizeof(T) * (size_t)cap;
  *so = reinterpret_cast<float*>(reinterpret_cast<char*>(L.P) + sizeof(T) * (size_t)cap);
  return L;
}

// Expands runs [r0, r1) into so[0..n); returns n, or -1 on a bad run length / overflow.
FSMI_DEV int expand_runs(const float* run_occ, const int32_t* run_len, int64_t r0, int64_t r1,
                         int cap, float* so, int* ss, int lane) {
  // run starts by an exclusive scan of the lengths (chunks of 64 runs)
  int carry = 0;
  bool bad = false;
  const int nr = (int)(r1 - r0);
  for (int base = 0; base < nr; base += kWave) {
    const int u = base + lane;
    int L = u < nr ? run_len[r0 + u] : 0;
    if (u < nr && L <= 0) bad = true;
    L = L > 0 ? L : 0;
    const int inc = wave_scan_incl<OpAdd>(L);
    const int s = carry + inc - L;
    if (u < nr && !bad && s + L <= cap) {
      const float o = run_occ[r0 + u];
      for (int t = 0; t < L; ++t) so[s + t] = o;
    }
    carry += wave_last(inc);
    if (carry > cap) bad = true;
  }
  (void)ss;
  if (__any(bad)) return -1;
  wave_sync();
  return carry;
}

template <typename T>
__global__ __launch_bounds__(kWave) void k_rle_beams(RleArgs a) {
  extern __shared__ __align__(16) char lds[];
  float* so;
  const CoreLds L = carve_rle<T>(lds, a.cap, &so);
  const RunLds R = carve_runs<T>(run_region(so, a.cap), a.cap, reinterpret_cast<int*>(L.C));
  const int lane = threadIdx.x;
  // runs of beams from the queue (guided self-scheduling)
  const int64_t n_waves = gridDim.x;
  int64_t kr = run_length(a.n_beams, 0, n_waves);
  for (int64_t start = wave_take64(a.counter, kr); start < a.n_beams;
       start = wave_take64(a.counter, kr)) {
    const int64_t it_end = min<int64_t>(start + kr, a.n_beams);
    kr = run_length(a.n_beams, it_end, n_waves);
    for (int64_t it = start; it < it_end; ++it) {
      const int64_t r0 = a.run_off[it], r1 = a.run_off[it + 1];
      double v;
      if (r1 < r0) {
        v = __builtin_nan("");
        if (lane == 0) latch(a.status, kErrLen);
      } else {
        const int nr = (int)min<int64_t>(r1 - r0, (int64_t)kRunCap + 1);
        const int n = nr <= kRunCap
                          ? runs_from_csr(a.run_occ, a.run_len, r0, r1, a.cap, so, R, lane)
                          : expand_runs(a.run_occ, a.run_len, r0, r1, a.cap, so, nullptr, lane);
        if (n < 0) {
          v = __builtin_nan("");
          if (lane == 0) latch(a.status, kErrLen);
        } else if (n == 0) {
          v = 0.0;
        } else {
          bool bad;
          if (use_run_engine(a.ec, n, nr))
            v = rle_core<T>(a.ec, n, so, nr, R, (double)a.sigma_p[it], L, lane, &bad);
          else
            v = beam_core<1, false, T>(a.ec, n, so, false, (double)a.sigma_p[it], L, nullptr,
                                       nullptr, lane, false, &bad);
          if (bad && lane == 0) latch(a.status, kErrOcc);
        }
      }
      if (lane == 0) a.mi[it] = v;
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------------
// Fused 3D: one wave per (pose, beam): yaw rotation, virtual cells (ray_dev.h),
// evaluation on the expanded virtual cells.
// ---------------------------------------------------------------------------
struct Pose3dArgs {
  EvalConst ec;
  const float* map;
  int64_t X, Y, Z;
  int64_t n_poses, n_beams;
  const double* poses;     // [n][5] x, y, z, cos, sin
  const double* beam_dir;  // [n][3]
  double sigma_p, R, w;
  int cap;
  double* mi_beam;
  int32_t* counter;
  uint32_t* status;
};

// RUNS: the instantiation that carries the run engine (FSMI_F_RLE_RUNS); the
// default one evaluates every beam on its expanded cells.  At the 3D
// workload's run lengths (15.6 cells on average) the run engine does not
// reach its measured crossover, and carrying it costs registers.
template <typename T, bool RUNS>
FSMI_DEV void poses3d_body(const Pose3dArgs& a) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) char lds[];
  float* so;
  const CoreLds L = carve_rle<T>(lds, a.cap, &so);
  const RunLds R = carve_runs<T>(run_region(so, a.cap), a.cap, reinterpret_cast<int*>(L.C));
  const int lane = threadIdx.x;
  const int64_t n_items = a.n_poses * a.n_beams;
  // runs of items from the queue (guided self-scheduling); k, start and the
  // loop bounds are wave-uniform
  const int64_t n_waves = gridDim.x;
  int64_t k = run_length(n_items, 0, n_waves);
  for (int64_t start = wave_take64(a.counter, k); start < n_items;
       start = wave_take64(a.counter, k)) {
    const int64_t it_end = min<int64_t>(start + k, n_items);
    k = run_length(n_items, it_end, n_waves);
    for (int64_t it = start; it < it_end; ++it) {
      const int64_t p = it / a.n_beams, b = it - p * a.n_beams;
      const double* ps = a.poses + 5 * p;
      const double* bd = a.beam_dir + 3 * b;
      const double m1 = ps[3] * bd[0], m2 = ps[4] * bd[1], m3 = ps[4] * bd[0], m4 = ps[3] * bd[1];
      const double d[3] = {m1 - m2, m3 + m4, bd[2]};
      bool ok;
      const int n = virtual3d_wave(a.map, a.X, a.Y, a.Z, ps, d, a.R, a.w, a.cap, so, nullptr, lane, &ok);
      double v;
      if (!ok) {
        v = __builtin_nan("");
        if (lane == 0) latch(a.status, kErrPose);
      } else if (n == 0) {
        v = 0.0;
      } else {
        wave_sync();
        bool bad;
        if constexpr (RUNS) {
          const int nr = runs_of_cells(so, n, R, lane);
          if (nr <= kRunCap)
            v = rle_core<T>(a.ec, n, so, nr, R, a.sigma_p, L, lane, &bad);
          else
            v = beam_core<1, false, T>(a.ec, n, so, false, a.sigma_p, L, nullptr, nullptr, lane,
                                       false, &bad);
        } else {
          v = beam_core<1, false, T>(a.ec, n, so, false, a.sigma_p, L, nullptr, nullptr, lane, false,
                                     &bad);
        }
        if (bad && lane == 0) latch(a.status, kErrOcc);
      }
      if (lane == 0) a.mi_beam[it] = v;
      wave_sync();
    }
  }
}

__global__ __launch_bounds__(kWave) void k_poses3d_f32(Pose3dArgs a) {
  poses3d_body<float, false>(a);
}
__global__ __launch_bounds__(kWave) void k_poses3d_f64(Pose3dArgs a) {
  poses3d_body<double, false>(a);
}
// With the run engine: FP32 held to 128 VGPRs (4 waves per SIMD, which the
// sampler's gathers need to hide their latency; two spilled registers).
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4)))
void k_poses3d_runs_f32(Pose3dArgs a) {
  poses3d_body<float, true>(a);
}
__global__ __launch_bounds__(kWave) void k_poses3d_runs_f64(Pose3dArgs a) {
  poses3d_body<double, true>(a);
}

__global__ void k_reset_counter64(int32_t* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

__global__ void k_rle_max_len(const int64_t* run_off, const int32_t* run_len, int64_t n_beams,
                              int32_t* out) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n_beams;
       b += (int64_t)gridDim.x * blockDim.x) {
    int64_t s = 0;
    for (int64_t u = run_off[b]; u < run_off[b + 1]; ++u) s += run_len[u] > 0 ? run_len[u] : 0;
    atomicMax(out, (int32_t)min<int64_t>(s, 0x7fffffff));
  }
}

__global__ void k_zero_i32(int32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

}  // namespace

hipError_t launch_rle_eval_beams(fsmi_ctx ctx, const EvalConst& ec, int64_t n_beams,
                                 const int64_t* run_off, const float* run_occ,
                                 const int32_t* run_len, const float* sigma_p, double* mi,
                                 int max_cells) {
  if (n_beams <= 0) return hipSuccess;
  hipError_t e;
  if (max_cells <= 0) {
    e = ensure_work(ctx, 64);
    if (e != hipSuccess) return e;
    int32_t* d = reinterpret_cast<int32_t*>(ctx->d_work);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, d);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_beams + 255) / 256, 1024));
    hipLaunchKernelGGL(k_rle_max_len, dim3(grid), dim3(256), 0, ctx->stream, run_off, run_len,
                       n_beams, d);
    int host = 0;
    e = hipMemcpyAsync(&host, d, 4, hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    max_cells = std::max(host, 1);
  }
  RleArgs a;
  a.ec = ec;
  a.n_beams = n_beams;
  a.run_off = run_off;
  a.run_occ = run_occ;
  a.run_len = run_len;
  a.sigma_p = sigma_p;
  a.mi = mi;
  a.cap = max_cells;
  a.counter = ctx->d_counters + 8;
  a.status = ctx->d_status;
  const bool fp64 = ec.precision == FSMI_FP64;
  const size_t lds = fp64 ? rle_lds<double>(a.cap) : rle_lds<float>(a.cap);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reset_counter64, dim3(1), dim3(64), 0, ctx->stream, a.counter);
  const int per_cu = std::max<int>(1, std::min<int>(16, (int)((160 * 1024) / (lds + 256))));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_beams, (int64_t)ctx->num_cu * per_cu));
  if (fp64) {
    (void)hipFuncSetAttribute((const void*)k_rle_beams<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_rle_beams<double>, dim3(grid), dim3(kWave), lds, ctx->stream, a);
  } else {
    (void)hipFuncSetAttribute((const void*)k_rle_beams<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_rle_beams<float>, dim3(grid), dim3(kWave), lds, ctx->stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_eval_poses_3d(fsmi_ctx ctx, const EvalConst& ec, const float* map, int64_t X,
                                int64_t Y, int64_t Z, int64_t n_poses, const double* poses,
                                int64_t n_beams, const double* beam_dir, double sigma, double R,
                                double w, double* mi_pose, double* mi_beam, const PoseScratch* ws) {
  const int64_t n_items = n_poses * n_beams;
  if (n_items <= 0) return hipSuccess;
  double* mb = mi_beam;
  if (!mb && ws) {
    mb = ws->beams;
  } else if (!mb) {
    hipError_t e = ensure_work(ctx, (size_t)n_items * 8);
    if (e != hipSuccess) return e;
    mb = reinterpret_cast<double*>(ctx->d_work);
  }
  Pose3dArgs a;
  a.ec = ec;
  a.map = map;
  a.X = X;
  a.Y = Y;
  a.Z = Z;
  a.n_poses = n_poses;
  a.n_beams = n_beams;
  a.poses = poses;
  a.beam_dir = beam_dir;
  a.sigma_p = sigma / w;
  a.R = R;
  a.w = w;
  a.cap = std::max(1, (int)floor(R / w));
  a.mi_beam = mb;
  a.counter = ws ? ws->counter : ctx->d_counters + 8;
  a.status = ctx->d_status;
  const bool fp64 = ec.precision == FSMI_FP64;
  const bool with_runs = (ec.flags & FSMI_F_RLE_RUNS) != 0;
  const size_t lds = fp64 ? rle_lds<double>(a.cap, with_runs) : rle_lds<float>(a.cap, with_runs);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reset_counter64, dim3(1), dim3(64), 0, ctx->stream, a.counter);
  const int per_cu = std::max<int>(1, std::min<int>(16, (int)((160 * 1024) / (lds + 256))));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_items, (int64_t)ctx->num_cu * per_cu));
  auto launch = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), lds, ctx->stream, a);
  };
  const bool runs = (ec.flags & FSMI_F_RLE_RUNS) != 0;
  if (fp64) {
    if (runs) launch(k_poses3d_runs_f64);
    else launch(k_poses3d_f64);
  } else {
    if (runs) launch(k_poses3d_runs_f32);
    else launch(k_poses3d_f32);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_pose_reduce(ctx, mb, n_poses, n_beams, mi_pose);
}

}  // namespace fsmi
