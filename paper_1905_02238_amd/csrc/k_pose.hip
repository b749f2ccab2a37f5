// k_pose.hip -- fsmi_eval_poses on 2D grids: the fused hot path.
//
// One wave per (pose, beam) item, popped from an atomic queue (items of one
// pose are adjacent, so neighbouring waves gather from the same map region).
// Per item: rotate the sensor direction by the pose's yaw, walk the grid
// (ray_dev.h) straight into LDS -- entry distances l_i and the gathered o_i --
// then evaluate the beam (beam_dev.h).  The per-beam MI goes to mi_beam (or a
// scratch array) and a second kernel sums each pose's beams in a fixed order
// in FP64 (Sec. 2.4: a scan's MI is the sum over its beams).
#include <math.h>

#include <algorithm>

#include "beam_dev.h"
#include "csqmi_dev.h"
#include "fsmi_internal.h"
#include "lut_dev.h"
#include "ray_dev.h"

namespace fsmi {
namespace {

struct Pose2dArgs {
  EvalConst ec;
  const float* map;
  int64_t X, Y;
  int64_t n_poses, n_beams;
  const double* poses;     // [n][4] x, y, cos, sin
  const double* beam_dir;  // [n][2]
  double sigma, R;
  int capa, ecap;
  double* mi_beam;         // [n_poses][n_beams]
  int32_t* counter;        // item queue head
  uint32_t* status;
  const float2* lut;       // the look-up tables in global memory (LUT mode)
};

// LDS of one wave: region 1 = the walk's tie counts, reused for C (and, in
// FP64, P) after the walk; region 2 = l (FP64 [ecap+1]) and o (FP32 [ecap]).
// In FP32, P(e_j) overwrites o in place (each lane reads o_i and writes P_i at
// the same index, and o is not read again).  The walk recomputes face times
// instead of storing them.
template <typename T>
__host__ __device__ inline size_t pose2d_region1(int capa, int ecap) {
  const size_t walk = (size_t)(capa + 1) * 4;
  const size_t cp = (sizeof(T) == 4 ? 1 : 2) * sizeof(T) * (size_t)ecap;
  return ((walk > cp ? walk : cp) + 15) / 16 * 16;
}
template <typename T>
__host__ __device__ inline size_t pose2d_lds(int capa, int ecap) {
  return pose2d_region1<T>(capa, ecap) + 8 * (size_t)(ecap + 1) + 4 * (size_t)ecap + 16;
}

// Waves per workgroup: one, or in the look-up-table mode four, which share one
// copy of the tables in LDS ahead of their own regions.
template <bool LUT> constexpr int pose2d_waves() { return LUT ? 4 : 1; }
template <bool LUT> constexpr size_t pose2d_shared() { return LUT ? kLutBytes : 0; }
template <typename T>
__host__ __device__ inline size_t pose2d_wave_bytes(int capa, int ecap) {
  return (pose2d_lds<T>(capa, ecap) + 15) / 16 * 16;
}

template <typename T, bool CSQ, bool LUT>
__global__ __launch_bounds__(kWave* pose2d_waves<LUT>()) void k_poses2d(Pose2dArgs a) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) char lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if constexpr (LUT) {
    lut_stage(reinterpret_cast<float2*>(lds), a.lut, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  char* r1 = lds + pose2d_shared<LUT>() + (size_t)wave * pose2d_wave_bytes<T>(a.capa, a.ecap);
  int* tie = reinterpret_cast<int*>(r1);
  double* sL = reinterpret_cast<double*>(r1 + pose2d_region1<T>(a.capa, a.ecap));
  float* so = reinterpret_cast<float*>(sL + a.ecap + 1);
  const int64_t n_items = a.n_poses * a.n_beams;
  // runs of items from the queue (guided self-scheduling); k, start and the
  // loop bounds are wave-uniform
  const int64_t n_waves = (int64_t)gridDim.x * pose2d_waves<LUT>();
  int64_t k = run_length(n_items, 0, n_waves);
  for (int64_t start = wave_take64(a.counter, k); start < n_items;
       start = wave_take64(a.counter, k)) {
    const int64_t it_end = min<int64_t>(start + k, n_items);
    k = run_length(n_items, it_end, n_waves);
    for (int64_t it = start; it < it_end; ++it) {
      const int64_t p = it / a.n_beams, b = it - p * a.n_beams;
      const double* ps = a.poses + 4 * p;
      const double bx = a.beam_dir[2 * b], by = a.beam_dir[2 * b + 1];
      const double m1 = ps[2] * bx, m2 = ps[3] * by, m3 = ps[3] * bx, m4 = ps[2] * by;
      const double dx = m1 - m2, dy = m3 + m4;
      const float* map = a.map;
      // the walk records entry distances and cell indices (in o's slots); the
      // occupancies are gathered afterwards, several loads in flight per lane
      int* sc = reinterpret_cast<int*>(so);
      auto emit = [&](int r, double t, int c) {
        sL[r + 1] = t > 0.0 ? t : 0.0;
        sc[r + 1] = c;
      };
      const Dda2dResult res =
          dda2d_wave(a.X, a.Y, ps[0], ps[1], dx, dy, a.R, a.capa, a.ecap, tie, emit, lane);
      double v;
      if (res.n < 0) {
        v = __builtin_nan("");
        if (lane == 0) latch(a.status, res.n == -1 ? kErrPose : kErrCap);
      } else {
        // cells 1 .. skip0 + n - 1 were entered by events before the walk's end
        const int hi = res.skip0 + res.n;
        for (int base = 1; base < hi; base += 4 * kWave) {
          int c[4];
          float o[4];
  #pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = base + u * kWave + lane;
            c[u] = i < hi ? sc[i] : -1;
          }
  #pragma unroll
          for (int u = 0; u < 4; ++u) o[u] = map[c[u] >= 0 ? c[u] : 0];
  #pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = base + u * kWave + lane;
            if (i < hi) so[i] = c[u] >= 0 ? o[u] : 0.0f;
          }
        }
        if (lane == 0) {
          sL[0] = 0.0;
          so[0] = map[res.cell0];
          sL[res.skip0 + res.n] = res.lend;
        }
        wave_sync();
        CoreLds L;
        L.A = sL + res.skip0;
        L.C = r1;
        L.P = sizeof(T) == 4 ? reinterpret_cast<void*>(so + res.skip0)
                             : reinterpret_cast<void*>(r1 + sizeof(T) * (size_t)a.ecap);
        if constexpr (LUT) L.lut = reinterpret_cast<const float2*>(lds);
        bool bad;
        v = beam_eval<1, false, T, CSQ, LUT>(a.ec, res.n, so + res.skip0, true, a.sigma, L, nullptr,
                                             nullptr, lane, false, &bad);
        if (bad && lane == 0) latch(a.status, kErrOcc);
      }
      if (lane == 0) a.mi_beam[it] = v;
      wave_sync();
    }
  }
}

// The look-up tables of lut_dev.h, computed in FP64 and rounded to FP32.
__global__ __launch_bounds__(256) void k_build_lut(double delta_occ, float2* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kLutPhiN) {
    const double s = (double)kInvSqrtL2E / (double)kLutInvH;   // table step in erfc's argument
    const double e0 = erfc(i * s);
    const double e1 = i + 1 < kLutPhiN ? erfc((i + 1) * s) : 0.0;
    out[i] = make_float2((float)e0, (float)(e1 - e0));
  } else if (i == kLutPhiN) {
    out[i] = make_float2(0.0f, 0.0f);
  } else if (i < kLutEntries) {
    const int k = i - kLutPhiN - 1;
    const double ld = log(delta_occ);
    const double h = 1.0 / (kLutFN - 1);
    const double f0 = f_cell<double>(delta_occ, ld, k * h);
    const double f1 = k + 1 < kLutFN ? f_cell<double>(delta_occ, ld, fmin(1.0, (k + 1) * h)) : f0;
    out[i] = make_float2((float)f0, (float)(f1 - f0));
  }
}

// mi_pose[p] = sum_b mi_beam[p][b], one wave per pose, fixed-order FP64 tree.
__global__ __launch_bounds__(kWave) void k_pose_reduce(const double* mi_beam, int64_t n_poses,
                                                       int64_t n_beams, double* mi_pose) {
  const int lane = threadIdx.x;
  for (int64_t p = blockIdx.x; p < n_poses; p += gridDim.x) {
    double s = 0.0;
    for (int64_t b = lane; b < n_beams; b += kWave) s += mi_beam[p * n_beams + b];
    s = wave_sum(s);
    if (lane == 0) mi_pose[p] = s;
  }
}

__global__ void k_reset_counter(int32_t* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

}  // namespace

size_t lut_bytes() { return kLutBytes; }

hipError_t launch_build_lut(hipStream_t st, double delta_occ, void* out) {
  const int n = kLutEntries;
  hipLaunchKernelGGL(k_build_lut, dim3((n + 255) / 256), dim3(256), 0, st, delta_occ,
                     reinterpret_cast<float2*>(out));
  return hipGetLastError();
}

hipError_t launch_pose_reduce(fsmi_ctx ctx, const double* mi_beam, int64_t n_poses,
                              int64_t n_beams, double* mi_pose) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_poses, 8192));
  hipLaunchKernelGGL(k_pose_reduce, dim3(grid), dim3(kWave), 0, ctx->stream, mi_beam, n_poses,
                     n_beams, mi_pose);
  return hipGetLastError();
}

hipError_t launch_eval_poses_2d(fsmi_ctx ctx, const EvalConst& ec, const float* map, int64_t X,
                                int64_t Y, int64_t n_poses, const double* poses, int64_t n_beams,
                                const double* beam_dir, double sigma, double R, double* mi_pose,
                                double* mi_beam, const PoseScratch* ws) {
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
  Pose2dArgs a;
  a.ec = ec;
  a.map = map;
  a.X = X;
  a.Y = Y;
  a.n_poses = n_poses;
  a.n_beams = n_beams;
  a.poses = poses;
  a.beam_dir = beam_dir;
  a.sigma = sigma;
  a.R = R;
  a.capa = dda2d_axis_cap(R);
  a.ecap = dda2d_event_cap(R);
  a.mi_beam = mb;
  a.counter = ws ? ws->counter : ctx->d_counters + 8;   // 64-bit head (counters[8..9])
  a.status = ctx->d_status;
  a.lut = reinterpret_cast<const float2*>(ctx->d_lut);
  const bool fp64 = ec.precision == FSMI_FP64;
  const bool lut = (ec.flags & FSMI_F_LUT) != 0;
  if (lut && (fp64 || ec.variant == FSMI_CSQMI)) return hipErrorInvalidValue;
  if (lut) {
    hipError_t e = launch_build_lut(ctx->stream, ec.delta_occ, ctx->d_lut);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, ctx->stream, a.counter);
  const size_t wb = fp64 ? pose2d_wave_bytes<double>(a.capa, a.ecap)
                         : pose2d_wave_bytes<float>(a.capa, a.ecap);
  const int waves = lut ? pose2d_waves<true>() : pose2d_waves<false>();
  const size_t lds = (lut ? pose2d_shared<true>() : 0) + (size_t)waves * wb;
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  const int per_cu = std::max<int>(1, std::min<int>(16 / waves, (int)((160 * 1024) / (lds + 256))));
  const int64_t groups = (n_items + waves - 1) / waves;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)ctx->num_cu * per_cu));
  auto launch = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * waves), lds, ctx->stream, a);
  };
  const bool csq = ec.variant == FSMI_CSQMI;
  if (fp64) {
    if (csq) launch(k_poses2d<double, true, false>);
    else launch(k_poses2d<double, false, false>);
  } else if (lut) {
    launch(k_poses2d<float, false, true>);
  } else {
    if (csq) launch(k_poses2d<float, true, false>);
    else launch(k_poses2d<float, false, false>);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_pose_reduce(ctx, mb, n_poses, n_beams, mi_pose);
}

}  // namespace fsmi
