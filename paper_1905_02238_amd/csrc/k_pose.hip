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

template <typename T, bool CSQ>
__global__ __launch_bounds__(kWave) void k_poses2d(Pose2dArgs a) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) char lds[];
  const int lane = threadIdx.x;
  char* r1 = lds;
  int* tie = reinterpret_cast<int*>(r1);
  double* sL = reinterpret_cast<double*>(lds + pose2d_region1<T>(a.capa, a.ecap));
  float* so = reinterpret_cast<float*>(sL + a.ecap + 1);
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
        bool bad;
        v = beam_eval<1, false, T, CSQ>(a.ec, res.n, so + res.skip0, true, a.sigma, L, nullptr, nullptr,
                                   lane, false, &bad);
        if (bad && lane == 0) latch(a.status, kErrOcc);
      }
      if (lane == 0) a.mi_beam[it] = v;
      wave_sync();
    }
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
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, ctx->stream, a.counter);
  const bool fp64 = ec.precision == FSMI_FP64;
  const size_t lds = fp64 ? pose2d_lds<double>(a.capa, a.ecap) : pose2d_lds<float>(a.capa, a.ecap);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  const int per_cu = std::max<int>(1, std::min<int>(16, (int)((160 * 1024) / (lds + 256))));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_items, (int64_t)ctx->num_cu * per_cu));
  auto launch = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), lds, ctx->stream, a);
  };
  const bool csq = ec.variant == FSMI_CSQMI;
  if (fp64) {
    if (csq) launch(k_poses2d<double, true>);
    else launch(k_poses2d<double, false>);
  } else {
    if (csq) launch(k_poses2d<float, true>);
    else launch(k_poses2d<float, false>);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_pose_reduce(ctx, mb, n_poses, n_beams, mi_pose);
}

}  // namespace fsmi
