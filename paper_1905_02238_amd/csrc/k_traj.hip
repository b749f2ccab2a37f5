// k_traj.hip -- trajectory MI with cell marking on 2D grids (Sec. 2.4):
// fsmi_eval_trajectories.
//
// A candidate trajectory is a sequence of states (2D poses) in travel order;
// its MI is the sum of its states' scan MI, with each cell's information
// counted only at the first state whose beams cross it.  The host reads the
// CSR offsets once, sets aside trajectories whose offsets are invalid (their
// MI is NaN and the call latches), and evaluates the rest in groups of up to
// G trajectories, G stamp maps side by side (G from a 1 GiB budget, at most
// 64).  Each group takes two persistent passes of one wave per (state, beam)
// item of all its trajectories:
//   1. stamp: walk every beam and raise the cell's 64-bit stamp in its
//      trajectory's map to (k << 32) | (2^32 - 1 - t) with an atomic max, so
//      after the pass a cell crossed by trajectory k holds k and the first
//      state t that crosses it (a later trajectory in the same slot has a
//      larger k, so the maps are cleared once per call, not per group);
//   2. evaluate: walk again, gather o and mark cell i counted iff its stamp
//      names this state, and run the beam engine with that mask (the f terms
//      of uncounted cells leave C_k; every cell still shapes P(e_j)).
// Per-state MI is the fixed-order FP64 sum of its beams, per-trajectory MI
// the fixed-order FP64 sum of its states.
#include <math.h>

#include <algorithm>
#include <vector>

#include "beam_dev.h"
#include "fsmi_internal.h"
#include "ray_dev.h"

namespace fsmi {
// Stamp maps side by side: at most kTrajSlots trajectories per group, within
// kStampBudget bytes of maps.
constexpr int64_t kTrajSlots = 64;
constexpr int64_t kStampBudget = (int64_t)1 << 30;
hipError_t launch_pose_reduce(fsmi_ctx ctx, const double* mi_beam, int64_t n_poses,
                              int64_t n_beams, double* mi_pose);
namespace {

// A group's table: record j < ng = {trajectory k, first state s0, states,
// items before slot j}; record ng holds the group's item count in its last
// field.
struct TrajArgs {
  EvalConst ec;
  const float* map;
  int64_t X, Y;
  const int64_t* gtab;       // [(ng + 1) * 4], device
  int ng;
  int64_t n_states, n_beams;
  const double* poses;       // [n_states][4] x, y, cos, sin
  const double* beam_dir;    // [n_beams][2]
  double sigma, R;
  int capa, ecap;
  unsigned long long* stamp; // [G][X * Y]: slot j of the group uses map j
  double* mi_beam;           // [n_states][n_beams]
  int32_t* counter;          // 64-bit queue head
  uint32_t* status;
};

// LDS of one wave: region 1 = the walk's tie counts, reused for C (and, in
// FP64, P); then l (FP64 [ecap + 1]), o (FP32 [ecap]; P in FP32 overwrites it
// in place) and the counted mask (bytes [ecap]).
template <typename T>
__host__ __device__ inline size_t traj_region1(int capa, int ecap) {
  const size_t walk = (size_t)(capa + 1) * 4;
  const size_t cp = (sizeof(T) == 4 ? 1 : 2) * sizeof(T) * (size_t)ecap;
  return ((walk > cp ? walk : cp) + 15) / 16 * 16;
}
template <typename T>
__host__ __device__ inline size_t traj_lds(int capa, int ecap) {
  return traj_region1<T>(capa, ecap) + 8 * (size_t)(ecap + 1) + 4 * (size_t)ecap + (size_t)ecap + 32;
}

// A value every lane loaded from the same address, as a wave-uniform scalar.
FSMI_DEV int64_t uniform_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

FSMI_DEV unsigned long long traj_key(int64_t k, int64_t t) {
  return ((unsigned long long)k << 32) | (unsigned long long)(0xffffffffu - (uint32_t)t);
}

template <typename T, bool STAMP>
__global__ __launch_bounds__(kWave) void k_traj2d(TrajArgs a) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) char lds[];
  const int lane = threadIdx.x;
  char* r1 = lds;
  int* tie = reinterpret_cast<int*>(r1);
  double* sL = reinterpret_cast<double*>(lds + traj_region1<T>(a.capa, a.ecap));
  float* so = reinterpret_cast<float*>(sL + a.ecap + 1);
  unsigned char* sm = reinterpret_cast<unsigned char*>(so + a.ecap);
  const int64_t n_items = uniform_i64(a.gtab[4 * a.ng + 3]);
  const int64_t n_waves = gridDim.x;
  int64_t kr = run_length(n_items, 0, n_waves);
  for (int64_t start = wave_take64(a.counter, kr); start < n_items;
       start = wave_take64(a.counter, kr)) {
    const int64_t it_end = min<int64_t>(start + kr, n_items);
    kr = run_length(n_items, it_end, n_waves);
    for (int64_t it = start; it < it_end; ++it) {
      // the item's slot: the last record whose item prefix is <= it
      int lo = 0, hi = a.ng;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (uniform_i64(a.gtab[4 * mid + 3]) <= it) lo = mid;
        else hi = mid;
      }
      const int64_t k = uniform_i64(a.gtab[4 * lo]);
      const int64_t s0 = uniform_i64(a.gtab[4 * lo + 1]);
      const int64_t local = it - uniform_i64(a.gtab[4 * lo + 3]);
      const int64_t t = local / a.n_beams, b = local - t * a.n_beams;
      unsigned long long* stamp = a.stamp + (int64_t)lo * a.X * a.Y;
      const double* ps = a.poses + 4 * (s0 + t);
      const double bx = a.beam_dir[2 * b], by = a.beam_dir[2 * b + 1];
      const double m1 = ps[2] * bx, m2 = ps[3] * by, m3 = ps[3] * bx, m4 = ps[2] * by;
      const double dx = m1 - m2, dy = m3 + m4;
      int* sc = reinterpret_cast<int*>(so);
      auto emit = [&](int r, double tt, int c) {
        sL[r + 1] = tt > 0.0 ? tt : 0.0;
        sc[r + 1] = c;
      };
      const Dda2dResult res =
          dda2d_wave(a.X, a.Y, ps[0], ps[1], dx, dy, a.R, a.capa, a.ecap, tie, emit, lane);
      const unsigned long long key = traj_key(k, t);
      if constexpr (STAMP) {
        if (res.n < 0) {
          if (lane == 0) latch(a.status, res.n == -1 ? kErrPose : kErrCap);
        } else {
          // the beam's cells: the origin cell (index 0) unless it has zero
          // length, then the cells entered by events 1 .. skip0 + n - 1
          const int hi = res.skip0 + res.n;
          for (int i = res.skip0 + lane; i < hi; i += kWave) {
            const int64_t c = i == 0 ? res.cell0 : (int64_t)sc[i];
            if (c >= 0) atomicMax(&stamp[c], key);
          }
        }
        wave_sync();
      } else {
        double v;
        if (res.n < 0) {
          v = __builtin_nan("");
        } else {
          const int hi = res.skip0 + res.n;
          for (int base = 1; base < hi; base += 4 * kWave) {
            int c[4];
            float o[4];
            unsigned long long st[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = base + u * kWave + lane;
              c[u] = i < hi ? sc[i] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              o[u] = a.map[c[u] >= 0 ? c[u] : 0];
              st[u] = stamp[c[u] >= 0 ? c[u] : 0];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = base + u * kWave + lane;
              if (i < hi) {
                so[i] = c[u] >= 0 ? o[u] : 0.0f;
                sm[i] = (c[u] >= 0 && st[u] == key) ? 1 : 0;
              }
            }
          }
          if (lane == 0) {
            sL[0] = 0.0;
            so[0] = a.map[res.cell0];
            sm[0] = stamp[res.cell0] == key ? 1 : 0;
            sL[res.skip0 + res.n] = res.lend;
          }
          wave_sync();
          CoreLds L;
          L.A = sL + res.skip0;
          L.C = r1;
          L.P = sizeof(T) == 4 ? reinterpret_cast<void*>(so + res.skip0)
                               : reinterpret_cast<void*>(r1 + sizeof(T) * (size_t)a.ecap);
          bool bad;
          v = beam_core<1, false, T, true>(a.ec, res.n, so + res.skip0, true, a.sigma, L, nullptr,
                                           nullptr, lane, false, &bad, sm + res.skip0);
          if (bad && lane == 0) latch(a.status, kErrOcc);
        }
        if (lane == 0) a.mi_beam[(s0 + t) * a.n_beams + b] = v;
        wave_sync();
      }
    }
  }
}

__global__ void k_latch(uint32_t* status, uint32_t bits) {
  if (threadIdx.x == 0) latch(status, bits);
}

__global__ void k_traj_reset64(int32_t* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

__global__ void k_fill_u64(int64_t n, unsigned long long* p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// mi_traj[k] = sum of mi_state over the trajectory's states, one wave per
// trajectory, fixed-order FP64 tree.
__global__ __launch_bounds__(kWave) void k_traj_reduce(const double* mi_state,
                                                       const int64_t* traj_off, int64_t n_traj,
                                                       int64_t n_states, double* mi_traj) {
  const int lane = threadIdx.x;
  for (int64_t k = blockIdx.x; k < n_traj; k += gridDim.x) {
    const int64_t s0 = traj_off[k], s1 = traj_off[k + 1];
    double s = 0.0;
    if (s0 >= 0 && s1 >= s0 && s1 <= n_states) {
      for (int64_t t = s0 + lane; t < s1; t += kWave) s += mi_state[t];
      s = wave_sum(s);
    } else {
      s = __builtin_nan("");
    }
    if (lane == 0) mi_traj[k] = s;
  }
}

}  // namespace

hipError_t launch_eval_trajectories_2d(fsmi_ctx ctx, const EvalConst& ec, const float* map,
                                       int64_t X, int64_t Y, int64_t n_traj,
                                       const int64_t* traj_off, int64_t n_states,
                                       const double* poses, int64_t n_beams,
                                       const double* beam_dir, double sigma, double R,
                                       double* mi_traj, double* mi_state, double* mi_beam) {
  if (n_traj <= 0) return hipSuccess;
  // the offsets, read once: the groups are laid out on the host
  std::vector<int64_t> off((size_t)n_traj + 1);
  hipError_t e = hipMemcpyAsync(off.data(), traj_off, sizeof(int64_t) * off.size(),
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return e;
  std::vector<int64_t> valid;
  bool any_bad = false;
  for (int64_t k = 0; k < n_traj; ++k) {
    if (off[k] >= 0 && off[k + 1] >= off[k] && off[k + 1] <= n_states) valid.push_back(k);
    else any_bad = true;
  }
  const int64_t cells = X * Y;
  const int64_t G = std::max<int64_t>(1, std::min<int64_t>({kTrajSlots, (kStampBudget / 8) / cells,
                                                            (int64_t)valid.size()}));
  const int64_t n_groups = ((int64_t)valid.size() + G - 1) / G;
  // group tables: (G + 1) records of 4 per group
  std::vector<int64_t> tab((size_t)std::max<int64_t>(n_groups, 1) * (G + 1) * 4, 0);
  for (int64_t gi = 0; gi < n_groups; ++gi) {
    int64_t* rec = tab.data() + gi * (G + 1) * 4;
    const int64_t j0 = gi * G, j1 = std::min<int64_t>(j0 + G, (int64_t)valid.size());
    int64_t items = 0;
    for (int64_t j = j0; j < j1; ++j) {
      const int64_t k = valid[(size_t)j];
      int64_t* r = rec + (j - j0) * 4;
      r[0] = k;
      r[1] = off[k];
      r[2] = off[k + 1] - off[k];
      r[3] = items;
      items += r[2] * n_beams;
    }
    rec[(j1 - j0) * 4 + 3] = items;
  }
  // work area: G stamp maps, the per-beam and per-state sums the caller does
  // not keep, the group tables; each on a 256-byte boundary
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t stamp_b = up((size_t)G * (size_t)cells * 8);
  const size_t beam_b = mi_beam ? 0 : up((size_t)n_states * (size_t)n_beams * 8);
  const size_t state_b = mi_state ? 0 : up((size_t)n_states * 8);
  const size_t tab_b = up(tab.size() * 8);
  e = ensure_work(ctx, stamp_b + beam_b + state_b + tab_b + 256);
  if (e != hipSuccess) return e;
  char* w = reinterpret_cast<char*>(ctx->d_work);
  int64_t* d_tab = reinterpret_cast<int64_t*>(w + stamp_b + beam_b + state_b);
  e = hipMemcpyAsync(d_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return e;
  TrajArgs a;
  a.ec = ec;
  a.map = map;
  a.X = X;
  a.Y = Y;
  a.n_states = n_states;
  a.n_beams = n_beams;
  a.poses = poses;
  a.beam_dir = beam_dir;
  a.sigma = sigma;
  a.R = R;
  a.capa = dda2d_axis_cap(R);
  a.ecap = dda2d_event_cap(R);
  a.stamp = reinterpret_cast<unsigned long long*>(w);
  a.mi_beam = mi_beam ? mi_beam : reinterpret_cast<double*>(w + stamp_b);
  double* ms = mi_state ? mi_state : reinterpret_cast<double*>(w + stamp_b + beam_b);
  a.counter = ctx->d_counters + 8;
  a.status = ctx->d_status;
  const bool fp64 = ec.precision == FSMI_FP64;
  const size_t lds = fp64 ? traj_lds<double>(a.capa, a.ecap) : traj_lds<float>(a.capa, a.ecap);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  const int per_cu = std::max<int>(1, std::min<int>(16, (int)((160 * 1024) / (lds + 256))));
  const int grid = std::max(1, ctx->num_cu * per_cu);
  if (any_bad) hipLaunchKernelGGL(k_latch, dim3(1), dim3(64), 0, ctx->stream, a.status, kErrLen);
  // per-state sums of states no valid trajectory reaches stay zero
  if (n_states > 0) {
    e = launch_fill_f64(ctx->stream, n_states * n_beams, 0.0, a.mi_beam);
    if (e != hipSuccess) return e;
  }
  {
    const int64_t n = G * cells;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(256), 0, ctx->stream, n, a.stamp);
  }
  auto launch = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_traj_reset64, dim3(1), dim3(64), 0, ctx->stream, a.counter);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), lds, ctx->stream, a);
  };
  for (int64_t gi = 0; gi < n_groups; ++gi) {
    a.gtab = d_tab + gi * (G + 1) * 4;
    a.ng = (int)(std::min<int64_t>((gi + 1) * G, (int64_t)valid.size()) - gi * G);
    if (fp64) {
      launch(k_traj2d<double, true>);
      launch(k_traj2d<double, false>);
    } else {
      launch(k_traj2d<float, true>);
      launch(k_traj2d<float, false>);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_states > 0) {
    e = launch_pose_reduce(ctx, a.mi_beam, n_states, n_beams, ms);
    if (e != hipSuccess) return e;
  }
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>(n_traj, 8192));
  hipLaunchKernelGGL(k_traj_reduce, dim3(g), dim3(kWave), 0, ctx->stream, ms, traj_off, n_traj,
                     n_states, mi_traj);
  return hipGetLastError();
}

}  // namespace fsmi
