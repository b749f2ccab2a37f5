// k_ray.hip -- fsmi_raycast: beam cell lists (2D grid walk) and 3D virtual
// cells / runs, one wave per ray, results written to caller buffers.
#include <math.h>

#include "fsmi_internal.h"
#include "ray_dev.h"

namespace fsmi {
namespace {

// LDS of the walk: ev [ecap] FP64, pc [ecap] int, tie [capa + 1] int.
static inline size_t raycast2d_lds(int capa, int ecap) {
  return (size_t)ecap * 8 + (size_t)ecap * 4 + (size_t)(capa + 1) * 4 + 16;
}

__global__ __launch_bounds__(kWave) void k_raycast2d(const float* __restrict__ map, int64_t X,
                                                     int64_t Y, int64_t n_rays,
                                                     const double* __restrict__ origin,
                                                     const double* __restrict__ dir, double R,
                                                     int capa, int ecap, int max_cells,
                                                     int32_t* count, int32_t* cell, double* entry,
                                                     float* occ_out, uint32_t* status) {
  extern __shared__ __align__(16) char lds[];
  double* ev = reinterpret_cast<double*>(lds);
  int* pc = reinterpret_cast<int*>(ev + ecap);
  int* tie = pc + ecap;
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n_rays; r += gridDim.x) {
    auto emit = [&](int rank, double t, int c) {
      ev[rank] = t;
      pc[rank] = c;
    };
    const Dda2dResult res = dda2d_wave(X, Y, origin[2 * r], origin[2 * r + 1], dir[2 * r],
                                       dir[2 * r + 1], R, capa, ecap, tie, emit, lane);
    if (res.n < 0 || res.n > max_cells) {
      if (lane == 0) {
        count[r] = res.n < 0 ? res.n : -2;
        latch(status, res.n == -1 ? kErrPose : kErrCap);
      }
      wave_sync();
      continue;
    }
    for (int q = lane; cell != nullptr && q < res.n; q += kWave) {
      const int k = q + res.skip0;
      int c;
      double e;
      if (k == 0) {
        c = (int)res.cell0;
        e = 0.0;
      } else {
        c = pc[k - 1];
        const double t = ev[k - 1];
        e = t > 0.0 ? t : 0.0;
      }
      cell[r * max_cells + q] = c;
      entry[r * (int64_t)(max_cells + 1) + q] = e;
      if (occ_out) occ_out[r * max_cells + q] = map[c];
    }
    if (lane == 0) {
      count[r] = res.n;
      if (entry) entry[r * (int64_t)(max_cells + 1) + res.n] = res.lend;
    }
    wave_sync();
  }
}

__global__ __launch_bounds__(kWave) void k_virtual3d(const float* __restrict__ map, int64_t X,
                                                     int64_t Y, int64_t Z, int64_t n_rays,
                                                     const double* __restrict__ origin,
                                                     const double* __restrict__ dir, double R,
                                                     double w, int max_cells, int rle,
                                                     int32_t* count, int32_t* cell, float* occ_out,
                                                     int32_t* run_len, uint32_t* status) {
  extern __shared__ __align__(16) char lds[];
  float* so = reinterpret_cast<float*>(lds);
  int* sc = reinterpret_cast<int*>(so + max_cells);
  float* ro = reinterpret_cast<float*>(sc + max_cells);
  int* rl = reinterpret_cast<int*>(ro + max_cells);
  int* rs = rl + max_cells;
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n_rays; r += gridDim.x) {
    bool ok;
    const int n = virtual3d_wave(map, X, Y, Z, origin + 3 * r, dir + 3 * r, R, w, max_cells, so, sc,
                                 lane, &ok);
    if (!ok) {
      if (lane == 0) {
        count[r] = -1;
        latch(status, kErrPose);
      }
      continue;
    }
    wave_sync();
    if (!rle) {
      for (int q = lane; q < n; q += kWave) {
        if (cell) cell[r * max_cells + q] = sc[q];
        if (occ_out) occ_out[r * max_cells + q] = so[q];
      }
      if (lane == 0) count[r] = n;
    } else {
      const int nr = runs_wave(so, n, ro, rl, rs, lane);
      for (int q = lane; q < nr; q += kWave) {
        if (occ_out) occ_out[r * max_cells + q] = ro[q];
        if (run_len) run_len[r * max_cells + q] = rl[q];
        if (cell) cell[r * max_cells + q] = sc[rs[q]];
      }
      if (lane == 0) count[r] = nr;
    }
    wave_sync();
  }
}

}  // namespace

hipError_t launch_raycast2d(fsmi_ctx ctx, const float* map, int64_t X, int64_t Y, int64_t n_rays,
                            const double* origin, const double* dir, double R, int max_cells,
                            int32_t* count, int32_t* cell, double* entry, float* occ_out) {
  if (n_rays <= 0) return hipSuccess;
  const int capa = dda2d_axis_cap(R);
  const int ecap = dda2d_event_cap(R);
  const size_t lds = raycast2d_lds(capa, ecap);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(n_rays, 65536);
  hipLaunchKernelGGL(k_raycast2d, dim3(grid), dim3(kWave), lds, ctx->stream, map, X, Y, n_rays,
                     origin, dir, R, capa, ecap, max_cells, count, cell, entry, occ_out,
                     ctx->d_status);
  return hipGetLastError();
}

hipError_t launch_virtual3d(fsmi_ctx ctx, const float* map, int64_t X, int64_t Y, int64_t Z,
                            int64_t n_rays, const double* origin, const double* dir, double R,
                            double w, int max_cells, int rle, int32_t* count, int32_t* cell,
                            float* occ_out, int32_t* run_len) {
  if (n_rays <= 0) return hipSuccess;
  const size_t lds = (size_t)max_cells * 20;
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(n_rays, 65536);
  hipLaunchKernelGGL(k_virtual3d, dim3(grid), dim3(kWave), lds, ctx->stream, map, X, Y, Z, n_rays,
                     origin, dir, R, w, max_cells, rle, count, cell, occ_out, run_len,
                     ctx->d_status);
  return hipGetLastError();
}

}  // namespace fsmi
