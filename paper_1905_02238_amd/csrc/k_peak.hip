// k_peak.hip -- the library's own microbenchmarks of the chip's ceilings, so
// that each path can be reported against a measured roof as well as against
// the published one: a plain HBM copy, scalar FP32 FMA issue, one erfc plus
// one FMA per pair with operands in registers (the Phi-pair ceiling of the
// exact double sum), and dense BF16 matrix-core products.
#include <hip/hip_runtime.h>

#include "fsmi_dev.h"
#include "fsmi_internal.h"

namespace fsmi {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Lane 0 of every wave adds its shader cycles and its constant-rate wall-clock
// ticks since (c0, w0) to acc[0], acc[1]: their ratio gives the shader clock
// the waves ran at.
__device__ inline void clock_note(unsigned long long* acc, long long c0, long long w0) {
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicAdd(acc, (unsigned long long)(clock64() - c0));
    atomicAdd(acc + 1, (unsigned long long)(wall_clock64() - w0));
  }
}

typedef float f4v_ __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_fill_f4(f4v_* p, int64_t n, float v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = f4v_{v, v, v, v};
}

// Non-temporal loads and stores: the copy streams through without filling the
// caches (the fastest form measured on this chip, about 5.9 TB/s).
typedef float f4v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_f4(const f4v* __restrict__ src, f4v* __restrict__ dst,
                                                 int64_t n, unsigned long long* clk) {
  const long long c0 = clock64(), w0 = wall_clock64();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  clock_note(clk, c0, w0);
}

// Eight independent FMA chains per lane; m and c arrive as arguments so the
// compiler cannot fold them.
constexpr int kFmaChains = 8;
__global__ __launch_bounds__(256) void k_fma_peak(int iters, float m, float c, float* out,
                                                  unsigned long long* clk) {
  const long long c0 = clock64(), w0 = wall_clock64();
  float a[kFmaChains];
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) a[k] = threadIdx.x * 1e-3f + k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) a[k] = fmaf(a[k], m, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) s += a[k];
  out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
  clock_note(clk, c0, w0);
}

// The Phi-pair ceiling: per pair one FP32 erfc of the library (erfc_pos_l2)
// and one FMA into an accumulator, the argument in a register (an FMA keeps it
// bounded), eight independent pairs per lane in flight.
constexpr int kPhiChains = 8;
__global__ __launch_bounds__(256) void k_phi_peak(int iters, float c, float* out,
                                                  unsigned long long* clk) {
  const long long c0 = clock64(), w0 = wall_clock64();
  float y[kPhiChains], acc[kPhiChains];
#pragma unroll
  for (int k = 0; k < kPhiChains; ++k) {
    y[k] = 0.25f * k + threadIdx.x * 1e-3f;
    acc[k] = 0.0f;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kPhiChains; ++k) {
      acc[k] = fmaf(c, erfc_pos_l2(y[k]), acc[k]);
      y[k] = fmaf(y[k], 0.999f, 0.0037f);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kPhiChains; ++k) s += acc[k];
  out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
  clock_note(clk, c0, w0);
}

// Four independent accumulators of v_mfma_f32_16x16x32_bf16 per wave (named
// variables: an array of accumulators makes the compiler rotate registers
// inside the loop).
constexpr int kMfmaAcc = 4;
__global__ __launch_bounds__(256) void k_mfma_peak(int iters, float* out, unsigned long long* clk) {
  const long long c0 = clock64(), w0 = wall_clock64();
  // distinct operands and starting values, so no two products are the same
  bf16x8 a, b0, b1, b2, b3;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = (__bf16)(0.001f * (float)(threadIdx.x + q));
    b0[q] = (__bf16)(0.002f * (float)q);
    b1[q] = (__bf16)(0.003f * (float)q);
    b2[q] = (__bf16)(0.004f * (float)q);
    b3[q] = (__bf16)(0.005f * (float)q);
  }
  floatx4 d0 = {0.0f, 0.0f, 0.0f, 0.0f}, d1 = {1.0f, 0.0f, 0.0f, 0.0f},
          d2 = {2.0f, 0.0f, 0.0f, 0.0f}, d3 = {3.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
    d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, d1, 0, 0, 0);
    d2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b2, d2, 0, 0, 0);
    d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b3, d3, 0, 0, 0);
  }
  const floatx4 d = d0 + d1 + d2 + d3;
  out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = d[0] + d[1] + d[2] + d[3];
  clock_note(clk, c0, w0);
}

// Mean seconds per launch of `launch` over `reps` launches after one warm one.
template <class F>
hipError_t time_launches(hipStream_t st, int reps, F launch, double* sec) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  launch();
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, st);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  *sec = (double)ms * 1e-3 / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

hipError_t run_peak(fsmi_ctx ctx, int kind, double* rate, double* clock_mhz) {
  hipStream_t st = ctx->stream;
  const int ncu = ctx->num_cu;
  double sec = 0.0;
  int wall_khz = 0;
  hipError_t e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ctx->device);
  if (e != hipSuccess) return e;
  unsigned long long* clk = nullptr;   // shader cycles, wall ticks
  e = hipMalloc(&clk, 2 * sizeof(unsigned long long));
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(clk, 0, 2 * sizeof(unsigned long long), st);
  void* buf[2] = {nullptr, nullptr};
  if (e == hipSuccess && kind == FSMI_PEAK_COPY) {
    const int64_t n = (int64_t)1 << 26;   // 16-byte vectors: 1 GiB per buffer
    e = hipMalloc(&buf[0], n * sizeof(f4v));
    if (e == hipSuccess) e = hipMalloc(&buf[1], n * sizeof(f4v));
    if (e == hipSuccess) {
      f4v* src = reinterpret_cast<f4v*>(buf[0]);
      f4v* dst = reinterpret_cast<f4v*>(buf[1]);
      const int grid = ncu * 4;
      hipLaunchKernelGGL(k_fill_f4, dim3(grid), dim3(256), 0, st, src, n, 1.0f);
      e = time_launches(st, 20, [&] {
        hipLaunchKernelGGL(k_copy_f4, dim3(grid), dim3(256), 0, st, src, dst, n, clk);
      }, &sec);
      if (e == hipSuccess) *rate = 2.0 * (double)n * sizeof(f4v) / sec;
    }
  } else if (e == hipSuccess) {
    const int grid = ncu * 8, threads = 256;
    e = hipMalloc(&buf[0], (size_t)grid * threads * sizeof(float));
    float* out = reinterpret_cast<float*>(buf[0]);
    if (e == hipSuccess && kind == FSMI_PEAK_FMA) {
      const int iters = 1 << 16;
      e = time_launches(st, 5, [&] {
        hipLaunchKernelGGL(k_fma_peak, dim3(grid), dim3(threads), 0, st, iters, 0.999f, 1e-3f, out,
                           clk);
      }, &sec);
      if (e == hipSuccess) *rate = 2.0 * kFmaChains * (double)iters * grid * threads / sec;
    } else if (e == hipSuccess && kind == FSMI_PEAK_PAIR) {
      const int iters = 1 << 13;
      e = time_launches(st, 5, [&] {
        hipLaunchKernelGGL(k_phi_peak, dim3(grid), dim3(threads), 0, st, iters, 0.01f, out, clk);
      }, &sec);
      if (e == hipSuccess) *rate = (double)kPhiChains * iters * grid * threads / sec;
    } else if (e == hipSuccess && kind == FSMI_PEAK_MFMA_BF16) {
      const int iters = 1 << 15;
      e = time_launches(st, 5, [&] {
        hipLaunchKernelGGL(k_mfma_peak, dim3(grid), dim3(threads), 0, st, iters, out, clk);
      }, &sec);
      const double waves = (double)grid * threads / kWave;
      if (e == hipSuccess) *rate = 2.0 * 16 * 16 * 32 * kMfmaAcc * (double)iters * waves / sec;
    } else if (e == hipSuccess) {
      e = hipErrorInvalidValue;
    }
  }
  unsigned long long h[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, clk, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && clock_mhz)
    *clock_mhz = h[1] ? (double)h[0] / (double)h[1] * (wall_khz * 1e-3) : 0.0;
  for (void* p : buf)
    if (p) (void)hipFree(p);
  (void)hipFree(clk);
  return e;
}

}  // namespace fsmi
