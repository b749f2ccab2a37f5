// k_beam.hip -- FSMI on batches of beams in CSR form (fsmi_eval_beams).
//
// Schedule: one persistent launch.  A device pass sorts beam ids into
// descending length bins, with every beam above the wave threshold ahead of
// every beam at or below it; beams above the threshold are taken by a whole
// workgroup (rows j split over all its lanes: tile-per-beam), the rest by
// single waves (wave-per-beam), in the same kernel (k_eval_fused).  Both pop
// items from atomic queue heads, so every wave exits once the queues are
// drained.
#include <math.h>

#include <algorithm>

#include "beam_dev.h"
#include "csqmi_dev.h"
#include "fsmi_internal.h"

namespace fsmi {

namespace {

constexpr int kNW = 4;          // waves per workgroup
constexpr int kHalf = 16;       // length bins per class (octaves, descending)
constexpr int kBins = 2 * kHalf;
constexpr int kMaxGrid = 4096;  // persistent workgroups
constexpr size_t kLdsLimit = 150 * 1024;   // dynamic LDS per workgroup

struct BeamArgs {
  EvalConst ec;
  int64_t n_beams;
  const int64_t* off;
  const float* occ;
  const double* bound;
  const float* sigma;
  double* mi;
  const int32_t* order;   // beam ids, longest first
  int32_t* counters;      // [0] block-queue head, [1] wave-queue head, [2] n_long
  uint32_t* status;
  int cap_block;          // cells of a workgroup item
  int cap_wave;           // cells of a wave item
};

template <typename T>
constexpr int bytes_per_cell() { return core_bytes_per_cell<T>() + 4; }   // + o

template <typename T>
FSMI_DEV CoreLds carve(char* p, int cap, float** so) {
  CoreLds L;
  L.A = reinterpret_cast<double*>(p);
  L.C = p + 8 * (size_t)(cap + 1);
  L.P = reinterpret_cast<char*>(L.C) + sizeof(T) * (size_t)cap;
  *so = reinterpret_cast<float*>(reinterpret_cast<char*>(L.P) + sizeof(T) * (size_t)cap);
  return L;
}

template <bool BLOCK, typename T, bool CSQ>
FSMI_DEV void process_beam(const BeamArgs& a, int b, char* lds, int cap, double* scratch,
                           int* flag, int tid) {
  constexpr int G = Grp<kNW, BLOCK>::size;
  const int64_t o0 = a.off[b];
  // wave-uniform length, clamped to [-1, 2^31): -1 flags a negative length
  const int n = __builtin_amdgcn_readfirstlane((int)min<int64_t>(
      max<int64_t>(a.off[b + 1] - o0, (int64_t)-1), (int64_t)0x7fffffff));
  double v = 0.0;
  uint32_t err = 0;
  if (n > 0 && n <= cap) {
    float* so;
    const CoreLds L = carve<T>(lds, cap, &so);
    const bool has_bound = a.bound != nullptr && a.ec.variant != FSMI_UNIFORM;
    // eight loads in flight per lane before any is stored: the beam's
    // occupancies come from HBM, and one round trip per element would
    // serialise a short beam's whole load
    for (int base = 0; base < n; base += 8 * G) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + u * G + tid;
        v[u] = a.occ[o0 + min(i, n - 1)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + u * G + tid;
        if (i < n) so[i] = v[u];
      }
    }
    if (has_bound) {
      const double* bp = a.bound + o0 + b;
      for (int base = 0; base <= n; base += 4 * G) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = base + u * G + tid;
          v[u] = bp[min(i, n)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = base + u * G + tid;
          if (i <= n) L.A[i] = v[u];
        }
      }
    }
    Grp<kNW, BLOCK>::sync();
    bool bad;
    v = beam_eval<kNW, BLOCK, T, CSQ>(a.ec, n, so, has_bound, (double)a.sigma[b], L, scratch, flag, tid,
                                 false, &bad);
    if (bad) err = kErrOcc;
  } else if (n != 0) {
    v = __builtin_nan("");
    err = n < 0 ? kErrLen : kErrCap;
  }
  if (tid == 0) {
    a.mi[b] = v;
    if (err) latch(a.status, err);
  }
}

// Both schedules in one persistent launch: every workgroup first takes beams
// above the wave threshold from the tile queue (all four waves on one beam),
// and once that queue is empty each of its waves takes beams from the wave
// queue on its own LDS slice.  A workgroup that finishes the long beams starts
// on the short ones at once, so no compute unit waits at a kernel boundary for
// the last long beams.  The LDS is the larger of the two phases' needs; the
// phases share it, and all waves leave the first phase together (its exit test
// is on a value read between two barriers), after the barrier that ends the
// last beam's use of the LDS.
template <typename T, bool CSQ>
__global__ __launch_bounds__(kWave* kNW) void k_eval_fused(BeamArgs a) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double scratch[kNW];
  __shared__ int s_item, s_flag;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int n_long = __builtin_amdgcn_readfirstlane(a.counters[2]);
  for (;;) {
    if (wave == 0) s_item = wave_pop(&a.counters[0]);   // every lane of wave 0 writes the same value
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_long) break;
    const int b = __builtin_amdgcn_readfirstlane(a.order[it]);
    process_beam<true, T, CSQ>(a, b, lds, a.cap_block, scratch, &s_flag, tid);
    __syncthreads();
  }
  const int n_short = (int)a.n_beams - n_long;
  char* my = lds + (size_t)wave * ((size_t)a.cap_wave * bytes_per_cell<T>() + 16);
  const int64_t n_waves = (int64_t)gridDim.x * kNW;
  int k = (int)run_length(n_short, 0, n_waves);
  for (int start = wave_take(&a.counters[1], k); start < n_short;
       start = wave_take(&a.counters[1], k)) {
    const int end = min(start + k, n_short);
    k = (int)run_length(n_short, end, n_waves);
    for (int it = start; it < end; ++it) {
      const int b = __builtin_amdgcn_readfirstlane(a.order[n_long + it]);
      process_beam<false, T, CSQ>(a, b, my, a.cap_wave, nullptr, nullptr, lane);
    }
  }
}

// ---------------------------------------------------------------------------
// Schedule on the device: a length histogram over bins ordered long-to-short
// (class "above the wave threshold" first, octaves descending within a class),
// exclusive bin offsets, and a scatter of beam ids.  counters[2] receives the
// number of beams above the threshold.
// ---------------------------------------------------------------------------
FSMI_DEV int len_bin(int64_t n, int wave_max) {
  const int cls = n > wave_max ? 0 : 1;
  int oct = n <= 1 ? 0 : 63 - __builtin_clzll((unsigned long long)n);   // floor(log2 n)
  oct = oct > kHalf - 1 ? kHalf - 1 : oct;
  return cls * kHalf + (kHalf - 1 - oct);
}

__global__ void k_sched_reset(int32_t* counters, int32_t* hist) {
  const int t = threadIdx.x;
  if (t < 8) counters[t] = 0;
  if (t < 2 * kBins) hist[t] = 0;
}

__global__ void k_queue_reset(int32_t* counters) {
  if (threadIdx.x < 2) counters[threadIdx.x] = 0;
}

__global__ void k_sched_count(const int64_t* off, int64_t n_beams, int wave_max, int32_t* hist,
                              int32_t* counters) {
  __shared__ int32_t h[kBins];
  __shared__ int32_t nl;
  if (threadIdx.x < kBins) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) nl = 0;
  __syncthreads();
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n_beams;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = off[b + 1] - off[b];
    atomicAdd(&h[len_bin(n, wave_max)], 1);
    if (n > wave_max) atomicAdd(&nl, 1);
  }
  __syncthreads();
  if (threadIdx.x < kBins && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 0 && nl) atomicAdd(&counters[2], nl);
}

__global__ void k_sched_scan(int32_t* hist) {
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int i = 0; i < kBins; ++i) {
      hist[kBins + i] = s;
      s += hist[i];
    }
  }
}

// Beams into their bins, a block of 256 at a time: ranks within the block
// from LDS atomics, one global atomic per bin and block for the block's range
// (order within a bin is arbitrary; every beam's result is independent of it).
__global__ __launch_bounds__(256) void k_sched_scatter(const int64_t* off, int64_t n_beams,
                                                       int wave_max, int32_t* hist,
                                                       int32_t* order) {
  __shared__ int32_t cnt[kBins], base[kBins];
  const int tid = threadIdx.x;
  for (int64_t chunk = (int64_t)blockIdx.x * 256; chunk < n_beams;
       chunk += (int64_t)gridDim.x * 256) {
    if (tid < kBins) cnt[tid] = 0;
    __syncthreads();
    const int64_t b = chunk + tid;
    int bin = -1, local = 0;
    if (b < n_beams) {
      bin = len_bin(off[b + 1] - off[b], wave_max);
      local = atomicAdd(&cnt[bin], 1);
    }
    __syncthreads();
    if (tid < kBins && cnt[tid]) base[tid] = atomicAdd(&hist[kBins + tid], cnt[tid]);
    __syncthreads();
    if (bin >= 0) order[base[bin] + local] = (int32_t)b;
    __syncthreads();
  }
}

__global__ void k_max_len(const int64_t* off, int64_t n_beams, int32_t* out) {
  int32_t m = 0;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n_beams;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = off[b + 1] - off[b];
    m = max(m, (int32_t)min<int64_t>(n, 0x7fffffff));
  }
  atomicMax(out, m);
}

__global__ void k_zero_i32(int32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_erfc_probe(int64_t n, const float* z, float* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = erfc_pos(z[i]);
}

__global__ void k_f_probe(FConst k, int64_t n, const float* o, double* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = f_cell_series(k, (double)o[i]);
}

}  // namespace

hipError_t launch_f_probe(fsmi_ctx ctx, double delta, int64_t n, const float* o, double* out) {
  if (n <= 0) return hipSuccess;
  const FConst k{delta, delta - 1.0, (delta - 1.0) / delta, log(delta)};
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_f_probe, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, k, n, o, out);
  return hipGetLastError();
}

hipError_t launch_erfc_probe(fsmi_ctx ctx, int64_t n, const float* z, float* out) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_erfc_probe, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, z, out);
  return hipGetLastError();
}

hipError_t launch_max_len(fsmi_ctx ctx, const int64_t* off, int64_t n_beams, int* host_out) {
  hipError_t e = ensure_work(ctx, 64);
  if (e != hipSuccess) return e;
  int32_t* d = reinterpret_cast<int32_t*>(ctx->d_work);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, d);
  const int grid = (int)std::min<int64_t>((n_beams + 255) / 256, 1024);
  hipLaunchKernelGGL(k_max_len, dim3(std::max(grid, 1)), dim3(256), 0, ctx->stream, off, n_beams, d);
  e = hipMemcpyAsync(host_out, d, 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(ctx->stream);
}

int beam_default_wave_max(int precision) { return precision == FSMI_FP64 ? 256 : 512; }

int beam_bytes_per_cell(int precision) {
  return precision == FSMI_FP64 ? bytes_per_cell<double>() : bytes_per_cell<float>();
}

bool beam_fits(int precision, int wave_max, int max_len) {
  const size_t bpc = (size_t)beam_bytes_per_cell(precision);
  return bpc * (size_t)std::max(max_len, 1) + 16 <= kLdsLimit &&
         (size_t)kNW * (bpc * (size_t)std::max(wave_max, 1) + 16) <= kLdsLimit;
}

size_t beam_sched_ints(int64_t n_beams) { return (size_t)n_beams + 2 * kBins + 16; }

hipError_t launch_beam_schedule(hipStream_t st, const int64_t* off, int64_t n_beams, int wave_max,
                                int32_t* sched) {
  int32_t* order = sched;
  int32_t* hist = sched + n_beams;
  int32_t* counters = hist + 2 * kBins;
  hipLaunchKernelGGL(k_sched_reset, dim3(1), dim3(64), 0, st, counters, hist);
  const int cb = (int)std::max<int64_t>(1, std::min<int64_t>((n_beams + 255) / 256, 1024));
  hipLaunchKernelGGL(k_sched_count, dim3(cb), dim3(256), 0, st, off, n_beams, wave_max, hist,
                     counters);
  hipLaunchKernelGGL(k_sched_scan, dim3(1), dim3(64), 0, st, hist);
  hipLaunchKernelGGL(k_sched_scatter, dim3(cb), dim3(256), 0, st, off, n_beams, wave_max, hist,
                     order);
  return hipGetLastError();
}

int64_t beam_sched_n_long_index(int64_t n_beams) { return n_beams + 2 * kBins + 2; }

hipError_t launch_beam_kernels(hipStream_t st, int num_cu, const EvalConst& ec, int64_t n_beams,
                               const int64_t* off, const float* occ, const double* bound,
                               const float* sigma, double* mi, const int32_t* sched,
                               uint32_t* status, int wave_max, int max_len) {
  BeamArgs a;
  a.ec = ec;
  a.n_beams = n_beams;
  a.off = off;
  a.occ = occ;
  a.bound = bound;
  a.sigma = sigma;
  a.mi = mi;
  a.order = sched;
  a.counters = const_cast<int32_t*>(sched) + n_beams + 2 * kBins;
  a.status = status;
  const bool fp64 = ec.precision == FSMI_FP64;
  const size_t bpc = (size_t)beam_bytes_per_cell(ec.precision);
  a.cap_wave = wave_max;
  a.cap_block = std::max(max_len, 1);
  const size_t lds_long = bpc * a.cap_block + 16;
  const size_t lds_short = (size_t)kNW * (bpc * a.cap_wave + 16);
  if (lds_long > kLdsLimit || lds_short > kLdsLimit) return hipErrorInvalidValue;
  // one persistent launch over both queues, sized for the larger phase
  const size_t lds = std::max(lds_long, lds_short);
  const int per_cu = std::max<int>(1, (int)((160 * 1024) / (lds + 512)));
  const int grid = std::max(1, std::min(kMaxGrid, num_cu * std::min(per_cu, 8)));
  // queue heads back to zero; the long-beam count written by the schedule stays
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, a.counters);
  auto launch = [&](auto kern) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * kNW), lds, st, a);
  };
  const bool csq = ec.variant == FSMI_CSQMI;
  if (fp64) {
    if (csq) launch(k_eval_fused<double, true>);
    else launch(k_eval_fused<double, false>);
  } else {
    if (csq) launch(k_eval_fused<float, true>);
    else launch(k_eval_fused<float, false>);
  }
  return hipGetLastError();
}

hipError_t launch_eval_beams(fsmi_ctx ctx, const EvalConst& ec, int64_t n_beams, const int64_t* off,
                             const float* occ, const double* bound, const float* sigma,
                             double* mi, int max_len, int wave_max) {
  if (n_beams <= 0) return hipSuccess;
  hipError_t e = ensure_work(ctx, beam_sched_ints(n_beams) * 4);
  if (e != hipSuccess) return e;
  int32_t* sched = reinterpret_cast<int32_t*>(ctx->d_work);
  e = launch_beam_schedule(ctx->stream, off, n_beams, wave_max, sched);
  if (e != hipSuccess) return e;
  return launch_beam_kernels(ctx->stream, ctx->num_cu, ec, n_beams, off, occ, bound, sigma, mi, sched,
                             ctx->d_status, wave_max, max_len);
}

__global__ void k_fill_f64(int64_t n, double v, double* p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_f64(hipStream_t st, int64_t n, double v, double* p) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill_f64, dim3(grid), dim3(256), 0, st, n, v, p);
  return hipGetLastError();
}

}  // namespace fsmi
