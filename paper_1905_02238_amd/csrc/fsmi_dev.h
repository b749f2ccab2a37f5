// fsmi_dev.h -- device-side building blocks of libfsmi (gfx950, wave64).
//
// Per-cell information function f (Sec. 2.2), the complementary error function
// used for the Gaussian weights G_{k,j} (Lemma on G, Sec. 3.3), wave-level
// prefix scans for the first-hit probabilities (Alg 2) and the info-gain
// terms (Alg 3), and small synchronisation helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FSMI_DEV __device__ __forceinline__

namespace fsmi {

constexpr int kWave = 64;

// Bits latched into the device status word.
enum : uint32_t {
  kErrOcc = 1u,      // an occupancy outside [0, 1] or NaN
  kErrLen = 2u,      // a negative beam length / run length <= 0 / bad offsets
  kErrPose = 4u,     // a pose outside the map
  kErrCap = 8u,      // a beam longer than the launch was sized for
  kErrBound = 16u,   // non-increasing cell boundaries
};

FSMI_DEV void latch(uint32_t* status, uint32_t bits) {
  if (status) atomicOr(status, bits);   // global (vector) atomic
}

// Makes LDS writes of one lane visible to later LDS reads of other lanes of the
// same wave (LDS executes a wave's operations in order; this stops the compiler
// from reordering across the exchange and waits for the writes to land).
FSMI_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

FSMI_DEV int lane_id() { return __lane_id(); }

// Work-queue pops, one ticket per wave, with no divergent branch: every lane
// issues the atomic but only lane 0 adds 1, and every lane takes lane 0's old
// value.  The result is wave-uniform (an SGPR), so loops over tickets are
// scalar loops.
FSMI_DEV int wave_pop(int32_t* counter) {
  const int inc = __lane_id() == 0 ? 1 : 0;
  const int old = atomicAdd(counter, inc);
  return __builtin_amdgcn_readfirstlane(old);
}
FSMI_DEV int64_t wave_pop64(int32_t* counter_pair) {
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counter_pair);
  const unsigned long long inc = __lane_id() == 0 ? 1ull : 0ull;
  const unsigned long long old = atomicAdd(c, inc);
  const int lo = __builtin_amdgcn_readfirstlane((int)(old & 0xffffffffull));
  const int hi = __builtin_amdgcn_readfirstlane((int)(old >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// ---------------------------------------------------------------------------
// Complementary error function, z >= 0, FP32.
// Chebyshev-fitted form of Press, Teukolsky, Vetterling & Flannery, Numerical
// Recipes (2nd ed.) Sec. 6.2: erfc(z) = t exp(-z^2 + P(t)), t = 1/(1 + z/2),
// fractional error below 1.2e-7 in exact arithmetic.  The polynomial is
// pre-scaled by log2(e) so the hardware 2^x instruction evaluates the exp.
// One branch-free path for all z, so lanes of a wave never diverge.
// ---------------------------------------------------------------------------
FSMI_DEV float erfc_pos(float z) {
  constexpr float L2E = 1.4426950408889634f;
  constexpr float c0 = -1.26551223f * L2E, c1 = 1.00002368f * L2E, c2 = 0.37409196f * L2E,
                  c3 = 0.09678418f * L2E, c4 = -0.18628806f * L2E, c5 = 0.27886807f * L2E,
                  c6 = -1.13520398f * L2E, c7 = 1.48851587f * L2E, c8 = -0.82215223f * L2E,
                  c9 = 0.17087277f * L2E;
  float t = __builtin_amdgcn_rcpf(fmaf(0.5f, z, 1.0f));
  float p = fmaf(t, c9, c8);
  p = fmaf(t, p, c7);
  p = fmaf(t, p, c6);
  p = fmaf(t, p, c5);
  p = fmaf(t, p, c4);
  p = fmaf(t, p, c3);
  p = fmaf(t, p, c2);
  p = fmaf(t, p, c1);
  p = fmaf(t, p, c0);
  float arg = fmaf(-z * L2E, z, p);
  return t * __builtin_amdgcn_exp2f(arg);
}

// The same function of x = z sqrt(log2 e): erfc(z) = t 2^(P2(t) - x^2), with
// t = 1/(1 + x / (2 sqrt(log2 e))) and P2 = log2(e) P.
FSMI_DEV float erfc_pos_l2(float x) {
  constexpr float L2E = 1.4426950408889634f;
  constexpr float c0 = -1.26551223f * L2E, c1 = 1.00002368f * L2E, c2 = 0.37409196f * L2E,
                  c3 = 0.09678418f * L2E, c4 = -0.18628806f * L2E, c5 = 0.27886807f * L2E,
                  c6 = -1.13520398f * L2E, c7 = 1.48851587f * L2E, c8 = -0.82215223f * L2E,
                  c9 = 0.17087277f * L2E;
  constexpr float kHalfInvSqrtL2E = 0.41627730557884884f;   // 1 / (2 sqrt(log2 e))
  float t = __builtin_amdgcn_rcpf(fmaf(kHalfInvSqrtL2E, x, 1.0f));
  float p = fmaf(t, c9, c8);
  p = fmaf(t, p, c7);
  p = fmaf(t, p, c6);
  p = fmaf(t, p, c5);
  p = fmaf(t, p, c4);
  p = fmaf(t, p, c3);
  p = fmaf(t, p, c2);
  p = fmaf(t, p, c1);
  p = fmaf(t, p, c0);
  return t * __builtin_amdgcn_exp2f(fmaf(-x, x, p));
}

// FP64 complementary error function (device libm), used by the FP64 mode.
FSMI_DEV double erfc_pos(double z) { return erfc(z); }

// ---------------------------------------------------------------------------
// f(delta, o) of Sec. 2.2 written in the occupancy o = r/(1+r).
// With s = 1 + o(delta-1): f = (o delta / s) ln(delta) - log1p(o (delta-1)).
// Near o = 1 both terms approach ln(delta) and cancel, so for o > 1/2 the
// equivalent form in u = 1 - o is used:
//   f = -log1p(-u a) - u ln(delta) / (delta (1 - u a)),  a = (delta-1)/delta.
// ---------------------------------------------------------------------------
template <typename T>
FSMI_DEV T f_cell(T delta, T ln_delta, T o);

template <>
FSMI_DEV float f_cell<float>(float delta, float ln_delta, float o) {
  if (o <= 0.5f) {
    float dm1 = delta - 1.0f;
    float s = fmaf(o, dm1, 1.0f);
    return (o * delta / s) * ln_delta - log1pf(o * dm1);
  }
  float u = 1.0f - o;
  float a = (delta - 1.0f) / delta;
  float ua = u * a;
  return -log1pf(-ua) - u * ln_delta / (delta * (1.0f - ua));
}

template <>
FSMI_DEV double f_cell<double>(double delta, double ln_delta, double o) {
  if (o <= 0.5) {
    double dm1 = delta - 1.0;
    double s = fma(o, dm1, 1.0);
    return (o * delta / s) * ln_delta - log1p(o * dm1);
  }
  double u = 1.0 - o;
  double a = (delta - 1.0) / delta;
  double ua = u * a;
  return -log1p(-ua) - u * ln_delta / (delta * (1.0 - ua));
}

// ---------------------------------------------------------------------------
// DPP wave scans (wave64, gfx9 DPP: row_shr within 16-lane rows, then
// row_bcast:15 and row_bcast:31 across rows).  Lanes whose DPP source is out of
// range receive the identity.
// ---------------------------------------------------------------------------
namespace dpp {
constexpr int row_shr1 = 0x111, row_shr2 = 0x112, row_shr4 = 0x114, row_shr8 = 0x118;
constexpr int row_bcast15 = 0x142, row_bcast31 = 0x143;
constexpr int wave_shr1 = 0x138;
}  // namespace dpp

template <int CTRL, int ROWMASK>
FSMI_DEV float dpp_f32(float v, float ident) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(ident), __float_as_int(v), CTRL,
                                                    ROWMASK, 0xf, false));
}

template <int CTRL, int ROWMASK>
FSMI_DEV double dpp_f64(double v, double ident) {
  int2 a = *reinterpret_cast<int2*>(&v);
  int2 i = *reinterpret_cast<int2*>(&ident);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(i.x, a.x, CTRL, ROWMASK, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(i.y, a.y, CTRL, ROWMASK, 0xf, false);
  return *reinterpret_cast<double*>(&r);
}

template <int CTRL, int ROWMASK>
FSMI_DEV int dpp_i32(int v, int ident) {
  return __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWMASK, 0xf, false);
}

struct OpAdd {
  template <typename T> FSMI_DEV static T apply(T a, T b) { return a + b; }
  template <typename T> FSMI_DEV static T ident() { return T(0); }
};
struct OpMul {
  template <typename T> FSMI_DEV static T apply(T a, T b) { return a * b; }
  template <typename T> FSMI_DEV static T ident() { return T(1); }
};
struct OpMinI {
  template <typename T> FSMI_DEV static T apply(T a, T b) { return a < b ? a : b; }
  template <typename T> FSMI_DEV static T ident() { return T(0x7fffffff); }
};

// Inclusive scan over the 64 lanes of a wave.
template <typename Op, typename T>
FSMI_DEV T wave_scan_incl(T v) {
  const T id = Op::template ident<T>();
  if constexpr (sizeof(T) == 8) {
    v = Op::apply(v, dpp_f64<dpp::row_shr1, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_shr2, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_shr4, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_shr8, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_bcast15, 0xa>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_bcast31, 0xc>(v, id));
  } else if constexpr (__is_same(T, float)) {
    v = Op::apply(v, dpp_f32<dpp::row_shr1, 0xf>(v, id));
    v = Op::apply(v, dpp_f32<dpp::row_shr2, 0xf>(v, id));
    v = Op::apply(v, dpp_f32<dpp::row_shr4, 0xf>(v, id));
    v = Op::apply(v, dpp_f32<dpp::row_shr8, 0xf>(v, id));
    v = Op::apply(v, dpp_f32<dpp::row_bcast15, 0xa>(v, id));
    v = Op::apply(v, dpp_f32<dpp::row_bcast31, 0xc>(v, id));
  } else {
    v = Op::apply(v, dpp_i32<dpp::row_shr1, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_shr2, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_shr4, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_shr8, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_bcast15, 0xa>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_bcast31, 0xc>(v, id));
  }
  return v;
}

// Exclusive version: the inclusive result shifted up one lane (lane 0 gets the identity).
template <typename Op, typename T>
FSMI_DEV T wave_shift_up(T inc) {
  const T id = Op::template ident<T>();
  if constexpr (sizeof(T) == 8) return dpp_f64<dpp::wave_shr1, 0xf>(inc, id);
  else if constexpr (__is_same(T, float)) return dpp_f32<dpp::wave_shr1, 0xf>(inc, id);
  else return dpp_i32<dpp::wave_shr1, 0xf>(inc, id);
}

// Value held by lane 63 (the wave total after an inclusive scan).
template <typename T>
FSMI_DEV T wave_last(T v) {
  if constexpr (sizeof(T) == 8) {
    int2 a = *reinterpret_cast<int2*>(&v);
    int2 r;
    r.x = __builtin_amdgcn_readlane(a.x, 63);
    r.y = __builtin_amdgcn_readlane(a.y, 63);
    return *reinterpret_cast<T*>(&r);
  } else if constexpr (__is_same(T, float)) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  } else {
    return __builtin_amdgcn_readlane(v, 63);
  }
}

// Sum over the wave, result in every lane (fixed-order tree, deterministic).
FSMI_DEV double wave_sum(double v) {
  v = wave_scan_incl<OpAdd>(v);
  return wave_last(v);
}
FSMI_DEV float wave_sum(float v) {
  v = wave_scan_incl<OpAdd>(v);
  return wave_last(v);
}
FSMI_DEV int wave_sum(int v) {
  v = wave_scan_incl<OpAdd>(v);
  return wave_last(v);
}

FSMI_DEV int wave_min(int v) {
  v = wave_scan_incl<OpMinI>(v);
  return wave_last(v);
}

// Kahan-compensated accumulator (FP32), used for the double sum.
struct Kahan {
  float s = 0.0f, c = 0.0f;
  FSMI_DEV void add(float x) {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
};

}  // namespace fsmi
