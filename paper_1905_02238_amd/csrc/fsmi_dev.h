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
// Longest run of (pose, beam) items one queue ticket takes in the fused pose
// kernels (guided self-scheduling, run_length below).
constexpr int kMaxRun = 32;

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
// Takes the next k items (k wave-uniform) from a 64-bit queue head: returns the
// first, the same in every lane.
FSMI_DEV int64_t wave_take64(int32_t* counter_pair, int64_t k) {
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counter_pair);
  const unsigned long long inc = __lane_id() == 0 ? (unsigned long long)k : 0ull;
  const unsigned long long old = atomicAdd(c, inc);
  const int lo = __builtin_amdgcn_readfirstlane((int)(old & 0xffffffffull));
  const int hi = __builtin_amdgcn_readfirstlane((int)(old >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The same on a 32-bit queue head.
FSMI_DEV int wave_take(int32_t* counter, int k) {
  const int inc = __lane_id() == 0 ? k : 0;
  const int old = atomicAdd(counter, inc);
  return __builtin_amdgcn_readfirstlane(old);
}

// Guided self-scheduling: a quarter of the remaining items' share per wave,
// between 1 and kMaxRun, so runs are long (few atomics on the queue head)
// while the queue is full and single items at the end (the last, possibly
// costly, items still spread over all waves).
FSMI_DEV int64_t run_length(int64_t n_items, int64_t taken, int64_t n_waves) {
  const int64_t r = (n_items - taken) / (4 * n_waves);
  return r < 1 ? 1 : (r > kMaxRun ? kMaxRun : r);
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
// Complementary error function, FP32, of y = z sqrt(log2 e) for z >= 0:
//   erfc(z) = t 2^(P2(t) - y^2),  t = 1 / (1 + kErfcA y),
// P2 a degree-6 polynomial (log2 e times a fit of ln(erfc(z)/t) + z^2 in t,
// with t = 1/(1 + 0.382 z)).  The constants and their fit are made by
// csrc/erfc_fit.py: relative error 1.2e-6 on z in [0, 10] in exact
// arithmetic, about 2e-6 once the FP32 exponent y^2 is rounded.  Degree 6
// is what the FP32 mode's 1e-5 bar on mutual information needs: with the
// fit's error alone, Thm 1 moved by at most 2.7e-6 relative on 2560 beams
// of the 2D timed workload (degree 7: 2.2e-7, for one more FMA per pair).
// The hardware reciprocal and 2^x run on the transcendental unit; the rest is
// seven FMAs and a multiply.  One branch-free path for all z, so lanes never
// diverge.
// ---------------------------------------------------------------------------
constexpr float kErfcA = 0.31803587079048157f;
constexpr float kErfcP0 = -2.2124266624450684f, kErfcP1 = 1.4149539470672607f,
                kErfcP2 = 0.802640438079834f, kErfcP3 = -0.38545480370521545f,
                kErfcP4 = 1.3409265279769897f, kErfcP5 = -1.3553467988967896f,
                kErfcP6 = 0.39470893144607544f;
constexpr float kSqrtL2E = 1.2011224087864498f;    // sqrt(log2 e)
constexpr float kInvSqrtL2E = 0.8325546111576977f;  // 1 / sqrt(log2 e)

FSMI_DEV float erfc_pos_l2(float y) {
  const float t = __builtin_amdgcn_rcpf(fmaf(kErfcA, y, 1.0f));
  float p = fmaf(t, kErfcP6, kErfcP5);
  p = fmaf(t, p, kErfcP4);
  p = fmaf(t, p, kErfcP3);
  p = fmaf(t, p, kErfcP2);
  p = fmaf(t, p, kErfcP1);
  p = fmaf(t, p, kErfcP0);
  return t * __builtin_amdgcn_exp2f(fmaf(-y, y, p));
}

// erfc(z), z >= 0, FP32.
FSMI_DEV float erfc_pos(float z) { return erfc_pos_l2(z * kSqrtL2E); }

// FP64 complementary error function (device libm), used by the FP64 mode.
FSMI_DEV double erfc_pos(double z) { return erfc(z); }

// ---------------------------------------------------------------------------
// f(delta, o) of Sec. 2.2 written in the occupancy o = r/(1+r).
// With s = 1 + o(delta-1): f = (o delta / s) ln(delta) - ln s.
// Near o = 1 both terms approach ln(delta) and cancel, so for o > 1/2 the
// equivalent form in u = 1 - o is used (s = delta (1 - u a)):
//   f = -log1p(-u a) - u ln(delta) / s,  a = (delta-1)/delta.
// ---------------------------------------------------------------------------
template <typename T>
FSMI_DEV T f_cell(T delta, T ln_delta, T o);

// FP64 mode: device libm.
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

// FP32 mode: the same two forms, chosen per lane by a select (no branch),
// in FP64 arithmetic with a short series for the logarithm, so that neither
// form's cancellation reaches FP32 precision (relative error about 1e-12 of f
// for delta in [1.001, 100]).
//   ln(1 + x) = e ln 2 + 2 atanh(z),  1 + x = m 2^e,  m in [sqrt(1/2), sqrt 2),
//   z = (m - 1)/(m + 1), or z = x/(2 + x) straight from x when e = 0, so a
//   small x keeps every digit; 2 atanh(z) = z sum_k 2 z^(2k)/(2k+1), k <= 6,
//   |z| <= 0.1716: truncation below 2e-12 relative.
// The quotients take the hardware reciprocal and one Newton step.
struct FConst {
  double delta, dm1, a, ln_delta;   // delta, delta - 1, (delta - 1)/delta, ln delta
};
FSMI_DEV FConst f_const(double delta) {
  return FConst{delta, delta - 1.0, (delta - 1.0) / delta, log(delta)};
}
FSMI_DEV double rcp_f64(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}
FSMI_DEV double ln1p_series(double x) {   // x > -1
  const double y = 1.0 + x;
  double m = __builtin_amdgcn_frexp_mant(y);   // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(y);
  if (m < 0.70710678118654752440) m += m, e -= 1;
  const bool e0 = e == 0;
  const double zn = e0 ? x : m - 1.0;
  const double zd = e0 ? 2.0 + x : m + 1.0;
  const double z = zn * rcp_f64(zd);
  const double w = z * z;
  double p = fma(w, 2.0 / 13.0, 2.0 / 11.0);
  p = fma(w, p, 2.0 / 9.0);
  p = fma(w, p, 2.0 / 7.0);
  p = fma(w, p, 2.0 / 5.0);
  p = fma(w, p, 2.0 / 3.0);
  p = fma(w, p, 2.0);
  return fma((double)e, 0.69314718055994530942, z * p);
}
FSMI_DEV double f_cell_series(const FConst& k, double o) {
  const bool lo = o <= 0.5;
  const double u = 1.0 - o;
  const double x = lo ? o * k.dm1 : -u * k.a;
  const double num = lo ? o * k.delta : -u;
  const double s = fma(o, k.dm1, 1.0);
  return fma(num, k.ln_delta * rcp_f64(s), -ln1p_series(x));
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
