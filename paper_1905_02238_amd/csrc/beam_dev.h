// beam_dev.h -- the per-beam FSMI evaluation run by a group of lanes (one wave,
// or a whole workgroup), on data staged in LDS.
//
// Steps (Sec. 3): per-cell f (Sec. 2.2) -> P(e_j) by a prefix product (Alg 2)
// -> C_k by a prefix sum (Alg 3) -> the double sum of Thm 1 with the Gaussian
// weights G_{k,j} (Eq. G_jk), its truncated form (Eq. fsmi_approx), or the
// uniform-noise form (Thm 4 / Alg 4).
//
// Numerics (FP32 mode): f is evaluated in FP64 (f_cell_series); the prefix
// product of (1 - o) and the C_k prefix are scanned in FP64; on explicit
// boundaries the O(n^2) loop is FP32 with one erfc per (row j, boundary),
// evaluated on the tail side of mu_j so that no digits cancel, and a
// Kahan-compensated sum over blocks of eight terms; each row's P_j S_j is
// accumulated in FP64 and the group total is a fixed-order tree.  On unit
// cells exact FSMI runs on the matrix cores (exact_unit_mfma): FP32 products
// accumulated in FP32 per 16 x 16 block offset, weighted and added in FP64.
#pragma once
#include <math.h>

#include "fsmi_dev.h"
#include "fsmi_internal.h"
#include "lut_dev.h"

namespace fsmi {

template <int NW, bool BLOCK>
struct Grp {
  static constexpr int size = BLOCK ? kWave * NW : kWave;
  FSMI_DEV static void sync() {
    if constexpr (BLOCK) __syncthreads();
    else wave_sync();
  }
};

// Exclusive scan across the group in thread order, carried across chunks.
template <int NW, bool BLOCK, typename Op>
FSMI_DEV double group_scan_excl(double v, double& carry, double* scratch, int tid) {
  double inc = wave_scan_incl<Op>(v);
  double exw = wave_shift_up<Op>(inc);
  double wtot = wave_last(inc);
  if constexpr (BLOCK) {
    const int w = tid >> 6;
    if ((tid & 63) == 0) scratch[w] = wtot;
    __syncthreads();
    double pre = Op::template ident<double>(), tot = Op::template ident<double>();
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      double x = scratch[i];
      if (i < w) pre = Op::apply(pre, x);
      tot = Op::apply(tot, x);
    }
    __syncthreads();
    double r = Op::apply(Op::apply(carry, pre), exw);
    carry = Op::apply(carry, tot);
    return r;
  } else {
    double r = Op::apply(carry, exw);
    carry = Op::apply(carry, wtot);
    return r;
  }
}

template <int NW, bool BLOCK>
FSMI_DEV double group_sum(double v, double* scratch, int tid) {
  double s = wave_sum(v);
  if constexpr (BLOCK) {
    const int w = tid >> 6;
    if ((tid & 63) == 0) scratch[w] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += scratch[i];
    __syncthreads();
    return t;
  }
  return s;
}

template <int NW, bool BLOCK>
FSMI_DEV bool group_any(bool b, int* flag, int tid) {
  bool w = __any(b);
  if constexpr (BLOCK) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    if (w && (tid & 63) == 0) *flag = 1;
    __syncthreads();
    const bool r = __builtin_amdgcn_readfirstlane(*flag) != 0;
    __syncthreads();
    return r;
  }
  return w;
}

// |x| as the VALU source modifier (no compare/select).
template <typename T> FSMI_DEV T tabs(T x) {
  if constexpr (sizeof(T) == 8) return __builtin_fabs(x);
  else return __builtin_fabsf(x);
}

template <typename T> FSMI_DEV T erf_t(T x);
template <> FSMI_DEV float erf_t<float>(float x) { return erff(x); }
template <> FSMI_DEV double erf_t<double>(double x) { return erf(x); }

template <typename T> struct Acc;
template <> struct Acc<float> {
  Kahan k;
  FSMI_DEV void add(float x) { k.add(x); }
  FSMI_DEV double value() const { return (double)k.s - (double)k.c; }
};
template <> struct Acc<double> {
  double s = 0.0, c = 0.0;
  FSMI_DEV void add(double x) {
    double y = x - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  FSMI_DEV double value() const { return s - c; }
};

// Explicit boundaries are pre-scaled once per beam (beam_core):
//   FP32: L = l c sqrt(log2 e), the argument erfc_pos_l2 takes;
//   FP64: L = l c;
// with c = 1/(sigma sqrt 2), so the weight argument of a boundary is |L - M|
// (M the scaled mid-point of the hit cell) with no multiply per pair.
// LUT (FP32 only): the boundaries are scaled by kLutInvH too and the tail is
// read from the table (lut_dev.h).
template <typename T, bool LUT = false>
FSMI_DEV T tail_E(double L, double M, const float2* lut = nullptr) {
  if constexpr (sizeof(T) == 8) {
    return erfc_pos(tabs(L - M));
  } else if constexpr (LUT) {
    return lut_tail(lut, (float)tabs(L - M));
  } else {
    return erfc_pos_l2((float)tabs(L - M));
  }
}
template <typename T, bool LUT = false> constexpr double unscale() {
  return sizeof(T) == 8 ? 1.0 : (LUT ? (double)kInvSqrtL2E / (double)kLutInvH : (double)kInvSqrtL2E);
}

// The erfc of a signed scaled distance d, on the tail side.
template <typename T>
FSMI_DEV T tail_Ed(double d) {
  if constexpr (sizeof(T) == 8) {
    return erfc_pos(tabs(d));
  } else {
    return erfc_pos_l2((float)tabs(d));
  }
}

// Row j's frame: the scaled distance of a boundary from mu_j.  With one sigma
// per beam the boundaries are pre-scaled and d(l) = l - M.  With
// range-dependent noise (sigma_j = sigma + slope mu_j, the per-event sigma_j
// of Alg 1) the boundaries stay in their own units and d(l) = l a_j + b_j,
// a_j = 1 / (sigma_j sqrt 2) (times sqrt(log2 e) in FP32), b_j = -mu_j a_j:
// one FMA in place of the subtraction.
template <typename T, bool RD>
struct RowFrame {
  double M = 0.0, a = 0.0, b = 0.0;
  FSMI_DEV double d(double l) const {
    if constexpr (RD) return fma(l, a, b);
    else return l - M;
  }
};
template <typename T, bool RD>
FSMI_DEV RowFrame<T, RD> row_frame(const double* sL, int j, double sigma, double slope) {
  RowFrame<T, RD> f;
  f.M = 0.5 * (sL[j - 1] + sL[j]);
  if constexpr (RD) {
    const double sj = sigma + slope * f.M;
    f.a = (sizeof(T) == 8 ? 1.0 : (double)kSqrtL2E) / (sj * 1.4142135623730951);
    f.b = -f.M * f.a;
  }
  return f;
}

// ---------------------------------------------------------------------------
// Row sums S_j = sum_k C_k G_{k,j} on scaled boundaries sL[0..n].
// G_{k,j} = (1/2)|E(l_{k+1}) - E(l_k)| for k != j (both boundaries on one side
// of mu_j), G_{j,j} = (1/2)(erf((l_{j+1}-mu)c) + erf((mu-l_j)c)).
// ---------------------------------------------------------------------------
template <typename T, bool LUT = false>
FSMI_DEV double diag_fix(Acc<T>& acc, const double* sL, const T* sC, int j, double M,
                         const float2* lut = nullptr) {
  // replace the k = j term the loop took by the exact diagonal weight
  T Ej = tail_E<T, LUT>(sL[j - 1], M, lut);
  T Ej1 = tail_E<T, LUT>(sL[j], M, lut);
  T Cj = sC[j - 1];
  acc.add(-(Cj * tabs(Ej1 - Ej)));
  constexpr double u = unscale<T, LUT>();
  T g2 = erf_t<T>((T)((sL[j] - M) * u)) + erf_t<T>((T)((M - sL[j - 1]) * u));
  acc.add(Cj * g2);
  return 0.5 * acc.value();
}

// Terms b0..b1 (1 <= b0 <= b1 <= n) of row j, halved, with the exact diagonal
// weight if the segment holds b = j.  Eight pairs per compensated add: the
// block of eight is an FP32 (or FP64) FMA chain, the blocks are Kahan-summed.
template <typename T, bool LUT = false>
FSMI_DEV double row_exact_seg(const double* sL, const T* sC, int j, int b0, int b1,
                              const float2* lut = nullptr) {
  const double M = 0.5 * (sL[j - 1] + sL[j]);
  Acc<T> acc;
  T Eprev = tail_E<T, LUT>(sL[b0 - 1], M, lut);
  int b = b0;
  for (; b + 7 <= b1; b += 8) {
    T E[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) E[q] = tail_E<T, LUT>(sL[b + q], M, lut);
    T p = sC[b - 1] * tabs(E[0] - Eprev);
#pragma unroll
    for (int q = 1; q < 8; ++q) p = fma(sC[b - 1 + q], tabs(E[q] - E[q - 1]), p);
    acc.add(p);
    Eprev = E[7];
  }
  for (; b <= b1; ++b) {
    T E = tail_E<T, LUT>(sL[b], M, lut);
    acc.add(sC[b - 1] * tabs(E - Eprev));
    Eprev = E;
  }
  if (j >= b0 && j <= b1) return diag_fix<T, LUT>(acc, sL, sC, j, M, lut);
  return 0.5 * acc.value();
}

// sum_j P_j S_j over the n rows of an n x n pair grid, on the G lanes of a
// group: whole sweeps of G rows (one row per lane), then the last R = n mod G
// rows, each cut into S = floor(G / R) equal runs of terms, lane l taking row
// (l mod R), run (l div R), so a partly filled sweep does not leave lanes idle.
template <int G, typename T, bool LUT = false>
FSMI_DEV double exact_rows(const double* sL, const T* sC, const T* sP, int n, int tid,
                           const float2* lut = nullptr) {
  double tot = 0.0;
  const int full = (n / G) * G;
  for (int j = tid + 1; j <= full; j += G)
    tot += (double)sP[j - 1] * row_exact_seg<T, LUT>(sL, sC, j, 1, n, lut);
  const int R = n - full;
  if (R > 0) {
    const int S = G / R;
    const int r = tid % R, s = tid / R;
    const int len = (n + S - 1) / S;
    const int b0 = s * len + 1, b1 = min(n, (s + 1) * len);
    if (s < S && b0 <= b1) {
      const int j = full + 1 + r;
      tot += (double)sP[j - 1] * row_exact_seg<T, LUT>(sL, sC, j, b0, b1, lut);
    }
  }
  return tot;
}

// ---------------------------------------------------------------------------
// The same rows in a row frame (range-dependent noise) and with the
// max-range return term; kept apart so the one-sigma loop above is unchanged.
// ---------------------------------------------------------------------------
template <typename T, bool RD>
FSMI_DEV double diag_fix_f(Acc<T>& acc, const double* sL, const T* sC, int j,
                           const RowFrame<T, RD>& f) {
  // replace the k = j term the loop took by the exact diagonal weight
  const double dl = f.d(sL[j - 1]), dr = f.d(sL[j]);
  T Ej = tail_Ed<T>(dl);
  T Ej1 = tail_Ed<T>(dr);
  T Cj = sC[j - 1];
  acc.add(-(Cj * tabs(Ej1 - Ej)));
  constexpr double u = unscale<T>();
  T g2 = erf_t<T>((T)(dr * u)) + erf_t<T>((T)(-dl * u));
  acc.add(Cj * g2);
  return 0.5 * acc.value();
}

// Terms b0..b1 (1 <= b0 <= b1 <= n) of row j, halved, with the exact diagonal
// weight if the segment holds b = j.  Eight pairs per compensated add: the
// block of eight is an FP32 (or FP64) FMA chain, the blocks are Kahan-summed.
template <typename T, bool RD>
FSMI_DEV double row_exact_seg_f(const double* sL, const T* sC, int j, int b0, int b1,
                                const RowFrame<T, RD>& f) {
  Acc<T> acc;
  T Eprev = tail_Ed<T>(f.d(sL[b0 - 1]));
  int b = b0;
  for (; b + 7 <= b1; b += 8) {
    T E[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) E[q] = tail_Ed<T>(f.d(sL[b + q]));
    T p = sC[b - 1] * tabs(E[0] - Eprev);
#pragma unroll
    for (int q = 1; q < 8; ++q) p = fma(sC[b - 1 + q], tabs(E[q] - E[q - 1]), p);
    acc.add(p);
    Eprev = E[7];
  }
  for (; b <= b1; ++b) {
    T E = tail_Ed<T>(f.d(sL[b]));
    acc.add(sC[b - 1] * tabs(E - Eprev));
    Eprev = E;
  }
  if (j >= b0 && j <= b1) return diag_fix_f<T, RD>(acc, sL, sC, j, f);
  return 0.5 * acc.value();
}

// sum_j P_j S_j over the n rows of an n x n pair grid, on the G lanes of a
// group: whole sweeps of G rows (one row per lane), then the last R = n mod G
// rows, each cut into S = floor(G / R) equal runs of terms, lane l taking row
// (l mod R), run (l div R), so a partly filled sweep does not leave lanes idle.
// With tq != 0 each row also adds P_j tq erfc(d(l_{n+1})): the max-range
// reading's probability under e_j (times 2) weighted by tq = q_n / 2.
template <int G, typename T, bool RD>
FSMI_DEV double exact_rows_ext(const double* sL, const T* sC, const T* sP, int n, int tid,
                               double sigma, double slope, double tq) {
  double tot = 0.0;
  const int full = (n / G) * G;
  for (int j = tid + 1; j <= full; j += G) {
    const RowFrame<T, RD> f = row_frame<T, RD>(sL, j, sigma, slope);
    double v = row_exact_seg_f<T, RD>(sL, sC, j, 1, n, f);
    if (tq != 0.0) v += tq * (double)tail_Ed<T>(f.d(sL[n]));
    tot += (double)sP[j - 1] * v;
  }
  const int R = n - full;
  if (R > 0) {
    const int S = G / R;
    const int r = tid % R, s = tid / R;
    const int len = (n + S - 1) / S;
    const int b0 = s * len + 1, b1 = min(n, (s + 1) * len);
    if (s < S && b0 <= b1) {
      const int j = full + 1 + r;
      const RowFrame<T, RD> f = row_frame<T, RD>(sL, j, sigma, slope);
      double v = row_exact_seg_f<T, RD>(sL, sC, j, b0, b1, f);
      if (tq != 0.0 && s == 0) v += tq * (double)tail_Ed<T>(f.d(sL[n]));
      tot += (double)sP[j - 1] * v;
    }
  }
  return tot;
}

// Skip-zero mode (FP32): only boundaries with |L_b - M_j| <= kSkipY, beyond
// which erfc is below the smallest normal float (erfc(9.3) < 2^-126), so the
// skipped terms add nothing at FP32 precision.  Cells kept: from the band's
// first boundary to one past its last (the cells at the edges of the band).
constexpr double kSkipY = 11.2;   // scaled units: 9.32 in units of sigma sqrt 2

FSMI_DEV int first_at_least(const double* sL, int n, double key) {   // in [0, n + 1]
  int lo = 0, hi = n + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sL[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename T>
FSMI_DEV double row_exact_band(const double* sL, const T* sC, int n, int j) {
  const double M = 0.5 * (sL[j - 1] + sL[j]);
  const int b_lo = first_at_least(sL, n, M - kSkipY);
  const int b_hi = first_at_least(sL, n, M + kSkipY + 1e-300) - 1;   // last with L_b <= M + Y
  const int k0 = max(1, b_lo), k1 = min(n, b_hi + 1);
  Acc<T> acc;
  T Eprev = tail_E<T>(sL[k0 - 1], M);
  int b = k0;
  for (; b + 7 <= k1; b += 8) {
    T E[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) E[q] = tail_E<T>(sL[b + q], M);
    T p = sC[b - 1] * tabs(E[0] - Eprev);
#pragma unroll
    for (int q = 1; q < 8; ++q) p = fma(sC[b - 1 + q], tabs(E[q] - E[q - 1]), p);
    acc.add(p);
    Eprev = E[7];
  }
  for (; b <= k1; ++b) {
    T E = tail_E<T>(sL[b], M);
    acc.add(sC[b - 1] * tabs(E - Eprev));
    Eprev = E;
  }
  return diag_fix<T>(acc, sL, sC, j, M);
}

// Cells k in [k0, k1) of row j on the tail side given by Eprev (the tail
// value at boundary k0 - 1): sum of C_k |E_k - E_{k-1}| in FMA chains of up
// to eight terms, each chain Kahan-added to acc.
template <typename T, bool LUT = false>
FSMI_DEV void row_side(const double* sL, const T* sC, double M, int k0, int k1, T Eprev,
                       Acc<T>& acc, const float2* lut = nullptr) {
  for (int b = k0; b < k1; b += 8) {
    const int e = min(b + 8, k1);
    T p = T(0);
    for (int k = b; k < e; ++k) {
      const T E = tail_E<T, LUT>(sL[k], M, lut);
      p = fma(sC[k - 1], tabs(E - Eprev), p);
      Eprev = E;
    }
    acc.add(p);
  }
}

template <typename T, bool LUT = false>
FSMI_DEV double row_approx_bound(const double* sL, const T* sC, int n, int j, int D,
                                 const float2* lut = nullptr) {
  const double M = 0.5 * (sL[j - 1] + sL[j]);
  // cells k = j-D..j+D inside the beam; the hit cell k = j takes the exact
  // weight of its two half widths, the others their tail differences
  const int k0 = max(1, j - D), k1 = min(n, j + D);
  Acc<T> acc;
  row_side<T, LUT>(sL, sC, M, k0, j, tail_E<T, LUT>(sL[k0 - 1], M, lut), acc, lut);
  row_side<T, LUT>(sL, sC, M, j + 1, k1 + 1, tail_E<T, LUT>(sL[j], M, lut), acc, lut);
  constexpr double u = unscale<T, LUT>();
  const T g2 = erf_t<T>((T)((sL[j] - M) * u)) + erf_t<T>((T)((M - sL[j - 1]) * u));
  acc.add(sC[j - 1] * g2);
  return 0.5 * acc.value();
}

// Unit cells: G_{k,j} = g(|k-j|), g from the per-beam table sG[0..n-1].
// The weight table of equal-width cells, seen from row j: w(k) = g(|k - j|).
// FP32 keeps the table mirrored (g(|d|) at off + d, d = -(n-1)..n-1), so a
// row reads consecutive addresses and an unrolled block needs no index
// arithmetic; off >= n - 1 puts sG + off on a 16-byte boundary
// (unit_origin).  FP64 keeps g(d), d = 0..n-1 (a mirror would not fit its
// LDS).
template <typename T> struct UnitRow;
template <> struct UnitRow<float> {
  const float* base;
  FSMI_DEV UnitRow(const float* sG, int off, int j) : base(sG + (off - j)) {}
  FSMI_DEV float operator()(int k) const { return base[k]; }
};
template <> struct UnitRow<double> {
  const double* g;
  int j;
  FSMI_DEV UnitRow(const double* sG, int, int jj) : g(sG), j(jj) {}
  FSMI_DEV double operator()(int k) const { return g[abs(k - j)]; }
};

// The mirror's origin: the least off >= n - 1 with sG + off 16-byte aligned
// (sG is at least 4-byte aligned).
FSMI_DEV int unit_origin(const float* sG, int n) {
  const int mis = (int)((reinterpret_cast<uintptr_t>(sG) >> 2) + (uintptr_t)(n - 1)) & 3;
  return n - 1 + ((4 - mis) & 3);
}

// Eight pairs per compensated add, as on explicit boundaries.
template <typename T>
FSMI_DEV double row_exact_unit(const T* sG, const T* sC, int off, int n, int j) {
  const UnitRow<T> w(sG, off, j);
  Acc<T> acc;
  int k = 1;
  for (; k + 7 <= n; k += 8) {
    T p = sC[k - 1] * w(k);
#pragma unroll
    for (int q = 1; q < 8; ++q) p = fma(sC[k - 1 + q], w(k + q), p);
    acc.add(p);
  }
  for (; k <= n; ++k) acc.add(sC[k - 1] * w(k));
  return acc.value();
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The FP32 unit-cell double sum of Thm 1, sum_j P_j sum_k C_k g(|j - k|), on
// the matrix cores.  With the cells in blocks of 16, the weight between a cell
// of row block r and one of column block s depends only on t = r - s and on
// the two offsets a, b within the blocks, so for each t >= 0
//   M_t[a][b] = sum_s P[16(s + t) + a] C[16 s + b]  (+ C[16(s + t) + a] P[16 s + b], t > 0)
// is a 16 x 16 product over the blocks s (the second term holds the pairs below
// the diagonal, which meet the same weight g(|16 t + a - b|)), and the sum is
// sum_t sum_{a,b} g(|16 t + a - b|) M_t[a][b]: every pair (j, k) once.
// v_mfma_f32_16x16x4f32 takes four blocks s per step: lane l gives the A
// value of row l % 16 and the B value of column l % 16 for block l / 16 of the
// step, so both operands are 64 consecutive floats, and it returns rows
// 4 (l / 16) .. + 3 of column l % 16.  Values past the beam read as zero.
// Four offsets t0 .. t0 + 3 go together: they share the column operands of a
// step (C and P at block s), and their eight products are independent chains.
// A group deals the sets of four to its waves in a snake order; a wave
// accumulates M_t in FP32 over the blocks, weights its four entries in FP32
// and adds that in FP64.  sG is the mirrored FP32 weight table (unit_origin).
template <int NW, bool BLOCK>
FSMI_DEV double exact_unit_mfma(const float* sG, const float* sC, const float* sP, int off, int n,
                                int tid) {
  const int lane = tid & 63;
  const int wv = BLOCK ? __builtin_amdgcn_readfirstlane(tid >> 6) : 0;
  const int nb = (n + 15) >> 4;
  const int ng = (nb + 3) >> 2;
  const int ra = 4 * (lane >> 4) - (lane & 15);   // row - column of this lane's first output
  double tot = 0.0;
  for (int g = 0; g < ng; ++g) {
    if constexpr (BLOCK) {
      const int r = g % (2 * NW);
      if ((r < NW ? r : 2 * NW - 1 - r) != wv) continue;
    }
    const int t0 = 4 * g;
    const int steps = (nb - t0 + 3) >> 2;
    // steps q < qf read only cells below n: 16 (t0 + 3) + 64 q + 63 < n
    const int rem = n - 16 * t0 - 112;
    const int qf = rem >= 0 ? min(steps, (rem >> 6) + 1) : 0;
    f32x4 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = f32x4{0.f, 0.f, 0.f, 0.f};
      b[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const float* pr = sP + 16 * t0 + lane;
    const float* cr = sC + 16 * t0 + lane;
    // full steps in pairs, software-pipelined: the operands of one step (ten
    // reads) are in flight while the other step's eight products run
    int q = 0;
    float ac = 0.f, ap = 0.f, ax[4], ay[4];
    auto load = [&](int qq, float& c0, float& p0, float (&x)[4], float (&y)[4]) {
      const int o = 64 * qq;
      c0 = sC[o + lane];
      p0 = sP[o + lane];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = pr[o + 16 * u];
        y[u] = cr[o + 16 * u];
      }
    };
    auto step = [&](float c0, float p0, const float (&x)[4], const float (&y)[4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u], c0, a[u], 0, 0, 0);
        b[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(y[u], p0, b[u], 0, 0, 0);
      }
    };
    if (qf > 0) load(0, ac, ap, ax, ay);
    for (; q + 1 < qf; q += 2) {
      float bc, bp, bx[4], by[4];
      load(q + 1, bc, bp, bx, by);
      step(ac, ap, ax, ay);
      if (q + 2 < qf) load(q + 2, ac, ap, ax, ay);
      step(bc, bp, bx, by);
    }
    if (q < qf) {
      step(ac, ap, ax, ay);
      ++q;
    }
    for (; q < steps; ++q) {   // the last steps: cells at n and beyond are zero
      const int ib = 64 * q + lane, jb = min(ib, n - 1);
      const float c0 = ib < n ? sC[jb] : 0.f, p0 = ib < n ? sP[jb] : 0.f;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (16 * (t0 + u) + 64 * q >= n) break;   // this offset's rows are all past the beam
        const int ia = 16 * (t0 + u) + ib, ja = min(ia, n - 1);
        const float x = ia < n ? sP[ja] : 0.f, y = ia < n ? sC[ja] : 0.f;
        a[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, c0, a[u], 0, 0, 0);
        b[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(y, p0, b[u], 0, 0, 0);
      }
    }
    // weights g(|16 t + a - b|); offsets of n or more meet products of zero
    // (weight zero); at t = 0 the second product repeats the first
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u;
      if (t >= nb) break;
      float w[4];
      if (16 * t + 15 < n && n >= 16) {
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = sG[off + 16 * t + ra + r];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int dd = 16 * t + ra + r;
          const int dc = max(-(n - 1), min(dd, n - 1));
          w[r] = (dd < n && dd > -n) ? sG[off + dc] : 0.f;
        }
      }
      const float k2 = t > 0 ? 1.f : 0.f;
      float acc = fmaf(k2, b[u][0], a[u][0]) * w[0];
#pragma unroll
      for (int r = 1; r < 4; ++r) acc = fmaf(fmaf(k2, b[u][r], a[u][r]), w[r], acc);
      tot += (double)acc;
    }
  }
  return tot;
}

template <typename T>
FSMI_DEV double row_approx_unit(const T* sG, const T* sC, int off, int n, int j, int D) {
  const UnitRow<T> w(sG, off, j);
  Acc<T> acc;
  const int k0 = max(1, j - D), k1 = min(n, j + D);
  for (int b = k0; b <= k1; b += 8) {
    const int e = min(b + 7, k1);
    T p = T(0);
    for (int k = b; k <= e; ++k) p = fma(sC[k - 1], w(k), p);
    acc.add(p);
  }
  return acc.value();
}

// LDS the core needs besides o: A = FP64 [cap+1], C and P = T [cap] each.
template <typename T>
__host__ __device__ constexpr int core_bytes_per_cell() { return 8 + 2 * (int)sizeof(T); }

struct CoreLds {
  double* A;   // boundaries l_1..l_{n+1} on entry (explicit bounds); D prefix; kernel table
  void* C;     // C_k
  void* P;     // P(e_j)
  const float2* lut = nullptr;   // the look-up tables in LDS (LUT mode)
};

// The beam's mutual information, valid in every lane of the group.
// so[0..n): occupancies; with explicit bounds A[0..n] holds l_1..l_{n+1}.
// *bad is set (group-uniform) when an input is invalid; the result is then NaN.
// MASK: only the cells i with counted[i] != 0 add their information (cell
// marking along a trajectory, Sec. 2.4): by Lemma 1 the f terms of the other
// cells leave C_k, while every cell still shapes P(e_j).
template <int NW, bool BLOCK, typename T, bool MASK = false, bool LUT = false>
FSMI_DEV double beam_core(const EvalConst& ec, int n, const float* so, bool has_bound, double sigma,
                          const CoreLds& L, double* scratch, int* flag, int tid, bool bad_in,
                          bool* bad_out, const unsigned char* counted = nullptr) {
  constexpr int G = Grp<NW, BLOCK>::size;
  double* sA = L.A;
  T* sC = reinterpret_cast<T*>(L.C);
  T* sP = reinterpret_cast<T*>(L.P);
  const double docc = ec.delta_occ, demp = 1.0 / ec.delta_occ;
  const double ldo = log(ec.delta_occ), lde = -ldo;
  const FConst ko = f_const(docc), ke = f_const(demp);
  const bool uni = ec.variant == FSMI_UNIFORM;
  bool bad = bad_in;
  if (!(sigma > 0.0) && !uni) bad = true;
  if (has_bound && !uni) {
    for (int i = tid + 1; i <= n; i += G)
      if (!(sA[i] >= sA[i - 1])) bad = true;
  }
  // ---- per-cell f, Alg 2 and Alg 3 (FP64 scans) ----
  // Each lane takes kv consecutive cells of a chunk of kv * G (kv <= 4, as
  // many as the cells left need, so a short tail does not evaluate f for
  // empty slots): it scans them in order itself, and one group scan over the
  // lanes' totals serves all kv.  A lane reads o_i and writes P_i only at its
  // own cells (P may share o's storage).
  double carryC = 0.0, carryE = 1.0, carryD = 0.0;
  for (int base = 0; base < n;) {
    const int kv = min(4, (n - base + G - 1) / G);   // group-uniform
    const int i0 = base + kv * tid;
    float of[4];
    double fo[4], qin[4], ein[4];
    double qs = 0.0, es = 1.0;   // this lane's running sum of f_emp, product of 1 - o
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= kv) break;
      const bool v = i0 + u < n;
      of[u] = v ? so[i0 + u] : 0.0f;
      if (v && !(of[u] >= 0.0f && of[u] <= 1.0f)) bad = true;
      const double o = (double)of[u];
      double fe;
      if constexpr (LUT) {
        fo[u] = lut_f(L.lut, o);
        fe = lut_f(L.lut, 1.0 - o);
      } else if constexpr (sizeof(T) == 4) {
        fo[u] = f_cell_series(ko, o);
        fe = f_cell_series(ke, o);
      } else {
        fo[u] = f_cell<double>(docc, ldo, o);
        fe = f_cell<double>(demp, lde, o);
      }
      if (!v) fo[u] = fe = 0.0;
      if constexpr (MASK) {
        if (v && !counted[i0 + u]) fo[u] = fe = 0.0;
      }
      qin[u] = qs;
      ein[u] = es;
      qs += fe;
      es *= v ? 1.0 - o : 1.0;
    }
    const double q = group_scan_excl<NW, BLOCK, OpAdd>(qs, carryC, scratch, tid);
    const double E = group_scan_excl<NW, BLOCK, OpMul>(es, carryE, scratch, tid);
    double Ck[4], ds = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= kv) break;
      Ck[u] = (q + qin[u]) + fo[u];
      if (i0 + u < n) {
        sC[i0 + u] = (T)Ck[u];
        sP[i0 + u] = (T)((E * ein[u]) * (double)of[u]);
        ds += Ck[u];
      }
    }
    if (uni) {  // D_k = sum_{i<=k} C_i in FP64 at A[k], A[0] = 0
      double d = group_scan_excl<NW, BLOCK, OpAdd>(ds, carryD, scratch, tid);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u >= kv) break;
        if (i0 + u < n) {
          d += Ck[u];
          sA[i0 + u + 1] = d;
        }
      }
      if (tid == 0 && base == 0) sA[0] = 0.0;
    }
    base += kv * G;
  }
  const double c = 1.0 / (sigma * 1.4142135623730951);
  if (!uni && !has_bound) {
    // g(d) = Phi((d+1/2)/sigma) - Phi((d-1/2)/sigma), d = 0..n-1; FP32 also
    // stores the mirror image (UnitRow), in the 2(n+1) floats of A
    T* sG = reinterpret_cast<T*>(sA);
    int off = 0;
    if constexpr (sizeof(T) == 4) off = unit_origin(sG, n);
    for (int d = tid; d < n; d += G) {
      T g;
      if (ec.kernel == FSMI_KERNEL_DENSITY) {
        // exp(-d^2 / (2 sigma^2)) / (sqrt(2 pi) sigma) = exp(-(d c)^2) c / sqrt(pi)
        const double z = d * c;
        g = (T)(exp(-z * z) * c * 0.56418958354775628695);
      } else if (d == 0) {
        g = erf_t<T>((T)(0.5 * c));
      } else {
        g = T(0.5) * (erfc_pos((T)((d - 0.5) * c)) - erfc_pos((T)((d + 0.5) * c)));
      }
      if constexpr (sizeof(T) == 4) {
        sG[off + d] = g;
        sG[off - d] = g;
      } else {
        sG[d] = g;
      }
    }
  }
  const bool any_bad = group_any<NW, BLOCK>(bad, flag, tid);
  *bad_out = any_bad;
  Grp<NW, BLOCK>::sync();
  // range-dependent noise keeps the boundaries in their own units (RowFrame)
  const bool rd = ec.slope != 0.0;
  if (has_bound && !uni && !any_bad && !rd) {
    // scale the boundaries once: the weight argument becomes |L_b - M_j|
    const double s = sizeof(T) == 8 ? c : c * (double)kSqrtL2E * (LUT ? (double)kLutInvH : 1.0);
    for (int i = tid; i <= n; i += G) sA[i] *= s;
    Grp<NW, BLOCK>::sync();
  }

  // ---- the double sum ----
  double tot = 0.0;
  if (!any_bad) {
    if (uni) {
      const double inv = 1.0 / (2.0 * ec.H + 1.0);
      for (int j = tid + 1; j <= n; j += G) {
        const int hi = min(n, j + ec.H), lo = max(0, j - ec.H - 1);
        tot += (double)sP[j - 1] * ((sA[hi] - sA[lo]) * inv);
      }
    } else if (has_bound) {
      if (ec.variant == FSMI_EXACT && (ec.flags & FSMI_F_SKIP_ZERO)) {
        for (int j = tid + 1; j <= n; j += G) tot += (double)sP[j - 1] * row_exact_band<T>(sA, sC, n, j);
      } else if (ec.variant == FSMI_EXACT && (rd || (ec.flags & FSMI_F_MAX_RANGE))) {
        // q_n = carryC (the sum of f_emp over the beam), P(e_0) = carryE
        const double tq = (ec.flags & FSMI_F_MAX_RANGE) ? 0.5 * carryC : 0.0;
        if (rd) tot = exact_rows_ext<G, T, true>(sA, sC, sP, n, tid, sigma, ec.slope, tq);
        else tot = exact_rows_ext<G, T, false>(sA, sC, sP, n, tid, sigma, 0.0, tq);
        if (tid == 0 && (ec.flags & FSMI_F_MAX_RANGE)) tot += carryC * carryE;
      } else if (ec.variant == FSMI_EXACT) {
        tot = exact_rows<G, T, LUT>(sA, sC, sP, n, tid, L.lut);
      } else {
        for (int j = tid + 1; j <= n; j += G)
          tot += (double)sP[j - 1] * row_approx_bound<T, LUT>(sA, sC, n, j, ec.Delta, L.lut);
      }
    } else {
      const T* sG = reinterpret_cast<const T*>(sA);
      int off = 0;
      if constexpr (sizeof(T) == 4) off = unit_origin(sG, n);
      if (ec.variant == FSMI_EXACT) {
        if constexpr (sizeof(T) == 4) {
          tot = exact_unit_mfma<NW, BLOCK>(sG, sC, sP, off, n, tid);
        } else {
          for (int j = tid + 1; j <= n; j += G) tot += (double)sP[j - 1] * row_exact_unit<T>(sG, sC, off, n, j);
        }
      } else {
        for (int j = tid + 1; j <= n; j += G)
          tot += (double)sP[j - 1] * row_approx_unit<T>(sG, sC, off, n, j, ec.Delta);
      }
    }
  }
  const double s = group_sum<NW, BLOCK>(tot, scratch, tid);
  Grp<NW, BLOCK>::sync();
  return any_bad ? __builtin_nan("") : s;
}

}  // namespace fsmi
