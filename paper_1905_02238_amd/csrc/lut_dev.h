// lut_dev.h -- the look-up-table mode of Sec. 3.3 (FSMI_F_LUT, opt-in): the
// normal distribution's tail and f(delta_occ, .) are tabulated once per call
// and read with linear interpolation, in place of one erfc per (row,
// boundary) pair and two f series per cell.
//
// Tail table: E_i = erfc(y_i / sqrt(log2 e)) at y_i = i / kLutInvH,
// i < kLutPhiN, on the FP32 mode's scaled argument y = |l - mu| c sqrt(log2 e)
// (c = 1/(sigma sqrt 2)); with the boundaries scaled by kLutInvH as well, a
// pair's table coordinate is x = |L - M| with no multiply.  Entry i holds
// (E_i, E_{i+1} - E_i), E_{kLutPhiN} = 0, and one more entry (0, 0) that
// every x >= kLutPhiN reads (erfc of y >= 12 is below FP32's normal range),
// so no select is needed.  Linear interpolation at this step is within 6e-6
// of erfc.
// f table: f(delta_occ, o) at o_i = i / (kLutFN - 1), entry i holding
// (f_i, f_{i+1} - f_i); f(delta_emp, o) = f(delta_occ, 1 - o) for
// delta_emp = 1 / delta_occ (the odds r become 1/r), so one table serves both.
// The tables are built in FP64 and rounded to FP32 (k_build_lut), and a
// kernel stages them into its LDS before its first beam.
#pragma once
#include "fsmi_dev.h"

namespace fsmi {

constexpr int kLutPhiN = 1536;
constexpr float kLutInvH = 128.0f;
constexpr int kLutFN = 512;
constexpr int kLutEntries = kLutPhiN + 1 + kLutFN;   // tail, its zero entry, f
constexpr size_t kLutBytes = 8 * (size_t)kLutEntries;

// erfc at table coordinate x >= 0.
FSMI_DEV float lut_tail(const float2* tab, float x) {
  const int i = min((int)x, kLutPhiN);
  const float2 e = tab[i];
  return fmaf(__builtin_amdgcn_fractf(x), e.y, e.x);
}

// f(delta_occ, o) for o in [0, 1].
FSMI_DEV double lut_f(const float2* tab, double o) {
  const float x = (float)o * (float)(kLutFN - 1);
  const int i = min((int)x, kLutFN - 2);
  const float2 e = tab[kLutPhiN + 1 + i];
  return (double)fmaf(x - (float)i, e.y, e.x);
}

// Copies the kLutBytes of tables from global memory into LDS (all threads of
// the workgroup take part; the caller synchronises).
FSMI_DEV void lut_stage(float2* dst, const float2* src, int tid, int nthreads) {
  for (int i = tid; i < kLutEntries; i += nthreads) dst[i] = src[i];
}

}  // namespace fsmi
