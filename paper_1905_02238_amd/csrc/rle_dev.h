// rle_dev.h -- FSMI-RLE (Thm 5) and Approx-FSMI-RLE (Thm 6) on a beam of equal-
// width virtual cells held as runs (Sec. 4), evaluated by one wave in the run
// domain.
//
// A run u covers cells k0_u .. k1_u (1-based) of one occupancy o_u.  Inside a
// run the info-gain term is linear in the cell's offset b = k - k0_u:
//   C_k = D_E(u) + b f(delta_emp, r_u) + f(delta_occ, r_u)        (Lemma 1, Alg 6),
// so a row j's inner sum S_j = sum_k C_k g(k - j) splits into one term per run,
//   S_j = sum_v [ (D_E(v) + f_occ(v)) W0_v(j) + f_emp(v) W1_v(j) ],
//   W0_v(j) = sum_{k in v} g(k - j),   W1_v(j) = sum_{k in v} (k - k0_v) g(k - j),
// the two block sums of the proof of Thm 5 for a single row.  Both come from
// two tail tables of the (symmetric) kernel, read at the run's ends:
//   Tg(d) = sum_{e >= d} g(e),   D1(d) = sum_{e >= d} e g(e),   d >= 1,
// with the part of run v right of j at distances dR0..dR1, the part left of j
// at eL0..eL1, and the cell k = j itself weighted g(0):
//   W0 = [j in v] g(0) + (Tg(dR0) - Tg(dR1 + 1)) + (Tg(eL0) - Tg(eL1 + 1)),
//   W1 = (j - k0_v) W0 + (D1(dR0) - D1(dR1 + 1)) - (D1(eL0) - D1(eL1 + 1)).
// Only differences of tails appear, and no power of x: the paper's block
// tables multiply by x^{-t}, which overflows and cancels (Sec. 4.1).  A row
// visits only the runs within the
// kernel's reach: Delta for Approx-FSMI-RLE (the kernel truncated at
// |d| <= Delta, Thm 6 read with the truncated kernel inside the blocks), and
// for FSMI-RLE the last distance at which the kernel table is non-zero in the
// working precision; pairs farther apart have a zero weight in the dense
// expanded sum as well, so the value is the expanded sum's up to rounding.
// P(e_j) comes from Alg 2 on the cells (one FP64 prefix product); f once per
// run; D_E by a prefix sum over runs (Alg 6).  The cost is O(n x runs in reach)
// instead of O(n^2).
#pragma once
#include <math.h>

#include "beam_dev.h"

namespace fsmi {

constexpr int kRunCap = 64;   // runs one wave evaluates in the run domain

// Maximum over the wave's lanes (wave-uniform).
FSMI_DEV int wave_max_i(int v) {
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return __builtin_amdgcn_readfirstlane(v);
}

struct RunLds {
  float* ro;   // [kRunCap] run values
  int* rs;     // [kRunCap + 1] run starts (0-based cell index), rs[nr] = n
  int* ru;     // [cap] run of each cell
  void* c0;    // [kRunCap] T: D_E(u) + f(delta_occ, r_u)
  void* fe;    // [kRunCap] T: f(delta_emp, r_u)
  void* tab;   // [2][cap + 2] T: Tg then D1
};

// Bytes of the run region: the per-run arrays and the two tail tables.
template <typename T>
__host__ __device__ constexpr size_t run_region_bytes(int cap) {
  return (size_t)4 * kRunCap + (size_t)4 * (kRunCap + 1) + 2 * sizeof(T) * (size_t)kRunCap +
         2 * sizeof(T) * ((size_t)cap + 2) + 16;
}

template <typename T>
FSMI_DEV RunLds carve_runs(char* p, int cap, int* ru) {
  RunLds R;
  R.c0 = p;
  R.fe = p + sizeof(T) * kRunCap;
  R.tab = p + 2 * sizeof(T) * kRunCap;
  char* q = p + 2 * sizeof(T) * kRunCap + 2 * sizeof(T) * ((size_t)cap + 2);
  R.ro = reinterpret_cast<float*>(q);
  R.rs = reinterpret_cast<int*>(q + 4 * kRunCap);
  R.ru = ru;
  return R;
}

// Maximal runs of bit-identical o in so[0..n) (Eq. occup_rle): the run of each
// cell, and the first kRunCap runs' values and starts.  Returns the number of
// runs (wave-uniform); more than kRunCap means the run arrays are incomplete.
FSMI_DEV int runs_of_cells(const float* so, int n, const RunLds& R, int lane) {
  int carry = 0;
  for (int base = 0; base < n; base += kWave) {
    const int i = base + lane;
    int head = 0;
    if (i < n) head = (i == 0 || __float_as_uint(so[i]) != __float_as_uint(so[i - 1])) ? 1 : 0;
    const int inc = wave_scan_incl<OpAdd>(head);
    const int r = carry + inc - 1;
    if (i < n) {
      R.ru[i] = r;
      if (head && r < kRunCap) {
        R.ro[r] = so[i];
        R.rs[r] = i;
      }
    }
    carry += wave_last(inc);
  }
  if (lane == 0 && carry <= kRunCap) R.rs[carry] = n;
  wave_sync();
  return carry;
}

// Given runs (values, starts and lengths) of an RLE beam: the runs' arrays and
// the run of each cell, for runs r0 .. r1 - 1 of the caller's CSR arrays.
// Returns the number of cells, or -1 (bad length or more than cap cells);
// the caller has checked r1 - r0 <= kRunCap.
FSMI_DEV int runs_from_csr(const float* run_occ, const int32_t* run_len, int64_t r0, int64_t r1,
                           int cap, float* so, const RunLds& R, int lane) {
  const int nr = (int)(r1 - r0);
  const int u = lane;
  int Lu = u < nr ? run_len[r0 + u] : 0;
  const bool bad = u < nr && Lu <= 0;
  Lu = Lu > 0 ? Lu : 0;
  const int inc = wave_scan_incl<OpAdd>(Lu);
  const int s = inc - Lu;
  const int n = wave_last(inc);
  if (__any(bad) || n > cap) return -1;
  if (u < nr) {
    const float o = run_occ[r0 + u];
    R.ro[u] = o;
    R.rs[u] = s;
    for (int t = 0; t < Lu; ++t) {
      so[s + t] = o;
      R.ru[s + t] = u;
    }
  }
  if (lane == 0) R.rs[nr] = n;
  wave_sync();
  return n;
}

// The beam's FSMI-RLE (EXACT) or Approx-FSMI-RLE (APPROX) value, valid in every
// lane; nr <= kRunCap runs set up by runs_of_cells / runs_from_csr; so[0..n)
// the expanded occupancies (P(e_j) is scanned over them).  *bad_out: an input
// is invalid (group-uniform); the result is then NaN.
template <typename T>
FSMI_DEV double rle_core(const EvalConst& ec, int n, const float* so, int nr, const RunLds& R,
                         double sigma, const CoreLds& L, int lane, bool* bad_out) {
  T* sP = reinterpret_cast<T*>(L.P);
  T* c0 = reinterpret_cast<T*>(R.c0);
  T* fe = reinterpret_cast<T*>(R.fe);
  T* Tg = reinterpret_cast<T*>(R.tab);
  T* D1 = Tg + (n + 2);
  const double docc = ec.delta_occ, demp = 1.0 / ec.delta_occ;
  const double ldo = log(ec.delta_occ), lde = -ldo;
  bool bad = !(sigma > 0.0);
  // ---- per run: f (Sec. 2.2) and D_E(u) = sum_{v<u} L_v f(delta_emp, r_v) (Alg 6) ----
  {
    double fo_u = 0.0, fe_u = 0.0, len = 0.0;
    if (lane < nr) {
      const float of = R.ro[lane];
      if (!(of >= 0.0f && of <= 1.0f)) bad = true;
      const double o = (double)of;
      if constexpr (sizeof(T) == 4) {
        fo_u = f_cell_series(f_const(docc), o);
        fe_u = f_cell_series(f_const(demp), o);
      } else {
        fo_u = f_cell<double>(docc, ldo, o);
        fe_u = f_cell<double>(demp, lde, o);
      }
      len = (double)(R.rs[lane + 1] - R.rs[lane]);
    }
    double carry = 0.0;
    const double DE = group_scan_excl<1, false, OpAdd>(len * fe_u, carry, nullptr, lane);
    if (lane < nr) {
      c0[lane] = (T)(DE + fo_u);
      fe[lane] = (T)fe_u;
    }
  }
  // ---- P(e_j) = o_j prod_{l<j} (1 - o_l) (Alg 2), FP64 prefix product ----
  double carryE = 1.0;
  for (int base = 0; base < n;) {
    const int kv = min(4, (n - base + kWave - 1) / kWave);   // wave-uniform
    const int i0 = base + kv * lane;
    double es = 1.0, ein[4];
    float of[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= kv) break;
      const bool v = i0 + u < n;
      of[u] = v ? so[i0 + u] : 0.0f;
      ein[u] = es;
      es *= v ? 1.0 - (double)of[u] : 1.0;
    }
    const double E = group_scan_excl<1, false, OpMul>(es, carryE, nullptr, lane);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= kv) break;
      if (i0 + u < n) sP[i0 + u] = (T)((E * ein[u]) * (double)of[u]);
    }
    base += kv * kWave;
  }
  // ---- the kernel g(d), d = 0 .. n-1 (Eq. G_jk on unit cells, or the density
  // form), truncated at Delta for APPROX; tails summed in FP64 from the far end ----
  const double c = 1.0 / (sigma * 1.4142135623730951);
  const bool trunc = ec.variant == FSMI_APPROX;
  int far = -1;   // the largest d with g(d) != 0
  for (int d = lane; d < n; d += kWave) {
    T g;
    if (trunc && d > ec.Delta) {
      g = T(0);
    } else if (ec.kernel == FSMI_KERNEL_DENSITY) {
      const double z = d * c;
      g = (T)(exp(-z * z) * c * 0.56418958354775628695);
    } else if (d == 0) {
      g = erf_t<T>((T)(0.5 * c));
    } else {
      g = T(0.5) * (erfc_pos((T)((d - 0.5) * c)) - erfc_pos((T)((d + 0.5) * c)));
    }
    Tg[d] = g;
    if (g != T(0)) far = d;
  }
  far = wave_max_i(far);
  if (lane < 2) {
    Tg[n + lane] = T(0);
    D1[n + lane] = T(0);
  }
  wave_sync();
  const T g0 = Tg[0];
  {
    // suffix sums over d = 1 .. n-1 in chunks of 64 from the far end; lane l
    // of a chunk takes d = top - l, so an inclusive lane scan is the suffix sum
    double cg = 0.0, cd = 0.0;
    for (int top = n - 1; top >= 1; top -= kWave) {
      const int d = top - lane;
      const double g = d >= 1 ? (double)Tg[d] : 0.0;
      const double sg = wave_scan_incl<OpAdd>(g) + cg;
      const double sd = wave_scan_incl<OpAdd>((double)d * g * (d >= 1 ? 1.0 : 0.0)) + cd;
      cg = wave_last(sg);
      cd = wave_last(sd);
      wave_sync();
      if (d >= 1) {
        Tg[d] = (T)sg;
        D1[d] = (T)sd;
      }
    }
  }
  wave_sync();
  const int reach = max(far, 0);
  const bool any_bad = __any(bad);
  *bad_out = any_bad;
  // ---- rows: S_j over the runs within reach of row j ----
  double tot = 0.0;
  if (!any_bad) {
    for (int j = lane + 1; j <= n; j += kWave) {
      const int i = j - 1;
      const int v0 = R.ru[max(0, i - reach)], v1 = R.ru[min(n - 1, i + reach)];
      T acc = T(0);
      for (int v = v0; v <= v1; ++v) {
        const int k0 = R.rs[v] + 1, k1 = R.rs[v + 1];
        const int dR0 = max(k0 - j, 1), dR1 = k1 - j;   // right of j
        const int eL0 = max(j - k1, 1), eL1 = j - k0;   // left of j
        const int rb = dR1 >= dR0 ? dR1 + 1 : dR0;     // an empty side reads one entry twice
        const int lb = eL1 >= eL0 ? eL1 + 1 : eL0;
        const T W0 = ((k0 <= j && j <= k1) ? g0 : T(0)) + (Tg[dR0] - Tg[rb]) + (Tg[eL0] - Tg[lb]);
        const T W1 = (T)(j - k0) * W0 + (D1[dR0] - D1[rb]) - (D1[eL0] - D1[lb]);
        acc = fma(c0[v], W0, acc);
        acc = fma(fe[v], W1, acc);
      }
      tot += (double)sP[i] * (double)acc;
    }
  }
  const double s = wave_sum(tot);
  wave_sync();
  return any_bad ? __builtin_nan("") : s;
}

}  // namespace fsmi
