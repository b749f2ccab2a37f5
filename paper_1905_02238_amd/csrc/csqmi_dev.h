// csqmi_dev.h -- the comparison metric of Sec. 2.3 (CSQMI) on one beam staged in
// LDS, evaluated by a group of lanes (one wave, or a whole workgroup):
// Eq. csqmi_exact with both double sums truncated to |l - j| <= Delta, the
// Approx-CSQMI of Sec. 2.3 / Sec. 3.4 (Delta >= n - 1 is the exact sum).
//
// With q_i = o_i^2 + (1 - o_i)^2 and Q = prod_i q_i, the weight of a first hit
// at l is w_l = P(e_l)^2 prod_{i>l} q_i (the sum of P(m)^2 over the maps whose
// first occupied cell is l), w_0 = P(e_0)^2.  All three sums of the equation
// carry the factors Q and N(0, 2 sigma^2), so with
//   u_l  = w_l / Q = (o_l^2 / q_l) prod_{i<l} (1 - o_i)^2 / q_i,
//   u_0  = prod_i (1 - o_i)^2 / q_i,
//   e_jl = exp(-(mu_l - mu_j)^2 / (4 sigma^2)),
//   C''  = P(e_0)^2 + sum_j sum_l P(e_j) P(e_l) e_jl,
//   A''  = P(e_0) u_0 + sum_j sum_l P(e_j) u_l e_jl,
// the value log B + log C - 2 log A is log(sum_{l=0}^{n} u_l) + log C'' -
// 2 log A'': the factors cancel exactly.  Every u_l lies in [0, 1], so no sum
// overflows or underflows however long the beam.  The all-free event e_0
// reads beyond the beam (as in Thm 1), so only its self terms remain.
//
// Numerics follow the FSMI engine: P(e_j) and the u_l prefix products are
// scanned in FP64; the pair loop runs in T with the Gaussian as one 2^(-y^2)
// (y the scaled distance of the two cell centres, formed in FP64), in chains
// of eight pairs added to FP64 row sums.
#pragma once
#include <math.h>

#include "beam_dev.h"

namespace fsmi {

template <typename T> FSMI_DEV T exp2_neg_sq(T y);
template <> FSMI_DEV float exp2_neg_sq<float>(float y) { return __builtin_amdgcn_exp2f(-(y * y)); }
template <> FSMI_DEV double exp2_neg_sq<double>(double y) { return exp2(-(y * y)); }

// The beam's CSQMI, valid in every lane of the group (NaN on bad input, with
// *bad_out set group-uniformly).  so[0..n): occupancies; with explicit bounds
// A[0..n] holds l_1..l_{n+1}.  LDS use: A -> scaled cell centres, C -> u_l,
// P -> P(e_j) (P may share o's storage: a lane writes P_i only where it read o_i).
template <int NW, bool BLOCK, typename T>
FSMI_DEV double csqmi_core(const EvalConst& ec, int n, const float* so, bool has_bound,
                           double sigma, const CoreLds& L, double* scratch, int* flag, int tid,
                           bool bad_in, bool* bad_out) {
  constexpr int G = Grp<NW, BLOCK>::size;
  double* sA = L.A;
  T* sU = reinterpret_cast<T*>(L.C);
  T* sP = reinterpret_cast<T*>(L.P);
  bool bad = bad_in;
  if (!(sigma > 0.0)) bad = true;
  if (has_bound) {
    for (int i = tid + 1; i <= n; i += G)
      if (!(sA[i] >= sA[i - 1])) bad = true;
  }
  // ---- P(e_j) (Alg 2) and u_l: FP64 prefix products, up to four cells per lane ----
  double carryE = 1.0, carryR = 1.0, usum = 0.0;
  for (int base = 0; base < n;) {
    const int kv = min(4, (n - base + G - 1) / G);   // group-uniform
    const int i0 = base + kv * tid;
    float of[4];
    double ein[4], rin[4];
    double es = 1.0, rs = 1.0;   // this lane's running products of 1 - o and (1 - o)^2 / q
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= kv) break;
      const bool v = i0 + u < n;
      of[u] = v ? so[i0 + u] : 0.0f;
      if (v && !(of[u] >= 0.0f && of[u] <= 1.0f)) bad = true;
      const double o = (double)of[u], om = 1.0 - o;
      const double q = fma(o, o, om * om);
      ein[u] = es;
      rin[u] = rs;
      es *= v ? om : 1.0;
      rs *= v ? (om * om) / q : 1.0;
    }
    const double E = group_scan_excl<NW, BLOCK, OpMul>(es, carryE, scratch, tid);
    const double R = group_scan_excl<NW, BLOCK, OpMul>(rs, carryR, scratch, tid);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= kv) break;
      if (i0 + u < n) {
        const double o = (double)of[u], om = 1.0 - o;
        const double q = fma(o, o, om * om);
        const double ul = (R * rin[u]) * ((o * o) / q);
        sP[i0 + u] = (T)((E * ein[u]) * o);
        sU[i0 + u] = (T)ul;
        usum += ul;
      }
    }
    base += kv * G;
  }
  // ---- scaled cell centres y_j = mu_j sqrt(log2 e) / (2 sigma), into A[j-1] ----
  const double hs = 0.6005612043932249 / sigma;   // sqrt(log2 e) / 2
  if (has_bound) {
    // in place, a chunk of G centres at a time: every lane reads its two
    // boundaries before any lane of the chunk overwrites one
    for (int base = 0; base < n; base += G) {
      const int j = base + tid + 1;
      double y = 0.0;
      if (j <= n) y = (0.5 * (sA[j - 1] + sA[j])) * hs;
      Grp<NW, BLOCK>::sync();
      if (j <= n) sA[j - 1] = y;
      Grp<NW, BLOCK>::sync();
    }
  } else {
    for (int j = tid + 1; j <= n; j += G) sA[j - 1] = ((double)j - 0.5) * hs;
  }
  const bool any_bad = group_any<NW, BLOCK>(bad, flag, tid);
  *bad_out = any_bad;
  Grp<NW, BLOCK>::sync();

  // ---- the two truncated double sums, one row j per lane ----
  const int D = ec.Delta;
  double Au = 0.0, Cp = 0.0;
  if (!any_bad) {
    for (int j = tid + 1; j <= n; j += G) {
      const double yj = sA[j - 1];
      const int k0 = D >= j - 1 ? 1 : j - D;
      const int k1 = D >= n - j ? n : j + D;
      double ru = 0.0, rp = 0.0;
      for (int b = k0; b <= k1; b += 8) {
        const int e = min(b + 7, k1);
        T su = T(0), sp = T(0);
        for (int k = b; k <= e; ++k) {
          const T w = exp2_neg_sq<T>((T)(sA[k - 1] - yj));
          su = fma(sU[k - 1], w, su);
          sp = fma(sP[k - 1], w, sp);
        }
        ru += (double)su;
        rp += (double)sp;
      }
      const double pj = (double)sP[j - 1];
      Au += pj * ru;
      Cp += pj * rp;
    }
  }
  const double us = group_sum<NW, BLOCK>(usum, scratch, tid);
  const double as = group_sum<NW, BLOCK>(Au, scratch, tid);
  const double cs = group_sum<NW, BLOCK>(Cp, scratch, tid);
  Grp<NW, BLOCK>::sync();
  if (any_bad) return __builtin_nan("");
  // e_0: P(e_0) = carryE, u_0 = carryR
  const double u_tot = us + carryR;
  const double a2 = as + carryE * carryR;
  const double c2 = cs + carryE * carryE;
  return log(u_tot) + log(c2) - 2.0 * log(a2);
}

}  // namespace fsmi

namespace fsmi {
// The per-beam evaluation of the 2D paths: FSMI's variants (beam_core) or, in
// kernels instantiated for it (CSQ), the CSQMI comparator, so the FSMI kernels
// compile without the comparator's code.
template <int NW, bool BLOCK, typename T, bool CSQ, bool LUT = false>
FSMI_DEV double beam_eval(const EvalConst& ec, int n, const float* so, bool has_bound,
                          double sigma, const CoreLds& L, double* scratch, int* flag, int tid,
                          bool bad_in, bool* bad_out) {
  if constexpr (CSQ)
    return csqmi_core<NW, BLOCK, T>(ec, n, so, has_bound, sigma, L, scratch, flag, tid, bad_in,
                                    bad_out);
  else
    return beam_core<NW, BLOCK, T, false, LUT>(ec, n, so, has_bound, sigma, L, scratch, flag, tid,
                                               bad_in, bad_out);
}
}  // namespace fsmi
