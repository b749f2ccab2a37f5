// k_rle_table.hip -- the paper's table route for Approx-FSMI-RLE: Alg 8 with the
// alpha/beta/theta/gamma tables of Alg 9 and 10, x = 1 - o quantised to a grid.
// It is kept beside the run engine (k_rle.hip) to reproduce the paper's
// run-length crossover and to measure the route's cancellation; the run engine
// is the accurate path.
//
// Tables, for x_i = i / levels, i = 0 .. levels, with the un-normalised
// Gaussian g(d) = exp(-d^2 / (2 sigma'^2)) truncated at |d| <= Delta (Thm 6's
// kernel):
//   alpha[x, P, Q] = sum_{a<P} sum_{b<Q} x^a g(a - b),  beta adds a factor b,
//     P, Q in [0, 2 Delta] (a block cropped by Eqs. su'..Lv' and shifted by t
//     reads entries up to 2 Delta);
//   theta[x, L] = alpha[x, L, L], gamma[x, L] = beta[x, L, L], L <= max_run.
// Per beam (one wave, the runs in LDS, a lane per run u):
//   I = (sum_u I_{u=v} + I_{u<v} + I_{u>v}) / (sqrt(2 pi) sigma'),
// with blocks cropped as in Thm 6, t = s'_u - s'_v:
//   t <= 0 (v after u):  A = alpha[L'_u, L'_v - t] - alpha[L'_u, -t],
//                        B = beta[L'_u, L'_v - t] - beta[L'_u, -t] + t A,
//                        weighted by P_E(u) (1 - o_u)^(s'_u - s_u);
//   t >= 1 (v before u): A = x^{-t} (alpha[t + L'_u, L'_v] - alpha[t, L'_v]),
//                        B = x^{-t} (beta[t + L'_u, L'_v] - beta[t, L'_v]),
//                        the route whose cancellation Sec. 4.1 warns about;
//                        at x = 0 the block is its first row,
//                        A = sum_{b<L'_v} g(t - b), B = sum_b b g(t - b).
// P_E, D_E and the crop factor use o itself; only table reads use the grid.
#include <math.h>

#include <algorithm>

#include "fsmi_dev.h"
#include "fsmi_internal.h"

namespace fsmi {
namespace {

constexpr int kTabRuns = 1024;     // runs per beam held in LDS (the larger of two kernels)
constexpr int kTabMaxRun = 4096;   // longest run the theta/gamma tables hold

// Neumaier-compensated FP64 sum.
struct CSum {
  double s = 0.0, c = 0.0;
  FSMI_DEV void add(double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  FSMI_DEV double value() const { return s + c; }
};

FSMI_DEV double gauss_trunc(double two_var, int Delta, int d) {
  if (d > Delta || d < -Delta) return 0.0;
  return exp(-((double)d * (double)d) / two_var);
}

// alpha and beta by their definitions: one thread per (i, P, Q).
__global__ void k_tab_alpha_beta(int levels, int Delta, double two_var, double* ab) {
  const int W = 2 * Delta + 1;
  const int64_t total = (int64_t)(levels + 1) * W * W;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / (W * W)), P = (int)(e / W % W), Q = (int)(e % W);
    const double x = (double)i / (double)levels;
    CSum sa, sb;
    for (int a = 0; a < P; ++a) {
      const double xa = pow(x, (double)a);
      for (int b = 0; b < Q; ++b) {
        const double w = gauss_trunc(two_var, Delta, a - b);
        sa.add(xa * w);
        sb.add((double)b * xa * w);
      }
    }
    double* t = ab + (int64_t)i * 2 * W * W;
    t[P * W + Q] = sa.value();
    t[W * W + P * W + Q] = sb.value();
  }
}

// theta and gamma.  theta[x, L] - theta[x, L - 1] is the new row a = L - 1
// (b < L) and the new column b = L - 1 (a < L - 1) of the band
// |a - b| <= Delta: first every increment, one thread per (i, L), then one
// thread per level adds them up in order (compensated).
__global__ void k_tab_tg_steps(int levels, int Delta, double two_var, int max_run, double* tg) {
  const int64_t total = (int64_t)(levels + 1) * max_run;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / max_run), L = (int)(e % max_run) + 1;
    const double x = (double)i / (double)levels;
    const int m = L - 1;
    const double xm = pow(x, (double)m);
    CSum st, sg;
    for (int b = max(0, m - Delta); b <= m; ++b) {   // row a = m
      const double w = gauss_trunc(two_var, Delta, m - b);
      st.add(xm * w);
      sg.add((double)b * xm * w);
    }
    for (int a = max(0, m - Delta); a < m; ++a) {    // column b = m
      const double w = pow(x, (double)a) * gauss_trunc(two_var, Delta, a - m);
      st.add(w);
      sg.add((double)m * w);
    }
    double* th = tg + (int64_t)i * 2 * (max_run + 1);
    th[L] = st.value();
    th[max_run + 1 + L] = sg.value();
  }
}

__global__ void k_tab_tg_prefix(int levels, int max_run, double* tg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > levels) return;
  double* th = tg + (int64_t)i * 2 * (max_run + 1);
  double* ga = th + (max_run + 1);
  th[0] = 0.0;
  ga[0] = 0.0;
  CSum st, sg;
  for (int L = 1; L <= max_run; ++L) {
    st.add(th[L]);
    sg.add(ga[L]);
    th[L] = st.value();
    ga[L] = sg.value();
  }
}

struct TabArgs {
  int64_t n_beams;
  const int64_t* run_off;
  const float* run_occ;
  const int32_t* run_len;
  double* mi;
  const double* ab;   // [levels + 1][2][W][W]
  const double* tg;   // [levels + 1][2][max_run + 1]
  double sigma_p, two_var, delta_occ, ln_occ, ln_emp;
  int Delta, levels, max_run;
  uint32_t* status;
};

// Run u's terms (Alg 8's u = v, v after u and v before u) of a beam whose
// nr runs sit in the LDS arrays s_*.
struct RunLds {
  const float* o;
  const int *L, *s;
  const double *P, *D, *fo, *fe;
};
FSMI_DEV double table_run_terms(const TabArgs& a, const RunLds& r, int u, int nr) {
  const int W = 2 * a.Delta + 1, Delta = a.Delta;
  const float* s_o = r.o;
  const int *s_L = r.L, *s_s = r.s;
  const double *s_P = r.P, *s_D = r.D, *s_fo = r.fo, *s_fe = r.fe;
  double acc = 0.0;
  const double ou = (double)s_o[u];
  const double x = 1.0 - ou;
  const int iq = (int)floor(x * (double)a.levels + 0.5);
  const double xq = (double)iq / (double)a.levels;
  const double* al = a.ab + (int64_t)iq * 2 * W * W;
  const double* be = al + W * W;
  const double* th = a.tg + (int64_t)iq * 2 * (a.max_run + 1);
  const double* ga = th + (a.max_run + 1);
  const int Lu = s_L[u], su = s_s[u];
  const double PE = s_P[u];
  acc += PE * ou * ((s_D[u] + s_fo[u]) * th[Lu] + s_fe[u] * ga[Lu]);
  // v after u: s_v increases with v
  for (int v = u + 1; v < nr && s_s[v] < su + Lu + Delta; ++v) {
    const int sv = s_s[v], Lv = s_L[v];
    const int su_p = max(su, sv - Delta);
    const int Lu_p = su + Lu - su_p;
    const int Lv_p = min(Lv, su + Lu + Delta - sv);
    const int t = su_p - sv;   // <= 0
    const double A = al[Lu_p * W + Lv_p - t] - al[Lu_p * W - t];
    const double B = be[Lu_p * W + Lv_p - t] - be[Lu_p * W - t] + (double)t * A;
    const double Pp = PE * pow(x, (double)(su_p - su));
    acc += Pp * ou * ((s_D[v] + s_fo[v]) * A + s_fe[v] * B);
  }
  // v before u: s_v + L_v decreases as v falls
  for (int v = u - 1; v >= 0 && su < s_s[v] + s_L[v] + Delta; --v) {
    const int sv = s_s[v], Lv = s_L[v];
    const int Lu_p = min(Lu, sv + Lv + Delta - su);
    const int sv_p = max(sv, su - Delta);
    const int Lv_p = sv + Lv - sv_p;
    const int t = su - sv_p;   // >= 1
    double A, B;
    if (iq == 0) {
      double sa = 0.0, sb = 0.0;
      for (int k = 0; k < Lv_p; ++k) {
        const double w = gauss_trunc(a.two_var, Delta, t - k);
        sa += w;
        sb += (double)k * w;
      }
      A = sa;
      B = sb;
    } else {
      const double xt = pow(xq, (double)(-t));
      A = xt * (al[(t + Lu_p) * W + Lv_p] - al[t * W + Lv_p]);
      B = xt * (be[(t + Lu_p) * W + Lv_p] - be[t * W + Lv_p]);
    }
    const double Dp = s_D[v] + (double)(sv_p - sv) * s_fe[v];
    acc += PE * ou * ((Dp + s_fo[v]) * A + s_fe[v] * B);
  }
  return acc;
}

template <int RUNS>
__global__ __launch_bounds__(kWave) void k_rle_table(TabArgs a) {
  __shared__ float s_o[RUNS];
  __shared__ int s_L[RUNS], s_s[RUNS];
  __shared__ double s_P[RUNS], s_D[RUNS], s_fo[RUNS], s_fe[RUNS];
  const int lane = threadIdx.x;
  const double delta_emp = 1.0 / a.delta_occ;
  for (int64_t it = blockIdx.x; it < a.n_beams; it += gridDim.x) {
    const int64_t r0 = a.run_off[it], r1 = a.run_off[it + 1];
    if (r1 < r0 || r1 - r0 > RUNS) {
      if (lane == 0) {
        latch(a.status, r1 < r0 ? kErrLen : kErrCap);
        a.mi[it] = __builtin_nan("");
      }
      continue;
    }
    const int nr = (int)(r1 - r0);
    // pass 1: the runs, their starts s, D_E (exclusive sums of L f_emp) and
    // P_E (exclusive products of (1 - o)^L), in chunks of 64 runs
    bool bad_o = false, bad_l = false, bad_c = false;
    int carry_s = 0;
    double carry_D = 0.0, carry_P = 1.0;
    for (int base = 0; base < nr; base += kWave) {
      const int u = base + lane;
      const bool valid = u < nr;
      const float o = valid ? a.run_occ[r0 + u] : 0.0f;
      int L = valid ? a.run_len[r0 + u] : 0;
      if (valid && !(o >= 0.0f && o <= 1.0f)) bad_o = true;
      if (valid && L <= 0) bad_l = true;
      if (valid && L > a.max_run) bad_c = true;
      L = (L > 0 && L <= a.max_run) ? L : 0;
      const double od = (o >= 0.0f && o <= 1.0f) ? (double)o : 0.0;
      const double fo = f_cell<double>(a.delta_occ, a.ln_occ, od);
      const double fe = f_cell<double>(delta_emp, a.ln_emp, od);
      const double eD = (double)L * fe;
      const double eP = valid ? pow(1.0 - od, (double)L) : 1.0;
      // the scans and shifts read other lanes: every lane takes part
      const int incS = wave_scan_incl<OpAdd>(L);
      const double incD = wave_scan_incl<OpAdd>(eD);
      const double incP = wave_scan_incl<OpMul>(eP);
      const double exD = wave_shift_up<OpAdd>(incD);
      const double exP = wave_shift_up<OpMul>(incP);
      if (valid) {
        s_o[u] = (float)od;
        s_L[u] = L;
        s_s[u] = carry_s + incS - L;
        s_D[u] = carry_D + exD;
        s_P[u] = carry_P * exP;
        s_fo[u] = fo;
        s_fe[u] = fe;
      }
      carry_s += wave_last(incS);
      carry_D += wave_last(incD);
      carry_P *= wave_last(incP);
    }
    const bool any_o = __any(bad_o), any_l = __any(bad_l), any_c = __any(bad_c);
    if (any_o || any_l || any_c) {
      if (lane == 0) {
        latch(a.status, (any_o ? kErrOcc : 0u) | (any_l ? kErrLen : 0u) | (any_c ? kErrCap : 0u));
        a.mi[it] = __builtin_nan("");
      }
      wave_sync();
      continue;
    }
    wave_sync();
    // pass 2: a lane per run u
    const RunLds rl{s_o, s_L, s_s, s_P, s_D, s_fo, s_fe};
    double acc = 0.0;
    for (int u = lane; u < nr; u += kWave) acc += table_run_terms(a, rl, u, nr);
    const double I = wave_sum(acc);
    if (lane == 0) a.mi[it] = I / (2.50662827463100050242 * a.sigma_p);
    wave_sync();   // the LDS arrays are refilled for the next beam
  }
}

// Scans within the 16-lane rows of a wave (DPP row shifts; a row's first
// lane gets the identity).
template <typename Op, typename T>
FSMI_DEV T row_scan_incl(T v) {
  const T id = Op::template ident<T>();
  if constexpr (sizeof(T) == 8) {
    v = Op::apply(v, dpp_f64<dpp::row_shr1, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_shr2, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_shr4, 0xf>(v, id));
    v = Op::apply(v, dpp_f64<dpp::row_shr8, 0xf>(v, id));
  } else {
    v = Op::apply(v, dpp_i32<dpp::row_shr1, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_shr2, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_shr4, 0xf>(v, id));
    v = Op::apply(v, dpp_i32<dpp::row_shr8, 0xf>(v, id));
  }
  return v;
}
template <typename Op>
FSMI_DEV double row_shift_up(double inc) {
  return dpp_f64<dpp::row_shr1, 0xf>(inc, Op::template ident<double>());
}

// Beams of at most 16 runs: four beams per wave, 16 lanes (one DPP row) each,
// a lane per run.  Beam 4 g + q of the launch's group g sits in row q.
__global__ __launch_bounds__(kWave) void k_rle_table16(TabArgs a) {
  __shared__ float s_o[kWave];
  __shared__ int s_L[kWave], s_s[kWave];
  __shared__ double s_P[kWave], s_D[kWave], s_fo[kWave], s_fe[kWave];
  const int lane = threadIdx.x, row = lane >> 4, u = lane & 15;
  const double delta_emp = 1.0 / a.delta_occ;
  const RunLds rl{s_o + 16 * row, s_L + 16 * row, s_s + 16 * row, s_P + 16 * row,
                  s_D + 16 * row, s_fo + 16 * row, s_fe + 16 * row};
  const int64_t n_groups = (a.n_beams + 3) / 4;
  for (int64_t gi = blockIdx.x; gi < n_groups; gi += gridDim.x) {
    const int64_t it = 4 * gi + row;
    const bool has_beam = it < a.n_beams;
    const int64_t r0 = has_beam ? a.run_off[it] : 0, r1 = has_beam ? a.run_off[it + 1] : 0;
    const bool bad_off = has_beam && (r1 < r0 || r1 - r0 > 16);
    const int nr = (has_beam && !bad_off) ? (int)(r1 - r0) : 0;
    const bool valid = u < nr;
    const float o = valid ? a.run_occ[r0 + u] : 0.0f;
    int L = valid ? a.run_len[r0 + u] : 0;
    const bool bad_o = valid && !(o >= 0.0f && o <= 1.0f);
    const bool bad_l = valid && L <= 0;
    const bool bad_c = valid && L > a.max_run;
    L = (L > 0 && L <= a.max_run) ? L : 0;
    const double od = (o >= 0.0f && o <= 1.0f) ? (double)o : 0.0;
    const double fo = f_cell<double>(a.delta_occ, a.ln_occ, od);
    const double fe = f_cell<double>(delta_emp, a.ln_emp, od);
    const double eD = (double)L * fe;
    const double eP = valid ? pow(1.0 - od, (double)L) : 1.0;
    // row-local scans: every lane takes part
    const int incS = row_scan_incl<OpAdd>(L);
    const double incD = row_scan_incl<OpAdd>(eD);
    const double incP = row_scan_incl<OpMul>(eP);
    const double exD = row_shift_up<OpAdd>(incD);
    const double exP = row_shift_up<OpMul>(incP);
    if (valid) {
      s_o[lane] = (float)od;
      s_L[lane] = L;
      s_s[lane] = incS - L;
      s_D[lane] = exD;
      s_P[lane] = exP;
      s_fo[lane] = fo;
      s_fe[lane] = fe;
    }
    // this row's flags
    const uint64_t mo = __ballot(bad_o), ml = __ballot(bad_l || bad_off), mc = __ballot(bad_c);
    const uint64_t rm = 0xffffull << (16 * row);
    const bool rbad = ((mo | ml | mc) & rm) != 0;
    wave_sync();
    const double acc = (valid && !rbad) ? table_run_terms(a, rl, u, nr) : 0.0;
    // the row's sum, in lane 15 of the row after the scan
    const double tot = __shfl(row_scan_incl<OpAdd>(acc), 16 * row + 15);
    if (u == 0 && has_beam) {
      if (rbad) {
        latch(a.status, ((mo & rm) ? kErrOcc : 0u) |
                            ((ml & rm) ? (bad_off && r1 - r0 > 16 ? kErrCap : kErrLen) : 0u) |
                            ((mc & rm) ? kErrCap : 0u));
        a.mi[it] = __builtin_nan("");
      } else {
        a.mi[it] = tot / (2.50662827463100050242 * a.sigma_p);
      }
    }
    wave_sync();   // the LDS rows are refilled for the next group
  }
}

// out[0] = the longest run, out[1] = the most runs in one beam.
__global__ void k_max_runs(const int64_t* run_off, const int32_t* run_len, int64_t n_beams,
                           int32_t* out) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n_beams;
       b += (int64_t)gridDim.x * blockDim.x) {
    int32_t m = 0;
    for (int64_t u = run_off[b]; u < run_off[b + 1]; ++u) m = max(m, run_len[u]);
    atomicMax(out, m);
    atomicMax(out + 1, (int32_t)min<int64_t>(run_off[b + 1] - run_off[b], 0x7fffffff));
  }
}

__global__ void k_zero_two(int32_t* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_rle_table(fsmi_ctx ctx, double delta_occ, int Delta, int levels,
                            double sigma_p, int64_t n_beams, const int64_t* run_off,
                            const float* run_occ, const int32_t* run_len, double* mi) {
  if (n_beams <= 0) return hipSuccess;
  hipStream_t st = ctx->stream;
  // the longest run of the batch sizes the theta/gamma tables
  hipError_t e = ensure_work(ctx, 64);
  if (e != hipSuccess) return e;
  int32_t* d = reinterpret_cast<int32_t*>(ctx->d_work);
  hipLaunchKernelGGL(k_zero_two, dim3(1), dim3(64), 0, st, d);
  const int g0 = (int)std::max<int64_t>(1, std::min<int64_t>((n_beams + 255) / 256, 1024));
  hipLaunchKernelGGL(k_max_runs, dim3(g0), dim3(256), 0, st, run_off, run_len, n_beams, d);
  int32_t host[2] = {0, 0};
  e = hipMemcpyAsync(host, d, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  const int max_run = std::max(1, std::min(host[0], kTabMaxRun));   // longer runs latch in the kernel
  const bool small = host[1] <= 256, tiny = host[1] <= 16;
  const int W = 2 * Delta + 1;
  const size_t ab_n = (size_t)(levels + 1) * 2 * W * W;
  const size_t tg_n = (size_t)(levels + 1) * 2 * (max_run + 1);
  e = ensure_work(ctx, sizeof(double) * (ab_n + tg_n));
  if (e != hipSuccess) return e;
  double* ab = reinterpret_cast<double*>(ctx->d_work);
  double* tg = ab + ab_n;
  const double two_var = 2.0 * sigma_p * sigma_p;
  const int g1 = (int)std::min<size_t>((ab_n / 2 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_tab_alpha_beta, dim3(std::max(g1, 1)), dim3(256), 0, st, levels, Delta,
                     two_var, ab);
  const int g2 = (int)std::min<int64_t>(((int64_t)(levels + 1) * max_run + 255) / 256, 4096);
  hipLaunchKernelGGL(k_tab_tg_steps, dim3(std::max(g2, 1)), dim3(256), 0, st, levels, Delta, two_var,
                     max_run, tg);
  hipLaunchKernelGGL(k_tab_tg_prefix, dim3((levels + 1 + 63) / 64), dim3(64), 0, st, levels, max_run, tg);
  TabArgs a;
  a.n_beams = n_beams;
  a.run_off = run_off;
  a.run_occ = run_occ;
  a.run_len = run_len;
  a.mi = mi;
  a.ab = ab;
  a.tg = tg;
  a.sigma_p = sigma_p;
  a.two_var = two_var;
  a.delta_occ = delta_occ;
  a.ln_occ = log(delta_occ);
  a.ln_emp = log(1.0 / delta_occ);
  a.Delta = Delta;
  a.levels = levels;
  a.max_run = max_run;
  a.status = ctx->d_status;
  // one-wave workgroups: 3 per SIMD fit the registers; the 1024-run kernel's
  // 45 KB of LDS allows 3 per CU
  const int per_cu = small ? 12 : 3;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_beams, (int64_t)ctx->num_cu * per_cu));
  if (tiny) {
    const int g16 = (int)std::max<int64_t>(1, std::min<int64_t>((n_beams + 3) / 4, (int64_t)ctx->num_cu * 12));
    hipLaunchKernelGGL(k_rle_table16, dim3(g16), dim3(kWave), 0, st, a);
  } else if (small)
    hipLaunchKernelGGL(k_rle_table<256>, dim3(grid), dim3(kWave), 0, st, a);
  else
    hipLaunchKernelGGL(k_rle_table<kTabRuns>, dim3(grid), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

}  // namespace fsmi
