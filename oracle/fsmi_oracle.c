/*
 * fsmi_oracle.c -- plain FP64 CPU oracle for FSMI (arXiv 1905.02238).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.  Build: gcc -O2 -fopenmp -ffp-contract=off.
 *
 * Notation follows the paper: cells 1..n along the beam, boundaries
 * l_1 = 0 < l_2 < ... < l_{n+1}, centres mu_j = (l_j + l_{j+1})/2, first-hit
 * probabilities P(e_j), info-gain terms C_k, Gaussian weights G_{k,j}.
 * Arrays are 0-based: o[j-1] = o_j, l[k-1] = l_k, C[k-1] = C_k.
 *
 * Parity status: every exported quantity here is pinned by a CPU test
 * (brute-force quadrature of the MI definition, closed forms, invariants,
 * identities between independent routes, hand-derived ray lists).
 */
#include "fsmi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Neumaier-compensated accumulator                                    */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* f(delta, r): Sec. 2.2, the per-cell information function             */
/* ------------------------------------------------------------------ */
/* Paper form: f = log((r+1)/(r+1/delta)) - log(delta)/(r*delta+1). */
double ora_f_odds(double delta, double r) {
  return log((r + 1.0) / (r + 1.0 / delta)) - log(delta) / (r * delta + 1.0);
}
/* Same function written in o = r/(1+r), which stays defined at o = 0 and 1:
   with s = 1 + o(delta-1),  f = (o*delta/s)*log(delta) - log1p(o(delta-1)). */
double ora_f(double delta, double o) {
  double s = 1.0 + o * (delta - 1.0);
  return (o * delta / s) * log(delta) - log1p(o * (delta - 1.0));
}

/* Alg 2: E_0 = 1, E_j = E_{j-1}(1-o_j), P(e_j) = E_{j-1} o_j, P(e_0) = E_n. */
void ora_first_hit(int n, const double* o, double* P) {
  double E = 1.0;
  for (int j = 1; j <= n; ++j) {
    P[j] = E * o[j - 1];
    E = E * (1.0 - o[j - 1]);
  }
  P[0] = E;
}

/* Alg 3: q_0 = 0, C_k = q_{k-1} + f(delta_occ, r_k), q_k = q_{k-1} + f(delta_emp, r_k). */
void ora_info_gain(int n, const double* o, double delta_occ, double* C) {
  double delta_emp = 1.0 / delta_occ;
  nsum q = {0.0, 0.0};
  for (int k = 1; k <= n; ++k) {
    C[k - 1] = nval(&q) + ora_f(delta_occ, o[k - 1]);
    nadd(&q, ora_f(delta_emp, o[k - 1]));
  }
}

/* Lemma (G_{k,j}): G = Phi(b) - Phi(a) with a = (l_k-mu)/sigma, b = (l_{k+1}-mu)/sigma.
   Written with erfc on the tail side of mu so no digits cancel away. */
double ora_G(double lk, double lk1, double mu, double sigma) {
  const double r2 = 0.70710678118654752440; /* 1/sqrt(2) */
  double a = (lk - mu) / sigma, b = (lk1 - mu) / sigma;
  if (a >= 0.0) return 0.5 * (erfc(a * r2) - erfc(b * r2));
  if (b <= 0.0) return 0.5 * (erfc(-b * r2) - erfc(-a * r2));
  return 1.0 - 0.5 * erfc(b * r2) - 0.5 * erfc(-a * r2);
}

/* Thm 1 (Eq. fast_exact_mi): I = sum_{j} sum_{k=1}^{n} P(e_j) C_k G_{k,j}.
   The j = 0 event (no cell hit) has its reading beyond l_{n+1}, outside the
   integration range [0, l_{n+1}), so G_{k,0} = 0 and the term vanishes. */
double ora_fsmi_exact(int n, const double* o, const double* l, double sigma, double delta_occ) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* C = (double*)malloc(sizeof(double) * n);
  ora_first_hit(n, o, P);
  ora_info_gain(n, o, delta_occ, C);
  nsum I = {0.0, 0.0};
  for (int j = 1; j <= n; ++j) {
    double mu = 0.5 * (l[j - 1] + l[j]);
    for (int k = 1; k <= n; ++k) {
      double G = ora_G(l[k - 1], l[k], mu, sigma);
      nadd(&I, P[j] * C[k - 1] * G);
    }
  }
  free(P);
  free(C);
  return nval(&I);
}

/* Two extensions of Thm 1 (readings the paper leaves open):
   - range-dependent noise: the reading of event e_j is N(mu_j, sigma_j^2) with
     sigma_j = sigma + slope * mu_j (the per-event sigma_j of Alg 1), so
     G_{k,j} uses sigma_j;
   - max-range returns (tail = 1): a reading at or beyond l_{n+1} is reported
     as "max range" and updates every cell of the beam as empty, an information
     gain of q_n = sum_{i=1}^{n} f(delta_emp, r_i).  Its probability is
     sum_j P(e_j) (1 - Phi((l_{n+1} - mu_j)/sigma_j)) + P(e_0) (e_0 reads max
     range with certainty), so the term added to Thm 1 is
     q_n [sum_j P(e_j) (1 - Phi((l_{n+1} - mu_j)/sigma_j)) + P(e_0)].
   With slope = 0 and tail = 0 this is ora_fsmi_exact. */
double ora_fsmi_exact_ext(int n, const double* o, const double* l, double sigma, double slope,
                          int tail, double delta_occ) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* C = (double*)malloc(sizeof(double) * n);
  ora_first_hit(n, o, P);
  ora_info_gain(n, o, delta_occ, C);
  nsum I = {0.0, 0.0};
  for (int j = 1; j <= n; ++j) {
    double mu = 0.5 * (l[j - 1] + l[j]);
    double sj = sigma + slope * mu;
    for (int k = 1; k <= n; ++k) {
      double G = ora_G(l[k - 1], l[k], mu, sj);
      nadd(&I, P[j] * C[k - 1] * G);
    }
  }
  if (tail) {
    const double r2 = 0.70710678118654752440; /* 1/sqrt(2) */
    double delta_emp = 1.0 / delta_occ;
    nsum q = {0.0, 0.0}, pmax = {0.0, 0.0};
    for (int i = 0; i < n; ++i) nadd(&q, ora_f(delta_emp, o[i]));
    for (int j = 1; j <= n; ++j) {
      double mu = 0.5 * (l[j - 1] + l[j]);
      double sj = sigma + slope * mu;
      nadd(&pmax, P[j] * 0.5 * erfc((l[n] - mu) / sj * r2));
    }
    nadd(&pmax, P[0]);
    nadd(&I, nval(&q) * nval(&pmax));
  }
  free(P);
  free(C);
  return nval(&I);
}

/* Eq. fsmi_approx: the k range is cut to [j-Delta, j+Delta] (clipped to 1..n),
   with no renormalisation of the remaining weights. */
double ora_fsmi_approx(int n, const double* o, const double* l, double sigma, double delta_occ,
                       int Delta) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* C = (double*)malloc(sizeof(double) * n);
  ora_first_hit(n, o, P);
  ora_info_gain(n, o, delta_occ, C);
  nsum I = {0.0, 0.0};
  for (int j = 1; j <= n; ++j) {
    double mu = 0.5 * (l[j - 1] + l[j]);
    int k0 = j - Delta < 1 ? 1 : j - Delta;
    int k1 = j + Delta > n ? n : j + Delta;
    for (int k = k0; k <= k1; ++k) {
      double G = ora_G(l[k - 1], l[k], mu, sigma);
      nadd(&I, P[j] * C[k - 1] * G);
    }
  }
  free(P);
  free(C);
  return nval(&I);
}

/* Thm 4 / Alg 4 (Uniform-FSMI): D_k = D_{k-1} + C_k, and
   I = sum_j P(e_j) (D_{min(n,j+H)} - D_{max(0,j-H-1)}) / (2H+1). */
double ora_fsmi_uniform(int n, const double* o, double delta_occ, int H) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* C = (double*)malloc(sizeof(double) * n);
  double* D = (double*)malloc(sizeof(double) * (n + 1));
  ora_first_hit(n, o, P);
  ora_info_gain(n, o, delta_occ, C);
  nsum acc = {0.0, 0.0};
  D[0] = 0.0;
  for (int k = 1; k <= n; ++k) {
    nadd(&acc, C[k - 1]);
    D[k] = nval(&acc);
  }
  nsum I = {0.0, 0.0};
  for (int j = 1; j <= n; ++j) {
    int hi = j + H > n ? n : j + H;
    int lo = j - H - 1 < 0 ? 0 : j - H - 1;
    nadd(&I, P[j] * (D[hi] - D[lo]) / (2.0 * H + 1.0));
  }
  free(P);
  free(C);
  free(D);
  return nval(&I);
}

/* ------------------------------------------------------------------ */
/* Equal-width cells: G_{k,j} depends on d = k - j only                 */
/* ------------------------------------------------------------------ */
/* ERF:     Phi((d+1/2)/sigma') - Phi((d-1/2)/sigma')   (Eq. G_jk on unit cells)
   DENSITY: exp(-d^2/(2 sigma'^2)) / (sqrt(2 pi) sigma')  (the density form in the
            proof of Thm 5)
   UNIFORM: [|d| <= H] / (2H+1)                          (Thm 4 noise model) */
double ora_kernel_weight(int kind, double sigma_p, int H, int d) {
  if (kind == ORA_K_ERF) return ora_G((double)d - 0.5, (double)d + 0.5, 0.0, sigma_p);
  if (kind == ORA_K_DENSITY) {
    const double s2pi = 2.50662827463100050242; /* sqrt(2 pi) */
    return exp(-((double)d * (double)d) / (2.0 * sigma_p * sigma_p)) / (s2pi * sigma_p);
  }
  return (d <= H && d >= -H) ? 1.0 / (2.0 * H + 1.0) : 0.0;
}

static double kernel_trunc(int kind, double sigma_p, int H, int trunc, int d) {
  if (trunc >= 0 && (d > trunc || d < -trunc)) return 0.0;
  return ora_kernel_weight(kind, sigma_p, H, d);
}

double ora_fsmi_eqwidth(int n, const double* o, double sigma_p, double delta_occ, int kind,
                        int trunc, int H) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* C = (double*)malloc(sizeof(double) * n);
  /* the weight of each distance d = k - j, evaluated once (w[d + n - 1]) */
  double* w = (double*)malloc(sizeof(double) * (2 * n - 1));
  ora_first_hit(n, o, P);
  ora_info_gain(n, o, delta_occ, C);
  for (int d = -(n - 1); d <= n - 1; ++d) w[d + n - 1] = kernel_trunc(kind, sigma_p, H, trunc, d);
  nsum I = {0.0, 0.0};
  for (int j = 1; j <= n; ++j)
    for (int k = 1; k <= n; ++k) {
      double wk = w[k - j + n - 1];
      if (wk != 0.0) nadd(&I, P[j] * C[k - 1] * wk);
    }
  free(P);
  free(C);
  free(w);
  return nval(&I);
}

/* ------------------------------------------------------------------ */
/* CSQMI (Sec. 2.3): the comparison metric, exact and Delta-truncated   */
/* ------------------------------------------------------------------ */
/* Density of N(0, 2 sigma^2) at x: the integral over z of the product of
   two N(z; mu, sigma^2) whose means differ by x. */
static double n2(double x, double sigma) {
  const double sqrt_pi = 1.77245385090551602730;
  return exp(-(x * x) / (4.0 * sigma * sigma)) / (2.0 * sigma * sqrt_pi);
}

/* Eq. csqmi_exact as printed: I = log B + log C - 2 log A with
     B = sum_{l=0}^{n} w_l N(0, 2 sigma^2),
     C = prod_i (o_i^2 + (1-o_i)^2) sum_j sum_l P(e_j) P(e_l) N(mu_l - mu_j, 2 sigma^2),
     A = sum_j sum_l P(e_j) w_l N(mu_l - mu_j, 2 sigma^2),
   j, l = 0..n.  Readings:
   - w_l = P(e_l)^2 prod_{i>l} (o_i^2 + (1-o_i)^2), w_0 = P(e_0)^2: the sum of
     P(m)^2 over the maps m whose first occupied cell is l (the cells after l
     are free), which the definition D_CS(P(Z, M), P(Z) P(M)) gives; the
     printed product runs over j < l;
   - e_0 (no cell occupied) reads beyond the beam, as in Thm 1: its cross
     terms with every cell vanish and its self terms carry N(0, 2 sigma^2);
   - the printed form is log B + log C - 2 log A, twice the -1/2 log of the
     divergence's definition; it is kept as printed.
   Delta >= 0 keeps only l in [j - Delta, j + Delta] in both double sums (the
   truncation of Sec. 2.3 that gives Approx-CSQMI); Delta < 0 is the exact sum.
   Valid while no sum underflows (returns NaN if one does). */
double ora_csqmi(int n, const double* o, const double* l, double sigma, int Delta) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* S = (double*)malloc(sizeof(double) * (n + 1));
  double* w = (double*)malloc(sizeof(double) * (n + 1));
  ora_first_hit(n, o, P);
  /* S[l] = prod_{i>l} q_i, q_i = o_i^2 + (1-o_i)^2; log prod_i q_i summed */
  S[n] = 1.0;
  for (int i = n; i >= 1; --i) {
    double q = o[i - 1] * o[i - 1] + (1.0 - o[i - 1]) * (1.0 - o[i - 1]);
    S[i - 1] = S[i] * q;
  }
  nsum logQ = {0.0, 0.0};
  for (int i = 1; i <= n; ++i) {
    double q = o[i - 1] * o[i - 1] + (1.0 - o[i - 1]) * (1.0 - o[i - 1]);
    nadd(&logQ, log(q));
  }
  w[0] = P[0] * P[0];
  for (int k = 1; k <= n; ++k) w[k] = P[k] * P[k] * S[k];
  const double g0 = n2(0.0, sigma);
  nsum B = {0.0, 0.0}, Cs = {0.0, 0.0}, A = {0.0, 0.0};
  for (int k = 0; k <= n; ++k) nadd(&B, w[k] * g0);
  nadd(&Cs, P[0] * P[0] * g0);
  nadd(&A, P[0] * w[0] * g0);
  for (int j = 1; j <= n; ++j) {
    double muj = 0.5 * (l[j - 1] + l[j]);
    int k0 = 1, k1 = n;
    if (Delta >= 0) {
      k0 = j - Delta < 1 ? 1 : j - Delta;
      k1 = j + Delta > n ? n : j + Delta;
    }
    for (int k = k0; k <= k1; ++k) {
      double muk = 0.5 * (l[k - 1] + l[k]);
      double g = n2(muk - muj, sigma);
      nadd(&Cs, P[j] * P[k] * g);
      nadd(&A, P[j] * w[k] * g);
    }
  }
  double b = nval(&B), c = nval(&Cs), a = nval(&A);
  free(P);
  free(S);
  free(w);
  if (!(a > 0.0) || !(b > 0.0) || !(c > 0.0)) return NAN;
  return log(b) + (nval(&logQ) + log(c)) - 2.0 * log(a);
}

/* ------------------------------------------------------------------ */
/* Trajectory MI with cell marking (Sec. 2.4)                           */
/* ------------------------------------------------------------------ */
/* A beam whose cells i with counted[i-1] == 0 have been counted before: their
   information is not added again, I = sum over counted cells i of I(M_i; Z).
   By Lemma 1 (F(z) = sum_i f(delta_i(z), r_i)) this removes the f terms of the
   uncounted cells from C_k; every cell still shapes P(e_j).  The variants
   follow Thm 1, Eq. fsmi_approx and Alg 4 with that C. */
static void info_gain_counted(int n, const double* o, double delta_occ,
                              const unsigned char* counted, double* C) {
  double delta_emp = 1.0 / delta_occ;
  nsum q = {0.0, 0.0};
  for (int k = 1; k <= n; ++k) {
    double focc = counted[k - 1] ? ora_f(delta_occ, o[k - 1]) : 0.0;
    C[k - 1] = nval(&q) + focc;
    if (counted[k - 1]) nadd(&q, ora_f(delta_emp, o[k - 1]));
  }
}

double ora_fsmi_counted(int variant, int n, const double* o, const double* l, double sigma,
                        double delta_occ, int Delta, int H, const unsigned char* counted) {
  if (n <= 0) return 0.0;
  double* P = (double*)malloc(sizeof(double) * (n + 1));
  double* C = (double*)malloc(sizeof(double) * n);
  ora_first_hit(n, o, P);
  info_gain_counted(n, o, delta_occ, counted, C);
  nsum I = {0.0, 0.0};
  if (variant == ORA_UNIFORM) {
    double* D = (double*)malloc(sizeof(double) * (n + 1));
    nsum acc = {0.0, 0.0};
    D[0] = 0.0;
    for (int k = 1; k <= n; ++k) {
      nadd(&acc, C[k - 1]);
      D[k] = nval(&acc);
    }
    for (int j = 1; j <= n; ++j) {
      int hi = j + H > n ? n : j + H;
      int lo = j - H - 1 < 0 ? 0 : j - H - 1;
      nadd(&I, P[j] * (D[hi] - D[lo]) / (2.0 * H + 1.0));
    }
    free(D);
  } else {
    for (int j = 1; j <= n; ++j) {
      double mu = 0.5 * (l[j - 1] + l[j]);
      int k0 = 1, k1 = n;
      if (variant == ORA_APPROX) {
        k0 = j - Delta < 1 ? 1 : j - Delta;
        k1 = j + Delta > n ? n : j + Delta;
      }
      for (int k = k0; k <= k1; ++k) nadd(&I, P[j] * C[k - 1] * ora_G(l[k - 1], l[k], mu, sigma));
    }
  }
  free(P);
  free(C);
  return nval(&I);
}

/* Candidate trajectories in CSR form: trajectory k has the states (2D poses
   [x, y, cos, sin]) traj_off[k] .. traj_off[k+1]-1, in travel order.  Each
   state's scan MI is the sum over its beams (Sec. 2.4); a cell's information
   counts only at the first state of the trajectory whose beams cross it, and
   there at every beam of that state that crosses it (within one scan beams
   are summed as they are, as in a single pose).  mi_state[t] = the state's
   MI, mi_traj[k] = the sum over its states; mi_beam [n_states][n_beams] may
   be NULL.  Returns -1 if a state lies outside the map. */
int ora_eval_trajectories_2d(int variant, int Delta, int H, double delta_occ, const float* map,
                             int64_t X, int64_t Y, int64_t n_traj, const int64_t* traj_off,
                             const double* poses, int64_t n_beams, const double* beam_dir,
                             double sigma, double R, double* mi_traj, double* mi_state,
                             double* mi_beam) {
  int max_cells = (int)floor(1.4142135623730951 * R) + 3;
  int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)(X * Y));
  int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * max_cells);
  double* entry = (double*)malloc(sizeof(double) * (max_cells + 1));
  float* of = (float*)malloc(sizeof(float) * max_cells);
  double* beam_val = (double*)malloc(sizeof(double) * (n_beams > 0 ? n_beams : 1));
  int bad = 0;
  for (int64_t k = 0; k < n_traj; ++k) {
    for (int64_t c = 0; c < X * Y; ++c) first[c] = -1;
    /* the first state of this trajectory whose beams cross each cell */
    for (int64_t t = traj_off[k]; t < traj_off[k + 1]; ++t) {
      const double* ps = poses + 4 * t;
      for (int64_t b = 0; b < n_beams; ++b) {
        double bx = beam_dir[2 * b], by = beam_dir[2 * b + 1];
        double m1 = ps[2] * bx, m2 = ps[3] * by, m3 = ps[3] * bx, m4 = ps[2] * by;
        int n = ora_raycast2d(map, X, Y, ps[0], ps[1], m1 - m2, m3 + m4, R, max_cells, cell,
                              entry, of);
        for (int i = 0; i < n; ++i)
          if (first[cell[i]] < 0) first[cell[i]] = (int32_t)(t - traj_off[k]);
      }
    }
    nsum tk = {0.0, 0.0};
    for (int64_t t = traj_off[k]; t < traj_off[k + 1]; ++t) {
      const double* ps = poses + 4 * t;
      /* the state's beams (independent of each other), then their sum in order */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
      for (int64_t b = 0; b < n_beams; ++b) {
        int32_t* bc = (int32_t*)malloc(sizeof(int32_t) * max_cells);
        double* be = (double*)malloc(sizeof(double) * (max_cells + 1));
        float* bof = (float*)malloc(sizeof(float) * max_cells);
        double* bo = (double*)malloc(sizeof(double) * max_cells);
        unsigned char* bm = (unsigned char*)malloc((size_t)max_cells);
        double bx = beam_dir[2 * b], by = beam_dir[2 * b + 1];
        double m1 = ps[2] * bx, m2 = ps[3] * by, m3 = ps[3] * bx, m4 = ps[2] * by;
        int n = ora_raycast2d(map, X, Y, ps[0], ps[1], m1 - m2, m3 + m4, R, max_cells, bc, be, bof);
        double v;
        if (n < 0) {
          v = NAN;
          bad = 1;
        } else {
          for (int i = 0; i < n; ++i) {
            bo[i] = (double)bof[i];
            bm[i] = first[bc[i]] == (int32_t)(t - traj_off[k]);
          }
          v = ora_fsmi_counted(variant, n, bo, be, sigma, delta_occ, Delta, H, bm);
        }
        beam_val[b] = v;
        free(bc);
        free(be);
        free(bof);
        free(bo);
        free(bm);
      }
      nsum ts = {0.0, 0.0};
      for (int64_t b = 0; b < n_beams; ++b) {
        if (mi_beam) mi_beam[t * n_beams + b] = beam_val[b];
        nadd(&ts, beam_val[b]);
      }
      if (mi_state) mi_state[t] = nval(&ts);
      nadd(&tk, nval(&ts));
    }
    mi_traj[k] = nval(&tk);
  }
  free(first);
  free(cell);
  free(entry);
  free(of);
  free(beam_val);
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Run-length encoded beams (Sec. 4)                                    */
/* ------------------------------------------------------------------ */
/* Primary route: expand the runs (Eq. occup_rle) and evaluate the plain sum. */
double ora_rle_expanded(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                        int kind, int trunc, int H) {
  int n = 0;
  for (int u = 0; u < nr; ++u) n += L[u];
  if (n <= 0) return 0.0;
  double* o = (double*)malloc(sizeof(double) * n);
  int p = 0;
  for (int u = 0; u < nr; ++u)
    for (int i = 0; i < L[u]; ++i) o[p++] = ro[u];
  double I = ora_fsmi_eqwidth(n, o, sigma_p, delta_occ, kind, trunc, H);
  free(o);
  return I;
}

/* Alg 5: P_E(1) = 1, P_E(u) = P_E(u-1) (1-o_{u-1})^{L_{u-1}}.
   Alg 6: D_E(1) = 0, D_E(v) = D_E(v-1) + L_{v-1} f(delta_emp, r_{v-1}).
   s_u = sum_{i<u} L_i. */
static void rle_prefix(int nr, const double* ro, const int* L, double delta_occ, double* PE,
                       double* DE, int* s) {
  double delta_emp = 1.0 / delta_occ;
  PE[0] = 1.0;
  DE[0] = 0.0;
  s[0] = 0;
  for (int u = 1; u < nr; ++u) {
    PE[u] = PE[u - 1] * pow(1.0 - ro[u - 1], (double)L[u - 1]);
    DE[u] = DE[u - 1] + (double)L[u - 1] * ora_f(delta_emp, ro[u - 1]);
    s[u] = s[u - 1] + L[u - 1];
  }
}

/* Block sums of the proof of Thm 5 with a general kernel w:
   A[x,Lu,Lv,t] = sum_{j<Lu} sum_{k<Lv} x^j w(j+t-k),  B = same with a factor k. */
static void block_AB(double x, int Lu, int Lv, int t, int kind, double sigma_p, int H, int trunc,
                     double* A, double* B) {
  nsum a = {0.0, 0.0}, b = {0.0, 0.0};
  for (int j = 0; j < Lu; ++j) {
    double xj = pow(x, (double)j);
    for (int k = 0; k < Lv; ++k) {
      double w = kernel_trunc(kind, sigma_p, H, trunc, j + t - k);
      nadd(&a, xj * w);
      nadd(&b, (double)k * xj * w);
    }
  }
  *A = nval(&a);
  *B = nval(&b);
}

/* Secondary route, Thm 5 (Eq. group_fsmi_rle_exact):
   I = sum_u sum_v P_E(u) o_u [ (D_E(v) + f(d_occ, r_v)) A + f(d_emp, r_v) B ]
   with x = 1 - o_u and t = s_u - s_v.  The kernel carries its own normalisation,
   so the paper's outer 1/(sqrt(2 pi) sigma') is inside w for the DENSITY kind. */
double ora_rle_thm5(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                    int kind, int trunc, int H) {
  if (nr <= 0) return 0.0;
  double delta_emp = 1.0 / delta_occ;
  double* PE = (double*)malloc(sizeof(double) * nr);
  double* DE = (double*)malloc(sizeof(double) * nr);
  int* s = (int*)malloc(sizeof(int) * nr);
  rle_prefix(nr, ro, L, delta_occ, PE, DE, s);
  nsum I = {0.0, 0.0};
  for (int u = 0; u < nr; ++u)
    for (int v = 0; v < nr; ++v) {
      double A, B;
      block_AB(1.0 - ro[u], L[u], L[v], s[u] - s[v], kind, sigma_p, H, trunc, &A, &B);
      double cv = DE[v] + ora_f(delta_occ, ro[v]);
      nadd(&I, PE[u] * ro[u] * (cv * A + ora_f(delta_emp, ro[v]) * B));
    }
  free(PE);
  free(DE);
  free(s);
  return nval(&I);
}

/* Thm 6 (Approx-FSMI-RLE), kernel truncated at |d| <= Delta inside every block:
   only pairs with u = v, or u < v and s_v < s_u + L_u + Delta, or v < u and
   s_u < s_v + L_v + Delta contribute (Lemma on non-zero block pairs), and each
   such block is cropped to the start/length s', L' of Eqs. su'..Lv'.  The
   cropped block's shift is t = s'_u - s'_v (the shift of the cropped start
   cells).  The u < v weight is (D_E(v) + f(d_occ, r_v)) A + f(d_emp, r_v) B. */
double ora_rle_thm6(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                    int kind, int Delta, int H) {
  if (nr <= 0) return 0.0;
  double delta_emp = 1.0 / delta_occ;
  double* PE = (double*)malloc(sizeof(double) * nr);
  double* DE = (double*)malloc(sizeof(double) * nr);
  int* s = (int*)malloc(sizeof(int) * nr);
  rle_prefix(nr, ro, L, delta_occ, PE, DE, s);
  nsum I = {0.0, 0.0};
  for (int u = 0; u < nr; ++u) {
    double x = 1.0 - ro[u];
    double A, B;
    /* u = v: theta = A[x,L,L,0], gamma = B[x,L,L,0] */
    block_AB(x, L[u], L[u], 0, kind, sigma_p, H, Delta, &A, &B);
    nadd(&I, PE[u] * ro[u] * ((DE[u] + ora_f(delta_occ, ro[u])) * A + ora_f(delta_emp, ro[u]) * B));
    for (int v = u + 1; v < nr; ++v) {
      if (!(s[v] < s[u] + L[u] + Delta)) continue;
      int su_p = s[u] > s[v] - Delta ? s[u] : s[v] - Delta;
      int Lu_p = s[u] + L[u] - su_p;
      int sv_p = s[v];
      int Lv_p = L[v] < s[u] + L[u] + Delta - s[v] ? L[v] : s[u] + L[u] + Delta - s[v];
      block_AB(x, Lu_p, Lv_p, su_p - sv_p, kind, sigma_p, H, Delta, &A, &B);
      double Pp = PE[u] * pow(x, (double)(su_p - s[u]));
      nadd(&I, Pp * ro[u] * ((DE[v] + ora_f(delta_occ, ro[v])) * A + ora_f(delta_emp, ro[v]) * B));
    }
    for (int v = 0; v < u; ++v) {
      if (!(s[u] < s[v] + L[v] + Delta)) continue;
      int su_p = s[u];
      int Lu_p = L[u] < s[v] + L[v] + Delta - s[u] ? L[u] : s[v] + L[v] + Delta - s[u];
      int sv_p = s[v] > s[u] - Delta ? s[v] : s[u] - Delta;
      int Lv_p = s[v] + L[v] - sv_p;
      block_AB(x, Lu_p, Lv_p, su_p - sv_p, kind, sigma_p, H, Delta, &A, &B);
      double Dp = DE[v] + (double)(sv_p - s[v]) * ora_f(delta_emp, ro[v]);
      nadd(&I, PE[u] * ro[u] * ((Dp + ora_f(delta_occ, ro[v])) * A + ora_f(delta_emp, ro[v]) * B));
    }
  }
  free(PE);
  free(DE);
  free(s);
  return nval(&I);
}

/* alpha[x,a,b] = sum_{j<a} sum_{k<b} x^j exp(-(j-k)^2/(2 sigma'^2)), beta adds a factor k
   (Eqs. alpha, beta; un-normalised Gaussian as in the paper). */
static double alpha_def(double x, int a, int b, double sp) {
  nsum s = {0.0, 0.0};
  for (int j = 0; j < a; ++j)
    for (int k = 0; k < b; ++k)
      nadd(&s, pow(x, (double)j) * exp(-((double)(j - k) * (j - k)) / (2.0 * sp * sp)));
  return nval(&s);
}
static double beta_def(double x, int a, int b, double sp) {
  nsum s = {0.0, 0.0};
  for (int j = 0; j < a; ++j)
    for (int k = 0; k < b; ++k)
      nadd(&s, (double)k * pow(x, (double)j) * exp(-((double)(j - k) * (j - k)) / (2.0 * sp * sp)));
  return nval(&s);
}

/* Tertiary route: A and B from alpha/beta via Eqs. compute_A / compute_B, chosen by
   the sign of t, then Thm 5 with the density kernel and the outer 1/(sqrt(2 pi) sigma').
   x^{-t} grows without bound for long beams, so this route is for tiny inputs only. */
double ora_rle_alpha_route(int nr, const double* ro, const int* L, double sigma_p,
                           double delta_occ) {
  if (nr <= 0) return 0.0;
  double delta_emp = 1.0 / delta_occ;
  double* PE = (double*)malloc(sizeof(double) * nr);
  double* DE = (double*)malloc(sizeof(double) * nr);
  int* s = (int*)malloc(sizeof(int) * nr);
  rle_prefix(nr, ro, L, delta_occ, PE, DE, s);
  nsum I = {0.0, 0.0};
  for (int u = 0; u < nr; ++u) {
    double x = 1.0 - ro[u];
    for (int v = 0; v < nr; ++v) {
      int t = s[u] - s[v];
      double A, B;
      if (t >= 1) {
        double xt = pow(x, (double)(-t));
        A = xt * (alpha_def(x, L[u] + t, L[v], sigma_p) - alpha_def(x, t, L[v], sigma_p));
        B = xt * (beta_def(x, L[u] + t, L[v], sigma_p) - beta_def(x, t, L[v], sigma_p));
      } else if (t == 0) {
        A = alpha_def(x, L[u], L[v], sigma_p);
        B = beta_def(x, L[u], L[v], sigma_p);
      } else {
        A = alpha_def(x, L[u], L[v] - t, sigma_p) - alpha_def(x, L[u], -t, sigma_p);
        B = beta_def(x, L[u], L[v] - t, sigma_p) - beta_def(x, L[u], -t, sigma_p) + (double)t * A;
      }
      nadd(&I, PE[u] * ro[u] * ((DE[v] + ora_f(delta_occ, ro[v])) * A + ora_f(delta_emp, ro[v]) * B));
    }
  }
  free(PE);
  free(DE);
  free(s);
  const double s2pi = 2.50662827463100050242;
  return nval(&I) / (s2pi * sigma_p);
}

/* ---- table mode of Approx-FSMI-RLE (Alg 8 with the tables of Alg 9 and 10) ----
   The tables hold the un-normalised Gaussian truncated at |a - b| <= Delta, Thm 6's
   kernel: alpha_D[x,P,Q] = sum_{a<P} sum_{b<Q, |a-b|<=Delta} x^a g(a-b), beta_D adds a
   factor b, g(d) = exp(-d^2 / (2 sigma'^2)).  A block cropped by Eqs. su'..Lv' and
   shifted by t reads entries up to 2 Delta. */
static double gauss_t(double sp, int Delta, int d) {
  if (d > Delta || d < -Delta) return 0.0;
  return exp(-((double)d * (double)d) / (2.0 * sp * sp));
}
static double alpha_trunc(double x, int P, int Q, double sp, int Delta) {
  nsum s = {0.0, 0.0};
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < Q; ++b) nadd(&s, pow(x, (double)a) * gauss_t(sp, Delta, a - b));
  return nval(&s);
}
static double beta_trunc(double x, int P, int Q, double sp, int Delta) {
  nsum s = {0.0, 0.0};
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < Q; ++b) nadd(&s, (double)b * pow(x, (double)a) * gauss_t(sp, Delta, a - b));
  return nval(&s);
}

/* Table mode: I = (I_{u=v} + I_{u<v} + I_{u>v}) / (sqrt(2 pi) sigma'), with every
   table read at x_u quantised to the grid i / levels, i = floor(levels (1 - o_u) + 1/2);
   P_E, D_E and the crop factor (1 - o_u)^(s'_u - s_u) use o itself.  Per pair, with
   t = s'_u - s'_v of the cropped block:
     t <= 0 (v after u):  A = alpha_D[L'_u, L'_v - t] - alpha_D[L'_u, -t],
                          B = beta_D[L'_u, L'_v - t] - beta_D[L'_u, -t] + t A;
     t >= 1 (v before u): A = x^{-t} (alpha_D[t + L'_u, L'_v] - alpha_D[t, L'_v]),
                          B = x^{-t} (beta_D[t + L'_u, L'_v] - beta_D[t, L'_v]),
   the second the algorithm's route whose cancellation Sec. 4.1 warns about.  At x = 0
   (o within 1/(2 levels) of 1) x^{-t} has no value; the block is then its a = 0 row,
   A = sum_{b<L'_v} g(t - b), B = sum_b b g(t - b).  theta[x, L] = alpha_D[L, L],
   gamma[x, L] = beta_D[L, L].  On a grid o (x = x_q) the value is Thm 6's with the
   density kernel. */
double ora_rle_table(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                     int Delta, int levels) {
  if (nr <= 0) return 0.0;
  double delta_emp = 1.0 / delta_occ;
  double* PE = (double*)malloc(sizeof(double) * nr);
  double* DE = (double*)malloc(sizeof(double) * nr);
  int* s = (int*)malloc(sizeof(int) * nr);
  rle_prefix(nr, ro, L, delta_occ, PE, DE, s);
  nsum I = {0.0, 0.0};
  for (int u = 0; u < nr; ++u) {
    const double x = 1.0 - ro[u];
    const int iq = (int)floor(x * (double)levels + 0.5);
    const double xq = (double)iq / (double)levels;
    /* u = v */
    double th = alpha_trunc(xq, L[u], L[u], sigma_p, Delta);
    double ga = beta_trunc(xq, L[u], L[u], sigma_p, Delta);
    nadd(&I, PE[u] * ro[u] * ((DE[u] + ora_f(delta_occ, ro[u])) * th + ora_f(delta_emp, ro[u]) * ga));
    /* v after u */
    for (int v = u + 1; v < nr; ++v) {
      if (!(s[v] < s[u] + L[u] + Delta)) continue;
      int su_p = s[u] > s[v] - Delta ? s[u] : s[v] - Delta;
      int Lu_p = s[u] + L[u] - su_p;
      int Lv_p = L[v] < s[u] + L[u] + Delta - s[v] ? L[v] : s[u] + L[u] + Delta - s[v];
      int t = su_p - s[v];
      double A = alpha_trunc(xq, Lu_p, Lv_p - t, sigma_p, Delta) - alpha_trunc(xq, Lu_p, -t, sigma_p, Delta);
      double B = beta_trunc(xq, Lu_p, Lv_p - t, sigma_p, Delta) - beta_trunc(xq, Lu_p, -t, sigma_p, Delta) +
                 (double)t * A;
      double Pp = PE[u] * pow(x, (double)(su_p - s[u]));
      nadd(&I, Pp * ro[u] * ((DE[v] + ora_f(delta_occ, ro[v])) * A + ora_f(delta_emp, ro[v]) * B));
    }
    /* v before u */
    for (int v = 0; v < u; ++v) {
      if (!(s[u] < s[v] + L[v] + Delta)) continue;
      int Lu_p = L[u] < s[v] + L[v] + Delta - s[u] ? L[u] : s[v] + L[v] + Delta - s[u];
      int sv_p = s[v] > s[u] - Delta ? s[v] : s[u] - Delta;
      int Lv_p = s[v] + L[v] - sv_p;
      int t = s[u] - sv_p;
      double A, B;
      if (iq == 0) {
        nsum a = {0.0, 0.0}, b = {0.0, 0.0};
        for (int k = 0; k < Lv_p; ++k) {
          nadd(&a, gauss_t(sigma_p, Delta, t - k));
          nadd(&b, (double)k * gauss_t(sigma_p, Delta, t - k));
        }
        A = nval(&a);
        B = nval(&b);
      } else {
        double xt = pow(xq, (double)(-t));
        A = xt * (alpha_trunc(xq, t + Lu_p, Lv_p, sigma_p, Delta) - alpha_trunc(xq, t, Lv_p, sigma_p, Delta));
        B = xt * (beta_trunc(xq, t + Lu_p, Lv_p, sigma_p, Delta) - beta_trunc(xq, t, Lv_p, sigma_p, Delta));
      }
      double Dp = DE[v] + (double)(sv_p - s[v]) * ora_f(delta_emp, ro[v]);
      nadd(&I, PE[u] * ro[u] * ((Dp + ora_f(delta_occ, ro[v])) * A + ora_f(delta_emp, ro[v]) * B));
    }
  }
  free(PE);
  free(DE);
  free(s);
  const double s2pi = 2.50662827463100050242;
  return nval(&I) / (s2pi * sigma_p);
}

/* alpha, beta, theta, gamma straight from their definitions. */
void ora_tab_definition(double x, double sp, int Lb, int Lmax, double* alpha, double* beta,
                        double* theta, double* gamma) {
  for (int a = 1; a <= Lb; ++a)
    for (int b = 1; b <= Lb; ++b) {
      alpha[a * (Lb + 1) + b] = alpha_def(x, a, b, sp);
      beta[a * (Lb + 1) + b] = beta_def(x, a, b, sp);
    }
  for (int L = 1; L <= Lmax; ++L) {
    theta[L] = alpha_def(x, L, L, sp);
    gamma[L] = beta_def(x, L, L, sp);
  }
}

/* The tabulation recurrences of Alg 9 and Alg 10 with the power of x on the row
   index j, as the definitions of alpha and beta require: the corner term added
   when the block grows to (Lu, Lv) is at j = Lu-1, k = Lv-1. */
void ora_tab_recurrence(double x, double sp, int Lb, int Lmax, double* alpha, double* beta,
                        double* theta, double* gamma) {
  const int W = Lb + 1;
#define EXPSQ(d) exp(-((double)(d) * (double)(d)) / (2.0 * sp * sp))
  alpha[1 * W + 1] = 1.0;
  beta[1 * W + 1] = 0.0;
  for (int Lu = 2; Lu <= Lb; ++Lu) {
    alpha[Lu * W + 1] = alpha[(Lu - 1) * W + 1] + pow(x, Lu - 1) * EXPSQ(Lu - 1);
    beta[Lu * W + 1] = 0.0;
  }
  for (int Lv = 2; Lv <= Lb; ++Lv) {
    alpha[1 * W + Lv] = alpha[1 * W + Lv - 1] + EXPSQ(1 - Lv);
    beta[1 * W + Lv] = beta[1 * W + Lv - 1] + (double)(Lv - 1) * EXPSQ(1 - Lv);
  }
  for (int Lu = 2; Lu <= Lb; ++Lu)
    for (int Lv = 2; Lv <= Lb; ++Lv) {
      alpha[Lu * W + Lv] = alpha[Lu * W + Lv - 1] + alpha[(Lu - 1) * W + Lv] -
                           alpha[(Lu - 1) * W + Lv - 1] + pow(x, Lu - 1) * EXPSQ(Lu - Lv);
      beta[Lu * W + Lv] = beta[Lu * W + Lv - 1] + beta[(Lu - 1) * W + Lv] -
                          beta[(Lu - 1) * W + Lv - 1] +
                          (double)(Lv - 1) * pow(x, Lu - 1) * EXPSQ(Lu - Lv);
    }
  for (int L = 1; L <= Lb && L <= Lmax; ++L) {
    theta[L] = alpha[L * W + L];
    gamma[L] = beta[L * W + L];
  }
  for (int L = Lb + 1; L <= Lmax; ++L) {
    theta[L] = theta[L - 1];
    gamma[L] = gamma[L - 1];
    for (int i = 1; i <= L - 1; ++i) {
      theta[L] += pow(x, L - 1) * EXPSQ(i - L); /* new row j = L-1, k = i-1 */
      theta[L] += pow(x, i - 1) * EXPSQ(i - L); /* new column k = L-1, j = i-1 */
      gamma[L] += (double)(i - 1) * pow(x, L - 1) * EXPSQ(i - L);
      gamma[L] += (double)(L - 1) * pow(x, i - 1) * EXPSQ(i - L);
    }
    theta[L] += pow(x, L - 1);
    gamma[L] += (double)(L - 1) * pow(x, L - 1);
  }
#undef EXPSQ
}

/* ------------------------------------------------------------------ */
/* Ray traversal.  The paper only says the beam's cells are listed in   */
/* ascending distance (Sec. 2.2, Sec. 3.1); this is a grid walk in the  */
/* style of Amanatides and Woo with every rounding pinned down:         */
/*  - face distance t_a = (face_a - p_a) * (1/d_a), two roundings, no FMA, */
/*    recomputed from the integer face after each step;                  */
/*  - a tie between axes steps all tied axes at once (diagonal step);     */
/*  - a cell is listed only if its [entry, exit) interval is non-empty;   */
/*  - the last cell is cut at R; the walk stops when it leaves the map.   */
/* ------------------------------------------------------------------ */
int ora_raycast2d(const float* map, int64_t X, int64_t Y, double px, double py, double dx,
                  double dy, double R, int max_cells, int32_t* cell, double* entry, float* occ) {
  if (!(px >= 0.0 && px < (double)X && py >= 0.0 && py < (double)Y)) return -1;
  if (dx == 0.0 && dy == 0.0) return -1;
  int64_t cx = (int64_t)floor(px), cy = (int64_t)floor(py);
  int sx = 0, sy = 0;
  double fx = 0.0, fy = 0.0, ix = 0.0, iy = 0.0, tx = INFINITY, ty = INFINITY;
  if (dx > 0.0) { sx = 1; fx = (double)(cx + 1); }
  if (dx < 0.0) { sx = -1; fx = (double)cx; }
  if (dy > 0.0) { sy = 1; fy = (double)(cy + 1); }
  if (dy < 0.0) { sy = -1; fy = (double)cy; }
  if (sx != 0) { ix = 1.0 / dx; tx = (fx - px) * ix; }
  if (sy != 0) { iy = 1.0 / dy; ty = (fy - py) * iy; }
  double tcur = 0.0;
  int n = 0;
  for (;;) {
    double tnext = (tx < ty) ? tx : ty;
    double end = (tnext < R) ? tnext : R;
    if (end > tcur) {
      if (n >= max_cells) return -2;
      cell[n] = (int32_t)(cx + X * cy);
      entry[n] = tcur;
      if (occ) occ[n] = map[cx + X * cy];
      ++n;
    }
    if (tnext >= R) {
      entry[n] = R;
      return n;
    }
    if (tx == tnext) { cx += sx; fx += (double)sx; tx = (fx - px) * ix; }
    if (ty == tnext) { cy += sy; fy += (double)sy; ty = (fy - py) * iy; }
    tcur = (tnext > tcur) ? tnext : tcur;
    if (cx < 0 || cx >= X || cy < 0 || cy >= Y) {
      entry[n] = tcur;
      return n;
    }
  }
}

/* Virtual cells (Sec. 4: the beam projected onto equally sized cells of width w):
   cell i = 1..floor(R/w) covers [(i-1)w, iw) and takes the occupancy of the voxel
   holding its midpoint q = p + t_i d, t_i = (i - 1/2) w (per axis, no FMA).  The
   beam ends at the first midpoint outside the map. */
int ora_virtual3d(const float* map, int64_t X, int64_t Y, int64_t Z, const double* p,
                  const double* d, double R, double w, int max_cells, int32_t* cell, float* occ) {
  if (!(p[0] >= 0.0 && p[0] < (double)X && p[1] >= 0.0 && p[1] < (double)Y && p[2] >= 0.0 &&
        p[2] < (double)Z))
    return -1;
  int64_t nmax = (int64_t)floor(R / w);
  int n = 0;
  for (int64_t i = 1; i <= nmax; ++i) {
    double t = ((double)i - 0.5) * w;
    double qx = p[0] + t * d[0];
    double qy = p[1] + t * d[1];
    double qz = p[2] + t * d[2];
    double vx = floor(qx), vy = floor(qy), vz = floor(qz);
    if (vx < 0.0 || vx >= (double)X || vy < 0.0 || vy >= (double)Y || vz < 0.0 || vz >= (double)Z)
      break;
    if (n >= max_cells) return -2;
    int64_t idx = (int64_t)vx + X * ((int64_t)vy + Y * (int64_t)vz);
    cell[n] = (int32_t)idx;
    occ[n] = map[idx];
    ++n;
  }
  return n;
}

/* Run-length encoding (Eq. occup_rle): maximal runs of bit-identical values. */
int ora_rle_runs(int n, const float* occ, float* run_o, int32_t* run_len) {
  int nr = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t a, b = 0;
    memcpy(&a, &occ[i], 4);
    if (nr > 0) memcpy(&b, &run_o[nr - 1], 4);
    if (nr > 0 && a == b) {
      run_len[nr - 1] += 1;
    } else {
      run_o[nr] = occ[i];
      run_len[nr] = 1;
      ++nr;
    }
  }
  return nr;
}

/* ------------------------------------------------------------------ */
/* Batches                                                             */
/* ------------------------------------------------------------------ */
int ora_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static double eval_one(int variant, int Delta, int H, double delta_occ, double slope, int tail,
                       int n, const double* o, const double* l, double sigma) {
  if (variant == ORA_EXACT && (slope != 0.0 || tail))
    return ora_fsmi_exact_ext(n, o, l, sigma, slope, tail, delta_occ);
  if (variant == ORA_EXACT) return ora_fsmi_exact(n, o, l, sigma, delta_occ);
  if (variant == ORA_APPROX) return ora_fsmi_approx(n, o, l, sigma, delta_occ, Delta);
  if (variant == ORA_CSQMI) return ora_csqmi(n, o, l, sigma, Delta);
  return ora_fsmi_uniform(n, o, delta_occ, H);
}

int ora_eval_beams(int variant, int Delta, int H, double delta_occ, double slope, int tail,
                   int64_t n_beams, const int64_t* off, const float* occ, const double* bound,
                   const float* sigma, double* mi, int threads) {
  if (threads <= 0) threads = ora_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads)
  for (int64_t b = 0; b < n_beams; ++b) {
    int n = (int)(off[b + 1] - off[b]);
    double* o = (double*)malloc(sizeof(double) * (n + 1));
    double* l = (double*)malloc(sizeof(double) * (n + 1));
    for (int i = 0; i < n; ++i) o[i] = (double)occ[off[b] + i];
    for (int i = 0; i <= n; ++i) l[i] = bound ? bound[off[b] + b + i] : (double)i;
    mi[b] = eval_one(variant, Delta, H, delta_occ, slope, tail, n, o, l, (double)sigma[b]);
    free(o);
    free(l);
  }
  return 0;
}

int ora_rle_eval_beams(int exact, int kind, int Delta, int H, double delta_occ, int64_t n_beams,
                       const int64_t* run_off, const float* run_occ, const int32_t* run_len,
                       const float* sigma_p, double* mi, int threads) {
  if (threads <= 0) threads = ora_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads)
  for (int64_t b = 0; b < n_beams; ++b) {
    int nr = (int)(run_off[b + 1] - run_off[b]);
    double* ro = (double*)malloc(sizeof(double) * (nr + 1));
    int* L = (int*)malloc(sizeof(int) * (nr + 1));
    for (int u = 0; u < nr; ++u) {
      ro[u] = (double)run_occ[run_off[b] + u];
      L[u] = run_len[run_off[b] + u];
    }
    mi[b] = ora_rle_expanded(nr, ro, L, (double)sigma_p[b], delta_occ, kind, exact ? -1 : Delta, H);
    free(ro);
    free(L);
  }
  return 0;
}

/* Per pose (Sec. 2.4: the scan's MI is the sum over its beams):
   world direction = R(yaw) * sensor direction, each product rounded on its own. */
int ora_eval_poses_2d(int variant, int Delta, int H, double delta_occ, double slope, int tail,
                      const float* map, int64_t X, int64_t Y, int64_t n_poses,
                      const double* poses, int64_t n_beams, const double* beam_dir, double sigma,
                      double R, double* mi_pose, double* mi_beam, int threads) {
  if (threads <= 0) threads = ora_max_threads();
  int max_cells = (int)floor(1.4142135623730951 * R) + 3;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(| : bad)
  for (int64_t p = 0; p < n_poses; ++p) {
    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * max_cells);
    double* entry = (double*)malloc(sizeof(double) * (max_cells + 1));
    float* of = (float*)malloc(sizeof(float) * max_cells);
    double* o = (double*)malloc(sizeof(double) * max_cells);
    const double* ps = poses + 4 * p;
    nsum tot = {0.0, 0.0};
    for (int64_t b = 0; b < n_beams; ++b) {
      double bx = beam_dir[2 * b], by = beam_dir[2 * b + 1];
      double m1 = ps[2] * bx, m2 = ps[3] * by, m3 = ps[3] * bx, m4 = ps[2] * by;
      double wx = m1 - m2, wy = m3 + m4;
      int n = ora_raycast2d(map, X, Y, ps[0], ps[1], wx, wy, R, max_cells, cell, entry, of);
      double v;
      if (n < 0) {
        v = NAN;
        bad = 1;
      } else {
        for (int i = 0; i < n; ++i) o[i] = (double)of[i];
        v = eval_one(variant, Delta, H, delta_occ, slope, tail, n, o, entry, sigma);
      }
      if (mi_beam) mi_beam[p * n_beams + b] = v;
      nadd(&tot, v);
    }
    mi_pose[p] = nval(&tot);
    free(cell);
    free(entry);
    free(of);
    free(o);
  }
  return bad ? -1 : 0;
}

int ora_eval_poses_3d(int exact, int kind, int Delta, int H, double delta_occ, const float* map,
                      int64_t X, int64_t Y, int64_t Z, int64_t n_poses, const double* poses,
                      int64_t n_beams, const double* beam_dir, double sigma, double R, double w,
                      double* mi_pose, double* mi_beam, int threads) {
  if (threads <= 0) threads = ora_max_threads();
  int max_cells = (int)floor(R / w) + 1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(| : bad)
  for (int64_t p = 0; p < n_poses; ++p) {
    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * max_cells);
    float* of = (float*)malloc(sizeof(float) * max_cells);
    double* o = (double*)malloc(sizeof(double) * max_cells);
    const double* ps = poses + 5 * p;
    nsum tot = {0.0, 0.0};
    for (int64_t b = 0; b < n_beams; ++b) {
      const double* bd = beam_dir + 3 * b;
      double m1 = ps[3] * bd[0], m2 = ps[4] * bd[1], m3 = ps[4] * bd[0], m4 = ps[3] * bd[1];
      double d[3] = {m1 - m2, m3 + m4, bd[2]};
      int n = ora_virtual3d(map, X, Y, Z, ps, d, R, w, max_cells, cell, of);
      double v;
      if (n < 0) {
        v = NAN;
        bad = 1;
      } else {
        for (int i = 0; i < n; ++i) o[i] = (double)of[i];
        v = ora_fsmi_eqwidth(n, o, sigma / w, delta_occ, kind, exact ? -1 : Delta, H);
      }
      if (mi_beam) mi_beam[p * n_beams + b] = v;
      nadd(&tot, v);
    }
    mi_pose[p] = nval(&tot);
    free(cell);
    free(of);
    free(o);
  }
  return bad ? -1 : 0;
}
