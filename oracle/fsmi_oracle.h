/*
 * fsmi_oracle.h -- plain FP64 CPU oracle for FSMI (arXiv 1905.02238).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library
 * against the paper.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Every function computes in double precision with sequential loops written
 * in the paper's order and notation; sums use Neumaier compensation.
 * Occupancies arrive as float (the maps are float) and are widened to double.
 *
 * Readings of the paper where it is silent or garbled (see the function
 * comments): the all-empty event e_0 contributes nothing (its range reading
 * lies beyond the beam), the z integral runs over [0, l_{n+1}), the
 * inverse-sensor odds are delta_emp = 1/delta_occ, logs are natural (nats).
 */
#ifndef FSMI_ORACLE_H
#define FSMI_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* ---- per-cell quantities (Sec. 2.2, Eq. for f(delta, r)) ---- */
double ora_f(double delta, double o);          /* o-form, defined on [0,1] */
double ora_f_odds(double delta, double r);     /* paper's r-form, r in (0,inf) */

/* Alg 2: P[0] = P(e_0), P[j] = P(e_j) for j = 1..n  (P has n+1 entries) */
void ora_first_hit(int n, const double* o, double* P);
/* Alg 3: C[k-1] = C_k for k = 1..n */
void ora_info_gain(int n, const double* o, double delta_occ, double* C);
/* G_{k,j} = Phi((l_{k+1}-mu_j)/sigma) - Phi((l_k-mu_j)/sigma), tail-split */
double ora_G(double lk, double lk1, double mu, double sigma);

/* ---- single beam, boundaries l[0..n] (l[0] = l_1 = 0) ---- */
double ora_fsmi_exact(int n, const double* o, const double* l, double sigma, double delta_occ);
/* Thm 1 with sigma_j = sigma + slope mu_j and, if tail, the max-range term */
double ora_fsmi_exact_ext(int n, const double* o, const double* l, double sigma, double slope,
                          int tail, double delta_occ);
double ora_fsmi_approx(int n, const double* o, const double* l, double sigma, double delta_occ, int Delta);
double ora_fsmi_uniform(int n, const double* o, double delta_occ, int H);

/* ---- equal-width (virtual) cells, kernel w(d) on the index distance ---- */
enum { ORA_K_ERF = 0, ORA_K_DENSITY = 1, ORA_K_UNIFORM = 2 };
double ora_kernel_weight(int kind, double sigma_p, int H, int d);
/* sum_j sum_k P_j C_k w(k-j), w truncated to |k-j| <= trunc when trunc >= 0 */
double ora_fsmi_eqwidth(int n, const double* o, double sigma_p, double delta_occ,
                        int kind, int trunc, int H);

/* ---- run-length encoded beams (Sec. 4) ---- */
double ora_rle_expanded(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                        int kind, int trunc, int H);
double ora_rle_thm5(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                    int kind, int trunc, int H);
double ora_rle_thm6(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                    int kind, int Delta, int H);
double ora_rle_alpha_route(int nr, const double* ro, const int* L, double sigma_p, double delta_occ);
/* table mode of Approx-FSMI-RLE: tables at x = 1 - o quantised to i / levels (see the .c) */
double ora_rle_table(int nr, const double* ro, const int* L, double sigma_p, double delta_occ,
                     int Delta, int levels);
/* alpha/beta/theta/gamma by their definitions and by the (corrected) Alg 9/10 recurrences;
   arrays are [Lb+1][Lb+1] (alpha, beta) and [Lmax+1] (theta, gamma), index 0 unused */
void ora_tab_definition(double x, double sigma_p, int Lb, int Lmax,
                        double* alpha, double* beta, double* theta, double* gamma);
void ora_tab_recurrence(double x, double sigma_p, int Lb, int Lmax,
                        double* alpha, double* beta, double* theta, double* gamma);

/* ---- CSQMI (Sec. 2.3): Eq. csqmi_exact, Delta-truncated when Delta >= 0 ---- */
double ora_csqmi(int n, const double* o, const double* l, double sigma, int Delta);

/* ---- trajectory MI with cell marking (Sec. 2.4) ---- */
/* one beam, information of the cells with counted[i] != 0 only (variant ORA_*) */
double ora_fsmi_counted(int variant, int n, const double* o, const double* l, double sigma,
                        double delta_occ, int Delta, int H, const unsigned char* counted);
int ora_eval_trajectories_2d(int variant, int Delta, int H, double delta_occ, const float* map,
                             int64_t X, int64_t Y, int64_t n_traj, const int64_t* traj_off,
                             const double* poses, int64_t n_beams, const double* beam_dir,
                             double sigma, double R, double* mi_traj, double* mi_state,
                             double* mi_beam);

/* ---- ray traversal and virtual sampling ---- */
/* returns n >= 0 cells, -1 origin outside map / bad direction, -2 capacity */
int ora_raycast2d(const float* map, int64_t X, int64_t Y, double px, double py,
                  double dx, double dy, double R, int max_cells,
                  int32_t* cell, double* entry /* max_cells+1 */, float* occ);
int ora_virtual3d(const float* map, int64_t X, int64_t Y, int64_t Z, const double* p,
                  const double* d, double R, double w, int max_cells,
                  int32_t* cell, float* occ);
int ora_rle_runs(int n, const float* occ, float* run_o, int32_t* run_len);

/* ---- batches (OpenMP over beams; threads <= 0 means the OpenMP default) ---- */
/* ORA_CSQMI: the comparison metric of Sec. 2.3 (ora_csqmi), truncated at Delta */
enum { ORA_EXACT = 0, ORA_APPROX = 1, ORA_UNIFORM = 2, ORA_CSQMI = 3 };
/* slope, tail: the extensions of ora_fsmi_exact_ext (EXACT only; 0, 0 = Thm 1) */
int ora_eval_beams(int variant, int Delta, int H, double delta_occ, double slope, int tail,
                   int64_t n_beams, const int64_t* off, const float* occ,
                   const double* bound /* or NULL */, const float* sigma, double* mi, int threads);
int ora_rle_eval_beams(int exact, int kind, int Delta, int H, double delta_occ, int64_t n_beams,
                       const int64_t* run_off, const float* run_occ, const int32_t* run_len,
                       const float* sigma_p, double* mi, int threads);
int ora_eval_poses_2d(int variant, int Delta, int H, double delta_occ, double slope, int tail,
                      const float* map, int64_t X, int64_t Y,
                      int64_t n_poses, const double* poses /* [n][4] x,y,cos,sin */,
                      int64_t n_beams, const double* beam_dir /* [n][2] */,
                      double sigma, double R, double* mi_pose, double* mi_beam, int threads);
int ora_eval_poses_3d(int exact, int kind, int Delta, int H, double delta_occ,
                      const float* map, int64_t X, int64_t Y, int64_t Z,
                      int64_t n_poses, const double* poses /* [n][5] x,y,z,cos,sin */,
                      int64_t n_beams, const double* beam_dir /* [n][3] */,
                      double sigma, double R, double w, double* mi_pose, double* mi_beam,
                      int threads);
int ora_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
