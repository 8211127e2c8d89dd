/*
 * oracle_common.h -- pieces shared by the 2D and 3D CPU oracles.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, FP64 CPU
 * implementation of the time-domain topology-optimization hot path of
 * Hassan & Cala Lesina, "Topology optimization of dispersive plasmonic
 * nanostructures in the time-domain" (arXiv 2203.01462): the Drude-ADE FDTD
 * forward solve, its exact discrete adjoint and the per-edge sensitivities.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may call it.  It shares no code, header, table or constant with the HIP
 * library; both are written independently from the paper.
 *
 * Precision: IEEE double, round to nearest; build with -O2 -ffp-contract=off.
 */
#ifndef ORACLE_COMMON_H
#define ORACLE_COMMON_H

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_C0 299792458.0
#define OR_MU0 (4.0e-7 * M_PI)
#define OR_EPS0 (1.0 / (OR_MU0 * OR_C0 * OR_C0))

enum { OR_OK = 0, OR_EINVAL = 1, OR_ESTATE = 2, OR_ENOMEM = 3, OR_EUNSTABLE = 5 };
enum { OR_SRC_GAUSS = 0, OR_SRC_SINC_HANN = 1, OR_SRC_NONE = 2 };
enum { OR_OBJ_DFT = 0, OR_OBJ_TIME_ENERGY = 1 };
enum { OR_W_ENHANCEMENT = 0, OR_W_UNIT = 1 };

/* Problem description.  Index triples are (x, y, z); 2D ignores z. */
typedef struct {
  int32_t dims, nx, ny, nz;
  int32_t n_steps, pml_cells, tfsf_margin, periodic_x;
  int32_t design_lo[3], design_n[3], gap_lo[3], gap_n[3];
  int32_t source_kind, objective_kind, weight_kind, n_freq;
  double dx, courant;
  double pml_order, pml_sigma_scale, pml_kappa_max, pml_alpha_max;
  double eps_s, eps_g, eps_inf, omega_p, gamma_p, gamma_mult, sigma_max, psi_s_ratio;
  double f_lo, f_hi, t0_over_tau, amplitude;
  const double *freqs_hz; /* NULL: n_freq frequencies uniform over [f_lo, f_hi] */
} or_cfg;

/* Excitation waveform (Sec. 2).  GAUSS: a carrier at the band centre under a
 * Gaussian envelope whose spectrum falls to half its peak at the band edges.
 * SINC_HANN: the paper's choice, a sinc envelope whose spectrum is the band,
 * cut after four lobes on each side, tapered by a Hann window, on the same
 * carrier.  Both start near zero at t = 0. */
static double or_source(const or_cfg *c, double t) {
  const double fc = 0.5 * (c->f_lo + c->f_hi);
  const double bw = c->f_hi - c->f_lo;
  if (c->source_kind == OR_SRC_NONE) return 0.0;
  if (c->source_kind == OR_SRC_GAUSS) {
    const double tau = sqrt(log(2.0)) / (M_PI * 0.5 * bw);
    const double t0 = c->t0_over_tau * tau;
    const double u = (t - t0) / tau;
    return c->amplitude * sin(2.0 * M_PI * fc * (t - t0)) * exp(-u * u);
  }
  /* SINC_HANN */
  const double half = 4.0 / bw; /* four lobes of width 1/bw on each side */
  const double t0 = half;
  const double s = t - t0;
  if (fabs(s) >= half) return 0.0;
  const double x = M_PI * bw * s;
  const double env = (fabs(x) < 1e-300) ? 1.0 : sin(x) / x;
  const double hann = 0.5 * (1.0 + cos(M_PI * s / half));
  return c->amplitude * env * hann * cos(2.0 * M_PI * fc * s);
}

/* Convolutional PML grading at depth d in (0,1] (1 at the wall): conductivity
 * rises as d^m to the usual optimum 0.8(m+1)/(eta dx); fills the
 * recursive-convolution coefficients b, a and the stretch kappa. */
static void or_pml_grade(const or_cfg *c, double dt, double d, double *b, double *a, double *kap) {
  const double m = c->pml_order;
  const double eta = sqrt(OR_MU0 / (OR_EPS0 * c->eps_s));
  const double smax = c->pml_sigma_scale * 0.8 * (m + 1.0) / (eta * c->dx);
  const double sig = smax * pow(d, m);
  const double k = 1.0 + (c->pml_kappa_max - 1.0) * pow(d, m);
  const double alp = c->pml_alpha_max * (1.0 - d);
  *kap = k;
  *b = exp(-(sig / k + alp) * dt / OR_EPS0);
  *a = (sig > 0.0) ? sig * (*b - 1.0) / (sig * k + k * k * alp) : 0.0;
}

/* Profile at coordinate `pos` (in cells, possibly half integer) on an axis
 * with nodes 0..n-1 whose outermost nodes are PEC walls; the absorber covers
 * the P cells next to each wall.  Returns 1 inside the absorber. */
static int or_pml_profile(const or_cfg *c, double dt, int n, int P, double pos,
                          double *b, double *a, double *kap) {
  double d = 0.0;
  if (P > 0) {
    if (pos < P) d = (P - pos) / P;
    else if (pos > (n - 1) - P) d = (pos - ((n - 1) - P)) / P;
  }
  if (d <= 0.0) { *b = 1.0; *a = 0.0; *kap = 1.0; return 0; }
  or_pml_grade(c, dt, d, b, a, kap);
  return 1;
}

/* One-dimensional incident-field line for the total-field/scattered-field
 * plane-wave injection (the injection boundary Gamma of Sec. 2).  The line
 * lies along the propagation axis in the background eps_s with the same dx and
 * dt as the main grid, so a plane wave on the main grid evolves exactly as on
 * this line.  Node 0 is driven by the waveform; the far end has a graded
 * absorber backed by a PEC node.
 *   einc[n*L + p], n = 0..N : transverse E at node p, time n dt
 *   hinc[n*L + p], n = 0..N-1: transverse H between nodes p and p+1, time (n+1/2) dt,
 *                              with the sign that makes E x H point along +axis.
 * Returns 0 on success. */
static int or_incident_line(const or_cfg *c, double dt, int L, int N,
                            double **einc_out, double **hinc_out) {
  const int P1 = 20;
  const int n1 = L + P1 + 1;
  double *e = (double *)calloc((size_t)n1, sizeof(double));
  double *h = (double *)calloc((size_t)n1, sizeof(double));
  double *pe = (double *)calloc((size_t)n1, sizeof(double));
  double *ph = (double *)calloc((size_t)n1, sizeof(double));
  double *be = (double *)malloc(sizeof(double) * n1), *ae = (double *)malloc(sizeof(double) * n1);
  double *ke = (double *)malloc(sizeof(double) * n1), *bh = (double *)malloc(sizeof(double) * n1);
  double *ah = (double *)malloc(sizeof(double) * n1), *kh = (double *)malloc(sizeof(double) * n1);
  double *einc = (double *)malloc(sizeof(double) * (size_t)(N + 1) * L);
  double *hinc = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * L);
  if (!e || !h || !pe || !ph || !be || !ae || !ke || !bh || !ah || !kh || !einc || !hinc) {
    free(e); free(h); free(pe); free(ph); free(be); free(ae); free(ke); free(bh); free(ah); free(kh);
    free(einc); free(hinc);
    return 1;
  }
  /* absorber only on the far side, graded towards the PEC node n1-1 */
  for (int p = 0; p < n1; ++p) {
    const double start = (double)(n1 - 1 - P1);
    const double de_ = (p - start) / P1, dh_ = (p + 0.5 - start) / P1;
    be[p] = 1; ae[p] = 0; ke[p] = 1; bh[p] = 1; ah[p] = 0; kh[p] = 1;
    if (de_ > 0.0) or_pml_grade(c, dt, de_, &be[p], &ae[p], &ke[p]);
    if (dh_ > 0.0) or_pml_grade(c, dt, dh_, &bh[p], &ah[p], &kh[p]);
  }
  const double ch = dt / (OR_MU0 * c->dx);
  const double ce = dt / (OR_EPS0 * c->eps_s * c->dx);
  e[0] = or_source(c, 0.0);
  for (int p = 0; p < L; ++p) einc[p] = e[p];
  for (int n = 0; n < N; ++n) {
    for (int p = 0; p < n1 - 1; ++p) {
      const double de = e[p + 1] - e[p];
      ph[p] = bh[p] * ph[p] + ah[p] * de / c->dx;
      h[p] -= ch * (de / kh[p]) + (dt / OR_MU0) * ph[p];
    }
    for (int p = 0; p < L; ++p) hinc[(size_t)n * L + p] = h[p];
    for (int p = 1; p < n1 - 1; ++p) {
      const double dh = h[p] - h[p - 1];
      pe[p] = be[p] * pe[p] + ae[p] * dh / c->dx;
      e[p] -= ce * (dh / ke[p]) + (dt / (OR_EPS0 * c->eps_s)) * pe[p];
    }
    e[0] = or_source(c, (n + 1) * dt);
    e[n1 - 1] = 0.0;
    for (int p = 0; p < L; ++p) einc[(size_t)(n + 1) * L + p] = e[p];
  }
  free(e); free(h); free(pe); free(ph); free(be); free(ae); free(ke); free(bh); free(ah); free(kh);
  *einc_out = einc;
  *hinc_out = hinc;
  return 0;
}

/* Band frequencies and objective weights.  Default frequencies are uniform
 * over [f_lo, f_hi] inclusive.  ENHANCEMENT weights are 1/|G(w_k)|^2 with G the
 * same running DFT of the excitation waveform, so each term is a field
 * enhancement; UNIT weights are 1 (also used when there is no excitation). */
static int or_freqs_weights(const or_cfg *c, double dt, double *f, double *w) {
  const int K = c->n_freq;
  for (int k = 0; k < K; ++k) {
    if (c->freqs_hz) f[k] = c->freqs_hz[k];
    else f[k] = (K == 1) ? 0.5 * (c->f_lo + c->f_hi) : c->f_lo + (c->f_hi - c->f_lo) * k / (K - 1);
  }
  for (int k = 0; k < K; ++k) {
    if (c->weight_kind == OR_W_UNIT || c->source_kind == OR_SRC_NONE) { w[k] = 1.0; continue; }
    double re = 0.0, im = 0.0;
    const double om = 2.0 * M_PI * f[k];
    for (int n = 1; n <= c->n_steps; ++n) {
      const double g = or_source(c, n * dt);
      re += dt * g * cos(om * n * dt);
      im -= dt * g * sin(om * n * dt);
    }
    const double m2 = re * re + im * im;
    if (!(m2 > 0.0)) return 1;
    w[k] = 1.0 / m2;
  }
  return 0;
}

#endif
