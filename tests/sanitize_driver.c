/*
 * Test driver of the CPU oracle for the sanitizer build (tests/test_sanitize_cpu.py):
 * reads one problem from stdin -- the fields of or_cfg in declaration order
 * (freqs_hz excluded, always NULL), the checkpoint interval, then the density
 * over the design box -- runs forward, adjoint and gradient, and prints F and
 * dF/drho, one value per line.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer, any out-of-bounds access, leak or undefined
 * operation of the oracle ends the run with a report and a non-zero status.
 */
#include "../oracle/oracle_common.h"

typedef struct or2d or2d;
typedef struct or3d or3d;
int or2d_create(const or_cfg *cfg, or2d **out);
int or2d_set_checkpoint(or2d *o, int every);
int or2d_set_density(or2d *o, const double *rho);
int or2d_forward(or2d *o, double *F);
int or2d_adjoint(or2d *o);
int or2d_gradient(or2d *o, double *grad, double *d_eps, double *d_psi, double *d_sig);
void or2d_destroy(or2d *o);
int or3d_create(const or_cfg *cfg, or3d **out);
int or3d_set_checkpoint(or3d *o, int every);
int or3d_set_density(or3d *o, const double *rho);
int or3d_forward(or3d *o, double *F);
int or3d_adjoint(or3d *o);
int or3d_gradient(or3d *o, double *grad, double *d_eps, double *d_psi, double *d_sig);
void or3d_destroy(or3d *o);

static int rd_i(int32_t *v) { return scanf("%d", v) == 1; }
static int rd_d(double *v) { return scanf("%lf", v) == 1; }

int main(void) {
  or_cfg c;
  memset(&c, 0, sizeof c);
  int ok = rd_i(&c.dims) && rd_i(&c.nx) && rd_i(&c.ny) && rd_i(&c.nz) && rd_i(&c.n_steps) && rd_i(&c.pml_cells) &&
           rd_i(&c.tfsf_margin) && rd_i(&c.periodic_x);
  for (int k = 0; k < 3 && ok; ++k) ok = rd_i(&c.design_lo[k]);
  for (int k = 0; k < 3 && ok; ++k) ok = rd_i(&c.design_n[k]);
  for (int k = 0; k < 3 && ok; ++k) ok = rd_i(&c.gap_lo[k]);
  for (int k = 0; k < 3 && ok; ++k) ok = rd_i(&c.gap_n[k]);
  ok = ok && rd_i(&c.source_kind) && rd_i(&c.objective_kind) && rd_i(&c.weight_kind) && rd_i(&c.n_freq);
  double *d[] = {&c.dx, &c.courant, &c.pml_order, &c.pml_sigma_scale, &c.pml_kappa_max, &c.pml_alpha_max,
                 &c.eps_s, &c.eps_g, &c.eps_inf, &c.omega_p, &c.gamma_p, &c.gamma_mult, &c.sigma_max,
                 &c.psi_s_ratio, &c.f_lo, &c.f_hi, &c.t0_over_tau, &c.amplitude};
  for (size_t k = 0; k < sizeof d / sizeof d[0] && ok; ++k) ok = rd_d(d[k]);
  int32_t ckpt = 0;
  ok = ok && rd_i(&ckpt);
  if (!ok) { fprintf(stderr, "bad input\n"); return 2; }
  c.freqs_hz = NULL;
  const int nd = c.design_n[0] * c.design_n[1] * (c.dims == 3 ? c.design_n[2] : 1);
  double *rho = (double *)malloc(sizeof(double) * nd), *g = (double *)malloc(sizeof(double) * nd);
  for (int i = 0; i < nd; ++i)
    if (!rd_d(&rho[i])) { fprintf(stderr, "bad density\n"); return 2; }
  double F = 0.0;
  int rc;
  if (c.dims == 2) {
    or2d *o = NULL;
    rc = or2d_create(&c, &o);
    if (!rc) rc = or2d_set_checkpoint(o, ckpt);
    if (!rc) rc = or2d_set_density(o, rho);
    if (!rc) rc = or2d_forward(o, &F);
    if (!rc) rc = or2d_adjoint(o);
    if (!rc) rc = or2d_gradient(o, g, NULL, NULL, NULL);
    or2d_destroy(o);
  } else {
    or3d *o = NULL;
    rc = or3d_create(&c, &o);
    if (!rc) rc = or3d_set_checkpoint(o, ckpt);
    if (!rc) rc = or3d_set_density(o, rho);
    if (!rc) rc = or3d_forward(o, &F);
    if (!rc) rc = or3d_adjoint(o);
    if (!rc) rc = or3d_gradient(o, g, NULL, NULL, NULL);
    or3d_destroy(o);
  }
  if (rc) { fprintf(stderr, "oracle status %d\n", rc); return 3; }
  printf("%.17g\n", F);
  for (int i = 0; i < nd; ++i) printf("%.17g\n", g[i]);
  free(rho);
  free(g);
  return 0;
}
