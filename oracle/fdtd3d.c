/*
 * fdtd3d.c -- 3D CPU oracle (FP64).  TEST INFRASTRUCTURE ONLY.
 *
 * The same method as fdtd2d.c on the full Yee cell (Sec. 3.2 of the paper):
 *   E_x at (i+1/2, j, k), E_y at (i, j+1/2, k), E_z at (i, j, k+1/2),
 *   H_x at (i, j+1/2, k+1/2), H_y at (i+1/2, j, k+1/2), H_z at (i+1/2, j+1/2, k),
 * arrays [k][j][i] with i fastest, all outer faces PEC.
 *   mu0 dH/dt = -curl E           (eq. (10c))
 *   eps0 eps_inf dE/dt + J + sigma E = curl H,  dJ/dt + gamma J = eps0 psi E   (eqs. (10a-b))
 * with the trapezoidal ADE update, the interpolation of eqs. (4)-(5) on every
 * Drude edge, a convolutional PML (one memory per curl term), and a plane
 * wave along +z with E along x injected on a total-field box.
 *
 * Design variables: cell (i,j,k) of the design box owns its three
 * index-aligned edges E_x[k][j][i], E_y[k][j][i], E_z[k][j][i], which share
 * rho_ijk; dF/drho of the cell is the sum over the three edges of eq. (27)
 * applied to the per-edge sensitivities of eq. (25).  Gap cells own three
 * non-dispersive edges (eps_g) observed by the monitor; the objective sums
 * over the gap cells and the three components.
 *
 * Adjoint: backwards in time with the same update; inside the absorber each
 * curl term is replaced by its exact transpose (grading and memory applied
 * to the differenced field before the difference).
 */
#include "oracle_common.h"

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct or3d {
  or_cfg c;
  double *freqs, *wts;
  int nx, ny, nz, N, K, nd, ng;
  double dt;
  int d0[3], dn[3], g0[3], gn[3];
  /* grading per axis at integer (e) and half-integer (h) positions: b, a, 1/kappa, in-absorber flag */
  double *be[3], *ae[3], *ike[3], *bh[3], *ah[3], *ikh[3];
  unsigned char *ine[3], *inh[3];
  double *E[3], *H[3], *J[3];
  /* absorber memories: pE[c][u] belongs to E component c, derivative axis u
   * (u != c); pH likewise.  Full-size arrays, used only inside the absorber. */
  double *pE[3][3], *pH[3][3];
  int tf_on, lo[3], hi[3], kref, L;
  double *einc, *hinc;
  double *rho;
  double *dft;   /* [K][ng][3][2] */
  double *gapE;  /* [N+1][ng][3] */
  double *hist;  /* [hist_steps][3][nd]: E^{n+1} on design edges, slot n - hist_base */
  int hist_steps, hist_base, hist_on, mon_on;
  double *gEps, *gSig, *gPsi; /* [3][nd] */
  /* segment checkpointing (ck > 0): a snapshot of the forward state at the
   * start of every ck-step segment, and a second state (rE, rH, rJ, rpE,
   * rpH) on which the adjoint re-runs each segment to refill the history */
  int ck, nseg;
  size_t snap_len;
  double *snap;
  double *rE[3], *rH[3], *rJ[3], *rpE[3][3], *rpH[3][3];
  int state;
  char err[256];
} or3d;

static char g_err3[256];

static int fail3(or3d *o, int code, const char *msg) {
  if (o) snprintf(o->err, sizeof o->err, "%s", msg);
  else snprintf(g_err3, sizeof g_err3, "%s", msg);
  return code;
}

const char *or3d_last_error(const or3d *o) { return o ? o->err : g_err3; }

#define IX3(o, i, j, k) (((size_t)(k) * (o)->ny + (j)) * (o)->nx + (i))

static inline int in_box(const int *lo, const int *n, int i, int j, int k) {
  return i >= lo[0] && i < lo[0] + n[0] && j >= lo[1] && j < lo[1] + n[1] && k >= lo[2] && k < lo[2] + n[2];
}
static inline int is_gap(const or3d *o, int i, int j, int k) { return in_box(o->g0, o->gn, i, j, k); }
static inline int is_drude(const or3d *o, int i, int j, int k) {
  return in_box(o->d0, o->dn, i, j, k) && !is_gap(o, i, j, k);
}
static inline int didx(const or3d *o, int i, int j, int k) {
  return ((k - o->d0[2]) * o->dn[1] + (j - o->d0[1])) * o->dn[0] + (i - o->d0[0]);
}

typedef struct { double eps, psi, sig, kp, beta, C1, C2; } coef3_t;

static coef3_t drude3(const or3d *o, double rho) {
  const or_cfg *c = &o->c;
  const double psi = c->omega_p * c->omega_p, psi_s = c->psi_s_ratio * psi;
  const double gam = c->gamma_mult * c->gamma_p, dt = o->dt;
  coef3_t k;
  k.eps = c->eps_s + rho * (c->eps_inf - c->eps_s);
  k.psi = psi_s + rho * (psi - psi_s);
  k.sig = rho * (1.0 - rho) * c->sigma_max;
  k.kp = (1.0 - gam * dt / 2.0) / (1.0 + gam * dt / 2.0);
  k.beta = (OR_EPS0 * k.psi * dt / 2.0) / (1.0 + gam * dt / 2.0);
  const double D = 2.0 * OR_EPS0 * k.eps + (k.beta + k.sig) * dt;
  k.C1 = (2.0 * OR_EPS0 * k.eps - (k.beta + k.sig) * dt) / D;
  k.C2 = 2.0 * dt / D;
  return k;
}

void or3d_destroy(or3d *o) {
  if (!o) return;
  free(o->freqs); free(o->wts);
  for (int a = 0; a < 3; ++a) {
    free(o->be[a]); free(o->ae[a]); free(o->ike[a]); free(o->bh[a]); free(o->ah[a]); free(o->ikh[a]);
    free(o->ine[a]); free(o->inh[a]); free(o->E[a]); free(o->H[a]); free(o->J[a]);
    for (int b = 0; b < 3; ++b) { free(o->pE[a][b]); free(o->pH[a][b]); }
    free(o->rE[a]); free(o->rH[a]); free(o->rJ[a]);
    for (int b = 0; b < 3; ++b) { free(o->rpE[a][b]); free(o->rpH[a][b]); }
  }
  free(o->snap);
  free(o->einc); free(o->hinc); free(o->rho); free(o->dft); free(o->gapE); free(o->hist);
  free(o->gEps); free(o->gSig); free(o->gPsi);
  free(o);
}

static int box3_ok(const int *lo, const int *n, const int *a, const int *b) {
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || lo[d] < a[d] || lo[d] + n[d] - 1 > b[d]) return 0;
  return 1;
}

int or3d_create(const or_cfg *cfg, or3d **out) {
  *out = NULL;
  if (!cfg) return fail3(NULL, OR_EINVAL, "null config");
  or_cfg c = *cfg;
  if (c.dims != 3) return fail3(NULL, OR_EINVAL, "dims must be 3");
  if (c.nx < 8 || c.ny < 8 || c.nz < 8) return fail3(NULL, OR_EINVAL, "grid too small");
  if (c.n_steps < 1) return fail3(NULL, OR_EINVAL, "n_steps < 1");
  if (!(c.courant > 0) || c.courant >= 1.0 / sqrt(3.0)) return fail3(NULL, OR_EINVAL, "Courant number outside (0, 1/sqrt(3))");
  if (c.n_freq < 1) return fail3(NULL, OR_EINVAL, "n_freq < 1");
  if (!(c.eps_s > 0) || !(c.eps_g > 0) || !(c.eps_inf > 0)) return fail3(NULL, OR_EINVAL, "permittivity <= 0");
  if (c.periodic_x) return fail3(NULL, OR_EINVAL, "periodic_x is 2D only");
  or3d *o = (or3d *)calloc(1, sizeof(or3d));
  if (!o) return fail3(NULL, OR_ENOMEM, "out of memory");
  o->c = c;
  o->nx = c.nx; o->ny = c.ny; o->nz = c.nz; o->N = c.n_steps; o->K = c.n_freq;
  o->dt = c.courant * c.dx / OR_C0;
  for (int d = 0; d < 3; ++d) { o->d0[d] = c.design_lo[d]; o->dn[d] = c.design_n[d]; o->g0[d] = c.gap_lo[d]; o->gn[d] = c.gap_n[d]; }
  o->nd = o->dn[0] * o->dn[1] * o->dn[2];
  o->ng = o->gn[0] * o->gn[1] * o->gn[2];
  const int P = c.pml_cells, m = c.tfsf_margin;
  const int n3[3] = {c.nx, c.ny, c.nz};
  o->tf_on = (c.source_kind != OR_SRC_NONE);
  int a[3], b[3];
  for (int d = 0; d < 3; ++d) {
    o->lo[d] = P + m; o->hi[d] = n3[d] - 1 - P - m;
    if (o->tf_on) { a[d] = o->lo[d] + 1; b[d] = o->hi[d] - 1; }
    else if (P == 0) { a[d] = 0; b[d] = n3[d] - 1; }   /* closed cavity: the design may fill the box */
    else { a[d] = P + 1; b[d] = n3[d] - 2 - P; }
  }
  int ok = 1;
  if (o->tf_on)
    for (int d = 0; d < 3; ++d) if (o->lo[d] < 3 || o->hi[d] - o->lo[d] < 2) ok = 0;
  if (!box3_ok(o->d0, o->dn, a, b)) ok = 0;
  if (o->ng > 0 && !box3_ok(o->g0, o->gn, a, b)) ok = 0;
  if (!ok) { or3d_destroy(o); return fail3(NULL, OR_EINVAL, "design/gap boxes must lie inside the interior (and the total-field box)"); }
  const size_t n = (size_t)c.nx * c.ny * c.nz;
  o->freqs = (double *)malloc(sizeof(double) * o->K);
  o->wts = (double *)malloc(sizeof(double) * o->K);
  int bad = !o->freqs || !o->wts;
  for (int d = 0; d < 3 && !bad; ++d) {
    const int nn = n3[d];
    o->be[d] = malloc(sizeof(double) * nn); o->ae[d] = malloc(sizeof(double) * nn); o->ike[d] = malloc(sizeof(double) * nn);
    o->bh[d] = malloc(sizeof(double) * nn); o->ah[d] = malloc(sizeof(double) * nn); o->ikh[d] = malloc(sizeof(double) * nn);
    o->ine[d] = malloc(nn); o->inh[d] = malloc(nn);
    o->E[d] = calloc(n, sizeof(double)); o->H[d] = calloc(n, sizeof(double)); o->J[d] = calloc(n, sizeof(double));
    for (int u = 0; u < 3; ++u)
      if (u != d) { o->pE[d][u] = calloc(n, sizeof(double)); o->pH[d][u] = calloc(n, sizeof(double)); bad |= !o->pE[d][u] || !o->pH[d][u]; }
    bad |= !o->be[d] || !o->ae[d] || !o->ike[d] || !o->bh[d] || !o->ah[d] || !o->ikh[d] || !o->ine[d] || !o->inh[d] ||
           !o->E[d] || !o->H[d] || !o->J[d];
  }
  o->rho = calloc((size_t)o->nd, sizeof(double));
  o->dft = calloc((size_t)o->K * (o->ng ? o->ng : 1) * 3 * 2, sizeof(double));
  o->gapE = calloc((size_t)(o->N + 1) * (o->ng ? o->ng : 1) * 3, sizeof(double));
  o->gEps = calloc(3 * (size_t)o->nd, sizeof(double));
  o->gSig = calloc(3 * (size_t)o->nd, sizeof(double));
  o->gPsi = calloc(3 * (size_t)o->nd, sizeof(double));
  if (bad || !o->rho || !o->dft || !o->gapE || !o->gEps || !o->gSig || !o->gPsi) {
    or3d_destroy(o);
    return fail3(NULL, OR_ENOMEM, "out of memory");
  }
  if (or_freqs_weights(&c, o->dt, o->freqs, o->wts)) { or3d_destroy(o); return fail3(NULL, OR_EINVAL, "zero source spectrum at a band frequency"); }
  o->c.freqs_hz = NULL;
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < n3[d]; ++q) {
      o->ine[d][q] = (unsigned char)or_pml_profile(&c, o->dt, n3[d], P, (double)q, &o->be[d][q], &o->ae[d][q], &o->ike[d][q]);
      o->inh[d][q] = (unsigned char)or_pml_profile(&c, o->dt, n3[d], P, q + 0.5, &o->bh[d][q], &o->ah[d][q], &o->ikh[d][q]);
      o->ike[d][q] = 1.0 / o->ike[d][q];
      o->ikh[d][q] = 1.0 / o->ikh[d][q];
    }
  o->kref = o->lo[2] - 2;
  o->L = o->hi[2] + 2 - o->kref + 1;
  if (o->tf_on && or_incident_line(&c, o->dt, o->L, o->N, &o->einc, &o->hinc)) {
    or3d_destroy(o);
    return fail3(NULL, OR_ENOMEM, "out of memory");
  }
  *out = o;
  return OR_OK;
}

int or3d_set_density(or3d *o, const double *rho) {
  for (int d = 0; d < o->nd; ++d)
    if (!(rho[d] >= 0.0 && rho[d] <= 1.0)) return fail3(o, OR_EINVAL, "density outside [0,1] or NaN");
  memcpy(o->rho, rho, sizeof(double) * o->nd);
  o->state = 1;
  return OR_OK;
}

static void zero3(or3d *o) {
  const size_t n = (size_t)o->nx * o->ny * o->nz;
  for (int d = 0; d < 3; ++d) {
    memset(o->E[d], 0, n * sizeof(double)); memset(o->H[d], 0, n * sizeof(double)); memset(o->J[d], 0, n * sizeof(double));
    for (int u = 0; u < 3; ++u) if (u != d) { memset(o->pE[d][u], 0, n * sizeof(double)); memset(o->pH[d][u], 0, n * sizeof(double)); }
  }
}

/* Update ranges of each component: E_c is tangential to the walls normal to
 * the two other axes (zero there) and lives at half positions along c; H_c
 * lives at half positions along the two other axes and is zero on the walls
 * normal to c. */
static void e_range(const or3d *o, int c, int *lo, int *hi) {
  const int n3[3] = {o->nx, o->ny, o->nz};
  for (int d = 0; d < 3; ++d) {
    if (d == c) { lo[d] = 0; hi[d] = n3[d] - 2; }
    else { lo[d] = 1; hi[d] = n3[d] - 2; }
  }
}
static void h_range(const or3d *o, int c, int *lo, int *hi) {
  const int n3[3] = {o->nx, o->ny, o->nz};
  for (int d = 0; d < 3; ++d) {
    if (d == c) { lo[d] = 1; hi[d] = n3[d] - 2; }
    else { lo[d] = 0; hi[d] = n3[d] - 2; }
  }
}

static const size_t *strides(const or3d *o, size_t *s) {
  s[0] = 1; s[1] = (size_t)o->nx; s[2] = (size_t)o->nx * o->ny;
  return s;
}

/* The two curl terms of component c: axes (u, v) and the other field's
 * components (f_u, f_v) with (curl X)_c = d_u X_{f_u} - d_v X_{f_v}. */
static void curl_axes(int c, int *u, int *v) {
  *u = (c + 1) % 3; *v = (c + 2) % 3;
}

/* Incident E_x at node row k, time n; incident H_y at k+1/2, time n+1/2. */
static inline double einc3(const or3d *o, int n, int k) { return o->einc[(size_t)n * o->L + (k - o->kref)]; }
static inline double hinc3(const or3d *o, int n, int k) { return o->hinc[(size_t)n * o->L + (k - o->kref)]; }

/* forward H^{n+1/2}: H_c -= dt/mu0 [ (d_u E_v)/kappa_u + psi_cu - (d_v E_u)/kappa_v - psi_cv ] */
static void fwd_h3(or3d *o, int n, int tf) {
  size_t st[3];
  strides(o, st);
  const double cm = o->dt / OR_MU0, dx = o->c.dx;
  for (int c = 0; c < 3; ++c) {
    int u, v, lo[3], hi[3];
    curl_axes(c, &u, &v);
    h_range(o, c, lo, hi);
    double *Hc = o->H[c];
    const double *Ev = o->E[v], *Eu = o->E[u];
#pragma omp parallel for schedule(static)
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          const int idx[3] = {i, j, k};
          const size_t q = IX3(o, i, j, k);
          const double du = (Ev[q + st[u]] - Ev[q]) / dx; /* d_u E_v at the H_c position */
          const double dv = (Eu[q + st[v]] - Eu[q]) / dx; /* d_v E_u */
          double tu = du * o->ikh[u][idx[u]], tv = dv * o->ikh[v][idx[v]];
          if (o->inh[u][idx[u]]) { o->pH[c][u][q] = o->bh[u][idx[u]] * o->pH[c][u][q] + o->ah[u][idx[u]] * du; tu += o->pH[c][u][q]; }
          if (o->inh[v][idx[v]]) { o->pH[c][v][q] = o->bh[v][idx[v]] * o->pH[c][v][q] + o->ah[v][idx[v]] * dv; tv += o->pH[c][v][q]; }
          Hc[q] -= cm * (tu - tv);
        }
  }
  if (tf) {
    const double ch = o->dt / (OR_MU0 * dx);
    /* H_y on the z-faces, H_z on the y-faces, fed by the incident E_x */
    for (int j = o->lo[1]; j <= o->hi[1]; ++j)
      for (int i = o->lo[0]; i <= o->hi[0] - 1; ++i) {
        o->H[1][IX3(o, i, j, o->lo[2] - 1)] += ch * einc3(o, n, o->lo[2]);
        o->H[1][IX3(o, i, j, o->hi[2])] -= ch * einc3(o, n, o->hi[2]);
      }
    for (int k = o->lo[2]; k <= o->hi[2]; ++k)
      for (int i = o->lo[0]; i <= o->hi[0] - 1; ++i) {
        o->H[2][IX3(o, i, o->lo[1] - 1, k)] -= ch * einc3(o, n, k);
        o->H[2][IX3(o, i, o->hi[1], k)] += ch * einc3(o, n, k);
      }
  }
}

/* forward E^{n+1}: (curl H)_c = d_u H_v - d_v H_u taken backwards, graded */
static void fwd_e3(or3d *o, int n, int tf, const double *qsrc, double *efull) {
  size_t st[3];
  strides(o, st);
  const double dx = o->c.dx, dt = o->dt;
  const size_t n3 = (size_t)o->nx * o->ny * o->nz;
  for (int c = 0; c < 3; ++c) {
    int u, v, lo[3], hi[3];
    curl_axes(c, &u, &v);
    e_range(o, c, lo, hi);
    double *Ec = o->E[c], *Jc = o->J[c];
    const double *Hv = o->H[v], *Hu = o->H[u];
#pragma omp parallel for schedule(static)
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          const int idx[3] = {i, j, k};
          const size_t q = IX3(o, i, j, k);
          const double du = (Hv[q] - Hv[q - st[u]]) / dx;
          const double dv = (Hu[q] - Hu[q - st[v]]) / dx;
          double tu = du * o->ike[u][idx[u]], tv = dv * o->ike[v][idx[v]];
          if (o->ine[u][idx[u]]) { o->pE[c][u][q] = o->be[u][idx[u]] * o->pE[c][u][q] + o->ae[u][idx[u]] * du; tu += o->pE[c][u][q]; }
          if (o->ine[v][idx[v]]) { o->pE[c][v][q] = o->be[v][idx[v]] * o->pE[c][v][q] + o->ae[v][idx[v]] * dv; tv += o->pE[c][v][q]; }
          double curl = tu - tv;
          if (tf) {
            if (c == 0 && i >= o->lo[0] && i <= o->hi[0] - 1 && j >= o->lo[1] && j <= o->hi[1]) {
              if (k == o->lo[2]) curl += hinc3(o, n, o->lo[2] - 1) / dx;
              if (k == o->hi[2]) curl -= hinc3(o, n, o->hi[2]) / dx;
            }
            if (c == 2 && j >= o->lo[1] && j <= o->hi[1] && k >= o->lo[2] && k <= o->hi[2] - 1) {
              if (i == o->lo[0]) curl -= hinc3(o, n, k) / dx;
              if (i == o->hi[0]) curl += hinc3(o, n, k) / dx;
            }
          }
          if (qsrc) curl += qsrc[(size_t)c * n3 + q];
          const double e0 = Ec[q];
          if (is_drude(o, i, j, k)) {
            const coef3_t kk = drude3(o, o->rho[didx(o, i, j, k)]);
            const double e1 = kk.C1 * e0 + kk.C2 * (curl - 0.5 * (1.0 + kk.kp) * Jc[q]);
            Jc[q] = kk.kp * Jc[q] + kk.beta * (e1 + e0);
            Ec[q] = e1;
          } else {
            const double eps = is_gap(o, i, j, k) ? o->c.eps_g : o->c.eps_s;
            Ec[q] = e0 + dt / (OR_EPS0 * eps) * curl;
          }
        }
  }
  for (int c = 0; c < 3; ++c) {
    for (int gk = 0; gk < (o->mon_on ? o->gn[2] : 0); ++gk)
      for (int gj = 0; gj < o->gn[1]; ++gj)
        for (int gi = 0; gi < o->gn[0]; ++gi) {
          const int g = (gk * o->gn[1] + gj) * o->gn[0] + gi;
          const double e = o->E[c][IX3(o, o->g0[0] + gi, o->g0[1] + gj, o->g0[2] + gk)];
          o->gapE[((size_t)(n + 1) * o->ng + g) * 3 + c] = e;
          for (int kf = 0; kf < o->K; ++kf) {
            const double ph = 2.0 * M_PI * o->freqs[kf] * (n + 1) * dt;
            o->dft[(((size_t)kf * o->ng + g) * 3 + c) * 2 + 0] += dt * e * cos(ph);
            o->dft[(((size_t)kf * o->ng + g) * 3 + c) * 2 + 1] -= dt * e * sin(ph);
          }
        }
    for (int dk = 0; dk < (o->hist_on ? o->dn[2] : 0); ++dk)
      for (int dj = 0; dj < o->dn[1]; ++dj)
        for (int di = 0; di < o->dn[0]; ++di)
          o->hist[((size_t)(n - o->hist_base) * 3 + c) * o->nd + (dk * o->dn[1] + dj) * o->dn[0] + di] =
              o->E[c][IX3(o, o->d0[0] + di, o->d0[1] + dj, o->d0[2] + dk)];
    if (efull) memcpy(efull + ((size_t)n * 3 + c) * n3, o->E[c], n3 * sizeof(double));
  }
}

static double objective3(const or3d *o) {
  double F = 0.0;
  if (o->c.objective_kind == OR_OBJ_TIME_ENERGY) {
    for (size_t q = 0; q < (size_t)(o->N + 1) * o->ng * 3; ++q) F += o->gapE[q] * o->gapE[q];
    return 0.5 * o->c.eps_g * o->dt * o->c.dx * o->c.dx * o->c.dx * F;
  }
  for (int k = 0; k < o->K; ++k)
    for (int g = 0; g < o->ng * 3; ++g) {
      const double re = o->dft[((size_t)k * o->ng * 3 + g) * 2], im = o->dft[((size_t)k * o->ng * 3 + g) * 2 + 1];
      F += o->wts[k] * (re * re + im * im);
    }
  return F;
}

/* ------------------------------------------------------- checkpointing */

/* Walk the forward state in a fixed order, copying it to (save) or from
 * (load) buf: E and H whole, J over the design box, and each absorber memory
 * only where its grading is active (it is zero elsewhere).  Returns the
 * number of doubles; buf = NULL only counts. */
static size_t snap_io3(or3d *o, double *buf, int save) {
  const size_t n = (size_t)o->nx * o->ny * o->nz;
  size_t k = 0;
  for (int c = 0; c < 3; ++c)
    for (int f = 0; f < 2; ++f) {
      double *a = f ? o->H[c] : o->E[c];
      if (buf) { if (save) memcpy(buf + k, a, n * sizeof(double)); else memcpy(a, buf + k, n * sizeof(double)); }
      k += n;
    }
  for (int c = 0; c < 3; ++c) {
    if (buf && !save) memset(o->J[c], 0, n * sizeof(double));
    for (int dk = 0; dk < o->dn[2]; ++dk)
      for (int dj = 0; dj < o->dn[1]; ++dj)
        for (int di = 0; di < o->dn[0]; ++di, ++k) {
          double *v = &o->J[c][IX3(o, o->d0[0] + di, o->d0[1] + dj, o->d0[2] + dk)];
          if (buf) { if (save) buf[k] = *v; else *v = buf[k]; }
        }
  }
  for (int c = 0; c < 3; ++c)
    for (int u = 0; u < 3; ++u) {
      if (u == c) continue;
      for (int f = 0; f < 2; ++f) {
        double *a = f ? o->pH[c][u] : o->pE[c][u];
        const unsigned char *flag = f ? o->inh[u] : o->ine[u];
        if (buf && !save) memset(a, 0, n * sizeof(double));
        for (int kk = 0; kk < o->nz; ++kk)
          for (int j = 0; j < o->ny; ++j)
            for (int i = 0; i < o->nx; ++i) {
              const int idx[3] = {i, j, kk};
              if (!flag[idx[u]]) continue;
              const size_t q = IX3(o, i, j, kk);
              if (buf) { if (save) buf[k] = a[q]; else a[q] = buf[k]; }
              ++k;
            }
      }
    }
  return k;
}

/* Exchange the working state with the re-run state. */
static void swap3(or3d *o) {
  for (int c = 0; c < 3; ++c) {
    double *t;
    t = o->E[c]; o->E[c] = o->rE[c]; o->rE[c] = t;
    t = o->H[c]; o->H[c] = o->rH[c]; o->rH[c] = t;
    t = o->J[c]; o->J[c] = o->rJ[c]; o->rJ[c] = t;
    for (int u = 0; u < 3; ++u) {
      t = o->pE[c][u]; o->pE[c][u] = o->rpE[c][u]; o->rpE[c][u] = t;
      t = o->pH[c][u]; o->pH[c][u] = o->rpH[c][u]; o->rpH[c][u] = t;
    }
  }
}

/* Full history (every = 0) or `every` steps of it plus segment snapshots;
 * see or2d_set_checkpoint.  Both give identical results. */
int or3d_set_checkpoint(or3d *o, int every) {
  if (every < 0) return fail3(o, OR_EINVAL, "negative checkpoint interval");
  o->ck = (every > 0 && every < o->N) ? every : 0;
  free(o->hist); o->hist = NULL; o->hist_steps = 0;
  free(o->snap); o->snap = NULL;
  if (o->state > 1) o->state = 1;
  return OR_OK;
}

static int ensure_history3(or3d *o) {
  const int steps = o->ck ? o->ck : o->N;
  o->nseg = o->ck ? (o->N + o->ck - 1) / o->ck : 1;
  o->snap_len = o->ck ? snap_io3(o, NULL, 1) : 0;
  const double bytes = 8.0 * (3.0 * steps * o->nd + (double)o->nseg * o->snap_len);
  if (bytes > 40e9) return fail3(o, OR_ENOMEM, "design history and snapshots would exceed 40 GB");
  if (!o->hist || o->hist_steps != steps) {
    free(o->hist);
    o->hist = (double *)malloc(sizeof(double) * 3 * (size_t)steps * (o->nd > 0 ? o->nd : 1));
    o->hist_steps = o->hist ? steps : 0;
    if (!o->hist) return fail3(o, OR_ENOMEM, "out of memory (history)");
  }
  if (o->ck && !o->snap) {
    const size_t n = (size_t)o->nx * o->ny * o->nz;
    o->snap = (double *)malloc(sizeof(double) * o->snap_len * o->nseg);
    int bad = !o->snap;
    for (int c = 0; c < 3; ++c) {
      if (!o->rE[c]) o->rE[c] = calloc(n, sizeof(double));
      if (!o->rH[c]) o->rH[c] = calloc(n, sizeof(double));
      if (!o->rJ[c]) o->rJ[c] = calloc(n, sizeof(double));
      bad |= !o->rE[c] || !o->rH[c] || !o->rJ[c];
      for (int u = 0; u < 3; ++u) {
        if (u == c) continue;
        if (!o->rpE[c][u]) o->rpE[c][u] = calloc(n, sizeof(double));
        if (!o->rpH[c][u]) o->rpH[c][u] = calloc(n, sizeof(double));
        bad |= !o->rpE[c][u] || !o->rpH[c][u];
      }
    }
    if (bad) return fail3(o, OR_ENOMEM, "out of memory (snapshots)");
  }
  return OR_OK;
}

static int run_fwd3(or3d *o, int tf, const double *q, double *efull) {
  int rc = ensure_history3(o);
  if (rc) return rc;
  zero3(o);
  memset(o->dft, 0, sizeof(double) * o->K * (o->ng ? o->ng : 1) * 6);
  memset(o->gapE, 0, sizeof(double) * (size_t)(o->N + 1) * (o->ng ? o->ng : 1) * 3);
  const size_t n3 = (size_t)o->nx * o->ny * o->nz;
  o->mon_on = 1;
  o->hist_on = !o->ck;
  o->hist_base = 0;
  for (int n = 0; n < o->N; ++n) {
    if (o->ck && n % o->ck == 0) snap_io3(o, o->snap + (size_t)(n / o->ck) * o->snap_len, 1);
    fwd_h3(o, n, tf);
    fwd_e3(o, n, tf, q ? q + (size_t)n * 3 * n3 : NULL, efull);
  }
  for (int c = 0; c < 3; ++c)
    for (size_t i = 0; i < n3; ++i)
      if (!isfinite(o->E[c][i])) return fail3(o, OR_EUNSTABLE, "non-finite field");
  return OR_OK;
}

int or3d_forward(or3d *o, double *F) {
  if (o->state < 1) return fail3(o, OR_ESTATE, "forward before set_density");
  int rc = run_fwd3(o, o->tf_on, NULL, NULL);
  if (rc) return rc;
  if (F) *F = objective3(o);
  o->state = 2;
  return OR_OK;
}

static double adj_src3(const or3d *o, int m, int g, int c) {
  if (o->c.objective_kind == OR_OBJ_TIME_ENERGY)
    return o->c.eps_g * o->dt * o->c.dx * o->c.dx * o->c.dx * o->gapE[((size_t)m * o->ng + g) * 3 + c];
  double s = 0.0;
  for (int k = 0; k < o->K; ++k) {
    const double ph = 2.0 * M_PI * o->freqs[k] * m * o->dt;
    const double re = o->dft[(((size_t)k * o->ng + g) * 3 + c) * 2], im = o->dft[(((size_t)k * o->ng + g) * 3 + c) * 2 + 1];
    s += o->wts[k] * (re * cos(ph) - im * sin(ph));
  }
  return 2.0 * o->dt * s;
}

/* One adjoint step m: (1) memories of the E* grading, (2) H*, (3) memories of
 * the H* grading, (4) E*, J* and the sensitivity sums with the stored E^m. */
static void adj_step3(or3d *o, int m, const double *ssrc, double *estar) {
  size_t st[3];
  strides(o, st);
  const double cm = o->dt / OR_MU0, dx = o->c.dx, dt = o->dt;
  const int n3a[3] = {o->nx, o->ny, o->nz};
  const size_t n3 = (size_t)o->nx * o->ny * o->nz;
  /* (1) nu for E_c graded along u: nu = b^e_u nu + a^e_u E*_c at every node */
  for (int c = 0; c < 3; ++c)
    for (int u = 0; u < 3; ++u) {
      if (u == c) continue;
      double *nu = o->pE[c][u];
      const double *Ec = o->E[c];
#pragma omp parallel for schedule(static)
      for (int k = 0; k < n3a[2]; ++k)
        for (int j = 0; j < n3a[1]; ++j)
          for (int i = 0; i < n3a[0]; ++i) {
            const int idx[3] = {i, j, k};
            if (!o->ine[u][idx[u]]) continue;
            const size_t q = IX3(o, i, j, k);
            nu[q] = o->be[u][idx[u]] * nu[q] + o->ae[u][idx[u]] * Ec[q];
          }
    }
  /* (2) H*_c -= dt/mu0 [ d_u G_u(E*_v) - d_v G_v(E*_u) ],  G_u(X) = X/kappa^e_u + nu */
  for (int c = 0; c < 3; ++c) {
    int u, v, lo[3], hi[3];
    curl_axes(c, &u, &v);
    h_range(o, c, lo, hi);
    double *Hc = o->H[c];
    const double *Ev = o->E[v], *Eu = o->E[u], *nv = o->pE[v][u], *nu_ = o->pE[u][v];
#pragma omp parallel for schedule(static)
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          const int idx[3] = {i, j, k};
          const size_t q = IX3(o, i, j, k);
          const int iu1 = idx[u] + 1, iv1 = idx[v] + 1;
          const double g1 = Ev[q + st[u]] * o->ike[u][iu1] + (o->ine[u][iu1] ? nv[q + st[u]] : 0.0);
          const double g0 = Ev[q] * o->ike[u][idx[u]] + (o->ine[u][idx[u]] ? nv[q] : 0.0);
          const double h1 = Eu[q + st[v]] * o->ike[v][iv1] + (o->ine[v][iv1] ? nu_[q + st[v]] : 0.0);
          const double h0 = Eu[q] * o->ike[v][idx[v]] + (o->ine[v][idx[v]] ? nu_[q] : 0.0);
          Hc[q] -= cm * ((g1 - g0) - (h1 - h0)) / dx;
        }
  }
  /* (3) nu for H_c graded along u: nu = b^h_u nu + a^h_u H*_c */
  for (int c = 0; c < 3; ++c)
    for (int u = 0; u < 3; ++u) {
      if (u == c) continue;
      double *nu = o->pH[c][u];
      const double *Hc = o->H[c];
#pragma omp parallel for schedule(static)
      for (int k = 0; k < n3a[2]; ++k)
        for (int j = 0; j < n3a[1]; ++j)
          for (int i = 0; i < n3a[0]; ++i) {
            const int idx[3] = {i, j, k};
            if (!o->inh[u][idx[u]]) continue;
            const size_t q = IX3(o, i, j, k);
            nu[q] = o->bh[u][idx[u]] * nu[q] + o->ah[u][idx[u]] * Hc[q];
          }
    }
  /* (4) E*_c += ... [ d_u G_u(H*_v) - d_v G_v(H*_u) + s ] (backward differences) */
  for (int c = 0; c < 3; ++c) {
    int u, v, lo[3], hi[3];
    curl_axes(c, &u, &v);
    e_range(o, c, lo, hi);
    double *Ec = o->E[c], *Jc = o->J[c];
    const double *Hv = o->H[v], *Hu = o->H[u], *nv = o->pH[v][u], *nu_ = o->pH[u][v];
    const double *Em = o->hist ? o->hist + ((size_t)(m - 1 - o->hist_base) * 3 + c) * o->nd : NULL;
#pragma omp parallel for schedule(static)
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          const int idx[3] = {i, j, k};
          const size_t q = IX3(o, i, j, k);
          const int iu0 = idx[u] - 1, iv0 = idx[v] - 1;
          const double g1 = Hv[q] * o->ikh[u][idx[u]] + (o->inh[u][idx[u]] ? nv[q] : 0.0);
          const double g0 = Hv[q - st[u]] * o->ikh[u][iu0] + (o->inh[u][iu0] ? nv[q - st[u]] : 0.0);
          const double h1 = Hu[q] * o->ikh[v][idx[v]] + (o->inh[v][idx[v]] ? nu_[q] : 0.0);
          const double h0 = Hu[q - st[v]] * o->ikh[v][iv0] + (o->inh[v][iv0] ? nu_[q - st[v]] : 0.0);
          double curl = ((g1 - g0) - (h1 - h0)) / dx;
          if (ssrc) curl += ssrc[(size_t)c * n3 + q];
          else if (is_gap(o, i, j, k))
            curl += adj_src3(o, m, ((k - o->g0[2]) * o->gn[1] + (j - o->g0[1])) * o->gn[0] + (i - o->g0[0]), c);
          const double e0 = Ec[q];
          if (is_drude(o, i, j, k)) {
            const int d = didx(o, i, j, k);
            const coef3_t kk = drude3(o, o->rho[d]);
            const double e1 = kk.C1 * e0 + kk.C2 * (curl - 0.5 * (1.0 + kk.kp) * Jc[q]);
            const double j1 = kk.kp * Jc[q] + kk.beta * (e1 + e0);
            if (!ssrc) {
              o->gEps[(size_t)c * o->nd + d] += Em[d] * (e1 - e0);
              o->gSig[(size_t)c * o->nd + d] += Em[d] * (e1 + e0);
              o->gPsi[(size_t)c * o->nd + d] += Em[d] * (j1 + Jc[q]);
            }
            Ec[q] = e1;
            Jc[q] = j1;
          } else {
            const double eps = is_gap(o, i, j, k) ? o->c.eps_g : o->c.eps_s;
            Ec[q] = e0 + dt / (OR_EPS0 * eps) * curl;
          }
        }
    if (estar) memcpy(estar + ((size_t)(m - 1) * 3 + c) * n3, Ec, n3 * sizeof(double));
  }
}

int or3d_adjoint(or3d *o) {
  if (o->state < 2) return fail3(o, OR_ESTATE, "adjoint before forward");
  zero3(o);
  memset(o->gEps, 0, sizeof(double) * 3 * o->nd);
  memset(o->gSig, 0, sizeof(double) * 3 * o->nd);
  memset(o->gPsi, 0, sizeof(double) * 3 * o->nd);
  if (!o->ck) {
    o->hist_base = 0;
    for (int m = o->N; m >= 1; --m) adj_step3(o, m, NULL, NULL);
  } else {
    /* newest segment first: re-run the forward over steps [a, b) from its
     * snapshot on the second state (history only), then adjoint m = b..a+1 */
    for (int s = o->nseg - 1; s >= 0; --s) {
      const int a = s * o->ck, b = a + o->ck < o->N ? a + o->ck : o->N;
      swap3(o);
      snap_io3(o, o->snap + (size_t)s * o->snap_len, 0);
      o->mon_on = 0; o->hist_on = 1; o->hist_base = a;
      for (int n = a; n < b; ++n) {
        fwd_h3(o, n, o->tf_on);
        fwd_e3(o, n, o->tf_on, NULL, NULL);
      }
      o->mon_on = 1;
      swap3(o);
      for (int m = b; m >= a + 1; --m) adj_step3(o, m, NULL, NULL);
    }
  }
  o->state = 3;
  return OR_OK;
}

/* dF/drho per design cell (sum of the three owned edges); optional per-edge
 * partials [3][nd] of eq. (25). */
int or3d_gradient(or3d *o, double *grad, double *d_eps, double *d_psi, double *d_sig) {
  if (o->state < 3) return fail3(o, OR_ESTATE, "gradient before adjoint");
  const or_cfg *c = &o->c;
  const double psi = c->omega_p * c->omega_p, psi_s = c->psi_s_ratio * psi;
  for (int dk = 0; dk < o->dn[2]; ++dk)
    for (int dj = 0; dj < o->dn[1]; ++dj)
      for (int di = 0; di < o->dn[0]; ++di) {
        const int d = (dk * o->dn[1] + dj) * o->dn[0] + di;
        const int gap = is_gap(o, o->d0[0] + di, o->d0[1] + dj, o->d0[2] + dk);
        const coef3_t kk = drude3(o, o->rho[d]);
        double g = 0.0;
        for (int cc = 0; cc < 3; ++cc) {
          const size_t e = (size_t)cc * o->nd + d;
          double fe = 0, fp = 0, fs = 0;
          if (!gap) {
            fe = -(OR_EPS0 / o->dt) * o->gEps[e];
            fs = -0.5 * o->gSig[e];
            fp = -o->gPsi[e] / (2.0 * kk.psi);
            g += (c->eps_inf - c->eps_s) * fe + (psi - psi_s) * fp + c->sigma_max * (1.0 - 2.0 * o->rho[d]) * fs;
          }
          if (d_eps) d_eps[e] = fe;
          if (d_psi) d_psi[e] = fp;
          if (d_sig) d_sig[e] = fs;
        }
        if (grad) grad[d] = g;
      }
  return OR_OK;
}

int or3d_get_dft(const or3d *o, double *out) {
  if (o->state < 2) return OR_ESTATE;
  memcpy(out, o->dft, sizeof(double) * o->K * o->ng * 6);
  return OR_OK;
}

int or3d_get_gap_series(const or3d *o, double *out) {
  if (o->state < 2) return OR_ESTATE;
  memcpy(out, o->gapE, sizeof(double) * (size_t)(o->N + 1) * o->ng * 3);
  return OR_OK;
}

void or3d_info(const or3d *o, double *dt, double *freqs, double *wts, int32_t *tf_box) {
  if (dt) *dt = o->dt;
  if (freqs) memcpy(freqs, o->freqs, sizeof(double) * o->K);
  if (wts) memcpy(wts, o->wts, sizeof(double) * o->K);
  if (tf_box) for (int d = 0; d < 3; ++d) { tf_box[2 * d] = o->lo[d]; tf_box[2 * d + 1] = o->hi[d]; }
}

int or3d_incident_column(const or3d *o, int k, double *out) {
  if (!o->tf_on) return OR_EINVAL;
  const int p = k - o->kref;
  if (p < 0 || p >= o->L) return OR_EINVAL;
  for (int n = 0; n <= o->N; ++n) out[n] = o->einc[(size_t)n * o->L + p];
  return OR_OK;
}

/* Test hooks: extra source q ([N][3][nz][ny][nx]) in the curl bracket with the
 * plane wave off, E over the whole grid to efull ([N][3][..]); the adjoint
 * driven by s ([N][3][..], index m-1) with E* to estar. */
int or3d_forward_ext(or3d *o, const double *q, double *efull) {
  if (o->state < 1) return fail3(o, OR_ESTATE, "forward before set_density");
  return run_fwd3(o, 0, q, efull);
}

int or3d_adjoint_ext(or3d *o, const double *s, double *estar) {
  if (o->state < 1) return fail3(o, OR_ESTATE, "adjoint before set_density");
  zero3(o);
  o->hist_base = 0;
  const size_t n3 = (size_t)o->nx * o->ny * o->nz;
  for (int m = o->N; m >= 1; --m) adj_step3(o, m, s + (size_t)(m - 1) * 3 * n3, estar);
  return OR_OK;
}

/* Full state (E, H, J components, each [nz][ny][nx]) for source-free tests. */
int or3d_set_state(or3d *o, const double *const *E, const double *const *H, const double *const *J) {
  const size_t n = (size_t)o->nx * o->ny * o->nz;
  zero3(o);
  for (int c = 0; c < 3; ++c) {
    memcpy(o->E[c], E[c], n * sizeof(double));
    memcpy(o->H[c], H[c], n * sizeof(double));
    memcpy(o->J[c], J[c], n * sizeof(double));
  }
  return OR_OK;
}

int or3d_get_state(const or3d *o, double *const *E, double *const *H, double *const *J) {
  const size_t n = (size_t)o->nx * o->ny * o->nz;
  for (int c = 0; c < 3; ++c) {
    memcpy(E[c], o->E[c], n * sizeof(double));
    memcpy(H[c], o->H[c], n * sizeof(double));
    memcpy(J[c], o->J[c], n * sizeof(double));
  }
  return OR_OK;
}

int or3d_step_free(or3d *o, int k) {
  if (o->state < 1) return fail3(o, OR_ESTATE, "step before set_density");
  o->mon_on = 0;  /* monitors and history off: only the fields evolve */
  o->hist_on = 0;
  for (int s = 0; s < k; ++s) {
    fwd_h3(o, 0, 0);
    fwd_e3(o, 0, 0, NULL, NULL);
  }
  return OR_OK;
}
