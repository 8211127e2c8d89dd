/*
 * fdtd2d.c -- 2D TMz CPU oracle (FP64).  TEST INFRASTRUCTURE ONLY.
 *
 * What it computes, step by step, following the paper:
 *   * Material map, eqs. (4)-(5): on each design edge i,
 *       eps_inf_i = eps_s + rho_i (eps_inf - eps_s)
 *       psi_i     = psi_s + rho_i (psi - psi_s),   psi = omega_p^2, psi_s = r_s psi
 *       sigma_i   = rho_i (1 - rho_i) sigma_max
 *     with the collision rate gamma = gamma_mult * gamma_p.
 *   * Governing equations (10a-c): eps0 eps_inf dE/dt + J + sigma E = curl H,
 *     dJ/dt + gamma J = eps0 psi E, mu0 dH/dt = -curl E, discretized on a Yee
 *     grid (Sec. 3.2): E and J at integer steps, H at half steps; the two
 *     E/J equations are trapezoidal in time (the auxiliary-differential-equation
 *     form of the Drude model), which makes the explicit update
 *       E^{n+1} = C1 E^n + C2 [curl H^{n+1/2} - (1+kp)/2 J^n]
 *       J^{n+1} = kp J^n + beta (E^{n+1} + E^n)
 *     with kp = (1 - gamma dt/2)/(1 + gamma dt/2), beta = eps0 psi_i dt/2/(1 + gamma dt/2),
 *     D = 2 eps0 eps_inf_i + (beta + sigma_i) dt, C1 = (2 eps0 eps_inf_i - (beta+sigma_i) dt)/D,
 *     C2 = 2 dt / D.  Outside the design box the medium is the plain
 *     dielectric eps_s (eps_g in the gap).
 *   * Open boundary: convolutional PML over pml_cells next to PEC walls (the
 *     paper uses a uniaxial PML; either is a perfectly matched absorber).
 *   * Plane-wave injection: total-field/scattered-field box fed by a 1D line.
 *   * Monitors: running DFT of E over the gap at the band frequencies,
 *       Ehat_g(w_k) = dt sum_{n=1..N} E_g^n exp(-j w_k n dt),
 *     objective F = sum_k w_k sum_g |Ehat_g(w_k)|^2; or the time-domain energy
 *     of eq. (24), W = eps_g dt dx^3 / 2 sum_g sum_{n=0..N} (E_g^n)^2.
 *   * Adjoint (eq. (20) and Sec. 3.2): the same update run backwards in time
 *     on (E*, H*, J*) with E*, J* at half steps and H* at integer steps,
 *     driven by s^m = dF/dE^m at the gap, from zero terminal state.  Inside the
 *     absorber the adjoint is the exact transpose of the forward recursion.
 *   * Sensitivities, eq. (25):
 *       dF/d eps_inf_i = -(eps0/dt) sum_{m=1..N} E_i^m (E*_i^{m-1/2} - E*_i^{m+1/2})
 *       dF/d sigma_i   = -1/2      sum_{m=1..N} E_i^m (E*_i^{m-1/2} + E*_i^{m+1/2})
 *       dF/d psi_i     = -1/(2 psi_i) sum_{m=1..N} E_i^m (J*_i^{m-1/2} + J*_i^{m+1/2})
 *     and the chain rule of eq. (27) with the filter taken as identity.
 *
 * Grid: nx x ny E_z nodes, E_z(i,j) at (i dx, j dx); H_x(i,j) at (i, j+1/2);
 * H_y(i,j) at (i+1/2, j); arrays are [j][i] with i fastest.  Outer nodes are
 * PEC (E_z = 0) unless periodic_x, which wraps the x axis (used only by the
 * reflection test).  The plane wave travels along +y with E along z.
 */
#include "oracle_common.h"

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct or2d {
  or_cfg c;
  double *freqs, *wts;
  int nx, ny, N, K, nd, ng;
  double dt;
  int dx0, dy0, dnx, dny; /* design box */
  int gx0, gy0, gnx, gny; /* gap box */
  /* per-axis absorber profiles at integer (e) and half-integer (h) positions */
  double *bxe, *axe, *kxe, *bxh, *axh, *kxh, *bye, *aye, *kye, *byh, *ayh, *kyh;
  unsigned char *inx_e, *inx_h, *iny_e, *iny_h;
  /* state (forward fields, or adjoint fields during the adjoint sweep) */
  double *Ez, *Hx, *Hy, *J;
  double *pHx, *pHy, *pEx, *pEy; /* absorber memory; nu variables in the adjoint */
  /* incident line */
  int tf_on, ia, ib, ja, jb, jref, L;
  double *einc, *hinc;
  /* density, monitors, history, sensitivities */
  double *rho;
  double *dft;   /* [K][ng][2] */
  double *gapE;  /* [N+1][ng] */
  double *hist;  /* [hist_steps][nd]: E^{n+1} on design edges, slot n - hist_base */
  int hist_steps, hist_base, hist_on, mon_on;
  double *gEps, *gSig, *gPsi;
  /* segment checkpointing (ck > 0): a snapshot of the forward state at the
   * start of every ck-step segment, and a second state (the r* arrays) on
   * which the adjoint re-runs each segment to refill a ck-step history */
  int ck, nseg;
  size_t snap_len;
  double *snap;
  double *rEz, *rHx, *rHy, *rJ, *rpHx, *rpHy, *rpEx, *rpEy;
  double F;
  int state; /* 0 created, 1 density set, 2 forward done, 3 adjoint done */
  char err[256];
} or2d;

static char g_err[256];

static int fail(or2d *o, int code, const char *msg) {
  if (o) snprintf(o->err, sizeof o->err, "%s", msg);
  else snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

const char *or2d_last_error(const or2d *o) { return o ? o->err : g_err; }

static inline size_t IX(const or2d *o, int i, int j) { return (size_t)j * o->nx + i; }
static inline int in_design(const or2d *o, int i, int j) {
  return i >= o->dx0 && i < o->dx0 + o->dnx && j >= o->dy0 && j < o->dy0 + o->dny;
}
static inline int in_gap(const or2d *o, int i, int j) {
  return i >= o->gx0 && i < o->gx0 + o->gnx && j >= o->gy0 && j < o->gy0 + o->gny;
}
/* Drude edge: in the design box and not in the gap */
static inline int is_drude(const or2d *o, int i, int j) { return in_design(o, i, j) && !in_gap(o, i, j); }

/* Material coefficients of eq. (5) and the trapezoidal ADE on one design edge. */
typedef struct { double eps, psi, sig, kp, beta, C1, C2; } coef_t;

static coef_t drude_coef(const or2d *o, double rho) {
  const or_cfg *c = &o->c;
  const double psi = c->omega_p * c->omega_p;
  const double psi_s = c->psi_s_ratio * psi;
  const double gam = c->gamma_mult * c->gamma_p;
  const double dt = o->dt;
  coef_t k;
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

static double eps_plain(const or2d *o, int i, int j) { return in_gap(o, i, j) ? o->c.eps_g : o->c.eps_s; }

void or2d_destroy(or2d *o) {
  if (!o) return;
  double **ptrs[] = {&o->freqs, &o->wts, &o->bxe, &o->axe, &o->kxe, &o->bxh, &o->axh, &o->kxh,
                     &o->bye, &o->aye, &o->kye, &o->byh, &o->ayh, &o->kyh, &o->Ez, &o->Hx, &o->Hy,
                     &o->J, &o->pHx, &o->pHy, &o->pEx, &o->pEy, &o->einc, &o->hinc, &o->rho,
                     &o->dft, &o->gapE, &o->hist, &o->gEps, &o->gSig, &o->gPsi, &o->snap,
                     &o->rEz, &o->rHx, &o->rHy, &o->rJ, &o->rpHx, &o->rpHy, &o->rpEx, &o->rpEy};
  for (size_t k = 0; k < sizeof ptrs / sizeof ptrs[0]; ++k) free(*ptrs[k]);
  free(o->inx_e); free(o->inx_h); free(o->iny_e); free(o->iny_h);
  free(o);
}

static int box_ok(int lo, int n, int a, int b) { return n >= 1 && lo >= a && lo + n - 1 <= b; }

int or2d_create(const or_cfg *cfg, or2d **out) {
  *out = NULL;
  if (!cfg) return fail(NULL, OR_EINVAL, "null config");
  or_cfg c = *cfg;
  if (c.dims != 2) return fail(NULL, OR_EINVAL, "dims must be 2");
  if ((c.periodic_x ? c.nx < 2 : c.nx < 8) || c.ny < 8) return fail(NULL, OR_EINVAL, "grid too small");
  if (c.n_steps < 1) return fail(NULL, OR_EINVAL, "n_steps < 1");
  if (!(c.dx > 0)) return fail(NULL, OR_EINVAL, "dx <= 0");
  if (!(c.courant > 0) || c.courant >= 1.0 / sqrt(2.0))
    return fail(NULL, OR_EINVAL, "Courant number outside (0, 1/sqrt(2))");
  if (c.n_freq < 1) return fail(NULL, OR_EINVAL, "n_freq < 1");
  if (!(c.eps_s > 0) || !(c.eps_g > 0) || !(c.eps_inf > 0)) return fail(NULL, OR_EINVAL, "permittivity <= 0");
  if (c.psi_s_ratio < 0 || c.sigma_max < 0 || c.gamma_mult < 0) return fail(NULL, OR_EINVAL, "negative material parameter");
  or2d *o = (or2d *)calloc(1, sizeof(or2d));
  if (!o) return fail(NULL, OR_ENOMEM, "out of memory");
  o->c = c;
  o->nx = c.nx; o->ny = c.ny; o->N = c.n_steps; o->K = c.n_freq;
  o->dt = c.courant * c.dx / OR_C0;
  o->dx0 = c.design_lo[0]; o->dy0 = c.design_lo[1]; o->dnx = c.design_n[0]; o->dny = c.design_n[1];
  o->gx0 = c.gap_lo[0]; o->gy0 = c.gap_lo[1]; o->gnx = c.gap_n[0]; o->gny = c.gap_n[1];
  o->nd = o->dnx * o->dny;
  o->ng = o->gnx * o->gny;
  const int P = c.pml_cells, m = c.tfsf_margin;
  /* total-field region (inclusive node ranges) */
  o->tf_on = (c.source_kind != OR_SRC_NONE);
  if (c.periodic_x) { o->ia = 0; o->ib = c.nx - 1; }
  else { o->ia = P + m; o->ib = c.nx - 1 - P - m; }
  o->ja = P + m; o->jb = c.ny - 1 - P - m;
  int ok = 1;
  /* boxes must avoid the absorber and the walls; with the plane wave on they
   * must also sit strictly inside the total-field region, off its lines.  An
   * empty gap (zero extent) is allowed: no monitor, F = 0. */
  int xlo, xhi, ylo, yhi;
  if (o->tf_on) {
    if (o->ja < 3 || o->jb - o->ja < 2) ok = 0;
    if (!c.periodic_x && (o->ia < 2 || o->ib - o->ia < 2)) ok = 0;
    xlo = c.periodic_x ? 0 : o->ia + 1; xhi = c.periodic_x ? c.nx - 1 : o->ib - 1;
    ylo = o->ja + 1; yhi = o->jb - 1;
  } else {
    xlo = c.periodic_x ? 0 : P + 1; xhi = c.periodic_x ? c.nx - 1 : c.nx - 2 - P;
    ylo = P + 1; yhi = c.ny - 2 - P;
  }
  if (!box_ok(o->dx0, o->dnx, xlo, xhi) || !box_ok(o->dy0, o->dny, ylo, yhi)) ok = 0;
  if (o->ng > 0 && (!box_ok(o->gx0, o->gnx, xlo, xhi) || !box_ok(o->gy0, o->gny, ylo, yhi))) ok = 0;
  if (o->gnx < 0 || o->gny < 0) ok = 0;
  if (!ok) { or2d_destroy(o); return fail(NULL, OR_EINVAL, "design/gap boxes must lie inside the interior (and the total-field region)"); }

  const size_t n2 = (size_t)c.nx * c.ny;
  o->freqs = (double *)malloc(sizeof(double) * o->K);
  o->wts = (double *)malloc(sizeof(double) * o->K);
  double **ax1[] = {&o->bxe, &o->axe, &o->kxe, &o->bxh, &o->axh, &o->kxh};
  double **ay1[] = {&o->bye, &o->aye, &o->kye, &o->byh, &o->ayh, &o->kyh};
  for (int k = 0; k < 6; ++k) { *ax1[k] = (double *)malloc(sizeof(double) * c.nx); *ay1[k] = (double *)malloc(sizeof(double) * c.ny); }
  o->inx_e = (unsigned char *)malloc(c.nx); o->inx_h = (unsigned char *)malloc(c.nx);
  o->iny_e = (unsigned char *)malloc(c.ny); o->iny_h = (unsigned char *)malloc(c.ny);
  double **fld[] = {&o->Ez, &o->Hx, &o->Hy, &o->J, &o->pHx, &o->pHy, &o->pEx, &o->pEy};
  for (int k = 0; k < 8; ++k) *fld[k] = (double *)calloc(n2, sizeof(double));
  o->rho = (double *)calloc((size_t)o->nd, sizeof(double));
  o->dft = (double *)calloc((size_t)o->K * (o->ng > 0 ? o->ng : 1) * 2, sizeof(double));
  o->gapE = (double *)calloc((size_t)(o->N + 1) * (o->ng > 0 ? o->ng : 1), sizeof(double));
  o->gEps = (double *)calloc((size_t)o->nd, sizeof(double));
  o->gSig = (double *)calloc((size_t)o->nd, sizeof(double));
  o->gPsi = (double *)calloc((size_t)o->nd, sizeof(double));
  if (!o->freqs || !o->wts || !o->Ez || !o->Hx || !o->Hy || !o->J || !o->pHx || !o->pHy || !o->pEx ||
      !o->pEy || !o->rho || !o->dft || !o->gapE || !o->gEps || !o->gSig || !o->gPsi ||
      !o->bxe || !o->kyh || !o->inx_e || !o->iny_h) {
    or2d_destroy(o);
    return fail(NULL, OR_ENOMEM, "out of memory");
  }
  if (or_freqs_weights(&c, o->dt, o->freqs, o->wts)) { or2d_destroy(o); return fail(NULL, OR_EINVAL, "zero source spectrum at a band frequency"); }
  o->c.freqs_hz = NULL;
  const int Px = c.periodic_x ? 0 : P;
  for (int i = 0; i < c.nx; ++i) {
    o->inx_e[i] = (unsigned char)or_pml_profile(&c, o->dt, c.nx, Px, (double)i, &o->bxe[i], &o->axe[i], &o->kxe[i]);
    o->inx_h[i] = (unsigned char)or_pml_profile(&c, o->dt, c.nx, Px, i + 0.5, &o->bxh[i], &o->axh[i], &o->kxh[i]);
  }
  for (int j = 0; j < c.ny; ++j) {
    o->iny_e[j] = (unsigned char)or_pml_profile(&c, o->dt, c.ny, P, (double)j, &o->bye[j], &o->aye[j], &o->kye[j]);
    o->iny_h[j] = (unsigned char)or_pml_profile(&c, o->dt, c.ny, P, j + 0.5, &o->byh[j], &o->ayh[j], &o->kyh[j]);
  }
  /* incident line: node p <-> row j = jref + p, starting two rows before the box */
  o->jref = o->ja - 2;
  o->L = o->jb + 2 - o->jref + 1;
  if (o->tf_on) {
    if (or_incident_line(&c, o->dt, o->L, o->N, &o->einc, &o->hinc)) { or2d_destroy(o); return fail(NULL, OR_ENOMEM, "out of memory"); }
  }
  o->state = 0;
  *out = o;
  return OR_OK;
}

int or2d_set_density(or2d *o, const double *rho) {
  for (int d = 0; d < o->nd; ++d)
    if (!(rho[d] >= 0.0 && rho[d] <= 1.0)) return fail(o, OR_EINVAL, "density outside [0,1] or NaN");
  memcpy(o->rho, rho, sizeof(double) * o->nd);
  o->state = 1;
  return OR_OK;
}

static void zero_state(or2d *o) {
  const size_t n2 = (size_t)o->nx * o->ny;
  double *f[] = {o->Ez, o->Hx, o->Hy, o->J, o->pHx, o->pHy, o->pEx, o->pEy};
  for (int k = 0; k < 8; ++k) memset(f[k], 0, n2 * sizeof(double));
}

/* ---------------------------------------------------------------- forward */

/* H^{n+1/2} from H^{n-1/2} and E^n (eq. 10c), with absorber memory and the
 * scattered-field corrections that use the incident E at step n. */
static void fwd_h(or2d *o, int n, int tf) {
  const int nx = o->nx, ny = o->ny, per = o->c.periodic_x;
  const double dx = o->c.dx, cm = o->dt / OR_MU0;
  double *Ez = o->Ez, *Hx = o->Hx, *Hy = o->Hy;
  const int i_lo = per ? 0 : 1, i_hi = per ? nx - 1 : nx - 2;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny - 1; ++j)
    for (int i = i_lo; i <= i_hi; ++i) {
      const size_t q = IX(o, i, j);
      const double dEy = (Ez[IX(o, i, j + 1)] - Ez[q]) / dx;
      double extra = 0.0;
      if (o->iny_h[j]) { o->pHx[q] = o->byh[j] * o->pHx[q] + o->ayh[j] * dEy; extra = o->pHx[q]; }
      Hx[q] -= cm * (dEy / o->kyh[j] + extra);
    }
#pragma omp parallel for schedule(static)
  for (int j = 1; j < ny - 1; ++j)
    for (int i = 0; i < (per ? nx : nx - 1); ++i) {
      const size_t q = IX(o, i, j);
      const int ip = (i + 1) % nx;
      const double dEx = (Ez[IX(o, ip, j)] - Ez[q]) / dx;
      double extra = 0.0;
      if (o->inx_h[i]) { o->pHy[q] = o->bxh[i] * o->pHy[q] + o->axh[i] * dEx; extra = o->pHy[q]; }
      Hy[q] += cm * (dEx / o->kxh[i] + extra);
    }
  if (tf) {
    const double c = o->dt / (OR_MU0 * dx);
    const double *e = o->einc + (size_t)n * o->L;
    for (int i = o->ia; i <= o->ib; ++i) {
      Hx[IX(o, i, o->ja - 1)] += c * e[o->ja - o->jref];
      Hx[IX(o, i, o->jb)] -= c * e[o->jb - o->jref];
    }
    if (!per)
      for (int j = o->ja; j <= o->jb; ++j) {
        Hy[IX(o, o->ia - 1, j)] -= c * e[j - o->jref];
        Hy[IX(o, o->ib, j)] += c * e[j - o->jref];
      }
  }
}

/* curl H at E node (i,j) including absorber memory update (forward). */
static inline double fwd_curl(or2d *o, int i, int j) {
  const int nx = o->nx;
  const int im = (i - 1 + nx) % nx;
  const size_t q = IX(o, i, j);
  const double dx = o->c.dx;
  const double dHy = (o->Hy[q] - o->Hy[IX(o, im, j)]) / dx;
  const double dHx = (o->Hx[q] - o->Hx[IX(o, i, j - 1)]) / dx;
  double cx = dHy / o->kxe[i], cy = dHx / o->kye[j];
  if (o->inx_e[i]) { o->pEx[q] = o->bxe[i] * o->pEx[q] + o->axe[i] * dHy; cx += o->pEx[q]; }
  if (o->iny_e[j]) { o->pEy[q] = o->bye[j] * o->pEy[q] + o->aye[j] * dHx; cy += o->pEy[q]; }
  return cx - cy;
}

/* E^{n+1}, J^{n+1} from E^n, J^n, H^{n+1/2} (eqs. 10a-b); q = optional extra
 * source in the curl bracket ([ny][nx] for this step); then monitors. */
static void fwd_e(or2d *o, int n, int tf, const double *qsrc, double *efull_out) {
  const int nx = o->nx, ny = o->ny, per = o->c.periodic_x;
  const double dt = o->dt, dx = o->c.dx;
  const int i_lo = per ? 0 : 1, i_hi = per ? nx - 1 : nx - 2;
  const double *hrow = tf ? o->hinc + (size_t)n * o->L : NULL;
#pragma omp parallel for schedule(static)
  for (int j = 1; j < ny - 1; ++j)
    for (int i = i_lo; i <= i_hi; ++i) {
      const size_t q = IX(o, i, j);
      double curl = fwd_curl(o, i, j);
      if (tf && i >= o->ia && i <= o->ib) {
        if (j == o->ja) curl += hrow[o->ja - 1 - o->jref] / dx;
        if (j == o->jb) curl -= hrow[o->jb - o->jref] / dx;
      }
      if (qsrc) curl += qsrc[q];
      const double e0 = o->Ez[q];
      if (is_drude(o, i, j)) {
        const int d = (j - o->dy0) * o->dnx + (i - o->dx0);
        const coef_t k = drude_coef(o, o->rho[d]);
        const double e1 = k.C1 * e0 + k.C2 * (curl - 0.5 * (1.0 + k.kp) * o->J[q]);
        o->J[q] = k.kp * o->J[q] + k.beta * (e1 + e0);
        o->Ez[q] = e1;
      } else {
        o->Ez[q] = e0 + dt / (OR_EPS0 * eps_plain(o, i, j)) * curl;
      }
    }
  /* monitors: gap time series and running DFT at time (n+1) dt; design history */
  for (int gj = 0; gj < (o->mon_on ? o->gny : 0); ++gj)
    for (int gi = 0; gi < o->gnx; ++gi) {
      const int g = gj * o->gnx + gi;
      const double e = o->Ez[IX(o, o->gx0 + gi, o->gy0 + gj)];
      o->gapE[(size_t)(n + 1) * o->ng + g] = e;
      for (int k = 0; k < o->K; ++k) {
        const double ph = 2.0 * M_PI * o->freqs[k] * (n + 1) * dt;
        o->dft[((size_t)k * o->ng + g) * 2 + 0] += dt * e * cos(ph);
        o->dft[((size_t)k * o->ng + g) * 2 + 1] -= dt * e * sin(ph);
      }
    }
  for (int dj = 0; dj < (o->hist_on ? o->dny : 0); ++dj)
    for (int di = 0; di < o->dnx; ++di)
      o->hist[(size_t)(n - o->hist_base) * o->nd + dj * o->dnx + di] = o->Ez[IX(o, o->dx0 + di, o->dy0 + dj)];
  if (efull_out) memcpy(efull_out + (size_t)n * nx * ny, o->Ez, sizeof(double) * nx * ny);
}

static double objective_from_monitors(const or2d *o) {
  double F = 0.0;
  if (o->c.objective_kind == OR_OBJ_TIME_ENERGY) {
    for (int n = 0; n <= o->N; ++n)
      for (int g = 0; g < o->ng; ++g) { const double e = o->gapE[(size_t)n * o->ng + g]; F += e * e; }
    return 0.5 * o->c.eps_g * o->dt * o->c.dx * o->c.dx * o->c.dx * F;
  }
  for (int k = 0; k < o->K; ++k)
    for (int g = 0; g < o->ng; ++g) {
      const double re = o->dft[((size_t)k * o->ng + g) * 2], im = o->dft[((size_t)k * o->ng + g) * 2 + 1];
      F += o->wts[k] * (re * re + im * im);
    }
  return F;
}

/* ------------------------------------------------------- checkpointing */

/* Walk the forward state in a fixed order, copying it to (save) or from
 * (load) buf: E_z, H_x, H_y whole, J over the design box, and each absorber
 * memory only on the rows/columns where its grading is active (it is zero
 * elsewhere).  Returns the number of doubles; buf = NULL only counts. */
static size_t snap_io(or2d *o, double *buf, int save) {
  const int nx = o->nx, ny = o->ny;
  const size_t n2 = (size_t)nx * ny;
  size_t k = 0;
  double *whole[3] = {o->Ez, o->Hx, o->Hy};
  for (int f = 0; f < 3; ++f) {
    if (buf) { if (save) memcpy(buf + k, whole[f], n2 * sizeof(double)); else memcpy(whole[f], buf + k, n2 * sizeof(double)); }
    k += n2;
  }
  if (buf && !save) memset(o->J, 0, n2 * sizeof(double));
  for (int dj = 0; dj < o->dny; ++dj)
    for (int di = 0; di < o->dnx; ++di, ++k) {
      double *v = &o->J[IX(o, o->dx0 + di, o->dy0 + dj)];
      if (buf) { if (save) buf[k] = *v; else *v = buf[k]; }
    }
  /* memory arrays and the flag that marks where each one is updated */
  double *mem[4] = {o->pHx, o->pHy, o->pEx, o->pEy};
  for (int f = 0; f < 4; ++f) {
    if (buf && !save) memset(mem[f], 0, n2 * sizeof(double));
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int on = f == 0 ? o->iny_h[j] : f == 1 ? o->inx_h[i] : f == 2 ? o->inx_e[i] : o->iny_e[j];
        if (!on) continue;
        if (buf) { if (save) buf[k] = mem[f][IX(o, i, j)]; else mem[f][IX(o, i, j)] = buf[k]; }
        ++k;
      }
  }
  return k;
}

/* Exchange the working state with the re-run state. */
static void swap_state(or2d *o) {
  double **a[8] = {&o->Ez, &o->Hx, &o->Hy, &o->J, &o->pHx, &o->pHy, &o->pEx, &o->pEy};
  double **b[8] = {&o->rEz, &o->rHx, &o->rHy, &o->rJ, &o->rpHx, &o->rpHy, &o->rpEx, &o->rpEy};
  for (int k = 0; k < 8; ++k) { double *t = *a[k]; *a[k] = *b[k]; *b[k] = t; }
}

/* Store E on the design edges for every step (every = 0), or only `every`
 * steps of it plus a snapshot of the state at the start of every segment of
 * `every` steps; the adjoint then re-runs each segment from its snapshot
 * before the adjoint steps that read it.  Both give identical results. */
int or2d_set_checkpoint(or2d *o, int every) {
  if (every < 0) return fail(o, OR_EINVAL, "negative checkpoint interval");
  o->ck = (every > 0 && every < o->N) ? every : 0;
  free(o->hist); o->hist = NULL; o->hist_steps = 0;
  free(o->snap); o->snap = NULL;
  if (o->state > 1) o->state = 1;
  return OR_OK;
}

/* Allocate the history (and, with checkpoints, the snapshots and the
 * re-run state) for the current checkpoint interval. */
static int ensure_history(or2d *o) {
  const int steps = o->ck ? o->ck : o->N;
  o->nseg = o->ck ? (o->N + o->ck - 1) / o->ck : 1;
  o->snap_len = o->ck ? snap_io(o, NULL, 1) : 0;
  const double bytes = 8.0 * ((double)steps * o->nd + (double)o->nseg * o->snap_len);
  if (bytes > 40e9) return fail(o, OR_ENOMEM, "design history and snapshots would exceed 40 GB");
  if (!o->hist || o->hist_steps != steps) {
    free(o->hist);
    o->hist = (double *)malloc(sizeof(double) * (size_t)steps * (o->nd > 0 ? o->nd : 1));
    o->hist_steps = o->hist ? steps : 0;
    if (!o->hist) return fail(o, OR_ENOMEM, "out of memory (history)");
  }
  if (o->ck && !o->snap) {
    const size_t n2 = (size_t)o->nx * o->ny;
    o->snap = (double *)malloc(sizeof(double) * o->snap_len * o->nseg);
    double **r[8] = {&o->rEz, &o->rHx, &o->rHy, &o->rJ, &o->rpHx, &o->rpHy, &o->rpEx, &o->rpEy};
    for (int k = 0; k < 8; ++k) if (!*r[k]) *r[k] = (double *)calloc(n2, sizeof(double));
    if (!o->snap || !o->rEz || !o->rHx || !o->rHy || !o->rJ || !o->rpHx || !o->rpHy || !o->rpEx || !o->rpEy)
      return fail(o, OR_ENOMEM, "out of memory (snapshots)");
  }
  return OR_OK;
}

static int run_forward(or2d *o, int tf, const double *qsrc, double *efull_out) {
  int rc = ensure_history(o);
  if (rc) return rc;
  zero_state(o);
  memset(o->dft, 0, sizeof(double) * o->K * o->ng * 2);
  memset(o->gapE, 0, sizeof(double) * (size_t)(o->N + 1) * o->ng);
  o->mon_on = 1;
  o->hist_on = !o->ck;
  o->hist_base = 0;
  for (int n = 0; n < o->N; ++n) {
    if (o->ck && n % o->ck == 0) snap_io(o, o->snap + (size_t)(n / o->ck) * o->snap_len, 1);
    fwd_h(o, n, tf);
    fwd_e(o, n, tf, qsrc ? qsrc + (size_t)n * o->nx * o->ny : NULL, efull_out);
  }
  for (size_t q = 0; q < (size_t)o->nx * o->ny; ++q)
    if (!isfinite(o->Ez[q])) return fail(o, OR_EUNSTABLE, "non-finite field");
  return OR_OK;
}

int or2d_forward(or2d *o, double *F_out) {
  if (o->state < 1) return fail(o, OR_ESTATE, "forward before set_density");
  int rc = run_forward(o, o->tf_on, NULL, NULL);
  if (rc) return rc;
  o->F = objective_from_monitors(o);
  if (F_out) *F_out = o->F;
  o->state = 2;
  return OR_OK;
}

/* ---------------------------------------------------------------- adjoint */

/* Adjoint source s^m = dF/dE_g^m at the gap. */
static double adj_source(const or2d *o, int m, int g) {
  if (o->c.objective_kind == OR_OBJ_TIME_ENERGY)
    return o->c.eps_g * o->dt * o->c.dx * o->c.dx * o->c.dx * o->gapE[(size_t)m * o->ng + g];
  double s = 0.0;
  for (int k = 0; k < o->K; ++k) {
    const double ph = 2.0 * M_PI * o->freqs[k] * m * o->dt;
    const double re = o->dft[((size_t)k * o->ng + g) * 2], im = o->dft[((size_t)k * o->ng + g) * 2 + 1];
    s += o->wts[k] * (re * cos(ph) - im * sin(ph));
  }
  return 2.0 * o->dt * s;
}

/* One adjoint step m (m = N..1): state holds E*^{m+1/2}, J*^{m+1/2},
 * H*^{m+1} and the absorber memories; leaves E*^{m-1/2}, J*^{m-1/2}, H*^m.
 * ssrc: optional full-grid source for this m; otherwise the objective's
 * gap source.  Sensitivity sums use the stored forward E^m. */
static void adj_step(or2d *o, int m, const double *ssrc, double *estar_out) {
  const int nx = o->nx, ny = o->ny, per = o->c.periodic_x;
  const double dt = o->dt, dx = o->c.dx, cm = dt / OR_MU0;
  double *Es = o->Ez, *Hx = o->Hx, *Hy = o->Hy, *Js = o->J;
  double *nEx = o->pEx, *nEy = o->pEy, *nHx = o->pHx, *nHy = o->pHy;
  const int i_lo = per ? 0 : 1, i_hi = per ? nx - 1 : nx - 2;
  /* (1) transposed absorber memory at E nodes, driven by E* itself */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t q = IX(o, i, j);
      if (o->inx_e[i]) nEx[q] = o->bxe[i] * nEx[q] + o->axe[i] * Es[q];
      if (o->iny_e[j]) nEy[q] = o->bye[j] * nEy[q] + o->aye[j] * Es[q];
    }
  /* (2) H*^m: the forward curl-E update applied to the graded E* */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny - 1; ++j)
    for (int i = i_lo; i <= i_hi; ++i) {
      const size_t q = IX(o, i, j), qu = IX(o, i, j + 1);
      const double gu = Es[qu] / o->kye[j + 1] + nEy[qu];
      const double g0 = Es[q] / o->kye[j] + nEy[q];
      Hx[q] -= cm * (gu - g0) / dx;
    }
#pragma omp parallel for schedule(static)
  for (int j = 1; j < ny - 1; ++j)
    for (int i = 0; i < (per ? nx : nx - 1); ++i) {
      const int ip = (i + 1) % nx;
      const size_t q = IX(o, i, j), qr = IX(o, ip, j);
      const double gr = Es[qr] / o->kxe[ip] + nEx[qr];
      const double g0 = Es[q] / o->kxe[i] + nEx[q];
      Hy[q] += cm * (gr - g0) / dx;
    }
  /* (3) transposed absorber memory at H positions, driven by H* */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t q = IX(o, i, j);
      if (o->iny_h[j]) nHx[q] = o->byh[j] * nHx[q] + o->ayh[j] * Hx[q];
      if (o->inx_h[i]) nHy[q] = o->bxh[i] * nHy[q] + o->axh[i] * Hy[q];
    }
  /* (4) E*^{m-1/2}, J*^{m-1/2}; sensitivity sums */
  const double *Em = o->hist ? o->hist + (size_t)(m - 1 - o->hist_base) * o->nd : NULL;
#pragma omp parallel for schedule(static)
  for (int j = 1; j < ny - 1; ++j)
    for (int i = i_lo; i <= i_hi; ++i) {
      const size_t q = IX(o, i, j);
      const int im = (i - 1 + nx) % nx;
      const size_t ql = IX(o, im, j), qd = IX(o, i, j - 1);
      const double cx = ((Hy[q] / o->kxh[i] + nHy[q]) - (Hy[ql] / o->kxh[im] + nHy[ql])) / dx;
      const double cy = ((Hx[q] / o->kyh[j] + nHx[q]) - (Hx[qd] / o->kyh[j - 1] + nHx[qd])) / dx;
      double curl = cx - cy;
      if (ssrc) curl += ssrc[q];
      else if (in_gap(o, i, j)) curl += adj_source(o, m, (j - o->gy0) * o->gnx + (i - o->gx0));
      const double e0 = Es[q];
      if (is_drude(o, i, j)) {
        const int d = (j - o->dy0) * o->dnx + (i - o->dx0);
        const coef_t k = drude_coef(o, o->rho[d]);
        const double e1 = k.C1 * e0 + k.C2 * (curl - 0.5 * (1.0 + k.kp) * Js[q]);
        const double j1 = k.kp * Js[q] + k.beta * (e1 + e0);
        if (!ssrc) {
          o->gEps[d] += Em[d] * (e1 - e0);
          o->gSig[d] += Em[d] * (e1 + e0);
          o->gPsi[d] += Em[d] * (j1 + Js[q]);
        }
        Es[q] = e1;
        Js[q] = j1;
      } else {
        Es[q] = e0 + dt / (OR_EPS0 * eps_plain(o, i, j)) * curl;
      }
    }
  if (estar_out) memcpy(estar_out + (size_t)(m - 1) * nx * ny, Es, sizeof(double) * nx * ny);
}

int or2d_adjoint(or2d *o) {
  if (o->state < 2) return fail(o, OR_ESTATE, "adjoint before forward");
  zero_state(o);
  memset(o->gEps, 0, sizeof(double) * o->nd);
  memset(o->gSig, 0, sizeof(double) * o->nd);
  memset(o->gPsi, 0, sizeof(double) * o->nd);
  if (!o->ck) {
    o->hist_base = 0;
    for (int m = o->N; m >= 1; --m) adj_step(o, m, NULL, NULL);
  } else {
    /* newest segment first: re-run the forward over steps [a, b) from the
     * snapshot on the second state (history only, monitors off), then the
     * adjoint steps m = b .. a+1 that read it */
    for (int s = o->nseg - 1; s >= 0; --s) {
      const int a = s * o->ck, b = a + o->ck < o->N ? a + o->ck : o->N;
      swap_state(o);
      snap_io(o, o->snap + (size_t)s * o->snap_len, 0);
      o->mon_on = 0; o->hist_on = 1; o->hist_base = a;
      for (int n = a; n < b; ++n) {
        fwd_h(o, n, o->tf_on);
        fwd_e(o, n, o->tf_on, NULL, NULL);
      }
      o->mon_on = 1;
      swap_state(o);
      for (int m = b; m >= a + 1; --m) adj_step(o, m, NULL, NULL);
    }
  }
  o->state = 3;
  return OR_OK;
}

/* dF/drho per design cell ([y][x] over the design box); optional partials
 * dF/deps_inf_i, dF/dpsi_i, dF/dsigma_i (eq. 25). */
int or2d_gradient(or2d *o, double *grad, double *d_eps, double *d_psi, double *d_sig) {
  if (o->state < 3) return fail(o, OR_ESTATE, "gradient before adjoint");
  const or_cfg *c = &o->c;
  const double psi = c->omega_p * c->omega_p, psi_s = c->psi_s_ratio * psi;
  for (int dj = 0; dj < o->dny; ++dj)
    for (int di = 0; di < o->dnx; ++di) {
      const int d = dj * o->dnx + di;
      const int i = o->dx0 + di, j = o->dy0 + dj;
      double fe = 0, fp = 0, fs = 0, g = 0;
      if (!in_gap(o, i, j)) {
        const coef_t k = drude_coef(o, o->rho[d]);
        fe = -(OR_EPS0 / o->dt) * o->gEps[d];
        fs = -0.5 * o->gSig[d];
        fp = -o->gPsi[d] / (2.0 * k.psi);
        g = (c->eps_inf - c->eps_s) * fe + (psi - psi_s) * fp + c->sigma_max * (1.0 - 2.0 * o->rho[d]) * fs;
      }
      if (grad) grad[d] = g;
      if (d_eps) d_eps[d] = fe;
      if (d_psi) d_psi[d] = fp;
      if (d_sig) d_sig[d] = fs;
    }
  return OR_OK;
}

int or2d_get_dft(const or2d *o, double *out) {
  if (o->state < 2) return OR_ESTATE;
  memcpy(out, o->dft, sizeof(double) * o->K * o->ng * 2);
  return OR_OK;
}

int or2d_get_gap_series(const or2d *o, double *out) {
  if (o->state < 2) return OR_ESTATE;
  memcpy(out, o->gapE, sizeof(double) * (size_t)(o->N + 1) * o->ng);
  return OR_OK;
}

void or2d_info(const or2d *o, double *dt, double *freqs, double *wts, int32_t *tf_box) {
  if (dt) *dt = o->dt;
  if (freqs) memcpy(freqs, o->freqs, sizeof(double) * o->K);
  if (wts) memcpy(wts, o->wts, sizeof(double) * o->K);
  if (tf_box) { tf_box[0] = o->ia; tf_box[1] = o->ib; tf_box[2] = o->ja; tf_box[3] = o->jb; }
}

/* Incident E along the propagation axis at row j for steps 0..N (test use). */
int or2d_incident_column(const or2d *o, int j, double *out) {
  if (!o->tf_on) return OR_EINVAL;
  const int p = j - o->jref;
  if (p < 0 || p >= o->L) return OR_EINVAL;
  for (int n = 0; n <= o->N; ++n) out[n] = o->einc[(size_t)n * o->L + p];
  return OR_OK;
}

/* ------------------------------------------------------------ test hooks */

/* Forward with the plane wave off and an extra source q^{n+1} ([N][ny][nx])
 * in the curl bracket; E^{n+1} over the whole grid to efull ([N][ny][nx]). */
int or2d_forward_ext(or2d *o, const double *q, double *efull) {
  if (o->state < 1) return fail(o, OR_ESTATE, "forward before set_density");
  return run_forward(o, 0, q, efull);
}

/* Adjoint driven by s^m ([N][ny][nx], index m-1) instead of the objective;
 * E*^{m-1/2} over the whole grid to estar ([N][ny][nx], index m-1). */
int or2d_adjoint_ext(or2d *o, const double *s, double *estar) {
  if (o->state < 1) return fail(o, OR_ESTATE, "adjoint before set_density");
  zero_state(o);
  o->hist_base = 0;
  for (int m = o->N; m >= 1; --m) adj_step(o, m, s + (size_t)(m - 1) * o->nx * o->ny, estar);
  return OR_OK;
}

/* State access for source-free evolution tests (plane wave off, monitors
 * still run).  Arrays are full [ny][nx]; absorber memories are cleared. */
int or2d_set_state(or2d *o, const double *Ez, const double *Hx, const double *Hy, const double *J) {
  const size_t n2 = (size_t)o->nx * o->ny;
  zero_state(o);
  memcpy(o->Ez, Ez, n2 * sizeof(double));
  memcpy(o->Hx, Hx, n2 * sizeof(double));
  memcpy(o->Hy, Hy, n2 * sizeof(double));
  memcpy(o->J, J, n2 * sizeof(double));
  return OR_OK;
}

int or2d_get_state(const or2d *o, double *Ez, double *Hx, double *Hy, double *J) {
  const size_t n2 = (size_t)o->nx * o->ny;
  memcpy(Ez, o->Ez, n2 * sizeof(double));
  memcpy(Hx, o->Hx, n2 * sizeof(double));
  memcpy(Hy, o->Hy, n2 * sizeof(double));
  memcpy(J, o->J, n2 * sizeof(double));
  return OR_OK;
}

int or2d_step_free(or2d *o, int k) {
  if (o->state < 1) return fail(o, OR_ESTATE, "step before set_density");
  /* monitors and history are off: only the fields evolve */
  o->mon_on = 0;
  o->hist_on = 0;
  for (int s = 0; s < k; ++s) {
    fwd_h(o, 0, 0);
    fwd_e(o, 0, 0, NULL, NULL);
  }
  return OR_OK;
}

int or2d_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
