/*
 * fdtd2d_te.c -- 2D TEz CPU oracle (FP64): E in the plane (E_x, E_y), H along
 * z.  TEST INFRASTRUCTURE ONLY.
 *
 * This is the paper's plasmonic 2D case (Sec. 4.1: in-plane E, the plane wave
 * travelling along +y with E along x), the polarization in which the metal
 * carries surface plasmons.  The same equations and discretization as the
 * TMz oracle (fdtd2d.c):
 *   * eqs. (4)-(5) map the density to eps_inf_i, psi_i, sigma_i on each
 *     design edge; eqs. (10a-c) with the trapezoidal Drude ADE give
 *       E^{n+1} = C1 E^n + C2 [curl H^{n+1/2} - (1+kp)/2 J^n]
 *       J^{n+1} = kp J^n + beta (E^{n+1} + E^n)
 *     on every E_x and E_y edge of the design box (Sec. 3.2: each design
 *     variable belongs to one Yee edge);
 *   * convolutional PML next to PEC walls; total-field/scattered-field
 *     injection fed by a 1D line;
 *   * monitors: running DFT of E over the gap edges, F = sum_k w_k sum_g
 *     |Ehat_g(w_k)|^2 (or the time-domain energy of eq. (24));
 *   * the adjoint: the exact transpose of the forward recursion, run
 *     backwards (eq. (20)), and the per-edge sensitivities of eq. (25) with
 *     the chain rule of eq. (27) (filter = identity).
 *
 * Grid: nx x ny nodes (i dx, j dx).  E_x(i,j) at ((i+1/2) dx, j dx), i <
 * nx-1; E_y(i,j) at (i dx, (j+1/2) dx), j < ny-1; H_z(i,j) at ((i+1/2) dx,
 * (j+1/2) dx).  All arrays are [ny][nx], i fastest, unused slots zero.  The
 * outer node lines are PEC: E_x = 0 on j = 0, ny-1 and E_y = 0 on i = 0,
 * nx-1.
 *
 * Design and gap boxes are given in cells (lower node (x0, y0), extent
 * (nx, ny)); their edges include both boundary lines: E_x edges i in [x0,
 * x0+nx-1], j in [y0, y0+ny]; E_y edges i in [x0, x0+nx], j in [y0,
 * y0+ny-1].  The density array holds the design box's E_x edges ([ny+1][nx])
 * followed by its E_y edges ([ny][nx+1]); gap edges are plain eps_g and keep
 * a zero gradient.  The gap monitors are the gap box's E_x edges followed by
 * its E_y edges.
 */
#include "oracle_common.h"

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct orte {
  or_cfg c;
  double *freqs, *wts;
  int nx, ny, N, K;
  double dt;
  int dx0, dy0, dnx, dny, gx0, gy0, gnx, gny;
  int ndx, nd, ngx, ng; /* design edges (E_x part, all), gap edges (E_x part, all) */
  double *bxe, *axe, *kxe, *bxh, *axh, *kxh, *bye, *aye, *kye, *byh, *ayh, *kyh;
  unsigned char *inx_e, *inx_h, *iny_e, *iny_h;
  /* state: fields, currents, absorber memories (adjoint: nu variables) */
  double *Ex, *Ey, *Hz, *Jx, *Jy;
  double *pHzx, *pHzy, *pEx, *pEy;
  int tf_on, ia, ib, ja, jb, jref, L;
  double *einc, *hinc;
  double *rho, *dft, *gapE, *hist;
  double *gEps, *gSig, *gPsi;
  double F;
  int state;
  char err[256];
} orte;

static char g_err[256];

static int fail(orte *o, int code, const char *msg) {
  if (o) snprintf(o->err, sizeof o->err, "%s", msg);
  else snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

const char *orte_last_error(const orte *o) { return o ? o->err : g_err; }

static inline size_t IX(const orte *o, int i, int j) { return (size_t)j * o->nx + i; }

/* Design-variable index of edge (comp, i, j) (comp 0: E_x, 1: E_y), or -1. */
static int design_index(const orte *o, int comp, int i, int j) {
  const int u = i - o->dx0, v = j - o->dy0;
  if (comp == 0) {
    if (u < 0 || u >= o->dnx || v < 0 || v > o->dny) return -1;
    return v * o->dnx + u;
  }
  if (u < 0 || u > o->dnx || v < 0 || v >= o->dny) return -1;
  return o->ndx + v * (o->dnx + 1) + u;
}

/* Monitor index of gap edge (comp, i, j), or -1. */
static int gap_index(const orte *o, int comp, int i, int j) {
  const int u = i - o->gx0, v = j - o->gy0;
  if (comp == 0) {
    if (u < 0 || u >= o->gnx || v < 0 || v > o->gny) return -1;
    return v * o->gnx + u;
  }
  if (u < 0 || u > o->gnx || v < 0 || v >= o->gny) return -1;
  return o->ngx + v * (o->gnx + 1) + u;
}

typedef struct { double eps, psi, sig, kp, beta, C1, C2; } coef_t;

/* Material coefficients of eq. (5) and the trapezoidal ADE on one design edge. */
static coef_t drude_coef(const orte *o, double rho) {
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

void orte_destroy(orte *o) {
  if (!o) return;
  double *p[] = {o->freqs, o->wts, o->bxe, o->axe, o->kxe, o->bxh, o->axh, o->kxh, o->bye, o->aye, o->kye,
                 o->byh, o->ayh, o->kyh, o->Ex, o->Ey, o->Hz, o->Jx, o->Jy, o->pHzx, o->pHzy, o->pEx, o->pEy,
                 o->einc, o->hinc, o->rho, o->dft, o->gapE, o->hist, o->gEps, o->gSig, o->gPsi};
  for (size_t k = 0; k < sizeof p / sizeof p[0]; ++k) free(p[k]);
  free(o->inx_e); free(o->inx_h); free(o->iny_e); free(o->iny_h);
  free(o);
}

static int box_ok(int lo, int n, int a, int b) { return n >= 1 && lo >= a && lo + n <= b; }

int orte_create(const or_cfg *cfg, orte **out) {
  *out = NULL;
  if (!cfg) return fail(NULL, OR_EINVAL, "null config");
  or_cfg c = *cfg;
  if (c.dims != 2) return fail(NULL, OR_EINVAL, "dims must be 2");
  if (c.periodic_x) return fail(NULL, OR_EINVAL, "no periodic axis in the TE oracle");
  if (c.nx < 8 || c.ny < 8) return fail(NULL, OR_EINVAL, "grid too small");
  if (c.n_steps < 1) return fail(NULL, OR_EINVAL, "n_steps < 1");
  if (!(c.dx > 0)) return fail(NULL, OR_EINVAL, "dx <= 0");
  if (!(c.courant > 0) || c.courant >= 1.0 / sqrt(2.0))
    return fail(NULL, OR_EINVAL, "Courant number outside (0, 1/sqrt(2))");
  if (c.n_freq < 1) return fail(NULL, OR_EINVAL, "n_freq < 1");
  if (!(c.eps_s > 0) || !(c.eps_g > 0) || !(c.eps_inf > 0)) return fail(NULL, OR_EINVAL, "permittivity <= 0");
  if (c.psi_s_ratio < 0 || c.sigma_max < 0 || c.gamma_mult < 0) return fail(NULL, OR_EINVAL, "negative material parameter");
  orte *o = (orte *)calloc(1, sizeof(orte));
  if (!o) return fail(NULL, OR_ENOMEM, "out of memory");
  o->c = c;
  o->nx = c.nx; o->ny = c.ny; o->N = c.n_steps; o->K = c.n_freq;
  o->dt = c.courant * c.dx / OR_C0;
  o->dx0 = c.design_lo[0]; o->dy0 = c.design_lo[1]; o->dnx = c.design_n[0]; o->dny = c.design_n[1];
  o->gx0 = c.gap_lo[0]; o->gy0 = c.gap_lo[1]; o->gnx = c.gap_n[0]; o->gny = c.gap_n[1];
  o->ndx = o->dnx * (o->dny + 1);
  o->nd = o->ndx + (o->dnx + 1) * o->dny;
  const int has_gap = o->gnx > 0 && o->gny > 0;
  o->ngx = has_gap ? o->gnx * (o->gny + 1) : 0;
  o->ng = has_gap ? o->ngx + (o->gnx + 1) * o->gny : 0;
  const int P = c.pml_cells, m = c.tfsf_margin;
  o->tf_on = (c.source_kind != OR_SRC_NONE);
  o->ia = P + m; o->ib = c.nx - 1 - P - m;
  o->ja = P + m; o->jb = c.ny - 1 - P - m;
  /* boxes (node ranges [lo, lo + n]) strictly inside the total-field region
   * with the plane wave on, else inside the absorber-free part of the grid */
  int ok = 1, lo, hix, hiy;
  if (o->tf_on) {
    if (o->ia < 2 || o->ib - o->ia < 3 || o->ja < 3 || o->jb - o->ja < 3) ok = 0;
    hix = o->ib - 1; hiy = o->jb - 1;
    if (!box_ok(o->dx0, o->dnx, o->ia + 1, hix) || !box_ok(o->dy0, o->dny, o->ja + 1, hiy)) ok = 0;
    if (has_gap && (!box_ok(o->gx0, o->gnx, o->ia + 1, hix) || !box_ok(o->gy0, o->gny, o->ja + 1, hiy))) ok = 0;
  } else {
    /* closed box: the boxes may fill the absorber-free interior, walls included */
    lo = P; hix = c.nx - 1 - P; hiy = c.ny - 1 - P;
    if (!box_ok(o->dx0, o->dnx, lo, hix) || !box_ok(o->dy0, o->dny, lo, hiy)) ok = 0;
    if (has_gap && (!box_ok(o->gx0, o->gnx, lo, hix) || !box_ok(o->gy0, o->gny, lo, hiy))) ok = 0;
  }
  if (o->gnx < 0 || o->gny < 0) ok = 0;
  if (!ok) { orte_destroy(o); return fail(NULL, OR_EINVAL, "design/gap boxes must lie inside the interior (and the total-field region)"); }

  const size_t n2 = (size_t)c.nx * c.ny;
  o->freqs = (double *)malloc(sizeof(double) * o->K);
  o->wts = (double *)malloc(sizeof(double) * o->K);
  double **ax1[] = {&o->bxe, &o->axe, &o->kxe, &o->bxh, &o->axh, &o->kxh};
  double **ay1[] = {&o->bye, &o->aye, &o->kye, &o->byh, &o->ayh, &o->kyh};
  for (int k = 0; k < 6; ++k) { *ax1[k] = (double *)malloc(sizeof(double) * c.nx); *ay1[k] = (double *)malloc(sizeof(double) * c.ny); }
  o->inx_e = (unsigned char *)malloc(c.nx); o->inx_h = (unsigned char *)malloc(c.nx);
  o->iny_e = (unsigned char *)malloc(c.ny); o->iny_h = (unsigned char *)malloc(c.ny);
  double **fld[] = {&o->Ex, &o->Ey, &o->Hz, &o->Jx, &o->Jy, &o->pHzx, &o->pHzy, &o->pEx, &o->pEy};
  for (int k = 0; k < 9; ++k) *fld[k] = (double *)calloc(n2, sizeof(double));
  o->rho = (double *)calloc((size_t)o->nd, sizeof(double));
  o->dft = (double *)calloc((size_t)o->K * (o->ng > 0 ? o->ng : 1) * 2, sizeof(double));
  o->gapE = (double *)calloc((size_t)(o->N + 1) * (o->ng > 0 ? o->ng : 1), sizeof(double));
  o->hist = (double *)calloc((size_t)o->N * o->nd, sizeof(double));
  o->gEps = (double *)calloc((size_t)o->nd, sizeof(double));
  o->gSig = (double *)calloc((size_t)o->nd, sizeof(double));
  o->gPsi = (double *)calloc((size_t)o->nd, sizeof(double));
  if (!o->freqs || !o->wts || !o->Ex || !o->Ey || !o->Hz || !o->Jx || !o->Jy || !o->pHzx || !o->pHzy ||
      !o->pEx || !o->pEy || !o->rho || !o->dft || !o->gapE || !o->hist || !o->gEps || !o->gSig || !o->gPsi ||
      !o->bxe || !o->kyh || !o->inx_e || !o->iny_h) {
    orte_destroy(o);
    return fail(NULL, OR_ENOMEM, "out of memory");
  }
  if (or_freqs_weights(&c, o->dt, o->freqs, o->wts)) { orte_destroy(o); return fail(NULL, OR_EINVAL, "zero source spectrum at a band frequency"); }
  o->c.freqs_hz = NULL;
  for (int i = 0; i < c.nx; ++i) {
    o->inx_e[i] = (unsigned char)or_pml_profile(&c, o->dt, c.nx, P, (double)i, &o->bxe[i], &o->axe[i], &o->kxe[i]);
    o->inx_h[i] = (unsigned char)or_pml_profile(&c, o->dt, c.nx, P, i + 0.5, &o->bxh[i], &o->axh[i], &o->kxh[i]);
  }
  for (int j = 0; j < c.ny; ++j) {
    o->iny_e[j] = (unsigned char)or_pml_profile(&c, o->dt, c.ny, P, (double)j, &o->bye[j], &o->aye[j], &o->kye[j]);
    o->iny_h[j] = (unsigned char)or_pml_profile(&c, o->dt, c.ny, P, j + 0.5, &o->byh[j], &o->ayh[j], &o->kyh[j]);
  }
  /* incident line: node p <-> row j = jref + p, starting two rows before the box */
  o->jref = o->ja - 2;
  o->L = o->jb + 2 - o->jref + 1;
  if (o->tf_on) {
    if (or_incident_line(&c, o->dt, o->L, o->N, &o->einc, &o->hinc)) { orte_destroy(o); return fail(NULL, OR_ENOMEM, "out of memory"); }
  }
  o->state = 0;
  *out = o;
  return OR_OK;
}

int orte_set_density(orte *o, const double *rho) {
  for (int d = 0; d < o->nd; ++d)
    if (!(rho[d] >= 0.0 && rho[d] <= 1.0)) return fail(o, OR_EINVAL, "density outside [0,1] or NaN");
  memcpy(o->rho, rho, sizeof(double) * o->nd);
  o->state = 1;
  return OR_OK;
}

static void zero_state(orte *o) {
  const size_t n2 = (size_t)o->nx * o->ny;
  double *f[] = {o->Ex, o->Ey, o->Hz, o->Jx, o->Jy, o->pHzx, o->pHzy, o->pEx, o->pEy};
  for (int k = 0; k < 9; ++k) memset(f[k], 0, n2 * sizeof(double));
}

/* Permittivity of a non-design edge: the gap's or the background's. */
static double eps_plain(const orte *o, int comp, int i, int j) {
  return gap_index(o, comp, i, j) >= 0 ? o->c.eps_g : o->c.eps_s;
}

/* ---------------------------------------------------------------- forward */

/* H_z^{n+1/2} from H_z^{n-1/2} and E^n (eq. 10c: mu0 dH_z/dt = -(dE_y/dx -
 * dE_x/dy)), with the absorber memories of both differences and the
 * scattered-field corrections that use the incident E_x at step n. */
static void fwd_h(orte *o, int n, int tf) {
  const int nx = o->nx, ny = o->ny;
  const double dx = o->c.dx, cm = o->dt / OR_MU0;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny - 1; ++j)
    for (int i = 0; i < nx - 1; ++i) {
      const size_t q = IX(o, i, j);
      const double dEy = (o->Ey[IX(o, i + 1, j)] - o->Ey[q]) / dx;
      const double dEx = (o->Ex[IX(o, i, j + 1)] - o->Ex[q]) / dx;
      double tx = dEy / o->kxh[i], ty = dEx / o->kyh[j];
      if (o->inx_h[i]) { o->pHzx[q] = o->bxh[i] * o->pHzx[q] + o->axh[i] * dEy; tx += o->pHzx[q]; }
      if (o->iny_h[j]) { o->pHzy[q] = o->byh[j] * o->pHzy[q] + o->ayh[j] * dEx; ty += o->pHzy[q]; }
      o->Hz[q] -= cm * (tx - ty);
    }
  if (tf) {
    /* the rows of H_z just outside the box read E_x on the box's lower and
     * upper lines, which holds the total field */
    const double c = o->dt / (OR_MU0 * dx);
    const double *e = o->einc + (size_t)n * o->L;
    for (int i = o->ia; i <= o->ib - 1; ++i) {
      o->Hz[IX(o, i, o->ja - 1)] -= c * e[o->ja - o->jref];
      o->Hz[IX(o, i, o->jb)] += c * e[o->jb - o->jref];
    }
  }
}

/* The curl of H at an E edge with its absorber memory updated (forward):
 * E_x: dH_z/dy; E_y: -dH_z/dx. */
static inline double fwd_curl(orte *o, int comp, int i, int j) {
  const size_t q = IX(o, i, j);
  const double dx = o->c.dx;
  if (comp == 0) {
    const double d = (o->Hz[q] - o->Hz[IX(o, i, j - 1)]) / dx;
    double t = d / o->kye[j];
    if (o->iny_e[j]) { o->pEx[q] = o->bye[j] * o->pEx[q] + o->aye[j] * d; t += o->pEx[q]; }
    return t;
  }
  const double d = (o->Hz[q] - o->Hz[IX(o, i - 1, j)]) / dx;
  double t = d / o->kxe[i];
  if (o->inx_e[i]) { o->pEy[q] = o->bxe[i] * o->pEy[q] + o->axe[i] * d; t += o->pEy[q]; }
  return -t;
}

/* One E edge: E^{n+1} (and J^{n+1} on a Drude edge) from its curl. */
static inline void e_update(orte *o, int comp, int i, int j, double curl) {
  const size_t q = IX(o, i, j);
  double *E = comp == 0 ? o->Ex : o->Ey, *Jc = comp == 0 ? o->Jx : o->Jy;
  const double e0 = E[q];
  const int d = design_index(o, comp, i, j);
  if (d >= 0 && gap_index(o, comp, i, j) < 0) {
    const coef_t k = drude_coef(o, o->rho[d]);
    const double e1 = k.C1 * e0 + k.C2 * (curl - 0.5 * (1.0 + k.kp) * Jc[q]);
    Jc[q] = k.kp * Jc[q] + k.beta * (e1 + e0);
    E[q] = e1;
  } else {
    E[q] = e0 + o->dt / (OR_EPS0 * eps_plain(o, comp, i, j)) * curl;
  }
}

/* E^{n+1}, J^{n+1} from E^n, J^n, H^{n+1/2} (eqs. 10a-b), the total-field
 * corrections that use the incident H_z at step n + 1/2; then monitors. */
static void fwd_e(orte *o, int n, int tf, const double *qsrc) {
  const int nx = o->nx, ny = o->ny;
  const double dx = o->c.dx;
  /* incident H_z = -(the line's transverse H): E_x H_z < 0 travels along +y */
  const double *hrow = tf ? o->hinc + (size_t)n * o->L : NULL;
  const size_t n2 = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int j = 1; j < ny - 1; ++j)
    for (int i = 0; i < nx - 1; ++i) {
      double curl = fwd_curl(o, 0, i, j);
      if (tf && i >= o->ia && i <= o->ib - 1) {
        if (j == o->ja) curl += hrow[o->ja - 1 - o->jref] / dx;
        if (j == o->jb) curl -= hrow[o->jb - o->jref] / dx;
      }
      if (qsrc) curl += qsrc[IX(o, i, j)];
      e_update(o, 0, i, j, curl);
    }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny - 1; ++j)
    for (int i = 1; i < nx - 1; ++i) {
      double curl = fwd_curl(o, 1, i, j);
      if (tf && j >= o->ja && j <= o->jb - 1) {
        if (i == o->ia) curl -= hrow[j - o->jref] / dx;
        if (i == o->ib) curl += hrow[j - o->jref] / dx;
      }
      if (qsrc) curl += qsrc[n2 + IX(o, i, j)];
      e_update(o, 1, i, j, curl);
    }
  /* monitors: gap series and running DFT at time (n+1) dt; design history */
  const double dt = o->dt;
  for (int g = 0; g < o->ng; ++g) {
    const int comp = g < o->ngx ? 0 : 1;
    const int r = comp == 0 ? g : g - o->ngx, w = comp == 0 ? o->gnx : o->gnx + 1;
    const double e = (comp == 0 ? o->Ex : o->Ey)[IX(o, o->gx0 + r % w, o->gy0 + r / w)];
    o->gapE[(size_t)(n + 1) * o->ng + g] = e;
    for (int k = 0; k < o->K; ++k) {
      const double ph = 2.0 * M_PI * o->freqs[k] * (n + 1) * dt;
      o->dft[((size_t)k * o->ng + g) * 2 + 0] += dt * e * cos(ph);
      o->dft[((size_t)k * o->ng + g) * 2 + 1] -= dt * e * sin(ph);
    }
  }
  for (int d = 0; d < o->nd; ++d) {
    const int comp = d < o->ndx ? 0 : 1;
    const int r = comp == 0 ? d : d - o->ndx, w = comp == 0 ? o->dnx : o->dnx + 1;
    o->hist[(size_t)n * o->nd + d] = (comp == 0 ? o->Ex : o->Ey)[IX(o, o->dx0 + r % w, o->dy0 + r / w)];
  }
}

static double objective_from_monitors(const orte *o) {
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

static int run_forward(orte *o, int tf, const double *q) {
  zero_state(o);
  memset(o->dft, 0, sizeof(double) * o->K * (o->ng > 0 ? o->ng : 1) * 2);
  memset(o->gapE, 0, sizeof(double) * (size_t)(o->N + 1) * (o->ng > 0 ? o->ng : 1));
  const size_t n2 = (size_t)o->nx * o->ny;
  for (int n = 0; n < o->N; ++n) {
    fwd_h(o, n, tf);
    fwd_e(o, n, tf, q ? q + (size_t)n * 2 * n2 : NULL);
  }
  for (size_t k = 0; k < n2; ++k)
    if (!isfinite(o->Ex[k]) || !isfinite(o->Ey[k])) return fail(o, OR_EUNSTABLE, "non-finite field");
  return OR_OK;
}

int orte_forward(orte *o, double *F_out) {
  if (o->state < 1) return fail(o, OR_ESTATE, "forward before set_density");
  int rc = run_forward(o, o->tf_on, NULL);
  if (rc) return rc;
  o->F = objective_from_monitors(o);
  if (F_out) *F_out = o->F;
  o->state = 2;
  return OR_OK;
}

/* ---------------------------------------------------------------- adjoint */

/* Adjoint source s^m = dF/dE_g^m at gap edge g. */
static double adj_source(const orte *o, int m, int g) {
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

/* One E* edge of the adjoint step: the E/J update with its sensitivity sums. */
static inline void adj_e_update(orte *o, int comp, int i, int j, double curl, const double *Em, int sens) {
  const size_t q = IX(o, i, j);
  double *E = comp == 0 ? o->Ex : o->Ey, *Jc = comp == 0 ? o->Jx : o->Jy;
  const double e0 = E[q];
  const int d = design_index(o, comp, i, j);
  if (d >= 0 && gap_index(o, comp, i, j) < 0) {
    const coef_t k = drude_coef(o, o->rho[d]);
    const double e1 = k.C1 * e0 + k.C2 * (curl - 0.5 * (1.0 + k.kp) * Jc[q]);
    const double j1 = k.kp * Jc[q] + k.beta * (e1 + e0);
    if (sens) {
      o->gEps[d] += Em[d] * (e1 - e0);
      o->gSig[d] += Em[d] * (e1 + e0);
      o->gPsi[d] += Em[d] * (j1 + Jc[q]);
    }
    E[q] = e1;
    Jc[q] = j1;
  } else {
    E[q] = e0 + o->dt / (OR_EPS0 * eps_plain(o, comp, i, j)) * curl;
  }
}

/* One adjoint step m (m = N..1): the state holds E*^{m+1/2}, J*^{m+1/2},
 * H_z*^{m+1} and the memories; leaves E*^{m-1/2}, J*^{m-1/2}, H_z*^m.  ssrc:
 * optional full-grid source ([2][ny][nx]) for this m; otherwise the
 * objective's gap source.  Each curl acts on the field graded by the other
 * field's absorber profile (the transpose of the forward recursion). */
static void adj_step(orte *o, int m, const double *ssrc, double *estar_out) {
  const int nx = o->nx, ny = o->ny;
  const double dx = o->c.dx, cm = o->dt / OR_MU0;
  const size_t n2 = (size_t)nx * ny;
  /* (1) memories at the E edges, driven by E* itself */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t q = IX(o, i, j);
      if (o->iny_e[j]) o->pEx[q] = o->bye[j] * o->pEx[q] + o->aye[j] * o->Ex[q];
      if (o->inx_e[i]) o->pEy[q] = o->bxe[i] * o->pEy[q] + o->axe[i] * o->Ey[q];
    }
  /* (2) H_z*^m: the forward curl-E update applied to the graded E* */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny - 1; ++j)
    for (int i = 0; i < nx - 1; ++i) {
      const size_t q = IX(o, i, j), qr = IX(o, i + 1, j), qu = IX(o, i, j + 1);
      const double gyr = o->Ey[qr] / o->kxe[i + 1] + o->pEy[qr], gy0 = o->Ey[q] / o->kxe[i] + o->pEy[q];
      const double gxu = o->Ex[qu] / o->kye[j + 1] + o->pEx[qu], gx0 = o->Ex[q] / o->kye[j] + o->pEx[q];
      o->Hz[q] -= cm * ((gyr - gy0) - (gxu - gx0)) / dx;
    }
  /* (3) memories at the H_z positions, driven by H_z* */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t q = IX(o, i, j);
      if (o->inx_h[i]) o->pHzx[q] = o->bxh[i] * o->pHzx[q] + o->axh[i] * o->Hz[q];
      if (o->iny_h[j]) o->pHzy[q] = o->byh[j] * o->pHzy[q] + o->ayh[j] * o->Hz[q];
    }
  /* (4) E*^{m-1/2}, J*^{m-1/2} and the sensitivity sums with the forward E^m */
  const double *Em = o->hist + (size_t)(m - 1) * o->nd;
  const int sens = ssrc == NULL;
#pragma omp parallel for schedule(static)
  for (int j = 1; j < ny - 1; ++j)
    for (int i = 0; i < nx - 1; ++i) {
      const size_t q = IX(o, i, j), qd = IX(o, i, j - 1);
      double curl = ((o->Hz[q] / o->kyh[j] + o->pHzy[q]) - (o->Hz[qd] / o->kyh[j - 1] + o->pHzy[qd])) / dx;
      if (ssrc) curl += ssrc[q];
      else {
        const int g = gap_index(o, 0, i, j);
        if (g >= 0) curl += adj_source(o, m, g);
      }
      adj_e_update(o, 0, i, j, curl, Em, sens);
    }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny - 1; ++j)
    for (int i = 1; i < nx - 1; ++i) {
      const size_t q = IX(o, i, j), ql = IX(o, i - 1, j);
      double curl = -((o->Hz[q] / o->kxh[i] + o->pHzx[q]) - (o->Hz[ql] / o->kxh[i - 1] + o->pHzx[ql])) / dx;
      if (ssrc) curl += ssrc[n2 + q];
      else {
        const int g = gap_index(o, 1, i, j);
        if (g >= 0) curl += adj_source(o, m, g);
      }
      adj_e_update(o, 1, i, j, curl, Em, sens);
    }
  if (estar_out) {
    memcpy(estar_out + (size_t)(m - 1) * 2 * n2, o->Ex, sizeof(double) * n2);
    memcpy(estar_out + (size_t)(m - 1) * 2 * n2 + n2, o->Ey, sizeof(double) * n2);
  }
}

int orte_adjoint(orte *o) {
  if (o->state < 2) return fail(o, OR_ESTATE, "adjoint before forward");
  zero_state(o);
  memset(o->gEps, 0, sizeof(double) * o->nd);
  memset(o->gSig, 0, sizeof(double) * o->nd);
  memset(o->gPsi, 0, sizeof(double) * o->nd);
  for (int m = o->N; m >= 1; --m) adj_step(o, m, NULL, NULL);
  o->state = 3;
  return OR_OK;
}

/* dF/drho per design edge (the density layout); optional partials
 * dF/deps_inf_i, dF/dpsi_i, dF/dsigma_i (eq. 25).  Gap edges: 0. */
int orte_gradient(orte *o, double *grad, double *d_eps, double *d_psi, double *d_sig) {
  if (o->state < 3) return fail(o, OR_ESTATE, "gradient before adjoint");
  const or_cfg *c = &o->c;
  const double psi = c->omega_p * c->omega_p, psi_s = c->psi_s_ratio * psi;
  for (int d = 0; d < o->nd; ++d) {
    const int comp = d < o->ndx ? 0 : 1;
    const int r = comp == 0 ? d : d - o->ndx, w = comp == 0 ? o->dnx : o->dnx + 1;
    const int i = o->dx0 + r % w, j = o->dy0 + r / w;
    double fe = 0, fp = 0, fs = 0, g = 0;
    if (gap_index(o, comp, i, j) < 0) {
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

int orte_get_dft(const orte *o, double *out) {
  if (o->state < 2) return OR_ESTATE;
  memcpy(out, o->dft, sizeof(double) * o->K * o->ng * 2);
  return OR_OK;
}

int orte_get_gap_series(const orte *o, double *out) {
  if (o->state < 2) return OR_ESTATE;
  memcpy(out, o->gapE, sizeof(double) * (size_t)(o->N + 1) * o->ng);
  return OR_OK;
}

/* Sizes: design edges (all, of which E_x), gap edges (all, of which E_x). */
void orte_sizes(const orte *o, int32_t *out) {
  out[0] = o->nd; out[1] = o->ndx; out[2] = o->ng; out[3] = o->ngx;
}

void orte_info(const orte *o, double *dt, double *freqs, double *wts, int32_t *tf_box) {
  if (dt) *dt = o->dt;
  if (freqs) memcpy(freqs, o->freqs, sizeof(double) * o->K);
  if (wts) memcpy(wts, o->wts, sizeof(double) * o->K);
  if (tf_box) { tf_box[0] = o->ia; tf_box[1] = o->ib; tf_box[2] = o->ja; tf_box[3] = o->jb; }
}

/* ------------------------------------------------------------ test hooks */

/* Forward with the plane wave off and an extra source q^{n+1} ([N][2][ny][nx]:
 * E_x, E_y) in the curl bracket; fields are not returned (use get_state). */
int orte_forward_ext(orte *o, const double *q, double *efull) {
  if (o->state < 1) return fail(o, OR_ESTATE, "forward before set_density");
  zero_state(o);
  const size_t n2 = (size_t)o->nx * o->ny;
  memset(o->dft, 0, sizeof(double) * o->K * (o->ng > 0 ? o->ng : 1) * 2);
  for (int n = 0; n < o->N; ++n) {
    fwd_h(o, n, 0);
    fwd_e(o, n, 0, q + (size_t)n * 2 * n2);
    if (efull) {
      memcpy(efull + (size_t)n * 2 * n2, o->Ex, sizeof(double) * n2);
      memcpy(efull + (size_t)n * 2 * n2 + n2, o->Ey, sizeof(double) * n2);
    }
  }
  return OR_OK;
}

/* Adjoint driven by s^m ([N][2][ny][nx], index m-1) instead of the objective;
 * E*^{m-1/2} to estar ([N][2][ny][nx], index m-1). */
int orte_adjoint_ext(orte *o, const double *s, double *estar) {
  if (o->state < 1) return fail(o, OR_ESTATE, "adjoint before set_density");
  zero_state(o);
  const size_t n2 = (size_t)o->nx * o->ny;
  for (int m = o->N; m >= 1; --m) adj_step(o, m, s + (size_t)(m - 1) * 2 * n2, estar);
  return OR_OK;
}

/* State access for source-free evolution tests.  Arrays are full [ny][nx];
 * absorber memories are cleared. */
int orte_set_state(orte *o, const double *Ex, const double *Ey, const double *Hz, const double *Jx,
                   const double *Jy) {
  const size_t n2 = (size_t)o->nx * o->ny;
  zero_state(o);
  memcpy(o->Ex, Ex, n2 * sizeof(double));
  memcpy(o->Ey, Ey, n2 * sizeof(double));
  memcpy(o->Hz, Hz, n2 * sizeof(double));
  memcpy(o->Jx, Jx, n2 * sizeof(double));
  memcpy(o->Jy, Jy, n2 * sizeof(double));
  return OR_OK;
}

int orte_get_state(const orte *o, double *Ex, double *Ey, double *Hz, double *Jx, double *Jy) {
  const size_t n2 = (size_t)o->nx * o->ny;
  memcpy(Ex, o->Ex, n2 * sizeof(double));
  memcpy(Ey, o->Ey, n2 * sizeof(double));
  memcpy(Hz, o->Hz, n2 * sizeof(double));
  memcpy(Jx, o->Jx, n2 * sizeof(double));
  memcpy(Jy, o->Jy, n2 * sizeof(double));
  return OR_OK;
}

/* k source-free steps of the set state (monitors and history untouched). */
int orte_step_free(orte *o, int k) {
  if (o->state < 1) return fail(o, OR_ESTATE, "step before set_density");
  const size_t n2 = (size_t)o->nx * o->ny;
  double *save_g = o->gapE, *save_d = o->dft, *save_h = o->hist;
  double *scratch = (double *)calloc((size_t)(o->ng > 0 ? o->ng : 1) * (o->K * 2 + 2) + (size_t)o->nd + n2, sizeof(double));
  if (!scratch) return fail(o, OR_ENOMEM, "out of memory");
  /* monitors write into scratch rows (slot n = 0 only) */
  o->gapE = scratch;
  o->dft = scratch + 2 * (o->ng > 0 ? o->ng : 1);
  o->hist = o->dft + (size_t)o->K * (o->ng > 0 ? o->ng : 1) * 2;
  for (int s = 0; s < k; ++s) {
    fwd_h(o, 0, 0);
    fwd_e(o, 0, 0, NULL);
  }
  o->gapE = save_g; o->dft = save_d; o->hist = save_h;
  free(scratch);
  return OR_OK;
}
