/*
 * fdtd_design.h -- C ABI of the design-update loop around the FDTD hot path.
 *
 * The paper's optimization (Methods: eqs. (26)-(28) and the optimization
 * flowchart) maximizes the discrete objective over the density rho with
 * box constraints.  Each iteration filters the design variables (eq. (26)),
 * runs the forward and adjoint FDTD solves on the filtered density
 * (fdtd.h), maps the gradient back through the filter (eq. (27)) and updates
 * rho with the globally convergent method of moving asymptotes.  The design
 * is declared converged by its level of non-discreteness and finally
 * thresholded at 0.5.  This header holds the per-element parts of that loop:
 *
 *   fdtd_filter_*   open-close filter: a cascade of four fW-mean filters
 *                   (erode, dilate, dilate, erode) and the transpose of its
 *                   Jacobian for the chain rule of eq. (27)
 *   fdtd_mma_*      one method-of-moving-asymptotes step for an objective with
 *                   box constraints only: asymptotes, the conservative
 *                   separable approximation and its closed-form minimizer,
 *                   with the sums the globally convergent variant needs
 *   fdtd_design_stats   non-discreteness and first-order optimality
 *
 * Conventions: all vectors are device pointers of the object's precision
 * (float or double) with one value per design cell, in the density layout of
 * fdtd.h; all work runs in order on the object's stream (NULL: the library
 * creates one); sums are deterministic (fixed-order FP64 reductions).
 * Functions return an fdtd_status and never abort.
 */
#ifndef FDTD_DESIGN_H
#define FDTD_DESIGN_H

#include <stdint.h>

#include "fdtd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_filter fdtd_filter; /* opaque */
typedef struct fdtd_mma fdtd_mma;       /* opaque */

/* Open-close filter over a box of n[0] x n[1] x n[2] cells (n[2] = 1 in 2D).
 * Each of the four stages is an fW-mean: e_i = f^-1( sum_j w_ij f(u_j) ) with
 * f(u) = 1/(u + alpha), cone weights w_ij proportional to max(0, radius - |x_i - x_j|)
 * over the cells of the box (normalised per cell), u = x for the erosion and
 * u = 1 - x, output 1 - e for the dilation.  radius in cells (the paper's
 * filter size 5 dx is radius 2.5).  EINVAL for a non-positive size or radius. */
fdtd_status fdtd_filter_create(const int32_t n[3], double radius, int32_t precision, void *stream, fdtd_filter **out);

/* rho_f = F(rho) with nonlinearity alpha > 0 (large alpha: nearly the linear
 * cone filter; small alpha: close to min/max morphology).  Keeps the stage
 * inputs for fdtd_filter_transpose. */
fdtd_status fdtd_filter_apply(fdtd_filter *f, const void *rho, void *rho_f, double alpha);

/* g = J^T g_f, J = dF/drho at the last fdtd_filter_apply (ESTATE before any). */
fdtd_status fdtd_filter_transpose(fdtd_filter *f, const void *g_f, void *g);

fdtd_status fdtd_filter_destroy(fdtd_filter *f);

/* MMA for: minimize f0(x) subject to xmin <= x <= xmax, n variables.
 * move: move limit as a fraction of xmax - xmin (0.5); asyinit, asyincr,
 * asydecr: initial asymptote distance and its growth / shrink factors on
 * monotone / oscillating variables (0.5, 1.2, 0.7). */
fdtd_status fdtd_mma_create(int64_t n, int32_t precision, double xmin, double xmax, double move, double asyinit,
                            double asyincr, double asydecr, void *stream, fdtd_mma **out);

/* Start an outer iteration at x with objective f0 and gradient df0: update the
 * asymptotes from the previous two accepted iterates, the move limits, and
 * return in *rho0 the initial curvature weight of the approximation. */
fdtd_status fdtd_mma_begin(fdtd_mma *m, const void *x, double f0, const void *df0, double *rho0);

/* Minimizer xnew of the separable approximation with curvature weight rho
 * (>= 0).  *approx = the approximation's value at xnew; *dist = the distance
 * measure sum (U-L)(xnew-x)^2 / ((U-xnew)(xnew-L)(xmax-xmin)) used to raise rho
 * when the approximation was not conservative. */
fdtd_status fdtd_mma_solve(fdtd_mma *m, double rho, void *xnew, double *approx, double *dist);

/* Accept xnew as the next iterate (shifts the iterate history). */
fdtd_status fdtd_mma_accept(fdtd_mma *m, const void *xnew);

fdtd_status fdtd_mma_destroy(fdtd_mma *m);

/* out[0] = 4 x^T (1 - x) / n (non-discreteness of a density x in [0,1]);
 * out[1] = || x - clamp(x - g, xmin, xmax) ||_2 (first-order optimality of a
 * box-constrained minimization with gradient g; g may be NULL: out[1] = 0). */
fdtd_status fdtd_design_stats(int64_t n, int32_t precision, const void *x, const void *g, double xmin, double xmax,
                              void *stream, double out[2]);

/* Message of the last failing call of this header's functions on the calling
 * thread. */
const char *fdtd_design_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_DESIGN_H */
