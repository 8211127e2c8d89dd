/*
 * fdtd.h -- C ABI of the MI355X Drude-FDTD topology-optimization hot path.
 *
 * One optimization iteration of time-domain topology optimization for
 * dispersive (Drude) nanostructures, after Hassan & Cala Lesina, "Topology
 * optimization of dispersive plasmonic nanostructures in the time-domain"
 * (arXiv 2203.01462):
 *
 *   fdtd_set_density   rho over the design box                  (eqs. (4)-(5))
 *   fdtd_forward       Drude-ADE FDTD forward solve, gap DFT, F (eqs. (10a-c), (3)/(24))
 *   fdtd_adjoint       adjoint FDTD solve, sensitivity sums      (eq. (20), eq. (25))
 *   fdtd_gradient      dF/drho per design cell                   (eq. (27), filter = identity)
 *
 * The conceptual problem is eq. (2) / its discrete form eq. (28): maximize an
 * electric-field objective in a gap region by choosing, per design cell, a
 * density rho in [0,1] that interpolates between a dielectric (eps_s) and a
 * Drude metal (eps_inf, omega_p, gamma_p; eq. (1)), with the artificial
 * damping of eq. (5c) (sigma_max) and/or a collision-rate multiplier
 * (gamma = gamma_mult * gamma_p).
 *
 * Conventions
 *   * Units are SI.  Grid nodes are indexed (x, y, z); arrays are row-major
 *     with x fastest: [y][x] in 2D, [z][y][x] in 3D.
 *   * dims = 2 is the TMz polarization: E along z (one E per cell, at the
 *     node), H in the plane; the plane wave travels along +y.
 *     dims = 3 is the full Yee cell; the plane wave travels along +z with E
 *     along x.  Each cell owns its three index-aligned E edges.
 *   * The outermost nodes are PEC walls; a convolutional PML of pml_cells
 *     lines the walls; a total-field/scattered-field box tfsf_margin cells
 *     inside the PML injects the plane wave.  Design and gap boxes must lie
 *     strictly inside the total-field box.
 *   * Gap cells are non-dispersive (eps_g) and carry no design variable even
 *     when they lie inside the design box; their gradient entry is 0.
 *   * Objective (objective_kind = DFT): F = sum_k w_k sum_{g,c} |Ehat_{g,c}(w_k)|^2,
 *     Ehat(w) = dt sum_{n=1..N} E^n exp(-j w n dt); w_k = 1/|Ghat(w_k)|^2
 *     (ENHANCEMENT: Ghat is the same DFT of the excitation waveform) or 1 (UNIT).
 *     objective_kind = TIME_ENERGY is eq. (24).
 *
 * Ownership and threading
 *   * The caller owns every buffer passed in or out; the library copies what
 *     it keeps (rho, freqs_hz).  A context owns all of its device memory and
 *     frees it in fdtd_destroy.
 *   * All device work of a context runs in order on its stream (config.stream,
 *     a hipStream_t the caller keeps alive; NULL: the library creates one).
 *     Calls on one context must not overlap; distinct contexts are
 *     independent.
 *   * Functions never abort or exit; they return an fdtd_status and leave a
 *     message readable with fdtd_last_error.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDTD_ABI_VERSION 5

typedef enum {
  FDTD_OK = 0,
  FDTD_EINVAL = 1,    /* invalid argument or configuration */
  FDTD_ESTATE = 2,    /* call out of order (e.g. adjoint before forward) */
  FDTD_ENOMEM = 3,    /* device memory or history budget exhausted */
  FDTD_EDEVICE = 4,   /* HIP runtime error (no device, launch failure) */
  FDTD_EUNSTABLE = 5  /* runaway or non-finite fields (in-solve watchdog), or a non-finite objective */
} fdtd_status;

/* Excitation: the Gaussian-modulated carrier, the paper's Hann-windowed sinc
 * (Sec. 2), or none (no plane wave: the fields evolve from the state given
 * by fdtd_set_state, zero otherwise; objective weights are then 1). */
enum { FDTD_SRC_GAUSS = 0, FDTD_SRC_SINC_HANN = 1, FDTD_SRC_NONE = 2 };
/* Axes of pol_axis / prop_axis. */
enum { FDTD_AXIS_DEFAULT = -1, FDTD_AXIS_X = 0, FDTD_AXIS_Y = 1, FDTD_AXIS_Z = 2 };
enum { FDTD_OBJ_DFT = 0, FDTD_OBJ_TIME_ENERGY = 1 };
enum { FDTD_W_ENHANCEMENT = 0, FDTD_W_UNIT = 1 };

typedef struct fdtd_ctx fdtd_ctx; /* opaque */

typedef struct {
  int32_t abi_version;   /* must be FDTD_ABI_VERSION */
  int32_t dims;          /* 2 (TMz, or TEz with pol_axis = x) or 3 */
  int32_t precision;     /* 32 or 64: field arithmetic and storage; DFT and sensitivity sums are always FP64 */
  int32_t n[3];          /* nodes along x, y, z (n[2] ignored in 2D) */
  int32_t n_steps;       /* N time steps of each solve */
  int32_t pml_cells;     /* CPML thickness (cells) next to each wall */
  int32_t tfsf_margin;   /* cells between the PML and the total-field box */
  int32_t pol_axis;      /* axis of the incident E.  dims 2: z selects TMz (E_z, H_x, H_y), x selects
                            TEz (E_x, E_y, H_z: E in the plane, the paper's plasmonic 2D case,
                            Sec. 4.1); dims 3: x.  FDTD_AXIS_DEFAULT (-1) takes z in 2D, x in 3D;
                            any other axis is EINVAL */
  int32_t prop_axis;     /* propagation axis of the plane wave (towards +): 2D y, 3D z; -1 default */
  int32_t design_lo[3], design_n[3]; /* design box, nodes [lo, lo+n) per axis.  TEz: a box of
                            design_n cells whose edges include both boundary lines; the density
                            holds one value per edge, its E_x edges [ny+1][nx] followed by its
                            E_y edges [ny][nx+1] (Sec. 3.2: one design variable per Yee edge);
                            the gap box's edges are plain eps_g, zero gradient, and are the
                            monitors (E_x edges, then E_y edges); no checkpointing, no batches */
  int32_t gap_lo[3], gap_n[3];       /* gap (observation) box */
  int32_t source_kind;   /* FDTD_SRC_*: Gaussian-modulated carrier, or the paper's Hann-windowed 4-lobe sinc */
  int32_t objective_kind;/* FDTD_OBJ_* */
  int32_t weight_kind;   /* FDTD_W_* */
  int32_t n_freq;        /* K >= 1 band frequencies */
  double dx;             /* cell size (m), equal along all axes */
  double courant;        /* c0 dt / dx, in (0, 1/sqrt(dims)) */
  double pml_order, pml_sigma_scale, pml_kappa_max, pml_alpha_max; /* CPML grading: order m, sigma_max/(0.8(m+1)/(eta_s dx)), kappa_max, alpha_max (S/m) */
  double eps_s;          /* background / rho = 0 relative permittivity */
  double eps_g;          /* gap relative permittivity */
  double eps_inf, omega_p, gamma_p; /* Drude metal (eq. (1)) at rho = 1 */
  double gamma_mult;     /* collision-rate multiplier (damping continuation) */
  double sigma_max;      /* artificial conductivity peak of eq. (5c), S/m */
  double psi_s_ratio;    /* psi_s / omega_p^2 (the paper uses 1/100) */
  double f_lo, f_hi;     /* band edges (Hz) of the excitation */
  double t0_over_tau;    /* Gaussian delay in units of its width */
  double amplitude;      /* incident amplitude (V/m) */
  const double *freqs_hz;/* K frequencies, or NULL for K uniform over [f_lo, f_hi]; copied */
  int64_t history_budget_bytes; /* cap on the forward history plus checkpoints; 0 = device limit */
  int32_t ckpt_every;    /* 0: store E on every design edge for all n_steps (the
                            sums of eq. (25) read it back in reverse).  K > 0:
                            store only K steps of it plus a full-state snapshot
                            every K steps; the adjoint re-runs each K-step
                            segment of the forward from its snapshot, newest
                            first, before the adjoint steps that need it (when
                            the budget holds a second K-step history, on a
                            stream of the context's own, beside the adjoint
                            sweep of the segment after it).  Both give
                            bit-identical gradients. */
  void *stream;          /* hipStream_t or NULL */
} fdtd_config;

/* Per-solve timing of the time-stepping kernel, from HIP events recorded on
 * the context stream right before the first and right after the last step
 * launch of the most recent forward and adjoint solves. */
typedef struct {
  double forward_ms, adjoint_ms;   /* event time over the step-kernel launches */
  int64_t forward_launches, adjoint_launches;
  int64_t cells;                   /* nodes of the grid */
  int64_t design_cells;            /* cells of the design box (Drude or gap) */
} fdtd_timing;

/* Version of this header the library was built from. */
int32_t fdtd_abi_version(void);

/* Validate `cfg`, allocate the context and all device memory, and compute the
 * ρ-independent tables (absorber grading, incident-field line, phasors,
 * weights).  Fails with EINVAL on: precision not 32/64, dims not 2/3,
 * Courant outside (0, 1/sqrt(dims)), n_steps < 1, n_freq < 1, non-positive
 * permittivities or negative material parameters, ckpt_every < 0, axes other
 * than the supported ones, ckpt_every > 0 on a TEz context, boxes outside
 * the total-field region (with FDTD_SRC_NONE: outside the nodes 1 +
 * pml_cells .. n - 2 - pml_cells; TEz: pml_cells .. n - 1 - pml_cells);
 * ENOMEM if the forward history (and, with ckpt_every > 0, the snapshots)
 * does not fit the budget or the device; EDEVICE without a usable HIP device.
 * *out is NULL on failure. */
fdtd_status fdtd_create(const fdtd_config *cfg, fdtd_ctx **out);

/* Set the density over the design box (eqs. (4)-(5)): `count` =
 * prod(design_n) values of the context precision (float or double), layout
 * [z][y][x] / [y][x].  on_device != 0: `rho` is a device pointer read in
 * stream order; else a host pointer copied before return.  Entries must lie
 * in [0,1] (NaN rejected) -> EINVAL.  Invalidates forward/adjoint results. */
fdtd_status fdtd_set_density(fdtd_ctx *ctx, const void *rho, int64_t count, int32_t on_device);

/* Forward FDTD solve over n_steps (eqs. (10a-c)) with the gap monitor;
 * writes the objective F to *objective_out (host; may be NULL) and returns
 * after the solve has finished.  Requires a density (ESTATE).  A watchdog
 * reads the largest |E| every 1024 steps while the solve runs; on a
 * non-finite value or one above 1e10 times the reference amplitude (the
 * incident amplitude, or with FDTD_SRC_NONE the largest value of the state
 * set by fdtd_set_state) the solve stops and returns EUNSTABLE, naming the
 * step, and the forward result is invalid. */
fdtd_status fdtd_forward(fdtd_ctx *ctx, double *objective_out);

/* Adjoint FDTD solve (eq. (20)): time-reversed, driven by dF/dE at the gap,
 * accumulating the sensitivity sums of eq. (25) on every Drude design edge.
 * Requires a forward solve on the current density (ESTATE).  Asynchronous
 * on the context stream, except that the watchdog (non-finite adjoint
 * fields, EUNSTABLE) keeps the host at most 2048 steps behind the device. */
fdtd_status fdtd_adjoint(fdtd_ctx *ctx);

/* dF/drho per design cell (eq. (27), filter = identity; in 3D the sum over the
 * cell's three edges), `count` = prod(design_n) values of the context
 * precision, same layout as the density.  on_device != 0: device pointer,
 * written in stream order; else host pointer, filled before return.
 * Requires an adjoint solve on the current density (ESTATE). */
fdtd_status fdtd_gradient(fdtd_ctx *ctx, void *grad_out, int64_t count, int32_t on_device);

/* Gap DFT after a forward solve: host array of count = K * n_gap_cells *
 * n_comp * 2 doubles, layout [k][gap cell][component][re, im]; n_comp = 1 in
 * 2D, 3 (Ex, Ey, Ez) in 3D. */
fdtd_status fdtd_get_dft(fdtd_ctx *ctx, double *re_im, int64_t count);

/* TEST ONLY (source-free evolution: eigenmode, energy and stability checks
 * of the update itself, eqs. (10a-c)).  Initial state of the following
 * forward solves instead of zero: `state` holds, on the host, count =
 * nf * nx * ny * nz doubles, nf full-grid arrays [z][y][x] in the order
 * E_z, H_x, H_y, J_z (TMz: nf = 4, z ignored), E_x, E_y, H_z, J_x, J_y (TEz:
 * nf = 5) or E_x, E_y, E_z, H_x, H_y, H_z, J_x, J_y, J_z (dims 3: nf = 9),
 * at the staggered positions of the Yee
 * cell: E^0 and J^0 at t = 0, H^{-1/2} at t = -dt/2.  Positions the update
 * never writes (E and H on the PEC walls) and J off the Drude design edges
 * are taken as zero; absorber memories start at zero.  The state is copied;
 * it applies to every forward until fdtd_set_state(ctx, NULL, 0) clears it.
 * EINVAL on a wrong count or a NULL pointer with count != 0. */
fdtd_status fdtd_set_state(fdtd_ctx *ctx, const double *state, int64_t count);

/* TEST ONLY.  The state at the end of the most recent forward solve (E^N,
 * H^{N-1/2}, J^N), same layout as fdtd_set_state, into the host array
 * `state` of count doubles.  ESTATE before a forward solve or after an
 * adjoint solve (which reuses the state buffers). */
fdtd_status fdtd_get_state(fdtd_ctx *ctx, double *state, int64_t count);

/* Timing of the most recent solves (see fdtd_timing). */
fdtd_status fdtd_get_timing(fdtd_ctx *ctx, fdtd_timing *out);

/* Release the context and its device memory.  NULL is accepted. */
fdtd_status fdtd_destroy(fdtd_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batches of 2D instances.  Uneven TMz problems (own grid size, density,
 * damping, band, objective) advance together: at temporal-block depth 1 each
 * time step of all instances is one launch per tile depth in use; at depth 2
 * the instances follow the blocked schedule of a single context (plain
 * background super-tiles advance two steps per pass, everything else one
 * step per launch, two launches per pair of steps for all instances
 * together).  The N steps of a forward (or adjoint) solve are captured once
 * into a HIP graph and replayed.  Every instance computes exactly what a
 * single context with the same config and tile depth computes.
 */
typedef struct fdtd_batch fdtd_batch; /* opaque */

typedef struct {
  int32_t rows;       /* nodes per thread along y in the 2D step (tile depth):
                         1, 2 or 4 for every instance; 0 = tune on the batch at
                         creation: time 20 batched steps at each uniform depth,
                         then try the other depths for each grid size in turn
                         and keep what is faster */
  int32_t use_graph;  /* 1: replay the captured step sequence; 0: launch eagerly */
  int32_t depth;      /* temporal-block depth: 1 = one step per launch; 2 = the
                         blocked schedule for every instance that has
                         plain-background super-tiles (needs rows 0 or 2; the
                         tile depth is then 2); 0 = tune at creation: time the
                         best depth-1 choice against depth 2, try depth 1 for
                         each grid size in turn inside the blocked schedule,
                         keep what is faster */
} fdtd_batch_options;

/* Create `count` >= 1 instances from cfgs[0..count-1]: all dims = 2, the same
 * precision and n_steps, ckpt_every = 0.  All instances run on one stream:
 * cfgs[0].stream (the other streams are ignored) or one the library creates.
 * opt may be NULL (rows = 0, use_graph = 1, depth = 0).  Fails like
 * fdtd_create (the message names the instance), or EINVAL for mixed
 * precision / step counts or options out of range. */
fdtd_status fdtd_batch_create(const fdtd_config *cfgs, int32_t count, const fdtd_batch_options *opt,
                              fdtd_batch **out);

/* Density of instance `index` (as fdtd_set_density). */
fdtd_status fdtd_batch_set_density(fdtd_batch *b, int32_t index, const void *rho, int64_t count, int32_t on_device);

/* Forward solve of every instance; objectives_out (host, may be NULL) gets
 * `count` values.  Requires a density on every instance. */
fdtd_status fdtd_batch_forward(fdtd_batch *b, double *objectives_out);

/* Adjoint solve of every instance (after fdtd_batch_forward). */
fdtd_status fdtd_batch_adjoint(fdtd_batch *b);

/* dF/drho of instance `index` (as fdtd_gradient). */
fdtd_status fdtd_batch_gradient(fdtd_batch *b, int32_t index, void *grad_out, int64_t count, int32_t on_device);

/* Tile depth used for instance `index`, and the event time (ms) of the last
 * batched forward and adjoint step sequences (all instances together). */
fdtd_status fdtd_batch_info(fdtd_batch *b, int32_t index, int32_t *rows_out, double *forward_ms, double *adjoint_ms);

/* Temporal-block depth (1 or 2) used for instance `index`. */
fdtd_status fdtd_batch_depth(fdtd_batch *b, int32_t index, int32_t *depth_out);

/* Release the batch and all instances.  NULL is accepted. */
fdtd_status fdtd_batch_destroy(fdtd_batch *b);

/* Message of the last failing call on `b` (or, when b is NULL, of the
 * calling thread's last failing fdtd_batch_create). */
const char *fdtd_batch_last_error(const fdtd_batch *b);

/* Message of the last failing call on `ctx` (or, when ctx is NULL, of the
 * calling thread's last failing fdtd_create).  Owned by the library; valid
 * until the next call on the same context (or the next fdtd_create on the
 * same thread). */
const char *fdtd_last_error(const fdtd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
