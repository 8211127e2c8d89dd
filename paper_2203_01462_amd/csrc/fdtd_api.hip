// fdtd_api.hip -- the C ABI of include/fdtd.h: context creation, validation,
// buffer management and the solve drivers.  The time loops only enqueue
// kernels on the context stream; all arithmetic of a solve runs on the GPU.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fdtd_2d.hpp"
#include "fdtd_3d.hpp"

using namespace fdtd;

struct fdtd_ctx {
  fdtd_config cfg{};
  std::vector<double> freqs;
  int dims = 2, prec = 64;
  size_t esz = 8;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int nx = 0, ny = 0, nz = 1, pitch = 0;
  Arena3 lay3{};
  int tn3 = 0;
  int N = 0, K = 0, nd = 0, ng = 0, ncomp = 1, nmon = 0;
  double dt = 0;
  int ia = 0, ib = 0, ja = 0, jb = 0, jref = 0, L = 0;
  bool te = false;  // 2D TEz (E in the plane along x): fdtd_te.hip, per-edge design variables
  int lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
  // device memory: 2D fields (Ez, Hx, Hy) and absorber memories (4), two
  // copies each; 3D: one arena per copy (fields and absorber slabs) and the
  // packed CPML tables
  DevBuf fld[2][6], pml[2][12], arena3[3], tab3, J, rho, hist, grad, dft, gapE, phasor, wts, dfreq, asrc, einc, hinc;
  DevBuf axis[18], gwave, lineprof, linescr, scal, bad, Fdev, gtmp;
  // checkpointed adjoint: a second state (both copies and J) for re-running
  // forward segments, and the snapshots [nseg-1][state copy + J]
  DevBuf fldR[2][6], pmlR[2][12], arenaR[3], JR, snap;
  // 2D two-step blocking of the plain background: a third copy of the fields
  // (main and re-run state), the super-tiles and the per-step tiles
  DevBuf fld3[3], fld3R[3], tbTiles, tbRest;
  DevBuf glist3;  // 3D: tile-chunk lists of the general update
  int gS = 0, gM = 0, gD = 0, gAxD = 0;  // lengths of the three lists in glist3
  // 3D two-step blocking of the plain background (FP32): the super-chunk
  // launch list and flag grid; with super-chunks the state rotates over
  // three arenas (the state after s steps lives in arena s mod 3)
  DevBuf sup_list, sup_flags;
  Aux3D sup{nullptr, nullptr, nullptr}, supR{nullptr, nullptr, nullptr};  // the pass's stream (main, re-run lane)
  int nSup = 0, so3[3] = {0, 0, 0}, sn3[3] = {0, 0, 0};
  bool sup_planned = false;
  int nTb = 0, nRest = 0, nEarly = 0;  // tbTiles = [interior super-tiles (run early) | border ones]
  int ck = 0, nseg = 1;  // segment length (steps) and count; nseg = 1: full history
  size_t snap_bytes = 0;
  Step2D<float> p2f{}, p2fR{};
  Step2D<double> p2d{}, p2dR{};
  Step3D<float> p3f{}, p3fR{};
  Step3D<double> p3d{}, p3dR{};
  int state = 0;  // 0 created, 1 density, 2 forward, 3 adjoint
  double F = 0;
  std::string err;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  Aux3D aux{nullptr, nullptr, nullptr};  // 3D: second stream and fork/join events
  // checkpointed adjoint with the re-runs on their own stream: a second
  // history buffer (segment s uses buffer s % 2), the re-run stream and its
  // 3D side stream, and the events that order the two streams
  DevBuf hist2;
  hipStream_t rr = nullptr;
  Aux3D auxR{nullptr, nullptr, nullptr};
  hipEvent_t evStart = nullptr, evRerun = nullptr, evAdj[2] = {nullptr, nullptr};
  fdtd_timing timing{};
  // initial state of the forward solves (fdtd_set_state; host, full grid,
  // double) and whether the main state buffers hold a finished forward
  std::vector<double> init_state;
  bool fwd_state_valid = false;
  // in-solve watchdog: one slot per check (device, then pinned host copy)
  DevBuf watch;
  unsigned long long *watch_host = nullptr;
  int watch_slots = 0;
  hipEvent_t evWatch[2] = {nullptr, nullptr};
};

namespace {

thread_local std::string g_create_error;  // per thread: creates may run on several threads

// Steps between two checks of the forward solve's watchdog.
constexpr int kWatchEvery = 1024;
// A passive medium driven by a plane wave of amplitude A keeps |E| far below
// this multiple of A; beyond it (or at a non-finite value) the solve is unstable.
constexpr double kWatchFactor = 1e10;

Error einval(const std::string &m) { return Error{FDTD_EINVAL, m}; }

// A roctx range over one entry point (host time of the call; visible to
// rocprofv3 --marker-trace, free when no tool is attached).
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

bool box_inside(int lo, int n, int a, int b) { return n >= 1 && lo >= a && lo + n - 1 <= b; }

void validate(const fdtd_config &c) {
  if (c.abi_version != FDTD_ABI_VERSION) throw einval("abi_version mismatch");
  if (c.dims != 2 && c.dims != 3) throw einval("dims must be 2 or 3");
  if (c.precision != 32 && c.precision != 64) throw einval("precision must be 32 or 64");
  if (c.n_steps < 1) throw einval("n_steps < 1");
  if (c.n_freq < 1) throw einval("n_freq < 1");
  if (!(c.dx > 0)) throw einval("dx <= 0");
  const double lim = 1.0 / std::sqrt((double)c.dims);
  if (!(c.courant > 0) || !(c.courant < lim)) throw einval("Courant number outside (0, 1/sqrt(dims))");
  if (!(c.eps_s > 0) || !(c.eps_g > 0) || !(c.eps_inf > 0)) throw einval("permittivity <= 0");
  if (c.psi_s_ratio < 0 || c.sigma_max < 0 || c.gamma_mult < 0 || c.gamma_p < 0 || c.omega_p < 0 ||
      !(c.psi_s_ratio > 0 || c.omega_p == 0))
    throw einval("invalid Drude parameters (psi_s_ratio must be > 0)");
  if (c.pml_cells < 0 || c.tfsf_margin < 0) throw einval("negative pml_cells / tfsf_margin");
  if (c.ckpt_every < 0) throw einval("ckpt_every < 0");
  if (c.source_kind != FDTD_SRC_GAUSS && c.source_kind != FDTD_SRC_SINC_HANN && c.source_kind != FDTD_SRC_NONE)
    throw einval("unknown source_kind");
  // the update kernels inject the plane wave with E along z travelling +y
  // (TMz), E along x travelling +y (TEz, pol_axis = x in 2D) or E along x
  // travelling +z (3D)
  const bool te2 = c.dims == 2 && c.pol_axis == FDTD_AXIS_X;
  const int pol = c.dims == 2 ? (te2 ? FDTD_AXIS_X : FDTD_AXIS_Z) : FDTD_AXIS_X;
  const int prop = c.dims == 2 ? FDTD_AXIS_Y : FDTD_AXIS_Z;
  if ((c.pol_axis != FDTD_AXIS_DEFAULT && c.pol_axis != pol) || (c.prop_axis != FDTD_AXIS_DEFAULT && c.prop_axis != prop))
    throw einval(c.dims == 2 ? "2D runs with pol_axis = z (TMz) or x (TEz) and prop_axis = y (or -1)"
                             : "3D runs with pol_axis = x and prop_axis = z (or -1)");
  if (te2 && c.ckpt_every > 0) throw einval("checkpointing is not built for TEz contexts");
  if (c.objective_kind != FDTD_OBJ_DFT && c.objective_kind != FDTD_OBJ_TIME_ENERGY) throw einval("unknown objective_kind");
  if (c.weight_kind != FDTD_W_ENHANCEMENT && c.weight_kind != FDTD_W_UNIT) throw einval("unknown weight_kind");
  if (!(c.f_hi > c.f_lo) || !(c.f_lo > 0)) throw einval("band edges must satisfy 0 < f_lo < f_hi");
  for (int a = 0; a < c.dims; ++a)
    if (c.n[a] < 8) throw einval("grid too small");
}

template <typename T>
void upload(hipStream_t s, DevBuf &b, const std::vector<T> &v) {
  b.alloc(v.size() * sizeof(T));
  FDTD_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

template <typename T>
void build_axis_tables(fdtd_ctx *c) {
  AxisTables<T> ax, ay;
  ax.build(c->cfg, c->dt, c->nx, c->cfg.pml_cells);
  ay.build(c->cfg, c->dt, c->ny, c->cfg.pml_cells);
  const std::vector<T> *v[12] = {&ax.be, &ax.ae, &ax.ike, &ax.bh, &ax.ah, &ax.ikh,
                                 &ay.be, &ay.ae, &ay.ike, &ay.bh, &ay.ah, &ay.ikh};
  for (int k = 0; k < 12; ++k) upload(c->stream, c->axis[k], *v[k]);
}

template <typename T>
void fill_params2d(fdtd_ctx *c, Step2D<T> &p, bool rerun) {
  const fdtd_config &g = c->cfg;
  p.nx = c->nx; p.ny = c->ny; p.pitch = c->pitch; p.P = g.pml_cells;
  p.dx0 = g.design_lo[0]; p.dy0 = g.design_lo[1]; p.dnx = g.design_n[0]; p.dny = g.design_n[1];
  p.gx0 = g.gap_lo[0]; p.gy0 = g.gap_lo[1]; p.gnx = g.gap_n[0]; p.gny = g.gap_n[1];
  p.ia = c->ia; p.ib = c->ib; p.ja = c->ja; p.jb = c->jb; p.jref = c->jref; p.L = c->L;
  p.tf_on = g.source_kind != FDTD_SRC_NONE;
  p.K = c->K; p.ng = c->ng;
  for (int b = 0; b < 2; ++b) {
    DevBuf *f = rerun ? c->fldR[b] : c->fld[b], *m = rerun ? c->pmlR[b] : c->pml[b];
    p.ez[b] = f[0].as<T>(); p.hx[b] = f[1].as<T>(); p.hy[b] = f[2].as<T>();
    p.pex[b] = m[0].as<T>(); p.pey[b] = m[1].as<T>();
    p.phx[b] = m[2].as<T>(); p.phy[b] = m[3].as<T>();
  }
  p.hist_base = 0;
  p.hist_on = 1;
  p.J = (rerun ? c->JR : c->J).as<T>(); p.rho = c->rho.as<T>(); p.hist = c->hist.as<T>(); p.grad = c->grad.as<double>();
  p.gapE = c->gapE.as<double>();
  p.asrc = c->asrc.as<T>(); p.einc = c->einc.as<T>(); p.hinc = c->hinc.as<T>();
  const T **ax[12] = {&p.bxe, &p.axe, &p.ikxe, &p.bxh, &p.axh, &p.ikxh, &p.bye, &p.aye, &p.ikye, &p.byh, &p.ayh, &p.ikyh};
  for (int k = 0; k < 12; ++k) *ax[k] = c->axis[k].as<T>();
  const double dt = c->dt, dx = g.dx;
  const double psi = g.omega_p * g.omega_p, psi_s = g.psi_s_ratio * psi;
  const double gam = g.gamma_mult * g.gamma_p;
  const double den = 1.0 + gam * dt / 2.0;
  p.chx = T(dt / (kMu0 * dx));
  p.ce_s = T(dt / (kEps0 * g.eps_s * dx));
  p.ce_g = T(dt / (kEps0 * g.eps_g * dx));
  p.A0 = T(2.0 * kEps0 * g.eps_s);
  p.A1 = T(2.0 * kEps0 * (g.eps_inf - g.eps_s));
  p.B0 = T(kEps0 * psi_s * dt / 2.0 / den);
  p.B1 = T(kEps0 * (psi - psi_s) * dt / 2.0 / den);
  p.Sg = T(g.sigma_max * dt);
  p.dt_ = T(dt);
  p.dtdx = T(dt / dx);
  p.kpm1 = T(-gam * dt / den);
  p.dthJ = T(dt * 0.5 * (1.0 + (1.0 - gam * dt / 2.0) / den));
  p.ga = T(-(kEps0 / dt) * (g.eps_inf - g.eps_s));
  p.gsm = T(-0.5 * g.sigma_max);
  p.rs = T(g.psi_s_ratio);
  p.dt = dt;
}

// Workgroups are dispatched round-robin to the 8 XCDs, each with its own L2,
// so list position k of a launch runs on XCD (k + const) mod 8.  Reorders
// v[lo, hi) so that the positions lo + k with one value of k mod 8 hold the
// elements of one group (group(i, e) in 0..7 for the i-th element e of the
// range; order within a group kept); positions whose group has run out take
// elements of the fullest other group.  Elements and count are unchanged.
template <typename G>
void deal_to_xcds(std::vector<int> &v, int lo, int hi, G group) {
  std::array<std::vector<int>, 8> q;
  for (int i = lo; i < hi; ++i) q[group(i - lo, v[i])].push_back(v[i]);
  std::array<size_t, 8> at{};
  for (int k = 0; k < hi - lo; ++k) {
    int x = k % 8;
    if (at[x] == q[x].size()) {
      x = -1;
      for (int y = 0; y < 8; ++y)
        if (at[y] < q[y].size() && (x < 0 || q[y].size() - at[y] > q[x].size() - at[x])) x = y;
    }
    v[lo + k] = q[x][at[x]++];
  }
}

// Two-step blocking of the plain background, read when a context is
// created: FDTD_TEMPORAL_BLOCKING=0 turns it off, =1 on; unset, 2D contexts
// use it (super-tiles) and 3D contexts do not (super-chunks: bit-identical
// but slower on the 256^3 workload, whose plain background is half the grid
// and a third of the step time).  Both schedules give the same results.
bool blocking_enabled(int dims) {
  const char *v = std::getenv("FDTD_TEMPORAL_BLOCKING");
  if (v && v[0] == '0') return false;
  if (v && v[0] == '1') return true;
  return dims == 2;
}

void create_2d(fdtd_ctx *c) {
  const fdtd_config &g = c->cfg;
  const int P = g.pml_cells, m = g.tfsf_margin;
  c->ia = P + m; c->ib = c->nx - 1 - P - m;
  c->ja = P + m; c->jb = c->ny - 1 - P - m;
  const bool tf = g.source_kind != FDTD_SRC_NONE;
  if (tf && (c->ia < 2 || c->ib - c->ia < 2 || c->ja < 3 || c->jb - c->ja < 2))
    throw einval("total-field box does not fit inside the absorber");
  // boxes: strictly inside the total-field box, or without a plane wave
  // anywhere off the absorber and the walls
  if (c->te) {
    // TEz boxes are cells whose edges include both boundary lines: node
    // ranges [lo, lo + n] strictly inside the total-field box, or without a
    // plane wave off the absorber (PEC walls allowed)
    const int xa = tf ? c->ia + 1 : P, xb = tf ? c->ib - 1 : c->nx - 1 - P;
    const int ya = tf ? c->ja + 1 : P, yb = tf ? c->jb - 1 : c->ny - 1 - P;
    const bool gap = g.gap_n[0] > 0 && g.gap_n[1] > 0;
    if (!box_inside(g.design_lo[0], g.design_n[0] + 1, xa, xb) || !box_inside(g.design_lo[1], g.design_n[1] + 1, ya, yb) ||
        (gap && (!box_inside(g.gap_lo[0], g.gap_n[0] + 1, xa, xb) || !box_inside(g.gap_lo[1], g.gap_n[1] + 1, ya, yb))))
      throw einval(tf ? "design/gap boxes must lie strictly inside the total-field box"
                      : "design/gap boxes must lie off the absorber");
  } else {
    const int xa = tf ? c->ia + 1 : P + 1, xb = tf ? c->ib - 1 : c->nx - 2 - P;
    const int ya = tf ? c->ja + 1 : P + 1, yb = tf ? c->jb - 1 : c->ny - 2 - P;
    if (!box_inside(g.design_lo[0], g.design_n[0], xa, xb) || !box_inside(g.design_lo[1], g.design_n[1], ya, yb) ||
        !box_inside(g.gap_lo[0], g.gap_n[0], xa, xb) || !box_inside(g.gap_lo[1], g.gap_n[1], ya, yb))
      throw einval(tf ? "design/gap boxes must lie strictly inside the total-field box"
                      : "design/gap boxes must lie inside the absorber and the walls");
  }
  c->pitch = (c->nx + 63) & ~63;
  if (c->te) {
    // per-edge layout: E_x edges [dny+1][dnx], then E_y edges [dny][dnx+1]
    const int dnx = g.design_n[0], dny = g.design_n[1], gnx = g.gap_n[0], gny = g.gap_n[1];
    c->nd = dnx * (dny + 1) + (dnx + 1) * dny;
    c->ng = gnx > 0 && gny > 0 ? gnx * (gny + 1) + (gnx + 1) * gny : 0;
  } else {
    c->nd = g.design_n[0] * g.design_n[1];
    c->ng = g.gap_n[0] * g.gap_n[1];
  }
  c->ncomp = 1;
  c->nmon = c->ng;
  c->jref = c->ja - 2;
  c->L = c->jb + 2 - c->jref + 1;
  const size_t n2 = (size_t)c->pitch * c->ny * c->esz;
  for (int b = 0; b < 2; ++b) {
    for (int k = 0; k < 3; ++k) c->fld[b][k].alloc(n2);
    for (int k = 0; k < 4; ++k) c->pml[b][k].alloc(n2);
    if (c->nseg > 1) {
      for (int k = 0; k < 3; ++k) c->fldR[b][k].alloc(n2);
      for (int k = 0; k < 4; ++k) c->pmlR[b][k].alloc(n2);
    }
  }
  if (c->prec == 32) build_axis_tables<float>(c); else build_axis_tables<double>(c);
  const int dbox[4] = {g.design_lo[0], g.design_lo[1], g.design_n[0], g.design_n[1]};
  const int gbox[4] = {g.gap_lo[0], g.gap_lo[1], g.gap_n[0], g.gap_n[1]};
  // without a plane wave there are no injection lines to keep clear
  Tb2dPlan pl = tf ? tb2d_plan(c->nx, c->ny, P, c->ia, c->ib, c->ja, c->jb, dbox, gbox)
                   : tb2d_plan(c->nx, c->ny, P, -8, -8, -8, -8, dbox, gbox);
  if (!pl.tb.empty() && blocking_enabled(2) && !c->te) {
    // the interior super-tiles run one launch early (beside the rest tiles'
    // second step of the previous pair), the border ones after them
    std::vector<int> order;
    for (int code : pl.tb)
      if (!(code & 1)) order.push_back(code);
    c->nEarly = (int)order.size();
    for (int code : pl.tb)
      if (code & 1) order.push_back(code);
    c->nTb = (int)order.size();
    c->nRest = (int)pl.rest.size();
    // L2 locality: each XCD takes one contiguous band of the row-major
    // super-tiles of each launch's share (neighbours' halo lines then sit in
    // the same L2), and whole rest tile-rows, the rows dealt round-robin (the
    // slow absorber and design rows spread over the XCDs).  On the 2048^2
    // workload this cut the bytes fetched per step by 41% and the time per
    // forward / adjoint step from 21.1 / 21.7 us (both lists in row-major
    // order) to 19.1 / 19.4 us.
    const int ne = c->nEarly, nl = c->nTb - c->nEarly, nbx = pl.nbx;
    deal_to_xcds(order, 0, ne, [&](int i, int) { return (int)((int64_t)i * 8 / ne); });
    deal_to_xcds(order, ne, c->nTb, [&](int i, int) { return (int)((int64_t)i * 8 / nl); });
    deal_to_xcds(pl.rest, 0, c->nRest, [&](int, int code) { return (code / nbx) % 8; });
    c->tbTiles.alloc(order.size() * sizeof(int));
    c->tbRest.alloc(std::max<size_t>(pl.rest.size(), 1) * sizeof(int));
    FDTD_HIP(hipMemcpy(c->tbTiles.p, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!pl.rest.empty())
      FDTD_HIP(hipMemcpy(c->tbRest.p, pl.rest.data(), pl.rest.size() * sizeof(int), hipMemcpyHostToDevice));
    for (int k = 0; k < 3; ++k) {
      c->fld3[k].alloc(n2);
      if (c->nseg > 1) c->fld3R[k].alloc(n2);
    }
  }
}

// Field copy holding the state after `s` steps of a solve: with two-step
// blocking three copies rotate (a pair of steps reads copy s and writes
// copy s+2, as two single steps would), else two.  Absorber memories always
// alternate between two copies.
int fcopy(const fdtd_ctx *c, int s) { return c->nTb > 0 ? s % 3 : s & 1; }

// 3D arena holding the state after `s` steps: three rotate with two-step
// blocking, else two.
int acopy(const fdtd_ctx *c, int s) { return c->nSup > 0 ? s % 3 : s & 1; }
DevBuf &arena(fdtd_ctx *c, bool rerun, int s) { return rerun ? c->arenaR[acopy(c, s)] : c->arena3[acopy(c, s)]; }


DevBuf *field_buf(fdtd_ctx *c, bool rerun, int copy, int k) {
  if (copy == 2) return rerun ? &c->fld3R[k] : &c->fld3[k];
  return rerun ? &c->fldR[copy][k] : &c->fld[copy][k];
}

template <typename T>
void build_axis_tables3(fdtd_ctx *c) {
  // packed [axis][b_E, a_E, 1/kappa_E, b_H, a_H, 1/kappa_H][tn]; entries past an
  // axis' end repeat the identity grading
  const int n3[3] = {c->nx, c->ny, c->nz};
  const int tn = std::max(c->nx, std::max(c->ny, c->nz));
  std::vector<T> all((size_t)18 * tn);
  for (int a = 0; a < 3; ++a) {
    AxisTables<T> t;
    t.build(c->cfg, c->dt, n3[a], c->cfg.pml_cells);
    const std::vector<T> *v[6] = {&t.be, &t.ae, &t.ike, &t.bh, &t.ah, &t.ikh};
    const T idv[6] = {T(1), T(0), T(1), T(1), T(0), T(1)};
    for (int k = 0; k < 6; ++k)
      for (int i = 0; i < tn; ++i) all[((size_t)a * 6 + k) * tn + i] = i < n3[a] ? (*v[k])[i] : idv[k];
  }
  c->tn3 = tn;
  upload(c->stream, c->tab3, all);
}

void release_one(Aux3D &a) {
  if (a.stream) (void)hipStreamSynchronize(a.stream);
  if (a.fork) (void)hipEventDestroy(a.fork);
  if (a.join) (void)hipEventDestroy(a.join);
  if (a.stream) (void)hipStreamDestroy(a.stream);
  a = Aux3D{nullptr, nullptr, nullptr};
}

void create_one(Aux3D &a) {
  FDTD_HIP(hipStreamCreate(&a.stream));
  FDTD_HIP(hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
  FDTD_HIP(hipEventCreateWithFlags(&a.join, hipEventDisableTiming));
}

void create_3d(fdtd_ctx *c) {
  const fdtd_config &g = c->cfg;
  const int P = g.pml_cells, m = g.tfsf_margin;
  const int n3[3] = {c->nx, c->ny, c->nz};
  const bool tf = g.source_kind != FDTD_SRC_NONE;
  for (int d = 0; d < 3; ++d) {
    c->lo3[d] = P + m;
    c->hi3[d] = n3[d] - 1 - P - m;
    if (tf && (c->lo3[d] < 3 || c->hi3[d] - c->lo3[d] < 2))
      throw einval("total-field box does not fit inside the absorber");
    const int a = tf ? c->lo3[d] + 1 : P + 1, b = tf ? c->hi3[d] - 1 : n3[d] - 2 - P;
    if (!box_inside(g.design_lo[d], g.design_n[d], a, b) || !box_inside(g.gap_lo[d], g.gap_n[d], a, b))
      throw einval(tf ? "design/gap boxes must lie strictly inside the total-field box"
                      : "design/gap boxes must lie inside the absorber and the walls");
  }
  c->pitch = ((c->nx + 31) & ~31) + FDTD3D_PITCH_PAD;
  c->nd = g.design_n[0] * g.design_n[1] * g.design_n[2];
  c->ng = g.gap_n[0] * g.gap_n[1] * g.gap_n[2];
  c->ncomp = 3;
  c->nmon = 3 * c->ng;
  c->jref = c->lo3[2] - 2;
  c->L = c->hi3[2] + 2 - c->jref + 1;
  c->lay3 = arena3_layout(c->ny, c->nz, c->pitch, P);
  // kernels address a copy with 32-bit byte offsets
  if (c->lay3.total * (uint64_t)c->esz >= (uint64_t(1) << 32))
    throw einval("3D state too large for one 4 GiB arena per copy (fields + absorber memories)");
  for (int b = 0; b < 2; ++b) {
    c->arena3[b].alloc((size_t)c->lay3.total * c->esz);
    if (c->nseg > 1) c->arenaR[b].alloc((size_t)c->lay3.total * c->esz);
  }
  if (c->prec == 32) build_axis_tables3<float>(c); else build_axis_tables3<double>(c);
  create_one(c->aux);
}

// Streams and events beyond the context stream (all at default priority).
void release_aux(fdtd_ctx *c) {
  release_one(c->aux);
  release_one(c->auxR);
  release_one(c->sup);
  release_one(c->supR);
  if (c->rr) (void)hipStreamSynchronize(c->rr);
  for (hipEvent_t *e : {&c->evStart, &c->evRerun, &c->evAdj[0], &c->evAdj[1]}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  if (c->rr) (void)hipStreamDestroy(c->rr);
  c->rr = nullptr;
  for (hipEvent_t *e : {&c->evWatch[0], &c->evWatch[1]}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  if (c->watch_host) (void)hipHostFree(c->watch_host);
  c->watch_host = nullptr;
}

template <typename T>
void fill_params3d(fdtd_ctx *c, Step3D<T> &p, bool rerun) {
  const fdtd_config &g = c->cfg;
  p.n[0] = c->nx; p.n[1] = c->ny; p.n[2] = c->nz;
  p.pitch = c->pitch;
  p.P = g.pml_cells;
  for (int d = 0; d < 3; ++d) {
    p.d0[d] = g.design_lo[d]; p.dn[d] = g.design_n[d];
    p.g0[d] = g.gap_lo[d]; p.gn[d] = g.gap_n[d];
    p.lo[d] = c->lo3[d]; p.hi[d] = c->hi3[d];
  }
  p.kref = c->jref; p.L = c->L; p.tf_on = g.source_kind != FDTD_SRC_NONE; p.ng = c->ng;
  const Arena3 &a = c->lay3;
  p.G0 = a.G0; p.S = a.S; p.PL = a.PL; p.xs = a.xs; p.ys = a.ys; p.zs = a.zs;
  p.XS = a.XS; p.YS = a.YS; p.ZS = a.ZS; p.W = a.W;
  p.A[0] = (rerun ? c->arenaR[0] : c->arena3[0]).as<T>();
  p.A[1] = (rerun ? c->arenaR[1] : c->arena3[1]).as<T>();
  p.hist_base = 0;
  p.hist_on = 1;
  p.J = (rerun ? c->JR : c->J).as<T>(); p.rho = c->rho.as<T>(); p.hist = c->hist.as<T>(); p.grad = c->grad.as<double>();
  p.gapE = c->gapE.as<double>(); p.asrc = c->asrc.as<T>(); p.einc = c->einc.as<T>(); p.hinc = c->hinc.as<T>();
  p.tab = c->tab3.as<T>();
  p.tn = c->tn3;
  if (!c->glist3.p) {
    int nS = 0, nM = 0, nD = 0, axD = 0;
    const std::vector<int> lists = gen3d_plan(p, nS, nM, nD, axD);
    upload(c->stream, c->glist3, lists);
    FDTD_HIP(hipStreamSynchronize(c->stream));
    c->gS = nS; c->gM = nM; c->gD = nD; c->gAxD = axD;
  }
  p.glist = c->glist3.as<int>();
  p.gS = c->gS; p.gM = c->gM; p.gD = c->gD; p.gAxD = c->gAxD;
  plain3d_box(p, p.pb);
  if (!c->sup_planned) {
    c->sup_planned = true;
    if (c->prec == 32 && blocking_enabled(3)) {
      std::vector<unsigned char> flags;
      const std::vector<int> list = plan3d_super(p, c->so3, c->sn3, flags);
      c->nSup = (int)list.size();
      if (c->nSup > 0) {
        upload(c->stream, c->sup_list, list);
        upload(c->stream, c->sup_flags, flags);
        FDTD_HIP(hipStreamSynchronize(c->stream));
        c->arena3[2].alloc((size_t)c->lay3.total * c->esz);
        if (c->nseg > 1) c->arenaR[2].alloc((size_t)c->lay3.total * c->esz);
        create_one(c->sup);
        if (c->nseg > 1) create_one(c->supR);
      }
    }
  }
  p.sflag = c->nSup > 0 ? c->sup_flags.as<unsigned char>() : nullptr;
  for (int a = 0; a < 3; ++a) {
    p.so[a] = c->so3[a];
    p.sn[a] = c->nSup > 0 ? c->sn3[a] : 0;
  }
  p.skip_super = 0;
  p.Amid = nullptr;
  const double dt = c->dt, dx = g.dx;
  const double psi = g.omega_p * g.omega_p, psi_s = g.psi_s_ratio * psi;
  const double gam = g.gamma_mult * g.gamma_p;
  const double den = 1.0 + gam * dt / 2.0;
  p.ch = T(dt / (kMu0 * dx));
  p.ce_s = T(dt / (kEps0 * g.eps_s * dx));
  p.ce_g = T(dt / (kEps0 * g.eps_g * dx));
  p.A0 = T(2.0 * kEps0 * g.eps_s);
  p.A1 = T(2.0 * kEps0 * (g.eps_inf - g.eps_s));
  p.B0 = T(kEps0 * psi_s * dt / 2.0 / den);
  p.B1 = T(kEps0 * (psi - psi_s) * dt / 2.0 / den);
  p.Sg = T(g.sigma_max * dt);
  p.dt_ = T(dt);
  p.dtdx = T(dt / dx);
  p.kpm1 = T(-gam * dt / den);
  p.dthJ = T(dt * 0.5 * (1.0 + (1.0 - gam * dt / 2.0) / den));
  p.ga = T(-(kEps0 / dt) * (g.eps_inf - g.eps_s));
  p.gsm = T(-0.5 * g.sigma_max);
  p.rs = T(g.psi_s_ratio);
}

void create_common(fdtd_ctx *c) {
  const fdtd_config &g = c->cfg;
  hipStream_t s = c->stream;
  c->J.alloc((size_t)c->nd * c->ncomp * c->esz);
  c->rho.alloc((size_t)c->nd * c->esz);
  c->grad.alloc((size_t)c->nd * c->ncomp * sizeof(double));
  // history of ck steps (all N without checkpoints) plus nseg-1 snapshots
  const int hist_steps = c->nseg > 1 ? c->ck : c->N;
  const double hist_bytes = (double)hist_steps * c->nd * c->ncomp * c->esz;
  if (c->nseg > 1) {
    c->JR.alloc(c->J.bytes);
    c->snap_bytes = c->J.bytes;
    for (int b = 0; b < 1; ++b) {
      if (c->dims == 2) {
        for (int k = 0; k < 3; ++k) c->snap_bytes += c->fld[b][k].bytes;
        for (int k = 0; k < 4; ++k) c->snap_bytes += c->pml[b][k].bytes;
      } else {
        c->snap_bytes += c->arena3[b].bytes;
      }
    }
  }
  const double snap_total = (double)(c->nseg - 1) * c->snap_bytes;
  if (g.history_budget_bytes > 0 && hist_bytes + snap_total > (double)g.history_budget_bytes)
    throw Error{FDTD_ENOMEM, "forward history and snapshots (" + std::to_string(hist_bytes + snap_total) +
                                 " bytes) exceed history_budget_bytes"};
  size_t fr = 0, tot = 0;
  FDTD_HIP(hipMemGetInfo(&fr, &tot));
  if (hist_bytes + snap_total > 0.92 * (double)fr)
    throw Error{FDTD_ENOMEM, "forward history and snapshots do not fit in device memory"};
  c->hist.alloc((size_t)hist_bytes);
  if (c->nseg > 1) c->snap.alloc((size_t)snap_total);
  // a second segment history lets the re-run of segment s-1 overlap the
  // adjoint of segment s, where the budget and the memory allow it
  const double two = 2 * hist_bytes + snap_total;
  if (c->nseg > 1 && (g.history_budget_bytes <= 0 || two <= (double)g.history_budget_bytes) && two <= 0.92 * (double)fr) {
    c->hist2.alloc((size_t)hist_bytes);
    FDTD_HIP(hipStreamCreate(&c->rr));
    for (hipEvent_t *e : {&c->evStart, &c->evRerun, &c->evAdj[0], &c->evAdj[1]})
      FDTD_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    if (c->dims == 3) create_one(c->auxR);
  }
  c->dft.alloc((size_t)c->K * c->nmon * 2 * sizeof(double));
  c->gapE.alloc((size_t)(c->N + 1) * c->nmon * sizeof(double));
  c->asrc.alloc((size_t)(c->N + 1) * c->nmon * c->esz);
  c->scal.alloc(64);
  c->bad.alloc(64);
  c->Fdev.alloc(64);
  c->gtmp.alloc((size_t)c->nd * c->esz);
  // excitation samples, frequencies, phasors, weights
  std::vector<double> wave(c->N + 2);
  for (int n = 0; n <= c->N + 1; ++n) wave[n] = source_wave(g, n * c->dt);
  upload(s, c->gwave, wave);
  upload(s, c->dfreq, c->freqs);
  c->phasor.alloc((size_t)(c->N + 1) * c->K * 2 * sizeof(double));
  launch_phasors(s, c->dfreq.as<double>(), c->K, c->N, c->dt, c->phasor.as<double>());
  c->wts.alloc((size_t)c->K * sizeof(double));
  launch_weights(s, c->gwave.as<double>(), c->dfreq.as<double>(), c->K, c->N, c->dt,
                 g.weight_kind == FDTD_W_UNIT || g.source_kind == FDTD_SRC_NONE, c->wts.as<double>());
  // watchdog slots: one per check of the forward solve (every kWatchEvery
  // steps and after the last)
  c->watch_slots = (c->N + kWatchEvery - 1) / kWatchEvery;
  c->watch.alloc((size_t)c->watch_slots * sizeof(unsigned long long));
  FDTD_HIP(hipHostMalloc((void **)&c->watch_host, (size_t)c->watch_slots * sizeof(unsigned long long),
                         hipHostMallocDefault));
  for (hipEvent_t *e : {&c->evWatch[0], &c->evWatch[1]}) FDTD_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  // incident line: node p <-> main-grid index jref + p; far-end absorber of 20 cells
  const int P1 = 20, n1 = c->L + P1 + 1;
  std::vector<double> prof(6 * (size_t)n1);
  for (int p = 0; p < n1; ++p) {
    const double start = n1 - 1 - P1;
    const double de = (p - start) / P1, dh = (p + 0.5 - start) / P1;
    Grade ge{1, 0, 1}, gh{1, 0, 1};
    if (de > 0) ge = pml_grade(g, c->dt, de);
    if (dh > 0) gh = pml_grade(g, c->dt, dh);
    prof[p] = ge.b; prof[n1 + p] = ge.a; prof[2 * n1 + p] = 1.0 / ge.kap;
    prof[3 * n1 + p] = gh.b; prof[4 * n1 + p] = gh.a; prof[5 * n1 + p] = 1.0 / gh.kap;
  }
  upload(s, c->lineprof, prof);
  c->linescr.alloc(4 * (size_t)n1 * sizeof(double));
  c->einc.alloc((size_t)(c->N + 1) * c->L * c->esz);
  c->hinc.alloc((size_t)c->N * c->L * c->esz);
  launch_incident_line(s, c->prec, c->gwave.as<double>(), c->N, n1, c->L, c->lineprof.as<double>(),
                       c->dt / (kMu0 * g.dx), c->dt / (kEps0 * g.eps_s * g.dx), 0.0, 0.0,
                       c->linescr.as<double>(), c->einc.p, c->hinc.p);
}

void zero(fdtd_ctx *c, DevBuf &b) { launch_fill_zero(c->stream, b.p, b.bytes); }

void zero_state(fdtd_ctx *c) {
  for (int b = 0; b < 2; ++b) {
    for (int k = 0; k < 6; ++k) if (c->fld[b][k].p) zero(c, c->fld[b][k]);
    for (int k = 0; k < 12; ++k) if (c->pml[b][k].p) zero(c, c->pml[b][k]);
  }
  for (int b = 0; b < 3; ++b)
    if (c->arena3[b].p) zero(c, c->arena3[b]);
  for (int k = 0; k < 3; ++k) if (c->fld3[k].p) zero(c, c->fld3[k]);
  zero(c, c->J);
}

// ------------------------------------------------ test-only state access
// Fields of the fdtd_set_state layout: 2D TMz E_z, H_x, H_y, J_z; 2D TEz E_x,
// E_y, H_z, J_x, J_y; 3D E_x, E_y, E_z, H_x, H_y, H_z, J_x, J_y, J_z.
int state_fields(const fdtd_ctx *c) { return c->te ? 5 : c->dims == 2 ? 4 : 9; }

// E and H fields of the layout (the rest are currents).
int state_efields(const fdtd_ctx *c) { return c->dims == 2 ? 3 : 6; }

// Is node (i, j, k) of E/H field f one the update writes (off the PEC walls)?
bool state_node(const fdtd_ctx *c, int f, int i, int j, int k) {
  const int n3[3] = {c->nx, c->ny, c->nz};
  const int x[3] = {i, j, k};
  if (c->te) {
    // E_x: [0, nx-2] x [1, ny-2]; E_y: [1, nx-2] x [0, ny-2]; H_z: [0, nx-2] x [0, ny-2]
    const bool ix = f == 1 ? i >= 1 && i <= c->nx - 2 : i <= c->nx - 2;
    const bool jy = f == 0 ? j >= 1 && j <= c->ny - 2 : j <= c->ny - 2;
    return ix && jy;
  }
  if (c->dims == 2) {
    const bool ix = f == 2 ? i <= c->nx - 2 : i >= 1 && i <= c->nx - 2;
    const bool jy = f == 1 ? j <= c->ny - 2 : j >= 1 && j <= c->ny - 2;
    return ix && jy;
  }
  const int comp = f % 3;
  const bool isE = f < 3;
  for (int d = 0; d < 3; ++d) {
    // E_c: [0, n-2] along c, [1, n-2] across; H_c: [1, n-2] along c, [0, n-2] across
    const int lo = (d == comp) == isE ? 0 : 1;
    if (x[d] < lo || x[d] > n3[d] - 2) return false;
  }
  return true;
}

// Index into the context's J array of the Drude edge of component `comp` at
// node (i, j, k), or -1 when the node is not a Drude design edge.
int64_t drude_index(const fdtd_ctx *c, int comp, int i, int j, int k) {
  const fdtd_config &g = c->cfg;
  if (c->te) {
    // the edge's density index (E_x block, then E_y block), off the gap's edges
    const int u = i - g.design_lo[0], v = j - g.design_lo[1], dnx = g.design_n[0], dny = g.design_n[1];
    const int gu = i - g.gap_lo[0], gv = j - g.gap_lo[1], gnx = g.gap_n[0], gny = g.gap_n[1];
    const bool gp = gnx > 0 && gny > 0;
    if (comp == 0) {
      if (u < 0 || u >= dnx || v < 0 || v > dny) return -1;
      if (gp && gu >= 0 && gu < gnx && gv >= 0 && gv <= gny) return -1;
      return (int64_t)v * dnx + u;
    }
    if (u < 0 || u > dnx || v < 0 || v >= dny) return -1;
    if (gp && gu >= 0 && gu <= gnx && gv >= 0 && gv < gny) return -1;
    return (int64_t)dnx * (dny + 1) + (int64_t)v * (dnx + 1) + u;
  }
  const int x[3] = {i, j, k};
  int64_t d = 0, stride = 1;
  bool gap = true;
  for (int a = 0; a < c->dims; ++a) {
    const int u = x[a] - g.design_lo[a];
    if (u < 0 || u >= g.design_n[a]) return -1;
    d += u * stride;
    stride *= g.design_n[a];
    gap = gap && x[a] >= g.gap_lo[a] && x[a] < g.gap_lo[a] + g.gap_n[a];
  }
  return gap ? -1 : (int64_t)comp * c->nd + d;
}

// Offset (elements) of node (i, j, k) of field f in one state copy: the
// pitched 2D array of that field, or the 3D arena.
size_t state_offset(const fdtd_ctx *c, int f, int i, int j, int k) {
  if (c->dims == 2) return (size_t)j * c->pitch + i;
  return (size_t)c->lay3.G0 + (size_t)f * c->lay3.S + (size_t)k * c->lay3.PL + (size_t)j * c->pitch + i;
}

// Copy the initial state (host, double) into state copy 0 and J.
template <typename T>
void upload_init_state(fdtd_ctx *c) {
  const size_t cells = (size_t)c->nx * c->ny * c->nz;
  const double *st = c->init_state.data();
  const int nfe = state_efields(c);
  std::vector<T> jv((size_t)c->nd * c->ncomp, T(0));
  for (int comp = 0; comp < state_fields(c) - nfe; ++comp)
    for (int k = 0; k < c->nz; ++k)
      for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
          const int64_t d = drude_index(c, c->dims == 2 && !c->te ? 0 : comp, i, j, k);
          if (d >= 0) jv[d] = T(st[(size_t)(nfe + comp) * cells + ((size_t)k * c->ny + j) * c->nx + i]);
        }
  std::vector<std::vector<T>> img(c->dims == 2 ? 3 : 1);
  for (auto &v : img) v.assign(c->dims == 2 ? (size_t)c->pitch * c->ny : (size_t)c->lay3.total, T(0));
  for (int f = 0; f < nfe; ++f)
    for (int k = 0; k < c->nz; ++k)
      for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i)
          if (state_node(c, f, i, j, k))
            img[c->dims == 2 ? f : 0][state_offset(c, f, i, j, k)] = T(st[(size_t)f * cells + ((size_t)k * c->ny + j) * c->nx + i]);
  for (size_t b = 0; b < img.size(); ++b) {
    DevBuf *dst = c->dims == 2 ? field_buf(c, false, 0, (int)b) : &c->arena3[0];
    FDTD_HIP(hipMemcpyAsync(dst->p, img[b].data(), img[b].size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  }
  FDTD_HIP(hipMemcpyAsync(c->J.p, jv.data(), jv.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  FDTD_HIP(hipStreamSynchronize(c->stream));
}

// The state after the last forward solve into `out` (fdtd_set_state layout).
template <typename T>
void download_state(fdtd_ctx *c, double *out) {
  const size_t cells = (size_t)c->nx * c->ny * c->nz;
  const int nfe = state_efields(c);
  std::vector<std::vector<T>> img(c->dims == 2 ? 3 : 1);
  for (size_t b = 0; b < img.size(); ++b) {
    DevBuf *src = c->dims == 2 ? field_buf(c, false, fcopy(c, c->N), (int)b) : &arena(c, false, c->N);
    img[b].resize(src->bytes / sizeof(T));
    FDTD_HIP(hipMemcpyAsync(img[b].data(), src->p, src->bytes, hipMemcpyDeviceToHost, c->stream));
  }
  std::vector<T> jv((size_t)c->nd * c->ncomp);
  FDTD_HIP(hipMemcpyAsync(jv.data(), c->J.p, jv.size() * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  FDTD_HIP(hipStreamSynchronize(c->stream));
  for (int f = 0; f < state_fields(c); ++f)
    for (int k = 0; k < c->nz; ++k)
      for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
          double v = 0.0;
          if (f < nfe) {
            if (state_node(c, f, i, j, k)) v = (double)img[c->dims == 2 ? f : 0][state_offset(c, f, i, j, k)];
          } else {
            const int64_t d = drude_index(c, c->dims == 2 && !c->te ? 0 : f - nfe, i, j, k);
            if (d >= 0) v = (double)jv[d];
          }
          out[(size_t)f * cells + ((size_t)k * c->ny + j) * c->nx + i] = v;
        }
}

template <typename T>
Step2D<T> &params2d(fdtd_ctx *c, bool rerun);
template <>
Step2D<float> &params2d<float>(fdtd_ctx *c, bool rerun) { return rerun ? c->p2fR : c->p2f; }
template <>
Step2D<double> &params2d<double>(fdtd_ctx *c, bool rerun) { return rerun ? c->p2dR : c->p2d; }
template <typename T>
Step3D<T> &params3d(fdtd_ctx *c, bool rerun);
template <>
Step3D<float> &params3d<float>(fdtd_ctx *c, bool rerun) { return rerun ? c->p3fR : c->p3f; }
template <>
Step3D<double> &params3d<double>(fdtd_ctx *c, bool rerun) { return rerun ? c->p3dR : c->p3d; }

// Where a block of steps runs: its stream, the 3D side streams (general
// launches; two-step pass), and the history buffer the design edges write
// (forward) or read (adjoint).
struct Lane {
  hipStream_t s;
  const Aux3D *aux, *sup;
  void *hist;
};
Lane main_lane(fdtd_ctx *c) { return Lane{c->stream, &c->aux, &c->sup, c->hist.p}; }

// 2D parameters of the step that follows `s` steps of a solve: copy 0 read,
// copy 1 written, parities resolved.
template <typename T>
Step2D<T> params2d_at(fdtd_ctx *c, bool rerun, int s, int hist_base, bool hist_on, void *hist) {
  Step2D<T> p = params2d<T>(c, rerun);
  p.hist = static_cast<T *>(hist);
  const int fr = fcopy(c, s), fw = fcopy(c, s + 1);
  p.ez[0] = field_buf(c, rerun, fr, 0)->as<T>(); p.ez[1] = field_buf(c, rerun, fw, 0)->as<T>();
  p.hx[0] = field_buf(c, rerun, fr, 1)->as<T>(); p.hx[1] = field_buf(c, rerun, fw, 1)->as<T>();
  p.hy[0] = field_buf(c, rerun, fr, 2)->as<T>(); p.hy[1] = field_buf(c, rerun, fw, 2)->as<T>();
  const int mr = s & 1, mw = mr ^ 1;
  DevBuf *m0 = rerun ? c->pmlR[mr] : c->pml[mr], *m1 = rerun ? c->pmlR[mw] : c->pml[mw];
  p.pex[0] = m0[0].as<T>(); p.pex[1] = m1[0].as<T>();
  p.pey[0] = m0[1].as<T>(); p.pey[1] = m1[1].as<T>();
  p.phx[0] = m0[2].as<T>(); p.phx[1] = m1[2].as<T>();
  p.phy[0] = m0[3].as<T>(); p.phy[1] = m1[3].as<T>();
  p.hist_base = hist_base;
  p.hist_on = hist_on;
  return p;
}

// One time step (step number n, the (s+1)-th of its solve) on the main state
// (rerun = false) or the re-run state.
template <typename T>
void launch_step(fdtd_ctx *c, bool rerun, int n, int s, bool adjoint, int hist_base, bool hist_on, const Lane &ln) {
  if (c->te) {
    launch_step_te<T>(params2d_at<T>(c, rerun, s, hist_base, hist_on, ln.hist), n, adjoint, ln.s);
  } else if (c->dims == 2) {
    // a single step updates every tile (the super-tiles take the background
    // update of the per-step kernel)
    launch_step2d<T>(params2d_at<T>(c, rerun, s, hist_base, hist_on, ln.hist), n, 0, adjoint, ln.s);
  } else {
    Step3D<T> p = params3d<T>(c, rerun);
    p.hist = static_cast<T *>(ln.hist);
    p.hist_base = hist_base;
    p.hist_on = hist_on;
    launch_step3d<T>(p, arena(c, rerun, s).as<T>(), arena(c, rerun, s + 1).as<T>(), n, adjoint, ln.s, *ln.aux);
  }
}

// `count` consecutive time steps of a solve, the first one the (s0+1)-th:
// step j has step number nof(j), history base hbase and history flag hon(j).
// With two-step blocking (2D, nTb > 0) the steps go in pairs, pipelined two
// launches per pair: launch A of pair q = the rest tiles' first step of q and
// the border super-tiles of q (all super-tiles for the first pair); launch B
// = the rest tiles' second step of q and the interior super-tiles of pair
// q+1, run early.  Those reach only other super-tiles, whose state after the
// pair is already written, and write their output into the copy that the
// rest tiles read in that launch only outside the super-tiles.  An odd last
// step is a full-grid single step.
//
// In 3D with super-chunks (FP32) a pair is the two-step pass over the
// super-chunks (state after s0+2q read, after s0+2q+2 written, border nodes
// also after s0+2q+1) on the lane's pass stream, beside the first per-step
// update of the other nodes, and the second per-step update after both.
// The three arenas make the pass's reads and writes disjoint from those of
// the first per-step update.
template <typename T, typename NOF, typename HON>
void run_block(fdtd_ctx *c, bool rerun, bool adjoint, int s0, int count, NOF nof, int hbase, HON hon,
               const Lane &ln) {
  if constexpr (std::is_same<T, float>::value) {
    if (c->dims == 3 && c->nSup > 0) {
      const int P = count / 2;
      for (int q = 0; q < P; ++q) {
        const int s = s0 + 2 * q;
        Step3D<float> p = params3d<float>(c, rerun);
        p.hist = static_cast<float *>(ln.hist);
        p.hist_base = hbase;
        const Aux3D &sp = *ln.sup;
        FDTD_HIP(hipEventRecord(sp.fork, ln.s));
        FDTD_HIP(hipStreamWaitEvent(sp.stream, sp.fork, 0));
        launch_step3d_super(p, arena(c, rerun, s).as<float>(), arena(c, rerun, s + 1).as<float>(),
                            arena(c, rerun, s + 2).as<float>(), c->sup_list.as<int>(), c->nSup, sp.stream);
        FDTD_HIP(hipEventRecord(sp.join, sp.stream));
        p.skip_super = 1;
        for (int h = 0; h < 2; ++h) {
          if (h == 1) FDTD_HIP(hipStreamWaitEvent(ln.s, sp.join, 0));
          p.hist_on = hon(2 * q + h);
          launch_step3d<float>(p, arena(c, rerun, s + h).as<float>(), arena(c, rerun, s + h + 1).as<float>(),
                               nof(2 * q + h), adjoint, ln.s, *ln.aux);
        }
      }
      if (count & 1) launch_step<T>(c, rerun, nof(count - 1), s0 + count - 1, adjoint, hbase, hon(count - 1), ln);
      return;
    }
  }
  if (c->dims != 2 || c->nTb == 0) {
    for (int j = 0; j < count; ++j) launch_step<T>(c, rerun, nof(j), s0 + j, adjoint, hbase, hon(j), ln);
    return;
  }
  const int P = count / 2;
  const int *tiles = c->tbTiles.as<int>();
  auto step = [&](int j) {
    Step2D<T> p = params2d_at<T>(c, rerun, s0 + j, hbase, hon(j), ln.hist);
    p.tlist = c->tbRest.as<int>();
    return p;
  };
  auto out = [&](int q, int k) { return field_buf(c, rerun, fcopy(c, s0 + 2 * q + 2), k)->as<T>(); };
  for (int q = 0; q < P; ++q) {
    // launch A of pair q
    const Step2D<T> pa = step(2 * q), pt = params2d_at<T>(c, rerun, s0 + 2 * q, hbase, hon(2 * q), ln.hist);
    const int first = q == 0 ? 0 : c->nEarly;
    launch_step2d_mix<T>(pa, nof(2 * q), c->nRest, pt, tiles + first, c->nTb - first, out(q, 0), out(q, 1),
                         out(q, 2), adjoint, ln.s);
    // launch B of pair q (+ the interior super-tiles of pair q+1)
    const Step2D<T> pb = step(2 * q + 1);
    const bool next = q + 1 < P;
    const Step2D<T> pn = next ? params2d_at<T>(c, rerun, s0 + 2 * q + 2, hbase, hon(2 * q + 2), ln.hist) : pt;
    launch_step2d_mix<T>(pb, nof(2 * q + 1), c->nRest, pn, tiles, next ? c->nEarly : 0,
                         next ? out(q + 1, 0) : nullptr, next ? out(q + 1, 1) : nullptr,
                         next ? out(q + 1, 2) : nullptr, adjoint, ln.s);
  }
  if (count & 1) launch_step<T>(c, rerun, nof(count - 1), s0 + count - 1, adjoint, hbase, hon(count - 1), ln);
}

// The buffers holding the state after `st` steps of a solve (fields and
// absorber memories) followed by J.
std::vector<DevBuf *> state_bufs(fdtd_ctx *c, int st, bool rerun) {
  std::vector<DevBuf *> v;
  if (c->dims == 2) {
    for (int k = 0; k < 3; ++k) v.push_back(field_buf(c, rerun, fcopy(c, st), k));
    for (int k = 0; k < 4; ++k) v.push_back(rerun ? &c->pmlR[st & 1][k] : &c->pml[st & 1][k]);
  } else {
    v.push_back(&arena(c, rerun, st));
  }
  v.push_back(rerun ? &c->JR : &c->J);
  return v;
}

// Snapshot s <- the main state after `st` steps (the start of segment s).
void snap_save(fdtd_ctx *c, int st, int s) {
  char *dst = (char *)c->snap.p + (size_t)s * c->snap_bytes;
  for (DevBuf *d : state_bufs(c, st, false)) {
    FDTD_HIP(hipMemcpyAsync(dst, d->p, d->bytes, hipMemcpyDeviceToDevice, c->stream));
    dst += d->bytes;
  }
}

// Re-run state after `st` steps <- snapshot s.
void snap_load(fdtd_ctx *c, int st, int s, hipStream_t stream) {
  const char *src = (const char *)c->snap.p + (size_t)s * c->snap_bytes;
  for (DevBuf *d : state_bufs(c, st, true)) {
    FDTD_HIP(hipMemcpyAsync(d->p, src, d->bytes, hipMemcpyDeviceToDevice, stream));
    src += d->bytes;
  }
}

// History buffer of segment s: with a second buffer, segments alternate.
void *seg_hist(fdtd_ctx *c, int s) { return c->hist2.p && (s & 1) ? c->hist2.p : c->hist.p; }

// Forward solve: step n reads the state after n steps and writes the state
// after n+1.  With checkpoints the state entering each segment but the last is
// saved, and only the last segment's history is kept.  With two-step
// blocking, steps go in pairs that never straddle a saved state.
// Watchdog of a forward solve.  After every chunk of steps the largest |E|
// of the state is reduced into a device slot and copied to pinned host
// memory behind an event; the host reads slot q-1 right after enqueueing
// chunk q, so the device always has a chunk queued and no step waits for
// the host.  A non-finite value or one above the limit stops the solve.
struct ForwardWatch {
  fdtd_ctx *c;
  double limit;
  int slots = 0;
  std::vector<int> step;  // step count each slot checked
  ForwardWatch(fdtd_ctx *ctx, double lim) : c(ctx), limit(lim) {
    launch_fill_zero(c->stream, c->watch.p, c->watch.bytes);
  }
  void enqueue(int s) {  // the state after s steps
    if (slots >= c->watch_slots) throw Error{FDTD_EDEVICE, "watchdog: more checks than slots"};
    unsigned long long *slot = c->watch.as<unsigned long long>() + slots;
    if (c->dims == 2) {
      // TMz: E_z; TEz: E_x and E_y (the two checks share the slot's maximum)
      for (int k = 0; k < (c->te ? 2 : 1); ++k) {
        DevBuf *e = field_buf(c, false, fcopy(c, s), k);
        launch_watch(c->stream, c->prec, e->p, e->bytes / c->esz, slot);
      }
    } else {
      const char *e = arena(c, false, s).as<char>() + (size_t)c->lay3.G0 * c->esz;
      launch_watch(c->stream, c->prec, e, (size_t)3 * c->lay3.S, slot);
    }
    FDTD_HIP(hipMemcpyAsync(c->watch_host + slots, slot, sizeof(*slot), hipMemcpyDeviceToHost, c->stream));
    FDTD_HIP(hipEventRecord(c->evWatch[slots & 1], c->stream));
    step.push_back(s);
    if (++slots >= 2) check(slots - 2);
  }
  void check(int q) {
    FDTD_HIP(hipEventSynchronize(c->evWatch[q & 1]));
    const unsigned long long bits = c->watch_host[q];
    double v;
    std::memcpy(&v, &bits, sizeof v);
    if (!(v <= limit)) {
      FDTD_HIP(hipStreamSynchronize(c->stream));
      char msg[160];
      std::snprintf(msg, sizeof msg, "watchdog: max |E| = %.3e after step %d (limit %.3e)", v, step[q], limit);
      throw Error{FDTD_EUNSTABLE, msg};
    }
  }
  void finish() {
    if (slots >= 1) check(slots - 1);
  }
};

template <typename T>
void run_forward(fdtd_ctx *c, double limit) {
  FDTD_HIP(hipEventRecord(c->ev[0], c->stream));
  const int K = c->ck, S = c->nseg, last = (S - 1) * K, N = c->N;
  const int seglen = S > 1 ? K : N;
  Lane ln = main_lane(c);
  ForwardWatch watch(c, limit);
  for (int a = 0; a < N; a += seglen) {
    const int b = std::min(a + seglen, N);
    if (S > 1 && a < last) snap_save(c, a, a / K);
    ln.hist = seg_hist(c, a / seglen);
    // blocks end at the segment's end and at every multiple of
    // kWatchEvery, where the state is checked (and after the last step)
    for (int a2 = a; a2 < b;) {
      const int b2 = std::min(b, (a2 / kWatchEvery + 1) * kWatchEvery);
      run_block<T>(c, false, false, a2, b2 - a2, [=](int j) { return a2 + j; }, last,
                   [=](int j) { return a2 + j >= last; }, ln);
      if (b2 % kWatchEvery == 0 || b2 == N) watch.enqueue(b2);
      a2 = b2;
    }
  }
  FDTD_HIP(hipGetLastError());
  FDTD_HIP(hipEventRecord(c->ev[1], c->stream));
  watch.finish();
}

// Adjoint solve, m = N..1 (eq. (20)); step m reads the forward E^m from the
// history.  With checkpoints, when m enters a segment whose history is not
// held, that segment of the forward is re-run from its snapshot on the re-run
// state, refilling a history buffer.  With two history buffers the re-run of
// segment s-1 runs on the re-run stream while the adjoint sweeps segment s
// on the context stream: the adjoint of s waits for the re-run of s, and the
// re-run of s-1 for the adjoint of s+1 (which read the buffer it refills).
template <typename T>
void run_adjoint(fdtd_ctx *c) {
  FDTD_HIP(hipEventRecord(c->ev[2], c->stream));
  const int K = c->ck, S = c->nseg, N = c->N;
  const int seglen = S > 1 ? K : N;
  Lane main = main_lane(c);
  auto rerun = [&](int s, const Lane &ln) {
    const int a = s * seglen, b = std::min(a + seglen, N);
    snap_load(c, a, s, ln.s);
    run_block<T>(c, true, false, a, b - a, [=](int j) { return a + j; }, a, [](int) { return true; }, ln);
  };
  auto adjoint = [&](int s) {
    const int a = s * seglen, b = std::min(a + seglen, N);
    main.hist = seg_hist(c, s);
    // adjoint steps m = b .. a+1 (the (N-b+1)-th .. (N-a)-th of the adjoint solve)
    run_block<T>(c, false, true, N - b, b - a, [=](int j) { return b - j; }, a, [](int) { return false; }, main);
  };
  if (S > 1 && c->hist2.p) {
    Lane rl{c->rr, &c->auxR, &c->supR, nullptr};
    FDTD_HIP(hipEventRecord(c->evStart, c->stream));
    FDTD_HIP(hipStreamWaitEvent(c->rr, c->evStart, 0));
    for (int s = S - 1; s >= 0; --s) {
      if (s != S - 1) FDTD_HIP(hipStreamWaitEvent(c->stream, c->evRerun, 0));
      adjoint(s);
      FDTD_HIP(hipEventRecord(c->evAdj[s & 1], c->stream));
      if (s >= 1) {
        if (s + 1 <= S - 1) FDTD_HIP(hipStreamWaitEvent(c->rr, c->evAdj[(s + 1) & 1], 0));
        rl.hist = seg_hist(c, s - 1);
        rerun(s - 1, rl);
        FDTD_HIP(hipEventRecord(c->evRerun, c->rr));
      }
    }
  } else {
    for (int s = S - 1; s >= 0; --s) {
      if (S > 1 && s != S - 1) {
        Lane ln = main_lane(c);
        ln.hist = seg_hist(c, s);
        rerun(s, ln);
      }
      adjoint(s);
    }
  }
  FDTD_HIP(hipGetLastError());
  FDTD_HIP(hipEventRecord(c->ev[3], c->stream));
}

template <typename F>
fdtd_status guard(fdtd_ctx *c, F &&f) {
  try {
    f();
    return FDTD_OK;
  } catch (const Error &e) {
    if (c) c->err = e.msg; else g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    if (c) c->err = "host out of memory"; else g_create_error = "host out of memory";
    return FDTD_ENOMEM;
  }
}

// Steps of a forward solve around the time stepping (shared by single
// contexts and batches).
void fwd_prepare(fdtd_ctx *c) {
  if (c->state < 1) throw Error{FDTD_ESTATE, "forward before set_density"};
  c->state = 1;
  c->fwd_state_valid = false;
  zero_state(c);
  zero(c, c->gapE);
  if (!c->init_state.empty()) {
    if (c->prec == 32) upload_init_state<float>(c); else upload_init_state<double>(c);
  }
}

// Watchdog limit of a forward solve: a multiple of the incident amplitude,
// or without a plane wave of the largest value of the initial state.
double watch_limit(const fdtd_ctx *c) {
  double ref = c->cfg.source_kind == FDTD_SRC_NONE ? 0.0 : std::fabs(c->cfg.amplitude);
  if (c->cfg.source_kind == FDTD_SRC_NONE)
    for (double v : c->init_state) ref = std::max(ref, std::fabs(v));
  return kWatchFactor * (ref > 0.0 ? ref : 1.0);
}

void fwd_objective(fdtd_ctx *c) {
  const fdtd_config &g = c->cfg;
  launch_dft(c->stream, c->gapE.as<double>(), c->phasor.as<double>(), c->K, c->nmon, c->N, c->dt, c->dft.as<double>());
  const double te_scale = 0.5 * g.eps_g * c->dt * g.dx * g.dx * g.dx;
  launch_objective(c->stream, c->dft.as<double>(), c->wts.as<double>(), c->gapE.as<double>(), c->K, c->nmon, c->N,
                   g.objective_kind == FDTD_OBJ_TIME_ENERGY, te_scale, c->Fdev.as<double>());
}

void fwd_finish(fdtd_ctx *c, double F) {
  if (!std::isfinite(F)) throw Error{FDTD_EUNSTABLE, "non-finite objective"};
  c->F = F;
  c->state = 2;
}

void adj_prepare(fdtd_ctx *c) {
  if (c->state < 2) throw Error{FDTD_ESTATE, "adjoint before forward"};
  c->fwd_state_valid = false;  // the adjoint reuses the state buffers
  const fdtd_config &g = c->cfg;
  const double te_coef = g.eps_g * c->dt * g.dx * g.dx * g.dx;
  launch_adjoint_source(c->stream, c->prec, c->dft.as<double>(), c->wts.as<double>(), c->phasor.as<double>(),
                        c->gapE.as<double>(), c->K, c->nmon, c->N, g.objective_kind == FDTD_OBJ_TIME_ENERGY, te_coef,
                        c->dt, g.dx, c->scal.as<double>(), c->asrc.p);
  zero_state(c);
  zero(c, c->grad);
}

}  // namespace

// ---------------------------------------------------------------- batches
struct fdtd_batch {
  std::vector<fdtd_ctx *> inst;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int prec = 64, N = 0;
  fdtd_batch_options opt{0, 1, 0};
  std::vector<int> rows;  // tile depth per instance
  // Two-step blocking: with `mix` every step goes through the blocked
  // schedule (two rows per thread everywhere); tb[k] = instance k advances
  // its plain-background super-tiles two steps per pass.
  bool mix = false;
  std::vector<int> tb;
  struct MixLaunch {  // descriptor table of one launch of the blocked schedule
    DevBuf desc, firstR, firstT;
    int nrest = 0, nblocks = 0;
  };
  std::map<int, MixLaunch> mixl;  // by launch kind * 6 + (step index mod 6)
  struct Group {          // instances sharing one tile depth: one launch per step
    int R = 2, nblocks = 0;
    std::vector<int> members;
    DevBuf params, first;
  };
  std::vector<Group> groups;
  hipGraph_t graph[2] = {nullptr, nullptr};  // forward, adjoint step sequences
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  double ms[2] = {0, 0};
  std::string err;
  ~fdtd_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (int k = 0; k < 2; ++k) {
      if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
    }
    for (int k = 0; k < 4; ++k) if (ev[k]) (void)hipEventDestroy(ev[k]);
    for (fdtd_ctx *c : inst) fdtd_destroy(c);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

thread_local std::string g_batch_error;

// Launch one time step of every instance (one launch per tile-depth group).
template <typename T>
void batch_step(fdtd_batch *b, int n, int par, bool adjoint) {
  for (auto &g : b->groups)
    launch_step2d_batch<T>(g.params.as<Step2D<T>>(), g.first.as<int>(), (int)g.members.size(), g.nblocks, n, par,
                           adjoint, g.R, b->stream);
}

// Launch kinds of the blocked schedule (see run_block): the first pair's
// launch A (every super-tile), launch A, launch B with the next pair's early
// super-tiles, the last pair's launch B, a full-grid single step.
enum { MIX_A0, MIX_A, MIX_B, MIX_BLAST, MIX_SINGLE };

// The descriptor table of launch `kind` whose per-step part is the (s+1)-th
// step of its solve (field copies repeat with period 3, absorber memories
// with period 2).  Built and uploaded on first use, outside graph capture.
template <typename T>
fdtd_batch::MixLaunch &mix_launch(fdtd_batch *b, int kind, int s) {
  const int key = kind * 6 + s % 6;
  auto it = b->mixl.find(key);
  if (it != b->mixl.end()) return it->second;
  const int cnt = (int)b->inst.size();
  std::vector<Mix2D<T>> ds(cnt);
  std::vector<int> fr(cnt), ft(cnt);
  int nr = 0, nt = 0;
  for (int k = 0; k < cnt; ++k) {
    fdtd_ctx *c = b->inst[k];
    const bool on = b->tb[k] && c->nTb > 0 && kind != MIX_SINGLE;
    Mix2D<T> d{};
    d.ps = params2d_at<T>(c, false, s, 0, true, c->hist.p);
    d.ps.tlist = on ? c->tbRest.as<int>() : nullptr;
    d.nrest = on ? c->nRest : step2d_blocks(c->nx, c->ny, 0);
    int first = 0, count = 0, sp = s;  // super-tiles [first, first+count) of the pair entered after sp steps
    if (on && kind == MIX_A0) count = c->nTb;
    if (on && kind == MIX_A) {
      first = c->nEarly;
      count = c->nTb - c->nEarly;
    }
    if (on && kind == MIX_B) {
      count = c->nEarly;
      sp = s + 1;
    }
    d.pt = params2d_at<T>(c, false, sp, 0, true, c->hist.p);
    if (count > 0) {
      d.tiles = c->tbTiles.as<int>() + first;
      d.ntb = count;
      d.ezo = field_buf(c, false, fcopy(c, sp + 2), 0)->as<T>();
      d.hxo = field_buf(c, false, fcopy(c, sp + 2), 1)->as<T>();
      d.hyo = field_buf(c, false, fcopy(c, sp + 2), 2)->as<T>();
    }
    ds[k] = d;
    fr[k] = nr;
    ft[k] = nt;
    nr += (d.nrest + 7) / 8 * 8;  // keeps the XCD in the low bits of a whole-grid tile index
    nt += (d.ntb + 7) / 8 * 8;
  }
  fdtd_batch::MixLaunch &m = b->mixl[key];
  upload(b->stream, m.desc, ds);
  upload(b->stream, m.firstR, fr);
  upload(b->stream, m.firstT, ft);
  FDTD_HIP(hipStreamSynchronize(b->stream));
  m.nrest = nr;
  m.nblocks = nr + nt;
  return m;
}

// `count` steps of the blocked schedule from the start of a solve (forward:
// step n = s; adjoint: m = N - s), as run_block pipelines them.  With
// `build_only` the descriptor tables are made and nothing is launched.
template <typename T>
void batch_mix_steps(fdtd_batch *b, bool adjoint, int count, bool build_only = false) {
  const int N = b->N, cnt = (int)b->inst.size();
  auto go = [&](int kind, int s) {
    fdtd_batch::MixLaunch &m = mix_launch<T>(b, kind, s);
    if (!build_only)
      launch_step2d_batch_mix<T>(m.desc.as<Mix2D<T>>(), m.firstR.as<int>(), m.firstT.as<int>(), cnt, m.nrest,
                                 m.nblocks, adjoint ? N - s : s, adjoint, b->stream);
  };
  const int P = count / 2;
  for (int q = 0; q < P; ++q) {
    go(q == 0 ? MIX_A0 : MIX_A, 2 * q);
    go(q + 1 < P ? MIX_B : MIX_BLAST, 2 * q + 1);
  }
  if (count & 1) go(MIX_SINGLE, count - 1);
}

template <typename T>
void batch_steps(fdtd_batch *b, bool adjoint) {
  const int N = b->N;
  if (b->mix) {
    batch_mix_steps<T>(b, adjoint, N);
    return;
  }
  if (!adjoint)
    for (int n = 0; n < N; ++n) batch_step<T>(b, n, n & 1, false);
  else
    for (int m = N; m >= 1; --m) batch_step<T>(b, m, (N - m) & 1, true);
}

// The N steps of a solve: captured into a graph on first use, then replayed.
template <typename T>
void batch_run(fdtd_batch *b, bool adjoint) {
  const int k = adjoint ? 1 : 0;
  if (b->opt.use_graph && !b->exec[k]) {
    FDTD_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    batch_steps<T>(b, adjoint);
    FDTD_HIP(hipStreamEndCapture(b->stream, &b->graph[k]));
    FDTD_HIP(hipGraphInstantiate(&b->exec[k], b->graph[k], nullptr, nullptr, 0));
  }
  FDTD_HIP(hipEventRecord(b->ev[2 * k], b->stream));
  if (b->opt.use_graph)
    FDTD_HIP(hipGraphLaunch(b->exec[k], b->stream));
  else
    batch_steps<T>(b, adjoint);
  FDTD_HIP(hipGetLastError());
  FDTD_HIP(hipEventRecord(b->ev[2 * k + 1], b->stream));
}

// Group the instances by tile depth (b->rows) and upload each group's
// parameter blocks and workgroup table.
template <typename T>
void build_groups(fdtd_batch *b) {
  b->groups.clear();
  const int cnt = (int)b->inst.size();
  for (int R : {1, 2, 4}) {
    fdtd_batch::Group g;
    g.R = R;
    std::vector<Step2D<T>> ps;
    std::vector<int> first;
    for (int k = 0; k < cnt; ++k) {
      if (b->rows[k] != R) continue;
      fdtd_ctx *c = b->inst[k];
      g.members.push_back(k);
      Step2D<T> p = params2d<T>(c, false);
      p.hist_base = 0;
      p.hist_on = 1;
      ps.push_back(p);
      first.push_back(g.nblocks);
      g.nblocks += (step2d_blocks(c->nx, c->ny, R) + 7) / 8 * 8;  // keeps the XCD in the low bits
    }
    if (g.members.empty()) continue;
    upload(b->stream, g.params, ps);
    upload(b->stream, g.first, first);
    b->groups.push_back(std::move(g));
  }
  FDTD_HIP(hipStreamSynchronize(b->stream));
}

// Event time of `steps` batched forward steps with the current grouping (the
// instances' states are scratch here: every forward starts by zeroing them).
template <typename T>
float time_batch(fdtd_batch *b, int steps) {
  build_groups<T>(b);
  for (int k = 0; k < 3; ++k) batch_step<T>(b, k % b->N, k & 1, false);
  FDTD_HIP(hipEventRecord(b->ev[0], b->stream));
  for (int k = 0; k < steps; ++k) batch_step<T>(b, k % b->N, k & 1, false);
  FDTD_HIP(hipEventRecord(b->ev[1], b->stream));
  FDTD_HIP(hipEventSynchronize(b->ev[1]));
  float ms = 0;
  FDTD_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
  return ms;
}

// Event time of `steps` forward steps of the blocked schedule with the
// current two-step flags (from the start of a solve; states are scratch).
template <typename T>
float time_mix(fdtd_batch *b, int steps) {
  b->mixl.clear();
  batch_mix_steps<T>(b, false, steps, true);
  batch_mix_steps<T>(b, false, std::min(4, steps));
  FDTD_HIP(hipEventRecord(b->ev[0], b->stream));
  batch_mix_steps<T>(b, false, steps);
  FDTD_HIP(hipEventRecord(b->ev[1], b->stream));
  FDTD_HIP(hipEventSynchronize(b->ev[1]));
  float ms = 0;
  FDTD_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
  return ms;
}

// Per-step tile depths tuned on the batch: the fastest uniform depth, then
// one pass over the grid sizes trying the other depths for all instances of
// that size.  Returns the time of `steps` batched steps with the choice.
template <typename T>
float tune_rows(fdtd_batch *b, const std::vector<std::pair<int, int>> &sizes, int steps) {
  const int cnt = (int)b->inst.size();
  float best = 1e30f;
  int bestR = 2;
  for (int R : {1, 2, 4}) {
    b->rows.assign(cnt, R);
    const float t = time_batch<T>(b, steps);
    if (t < best) {
      best = t;
      bestR = R;
    }
  }
  b->rows.assign(cnt, bestR);
  if (sizes.size() > 1) {
    for (auto sz : sizes) {
      for (int R : {1, 2, 4}) {
        std::vector<int> trial = b->rows;
        bool changed = false;
        for (int k = 0; k < cnt; ++k)
          if (b->inst[k]->nx == sz.first && b->inst[k]->ny == sz.second && trial[k] != R) {
            trial[k] = R;
            changed = true;
          }
        if (!changed) continue;
        const std::vector<int> keep = b->rows;
        b->rows = trial;
        const float t = time_batch<T>(b, steps);
        if (t < best) best = t;
        else b->rows = keep;
      }
    }
  }
  return best;
}

// Temporal-block depth and tile depth: fixed by the options, or tuned on the
// batch.  Depth 1 = one launch per tile-depth group per step; depth 2 = the
// blocked schedule, where instances with plain-background super-tiles
// advance them two steps per pass (the others take per-step launches inside
// it).  Tuning times the best depth-1 choice against depth 2, then tries
// depth 1 for the instances of each grid size in turn within the blocked
// schedule and keeps what is faster.
template <typename T>
void batch_setup(fdtd_batch *b) {
  const int cnt = (int)b->inst.size();
  const int steps = std::min(20, b->N);
  std::vector<std::pair<int, int>> sizes;
  bool any_tb = false;
  for (fdtd_ctx *c : b->inst) {
    any_tb = any_tb || c->nTb > 0;
    if (std::find(sizes.begin(), sizes.end(), std::make_pair(c->nx, c->ny)) == sizes.end()) sizes.push_back({c->nx, c->ny});
  }
  b->mix = false;
  b->tb.assign(cnt, 0);
  const bool can_mix = any_tb && b->opt.depth != 1 && (b->opt.rows == 0 || b->opt.rows == 2);
  if (b->opt.depth == 2 && can_mix) {
    b->mix = true;
  } else if (b->opt.depth == 0 && can_mix) {
    float t1;
    if (b->opt.rows > 0) {
      b->rows.assign(cnt, b->opt.rows);
      t1 = time_batch<T>(b, steps);
    } else {
      t1 = tune_rows<T>(b, sizes, steps);
    }
    for (int k = 0; k < cnt; ++k) b->tb[k] = b->inst[k]->nTb > 0;
    float t2 = time_mix<T>(b, steps);
    if (sizes.size() > 1) {
      for (auto sz : sizes) {
        const std::vector<int> keep = b->tb;
        bool changed = false;
        for (int k = 0; k < cnt; ++k)
          if (b->inst[k]->nx == sz.first && b->inst[k]->ny == sz.second && b->tb[k]) {
            b->tb[k] = 0;
            changed = true;
          }
        if (!changed) continue;
        const float t = time_mix<T>(b, steps);
        if (t < t2) t2 = t;
        else b->tb = keep;
      }
    }
    b->mix = t2 < t1 && std::find(b->tb.begin(), b->tb.end(), 1) != b->tb.end();
  }
  if (b->mix) {
    if (std::find(b->tb.begin(), b->tb.end(), 1) == b->tb.end())
      for (int k = 0; k < cnt; ++k) b->tb[k] = b->inst[k]->nTb > 0;
    b->rows.assign(cnt, 2);
    b->groups.clear();
    b->mixl.clear();
    batch_mix_steps<T>(b, false, b->N, true);  // the adjoint uses the same tables
    return;
  }
  b->tb.assign(cnt, 0);
  b->mixl.clear();
  if (b->opt.rows > 0) b->rows.assign(cnt, b->opt.rows);
  else if (b->rows.size() != (size_t)cnt) tune_rows<T>(b, sizes, steps);
  build_groups<T>(b);
}

template <typename F>
fdtd_status bguard(fdtd_batch *b, F &&f) {
  try {
    f();
    return FDTD_OK;
  } catch (const Error &e) {
    if (b) b->err = e.msg; else g_batch_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    if (b) b->err = "host out of memory"; else g_batch_error = "host out of memory";
    return FDTD_ENOMEM;
  }
}

fdtd_ctx *instance(fdtd_batch *b, int32_t index) {
  if (index < 0 || index >= (int32_t)b->inst.size()) throw einval("instance index out of range");
  return b->inst[index];
}

}  // namespace

extern "C" {

int32_t fdtd_abi_version(void) { return FDTD_ABI_VERSION; }

const char *fdtd_last_error(const fdtd_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

fdtd_status fdtd_create(const fdtd_config *cfg, fdtd_ctx **out) {
  Range range("fdtd_create");
  if (!out) { g_create_error = "null out pointer"; return FDTD_EINVAL; }
  *out = nullptr;
  if (!cfg) { g_create_error = "null config"; return FDTD_EINVAL; }
  std::unique_ptr<fdtd_ctx> c(new fdtd_ctx());
  fdtd_status st = guard(nullptr, [&] {
    validate(*cfg);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      throw Error{FDTD_EDEVICE, "no HIP device"};
    }
    FDTD_HIP(hipGetDevice(&c->device));
    c->cfg = *cfg;
    c->dims = cfg->dims;
    c->te = cfg->dims == 2 && cfg->pol_axis == FDTD_AXIS_X;
    c->prec = cfg->precision;
    c->esz = c->prec == 32 ? 4 : 8;
    c->nx = cfg->n[0]; c->ny = cfg->n[1]; c->nz = cfg->dims == 3 ? cfg->n[2] : 1;
    c->N = cfg->n_steps; c->K = cfg->n_freq;
    c->ck = cfg->ckpt_every > 0 && cfg->ckpt_every < c->N ? cfg->ckpt_every : c->N;
    c->nseg = (c->N + c->ck - 1) / c->ck;
    c->dt = cfg->courant * cfg->dx / kC0;
    c->freqs.resize(c->K);
    for (int k = 0; k < c->K; ++k)
      c->freqs[k] = cfg->freqs_hz ? cfg->freqs_hz[k]
                                  : (c->K == 1 ? 0.5 * (cfg->f_lo + cfg->f_hi)
                                               : cfg->f_lo + (cfg->f_hi - cfg->f_lo) * k / (c->K - 1));
    c->cfg.freqs_hz = nullptr;
    if (cfg->stream) {
      c->stream = (hipStream_t)cfg->stream;
    } else {
      FDTD_HIP(hipStreamCreate(&c->stream));
      c->own_stream = true;
    }
    for (int k = 0; k < 4; ++k) FDTD_HIP(hipEventCreate(&c->ev[k]));
    if (c->dims == 2) create_2d(c.get()); else create_3d(c.get());
    create_common(c.get());
    if (c->dims == 2) {
      if (c->prec == 32) fill_params2d(c.get(), c->p2f, false); else fill_params2d(c.get(), c->p2d, false);
      if (c->prec == 32) fill_params2d(c.get(), c->p2fR, true); else fill_params2d(c.get(), c->p2dR, true);
    } else {
      if (c->prec == 32) fill_params3d(c.get(), c->p3f, false); else fill_params3d(c.get(), c->p3d, false);
      if (c->prec == 32) fill_params3d(c.get(), c->p3fR, true); else fill_params3d(c.get(), c->p3dR, true);
    }
    if (c->nseg > 1) {  // the re-run state's never-written nodes (walls, guards) stay zero
      for (int b = 0; b < 2; ++b) {
        for (int k = 0; k < 6; ++k) if (c->fldR[b][k].p) zero(c.get(), c->fldR[b][k]);
        for (int k = 0; k < 12; ++k) if (c->pmlR[b][k].p) zero(c.get(), c->pmlR[b][k]);
      }
      for (int b = 0; b < 3; ++b)
        if (c->arenaR[b].p) zero(c.get(), c->arenaR[b]);
      // the third field copy of the two-step schedule: a re-run whose
      // segment starts in copy 0 or 1 reads this copy's wall nodes before
      // any step has written them
      for (int k = 0; k < 3; ++k) if (c->fld3R[k].p) zero(c.get(), c->fld3R[k]);
    }
    FDTD_HIP(hipStreamSynchronize(c->stream));
    FDTD_HIP(hipGetLastError());
  });
  if (st != FDTD_OK) {
    release_aux(c.get());
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    for (int k = 0; k < 4; ++k) if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    return st;
  }
  *out = c.release();
  return FDTD_OK;
}

fdtd_status fdtd_destroy(fdtd_ctx *ctx) {
  if (!ctx) return FDTD_OK;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  release_aux(ctx);
  for (int k = 0; k < 4; ++k) if (ctx->ev[k]) (void)hipEventDestroy(ctx->ev[k]);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return FDTD_OK;
}

fdtd_status fdtd_set_density(fdtd_ctx *ctx, const void *rho, int64_t count, int32_t on_device) {
  if (!ctx) return FDTD_EINVAL;
  return guard(ctx, [&] {
    if (!rho) throw einval("null density");
    if (count != (int64_t)ctx->nd) throw einval("density count must equal the number of design cells");
    if (!on_device) {
      if (ctx->prec == 32) {
        const float *r = (const float *)rho;
        for (int64_t i = 0; i < count; ++i) if (!(r[i] >= 0.0f && r[i] <= 1.0f)) throw einval("density outside [0,1] or NaN");
      } else {
        const double *r = (const double *)rho;
        for (int64_t i = 0; i < count; ++i) if (!(r[i] >= 0.0 && r[i] <= 1.0)) throw einval("density outside [0,1] or NaN");
      }
      FDTD_HIP(hipMemcpyAsync(ctx->rho.p, rho, (size_t)count * ctx->esz, hipMemcpyHostToDevice, ctx->stream));
      FDTD_HIP(hipStreamSynchronize(ctx->stream));
    } else {
      launch_check_density(ctx->stream, ctx->prec, rho, count, ctx->bad.as<int>());
      int bad = 0;
      FDTD_HIP(hipMemcpyAsync(&bad, ctx->bad.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
      FDTD_HIP(hipStreamSynchronize(ctx->stream));
      if (bad) throw einval("density outside [0,1] or NaN");
      launch_copy_density(ctx->stream, ctx->prec, rho, ctx->rho.p, count);
    }
    ctx->state = 1;
  });
}

fdtd_status fdtd_forward(fdtd_ctx *ctx, double *objective_out) {
  if (!ctx) return FDTD_EINVAL;
  Range range("fdtd_forward");
  return guard(ctx, [&] {
    fwd_prepare(ctx);
    const double limit = watch_limit(ctx);
    if (ctx->prec == 32) run_forward<float>(ctx, limit); else run_forward<double>(ctx, limit);
    fwd_objective(ctx);
    double F = 0;
    FDTD_HIP(hipMemcpyAsync(&F, ctx->Fdev.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    FDTD_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0;
    FDTD_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    ctx->timing.forward_ms = ms;
    ctx->timing.forward_launches = ctx->N;
    fwd_finish(ctx, F);
    ctx->fwd_state_valid = true;
    if (objective_out) *objective_out = F;
  });
}

fdtd_status fdtd_adjoint(fdtd_ctx *ctx) {
  if (!ctx) return FDTD_EINVAL;
  Range range("fdtd_adjoint");
  return guard(ctx, [&] {
    adj_prepare(ctx);
    if (ctx->prec == 32) run_adjoint<float>(ctx); else run_adjoint<double>(ctx);
    ctx->timing.adjoint_launches = ctx->N;
    ctx->state = 3;
  });
}

fdtd_status fdtd_gradient(fdtd_ctx *ctx, void *grad_out, int64_t count, int32_t on_device) {
  if (!ctx) return FDTD_EINVAL;
  Range range("fdtd_gradient");
  return guard(ctx, [&] {
    if (ctx->state < 3) throw Error{FDTD_ESTATE, "gradient before adjoint"};
    if (!grad_out) throw einval("null gradient buffer");
    if (count != (int64_t)ctx->nd) throw einval("gradient count must equal the number of design cells");
    const fdtd_config &g = ctx->cfg;
    void *dst = on_device ? grad_out : ctx->gtmp.p;
    if (ctx->te)  // one sum per design edge; the gap's edges never accumulate
      launch_grad_finalize(ctx->stream, ctx->prec, ctx->grad.as<double>(), ctx->scal.as<double>(), 1, ctx->nd, 1, 1,
                           0, 0, 0, 0, 0, 0, dst);
    else
      launch_grad_finalize(ctx->stream, ctx->prec, ctx->grad.as<double>(), ctx->scal.as<double>(), ctx->ncomp,
                           g.design_n[0], g.design_n[1], ctx->dims == 3 ? g.design_n[2] : 1,
                           g.gap_lo[0] - g.design_lo[0], g.gap_lo[1] - g.design_lo[1],
                           ctx->dims == 3 ? g.gap_lo[2] - g.design_lo[2] : 0, g.gap_n[0], g.gap_n[1],
                           ctx->dims == 3 ? g.gap_n[2] : 1, dst);
    if (!on_device) {
      FDTD_HIP(hipMemcpyAsync(grad_out, ctx->gtmp.p, (size_t)count * ctx->esz, hipMemcpyDeviceToHost, ctx->stream));
      FDTD_HIP(hipStreamSynchronize(ctx->stream));
    }
    float ms = 0;
    FDTD_HIP(hipEventSynchronize(ctx->ev[3]));
    FDTD_HIP(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
    ctx->timing.adjoint_ms = ms;
  });
}

fdtd_status fdtd_get_dft(fdtd_ctx *ctx, double *re_im, int64_t count) {
  if (!ctx) return FDTD_EINVAL;
  return guard(ctx, [&] {
    if (ctx->state < 2) throw Error{FDTD_ESTATE, "get_dft before forward"};
    if (!re_im || count != (int64_t)ctx->K * ctx->nmon * 2) throw einval("dft buffer size must be K * n_gap * n_comp * 2");
    FDTD_HIP(hipMemcpyAsync(re_im, ctx->dft.p, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    FDTD_HIP(hipStreamSynchronize(ctx->stream));
  });
}

fdtd_status fdtd_set_state(fdtd_ctx *ctx, const double *state, int64_t count) {
  if (!ctx) return FDTD_EINVAL;
  return guard(ctx, [&] {
    if (count == 0 && !state) {
      ctx->init_state.clear();
      return;
    }
    const int64_t need = (int64_t)state_fields(ctx) * ctx->nx * ctx->ny * ctx->nz;
    if (!state || count != need) throw einval("state count must be n_fields * nx * ny * nz (or NULL, 0 to clear)");
    ctx->init_state.assign(state, state + count);
    ctx->fwd_state_valid = false;
  });
}

fdtd_status fdtd_get_state(fdtd_ctx *ctx, double *state, int64_t count) {
  if (!ctx) return FDTD_EINVAL;
  return guard(ctx, [&] {
    if (!ctx->fwd_state_valid) throw Error{FDTD_ESTATE, "get_state needs a forward solve (and no adjoint since)"};
    const int64_t need = (int64_t)state_fields(ctx) * ctx->nx * ctx->ny * ctx->nz;
    if (!state || count != need) throw einval("state count must be n_fields * nx * ny * nz");
    if (ctx->prec == 32) download_state<float>(ctx, state); else download_state<double>(ctx, state);
  });
}

fdtd_status fdtd_get_timing(fdtd_ctx *ctx, fdtd_timing *out) {
  if (!ctx || !out) return FDTD_EINVAL;
  *out = ctx->timing;
  out->cells = (int64_t)ctx->nx * ctx->ny * ctx->nz;
  out->design_cells = ctx->nd;
  return FDTD_OK;
}

fdtd_status fdtd_batch_create(const fdtd_config *cfgs, int32_t count, const fdtd_batch_options *opt, fdtd_batch **out) {
  if (!out) { g_batch_error = "null out pointer"; return FDTD_EINVAL; }
  *out = nullptr;
  std::unique_ptr<fdtd_batch> b(new fdtd_batch());
  fdtd_status st = bguard(nullptr, [&] {
    if (!cfgs || count < 1) throw einval("need at least one config");
    if (opt) b->opt = *opt;
    if (b->opt.rows != 0 && b->opt.rows != 1 && b->opt.rows != 2 && b->opt.rows != 4)
      throw einval("batch rows must be 0, 1, 2 or 4");
    if (b->opt.depth < 0 || b->opt.depth > 2) throw einval("batch depth must be 0, 1 or 2");
    if (b->opt.depth == 2 && b->opt.rows != 0 && b->opt.rows != 2)
      throw einval("two-step blocking runs two rows per thread (rows 0 or 2)");
    for (int k = 0; k < count; ++k) {
      if (cfgs[k].dims != 2 || cfgs[k].pol_axis == FDTD_AXIS_X)
        throw einval("batch instance " + std::to_string(k) + ": batches hold 2D TMz instances");
      if (cfgs[k].precision != cfgs[0].precision) throw einval("batch instances must share the precision");
      if (cfgs[k].n_steps != cfgs[0].n_steps) throw einval("batch instances must share n_steps");
      if (cfgs[k].ckpt_every != 0) throw einval("batch instances keep the full history (ckpt_every = 0)");
    }
    if (cfgs[0].stream) {
      b->stream = (hipStream_t)cfgs[0].stream;
    } else {
      FDTD_HIP(hipStreamCreate(&b->stream));
      b->own_stream = true;
    }
    for (int k = 0; k < 4; ++k) FDTD_HIP(hipEventCreate(&b->ev[k]));
    b->prec = cfgs[0].precision;
    b->N = cfgs[0].n_steps;
    for (int k = 0; k < count; ++k) {
      fdtd_config c = cfgs[k];
      c.stream = b->stream;
      fdtd_ctx *ctx = nullptr;
      const fdtd_status s2 = fdtd_create(&c, &ctx);
      if (s2 != FDTD_OK) throw Error{s2, "batch instance " + std::to_string(k) + ": " + g_create_error};
      b->inst.push_back(ctx);
    }
    if (b->prec == 32) batch_setup<float>(b.get()); else batch_setup<double>(b.get());
  });
  if (st != FDTD_OK) return st;
  *out = b.release();
  return FDTD_OK;
}

fdtd_status fdtd_batch_set_density(fdtd_batch *b, int32_t index, const void *rho, int64_t count, int32_t on_device) {
  if (!b) return FDTD_EINVAL;
  return bguard(b, [&] {
    fdtd_ctx *c = instance(b, index);
    const fdtd_status s = fdtd_set_density(c, rho, count, on_device);
    if (s != FDTD_OK) throw Error{s, c->err};
  });
}

fdtd_status fdtd_batch_forward(fdtd_batch *b, double *objectives_out) {
  if (!b) return FDTD_EINVAL;
  Range range("fdtd_batch_forward");
  return bguard(b, [&] {
    for (fdtd_ctx *c : b->inst) fwd_prepare(c);
    if (b->prec == 32) batch_run<float>(b, false); else batch_run<double>(b, false);
    const size_t cnt = b->inst.size();
    std::vector<double> F(cnt, 0.0);
    for (size_t k = 0; k < cnt; ++k) {
      fwd_objective(b->inst[k]);
      FDTD_HIP(hipMemcpyAsync(&F[k], b->inst[k]->Fdev.p, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    FDTD_HIP(hipStreamSynchronize(b->stream));
    float ms = 0;
    FDTD_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
    b->ms[0] = ms;
    for (size_t k = 0; k < cnt; ++k) {
      b->inst[k]->err.clear();
      fwd_finish(b->inst[k], F[k]);
      if (objectives_out) objectives_out[k] = F[k];
    }
  });
}

fdtd_status fdtd_batch_adjoint(fdtd_batch *b) {
  if (!b) return FDTD_EINVAL;
  Range range("fdtd_batch_adjoint");
  return bguard(b, [&] {
    for (fdtd_ctx *c : b->inst) adj_prepare(c);
    if (b->prec == 32) batch_run<float>(b, true); else batch_run<double>(b, true);
    FDTD_HIP(hipStreamSynchronize(b->stream));
    float ms = 0;
    FDTD_HIP(hipEventElapsedTime(&ms, b->ev[2], b->ev[3]));
    b->ms[1] = ms;
    for (fdtd_ctx *c : b->inst) {
      c->state = 3;
      c->timing.adjoint_ms = 0;
    }
  });
}

fdtd_status fdtd_batch_gradient(fdtd_batch *b, int32_t index, void *grad_out, int64_t count, int32_t on_device) {
  if (!b) return FDTD_EINVAL;
  return bguard(b, [&] {
    fdtd_ctx *c = instance(b, index);
    if (c->state < 3) throw Error{FDTD_ESTATE, "gradient before adjoint"};
    if (!grad_out) throw einval("null gradient buffer");
    if (count != (int64_t)c->nd) throw einval("gradient count must equal the number of design cells");
    const fdtd_config &g = c->cfg;
    void *dst = on_device ? grad_out : c->gtmp.p;
    launch_grad_finalize(c->stream, c->prec, c->grad.as<double>(), c->scal.as<double>(), c->ncomp, g.design_n[0],
                         g.design_n[1], 1, g.gap_lo[0] - g.design_lo[0], g.gap_lo[1] - g.design_lo[1], 0, g.gap_n[0],
                         g.gap_n[1], 1, dst);
    if (!on_device) {
      FDTD_HIP(hipMemcpyAsync(grad_out, c->gtmp.p, (size_t)count * c->esz, hipMemcpyDeviceToHost, c->stream));
      FDTD_HIP(hipStreamSynchronize(c->stream));
    }
  });
}

fdtd_status fdtd_batch_info(fdtd_batch *b, int32_t index, int32_t *rows_out, double *forward_ms, double *adjoint_ms) {
  if (!b) return FDTD_EINVAL;
  return bguard(b, [&] {
    (void)instance(b, index);
    if (rows_out) *rows_out = b->rows[index];
    if (forward_ms) *forward_ms = b->ms[0];
    if (adjoint_ms) *adjoint_ms = b->ms[1];
  });
}

fdtd_status fdtd_batch_depth(fdtd_batch *b, int32_t index, int32_t *depth_out) {
  if (!b) return FDTD_EINVAL;
  return bguard(b, [&] {
    fdtd_ctx *c = instance(b, index);
    if (!depth_out) throw einval("null depth pointer");
    *depth_out = b->mix && b->tb[index] && c->nTb > 0 ? 2 : 1;
  });
}

fdtd_status fdtd_batch_destroy(fdtd_batch *b) {
  delete b;
  return FDTD_OK;
}

const char *fdtd_batch_last_error(const fdtd_batch *b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"
