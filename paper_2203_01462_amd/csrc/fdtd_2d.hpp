// fdtd_2d.hpp -- parameters of the 2D TMz step kernel.
#pragma once

#include <vector>

#include "fdtd_internal.hpp"

namespace fdtd {

// Everything one launch of the fused 2D step reads.  Field and
// absorber-memory arrays are given as a read copy [par] and a write copy
// [par^1] because a tile recomputes its halo of H from the previous step's
// values while neighbouring tiles are already writing theirs (the host
// resolves which physical copies these are: two rotating copies, or three
// for the fields under two-step blocking).
template <typename T>
struct Step2D {
  int nx, ny, pitch, P;
  int dx0, dy0, dnx, dny;  // design box
  int gx0, gy0, gnx, gny;  // gap box
  int ia, ib, ja, jb, jref, L, tf_on;
  int K, ng;
  T *ez[2], *hx[2], *hy[2];
  T *pex[2], *pey[2], *phx[2], *phy[2];  // absorber memories (forward psi*dx; adjoint nu)
  T *J;                                  // Drude current over the design box [dny][dnx]
  const T *rho;                          // density over the design box
  T *hist;                               // forward E over the design box, [N][dny][dnx]
  double *grad;                          // sensitivity sums over the design box (adjoint)
  int hist_base, hist_on;  // history slot of step n is n - hist_base; the forward writes it when hist_on
  double *gapE;                          // gap time series [N+1][ng] (the DFT is taken after the solve)
  const T *asrc;                         // adjoint source table [N+1][ng] (scaled by dx and S')
  const T *einc, *hinc;                  // incident line [N+1][L], [N][L]
  const T *bxe, *axe, *ikxe, *bxh, *axh, *ikxh;  // x grading at nodes / half nodes
  const T *bye, *aye, *ikye, *byh, *ayh, *ikyh;  // y grading
  T chx;          // dt / (mu0 dx)
  T ce_s, ce_g;   // dt / (eps0 eps dx): background, gap
  T A0, A1;       // 2 eps0 eps_inf_i = A0 + rho A1
  T B0, B1;       // beta_i = B0 + rho B1
  T Sg;           // sigma_i dt = Sg rho (1 - rho)
  T dt_, dtdx, dthJ, kpm1;  // kpm1 = kp - 1 = -gamma dt / (1 + gamma dt / 2), rounded once from FP64
  T ga, gsm, rs;  // sensitivity: ga = -(eps0/dt)(eps_inf - eps_s); gsm = -sigma_max/2; rs = psi_s/psi
  double dt;
  const int *tlist;  // per-step launch over these workgroup tiles (ty * nbx + tx), or all when null
};

// One time step; rows = nodes per thread along y (1, 2 or 4; 0 = default).
template <typename T>
void launch_step2d(const Step2D<T> &p, int n, int par, bool adjoint, hipStream_t s, int rows = 0);

// One time step of the 2D TEz solve (E_x, E_y, H_z; fdtd_te.hip) on the
// same parameter block: ez = E_x, hx = E_y, hy = H_z (copy 0 read, copy 1
// written), pex / pey = H_z's x / y difference memories, phx = E_x's, phy =
// E_y's; rho, J, history and sensitivity sums per design edge, ng = gap edges.
template <typename T>
void launch_step_te(const Step2D<T> &p, int n, bool adjoint, hipStream_t s);

// Workgroups of one instance's step launch (rows <= 0: the default depth).
int step2d_blocks(int nx, int ny, int rows);

// Two-step blocking of the plain background.  Super-tiles of 64 x 16 nodes
// whose reach (three nodes around them) holds only background dielectric --
// no absorber, wall, injection line, design or gap -- advance two time steps
// at once from an LDS copy of their tile with a two-node halo; the other
// workgroup tiles of the default tiling (the "rest") take the per-step
// update.  Super-tiles next to a rest tile (border) also store their
// intermediate state, which the rest tiles' second step reads.
struct Tb2dPlan {
  std::vector<int> tb;    // super-tiles: ((sy * nbx + tx) << 1) | border
  std::vector<int> rest;  // per-step workgroup tiles (ty * nbx + tx) outside the super-tiles
  int nbx = 0;            // workgroup tile columns (64 nodes wide)
};
Tb2dPlan tb2d_plan(int nx, int ny, int P, int ia, int ib, int ja, int jb, const int dbox[4], const int gbox[4]);

// One launch of the blocked schedule: nrest workgroups update the rest
// tiles listed in ps.tlist by one step (step n; copy 0 read, copy 1 written),
// ntb workgroups advance the super-tiles tiles[0..ntb) by two steps of the
// pair described by pt (copy 0: E^m, H^{m-1/2}; copy 1 receives the border
// super-tiles' intermediate state; ezo, hxo, hyo the state after the pair).
// Either count may be zero.  The two-step update is the background update,
// identical in the forward and the adjoint.
template <typename T>
void launch_step2d_mix(const Step2D<T> &ps, int n, int nrest, const Step2D<T> &pt, const int *tiles, int ntb, T *ezo,
                       T *hxo, T *hyo, bool adjoint, hipStream_t s);

// One instance's part of a batched launch of the blocked schedule: nrest
// workgroups take the per-step update of the tiles in ps.tlist (the whole
// grid when null), ntb workgroups advance tiles[0..ntb) by the pair
// described by pt (as in launch_step2d_mix).  Parities are resolved.
template <typename T>
struct Mix2D {
  Step2D<T> ps, pt;
  T *ezo, *hxo, *hyo;
  const int *tiles;
  int nrest, ntb;
};

// One launch of the blocked schedule over several instances (device array
// `ds`): the per-step workgroups of all instances first (instance k from
// firstR[k], nrest_total in all), then their two-step workgroups (instance k
// from nrest_total + firstT[k]); each instance's counts padded to a multiple
// of 8.
template <typename T>
void launch_step2d_batch_mix(const Mix2D<T> *ds, const int *firstR, const int *firstT, int ninst, int nrest_total,
                             int nblocks, int n, bool adjoint, hipStream_t s);

// One time step of several instances (device array `ps` of their parameters,
// `first[k]` = first workgroup of instance k, blocks of each instance padded
// to a multiple of 8; `nblocks` = total), all with the same tile depth.
template <typename T>
void launch_step2d_batch(const Step2D<T> *ps, const int *first, int ninst, int nblocks, int n, int par, bool adjoint,
                         int rows, hipStream_t s);

}  // namespace fdtd
