// fdtd_3d.hpp -- parameters of the 3D step kernels.
#pragma once

#include "fdtd_internal.hpp"

namespace fdtd {

// Everything one launch of the 3D step reads.  Index (i, j, k) with
// i fastest; element (i, j, k) of an array is at k*sz + j*pitch + i.
// Components: E_x (i+1/2, j, k), E_y (i, j+1/2, k), E_z (i, j, k+1/2),
// H_x (i, j+1/2, k+1/2), H_y (i+1/2, j, k+1/2), H_z (i+1/2, j+1/2, k).
// Fields and absorber memories come in two copies (read par, write par^1).
template <typename T>
struct Step3D {
  int n[3];            // nodes per axis
  int pitch;           // row pitch (elements)
  long long sz;        // plane stride (elements)
  int P;               // CPML cells
  int d0[3], dn[3];    // design box
  int g0[3], gn[3];    // gap box
  int lo[3], hi[3];    // total-field box (inclusive nodes)
  int kref, L, tf_on;
  int ng;              // gap cells
  T *E[2][3], *H[2][3];
  // absorber memory of component c along axis u (u != c), slot [c][u]; the
  // forward uses them as psi*dx of the curl terms, the adjoint as nu
  T *pE[2][3][3], *pH[2][3][3];
  T *J;                // Drude currents [3][nd] over the design box
  const T *rho;        // density [nd]
  T *hist;             // forward E on design edges [N][3][nd]
  double *grad;        // sensitivity sums [3][nd]
  double *gapE;        // gap monitor series [N+1][ng][3]
  const T *asrc;       // adjoint source [N+1][ng][3] (scaled by dx and S')
  const T *einc, *hinc;// incident line along z: [N+1][L], [N][L]
  const T *be[3], *ae[3], *ike[3];  // grading per axis at integer positions
  const T *bh[3], *ah[3], *ikh[3];  // and at half positions
  T ch;                // dt / (mu0 dx)
  T ce_s, ce_g;        // dt / (eps0 eps dx)
  T A0, A1, B0, B1, Sg, dt_, dtdx, dthJ, kp;
  T ga, gsm, rs;
};

template <typename T>
void launch_step3d(const Step3D<T> &p, int n, int par, bool adjoint, hipStream_t s);

}  // namespace fdtd
