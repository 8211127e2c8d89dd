// fdtd_3d.hpp -- state layout and parameters of the 3D step kernels.
#pragma once

#include <cstdint>
#include <vector>

#include "fdtd_internal.hpp"

namespace fdtd {

// One copy of the 3D state lives in one device allocation (an "arena"), so a
// kernel reaches every field and absorber memory through a single base
// pointer and 32-bit element offsets.  Offsets in elements:
//   [0, G0)          guard, permanently zero: every neighbour offset of an
//                    in-grid node stays inside the arena, and predicated-off
//                    loads read element 0
//   G0 + c*S         field c = E_x, E_y, E_z, H_x, H_y, H_z; node (i, j, k)
//                    at k*PL + j*pitch + i.  E_x sits at (i+1/2, j, k),
//                    H_x at (i, j+1/2, k+1/2), and so on (full Yee cell).
//   xs + s*XS        x-absorber memories s = H_y, H_z, E_y, E_z along x,
//                    node at (k*ny + j)*W + sx(i)
//   ys + s*YS        y-absorber memories s = H_x, H_z, E_x, E_z along y,
//                    node at (k*W + sy(j))*pitch + i
//   zs + s*ZS        z-absorber memories s = H_x, H_y, E_x, E_y along z,
//                    node at (sz(k)*ny + j)*pitch + i
//   ... tail guard
// W = 2P + 1 nodes per axis hold every absorber position of E (integer
// positions i < P or i > n-1-P) and of H (half positions, i < P or
// i >= n-1-P): s?(i) = i for i < P, i - (n - 1 - 2P) otherwise.
#ifndef FDTD3D_SKEW
#define FDTD3D_SKEW 4160
#endif
#ifndef FDTD3D_PITCH_PAD
#define FDTD3D_PITCH_PAD 0
#endif

struct Arena3 {
  uint32_t G0, S, PL, xs, ys, zs, XS, YS, ZS, W;
  uint64_t total;  // elements
};

inline Arena3 arena3_layout(int ny, int nz, int pitch, int P) {
  auto up = [](uint64_t v) { return (v + 63) & ~uint64_t(63); };
  Arena3 a{};
  const uint64_t PL = (uint64_t)pitch * ny;
  const uint64_t G0 = up(PL + pitch + 64);
  // arrays are skewed off power-of-two strides so that the same node of the
  // six fields does not land in one L2 set
  const uint64_t S = up(PL * nz) + FDTD3D_SKEW;
  const uint64_t W = P > 0 ? 2 * (uint64_t)P + 1 : 0;
  const uint64_t XS = up((uint64_t)nz * ny * W), YS = up((uint64_t)nz * W * pitch), ZS = up(W * PL);
  const uint64_t xs = G0 + 6 * S, ys = xs + 4 * XS, zs = ys + 4 * YS, end = zs + 4 * ZS + G0;
  a.G0 = (uint32_t)G0; a.S = (uint32_t)S; a.PL = (uint32_t)PL;
  a.xs = (uint32_t)xs; a.ys = (uint32_t)ys; a.zs = (uint32_t)zs;
  a.XS = (uint32_t)XS; a.YS = (uint32_t)YS; a.ZS = (uint32_t)ZS; a.W = (uint32_t)W;
  a.total = end;
  return a;
}

// Everything one launch of the 3D step reads.
template <typename T>
struct Step3D {
  int n[3];            // nodes per axis
  int pitch;           // row pitch (elements)
  int P;               // CPML cells
  int d0[3], dn[3];    // design box
  int g0[3], gn[3];    // gap box
  int lo[3], hi[3];    // total-field box (inclusive nodes)
  int kref, L, tf_on;
  int ng;              // gap cells
  uint32_t G0, S, PL, xs, ys, zs, XS, YS, ZS, W;  // arena layout
  T *A[2];             // the two state copies; the launcher passes read in A[0], write in A[1]
  T *J;                // Drude currents [3][nd] over the design box
  const T *rho;        // density [nd]
  T *hist;             // forward E on design edges [N][3][nd]
  double *grad;        // sensitivity sums [3][nd]
  int hist_base, hist_on;  // history slot of step n is n - hist_base; the forward writes it when hist_on
  double *gapE;        // gap monitor series [N+1][ng][3]
  const T *asrc;       // adjoint source [N+1][ng][3] (scaled by dx and S')
  const T *einc, *hinc;// incident line along z: [N+1][L], [N][L]
  const T *tab;        // CPML tables [axis][b_E, a_E, 1/kappa_E, b_H, a_H, 1/kappa_H][tn]
  int tn;              // table length (largest axis)
  T ch;                // dt / (mu0 dx)
  T ce_s, ce_g;        // dt / (eps0 eps dx)
  T A0, A1, B0, B1, Sg, dt_, dtdx, dthJ, kpm1;  // kpm1 = kp - 1 = -gamma dt / (1 + gamma dt / 2), rounded once from FP64
  T ga, gsm, rs;
  // tile-chunk lists of the general update (device, from gen3d_plan):
  // [single-axis | multi-axis | design], lengths gS, gM, gD; gAxD = the
  // absorber axes the design chunks reach (0 or 7)
  const int *glist;
  int gS, gM, gD, gAxD;
  int pb[6];  // bounding box of the plain tile-planes: origin x, y, z, extent x, y, z (from plain3d_box)
  // Two-step blocking of the plain background (see plan3d_super): the grid of
  // super-chunks (origin so, chunk counts sn), one flag byte per chunk
  // (non-zero: the chunk advances two steps per pass), and whether a
  // per-step launch leaves the super-chunks' nodes to the two-step pass.
  const unsigned char *sflag;
  int so[3], sn[3];
  int skip_super;
  T *Amid;  // two-step pass: the copy that receives the intermediate state of the chunks' border nodes
};

// Two-step super-chunks: 60 x 16 x 8 nodes (a wavefront spans 64 columns, two
// of halo on each side; four wavefronts of four rows each).
constexpr int SCX = 60, SCY = 16, SCZ = 8;

// The chunks of plain background that advance two time steps per pass: every
// node of the chunk lies in a plain tile-plane of the general tiling and all
// nodes within three of it (in each axis) are plain background (no absorber,
// wall, injection line or face, design or gap).  Fills the grid (origin so,
// counts sn, flags per chunk) and returns the launch list: per chunk
// (index << 6) | border faces (bit f set: face f = x-, x+, y-, y+, z-, z+
// touches a node outside the super-chunks, whose neighbours read the chunk's
// intermediate state there), ordered for the 8 XCDs and padded with -1.
template <typename T>
std::vector<int> plan3d_super(const Step3D<T> &p, int so[3], int sn[3], std::vector<unsigned char> &flags);

// Tile-chunks of the general update, sorted by what they need: one or no
// absorber axis (code 4c + axis, axis 3 = none), several axes, the design or
// gap boxes (code c); chunks without a general plane are left out.  Each
// list is ordered for the 8 XCDs (groups of neighbouring chunks dealt to
// the XCD with the least work so far, then interleaved) and padded with -1
// to a multiple of 8.  The geometry fields of p are read (not the pointers).
template <typename T>
std::vector<int> gen3d_plan(const Step3D<T> &p, int &nS, int &nM, int &nD, int &axD);

// Bounding box of the tile-planes that take the plain update (extent 0
// when there are none); the plain launch covers only this box.
template <typename T>
void plain3d_box(const Step3D<T> &p, int pb[6]);

// A second stream and two events (created without timing) of a context:
// where the general update is three launches (the adjoint, FP64), the one
// over multi-axis chunks runs on `stream` beside the design and single-axis
// launches on the main stream, joined before the plain launch.  A null
// stream keeps all launches on the main stream.
struct Aux3D {
  hipStream_t stream;
  hipEvent_t fork, join;
};

// One time step: copy rd read, copy wr written (general launches, then the
// plain launch, which skips the super-chunks when p.skip_super is set).
template <typename T>
void launch_step3d(const Step3D<T> &p, T *rd, T *wr, int n, bool adjoint, hipStream_t s, const Aux3D &aux);

// The two-step pass over `count` listed super-chunks: reads copy rd (state
// after s steps), writes the state after s + 2 into out and the border nodes'
// state after s + 1 into mid.  FP32 only.
void launch_step3d_super(const Step3D<float> &p, const float *rd, float *mid, float *out, const int *list, int count,
                         hipStream_t s);

}  // namespace fdtd
