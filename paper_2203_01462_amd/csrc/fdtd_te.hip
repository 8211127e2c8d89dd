// fdtd_te.hip -- fused time step of the 2D TEz Drude-FDTD solve (E in the
// plane: E_x, E_y; H along z) and of its adjoint: the paper's plasmonic 2D
// polarization (Sec. 4.1, plane wave along +y with E along x).
//
// Per step (Sec. 3.2 staggering), on the Yee cell E_x(i+1/2, j), E_y(i,
// j+1/2), H_z(i+1/2, j+1/2):
//   H_z^{n+1/2} = H_z^{n-1/2} - dt/mu0 (dE_y/dx - dE_x/dy)            (eq. (10c))
//   E_x: curl H = dH_z/dy;  E_y: curl H = -dH_z/dx;  then the trapezoidal
//   Drude ADE of eqs. (10a-b) on every design edge (one density per edge):
//   E^{n+1} = E^n + dE,  dE = 2/D [dt curl H - dt (1+kp)/2 J^n - (beta+sigma) dt E^n],
//   J^{n+1} = J^n + (kp - 1) J^n + beta (E^{n+1} + E^n).
// CPML memories: H_z's x and y differences, E_x's y difference, E_y's x
// difference; total-field/scattered-field corrections on the box lines.  The
// adjoint (eq. (20)) runs the same update on (E*, H*, J*), each curl acting
// on the field graded by the other field's absorber profile (the exact
// transpose), driven by the gap source, and accumulates the per-edge
// sensitivity of eq. (25) folded with eq. (27) into one FP64 sum.
//
// One lane per column: a wavefront covers 64 columns, lane 0 the halo
// column left of the 63 it updates, and walks a segment of TER rows; at node
// (i, j) a lane updates H_z(i, j), E_x(i, j) and E_y(i, j).  The lower
// neighbour's new H_z is the lane's own from the previous row (the segment's
// first row recomputes it from the read copy), the left neighbour's comes
// from lane - 1 by a cross-lane shuffle; the next row's field values are
// loaded before the current row's arithmetic.  Blocks whose nodes reach the
// design or gap box take one row per wavefront and a body with the design
// and gap code; all other blocks a body without it.  Every array a halo
// reads has a read and a write copy.  This polarization's workloads are small (the
// paper's 2D designs), so the step is a plain per-step kernel without
// temporal blocking.

// Design layout (per edge): the design box of dnx x dny cells holds its E_x
// edges [dny+1][dnx] (density indices 0 .. ndx-1) followed by its E_y edges
// [dny][dnx+1]; the gap box's edges likewise give the monitor order.
#include <algorithm>
#include <cstdint>

#include "fdtd_2d.hpp"

namespace fdtd {
namespace {

#ifndef FDTD_TE_ROWS
#define FDTD_TE_ROWS 4
#endif
#ifndef FDTD_TE_WAVES
#define FDTD_TE_WAVES 4
#endif
// lanes (= columns, the first a halo) per wavefront, wavefronts per
// workgroup, rows per wavefront
constexpr int TEX = 64, TEW = FDTD_TE_WAVES, TER = FDTD_TE_ROWS, TEC = TEX - 1;

// A rectangle of blocks of the per-step tiling: columns [bx0, bx1), row
// bands [by0, by1).
struct TeRect {
  int bx0, bx1, by0, by1;
};

__device__ __forceinline__ bool te_pml_e(int i, int n, int P) { return P > 0 && (i < P || i > n - 1 - P); }
__device__ __forceinline__ bool te_pml_h(int i, int n, int P) { return P > 0 && (i < P || i >= n - 1 - P); }

// Density index of edge (comp, i, j) (comp 0: E_x, 1: E_y), or -1.
template <typename T>
__device__ __forceinline__ int te_design(const Step2D<T> &p, int comp, int i, int j) {
  const int u = i - p.dx0, v = j - p.dy0;
  if (comp == 0) return (u >= 0 && u < p.dnx && v >= 0 && v <= p.dny) ? v * p.dnx + u : -1;
  return (u >= 0 && u <= p.dnx && v >= 0 && v < p.dny) ? p.dnx * (p.dny + 1) + v * (p.dnx + 1) + u : -1;
}

// Monitor index of gap edge (comp, i, j), or -1.
template <typename T>
__device__ __forceinline__ int te_gap(const Step2D<T> &p, int comp, int i, int j) {
  if (p.gnx <= 0 || p.gny <= 0) return -1;
  const int u = i - p.gx0, v = j - p.gy0;
  if (comp == 0) return (u >= 0 && u < p.gnx && v >= 0 && v <= p.gny) ? v * p.gnx + u : -1;
  return (u >= 0 && u <= p.gnx && v >= 0 && v < p.gny) ? p.gnx * (p.gny + 1) + v * (p.gnx + 1) + u : -1;
}

// The E (and J) update of one edge from its curl (raw difference); the
// adjoint also adds the edge's sensitivity term to its FP64 sum.
template <typename T, bool ADJ, bool DES>
__device__ __forceinline__ T te_e(const Step2D<T> &p, int n, int comp, int i, int j, T e0, T curl) {
  const int d = DES ? te_design(p, comp, i, j) : -1, g = DES ? te_gap(p, comp, i, j) : -1;
  const int nd = p.dnx * (p.dny + 1) + (p.dnx + 1) * p.dny;
  if (ADJ && g >= 0) curl += p.asrc[(size_t)n * p.ng + g];
  T e1;
  if (d >= 0 && g < 0) {
    const T x = p.rho[d];
    const T eps2 = p.A0 + x * p.A1;
    const T beta = p.B0 + x * p.B1;
    const T bs = beta * p.dt_ + p.Sg * x * (T(1) - x);
    const T inv = T(2) / (eps2 + bs);
    const T Jo = p.J[d];
    const T dE = inv * (p.dtdx * curl - p.dthJ * Jo - bs * e0);
    e1 = e0 + dE;
    const T Jn = Jo + (p.kpm1 * Jo + beta * (e0 + e1));
    p.J[d] = Jn;
    if (ADJ) {
      const T Em = p.hist[(size_t)(n - 1 - p.hist_base) * nd + d];
      const T gc = -(T(1) - p.rs) / (T(2) * (p.rs + x * (T(1) - p.rs)));
      const T gb = p.gsm * (T(1) - T(2) * x);
      p.grad[d] += (double)(Em * (p.ga * dE + gb * (e0 + e1) + gc * (Jn + Jo)));
    }
  } else {
    e1 = e0 + (g >= 0 ? p.ce_g : p.ce_s) * curl;
  }
  if (!ADJ) {
    if (d >= 0 && p.hist_on) p.hist[(size_t)(n - p.hist_base) * nd + d] = e1;
    if (g >= 0) p.gapE[(size_t)(n + 1) * p.ng + g] = (double)e1;
  }
  return e1;
}

// One launch per step, two kinds of block.  The blocks of the per-step
// tiling (TEC columns by TEW * TER rows) inside the rectangle `dr` -- those
// whose updated nodes reach the design or gap box -- run the body with DES =
// true: design edges (Drude current, history, FP64 sensitivity sums) and gap
// edges compiled in, R = TE_DES_ROWS rows per wavefront.  Every other block
// runs the DES = false body, which has neither.  The design blocks come
// first in the launch, so their dependent loads overlap the background
// blocks, and the background blocks skip the design and gap index tests of
// every edge.  Measured on the 2048^2 workload: 36.0 / 47.0 us per forward
// / adjoint step against 40.7 / 55.7 with the design code in every block
// (64 / 89 VGPRs against 67 / 93), and against 41.0 / 48.5 with the design
// blocks as a launch of their own (9-11 us each, serialized with the
// background launch).  Blocks read only the read copy and write only their
// own nodes.
#ifndef FDTD_TE_DES_ROWS
#define FDTD_TE_DES_ROWS 1
#endif
constexpr int TE_DES_ROWS = FDTD_TE_DES_ROWS;
static_assert(TER % TE_DES_ROWS == 0, "design-block rows must divide the per-step rows");

// Block b of the launch: the first nD are design blocks (gdx columns of
// them), the rest the per-step grid (gx columns) less the rectangle.
struct TeGrid {
  TeRect dr;
  int nD, gdx, gx;
};

// The block's kind (1: design, 0: background, -1: none), its column offset
// and its wavefront's first row.
__device__ __forceinline__ int te_block(const TeGrid &g, int &bx, int &j0) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int b = (int)blockIdx.x;
  if (b < g.nD) {
    bx = g.dr.bx0 + b % g.gdx;
    j0 = g.dr.by0 * TEW * TER + ((b / g.gdx) * TEW + wv) * TE_DES_ROWS;
    return 1;
  }
  b -= g.nD;
  bx = b % g.gx;
  const int by = b / g.gx;
  j0 = (by * TEW + wv) * TER;
  return bx >= g.dr.bx0 && bx < g.dr.bx1 && by >= g.dr.by0 && by < g.dr.by1 ? -1 : 0;
}

// Forward.  Copy 0 read, copy 1 written.  Memories: pex = H_z's x
// difference, pey = H_z's y difference, phx = E_x's (y), phy = E_y's (x).
template <typename T, bool DES, int R>
__device__ __forceinline__ void te_fwd_body(const Step2D<T> &p, int n, int bx, int j0) {
  const int lane = threadIdx.x & 63;
  const int i = bx * TEC + lane - 1;
  const int nx = p.nx, ny = p.ny, P = p.P;
  // rows with an H_z cell or an E edge to update: 0 .. ny-2
  if (j0 > ny - 2) return;  // whole wavefront
  const int j1 = min(j0 + R, ny - 1);
  const size_t pitch = p.pitch;
  const T *__restrict__ Ex = p.ez[0];
  const T *__restrict__ Ey = p.hx[0];
  const T *__restrict__ Hz = p.hy[0];
  const T *__restrict__ mhx = p.pex[0];
  const T *__restrict__ mhy = p.pey[0];
  const T *__restrict__ mex = p.phx[0];
  const T *__restrict__ mey = p.phy[0];
  T *__restrict__ Exw = p.ez[1];
  T *__restrict__ Eyw = p.hx[1];
  T *__restrict__ Hzw = p.hy[1];
  T *__restrict__ mhxw = p.pex[1];
  T *__restrict__ mhyw = p.pey[1];
  T *__restrict__ mexw = p.phx[1];
  T *__restrict__ meyw = p.phy[1];
  const T *ei = p.einc + (size_t)n * p.L, *hi = p.hinc + (size_t)n * p.L;
  const bool hcol = i >= 0 && i <= nx - 2;  // the column holds H_z cells and E_x edges
  const bool own = lane > 0 && hcol;        // ... and is updated by this lane
  const bool ecol = own && i >= 1;          // ... with E_y edges
  const bool pmh = hcol && te_pml_h(i, nx, P), pme = ecol && te_pml_e(i, nx, P);
  const T kxh = hcol ? p.ikxh[i] : T(0), kxe = ecol ? p.ikxe[i] : T(0);
  const bool tfx = p.tf_on && i >= p.ia && i <= p.ib - 1;
  // new H_z at cell (i, b) from its five inputs (and its memories)
  auto hz_of = [&](int b, T eyc, T eyr, T exc, T exn, T hzc, T &sx, T &sy) {
    const size_t r = (size_t)b * pitch + i;
    const T dEy = eyr - eyc;
    const T dEx = exn - exc;
    T tx = dEy * kxh, ty = dEx * p.ikyh[b];
    sx = T(0);
    sy = T(0);
    if (pmh) { sx = p.bxh[i] * mhx[r] + p.axh[i] * dEy; tx += sx; }
    if (te_pml_h(b, ny, P)) { sy = p.byh[b] * mhy[r] + p.ayh[b] * dEx; ty += sy; }
    T h = hzc - p.chx * (tx - ty);
    // the H_z rows just outside the box read E_x on its lower and upper lines
    if (tfx) {
      if (b == p.ja - 1) h -= p.chx * ei[p.ja - p.jref];
      if (b == p.jb) h += p.chx * ei[p.jb - p.jref];
    }
    return h;
  };
  // the lane's column, row j: E_y(i), E_y(i+1), E_x(j), E_x(j+1), H_z
  T eyc = T(0), eyr = T(0), exc = T(0), exn = T(0), hzc = T(0);
  auto load_row = [&](int j, T &a, T &b, T &c, T &d, T &e) {
    const size_t r = (size_t)j * pitch + i;
    a = Ey[r];
    b = Ey[r + 1];
    c = Ex[r];
    d = Ex[r + pitch];
    e = Hz[r];
  };
  // new H_z of the row below the segment
  T hb = T(0);
  if (hcol && j0 >= 1) {
    T a, b, c, d, e, t0, t1;
    load_row(j0 - 1, a, b, c, d, e);
    hb = hz_of(j0 - 1, a, b, c, d, e, t0, t1);
  }
  if (hcol) load_row(j0, eyc, eyr, exc, exn, hzc);
  for (int j = j0; j < j1; ++j) {
    const size_t q = (size_t)j * pitch + i;
    // the next row's values, in flight during this row's arithmetic
    T eyc2 = T(0), eyr2 = T(0), exc2 = T(0), exn2 = T(0), hzc2 = T(0);
    if (hcol && j + 1 < j1) load_row(j + 1, eyc2, eyr2, exc2, exn2, hzc2);
    T h00 = T(0), sx = T(0), sy = T(0);
    if (hcol) h00 = hz_of(j, eyc, eyr, exc, exn, hzc, sx, sy);
    // the left neighbour's new H_z
    const T hl = __shfl_up(h00, 1, 64);
    if (own) {
      Hzw[q] = h00;
      if (pmh) mhxw[q] = sx;
      if (te_pml_h(j, ny, P)) mhyw[q] = sy;
      // E_x(i, j): curl = dH_z/dy; incident H_z = -(the line's transverse H)
      if (j >= 1) {
        const T d = h00 - hb;
        T c = d * p.ikye[j];
        if (te_pml_e(j, ny, P)) {
          const T s = p.bye[j] * mex[q] + p.aye[j] * d;
          mexw[q] = s;
          c += s;
        }
        if (tfx) {
          if (j == p.ja) c += hi[p.ja - 1 - p.jref];
          if (j == p.jb) c -= hi[p.jb - p.jref];
        }
        Exw[q] = te_e<T, false, DES>(p, n, 0, i, j, exc, c);
      }
      // E_y(i, j): curl = -dH_z/dx
      if (ecol) {
        const T d = h00 - hl;
        T g = d * kxe;
        if (pme) {
          const T s = p.bxe[i] * mey[q] + p.axe[i] * d;
          meyw[q] = s;
          g += s;
        }
        T c = -g;
        if (p.tf_on && j >= p.ja && j <= p.jb - 1) {
          if (i == p.ia) c -= hi[j - p.jref];
          if (i == p.ib) c += hi[j - p.jref];
        }
        Eyw[q] = te_e<T, false, DES>(p, n, 1, i, j, eyc, c);
      }
    }
    hb = h00;
    eyc = eyc2;
    eyr = eyr2;
    exc = exc2;
    exn = exn2;
    hzc = hzc2;
  }
}

// Adjoint step m = n: copy 0 holds E*^{m+1/2}, H_z*^{m+1} and the memories
// (nu), copy 1 receives E*^{m-1/2}, H_z*^m.
template <typename T, bool DES, int R>
__device__ __forceinline__ void te_adj_body(const Step2D<T> &p, int n, int bx, int j0) {
  const int lane = threadIdx.x & 63;
  const int i = bx * TEC + lane - 1;
  const int nx = p.nx, ny = p.ny, P = p.P;
  if (j0 > ny - 2) return;  // whole wavefront
  const int j1 = min(j0 + R, ny - 1);
  const size_t pitch = p.pitch;
  const T *__restrict__ Ex = p.ez[0];
  const T *__restrict__ Ey = p.hx[0];
  const T *__restrict__ Hz = p.hy[0];
  const T *__restrict__ mhx = p.pex[0];
  const T *__restrict__ mhy = p.pey[0];
  const T *__restrict__ mex = p.phx[0];
  const T *__restrict__ mey = p.phy[0];
  T *__restrict__ Exw = p.ez[1];
  T *__restrict__ Eyw = p.hx[1];
  T *__restrict__ Hzw = p.hy[1];
  T *__restrict__ mhxw = p.pex[1];
  T *__restrict__ mhyw = p.pey[1];
  T *__restrict__ mexw = p.phx[1];
  T *__restrict__ meyw = p.phy[1];
  const bool hcol = i >= 0 && i <= nx - 2;
  const bool own = lane > 0 && hcol;
  const bool ecol = own && i >= 1;
  const bool pmh = hcol && te_pml_h(i, nx, P);
  // E* graded by the E update's absorber profile (new memory from E* itself);
  // zero on the walls and the unused slots.  gx: E_x* at (i, b), value e;
  // gy: E_y* at (a, b) in this row, value e.
  auto gx = [&](int b, T e) {
    if (!hcol || b < 1 || b > ny - 2) return T(0);
    return e * p.ikye[b] + (te_pml_e(b, ny, P) ? p.bye[b] * mex[(size_t)b * pitch + i] + p.aye[b] * e : T(0));
  };
  auto gy = [&](int a, int b, T e) {
    if (a < 1 || a > nx - 2) return T(0);
    return e * p.ikxe[a] + (te_pml_e(a, nx, P) ? p.bxe[a] * mey[(size_t)b * pitch + a] + p.axe[a] * e : T(0));
  };
  // new H_z* at cell (i, b): the forward curl-E update on the graded E*
  auto hz_of = [&](int b, T eyc, T eyr, T exc, T exn, T hzc) {
    return hzc - p.chx * ((gy(i + 1, b, eyr) - gy(i, b, eyc)) - (gx(b + 1, exn) - gx(b, exc)));
  };
  // H_z* graded by the H update's profile along x (for dH/dx) and y (dH/dy)
  auto hxg = [&](int b, T h) {
    return h * p.ikxh[i] + (pmh ? p.bxh[i] * mhx[(size_t)b * pitch + i] + p.axh[i] * h : T(0));
  };
  auto hyg = [&](int b, T h) {
    return h * p.ikyh[b] + (te_pml_h(b, ny, P) ? p.byh[b] * mhy[(size_t)b * pitch + i] + p.ayh[b] * h : T(0));
  };
  T eyc = T(0), eyr = T(0), exc = T(0), exn = T(0), hzc = T(0);
  auto load_row = [&](int j, T &a, T &b, T &c, T &d, T &e) {
    const size_t r = (size_t)j * pitch + i;
    a = Ey[r];
    b = Ey[r + 1];
    c = Ex[r];
    d = Ex[r + pitch];
    e = Hz[r];
  };
  // y-graded new H_z* of the row below the segment
  T gb = T(0);
  if (hcol && j0 >= 1) {
    T a, b, c, d, e;
    load_row(j0 - 1, a, b, c, d, e);
    gb = hyg(j0 - 1, hz_of(j0 - 1, a, b, c, d, e));
  }
  if (hcol) load_row(j0, eyc, eyr, exc, exn, hzc);
  for (int j = j0; j < j1; ++j) {
    const size_t q = (size_t)j * pitch + i;
    T eyc2 = T(0), eyr2 = T(0), exc2 = T(0), exn2 = T(0), hzc2 = T(0);
    if (hcol && j + 1 < j1) load_row(j + 1, eyc2, eyr2, exc2, exn2, hzc2);
    T h00 = T(0), gyo = T(0), gxo = T(0);
    if (hcol) {
      h00 = hz_of(j, eyc, eyr, exc, exn, hzc);
      gyo = hyg(j, h00);
      gxo = hxg(j, h00);
    }
    // the left neighbour's x-graded new H_z*
    const T gl = __shfl_up(gxo, 1, 64);
    if (own) {
      // own memories of E* (driven by E* of copy 0)
      if (j >= 1 && te_pml_e(j, ny, P)) mexw[q] = p.bye[j] * mex[q] + p.aye[j] * exc;
      if (ecol && te_pml_e(i, nx, P)) meyw[q] = p.bxe[i] * mey[q] + p.axe[i] * eyc;
      Hzw[q] = h00;
      if (pmh) mhxw[q] = p.bxh[i] * mhx[q] + p.axh[i] * h00;
      if (te_pml_h(j, ny, P)) mhyw[q] = p.byh[j] * mhy[q] + p.ayh[j] * h00;
      if (j >= 1) Exw[q] = te_e<T, true, DES>(p, n, 0, i, j, exc, gyo - gb);
      if (ecol) Eyw[q] = te_e<T, true, DES>(p, n, 1, i, j, eyc, -(gxo - gl));
    }
    gb = gyo;
    eyc = eyc2;
    eyr = eyr2;
    exc = exc2;
    exn = exn2;
    hzc = hzc2;
  }
}

template <typename T>
__global__ void __launch_bounds__(TEX * TEW) step_te_fwd(const Step2D<T> p, int n, TeGrid g) {
  int bx, j0;
  const int kind = te_block(g, bx, j0);
  if (kind == 1) te_fwd_body<T, true, TE_DES_ROWS>(p, n, bx, j0);
  else if (kind == 0) te_fwd_body<T, false, TER>(p, n, bx, j0);
}

template <typename T>
__global__ void __launch_bounds__(TEX * TEW) step_te_adj(const Step2D<T> p, int n, TeGrid g) {
  int bx, j0;
  const int kind = te_block(g, bx, j0);
  if (kind == 1) te_adj_body<T, true, TE_DES_ROWS>(p, n, bx, j0);
  else if (kind == 0) te_adj_body<T, false, TER>(p, n, bx, j0);
}

// The blocks whose updated nodes (i, j) reach the design box's edges (i in
// dx0 .. dx0+dnx, j in dy0 .. dy0+dny) or the gap box's; empty if neither
// box is.
template <typename T>
TeRect te_rect(const Step2D<T> &p) {
  int ilo = INT32_MAX, ihi = -1, jlo = INT32_MAX, jhi = -1;
  auto box = [&](int x0, int nxb, int y0, int nyb) {
    if (nxb <= 0 || nyb <= 0) return;
    ilo = std::min(ilo, x0);
    ihi = std::max(ihi, x0 + nxb);
    jlo = std::min(jlo, y0);
    jhi = std::max(jhi, y0 + nyb);
  };
  box(p.dx0, p.dnx, p.dy0, p.dny);
  box(p.gx0, p.gnx, p.gy0, p.gny);
  if (ihi < 0) return TeRect{0, 0, 0, 0};
  const int rows = TEW * TER;
  return TeRect{ilo / TEC, ihi / TEC + 1, jlo / rows, jhi / rows + 1};
}

}  // namespace

template <typename T>
void launch_step_te(const Step2D<T> &p, int n, bool adjoint, hipStream_t s) {
  TeGrid g;
  g.dr = te_rect(p);
  g.gx = (p.nx + TEC - 1) / TEC;
  g.gdx = g.dr.bx1 - g.dr.bx0;
  g.nD = g.gdx * (g.dr.by1 - g.dr.by0) * (TER / TE_DES_ROWS);
  const int gy = (p.ny + TEW * TER - 1) / (TEW * TER);
  const dim3 grid((unsigned)(g.nD + g.gx * gy));
  if (adjoint) hipLaunchKernelGGL(step_te_adj<T>, grid, dim3(TEX * TEW), 0, s, p, n, g);
  else hipLaunchKernelGGL(step_te_fwd<T>, grid, dim3(TEX * TEW), 0, s, p, n, g);
}

template void launch_step_te<float>(const Step2D<float> &, int, bool, hipStream_t);
template void launch_step_te<double>(const Step2D<double> &, int, bool, hipStream_t);

}  // namespace fdtd
