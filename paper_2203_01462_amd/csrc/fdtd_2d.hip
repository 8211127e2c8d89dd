// fdtd_2d.hip -- fused time step of the 2D TMz Drude-FDTD solve and of its
// adjoint: one launch per time step (step2d_kernel), or, with two-step
// blocking of the plain background, two launches per two time steps
// (step2d_mix_kernel, see the two-step section below).
//
// Per step (Sec. 3.2 staggering: E, J at integer steps, H at half steps):
//   H^{n+1/2} = H^{n-1/2} - dt/mu0 curl E^n                 (eq. (10c), CPML, TFSF)
//   E^{n+1}   = E^n + dE,  dE = 2/D [dt curl H^{n+1/2} - dt (1+kp)/2 J^n - (beta+sigma) dt E^n]
//   J^{n+1}   = J^n + (kp - 1) J^n + beta (E^{n+1} + E^n)   (eqs. (10a-b), trapezoidal ADE)
// with the per-edge coefficients of eqs. (4)-(5) evaluated in registers from
// rho (D = 2 eps0 eps_inf_i + (beta_i + sigma_i) dt).  The adjoint step
// (eq. (20)) is the same update on (E*, H*, J*) driven by the gap source, with
// the absorber replaced by its exact transpose: the grading 1/kappa and the
// recursive memory act on the field before the difference, not after it.
// The adjoint also accumulates the sensitivity of eq. (25), folded with the
// chain rule of eq. (27) into one FP64 sum per design edge:
//   g_i += E_i^m [ga dE*_i + gb (E*_i^{m-1/2} + E*_i^{m+1/2}) + gc (J*_i^{m-1/2} + J*_i^{m+1/2})].
//
// Layout: a wavefront owns a 64 x 2 tile of E nodes (four wavefronts stacked
// along y form a workgroup); each thread owns one column segment of 2 nodes.
// Wavefronts whose tile (with its halo) touches only the plain background take
// a lean path with the dielectric update alone.  It issues all of its loads at once (E over the
// segment plus one node above/below/left/right, the old H it needs), computes
// H for its segment plus the low-side halo (H_x one row below, H_y one column
// to the left) from those values, writes its own H, then updates E.  No LDS
// and no barrier: neighbour values come through the caches.  All arrays that
// a halo reads come in a read and a write copy, so the step needs no
// grid-wide synchronisation.
#include <utility>

#include "fdtd_2d.hpp"

namespace fdtd {
namespace {

#ifndef FDTD2D_ROWS
#define FDTD2D_ROWS 2
#endif
#ifndef FDTD2D_MIN_WAVES
#define FDTD2D_MIN_WAVES 1
#endif
#ifndef FDTD2D_XCD_REMAP
#define FDTD2D_XCD_REMAP 2
#endif
constexpr int WAVES = 4;          // wavefronts per workgroup, stacked along y
constexpr int NT = 64 * WAVES;    // threads per workgroup
constexpr int TXW = 64;           // tile width (nodes along x): one wavefront
constexpr int RDEF = FDTD2D_ROWS; // default rows per thread; a wavefront covers 64 x R nodes

__device__ __forceinline__ bool pml_e(int i, int n, int P) { return P > 0 && (i < P || i > n - 1 - P); }
__device__ __forceinline__ bool pml_h(int i, int n, int P) { return P > 0 && (i < P || i >= n - 1 - P); }

// Workgroup -> tile map.  Consecutive dispatch slots go round-robin over the
// 8 XCDs (each with its own L2).  Mode 2 (default) gives XCD x whole tile-rows
// x, x+8, x+16, ...: horizontal neighbours share an L2, and the absorber,
// design and gap rows (the slower wavefronts) spread evenly over the XCDs.
// Mode 1 gives each XCD one contiguous band of tile-rows; mode 0 keeps the
// plain order.
__device__ __forceinline__ void tile_of(int bid, int nbx, int nby, int &tx, int &ty) {
  int t = bid;
  if (FDTD2D_XCD_REMAP == 1 && (nby * nbx) % 8 == 0) t = (bid & 7) * (nbx * nby / 8) + (bid >> 3);
  if (FDTD2D_XCD_REMAP == 2 && nby % 8 == 0) {
    const int k = bid >> 3;
    tx = k % nbx;
    ty = (bid & 7) + 8 * (k / nbx);
    return;
  }
  tx = t % nbx;
  ty = t / nbx;
}

// Every array a step touches is device memory.  The batched kernels copy
// their parameter blocks from device memory, which leaves the compiler
// unable to tell where the pointers point: it would reach the arrays with
// flat instructions, which also count against the LDS wait counter.  With
// G their update code addresses the arrays through global-space pointers.
// (The single-context kernels get their pointers as kernel arguments, which
// the compiler already knows to be global; there the casts only add scalar
// register pressure.)
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <bool G, typename T>
__device__ __forceinline__ auto gp(T *q) {
  if constexpr (G) return (gptr<T>)q;
  else return q;
}

// Branch-free predicated load: reads base[q] when `on`, else base[0] (always
// a valid address) and returns 0.
template <typename T>
__device__ __forceinline__ T ldp(const T *__restrict__ base, size_t q, bool on) {
  const T v = base[on ? q : 0];
  return on ? v : T(0);
}
template <typename T>
__device__ __forceinline__ T ldp(const gptr<const T> __restrict__ base, size_t q, bool on) {
  const T v = base[on ? q : 0];
  return on ? v : T(0);
}

// The step kernel is latency-bound unless every global load of a column
// segment is in flight before the first dependent use: all workgroups are
// resident at once on this grid, so the slowest column (absorber, design or
// gap) sets the launch time.  Hence three phases -- predicated loads, pure
// register arithmetic, stores -- with restrict-qualified pointers.
// A wavefront tile is an edge tile if it (or its one-node halo) touches an
// absorber cell, a wall or a total-field line.
template <int R>
__device__ __forceinline__ bool wave_is_edge(const int nx, const int ny, const int P, const int i0, const int jb,
                                             const int ia, const int ib, const int ja, const int jbt) {
  if (i0 < P + 2 || i0 + TXW > nx - 2 - P || jb < P + 2 || jb + R > ny - 2 - P) return true;
  const int x0 = i0 - 1, x1 = i0 + TXW, y0 = jb - 1, y1 = jb + R;
  auto hit = [](int lo, int hi, int v) { return v >= lo && v <= hi; };
  if (hit(x0, x1, ia - 1) || hit(x0, x1, ia) || hit(x0, x1, ib) || hit(x0, x1, ib + 1)) return true;
  return hit(y0, y1, ja - 1) || hit(y0, y1, ja) || hit(y0, y1, jbt) || hit(y0, y1, jbt + 1);
}

// Does the wavefront's 64 x R block of E nodes meet the box [x0,x0+nx) x [y0,y0+ny)?
template <int R>
__device__ __forceinline__ bool wave_touches_box(const int i0, const int jb, const int x0, const int y0, const int bnx,
                                                 const int bny) {
  return i0 + TXW - 1 >= x0 && i0 < x0 + bnx && jb + R - 1 >= y0 && jb < y0 + bny;
}

// Tiles that are neither edge tiles nor touch the design or gap box need only
// the plain dielectric update, identical in the forward and adjoint solves.
template <typename T, int R, bool G>
__device__ __forceinline__ void step_bulk(const Step2D<T> &p, const int par, const int i, const int jb) {
  const int pitch = p.pitch;
  auto *__restrict__ ez = gp<G>((const T *)p.ez[par]);
  auto *__restrict__ hxo = gp<G>((const T *)p.hx[par]);
  auto *__restrict__ hyo = gp<G>((const T *)p.hy[par]);
  auto *__restrict__ ezw = gp<G>(p.ez[par ^ 1]);
  auto *__restrict__ hxw = gp<G>(p.hx[par ^ 1]);
  auto *__restrict__ hyw = gp<G>(p.hy[par ^ 1]);
  const size_t q0 = (size_t)jb * pitch + i;
  T e[R + 2], er[R], el[R], hx[R + 1], hy[R], hyl[R];
#pragma unroll
  for (int r = 0; r < R + 2; ++r) e[r] = ez[q0 + (size_t)(r - 1) * pitch];
#pragma unroll
  for (int r = 0; r < R + 1; ++r) hx[r] = hxo[q0 + (size_t)(r - 1) * pitch];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const size_t q = q0 + (size_t)r * pitch;
    er[r] = ez[q + 1];
    el[r] = ez[q - 1];
    hy[r] = hyo[q];
    hyl[r] = hyo[q - 1];
  }
  const T ch = p.chx, ce = p.ce_s;
  T hxn[R + 1];
#pragma unroll
  for (int r = 0; r < R + 1; ++r) hxn[r] = hx[r] - ch * (e[r + 1] - e[r]);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const size_t q = q0 + (size_t)r * pitch;
    const T h = hy[r] + ch * (er[r] - e[r + 1]);
    const T hl = hyl[r] + ch * (e[r + 1] - el[r]);
    hxw[q] = hxn[r + 1];
    hyw[q] = h;
    ezw[q] = e[r + 1] + ce * ((h - hl) - (hxn[r + 1] - hxn[r]));
  }
}

// Absorber, wall, total-field, design and gap nodes.  EDGE = false compiles
// the absorber and plane-wave terms out (interior design/gap wavefronts),
// DES = false the design and gap terms (edge wavefronts away from both
// boxes: their loads, arithmetic and stores).
template <typename T, bool ADJ, bool EDGE, int R, bool G, bool DES = true>
__device__ __forceinline__ void step_general(const Step2D<T> &p, const int n, const int par, const int i,
                                             const int jb) {
  const int nx = p.nx, ny = p.ny, pitch = p.pitch, P = EDGE ? p.P : 0;
  if (i >= nx) return;
  const int wr = par ^ 1;
  auto *__restrict__ ez = gp<G>((const T *)p.ez[par]);
  auto *__restrict__ hxo = gp<G>((const T *)p.hx[par]);
  auto *__restrict__ hyo = gp<G>((const T *)p.hy[par]);
  auto *__restrict__ pexo = gp<G>((const T *)p.pex[par]);
  auto *__restrict__ peyo = gp<G>((const T *)p.pey[par]);
  auto *__restrict__ phxo = gp<G>((const T *)p.phx[par]);
  auto *__restrict__ phyo = gp<G>((const T *)p.phy[par]);
  auto *__restrict__ ezw = gp<G>(p.ez[wr]);
  auto *__restrict__ hxw = gp<G>(p.hx[wr]);
  auto *__restrict__ hyw = gp<G>(p.hy[wr]);
  auto *__restrict__ pexw = gp<G>(p.pex[wr]);
  auto *__restrict__ peyw = gp<G>(p.pey[wr]);
  auto *__restrict__ phxw = gp<G>(p.phx[wr]);
  auto *__restrict__ phyw = gp<G>(p.phy[wr]);
  auto *__restrict__ rho = gp<G>((const T *)p.rho);
  auto *__restrict__ Jc = gp<G>(p.J);
  auto *__restrict__ hist = gp<G>(p.hist);
  auto *__restrict__ grad = gp<G>(p.grad);

  const bool hasl = i >= 1, hasr = i + 1 < nx;
  const bool colx = i >= 1 && i <= nx - 2;       // E node column / H_x column
  const bool coly = i <= nx - 2;                  // H_y at (i+1/2)
  const bool pxe = pml_e(i, nx, P), pxh = pml_h(i, nx, P);
  const bool pxhl = hasl && pml_h(i - 1, nx, P);
  const bool pxel = hasl && pml_e(i - 1, nx, P), pxer = hasr && pml_e(i + 1, nx, P);
  const int nd = p.dnx * p.dny;
  const int di = i - p.dx0, gi = i - p.gx0;
  const bool dcol = DES && colx && di >= 0 && di < p.dnx, gcol = DES && colx && gi >= 0 && gi < p.gnx;
  const bool tfx = (EDGE && p.tf_on) && i >= p.ia && i <= p.ib;
  const bool tfy = (EDGE && p.tf_on) && (i == p.ia - 1 || i == p.ia || i == p.ib || i == p.ib + 1);

  // ---------------------------------------------------------------- loads
  // Every load is unconditional: a predicated-off load reads element 0 of its
  // array (one cache line for the whole wavefront) and its value is dropped.
  // Branch-free loads stay in flight together; branches around them would
  // make the compiler wait at every join.
  T e[R + 2], er[R], el[R], hx[R + 1], hy[R], hyl[R];
  T phx[R + 1], phy[R], phyl[R], pex[R], pey[R + 2], pexr[R], pexl[R];
  T rr[R], Jo[R], Em[R], src[R], einc_r[R];
  double gacc[R];
#pragma unroll
  for (int r = 0; r < R + 2; ++r) {
    const int j = jb - 1 + r;
    const bool ok = j >= 0 && j < ny;
    const size_t q = (size_t)(ok ? j : 0) * pitch + i;
    e[r] = ldp(ez, q, ok);
    const bool wpe = ADJ ? (ok && pml_e(j, ny, P)) : (r >= 1 && r <= R && colx && j <= ny - 2 && ok && pml_e(j, ny, P));
    pey[r] = ldp(peyo, q, wpe);
    if (r <= R) {
      hx[r] = ldp(hxo, q, ok);
      phx[r] = ldp(phxo, q, colx && ok && j <= ny - 2 && pml_h(j, ny, P));
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = jb + r;
    const bool ok = j < ny;
    const bool inner = j >= 1 && j <= ny - 2;
    const size_t q = (size_t)(ok ? j : 0) * pitch + i;
    er[r] = ldp(ez, q + 1, ok && hasr);
    el[r] = ldp(ez, q - 1, ok && hasl);
    hy[r] = ldp(hyo, q, ok);
    hyl[r] = ldp(hyo, q - 1, ok && hasl);
    phy[r] = ldp(phyo, q, inner && coly && pxh);
    phyl[r] = ldp(phyo, q - 1, inner && pxhl);
    pex[r] = ldp(pexo, q, ok && pxe && (ADJ || (colx && inner)));
    pexr[r] = ldp(pexo, q + 1, ADJ && ok && pxer);
    pexl[r] = ldp(pexo, q - 1, ADJ && ok && pxel);
    const int dj = j - p.dy0, gj = j - p.gy0;
    const bool des = dcol && inner && dj >= 0 && dj < p.dny;
    const bool gap = gcol && inner && gj >= 0 && gj < p.gny;
    const size_t d = (size_t)(des ? dj * p.dnx + di : 0);
    rr[r] = ldp(rho, d, des);
    Jo[r] = ldp(gp<G>((const T *)p.J), d, des && !gap);
    Em[r] = ldp(gp<G>((const T *)p.hist), (size_t)(n - 1 - p.hist_base) * nd + d, ADJ && des && !gap);
    gacc[r] = ldp(gp<G>((const double *)p.grad), d, ADJ && des && !gap);
    src[r] = ldp(gp<G>(p.asrc), (size_t)n * p.ng + (gap ? gj * p.gnx + gi : 0), ADJ && gap);
    const bool tfr = !ADJ && tfy && j >= p.ja && j <= p.jb;
    einc_r[r] = ldp(gp<G>(p.einc), (size_t)n * p.L + (tfr ? j - p.jref : 0), tfr);
  }
  T eA = T(0), eB = T(0), hA = T(0), hB = T(0);
  if (!ADJ && EDGE && p.tf_on) {
    eA = gp<G>(p.einc)[(size_t)n * p.L + (p.ja - p.jref)];
    eB = gp<G>(p.einc)[(size_t)n * p.L + (p.jb - p.jref)];
    hA = gp<G>(p.hinc)[(size_t)n * p.L + (p.ja - 1 - p.jref)];
    hB = gp<G>(p.hinc)[(size_t)n * p.L + (p.jb - p.jref)];
  }

  // ---------------------------------------------------------------- H
  // hxv[r]: H_x at (i, jb-1+r); hyv/hylv[r]: H_y at (i+1/2, jb+r) / (i-1/2, jb+r).
  // Forward: the new field.  Adjoint: the graded new field H*/kappa + nu.
  T hxv[R + 1], hxn[R + 1], hyv[R], hyn[R], hylv[R];
  T phxn[R + 1], phyn[R], peyn[R + 2], pexn[R];
  if (!ADJ) {
#pragma unroll
    for (int r = 0; r < R + 1; ++r) {
      const int j = jb - 1 + r;
      T h = T(0), ps = T(0);
      if (colx && j >= 0 && j <= ny - 2) {
        const T dE = e[r + 1] - e[r];
        if (pml_h(j, ny, P)) {
          ps = gp<G>(p.byh)[j] * phx[r] + gp<G>(p.ayh)[j] * dE;
          h = hx[r] - p.chx * (dE * gp<G>(p.ikyh)[j] + ps);
        } else {
          h = hx[r] - p.chx * dE;
        }
        if (tfx && j == p.ja - 1) h += p.chx * eA;
        if (tfx && j == p.jb) h -= p.chx * eB;
      }
      hxv[r] = h;
      hxn[r] = h;
      phxn[r] = ps;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = jb + r;
      T h = T(0), hl = T(0), ps = T(0);
      if (j >= 1 && j <= ny - 2) {
        const bool tfr = j >= p.ja && j <= p.jb;
        if (coly) {
          const T dE = er[r] - e[r + 1];
          if (pxh) {
            ps = gp<G>(p.bxh)[i] * phy[r] + gp<G>(p.axh)[i] * dE;
            h = hy[r] + p.chx * (dE * gp<G>(p.ikxh)[i] + ps);
          } else {
            h = hy[r] + p.chx * dE;
          }
          if (tfr && i == p.ia - 1) h -= p.chx * einc_r[r];
          if (tfr && i == p.ib) h += p.chx * einc_r[r];
        }
        if (hasl) {
          const T dE = e[r + 1] - el[r];
          if (pxhl) {
            const T psl = gp<G>(p.bxh)[i - 1] * phyl[r] + gp<G>(p.axh)[i - 1] * dE;
            hl = hyl[r] + p.chx * (dE * gp<G>(p.ikxh)[i - 1] + psl);
          } else {
            hl = hyl[r] + p.chx * dE;
          }
          if (tfr && i - 1 == p.ia - 1) hl -= p.chx * einc_r[r];
          if (tfr && i - 1 == p.ib) hl += p.chx * einc_r[r];
        }
      }
      hyv[r] = h;
      hyn[r] = h;
      hylv[r] = hl;
      phyn[r] = ps;
    }
  } else {
    T gy[R + 2], gx[R], gxr[R], gxl[R];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
      const int j = jb - 1 + r;
      gy[r] = e[r];
      peyn[r] = T(0);
      if (j >= 0 && j < ny && pml_e(j, ny, P)) {
        peyn[r] = gp<G>(p.bye)[j] * pey[r] + gp<G>(p.aye)[j] * e[r];
        gy[r] = e[r] * gp<G>(p.ikye)[j] + peyn[r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      gx[r] = e[r + 1];
      pexn[r] = T(0);
      if (pxe) {
        pexn[r] = gp<G>(p.bxe)[i] * pex[r] + gp<G>(p.axe)[i] * e[r + 1];
        gx[r] = e[r + 1] * gp<G>(p.ikxe)[i] + pexn[r];
      }
      gxr[r] = pxer ? er[r] * gp<G>(p.ikxe)[i + 1] + (gp<G>(p.bxe)[i + 1] * pexr[r] + gp<G>(p.axe)[i + 1] * er[r]) : er[r];
      gxl[r] = pxel ? el[r] * gp<G>(p.ikxe)[i - 1] + (gp<G>(p.bxe)[i - 1] * pexl[r] + gp<G>(p.axe)[i - 1] * el[r]) : el[r];
    }
#pragma unroll
    for (int r = 0; r < R + 1; ++r) {
      const int j = jb - 1 + r;
      T h = T(0), g = T(0), nu = T(0);
      if (colx && j >= 0 && j <= ny - 2) {
        h = hx[r] - p.chx * (gy[r + 1] - gy[r]);
        g = h;
        if (pml_h(j, ny, P)) {
          nu = gp<G>(p.byh)[j] * phx[r] + gp<G>(p.ayh)[j] * h;
          g = h * gp<G>(p.ikyh)[j] + nu;
        }
      }
      hxn[r] = h;
      hxv[r] = g;
      phxn[r] = nu;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = jb + r;
      T h = T(0), g = T(0), gl = T(0), nu = T(0);
      if (j >= 1 && j <= ny - 2) {
        if (coly) {
          h = hy[r] + p.chx * (gxr[r] - gx[r]);
          g = h;
          if (pxh) {
            nu = gp<G>(p.bxh)[i] * phy[r] + gp<G>(p.axh)[i] * h;
            g = h * gp<G>(p.ikxh)[i] + nu;
          }
        }
        if (hasl) {
          const T hl = hyl[r] + p.chx * (gx[r] - gxl[r]);
          gl = hl;
          if (pxhl) gl = hl * gp<G>(p.ikxh)[i - 1] + (gp<G>(p.bxh)[i - 1] * phyl[r] + gp<G>(p.axh)[i - 1] * hl);
        }
      }
      hyn[r] = h;
      hyv[r] = g;
      hylv[r] = gl;
      phyn[r] = nu;
    }
  }

  // ---------------------------------------------------------------- E, J
  T en[R], Jn[R], pexf[R], peyf[R];
  double gnew[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = jb + r;
    const T dHy = hyv[r] - hylv[r];
    const T dHx = hxv[r + 1] - hxv[r];
    T curl;
    pexf[r] = T(0);
    peyf[r] = T(0);
    if (!ADJ) {
      T cx = dHy, cy = dHx;
      if (pxe) {
        pexf[r] = gp<G>(p.bxe)[i] * pex[r] + gp<G>(p.axe)[i] * dHy;
        cx = dHy * gp<G>(p.ikxe)[i] + pexf[r];
      }
      if (pml_e(j, ny, P)) {
        peyf[r] = gp<G>(p.bye)[j] * pey[r + 1] + gp<G>(p.aye)[j] * dHx;
        cy = dHx * gp<G>(p.ikye)[j] + peyf[r];
      }
      curl = cx - cy;
      if (tfx && j == p.ja) curl += hA;
      if (tfx && j == p.jb) curl -= hB;
    } else {
      curl = dHy - dHx + src[r];
    }
    const int gj = j - p.gy0, dj = j - p.dy0;
    const bool gap = gcol && gj >= 0 && gj < p.gny;
    const bool des = dcol && dj >= 0 && dj < p.dny;
    const T e0 = e[r + 1];
    T e1;
    Jn[r] = T(0);
    gnew[r] = 0.0;
    if (des && !gap) {
      const T x = rr[r];
      const T eps2 = p.A0 + x * p.A1;
      const T beta = p.B0 + x * p.B1;
      const T bs = beta * p.dt_ + p.Sg * x * (T(1) - x);
      const T inv = T(2) / (eps2 + bs);
      const T dE = inv * (p.dtdx * curl - p.dthJ * Jo[r] - bs * e0);
      e1 = e0 + dE;
      Jn[r] = Jo[r] + (p.kpm1 * Jo[r] + beta * (e0 + e1));  // increment form: kp - 1 ~ -gamma dt is kept exactly
      if (ADJ) {
        const T gc = -(T(1) - p.rs) / (T(2) * (p.rs + x * (T(1) - p.rs)));
        const T gb = p.gsm * (T(1) - T(2) * x);
        gnew[r] = gacc[r] + (double)(Em[r] * (p.ga * dE + gb * (e0 + e1) + gc * (Jn[r] + Jo[r])));
      }
    } else {
      e1 = e0 + (gap ? p.ce_g : p.ce_s) * curl;
    }
    en[r] = e1;
  }

  // ---------------------------------------------------------------- stores
#pragma unroll
  for (int r = 1; r < R + 1; ++r) {
    const int j = jb - 1 + r;
    if (colx && j <= ny - 2) {
      const size_t q = (size_t)j * pitch + i;
      hxw[q] = hxn[r];
      if (pml_h(j, ny, P)) phxw[q] = phxn[r];
    }
  }
  if (ADJ) {
#pragma unroll
    for (int r = 1; r <= R; ++r) {
      const int j = jb - 1 + r;
      if (j < ny && pml_e(j, ny, P)) peyw[(size_t)j * pitch + i] = peyn[r];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = jb + r;
    if (j >= ny) continue;
    const size_t q = (size_t)j * pitch + i;
    const bool inner = j >= 1 && j <= ny - 2;
    if (ADJ && pxe) pexw[q] = pexn[r];
    if (inner && coly) {
      hyw[q] = hyn[r];
      if (pxh) phyw[q] = phyn[r];
    }
    if (!(inner && colx)) continue;
    ezw[q] = en[r];
    if (!ADJ) {
      if (pxe) pexw[q] = pexf[r];
      if (pml_e(j, ny, P)) peyw[q] = peyf[r];
    }
    const int gj = j - p.gy0, dj = j - p.dy0;
    const bool gap = gcol && gj >= 0 && gj < p.gny;
    const bool des = dcol && dj >= 0 && dj < p.dny;
    const int d = dj * p.dnx + di;
    if (des && !gap) {
      Jc[d] = Jn[r];
      if (ADJ) grad[d] = gnew[r];
    }
    if (!ADJ && des && p.hist_on) hist[(size_t)(n - p.hist_base) * nd + d] = en[r];
    if (!ADJ && gap) gp<G>(p.gapE)[(size_t)(n + 1) * p.ng + gj * p.gnx + gi] = (double)en[r];
  }
}

// One workgroup's tile: block `bid` of the grid of one instance.
template <typename T, bool ADJ, int R, bool G>
__device__ __forceinline__ void step2d_block(const Step2D<T> &p, const int n, const int par, const int bid) {
  constexpr int TYB = WAVES * R;
  const int nx = p.nx, ny = p.ny, P = p.P;
  const int nbx = (nx + TXW - 1) / TXW, nby = (ny + TYB - 1) / TYB;
  int tx, ty;
  if (p.tlist) {
    const int t = gp<G>(p.tlist)[bid];
    tx = t % nbx;
    ty = t / nbx;
  } else {
    tile_of(bid, nbx, nby, tx, ty);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = tx * TXW;
  const int i = i0 + lane;
  const int jb = ty * TYB + wave * R;
  if (jb >= ny) return;  // no barriers in these kernels
  const int ia = p.tf_on ? p.ia : -8, ib = p.tf_on ? p.ib : -8, ja = p.tf_on ? p.ja : -8, jbt = p.tf_on ? p.jb : -8;
  if constexpr (G && ADJ) {
    // The batched adjoint's edge wavefronts away from the design and gap
    // boxes skip their terms (measured on 64 uneven instances: 158 -> 146 us
    // per adjoint step; in the forward and in the single-context kernels the
    // extra body measured slower).
    const bool box = wave_touches_box<R>(i0, jb, p.dx0, p.dy0, p.dnx, p.dny) ||
                     wave_touches_box<R>(i0, jb, p.gx0, p.gy0, p.gnx, p.gny);
    if (!wave_is_edge<R>(nx, ny, P, i0, jb, ia, ib, ja, jbt)) {
      if (!box)
        step_bulk<T, R, G>(p, par, i, jb);
      else
        step_general<T, ADJ, false, R, G>(p, n, par, i, jb);
    } else if (!box) {
      step_general<T, ADJ, true, R, G, false>(p, n, par, i, jb);
    } else {
      step_general<T, ADJ, true, R, G>(p, n, par, i, jb);
    }
    return;
  }
  if (!wave_is_edge<R>(nx, ny, P, i0, jb, ia, ib, ja, jbt)) {
    if (!wave_touches_box<R>(i0, jb, p.dx0, p.dy0, p.dnx, p.dny) &&
        !wave_touches_box<R>(i0, jb, p.gx0, p.gy0, p.gnx, p.gny))
      step_bulk<T, R, G>(p, par, i, jb);
    else
      step_general<T, ADJ, false, R, G>(p, n, par, i, jb);
    return;
  }
  step_general<T, ADJ, true, R, G>(p, n, par, i, jb);
}

template <typename T, bool ADJ, int R>
__global__ void __launch_bounds__(NT, FDTD2D_MIN_WAVES) step2d_kernel(const Step2D<T> p, const int n) {
  step2d_block<T, ADJ, R, false>(p, n, 0, blockIdx.x);
}

// Several instances in one launch: instance k owns workgroups
// [first[k], first[k+1]); its parameters are read with scalar loads.  Each
// instance's block count is a multiple of 8, so its local block id keeps the
// hardware XCD in its low bits (see tile_of).
template <typename T>
using cptr2 = const __attribute__((address_space(4))) T *;

template <typename T, bool ADJ, int R>
__global__ void __launch_bounds__(NT, FDTD2D_MIN_WAVES)
    step2d_batch_kernel(const Step2D<T> *ps, const int *first, const int ninst, const int n, const int par) {
  const cptr2<int> f = (cptr2<int>)first;
  const int b = blockIdx.x;
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {  // last k with first[k] <= b
    const int mid = (lo + hi + 1) >> 1;
    if (f[mid] <= b) lo = mid; else hi = mid - 1;
  }
  Step2D<T> p;
  static_assert(sizeof(Step2D<T>) % 4 == 0, "parameter block copied as 32-bit words");
  int *dst = reinterpret_cast<int *>(&p);
  const cptr2<int> src = (cptr2<int>)(ps + lo);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Step2D<T>) / 4); ++k) dst[k] = src[k];
  // resolve the ping-pong parity here (copy 0 read, copy 1 written) so the
  // block body indexes the copies with constants and p stays in registers
  T *const *arr[7] = {p.ez, p.hx, p.hy, p.pex, p.pey, p.phx, p.phy};
  T *rd[7], *wr[7];
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    rd[a] = par ? arr[a][1] : arr[a][0];
    wr[a] = par ? arr[a][0] : arr[a][1];
  }
  p.ez[0] = rd[0]; p.ez[1] = wr[0];
  p.hx[0] = rd[1]; p.hx[1] = wr[1];
  p.hy[0] = rd[2]; p.hy[1] = wr[2];
  p.pex[0] = rd[3]; p.pex[1] = wr[3];
  p.pey[0] = rd[4]; p.pey[1] = wr[4];
  p.phx[0] = rd[5]; p.phx[1] = wr[5];
  p.phy[0] = rd[6]; p.phy[1] = wr[6];
  step2d_block<T, ADJ, R, true>(p, n, 0, b - f[lo]);
}

// ---------------------------------------------------------------- two-step
// Background update (as in step_bulk) applied twice to a TBX x TBY
// super-tile from an LDS copy of its region with a TBH = 2 node halo (LDS
// rows 0..TLY-1, columns 0..TLX-1; the super-tile is rows 2..TLY-3,
// columns 2..TLX-3).  Each phase updates in place over the nodes whose
// inputs the previous phases made valid:
//   H^{n+1/2}: H_x rows 0..TLY-2, H_y columns 0..TLX-2
//   E^{n+1}:   rows 1..TLY-2, columns 1..TLX-2
//   H^{n+3/2}: H_x rows 1..TLY-3 (columns 1..TLX-2), H_y rows 1..TLY-2 (columns 1..TLX-3)
//   E^{n+2}:   the super-tile
// The expressions are those of step_bulk, so the result is the per-step
// update's to the last bit.  64 x 16 super-tiles (17 KB of LDS in FP32)
// measured faster than 64 x 32 (more LDS per workgroup, fewer resident) and
// 64 x 8 (more halo).
constexpr int TBX = 64, TBY = 16, TBH = 2;
constexpr int TLX = TBX + 2 * TBH, TLY = TBY + 2 * TBH;  // 68 x 20
constexpr int TLS = TLX + 1;                               // LDS row stride

template <typename T, bool G>
__device__ __forceinline__ void tb_block(const Step2D<T> &p, const int code, T *ezo, T *hxo, T *hyo, T *E, T *HX,
                                         T *HY) {
  const int nbx = (p.nx + TXW - 1) / TXW;
  const bool mid = code & 1;
  const int st = code >> 1, sx = st % nbx, sy = st / nbx;
  const int x0 = sx * TBX - TBH, y0 = sy * TBY - TBH;  // global origin of LDS (0, 0)
  const int pitch = p.pitch;
  auto *__restrict__ ez = gp<G>((const T *)p.ez[0]);
  auto *__restrict__ hx = gp<G>((const T *)p.hx[0]);
  auto *__restrict__ hy = gp<G>((const T *)p.hy[0]);
  const T ch = p.chx, ce = p.ce_s;
  const int t = threadIdx.x;
  // all of a thread's loads in flight before the first LDS store
  constexpr int NL = (TLY * TLX + NT - 1) / NT;
  T ve[NL], vx[NL], vy[NL];
#pragma unroll
  for (int it = 0; it < NL; ++it) {
    const int e = t + it * NT;
    const int r = e / TLX, c = e - r * TLX;
    const bool on = e < TLY * TLX;
    const size_t q = on ? (size_t)(y0 + r) * pitch + (x0 + c) : (size_t)(y0 * pitch + x0);
    ve[it] = ez[q];
    vx[it] = hx[q];
    vy[it] = hy[q];
  }
#pragma unroll
  for (int it = 0; it < NL; ++it) {
    const int e = t + it * NT;
    if (e < TLY * TLX) {
      const int r = e / TLX, c = e - r * TLX;
      E[r * TLS + c] = ve[it];
      HX[r * TLS + c] = vx[it];
      HY[r * TLS + c] = vy[it];
    }
  }
  __syncthreads();
  // H^{n+1/2}
  for (int e = t; e < TLY * TLX; e += NT) {
    const int r = e / TLX, c = e - r * TLX, k = r * TLS + c;
    if (r < TLY - 1) HX[k] = HX[k] - ch * (E[k + TLS] - E[k]);
    if (c < TLX - 1) HY[k] = HY[k] + ch * (E[k + 1] - E[k]);
  }
  __syncthreads();
  // E^{n+1}
  for (int e = t; e < (TLY - 2) * (TLX - 2); e += NT) {
    const int r = 1 + e / (TLX - 2), c = 1 + e % (TLX - 2), k = r * TLS + c;
    E[k] = E[k] + ce * ((HY[k] - HY[k - 1]) - (HX[k] - HX[k - TLS]));
  }
  __syncthreads();
  if (mid) {  // the intermediate state of the super-tile, for the per-step neighbours
    auto *__restrict__ ezm = gp<G>(p.ez[1]);
    auto *__restrict__ hxm = gp<G>(p.hx[1]);
    auto *__restrict__ hym = gp<G>(p.hy[1]);
    for (int e = t; e < TBY * TBX; e += NT) {
      const int r = TBH + e / TBX, c = TBH + e % TBX, k = r * TLS + c;
      const size_t q = (size_t)(y0 + r) * pitch + (x0 + c);
      ezm[q] = E[k];
      hxm[q] = HX[k];
      hym[q] = HY[k];
    }
    __syncthreads();
  }
  // H^{n+3/2}
  for (int e = t; e < (TLY - 2) * (TLX - 2); e += NT) {
    const int r = 1 + e / (TLX - 2), c = 1 + e % (TLX - 2), k = r * TLS + c;
    if (r < TLY - 2) HX[k] = HX[k] - ch * (E[k + TLS] - E[k]);
    if (c < TLX - 2) HY[k] = HY[k] + ch * (E[k + 1] - E[k]);
  }
  __syncthreads();
  // E^{n+2} on the super-tile, stored with the new H
  for (int e = t; e < TBY * TBX; e += NT) {
    const int r = TBH + e / TBX, c = TBH + e % TBX, k = r * TLS + c;
    const size_t q = (size_t)(y0 + r) * pitch + (x0 + c);
    gp<G>(ezo)[q] = E[k] + ce * ((HY[k] - HY[k - 1]) - (HX[k] - HX[k - TLS]));
    gp<G>(hxo)[q] = HX[k];
    gp<G>(hyo)[q] = HY[k];
  }
}
// One launch of the blocked schedule: workgroups [0, nrest) take one
// per-step update of the tiles in ps.tlist (step n), the others two steps of
// the super-tiles tiles[0, ntb) of the pair described by pt.
template <typename T, bool ADJ>
__global__ void __launch_bounds__(NT, FDTD2D_MIN_WAVES)
    step2d_mix_kernel(const Step2D<T> ps, const int n, const int nrest, const Step2D<T> pt,
                      const int *__restrict__ tiles, T *ezo, T *hxo, T *hyo) {
  __shared__ T E[TLY * TLS], HX[TLY * TLS], HY[TLY * TLS];
  const int b = blockIdx.x;
  // per-step workgroups first: their slow design and absorber tiles start
  // early and the two-step workgroups fill the machine around them
  if (b < nrest) {
    step2d_block<T, ADJ, RDEF, false>(ps, n, 0, b);
    return;
  }
  tb_block<T, false>(pt, tiles[b - nrest], ezo, hxo, hyo, E, HX, HY);
}

// Last k with f[k] <= b.
__device__ __forceinline__ int owner(const cptr2<int> f, const int ninst, const int b) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (f[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The blocked schedule of several instances in one launch: the per-step
// workgroups of every instance, then the two-step ones.  An instance's
// descriptor part is copied into registers with scalar loads.
template <typename T, bool ADJ>
__global__ void __launch_bounds__(NT, FDTD2D_MIN_WAVES)
    step2d_batch_mix_kernel(const Mix2D<T> *ds, const int *firstR, const int *firstT, const int ninst,
                            const int nrest_total, const int n) {
  __shared__ T E[TLY * TLS], HX[TLY * TLS], HY[TLY * TLS];
  static_assert(sizeof(Step2D<T>) % 4 == 0, "parameter block copied as 32-bit words");
  const int b = blockIdx.x;
  const bool rest = b < nrest_total;
  const cptr2<int> f = (cptr2<int>)(rest ? firstR : firstT);
  const int bb = rest ? b : b - nrest_total;
  const int k = owner(f, ninst, bb);
  const int lb = bb - f[k];
  const cptr2<Mix2D<T>> d = (cptr2<Mix2D<T>>)(ds + k);
  Step2D<T> p;
  int *dst = reinterpret_cast<int *>(&p);
  if (rest) {
    if (lb >= d->nrest) return;  // padding
    const cptr2<int> src = (cptr2<int>)(&(ds + k)->ps);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(Step2D<T>) / 4); ++w) dst[w] = src[w];
      step2d_block<T, ADJ, RDEF, true>(p, n, 0, lb);
    return;
  }
  if (lb >= d->ntb) return;
  const cptr2<int> src = (cptr2<int>)(&(ds + k)->pt);
#pragma unroll
  for (int w = 0; w < (int)(sizeof(Step2D<T>) / 4); ++w) dst[w] = src[w];
  tb_block<T, true>(p, d->tiles[lb], d->ezo, d->hxo, d->hyo, E, HX, HY);
}


}  // namespace

int step2d_blocks(int nx, int ny, int rows) {
  if (rows <= 0) rows = RDEF;
  const int nbx = (nx + TXW - 1) / TXW, nby = (ny + WAVES * rows - 1) / (WAVES * rows);
  return nbx * nby;
}

// The ping-pong parity is resolved here (copy 0 read, copy 1 written), so
// the kernel indexes the copies with constants.
template <typename T, bool ADJ>
static void launch_one(const Step2D<T> &p0, int n, int par, int rows, hipStream_t s) {
  Step2D<T> p = p0;
  if (par) {
    std::swap(p.ez[0], p.ez[1]);
    std::swap(p.hx[0], p.hx[1]);
    std::swap(p.hy[0], p.hy[1]);
    std::swap(p.pex[0], p.pex[1]);
    std::swap(p.pey[0], p.pey[1]);
    std::swap(p.phx[0], p.phx[1]);
    std::swap(p.phy[0], p.phy[1]);
  }
  const dim3 grid(step2d_blocks(p.nx, p.ny, rows));
  if (rows == 1) hipLaunchKernelGGL((step2d_kernel<T, ADJ, 1>), grid, dim3(NT), 0, s, p, n);
  else if (rows == 4) hipLaunchKernelGGL((step2d_kernel<T, ADJ, 4>), grid, dim3(NT), 0, s, p, n);
  else hipLaunchKernelGGL((step2d_kernel<T, ADJ, 2>), grid, dim3(NT), 0, s, p, n);
}

Tb2dPlan tb2d_plan(int nx, int ny, int P, int ia, int ib, int ja, int jb, const int dbox[4], const int gbox[4]) {
  Tb2dPlan pl;
  const int nbx = (nx + TXW - 1) / TXW, nsy = ny / TBY;
  pl.nbx = nbx;
  const int tyb = WAVES * RDEF, nby = (ny + tyb - 1) / tyb;
  std::vector<char> ok((size_t)nbx * std::max(nsy, 1), 0);
  auto meets = [](int a0, int a1, int b0, int bn) { return bn > 0 && a1 >= b0 && a0 <= b0 + bn - 1; };
  for (int sy = 0; sy < nsy; ++sy)
    for (int tx = 0; tx < nbx; ++tx) {
      // reach: the super-tile grown by three nodes
      const int x0 = tx * TBX - 3, x1 = tx * TBX + TBX + 2, y0 = sy * TBY - 3, y1 = sy * TBY + TBY + 2;
      bool g = tx * TBX + TBX <= nx && x0 >= P + 2 && x1 <= nx - 3 - P && y0 >= P + 2 && y1 <= ny - 3 - P;
      for (int v : {ia - 1, ia, ib, ib + 1}) g = g && !(v >= x0 && v <= x1);
      for (int v : {ja - 1, ja, jb, jb + 1}) g = g && !(v >= y0 && v <= y1);
      g = g && !(meets(x0, x1, dbox[0], dbox[2]) && meets(y0, y1, dbox[1], dbox[3]));
      g = g && !(meets(x0, x1, gbox[0], gbox[2]) && meets(y0, y1, gbox[1], gbox[3]));
      ok[(size_t)sy * nbx + tx] = g;
    }
  auto at = [&](int sy, int tx) { return sy >= 0 && sy < nsy && tx >= 0 && tx < nbx && ok[(size_t)sy * nbx + tx]; };
  for (int sy = 0; sy < nsy; ++sy)
    for (int tx = 0; tx < nbx; ++tx) {
      if (!at(sy, tx)) continue;
      bool inner = true;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) inner = inner && at(sy + dy, tx + dx);
      pl.tb.push_back(((sy * nbx + tx) << 1) | (inner ? 0 : 1));
    }
  static_assert(TBY % (WAVES * RDEF) == 0, "super-tiles are whole workgroup tiles");
  for (int ty = 0; ty < nby; ++ty)
    for (int tx = 0; tx < nbx; ++tx)
      if (!at(ty * tyb / TBY, tx) || (ty + 1) * tyb > nsy * TBY) pl.rest.push_back(ty * nbx + tx);
  return pl;
}

template <typename T>
void launch_step2d_mix(const Step2D<T> &ps, int n, int nrest, const Step2D<T> &pt, const int *tiles, int ntb, T *ezo,
                       T *hxo, T *hyo, bool adjoint, hipStream_t s) {
  const int nb = nrest + ntb;
  if (nb <= 0) return;
  if (adjoint)
    hipLaunchKernelGGL((step2d_mix_kernel<T, true>), dim3(nb), dim3(NT), 0, s, ps, n, nrest, pt, tiles, ezo, hxo, hyo);
  else
    hipLaunchKernelGGL((step2d_mix_kernel<T, false>), dim3(nb), dim3(NT), 0, s, ps, n, nrest, pt, tiles, ezo, hxo, hyo);
}

template <typename T>
void launch_step2d_batch_mix(const Mix2D<T> *ds, const int *firstR, const int *firstT, int ninst, int nrest_total,
                             int nblocks, int n, bool adjoint, hipStream_t s) {
  if (nblocks <= 0) return;
  if (adjoint)
    hipLaunchKernelGGL((step2d_batch_mix_kernel<T, true>), dim3(nblocks), dim3(NT), 0, s, ds, firstR, firstT, ninst,
                       nrest_total, n);
  else
    hipLaunchKernelGGL((step2d_batch_mix_kernel<T, false>), dim3(nblocks), dim3(NT), 0, s, ds, firstR, firstT, ninst,
                       nrest_total, n);
}

template <typename T>
void launch_step2d(const Step2D<T> &p, int n, int par, bool adjoint, hipStream_t s, int rows) {
  if (rows <= 0) rows = RDEF;
  if (adjoint) launch_one<T, true>(p, n, par, rows, s);
  else launch_one<T, false>(p, n, par, rows, s);
}

template <typename T, bool ADJ>
static void launch_batch(const Step2D<T> *ps, const int *first, int ninst, int nblocks, int n, int par, int rows,
                         hipStream_t s) {
  const dim3 grid(nblocks);
  if (rows == 1) hipLaunchKernelGGL((step2d_batch_kernel<T, ADJ, 1>), grid, dim3(NT), 0, s, ps, first, ninst, n, par);
  else if (rows == 4) hipLaunchKernelGGL((step2d_batch_kernel<T, ADJ, 4>), grid, dim3(NT), 0, s, ps, first, ninst, n, par);
  else hipLaunchKernelGGL((step2d_batch_kernel<T, ADJ, 2>), grid, dim3(NT), 0, s, ps, first, ninst, n, par);
}

template <typename T>
void launch_step2d_batch(const Step2D<T> *ps, const int *first, int ninst, int nblocks, int n, int par, bool adjoint,
                         int rows, hipStream_t s) {
  if (adjoint) launch_batch<T, true>(ps, first, ninst, nblocks, n, par, rows, s);
  else launch_batch<T, false>(ps, first, ninst, nblocks, n, par, rows, s);
}

template void launch_step2d_mix<float>(const Step2D<float> &, int, int, const Step2D<float> &, const int *, int,
                                       float *, float *, float *, bool, hipStream_t);
template void launch_step2d_mix<double>(const Step2D<double> &, int, int, const Step2D<double> &, const int *, int,
                                        double *, double *, double *, bool, hipStream_t);
template void launch_step2d_batch_mix<float>(const Mix2D<float> *, const int *, const int *, int, int, int, int, bool,
                                             hipStream_t);
template void launch_step2d_batch_mix<double>(const Mix2D<double> *, const int *, const int *, int, int, int, int,
                                              bool, hipStream_t);
template void launch_step2d<float>(const Step2D<float> &, int, int, bool, hipStream_t, int);
template void launch_step2d<double>(const Step2D<double> &, int, int, bool, hipStream_t, int);
template void launch_step2d_batch<float>(const Step2D<float> *, const int *, int, int, int, int, bool, int, hipStream_t);
template void launch_step2d_batch<double>(const Step2D<double> *, const int *, int, int, int, int, bool, int, hipStream_t);

}  // namespace fdtd
