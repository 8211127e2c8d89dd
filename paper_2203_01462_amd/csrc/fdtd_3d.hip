// fdtd_3d.hip -- time step of the 3D Drude-FDTD solve and its adjoint.
//
// Per step, on the full Yee cell (Sec. 3.2; eqs. (10a-c)):
//   H^{n+1/2} = H^{n-1/2} - dt/mu0 curl E^n                (CPML, total-field faces)
//   E^{n+1} = E^n + 2/D [dt curl H^{n+1/2} - dt (1+kp)/2 J^n - (beta+sigma) dt E^n]
//   J^{n+1} = J^n + (kp - 1) J^n + beta (E^{n+1} + E^n)     (Drude edges, eqs. (4)-(5))
// The adjoint step (eq. (20)) is the same update on (E*, H*, J*) driven by
// the gap source, with each CPML term replaced by its exact transpose (the
// grading and the recursive memory act on the differenced field before the
// difference), and it accumulates the per-edge sensitivity of eq. (25) folded
// with eq. (27) into one FP64 sum per edge.
//
// Work split.  A workgroup owns a 32 x 8 column tile (one thread per (i, j))
// and marches through KC planes along z, carrying the new H_x, H_y of the
// plane below (needed by the E update) between planes.  The x/y halo (new H
// one node to the left and one row down) is recomputed from the previous
// step's values, which the ping-pong copies keep intact.  A tile-plane is
// "plain" when its whole reach is background dielectric; all others
// (absorber, walls, injection faces, Drude design edges, gap) are "general".
// One step is the general update over three host-built lists of
// tile-chunks (one absorber axis or none; several axes; design and gap) --
// one launch of step3d_general_fwd in the FP32 forward (design box clear of
// the absorber), else three launches of step3d_general, the multi-axis one
// on a second stream -- then step3d_plain, which reads back the general
// update's new H where a plain plane sits on a general one.  The general path keeps its cost down by
// loading each group of absorber memories only in tiles/planes that reach
// that absorber (uniform branches), by addressing the whole state of a copy
// through one base pointer with 32-bit offsets, and by CPML tables that are
// the identity outside the absorber, so the graded differences need no
// per-lane branches.
#include <cstdint>
#include <type_traits>

#include <algorithm>

#include "fdtd_3d.hpp"

namespace fdtd {
namespace {

constexpr int TX = 32, TY = 8, NT = TX * TY;
#ifndef FDTD3D_KC
#define FDTD3D_KC 4
#endif
constexpr int KC = FDTD3D_KC;  // planes per workgroup

// Read-only data with wave-uniform addresses goes through the constant
// address space, which lets the compiler use scalar loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

__host__ __device__ inline bool pml_e(int i, int n, int P) { return P > 0 && (i < P || i > n - 1 - P); }
__host__ __device__ inline bool pml_h(int i, int n, int P) { return P > 0 && (i < P || i >= n - 1 - P); }
__device__ __forceinline__ int slab(int i, int n, int P) { return i < P ? i : i - (n - 1 - 2 * P); }

// Element e of an arena (32-bit byte offsets).
template <typename T>
__device__ __forceinline__ T ld(const T *a, uint32_t e) {
  return *(const T *)((const char *)a + e * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st(T *a, uint32_t e, T v) {
  *(T *)((char *)a + e * (uint32_t)sizeof(T)) = v;
}

// Workgroup -> (bx, by, bz).  Dispatch slots go round-robin over the 8 XCDs
// (each with its own L2); XCD x takes z-chunks x, x+8, ..., and inside an XCD
// tiles run x fastest, then y, so in-plane neighbours share an L2.
__device__ __forceinline__ void block_of(int bid, int nbx, int nby, int nbz, int &bx, int &by, int &bz) {
  const int per = nbx * nby;
  if (nbz % 8 == 0) {
    const int k = bid >> 3;
    bx = k % nbx;
    by = (k / nbx) % nby;
    bz = (bid & 7) + 8 * (k / per);
    return;
  }
  bx = bid % nbx;
  by = (bid / nbx) % nby;
  bz = bid / per;
}

struct Tile {
  int i0, j0, kb, ke;
  bool xy_plain;     // x/y reach holds no absorber, wall or injection face
  bool tf_hit;       // x/y reach meets an injection face line
  bool tf_meet;      // x/y reach overlaps the total-field box grown by one node
  bool dxy, gxy;     // tile meets the design / gap box in x/y
};

// x/y classification of the general kernel's tile with origin (i0, j0).
template <typename T>
__host__ __device__ inline Tile tile_xy(const Step3D<T> &p, int i0, int j0) {
  const int nx = p.n[0], ny = p.n[1], P = p.P;
  Tile t;
  t.i0 = i0;
  t.j0 = j0;
  t.kb = t.ke = 0;
  const int x0 = i0 - 1, x1 = i0 + TX, y0 = j0 - 1, y1 = j0 + TY;
  auto hit = [](int lo, int hi, int v) { return v >= lo && v <= hi; };
  t.tf_hit = p.tf_on &&
             (hit(x0, x1, p.lo[0] - 1) || hit(x0, x1, p.lo[0]) || hit(x0, x1, p.hi[0]) || hit(x0, x1, p.hi[0] + 1) ||
              hit(y0, y1, p.lo[1] - 1) || hit(y0, y1, p.lo[1]) || hit(y0, y1, p.hi[1]) || hit(y0, y1, p.hi[1] + 1));
  t.tf_meet = p.tf_on && x1 >= p.lo[0] - 1 && x0 <= p.hi[0] + 1 && y1 >= p.lo[1] - 1 && y0 <= p.hi[1] + 1;
  t.xy_plain = i0 >= P + 1 && i0 + TX <= nx - 1 - P && j0 >= P + 1 && j0 + TY <= ny - 1 - P && !t.tf_hit;
  t.dxy = i0 + TX - 1 >= p.d0[0] && i0 < p.d0[0] + p.dn[0] && j0 + TY - 1 >= p.d0[1] && j0 < p.d0[1] + p.dn[1];
  t.gxy = i0 + TX - 1 >= p.g0[0] && i0 < p.g0[0] + p.gn[0] && j0 + TY - 1 >= p.g0[1] && j0 < p.g0[1] + p.gn[1];
  return t;
}

// Does the tile's z-chunk meet the design or the gap box?
template <typename T>
__host__ __device__ inline bool design_chunk(const Step3D<T> &p, const Tile &t) {
  return (t.dxy && t.ke > p.d0[2] && t.kb < p.d0[2] + p.dn[2]) || (t.gxy && t.ke > p.g0[2] && t.kb < p.g0[2] + p.gn[2]);
}

// Absorber axes whose tables and memories the general update of tile t
// needs in x and y (bit 0: x, bit 1: y), and along z at plane k (bit 2).
template <typename T>
__host__ __device__ inline int tile_axes(const Step3D<T> &p, const Tile &t) {
  const int P = p.P, nx = p.n[0], ny = p.n[1];
  const bool tx = P > 0 && (t.i0 <= P || t.i0 + TX >= nx - 1 - P);
  const bool ty = P > 0 && (t.j0 <= P || t.j0 + TY >= ny - 1 - P);
  return (tx ? 1 : 0) | (ty ? 2 : 0);
}
template <typename T>
__host__ __device__ inline int plane_axes(const Step3D<T> &p, int k) {
  const int P = p.P, nz = p.n[2];
  return pml_h(k, nz, P) || pml_e(k, nz, P) || (k + 1 < nz && pml_e(k + 1, nz, P)) ? 4 : 0;
}

// Plane k of tile t takes the plain update: x/y reach plain, k and its two z
// neighbours outside the absorber and the walls (so the new H of plane k-1 is
// ungraded in the adjoint too), k not an injection plane, and the tile-plane
// misses the design and gap boxes.  Every other tile-plane belongs to the
// general kernel.
template <typename T>
__host__ __device__ inline bool plane_plain(const Step3D<T> &p, const Tile &t, int k) {
  const int P = p.P, nz = p.n[2];
  bool pl = t.xy_plain && k >= P + 1 && k <= nz - 2 - P;
  if (p.tf_on && (k == p.lo[2] - 1 || k == p.lo[2] || k == p.hi[2])) pl = false;
  if (t.dxy && k >= p.d0[2] && k < p.d0[2] + p.dn[2]) pl = false;
  if (t.gxy && k >= p.g0[2] && k < p.g0[2] + p.gn[2]) pl = false;
  return pl;
}

// CPML grading of one axis at one position: (1/kappa, b, a).  The tables hold
// (1, 1, 0) outside the absorber, where the memories are zero, so grading is
// the identity there.
template <typename T>
struct Ax {
  T ik, b, a;
};
template <typename T>
__device__ __forceinline__ Ax<T> ax_id() {
  return {T(1), T(0), T(0)};
}
// kind 0: E (integer) positions, 1: H (half) positions
template <typename T>
__device__ __forceinline__ Ax<T> ax_ld(const Step3D<T> &p, int axis, int kind, int i) {
  const T *t = p.tab + (size_t)(axis * 6 + kind * 3) * p.tn;
  return {t[2 * p.tn + i], t[i], t[p.tn + i]};
}
template <typename T>
__device__ __forceinline__ Ax<T> ax_ld_uniform(const Step3D<T> &p, int axis, int kind, int i) {
  const cptr<T> t = (cptr<T>)(p.tab + (size_t)(axis * 6 + kind * 3) * p.tn);
  return {t[2 * p.tn + i], t[i], t[p.tn + i]};
}

// Graded value v/kappa + m_new with m_new = b m + a v: in the forward v is a
// difference and m its memory psi; in the adjoint v is the field itself and m
// its memory nu.
template <typename T>
__device__ __forceinline__ T gr(T v, T m, const Ax<T> &x, T &mn) {
  mn = x.b * m + x.a * v;
  return v * x.ik + mn;
}

// ---------------------------------------------------------------- general
// One tile-chunk of the general update.  DES compiles in the design and gap
// code; AX is the set of absorber axes compiled in (bit 0: x, 1: y, 2: z):
// a chunk whose planes reach no absorber along an axis needs no grading,
// memories or tables of that axis, and the variants without them hold fewer
// registers.  The host sorts the chunks by what they need (see
// gen3d_plan), so no variant meets a chunk it cannot update.
template <bool G, typename T>
__device__ __forceinline__ T grc(T v, T m, const Ax<T> &x, T &mn) {
  if constexpr (G) {
    return gr(v, m, x, mn);
  } else {
    mn = T(0);
    return v;
  }
}

template <typename T, bool ADJ, bool DES, int AX>
__device__ __forceinline__ void general_chunk(const Step3D<T> &p, const int n, const Tile &tl) {
  const int nx = p.n[0], ny = p.n[1], nz = p.n[2], P = p.P;
  auto gx = [](T v, T m, const Ax<T> &x, T &mn) { return grc<(AX & 1) != 0>(v, m, x, mn); };
  auto gy = [](T v, T m, const Ax<T> &x, T &mn) { return grc<(AX & 2) != 0>(v, m, x, mn); };
  auto gz = [](T v, T m, const Ax<T> &x, T &mn) { return grc<(AX & 4) != 0>(v, m, x, mn); };
  const int i = tl.i0 + (threadIdx.x % TX), j = tl.j0 + (threadIdx.x / TX);
  if (i >= nx || j >= ny) return;  // no barriers in this kernel
  const T *__restrict__ R = p.A[0];
  T *__restrict__ Wr = p.A[1];
  const uint32_t pitch = p.pitch, PL = p.PL, S = p.S, W = p.W;
  const uint32_t EX = 0, EY = S, EZ = 2 * S, HX = 3 * S, HY = 4 * S, HZ = 5 * S;
  const uint32_t qxy = p.G0 + (uint32_t)j * pitch + (uint32_t)i;

  // absorber groups reached by this tile (uniform)
  const int taxes = tile_axes(p, tl);
  const bool tx = (AX & 1) && (taxes & 1);
  const bool ty = (AX & 2) && (taxes & 2);
  // per-lane absorber flags along x and y
  const bool okL = i >= 1, okR = i + 1 < nx, okS = j >= 1, okN = j + 1 < ny;
  const bool hx_i = pml_h(i, nx, P), hx_im = okL && pml_h(i - 1, nx, P);
  const bool ex_i = pml_e(i, nx, P), ex_im = okL && pml_e(i - 1, nx, P), ex_ip = okR && pml_e(i + 1, nx, P);
  const bool hy_j = pml_h(j, ny, P), hy_jm = okS && pml_h(j - 1, ny, P);
  const bool ey_j = pml_e(j, ny, P), ey_jm = okS && pml_e(j - 1, ny, P), ey_jp = okN && pml_e(j + 1, ny, P);
  Ax<T> xh0 = ax_id<T>(), xhm = ax_id<T>(), xe0 = ax_id<T>(), xem = ax_id<T>(), xep = ax_id<T>();
  Ax<T> yh0 = ax_id<T>(), yhm = ax_id<T>(), ye0 = ax_id<T>(), yem = ax_id<T>(), yep = ax_id<T>();
  if (tx) {
    const int im = max(i - 1, 0), ip = min(i + 1, nx - 1);
    xh0 = ax_ld(p, 0, 1, i);
    xhm = ax_ld(p, 0, 1, im);
    xe0 = ax_ld(p, 0, 0, i);
    if (ADJ) {
      xem = ax_ld(p, 0, 0, im);
      xep = ax_ld(p, 0, 0, ip);
    }
  }
  if (ty) {
    const int jm = max(j - 1, 0), jp = min(j + 1, ny - 1);
    yh0 = ax_ld(p, 1, 1, j);
    yhm = ax_ld(p, 1, 1, jm);
    ye0 = ax_ld(p, 1, 0, j);
    if (ADJ) {
      yem = ax_ld(p, 1, 0, jm);
      yep = ax_ld(p, 1, 0, jp);
    }
  }
  // slab offsets of this column (meaningful only where the matching flag is set)
  const uint32_t oX0 = (uint32_t)j * W + (uint32_t)slab(i, nx, P);
  const uint32_t oXm = (uint32_t)j * W + (uint32_t)slab(i - 1, nx, P);
  const uint32_t oXp = (uint32_t)j * W + (uint32_t)slab(i + 1, nx, P);
  const uint32_t oY0 = (uint32_t)slab(j, ny, P) * pitch + (uint32_t)i;
  const uint32_t oYm = (uint32_t)slab(j - 1, ny, P) * pitch + (uint32_t)i;
  const uint32_t oYp = (uint32_t)slab(j + 1, ny, P) * pitch + (uint32_t)i;
  const uint32_t oZ = (uint32_t)j * pitch + (uint32_t)i;
  // wall validity along x and y of the owned and neighbour positions
  auto rng = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
  const bool xa1 = rng(i, 1, nx - 2), xa0 = rng(i, 0, nx - 2), xm0 = rng(i - 1, 0, nx - 2);
  const bool ya1 = rng(j, 1, ny - 2), ya0 = rng(j, 0, ny - 2), ym0 = rng(j - 1, 0, ny - 2);
  // design and gap columns
  const int nd = p.dn[0] * p.dn[1] * p.dn[2];
  const int di = i - p.d0[0], dj = j - p.d0[1], gi = i - p.g0[0], gj = j - p.g0[1];
  const bool dcol = di >= 0 && di < p.dn[0] && dj >= 0 && dj < p.dn[1];
  const bool gcol = gi >= 0 && gi < p.gn[0] && gj >= 0 && gj < p.gn[1];

  // new H_x, H_y of the plane below (adjoint: graded along z), carried
  T hxp = T(0), hyp = T(0);

  auto plane = [&](auto store_tag, const int k) {
    constexpr bool STORE = decltype(store_tag)::value;
    if (k < 0) {  // below the grid: no H
      hxp = hyp = T(0);
      return;
    }
    const bool kh = k <= nz - 2, kz = k >= 1 && k <= nz - 2, okU = k + 1 < nz;
    const bool vx00 = xa1 && ya0 && kh, vx0m = xa1 && ym0 && kh;
    const bool vy00 = xa0 && ya1 && kh, vym0 = xm0 && ya1 && kh;
    const bool vz00 = xa0 && ya0 && kz, vz0m = xa0 && ym0 && kz, vzm0 = xm0 && ya0 && kz;
    const bool vex = xa0 && ya1 && kz, vey = xa1 && ya0 && kz, vez = xa1 && ya1 && kh;
    // absorber along z at this plane (uniform)
    const bool hz_k = pml_h(k, nz, P), ez_k = pml_e(k, nz, P), ez_k1 = okU && pml_e(k + 1, nz, P);
    const bool tz = (AX & 4) && plane_axes(p, k);
    Ax<T> zh = ax_id<T>(), ze = ax_id<T>(), ze1 = ax_id<T>();
    uint32_t zb = 0, zb1 = 0;
    if (tz) {
      zh = ax_ld_uniform(p, 2, 1, k);
      ze = ax_ld_uniform(p, 2, 0, k);
      if (ADJ) ze1 = ax_ld_uniform(p, 2, 0, min(k + 1, nz - 1));
      zb = p.zs + (uint32_t)slab(k, nz, P) * PL + oZ;
      zb1 = p.zs + (uint32_t)slab(k + 1, nz, P) * PL + oZ;
    }
    const uint32_t xb = p.xs + (uint32_t)k * ny * W, yb = p.ys + (uint32_t)k * W * pitch;
    // injection, design and gap at this tile-plane (uniform)
    const bool tfp = tl.tf_meet && k >= p.lo[2] - 1 && k <= p.hi[2] &&
                     (tl.tf_hit || k == p.lo[2] - 1 || k == p.lo[2] || k == p.hi[2]);
    const bool dp = DES && tl.dxy && k >= p.d0[2] && k < p.d0[2] + p.dn[2];
    const bool gp = DES && tl.gxy && k >= p.g0[2] && k < p.g0[2] + p.gn[2];
    const bool des = dp && dcol, gap = gp && gcol, drude = des && !gap;
    const uint32_t d = des ? (uint32_t)(((k - p.d0[2]) * p.dn[1] + dj) * p.dn[0] + di) : 0u;
    const uint32_t g = gap ? (uint32_t)(((k - p.g0[2]) * p.gn[1] + gj) * p.gn[0] + gi) : 0u;

    const uint32_t q = qxy + (uint32_t)k * PL;
    // fields (the guard keeps every neighbour offset inside the arena; values
    // read across an edge only feed nodes that the wall masks discard)
    const T exC = ld(R, EX + q), exLl = ld(R, EX + q - 1), exN = ld(R, EX + q + pitch), exS = ld(R, EX + q - pitch);
    const T exLN = ld(R, EX + q + pitch - 1), exc1 = ld(R, EX + q + PL), exl1 = ld(R, EX + q + PL - 1);
    const T eyC = ld(R, EY + q), eySl = ld(R, EY + q - pitch), eyR = ld(R, EY + q + 1), eyRS = ld(R, EY + q + 1 - pitch);
    const T eyL = ld(R, EY + q - 1), eyc1 = ld(R, EY + q + PL), eys1 = ld(R, EY + q + PL - pitch);
    const T ezC = ld(R, EZ + q), ezN = ld(R, EZ + q + pitch), ezR = ld(R, EZ + q + 1), ezS = ld(R, EZ + q - pitch);
    const T ezL = ld(R, EZ + q - 1);
    const T hxC = ld(R, HX + q), hxS = ld(R, HX + q - pitch), hyC = ld(R, HY + q), hyL = ld(R, HY + q - 1);
    const T hzC = ld(R, HZ + q), hzS = ld(R, HZ + q - pitch), hzL = ld(R, HZ + q - 1);
    // design edges and gap
    const T rr = dp ? ld(p.rho, d) : T(0);
    T Jo[3] = {T(0), T(0), T(0)}, Em[3] = {T(0), T(0), T(0)}, src[3] = {T(0), T(0), T(0)};
    double gacc[3] = {0.0, 0.0, 0.0};
    if (dp) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Jo[c] = ld(p.J, drude ? (uint32_t)c * nd + d : 0u);
        if (ADJ) {
          Em[c] = p.hist[drude ? ((size_t)(n - 1 - p.hist_base) * 3 + c) * nd + d : 0];
          gacc[c] = p.grad[drude ? (size_t)c * nd + d : 0];
        }
      }
    }
    if (ADJ && gp) {
#pragma unroll
      for (int c = 0; c < 3; ++c) src[c] = gap ? p.asrc[((size_t)n * p.ng + g) * 3 + c] : T(0);
    }

    T hx00, hx0m, hy00, hym0, hz00, hz0m, hzm0;  // forward: new H; adjoint: new H*
    T cx, cy, cz;                                  // curl brackets of the three E updates
    T sn[12];                                      // new memories of the owned nodes
    T t;
    if constexpr (!ADJ) {
      // old memories of the differences below
      T s_hx00y = 0, s_hx0my = 0, s_hz00y = 0, s_hz0my = 0, s_hzm0y = 0, s_exy = 0, s_ezy = 0;
      T s_hy00x = 0, s_hym0x = 0, s_hz00x = 0, s_hz0mx = 0, s_hzm0x = 0, s_eyx = 0, s_ezx = 0;
      T s_hx00z = 0, s_hx0mz = 0, s_hy00z = 0, s_hym0z = 0, s_exz = 0, s_eyz = 0;
      if (ty) {
        s_hx00y = ld(R, vx00 && hy_j ? yb + oY0 : 0u);
        s_hx0my = ld(R, vx0m && hy_jm ? yb + oYm : 0u);
        s_hz00y = ld(R, vz00 && hy_j ? yb + p.YS + oY0 : 0u);
        s_hz0my = ld(R, vz0m && hy_jm ? yb + p.YS + oYm : 0u);
        s_hzm0y = ld(R, vzm0 && hy_j ? yb + p.YS + oY0 - 1 : 0u);
        s_exy = ld(R, vex && ey_j ? yb + 2 * p.YS + oY0 : 0u);
        s_ezy = ld(R, vez && ey_j ? yb + 3 * p.YS + oY0 : 0u);
      }
      if (tx) {
        s_hy00x = ld(R, vy00 && hx_i ? xb + oX0 : 0u);
        s_hym0x = ld(R, vym0 && hx_im ? xb + oXm : 0u);
        s_hz00x = ld(R, vz00 && hx_i ? xb + p.XS + oX0 : 0u);
        s_hz0mx = ld(R, vz0m && hx_i ? xb + p.XS + oX0 - W : 0u);
        s_hzm0x = ld(R, vzm0 && hx_im ? xb + p.XS + oXm : 0u);
        s_eyx = ld(R, vey && ex_i ? xb + 2 * p.XS + oX0 : 0u);
        s_ezx = ld(R, vez && ex_i ? xb + 3 * p.XS + oX0 : 0u);
      }
      if (tz) {
        s_hx00z = ld(R, vx00 && hz_k ? zb : 0u);
        s_hx0mz = ld(R, vx0m && hz_k ? zb - pitch : 0u);
        s_hy00z = ld(R, vy00 && hz_k ? zb + p.ZS : 0u);
        s_hym0z = ld(R, vym0 && hz_k ? zb + p.ZS - 1 : 0u);
        s_exz = ld(R, vex && ez_k ? zb + 2 * p.ZS : 0u);
        s_eyz = ld(R, vey && ez_k ? zb + 3 * p.ZS : 0u);
      }
      const T ch = p.ch;
      // H_x: d_y E_z - d_z E_y;  H_y: d_z E_x - d_x E_z;  H_z: d_x E_y - d_y E_x
      hx00 = hxC - ch * (gy(ezN - ezC, s_hx00y, yh0, sn[0]) - gz(eyc1 - eyC, s_hx00z, zh, sn[1]));
      hx0m = hxS - ch * (gy(ezC - ezS, s_hx0my, yhm, t) - gz(eys1 - eySl, s_hx0mz, zh, t));
      hy00 = hyC - ch * (gz(exc1 - exC, s_hy00z, zh, sn[2]) - gx(ezR - ezC, s_hy00x, xh0, sn[3]));
      hym0 = hyL - ch * (gz(exl1 - exLl, s_hym0z, zh, t) - gx(ezC - ezL, s_hym0x, xhm, t));
      hz00 = hzC - ch * (gx(eyR - eyC, s_hz00x, xh0, sn[4]) - gy(exN - exC, s_hz00y, yh0, sn[5]));
      hz0m = hzS - ch * (gx(eyRS - eySl, s_hz0mx, xh0, t) - gy(exC - exS, s_hz0my, yhm, t));
      hzm0 = hzL - ch * (gx(eyC - eyL, s_hzm0x, xhm, t) - gy(exLN - exLl, s_hzm0y, yh0, t));
      T hA = T(0), hB = T(0), hK = T(0);
      if (tfp) {
        // total-field / scattered-field corrections from the incident line
        const cptr<T> ei = (cptr<T>)(p.einc + (size_t)n * p.L);
        const cptr<T> hi = (cptr<T>)(p.hinc + (size_t)n * p.L);
        const bool kin = k >= p.lo[2] && k <= p.hi[2];
        const T eA = ei[p.lo[2] - p.kref], eB = ei[p.hi[2] - p.kref], eK = kin ? ei[k - p.kref] : T(0);
        hA = hi[p.lo[2] - 1 - p.kref];
        hB = hi[p.hi[2] - p.kref];
        hK = kin ? hi[k - p.kref] : T(0);
        const bool xin0 = i >= p.lo[0] && i <= p.hi[0] - 1, xinm = i - 1 >= p.lo[0] && i - 1 <= p.hi[0] - 1;
        const bool yin = j >= p.lo[1] && j <= p.hi[1];
        if (yin && k == p.lo[2] - 1) {
          if (xin0) hy00 += ch * eA;
          if (xinm) hym0 += ch * eA;
        }
        if (yin && k == p.hi[2]) {
          if (xin0) hy00 -= ch * eB;
          if (xinm) hym0 -= ch * eB;
        }
        if (kin) {
          if (xin0 && j == p.lo[1] - 1) hz00 -= ch * eK;
          if (xin0 && j == p.hi[1]) hz00 += ch * eK;
          if (xin0 && j - 1 == p.lo[1] - 1) hz0m -= ch * eK;
          if (xin0 && j - 1 == p.hi[1]) hz0m += ch * eK;
          if (xinm && j == p.lo[1] - 1) hzm0 -= ch * eK;
          if (xinm && j == p.hi[1]) hzm0 += ch * eK;
        }
      }
      // walls hold no H
      hx00 = vx00 ? hx00 : T(0);
      hx0m = vx0m ? hx0m : T(0);
      hy00 = vy00 ? hy00 : T(0);
      hym0 = vym0 ? hym0 : T(0);
      hz00 = vz00 ? hz00 : T(0);
      hz0m = vz0m ? hz0m : T(0);
      hzm0 = vzm0 ? hzm0 : T(0);
      // E_x: d_y H_z - d_z H_y;  E_y: d_z H_x - d_x H_z;  E_z: d_x H_y - d_y H_x
      cx = gy(hz00 - hz0m, s_exy, ye0, sn[6]) - gz(hy00 - hyp, s_exz, ze, sn[7]);
      cy = gz(hx00 - hxp, s_eyz, ze, sn[8]) - gx(hz00 - hzm0, s_eyx, xe0, sn[9]);
      cz = gx(hy00 - hym0, s_ezx, xe0, sn[10]) - gy(hx00 - hx0m, s_ezy, ye0, sn[11]);
      if (tfp) {
        if (i >= p.lo[0] && i <= p.hi[0] - 1 && j >= p.lo[1] && j <= p.hi[1]) {
          if (k == p.lo[2]) cx += hA;
          if (k == p.hi[2]) cx -= hB;
        }
        if (j >= p.lo[1] && j <= p.hi[1] && k >= p.lo[2] && k <= p.hi[2] - 1) {
          if (i == p.lo[0]) cz -= hK;
          if (i == p.hi[0]) cz += hK;
        }
      }
      hxp = hx00;
      hyp = hy00;
    } else {
      // old memories of the E* values graded below (transposed CPML) and of the new H*
      T n_ezyN = 0, n_ezyC = 0, n_ezyS = 0, n_exyN = 0, n_exyC = 0, n_exyS = 0, n_exyLN = 0, n_exyL = 0;
      T n_hx00y = 0, n_hx0my = 0, n_hz00y = 0, n_hz0my = 0;
      T n_ezxR = 0, n_ezxC = 0, n_ezxL = 0, n_eyxR = 0, n_eyxC = 0, n_eyxRS = 0, n_eyxS = 0, n_eyxL = 0;
      T n_hy00x = 0, n_hym0x = 0, n_hz00x = 0, n_hzm0x = 0;
      T n_eyzU = 0, n_eyzC = 0, n_eyzSU = 0, n_eyzS = 0, n_exzU = 0, n_exzC = 0, n_exzLU = 0, n_exzL = 0;
      T n_hx00z = 0, n_hy00z = 0;
      if (ty) {
        const uint32_t yEx = yb + 2 * p.YS, yEz = yb + 3 * p.YS;
        n_ezyN = ld(R, ey_jp ? yEz + oYp : 0u);
        n_ezyC = ld(R, ey_j ? yEz + oY0 : 0u);
        n_ezyS = ld(R, ey_jm ? yEz + oYm : 0u);
        n_exyN = ld(R, ey_jp ? yEx + oYp : 0u);
        n_exyC = ld(R, ey_j ? yEx + oY0 : 0u);
        n_exyS = ld(R, ey_jm ? yEx + oYm : 0u);
        n_exyLN = ld(R, okL && ey_jp ? yEx + oYp - 1 : 0u);
        n_exyL = ld(R, okL && ey_j ? yEx + oY0 - 1 : 0u);
        n_hx00y = ld(R, vx00 && hy_j ? yb + oY0 : 0u);
        n_hx0my = ld(R, vx0m && hy_jm ? yb + oYm : 0u);
        n_hz00y = ld(R, vz00 && hy_j ? yb + p.YS + oY0 : 0u);
        n_hz0my = ld(R, vz0m && hy_jm ? yb + p.YS + oYm : 0u);
      }
      if (tx) {
        const uint32_t xEy = xb + 2 * p.XS, xEz = xb + 3 * p.XS;
        n_ezxR = ld(R, ex_ip ? xEz + oXp : 0u);
        n_ezxC = ld(R, ex_i ? xEz + oX0 : 0u);
        n_ezxL = ld(R, ex_im ? xEz + oXm : 0u);
        n_eyxR = ld(R, ex_ip ? xEy + oXp : 0u);
        n_eyxC = ld(R, ex_i ? xEy + oX0 : 0u);
        n_eyxRS = ld(R, okS && ex_ip ? xEy + oXp - W : 0u);
        n_eyxS = ld(R, okS && ex_i ? xEy + oX0 - W : 0u);
        n_eyxL = ld(R, ex_im ? xEy + oXm : 0u);
        n_hy00x = ld(R, vy00 && hx_i ? xb + oX0 : 0u);
        n_hym0x = ld(R, vym0 && hx_im ? xb + oXm : 0u);
        n_hz00x = ld(R, vz00 && hx_i ? xb + p.XS + oX0 : 0u);
        n_hzm0x = ld(R, vzm0 && hx_im ? xb + p.XS + oXm : 0u);
      }
      if (tz) {
        n_eyzU = ld(R, ez_k1 ? zb1 + 3 * p.ZS : 0u);
        n_eyzC = ld(R, ez_k ? zb + 3 * p.ZS : 0u);
        n_eyzSU = ld(R, okS && ez_k1 ? zb1 + 3 * p.ZS - pitch : 0u);
        n_eyzS = ld(R, okS && ez_k ? zb + 3 * p.ZS - pitch : 0u);
        n_exzU = ld(R, ez_k1 ? zb1 + 2 * p.ZS : 0u);
        n_exzC = ld(R, ez_k ? zb + 2 * p.ZS : 0u);
        n_exzLU = ld(R, okL && ez_k1 ? zb1 + 2 * p.ZS - 1 : 0u);
        n_exzL = ld(R, okL && ez_k ? zb + 2 * p.ZS - 1 : 0u);
        n_hx00z = ld(R, vx00 && hz_k ? zb : 0u);
        n_hy00z = ld(R, vy00 && hz_k ? zb + p.ZS : 0u);
      }
      // graded E*
      const T gyEzN = gy(ezN, n_ezyN, yep, t), gyEzC = gy(ezC, n_ezyC, ye0, sn[11]), gyEzS = gy(ezS, n_ezyS, yem, t);
      const T gzEyU = gz(eyc1, n_eyzU, ze1, t), gzEyC = gz(eyC, n_eyzC, ze, sn[8]);
      const T gzEySU = gz(eys1, n_eyzSU, ze1, t), gzEyS = gz(eySl, n_eyzS, ze, t);
      const T gzExU = gz(exc1, n_exzU, ze1, t), gzExC = gz(exC, n_exzC, ze, sn[7]);
      const T gzExLU = gz(exl1, n_exzLU, ze1, t), gzExL = gz(exLl, n_exzL, ze, t);
      const T gxEzR = gx(ezR, n_ezxR, xep, t), gxEzC = gx(ezC, n_ezxC, xe0, sn[10]), gxEzL = gx(ezL, n_ezxL, xem, t);
      const T gxEyR = gx(eyR, n_eyxR, xep, t), gxEyC = gx(eyC, n_eyxC, xe0, sn[9]);
      const T gxEyRS = gx(eyRS, n_eyxRS, xep, t), gxEyS = gx(eySl, n_eyxS, xe0, t), gxEyL = gx(eyL, n_eyxL, xem, t);
      const T gyExN = gy(exN, n_exyN, yep, t), gyExC = gy(exC, n_exyC, ye0, sn[6]), gyExS = gy(exS, n_exyS, yem, t);
      const T gyExLN = gy(exLN, n_exyLN, yep, t), gyExL = gy(exLl, n_exyL, ye0, t);
      const T ch = p.ch;
      hx00 = vx00 ? hxC - ch * ((gyEzN - gyEzC) - (gzEyU - gzEyC)) : T(0);
      hx0m = vx0m ? hxS - ch * ((gyEzC - gyEzS) - (gzEySU - gzEyS)) : T(0);
      hy00 = vy00 ? hyC - ch * ((gzExU - gzExC) - (gxEzR - gxEzC)) : T(0);
      hym0 = vym0 ? hyL - ch * ((gzExLU - gzExL) - (gxEzC - gxEzL)) : T(0);
      hz00 = vz00 ? hzC - ch * ((gxEyR - gxEyC) - (gyExN - gyExC)) : T(0);
      hz0m = vz0m ? hzS - ch * ((gxEyRS - gxEyS) - (gyExC - gyExS)) : T(0);
      hzm0 = vzm0 ? hzL - ch * ((gxEyC - gxEyL) - (gyExLN - gyExL)) : T(0);
      // graded H* for the E* brackets
      const T gyHx00 = gy(hx00, n_hx00y, yh0, sn[0]), gzHx00 = gz(hx00, n_hx00z, zh, sn[1]);
      const T gyHx0m = gy(hx0m, n_hx0my, yhm, t);
      const T gzHy00 = gz(hy00, n_hy00z, zh, sn[2]), gxHy00 = gx(hy00, n_hy00x, xh0, sn[3]);
      const T gxHym0 = gx(hym0, n_hym0x, xhm, t);
      const T gxHz00 = gx(hz00, n_hz00x, xh0, sn[4]), gyHz00 = gy(hz00, n_hz00y, yh0, sn[5]);
      const T gyHz0m = gy(hz0m, n_hz0my, yhm, t), gxHzm0 = gx(hzm0, n_hzm0x, xhm, t);
      cx = (gyHz00 - gyHz0m) - (gzHy00 - hyp) + src[0];
      cy = (gzHx00 - hxp) - (gxHz00 - gxHzm0) + src[1];
      cz = (gxHy00 - gxHym0) - (gyHx00 - gyHx0m) + src[2];
      hxp = gzHx00;
      hyp = gzHy00;
    }
    if constexpr (!STORE) return;

    // E (or E*) and J on the owned edges
    const T e0[3] = {exC, eyC, ezC};
    const T curl[3] = {cx, cy, cz};
    const bool ev[3] = {vex, vey, vez};
    const T ce = gap ? p.ce_g : p.ce_s;
    T e1[3], Jn[3];
    double gn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Jn[c] = T(0);
      gn[c] = gacc[c];
      e1[c] = e0[c] + ce * curl[c];
      if (dp && drude) {
        const T eps2 = p.A0 + rr * p.A1;
        const T beta = p.B0 + rr * p.B1;
        const T bs = beta * p.dt_ + p.Sg * rr * (T(1) - rr);
        const T inv = T(2) / (eps2 + bs);
        const T dE = inv * (p.dtdx * curl[c] - p.dthJ * Jo[c] - bs * e0[c]);
        e1[c] = e0[c] + dE;
        Jn[c] = Jo[c] + (p.kpm1 * Jo[c] + beta * (e0[c] + e1[c]));  // increment form
        if (ADJ) {
          const T gc = -(T(1) - p.rs) / (T(2) * (p.rs + rr * (T(1) - p.rs)));
          const T gb = p.gsm * (T(1) - T(2) * rr);
          gn[c] = gacc[c] + (double)(Em[c] * (p.ga * dE + gb * (e0[c] + e1[c]) + gc * (Jn[c] + Jo[c])));
        }
      }
    }

    // ---- stores
    if (vx00) st(Wr, HX + q, hx00);
    if (vy00) st(Wr, HY + q, hy00);
    if (vz00) st(Wr, HZ + q, hz00);
    if (vex) st(Wr, EX + q, e1[0]);
    if (vey) st(Wr, EY + q, e1[1]);
    if (vez) st(Wr, EZ + q, e1[2]);
    // memories: the H ones on valid nodes; the forward E ones on valid
    // nodes, the adjoint E ones on every in-grid node (zero on the walls)
    const bool wex = ADJ || vex, wey = ADJ || vey, wez = ADJ || vez;
    if (ty) {
      if (vx00 && hy_j) st(Wr, yb + oY0, sn[0]);
      if (vz00 && hy_j) st(Wr, yb + p.YS + oY0, sn[5]);
      if (wex && ey_j) st(Wr, yb + 2 * p.YS + oY0, sn[6]);
      if (wez && ey_j) st(Wr, yb + 3 * p.YS + oY0, sn[11]);
    }
    if (tx) {
      if (vy00 && hx_i) st(Wr, xb + oX0, sn[3]);
      if (vz00 && hx_i) st(Wr, xb + p.XS + oX0, sn[4]);
      if (wey && ex_i) st(Wr, xb + 2 * p.XS + oX0, sn[9]);
      if (wez && ex_i) st(Wr, xb + 3 * p.XS + oX0, sn[10]);
    }
    if (tz) {
      if (vx00 && hz_k) st(Wr, zb, sn[1]);
      if (vy00 && hz_k) st(Wr, zb + p.ZS, sn[2]);
      if (wex && ez_k) st(Wr, zb + 2 * p.ZS, sn[7]);
      if (wey && ez_k) st(Wr, zb + 3 * p.ZS, sn[8]);
    }
    if (dp) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (!ev[c] || !des) continue;
        if (drude) {
          p.J[(size_t)c * nd + d] = Jn[c];
          if (ADJ) p.grad[(size_t)c * nd + d] = gn[c];
        }
        if (!ADJ && p.hist_on) p.hist[((size_t)(n - p.hist_base) * 3 + c) * nd + d] = e1[c];
      }
    }
    if (!ADJ && gp && gap) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (ev[c]) p.gapE[((size_t)(n + 1) * p.ng + g) * 3 + c] = (double)e1[c];
    }
  };

  bool have = false;  // carried values hold plane k-1
  for (int k = tl.kb; k < tl.ke; ++k) {
    if (plane_plain(p, tl, k)) {
      have = false;
      continue;
    }
    if (!have) plane(std::integral_constant<bool, false>(), k - 1);  // new H of plane k-1, not stored
    plane(std::integral_constant<bool, true>(), k);
    have = true;
  }
}

// Workgroup b updates tile-chunk list[b] (-1: none).  Chunk code c = (bz *
// nby + by) * nbx + bx; with AX = 8 the code is 4c + a, a = the one absorber
// axis the chunk needs (0 x, 1 y, 2 z) or 3 for none.
#ifndef FDTD3D_WPE_F8
#define FDTD3D_WPE_F8 4
#endif
#ifndef FDTD3D_WPE_A8
#define FDTD3D_WPE_A8 4
#endif
template <typename T, bool ADJ, bool DES, int AX>
constexpr int gen_waves() {
  if (sizeof(T) != 4) return 1;
  if (AX == 8) return ADJ ? FDTD3D_WPE_A8 : FDTD3D_WPE_F8;
  return 1;
}

template <typename T, bool ADJ, bool DES, int AX>
__device__ __forceinline__ void general_body(const Step3D<T> &p, const int n, const int code) {
  const int c = AX == 8 ? code >> 2 : code;
  const int nbx = (p.n[0] + TX - 1) / TX, nby = (p.n[1] + TY - 1) / TY;
  const int bx = c % nbx, by = (c / nbx) % nby, bz = c / (nbx * nby);
  Tile tl = tile_xy(p, bx * TX, by * TY);
  tl.kb = bz * KC;
  tl.ke = min(tl.kb + KC, p.n[2]);
  if constexpr (AX == 8) {
    switch (code & 3) {
      case 0: general_chunk<T, ADJ, DES, 1>(p, n, tl); break;
      case 1: general_chunk<T, ADJ, DES, 2>(p, n, tl); break;
      case 2: general_chunk<T, ADJ, DES, 4>(p, n, tl); break;
      default: general_chunk<T, ADJ, DES, 0>(p, n, tl); break;
    }
  } else {
    general_chunk<T, ADJ, DES, AX>(p, n, tl);
  }
}

template <typename T, bool ADJ, bool DES, int AX>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(gen_waves<T, ADJ, DES, AX>())))
step3d_general(const Step3D<T> p, const int n, const int *__restrict__ list) {
  const int code = ((cptr<int>)list)[blockIdx.x];
  if (code < 0) return;
  general_body<T, ADJ, DES, AX>(p, n, code);
}

// The FP32 forward's three lists in one launch, in list order (single-axis,
// multi-axis, design), when no design chunk reaches the absorber (gAxD = 0):
// workgroup b takes entry b, and the body follows the list the entry sits in
// (a uniform branch).  Each list's length is a multiple of 8, so every entry
// keeps the XCD slot its list gave it.  The union of the bodies fits 4 waves
// per SIMD (119 VGPRs; with the design-with-absorber body as well it needed
// 137 and spilled at 128).  Measured on the 256^3 workload it beats the
// three launches on two streams, whose fork and join each left the machine
// idle for ~6 us.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
step3d_general_fwd(const Step3D<float> p, const int n, const int *__restrict__ list) {
  const int b = blockIdx.x;
  const int code = ((cptr<int>)list)[b];
  if (code < 0) return;
  if (b < p.gS) general_body<float, false, false, 8>(p, n, code);
  else if (b < p.gS + p.gM) general_body<float, false, false, 7>(p, n, code);
  else general_body<float, false, true, 0>(p, n, code);
}

// ---------------------------------------------------------------- plain
// Background dielectric only, identical for the forward and the adjoint.
// Launched after the general update of the same step, so where plane k-1 was
// general its new H is read back from the write copy.  Its own tiling
// (64 x 8 columns, 4-plane chunks) covers the bounding box of the plain
// tile-planes only; each lane takes the nodes whose general-kernel
// tile-plane is plain.
#ifndef FDTD3D_PTX
#define FDTD3D_PTX 64
#endif
#ifndef FDTD3D_PTY
#define FDTD3D_PTY 8
#endif
#ifndef FDTD3D_PKC
#define FDTD3D_PKC 4
#endif
constexpr int PTX = FDTD3D_PTX, PTY = FDTD3D_PTY, PNT = PTX * PTY, PKC = FDTD3D_PKC;

// Workgroups of the plain launch over the box pb (z-chunks rounded up to a
// multiple of 8 for the XCD-aware order of block_of).
__host__ __device__ inline void plain_grid(const int pb[6], int &nbx, int &nby, int &nbz) {
  nbx = (pb[3] + PTX - 1) / PTX;
  nby = (pb[4] + PTY - 1) / PTY;
  nbz = (pb[5] + PKC - 1) / PKC;
  nbz = (nbz + 7) / 8 * 8;
}

// Does node (i, j, k) belong to a two-step super-chunk?
template <typename T>
__device__ __forceinline__ bool in_super(const Step3D<T> &p, int i, int j, int k) {
  const int u = i - p.so[0], v = j - p.so[1], w = k - p.so[2];
  if (u < 0 || v < 0 || w < 0) return false;
  const int cx = u / SCX, cy = v / SCY, cz = w / SCZ;
  if (cx >= p.sn[0] || cy >= p.sn[1] || cz >= p.sn[2]) return false;
  return p.sflag[(cz * p.sn[1] + cy) * p.sn[0] + cx] != 0;
}

// Does the box [x0, x1) x [y0, y1) x [z0, z1) lie inside two-step
// super-chunks only?  (At most two chunks per axis for boxes no larger
// than a chunk.)
template <typename T>
__device__ __forceinline__ bool all_super(const Step3D<T> &p, int x0, int x1, int y0, int y1, int z0, int z1) {
  const int lo[3] = {x0, y0, z0}, hi[3] = {x1, y1, z1}, sc[3] = {SCX, SCY, SCZ};
  int c0[3], c1[3];
  for (int a = 0; a < 3; ++a) {
    if (lo[a] < p.so[a] || hi[a] > p.so[a] + p.sn[a] * sc[a]) return false;
    c0[a] = (lo[a] - p.so[a]) / sc[a];
    c1[a] = (hi[a] - 1 - p.so[a]) / sc[a];
  }
  for (int cz = c0[2]; cz <= c1[2]; ++cz)
    for (int cy = c0[1]; cy <= c1[1]; ++cy)
      for (int cx = c0[0]; cx <= c1[0]; ++cx)
        if (!p.sflag[(cz * p.sn[1] + cy) * p.sn[0] + cx]) return false;
  return true;
}

template <typename T>
__global__ void __launch_bounds__(PNT) step3d_plain(const Step3D<T> p) {
  const int nx = p.n[0], ny = p.n[1];
  int nbx, nby, nbz, bx, by, bz;
  plain_grid(p.pb, nbx, nby, nbz);
  block_of(blockIdx.x, nbx, nby, nbz, bx, by, bz);
  if (p.skip_super) {
    // a tile held wholly by super-chunks has nothing to do (uniform exit)
    const int x0 = p.pb[0] + bx * PTX, y0 = p.pb[1] + by * PTY, z0 = p.pb[2] + bz * PKC;
    if (all_super(p, x0, min(x0 + PTX, nx), y0, min(y0 + PTY, ny), z0, min(z0 + PKC, p.pb[2] + p.pb[5]))) return;
  }
  const int i = p.pb[0] + bx * PTX + (threadIdx.x % PTX), j = p.pb[1] + by * PTY + (threadIdx.x / PTX);
  if (i >= nx || j >= ny) return;  // no barriers in this kernel
  const Tile tl = tile_xy(p, i - i % TX, j - j % TY);
  if (!tl.xy_plain) return;
  const int kb = p.pb[2] + bz * PKC, ke = min(kb + PKC, p.pb[2] + p.pb[5]);
  const uint32_t pitch = p.pitch, PL = p.PL, S = p.S;
  const T *__restrict__ Ex = p.A[0] + p.G0;
  const T *__restrict__ Ey = Ex + S;
  const T *__restrict__ Ez = Ex + 2 * (size_t)S;
  const T *__restrict__ Hx = Ex + 3 * (size_t)S;
  const T *__restrict__ Hy = Ex + 4 * (size_t)S;
  const T *__restrict__ Hz = Ex + 5 * (size_t)S;
  T *__restrict__ Exw = p.A[1] + p.G0;
  T *__restrict__ Eyw = Exw + S;
  T *__restrict__ Ezw = Exw + 2 * (size_t)S;
  T *__restrict__ Hxw = Exw + 3 * (size_t)S;
  T *__restrict__ Hyw = Exw + 4 * (size_t)S;
  T *__restrict__ Hzw = Exw + 5 * (size_t)S;
  const T ch = p.ch, ce = p.ce_s;
  T hxp = T(0), hyp = T(0), exc = T(0), exl = T(0), eyc = T(0), eys = T(0);
  bool have = false;
  for (int k = kb; k < ke; ++k) {
    // general planes belong to the general launches, super-chunk nodes to the
    // two-step pass; a plane that follows a super node recomputes its new H
    // (plane_plain holds there) from the read copy
    if (!plane_plain(p, tl, k) || (p.skip_super && in_super(p, i, j, k))) {
      have = false;
      continue;
    }
    const uint32_t q = (uint32_t)k * PL + (uint32_t)j * pitch + (uint32_t)i;
    if (!have) {
      exc = Ex[q];
      exl = Ex[q - 1];
      eyc = Ey[q];
      eys = Ey[q - pitch];
      if (plane_plain(p, tl, k - 1)) {
        const uint32_t r = q - PL;
        const T ezr = Ez[r];
        hxp = Hx[r] - ch * ((Ez[r + pitch] - ezr) - (eyc - Ey[r]));
        hyp = Hy[r] - ch * ((exc - Ex[r]) - (Ez[r + 1] - ezr));
      } else {
        hxp = Hxw[q - PL];
        hyp = Hyw[q - PL];
      }
      have = true;
    }
    const T exN = Ex[q + pitch], exS = Ex[q - pitch], exLN = Ex[q + pitch - 1];
    const T eyR = Ey[q + 1], eyRS = Ey[q + 1 - pitch], eyL = Ey[q - 1];
    const T ezC = Ez[q], ezN = Ez[q + pitch], ezR = Ez[q + 1], ezS = Ez[q - pitch], ezL = Ez[q - 1];
    const T exc1 = Ex[q + PL], exl1 = Ex[q + PL - 1], eyc1 = Ey[q + PL], eys1 = Ey[q + PL - pitch];
    const T hxC = Hx[q], hxS = Hx[q - pitch], hyC = Hy[q], hyL = Hy[q - 1];
    const T hzC = Hz[q], hzS = Hz[q - pitch], hzL = Hz[q - 1];
    const T hx00 = hxC - ch * ((ezN - ezC) - (eyc1 - eyc));
    const T hx0m = hxS - ch * ((ezC - ezS) - (eys1 - eys));
    const T hy00 = hyC - ch * ((exc1 - exc) - (ezR - ezC));
    const T hym0 = hyL - ch * ((exl1 - exl) - (ezC - ezL));
    const T hz00 = hzC - ch * ((eyR - eyc) - (exN - exc));
    const T hz0m = hzS - ch * ((eyRS - eys) - (exc - exS));
    const T hzm0 = hzL - ch * ((eyc - eyL) - (exLN - exl));
    // streaming stores: the new copy is not read again in this step
    __builtin_nontemporal_store(hx00, &Hxw[q]);
    __builtin_nontemporal_store(hy00, &Hyw[q]);
    __builtin_nontemporal_store(hz00, &Hzw[q]);
    __builtin_nontemporal_store(exc + ce * ((hz00 - hz0m) - (hy00 - hyp)), &Exw[q]);
    __builtin_nontemporal_store(eyc + ce * ((hx00 - hxp) - (hz00 - hzm0)), &Eyw[q]);
    __builtin_nontemporal_store(ezC + ce * ((hy00 - hym0) - (hx00 - hx0m)), &Ezw[q]);
    hxp = hx00;
    hyp = hy00;
    exc = exc1;
    exl = exl1;
    eyc = eyc1;
    eys = eys1;
  }
}

// ---------------------------------------------------------------- two-step
// Two time steps of the plain background per pass over a super-chunk
// (60 x 16 x 8 nodes): the update of step3d_plain applied twice, to the last
// bit.  A wavefront covers 64 consecutive columns c = a - 2 + lane (outputs
// for lanes 2..61; neighbours along x come from the adjacent lane by DPP wave
// shifts) and four output rows, holding the two rows below and above them in
// registers; it marches through planes kb-2 .. ke, carrying E^n, H^{n+1/2},
// E^{n+1} and the x, y components of H^{n+3/2} of the planes below, with the
// next plane's loads issued one iteration ahead.  Validity shrinks by one
// column per half step (H^{n+1/2}: lanes 0..62, E^{n+1}: 1..62, H^{n+3/2}:
// 1..61, E^{n+2}: 2..61), by one row per half step in y and one plane in z.
// Border nodes (faces flagged by the planner) also store E^{n+1}, H^{n+1/2}
// into the intermediate copy, which the per-step launches of the second step
// read.  No LDS and no barriers.
constexpr int SR = 4, SW = SCY / SR;  // rows per wavefront, wavefronts per workgroup

// v of lane l-1 (wave_shr:1) and of lane l+1 (wave_shl:1); the lane without
// a source gets 0, which only feeds values outside the valid lanes.
__device__ __forceinline__ float lane_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__global__ void __launch_bounds__(64 * SW) step3d_super(const Step3D<float> p, const float *__restrict__ rd,
                                                        float *__restrict__ mid, float *__restrict__ out,
                                                        const int *__restrict__ list) {
  const int code = ((cptr<int>)list)[blockIdx.x];
  if (code < 0) return;
  const int faces = code & 63, cidx = code >> 6;
  const int cx = cidx % p.sn[0], cy = (cidx / p.sn[0]) % p.sn[1], cz = cidx / (p.sn[0] * p.sn[1]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int a = p.so[0] + cx * SCX, c = a - 2 + lane;
  const int b = p.so[1] + cy * SCY, y0 = b + wv * SR;
  const int kb = p.so[2] + cz * SCZ, ke = kb + SCZ;
  const uint32_t pitch = p.pitch, PL = p.PL, S = p.S;
  const float *__restrict__ Ex = rd + p.G0;
  const float *__restrict__ Ey = Ex + S;
  const float *__restrict__ Ez = Ex + 2 * (size_t)S;
  const float *__restrict__ Hx = Ex + 3 * (size_t)S;
  const float *__restrict__ Hy = Ex + 4 * (size_t)S;
  const float *__restrict__ Hz = Ex + 5 * (size_t)S;
  float *__restrict__ O = out + p.G0;
  float *__restrict__ M = mid + p.G0;
  const float ch = p.ch, ce = p.ce_s;
  auto at = [&](int t, int k) { return (uint32_t)k * PL + (uint32_t)(y0 - 2 + t) * pitch + (uint32_t)c; };
  const bool own = lane >= 2 && lane < 2 + SCX;
  const bool bxf = (lane == 2 && (faces & 1)) || (lane == 1 + SCX && (faces & 2));
  constexpr int NE = SR + 4, NH = SR + 3;
  // E^n(m) rows 0..NE-1; H^{n+1/2}(m-1) rows 0..NH-1; E^{n+1}(m-1) rows 1..NH-1; H^{n+3/2}(m-2) x, y rows 2..SR+1
  float ex0[NE], ey0[NE], ez0[NE], h1x[NH], h1y[NH], h1z[NH], e1x[NH], e1y[NH], e1z[NH], h2x[SR + 2], h2y[SR + 2];
  float exn[NE], eyn[NE], ezn[NE], hxo[NH], hyo[NH], hzo[NH];
#pragma unroll
  for (int t = 0; t < NH; ++t) h1x[t] = h1y[t] = h1z[t] = e1x[t] = e1y[t] = e1z[t] = 0.f;
#pragma unroll
  for (int t = 0; t < SR + 2; ++t) h2x[t] = h2y[t] = 0.f;
  int m = kb - 2;
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const uint32_t q = at(t, m);
    ex0[t] = Ex[q]; ey0[t] = Ey[q]; ez0[t] = Ez[q];
  }
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const uint32_t q = at(t, m + 1);
    exn[t] = Ex[q]; eyn[t] = Ey[q]; ezn[t] = Ez[q];
  }
#pragma unroll
  for (int t = 0; t < NH; ++t) {
    const uint32_t q = at(t, m);
    hxo[t] = Hx[q]; hyo[t] = Hy[q]; hzo[t] = Hz[q];
  }
  for (; m <= ke; ++m) {
    // next plane's E^n(m+2) and H^{n-1/2}(m+1), one iteration ahead
    float pxn[NE], pyn[NE], pzn[NE], pxo[NH], pyo[NH], pzo[NH];
    if (m < ke) {
#pragma unroll
      for (int t = 0; t < NE; ++t) {
        const uint32_t q = at(t, m + 2);
        pxn[t] = Ex[q]; pyn[t] = Ey[q]; pzn[t] = Ez[q];
      }
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        const uint32_t q = at(t, m + 1);
        pxo[t] = Hx[q]; pyo[t] = Hy[q]; pzo[t] = Hz[q];
      }
    } else {
#pragma unroll
      for (int t = 0; t < NE; ++t) pxn[t] = pyn[t] = pzn[t] = 0.f;
#pragma unroll
      for (int t = 0; t < NH; ++t) pxo[t] = pyo[t] = pzo[t] = 0.f;
    }
    // H^{n+1/2}(m): Hx: d_y Ez - d_z Ey; Hy: d_z Ex - d_x Ez; Hz: d_x Ey - d_y Ex
    float hx[NH], hy[NH], hz[NH];
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const float ezR = lane_right(ez0[t]), eyR = lane_right(ey0[t]);
      hx[t] = hxo[t] - ch * ((ez0[t + 1] - ez0[t]) - (eyn[t] - ey0[t]));
      hy[t] = hyo[t] - ch * ((exn[t] - ex0[t]) - (ezR - ez0[t]));
      hz[t] = hzo[t] - ch * ((eyR - ey0[t]) - (ex0[t + 1] - ex0[t]));
    }
    // E^{n+1}(m): Ex: d_y Hz - d_z Hy; Ey: d_z Hx - d_x Hz; Ez: d_x Hy - d_y Hx
    float ex[NH], ey[NH], ez[NH];
#pragma unroll
    for (int t = 1; t < NH; ++t) {
      const float hzL = lane_left(hz[t]), hyL = lane_left(hy[t]);
      ex[t] = ex0[t] + ce * ((hz[t] - hz[t - 1]) - (hy[t] - h1y[t]));
      ey[t] = ey0[t] + ce * ((hx[t] - h1x[t]) - (hz[t] - hzL));
      ez[t] = ez0[t] + ce * ((hy[t] - hyL) - (hx[t] - hx[t - 1]));
    }
    if (m >= kb && m < ke) {
      // border nodes: the state after the first step, for the per-step launches
#pragma unroll
      for (int t = 2; t < SR + 2; ++t) {
        const int j = y0 - 2 + t;
        const bool border = bxf || (j == b && (faces & 4)) || (j == b + SCY - 1 && (faces & 8)) ||
                            (m == kb && (faces & 16)) || (m == ke - 1 && (faces & 32));
        if (own && border) {
          const uint32_t q = at(t, m);
          M[q] = ex[t];
          M[q + S] = ey[t];
          M[q + 2 * S] = ez[t];
          M[q + 3 * S] = hx[t];
          M[q + 4 * S] = hy[t];
          M[q + 5 * S] = hz[t];
        }
      }
    }
    if (m >= kb) {
      // H^{n+3/2}(m-1) from E^{n+1}(m-1) (carried) and E^{n+1}(m)
      float gx[SR + 2], gy[SR + 2], gz[SR + 2];
#pragma unroll
      for (int t = 1; t < SR + 2; ++t) {
        const float ezR = lane_right(e1z[t]), eyR = lane_right(e1y[t]);
        gx[t] = h1x[t] - ch * ((e1z[t + 1] - e1z[t]) - (ey[t] - e1y[t]));
        gy[t] = h1y[t] - ch * ((ex[t] - e1x[t]) - (ezR - e1z[t]));
        gz[t] = h1z[t] - ch * ((eyR - e1y[t]) - (e1x[t + 1] - e1x[t]));
      }
      if (m >= kb + 1) {
        // E^{n+2}(m-1); store it and H^{n+3/2}(m-1)
#pragma unroll
        for (int t = 2; t < SR + 2; ++t) {
          const float gzL = lane_left(gz[t]), gyL = lane_left(gy[t]);
          const float fx = e1x[t] + ce * ((gz[t] - gz[t - 1]) - (gy[t] - h2y[t]));
          const float fy = e1y[t] + ce * ((gx[t] - h2x[t]) - (gz[t] - gzL));
          const float fz = e1z[t] + ce * ((gy[t] - gyL) - (gx[t] - gx[t - 1]));
          if (own) {
            const uint32_t q = at(t, m - 1);
            __builtin_nontemporal_store(fx, &O[q]);
            __builtin_nontemporal_store(fy, &O[q + S]);
            __builtin_nontemporal_store(fz, &O[q + 2 * S]);
            __builtin_nontemporal_store(gx[t], &O[q + 3 * S]);
            __builtin_nontemporal_store(gy[t], &O[q + 4 * S]);
            __builtin_nontemporal_store(gz[t], &O[q + 5 * S]);
          }
        }
      }
#pragma unroll
      for (int t = 2; t < SR + 2; ++t) {
        h2x[t] = gx[t];
        h2y[t] = gy[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      ex0[t] = exn[t]; ey0[t] = eyn[t]; ez0[t] = ezn[t];
      exn[t] = pxn[t]; eyn[t] = pyn[t]; ezn[t] = pzn[t];
    }
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      h1x[t] = hx[t]; h1y[t] = hy[t]; h1z[t] = hz[t];
      hxo[t] = pxo[t]; hyo[t] = pyo[t]; hzo[t] = pzo[t];
    }
#pragma unroll
    for (int t = 1; t < NH; ++t) {
      e1x[t] = ex[t]; e1y[t] = ey[t]; e1z[t] = ez[t];
    }
  }
}

}  // namespace

namespace {

// Deal the chunks (codes in (bz, by, bx) order) to the 8 XCDs: groups of
// neighbouring chunks (one z-chunk, four tile rows) go whole to the XCD with
// the least work so far, largest group first, so neighbours share an L2;
// slot b of the launch runs on XCD b mod 8.
std::vector<int> xcd_order(const std::vector<int> &codes, const std::vector<int> &group, const std::vector<int> &work) {
  std::vector<std::pair<int, int>> gs;  // (group, first index)
  for (size_t i = 0; i < codes.size(); ++i)
    if (i == 0 || group[i] != group[i - 1]) gs.push_back({group[i], (int)i});
  std::vector<int> gw(gs.size(), 0), ge(gs.size(), 0);
  for (size_t g = 0; g < gs.size(); ++g) {
    ge[g] = g + 1 < gs.size() ? gs[g + 1].second : (int)codes.size();
    for (int i = gs[g].second; i < ge[g]; ++i) gw[g] += work[i];
  }
  std::vector<int> ord(gs.size());
  for (size_t g = 0; g < gs.size(); ++g) ord[g] = (int)g;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return gw[a] > gw[b]; });
  std::vector<int> load(8, 0);
  std::vector<std::vector<int>> per(8);
  std::vector<std::vector<int>> mine(8);
  for (int g : ord) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += gw[g];
    mine[x].push_back(g);
  }
  size_t len = 0;
  for (int x = 0; x < 8; ++x) {
    std::sort(mine[x].begin(), mine[x].end());
    for (int g : mine[x])
      for (int i = gs[g].second; i < ge[g]; ++i) per[x].push_back(codes[i]);
    len = std::max(len, per[x].size());
  }
  std::vector<int> out(len * 8, -1);
  for (int x = 0; x < 8; ++x)
    for (size_t t = 0; t < per[x].size(); ++t) out[t * 8 + x] = per[x][t];
  return out;
}

}  // namespace

template <typename T>
std::vector<int> gen3d_plan(const Step3D<T> &p, int &nS, int &nM, int &nD, int &axD) {
  const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
  const int nbx = (nx + TX - 1) / TX, nby = (ny + TY - 1) / TY, nbz = (nz + KC - 1) / KC;
  std::vector<int> cS, cM, cD, gS, gM, gD, wS, wM, wD;
  axD = 0;
  for (int bz = 0; bz < nbz; ++bz)
    for (int by = 0; by < nby; ++by)
      for (int bx = 0; bx < nbx; ++bx) {
        Tile tl = tile_xy(p, bx * TX, by * TY);
        tl.kb = bz * KC;
        tl.ke = std::min(tl.kb + KC, nz);
        // the planes the chunk updates and the planes below them whose new H
        // it recomputes (as the kernel's march does)
        int ax = 0, planes = 0;
        bool have = false;
        for (int k = tl.kb; k < tl.ke; ++k) {
          if (plane_plain(p, tl, k)) {
            have = false;
            continue;
          }
          if (!have && k >= 1) ax |= plane_axes(p, k - 1);
          ax |= plane_axes(p, k);
          have = true;
          ++planes;
        }
        if (planes == 0) continue;
        ax |= tile_axes(p, tl);
        const int c = (bz * nby + by) * nbx + bx, grp = bz * ((nby + 3) / 4) + by / 4;
        if (design_chunk(p, tl)) {
          axD |= ax;
          cD.push_back(c); gD.push_back(grp); wD.push_back(planes);
        } else if (ax == 0 || ax == 1 || ax == 2 || ax == 4) {
          const int a = ax == 1 ? 0 : ax == 2 ? 1 : ax == 4 ? 2 : 3;
          cS.push_back(4 * c + a); gS.push_back(grp); wS.push_back(planes);
        } else {
          cM.push_back(c); gM.push_back(grp); wM.push_back(planes);
        }
      }
  if (axD) axD = 7;
  std::vector<int> out = xcd_order(cS, gS, wS);
  nS = (int)out.size();
  const std::vector<int> m = xcd_order(cM, gM, wM), d = xcd_order(cD, gD, wD);
  nM = (int)m.size();
  nD = (int)d.size();
  out.insert(out.end(), m.begin(), m.end());
  out.insert(out.end(), d.begin(), d.end());
  return out;
}

template <typename T>
std::vector<int> plan3d_super(const Step3D<T> &p, int so[3], int sn[3], std::vector<unsigned char> &flags) {
  const int n3[3] = {p.n[0], p.n[1], p.n[2]}, nx = n3[0], ny = n3[1], nz = n3[2], P = p.P;
  const size_t tot = (size_t)nx * ny * nz;
  auto id = [&](int i, int j, int k) { return ((size_t)k * ny + j) * nx + i; };
  // nodes of plain tile-planes (general tiling)
  std::vector<unsigned char> ok(tot, 0);
  for (int j0 = 0; j0 < ny; j0 += TY)
    for (int i0 = 0; i0 < nx; i0 += TX) {
      const Tile tl = tile_xy(p, i0, j0);
      if (!tl.xy_plain) continue;
      for (int k = 0; k < nz; ++k)
        if (plane_plain(p, tl, k))
          for (int j = j0; j < std::min(j0 + TY, ny); ++j)
            for (int i = i0; i < std::min(i0 + TX, nx); ++i) ok[id(i, j, k)] = 1;
    }
  // plain background: off the walls and absorber (E and H), injection lines
  // and faces, design and gap; then every node within three of it too
  std::vector<unsigned char> ph(tot, 0);
  std::vector<char> axok[3];
  for (int a = 0; a < 3; ++a) {
    axok[a].assign(n3[a], 0);
    for (int i = 1; i <= n3[a] - 2; ++i) {
      bool g = !pml_e(i, n3[a], P) && !pml_h(i, n3[a], P);
      if (p.tf_on) g = g && i != p.lo[a] - 1 && i != p.lo[a] && i != p.hi[a] && i != p.hi[a] + 1;
      axok[a][i] = g;
    }
  }
  auto inbox = [](const int *lo, const int *n, int i, int j, int k) {
    return i >= lo[0] && i < lo[0] + n[0] && j >= lo[1] && j < lo[1] + n[1] && k >= lo[2] && k < lo[2] + n[2];
  };
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        ph[id(i, j, k)] = axok[0][i] && axok[1][j] && axok[2][k] && !inbox(p.d0, p.dn, i, j, k) &&
                          !inbox(p.g0, p.gn, i, j, k);
  // erosion by 3 along each axis in turn (a box of side 7): a node stays when
  // the 7 nodes of its line centred on it are all plain
  std::vector<unsigned char> tmp(tot);
  const size_t st[3] = {1, (size_t)nx, (size_t)nx * ny};
  for (int a = 0; a < 3; ++a) {
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    for (int u = 0; u < n3[b1]; ++u)
      for (int v = 0; v < n3[b2]; ++v) {
        const size_t base = (size_t)u * st[b1] + (size_t)v * st[b2];
        int run = 0;  // plain nodes in a row ending at x + 3
        for (int x = -3; x < n3[a]; ++x) {
          const int y = x + 3;
          run = (y < n3[a] && ph[base + (size_t)y * st[a]]) ? run + 1 : 0;
          if (x >= 0) tmp[base + (size_t)x * st[a]] = x >= 3 && x + 3 < n3[a] && run >= 7;
        }
      }
    ph.swap(tmp);
  }
  // prefix sums of ineligible nodes, for O(1) chunk tests
  std::vector<int> pre((size_t)(nx + 1) * (ny + 1) * (nz + 1), 0);
  auto P3 = [&](int i, int j, int k) -> int & { return pre[((size_t)k * (ny + 1) + j) * (nx + 1) + i]; };
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int bad = !(ok[id(i, j, k)] && ph[id(i, j, k)]);
        P3(i + 1, j + 1, k + 1) = bad + P3(i, j + 1, k + 1) + P3(i + 1, j, k + 1) + P3(i + 1, j + 1, k) -
                                  P3(i, j, k + 1) - P3(i, j + 1, k) - P3(i + 1, j, k) + P3(i, j, k);
      }
  auto clean = [&](int x, int y, int z) {  // chunk with origin (x, y, z) has no ineligible node
    const int X = x + SCX, Y = y + SCY, Z = z + SCZ;
    if (x < 0 || y < 0 || z < 0 || X > nx || Y > ny || Z > nz) return false;
    return P3(X, Y, Z) - P3(x, Y, Z) - P3(X, y, Z) - P3(X, Y, z) + P3(x, y, Z) + P3(x, Y, z) + P3(X, y, z) -
               P3(x, y, z) == 0;
  };
  // origin of the chunk grid: a few offsets from the plain box, the one
  // covering the most nodes
  int best = -1;
  for (int dz = 0; dz < SCZ; dz += 2)
    for (int dy = 0; dy < SCY; dy += 2)
      for (int dx = 0; dx < 12; dx += 2) {
        const int o[3] = {p.pb[0] + dx, p.pb[1] + dy, p.pb[2] + dz};
        int cnt = 0;
        for (int z = o[2]; z + SCZ <= nz; z += SCZ)
          for (int y = o[1]; y + SCY <= ny; y += SCY)
            for (int x = o[0]; x + SCX <= nx; x += SCX) cnt += clean(x, y, z);
        if (cnt > best) {
          best = cnt;
          for (int a = 0; a < 3; ++a) so[a] = o[a];
        }
      }
  const int sc[3] = {SCX, SCY, SCZ};
  for (int a = 0; a < 3; ++a) sn[a] = best > 0 ? std::max(0, (n3[a] - so[a]) / sc[a]) : 0;
  flags.assign((size_t)std::max(1, sn[0] * sn[1] * sn[2]), 0);
  if (best <= 0) return {};
  for (int cz = 0; cz < sn[2]; ++cz)
    for (int cy = 0; cy < sn[1]; ++cy)
      for (int cx = 0; cx < sn[0]; ++cx)
        flags[((size_t)cz * sn[1] + cy) * sn[0] + cx] =
            clean(so[0] + cx * SCX, so[1] + cy * SCY, so[2] + cz * SCZ);
  auto sup = [&](int cx, int cy, int cz) {
    return cx >= 0 && cy >= 0 && cz >= 0 && cx < sn[0] && cy < sn[1] && cz < sn[2] &&
           flags[((size_t)cz * sn[1] + cy) * sn[0] + cx];
  };
  std::vector<int> codes, group, work;
  for (int cz = 0; cz < sn[2]; ++cz)
    for (int cy = 0; cy < sn[1]; ++cy)
      for (int cx = 0; cx < sn[0]; ++cx) {
        if (!sup(cx, cy, cz)) continue;
        // face f (axis f/2, side f%2) is a border when any of the nine chunks
        // across it (edges and corners included) is not a super-chunk
        int faces = 0;
        for (int f = 0; f < 6; ++f) {
          const int ax = f / 2, sd = f % 2 ? 1 : -1;
          bool border = false;
          for (int u = -1; u <= 1; ++u)
            for (int v = -1; v <= 1; ++v) {
              int d[3];
              d[ax] = sd;
              d[(ax + 1) % 3] = u;
              d[(ax + 2) % 3] = v;
              border = border || !sup(cx + d[0], cy + d[1], cz + d[2]);
            }
          if (border) faces |= 1 << f;
        }
        codes.push_back((((cz * sn[1] + cy) * sn[0] + cx) << 6) | faces);
        group.push_back(cz * ((sn[1] + 1) / 2) + cy / 2);
        work.push_back(1);
      }
  return xcd_order(codes, group, work);
}

#ifndef FDTD3D_AUX
#define FDTD3D_AUX 1
#endif
#ifndef FDTD3D_MERGE
#define FDTD3D_MERGE 1
#endif

// The three general lists write disjoint tile-chunks of the write copy and
// read only the read copy, so they may run in any order or side by side.
// FP32 forward with no design chunk in the absorber: one launch over all
// three.  Otherwise three launches: the
// multi-axis list on the second stream, beside the design list and then the
// single-axis list on the context stream (the order measured fastest for
// the FP32 adjoint, whose multi-axis body is the longest).
template <typename T, bool ADJ>
static void launch_general(const Step3D<T> &q, int n, hipStream_t s, const Aux3D &aux) {
  const int *L = q.glist;
  if constexpr (std::is_same<T, float>::value && !ADJ) {
    const int tot = q.gS + q.gM + q.gD;
    if (FDTD3D_MERGE && tot > 0 && !q.gAxD) {
      hipLaunchKernelGGL(step3d_general_fwd, dim3(tot), dim3(NT), 0, s, q, n, L);
      return;
    }
  }
  const bool two = FDTD3D_AUX && aux.stream && q.gM > 0;
  hipStream_t s2 = s;
  if (two) {
    FDTD_HIP(hipEventRecord(aux.fork, s));
    FDTD_HIP(hipStreamWaitEvent(aux.stream, aux.fork, 0));
    s2 = aux.stream;
  }
  if (q.gM > 0) hipLaunchKernelGGL((step3d_general<T, ADJ, false, 7>), dim3(q.gM), dim3(NT), 0, s2, q, n, L + q.gS);
  if (q.gD > 0) {
    if (q.gAxD)
      hipLaunchKernelGGL((step3d_general<T, ADJ, true, 7>), dim3(q.gD), dim3(NT), 0, s, q, n, L + q.gS + q.gM);
    else
      hipLaunchKernelGGL((step3d_general<T, ADJ, true, 0>), dim3(q.gD), dim3(NT), 0, s, q, n, L + q.gS + q.gM);
  }
  if (q.gS > 0) hipLaunchKernelGGL((step3d_general<T, ADJ, false, 8>), dim3(q.gS), dim3(NT), 0, s, q, n, L);
  if (two) {
    FDTD_HIP(hipEventRecord(aux.join, aux.stream));
    FDTD_HIP(hipStreamWaitEvent(s, aux.join, 0));
  }
}

template <typename T>
void launch_step3d(const Step3D<T> &p, T *rd, T *wr, int n, bool adjoint, hipStream_t s, const Aux3D &aux) {
  Step3D<T> q = p;  // copy 0 is read, copy 1 written
  q.A[0] = rd;
  q.A[1] = wr;
  // the general tile-chunks (one launch, or three by what they need), then
  // the plain ones, which read back the new H of a general plane below them
  if (adjoint) launch_general<T, true>(q, n, s, aux);
  else launch_general<T, false>(q, n, s, aux);
  int pbx, pby, pbz;
  plain_grid(p.pb, pbx, pby, pbz);
  if (p.pb[3] > 0 && p.pb[4] > 0 && p.pb[5] > 0)
    hipLaunchKernelGGL(step3d_plain<T>, dim3(pbx * pby * pbz), dim3(PNT), 0, s, q);
}

template <typename T>
void plain3d_box(const Step3D<T> &p, int pb[6]) {
  const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
  int lo[3] = {nx, ny, nz}, hi[3] = {0, 0, 0};
  for (int j0 = 0; j0 < ny; j0 += TY)
    for (int i0 = 0; i0 < nx; i0 += TX) {
      const Tile tl = tile_xy(p, i0, j0);
      if (!tl.xy_plain) continue;
      for (int k = 0; k < nz; ++k) {
        if (!plane_plain(p, tl, k)) continue;
        lo[0] = std::min(lo[0], i0);
        hi[0] = std::max(hi[0], std::min(i0 + TX, nx));
        lo[1] = std::min(lo[1], j0);
        hi[1] = std::max(hi[1], std::min(j0 + TY, ny));
        lo[2] = std::min(lo[2], k);
        hi[2] = std::max(hi[2], k + 1);
      }
    }
  for (int a = 0; a < 3; ++a) {
    pb[a] = hi[a] > lo[a] ? lo[a] : 0;
    pb[3 + a] = hi[a] > lo[a] ? hi[a] - lo[a] : 0;
  }
}

template std::vector<int> gen3d_plan<float>(const Step3D<float> &, int &, int &, int &, int &);
template std::vector<int> gen3d_plan<double>(const Step3D<double> &, int &, int &, int &, int &);
template void plain3d_box<float>(const Step3D<float> &, int *);
template void plain3d_box<double>(const Step3D<double> &, int *);
template void launch_step3d<float>(const Step3D<float> &, float *, float *, int, bool, hipStream_t, const Aux3D &);
template void launch_step3d<double>(const Step3D<double> &, double *, double *, int, bool, hipStream_t, const Aux3D &);
template std::vector<int> plan3d_super<float>(const Step3D<float> &, int *, int *, std::vector<unsigned char> &);
template std::vector<int> plan3d_super<double>(const Step3D<double> &, int *, int *, std::vector<unsigned char> &);

void launch_step3d_super(const Step3D<float> &p, const float *rd, float *mid, float *out, const int *list, int count,
                         hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(step3d_super, dim3(count), dim3(64 * SW), 0, s, p, rd, mid, out, list);
}

}  // namespace fdtd
