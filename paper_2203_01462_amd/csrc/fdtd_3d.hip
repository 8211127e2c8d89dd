// fdtd_3d.hip -- fused time step of the 3D Drude-FDTD solve and its adjoint.
//
// Per step, on the full Yee cell (Sec. 3.2; eqs. (10a-c)):
//   H^{n+1/2} = H^{n-1/2} - dt/mu0 curl E^n                (CPML, total-field faces)
//   E^{n+1} = E^n + 2/D [dt curl H^{n+1/2} - dt (1+kp)/2 J^n - (beta+sigma) dt E^n]
//   J^{n+1} = kp J^n + beta (E^{n+1} + E^n)                 (Drude edges, eqs. (4)-(5))
// The adjoint step (eq. (20)) is the same update on (E*, H*, J*) driven by
// the gap source, with each CPML term replaced by its exact transpose, and it
// accumulates the per-edge sensitivity of eq. (25) folded with eq. (27).
//
// Work split: a workgroup owns a 32 x 8 x 2 block of cells (one thread per
// (i, j) column, two cells along z).  Each thread recomputes the new H it
// needs on the low side (j-1, i-1, k-1) instead of waiting for another
// workgroup, so a step is one pass over two copies of every array.  Blocks
// whose reach holds only background dielectric run step3d_bulk (one batch
// of loads, the plain update, identical for forward and adjoint); all other
// blocks run step3d_general.  The two kernels are launched back to back on
// complementary block sets.
#include "fdtd_3d.hpp"

namespace fdtd {
namespace {

constexpr int TX = 32, TY = 8, R = 2, NT = TX * TY;

__device__ __forceinline__ bool pml_e(int i, int n, int P) { return P > 0 && (i < P || i > n - 1 - P); }
__device__ __forceinline__ bool pml_h(int i, int n, int P) { return P > 0 && (i < P || i >= n - 1 - P); }

#ifndef FDTD3D_MAP
#define FDTD3D_MAP 1
#endif
#ifndef FDTD3D_GROUP
#define FDTD3D_GROUP 4
#endif

// Block -> (bx, by, bz).  Consecutive dispatch slots go round-robin over the
// 8 XCDs (each with its own L2).  Within an XCD blocks are taken x fastest,
// then y, so in-plane neighbours share an L2.  Mode 1: XCD x takes z-slabs
// x, x+8, ...; mode 2: one contiguous z-band per XCD; mode 3: runs of
// FDTD3D_GROUP consecutive z-slabs dealt round-robin to the XCDs (z-halos
// shared inside a run, slow slabs spread over the XCDs).
__device__ __forceinline__ void block_of(int bid, int nbx, int nby, int nbz, int &bx, int &by, int &bz) {
  const int per = nbx * nby;
  const int x = bid & 7, k = bid >> 3;
  if (FDTD3D_MAP == 1 && nbz % 8 == 0) {
    bx = k % nbx; by = (k / nbx) % nby; bz = x + 8 * (k / per);
    return;
  }
  if (FDTD3D_MAP == 2 && nbz % 8 == 0) {
    bx = k % nbx; by = (k / nbx) % nby; bz = x * (nbz / 8) + k / per;
    return;
  }
  if (FDTD3D_MAP == 3 && nbz % (8 * FDTD3D_GROUP) == 0) {
    const int zl = k / per, c = zl / FDTD3D_GROUP, s = zl % FDTD3D_GROUP;
    bx = k % nbx; by = (k / nbx) % nby; bz = (c * 8 + x) * FDTD3D_GROUP + s;
    return;
  }
  bx = bid % nbx;
  by = (bid / nbx) % nby;
  bz = bid / per;
}

template <typename T>
__device__ __forceinline__ bool block_is_bulk(const Step3D<T> &p, int i0, int j0, int k0) {
  const int P = p.P;
  if (i0 < P + 1 || i0 + TX > p.n[0] - 1 - P) return false;
  if (j0 < P + 1 || j0 + TY > p.n[1] - 1 - P) return false;
  if (k0 < P + 1 || k0 + R > p.n[2] - 1 - P) return false;
  auto hit = [](int lo, int hi, int v) { return v >= lo && v <= hi; };
  if (p.tf_on) {
    const int x0 = i0 - 1, x1 = i0 + TX, y0 = j0 - 1, y1 = j0 + TY, z0 = k0 - 1, z1 = k0 + R;
    for (int d = -1; d <= 0; ++d) {
      if (hit(x0, x1, p.lo[0] + d) || hit(x0, x1, p.hi[0] + 1 + d)) return false;
      if (hit(y0, y1, p.lo[1] + d) || hit(y0, y1, p.hi[1] + 1 + d)) return false;
      if (hit(z0, z1, p.lo[2] + d) || hit(z0, z1, p.hi[2] + 1 + d)) return false;
    }
  }
  auto meets = [&](const int *b0, const int *bn) {
    return i0 + TX - 1 >= b0[0] && i0 < b0[0] + bn[0] && j0 + TY - 1 >= b0[1] && j0 < b0[1] + bn[1] &&
           k0 + R - 1 >= b0[2] && k0 < b0[2] + bn[2];
  };
  return !meets(p.d0, p.dn) && !meets(p.g0, p.gn);
}

// ---------------------------------------------------------------- bulk
template <typename T>
__global__ void __launch_bounds__(NT) step3d_bulk(const Step3D<T> p, const int par) {
  const int nbx = (p.n[0] + TX - 1) / TX, nby = (p.n[1] + TY - 1) / TY, nbz = (p.n[2] + R - 1) / R;
  int bx, by, bz;
  block_of(blockIdx.x, nbx, nby, nbz, bx, by, bz);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * R;
  if (!block_is_bulk(p, i0, j0, k0)) return;
  const int i = i0 + (threadIdx.x % TX), j = j0 + (threadIdx.x / TX);
  const long long sy = p.pitch, sz = p.sz;
  const long long q = (long long)k0 * sz + (long long)j * sy + i;
  const T *__restrict__ Ex = p.E[par][0];
  const T *__restrict__ Ey = p.E[par][1];
  const T *__restrict__ Ez = p.E[par][2];
  const T *__restrict__ Hx = p.H[par][0];
  const T *__restrict__ Hy = p.H[par][1];
  const T *__restrict__ Hz = p.H[par][2];
  T *__restrict__ Exw = p.E[par ^ 1][0];
  T *__restrict__ Eyw = p.E[par ^ 1][1];
  T *__restrict__ Ezw = p.E[par ^ 1][2];
  T *__restrict__ Hxw = p.H[par ^ 1][0];
  T *__restrict__ Hyw = p.H[par ^ 1][1];
  T *__restrict__ Hzw = p.H[par ^ 1][2];
#define A3(arr, di, dj, dk) arr[q + (di) + (long long)(dj) * sy + (long long)(dk) * sz]
  T exC[4], exL[3], exN[2], exS[2], exLN[2];
  T eyC[4], eyS[3], eyR[2], eyRS[2], eyL[2];
  T ezC[3], ezN[3], ezR[3], ezS[2], ezL[2];
  T hxC[3], hxS[2], hyC[3], hyL[2], hzC[2], hzS[2], hzL[2];
#pragma unroll
  for (int r = 0; r < 4; ++r) { exC[r] = A3(Ex, 0, 0, r - 1); eyC[r] = A3(Ey, 0, 0, r - 1); }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    exL[r] = A3(Ex, -1, 0, r); eyS[r] = A3(Ey, 0, -1, r);
    ezC[r] = A3(Ez, 0, 0, r - 1); ezN[r] = A3(Ez, 0, 1, r - 1); ezR[r] = A3(Ez, 1, 0, r - 1);
    hxC[r] = A3(Hx, 0, 0, r - 1); hyC[r] = A3(Hy, 0, 0, r - 1);
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    exN[s] = A3(Ex, 0, 1, s); exS[s] = A3(Ex, 0, -1, s); exLN[s] = A3(Ex, -1, 1, s);
    eyR[s] = A3(Ey, 1, 0, s); eyRS[s] = A3(Ey, 1, -1, s); eyL[s] = A3(Ey, -1, 0, s);
    ezS[s] = A3(Ez, 0, -1, s); ezL[s] = A3(Ez, -1, 0, s);
    hxS[s] = A3(Hx, 0, -1, s); hyL[s] = A3(Hy, -1, 0, s);
    hzC[s] = A3(Hz, 0, 0, s); hzS[s] = A3(Hz, 0, -1, s); hzL[s] = A3(Hz, -1, 0, s);
  }
  const T ch = p.ch, ce = p.ce_s;
  T hx00[3], hy00[3], hx0m[2], hym0[2], hz00[2], hz0m[2], hzm0[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    hx00[r] = hxC[r] - ch * ((ezN[r] - ezC[r]) - (eyC[r + 1] - eyC[r]));
    hy00[r] = hyC[r] - ch * ((exC[r + 1] - exC[r]) - (ezR[r] - ezC[r]));
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    hx0m[s] = hxS[s] - ch * ((ezC[s + 1] - ezS[s]) - (eyS[s + 1] - eyS[s]));
    hym0[s] = hyL[s] - ch * ((exL[s + 1] - exL[s]) - (ezC[s + 1] - ezL[s]));
    hz00[s] = hzC[s] - ch * ((eyR[s] - eyC[s + 1]) - (exN[s] - exC[s + 1]));
    hz0m[s] = hzS[s] - ch * ((eyRS[s] - eyS[s]) - (exC[s + 1] - exS[s]));
    hzm0[s] = hzL[s] - ch * ((eyC[s + 1] - eyL[s]) - (exLN[s] - exL[s]));
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    A3(Hxw, 0, 0, s) = hx00[s + 1];
    A3(Hyw, 0, 0, s) = hy00[s + 1];
    A3(Hzw, 0, 0, s) = hz00[s];
    A3(Exw, 0, 0, s) = exC[s + 1] + ce * ((hz00[s] - hz0m[s]) - (hy00[s + 1] - hy00[s]));
    A3(Eyw, 0, 0, s) = eyC[s + 1] + ce * ((hx00[s + 1] - hx00[s]) - (hz00[s] - hzm0[s]));
    A3(Ezw, 0, 0, s) = ezC[s + 1] + ce * ((hy00[s + 1] - hym0[s]) - (hx00[s + 1] - hx0m[s]));
  }
#undef A3
}

// ---------------------------------------------------------------- general
// Indexing helper: components, validity ranges, bounds-checked loads.
template <typename T>
struct G3 {
  const Step3D<T> &p;
  int par;
  long long sy, sz;
  __device__ G3(const Step3D<T> &p_, int par_) : p(p_), par(par_), sy(p_.pitch), sz(p_.sz) {}
  __device__ long long at(int i, int j, int k) const { return (long long)k * sz + (long long)j * sy + i; }
  __device__ bool inside(int i, int j, int k) const {
    return i >= 0 && i < p.n[0] && j >= 0 && j < p.n[1] && k >= 0 && k < p.n[2];
  }
  // E_c is updated for index c in [0, n-2] and the others in [1, n-2];
  // H_c for index c in [1, n-2] and the others in [0, n-2].
  __device__ bool evalid(int c, int i, int j, int k) const {
    const int x[3] = {i, j, k};
    for (int d = 0; d < 3; ++d)
      if (x[d] < (d == c ? 0 : 1) || x[d] > p.n[d] - 2) return false;
    return true;
  }
  __device__ bool hvalid(int c, int i, int j, int k) const {
    const int x[3] = {i, j, k};
    for (int d = 0; d < 3; ++d)
      if (x[d] < (d == c ? 1 : 0) || x[d] > p.n[d] - 2) return false;
    return true;
  }
  __device__ T ld(const T *a, int i, int j, int k) const { return inside(i, j, k) ? a[at(i, j, k)] : T(0); }
  __device__ T einc(int n, int k) const { return p.einc[(long long)n * p.L + (k - p.kref)]; }
  __device__ T hinc(int n, int k) const { return p.hinc[(long long)n * p.L + (k - p.kref)]; }
};

// Forward: new H_c at (i,j,k) with CPML and the total-field corrections.
template <typename T, int C>
__device__ T h_fwd(const G3<T> &g, int n, int i, int j, int k, bool own) {
  if (!g.hvalid(C, i, j, k)) return T(0);
  constexpr int u = (C + 1) % 3, v = (C + 2) % 3;
  const Step3D<T> &p = g.p;
  const int x[3] = {i, j, k};
  int pu[3] = {i, j, k}, pv[3] = {i, j, k};
  pu[u] += 1;
  pv[v] += 1;
  const T *Ev = p.E[g.par][v], *Eu = p.E[g.par][u];
  const T du = g.ld(Ev, pu[0], pu[1], pu[2]) - g.ld(Ev, i, j, k);
  const T dv = g.ld(Eu, pv[0], pv[1], pv[2]) - g.ld(Eu, i, j, k);
  const long long q = g.at(i, j, k);
  T tu = du * p.ikh[u][x[u]], tv = dv * p.ikh[v][x[v]];
  if (pml_h(x[u], p.n[u], p.P)) {
    const T ps = p.bh[u][x[u]] * p.pH[g.par][C][u][q] + p.ah[u][x[u]] * du;
    tu += ps;
    if (own) p.pH[g.par ^ 1][C][u][q] = ps;
  }
  if (pml_h(x[v], p.n[v], p.P)) {
    const T ps = p.bh[v][x[v]] * p.pH[g.par][C][v][q] + p.ah[v][x[v]] * dv;
    tv += ps;
    if (own) p.pH[g.par ^ 1][C][v][q] = ps;
  }
  T h = p.H[g.par][C][q] - p.ch * (tu - tv);
  if (p.tf_on) {
    if (C == 1 && i >= p.lo[0] && i <= p.hi[0] - 1 && j >= p.lo[1] && j <= p.hi[1]) {
      if (k == p.lo[2] - 1) h += p.ch * g.einc(n, p.lo[2]);
      if (k == p.hi[2]) h -= p.ch * g.einc(n, p.hi[2]);
    }
    if (C == 2 && i >= p.lo[0] && i <= p.hi[0] - 1 && k >= p.lo[2] && k <= p.hi[2]) {
      if (j == p.lo[1] - 1) h -= p.ch * g.einc(n, k);
      if (j == p.hi[1]) h += p.ch * g.einc(n, k);
    }
  }
  if (own) p.H[g.par ^ 1][C][q] = h;
  return h;
}

// Adjoint: E*_V graded along axis U at node (i,j,k): E*/kappa + nu (nu new).
template <typename T, int V, int U>
__device__ T ge_adj(const G3<T> &g, int i, int j, int k) {
  const Step3D<T> &p = g.p;
  const int x[3] = {i, j, k};
  const T e = g.ld(p.E[g.par][V], i, j, k);
  if (!pml_e(x[U], p.n[U], p.P) || !g.inside(i, j, k)) return e;
  const T nu = p.be[U][x[U]] * p.pE[g.par][V][U][g.at(i, j, k)] + p.ae[U][x[U]] * e;
  return e * p.ike[U][x[U]] + nu;
}

// Adjoint: new H*_C at (i,j,k); graded values along its two axes to gu, gv.
template <typename T, int C>
__device__ void h_adj(const G3<T> &g, int i, int j, int k, bool own, T &gu, T &gv) {
  gu = gv = T(0);
  if (!g.hvalid(C, i, j, k)) return;
  constexpr int u = (C + 1) % 3, v = (C + 2) % 3;
  const Step3D<T> &p = g.p;
  const int x[3] = {i, j, k};
  int pu[3] = {i, j, k}, pv[3] = {i, j, k};
  pu[u] += 1;
  pv[v] += 1;
  const T du = ge_adj<T, v, u>(g, pu[0], pu[1], pu[2]) - ge_adj<T, v, u>(g, i, j, k);
  const T dv = ge_adj<T, u, v>(g, pv[0], pv[1], pv[2]) - ge_adj<T, u, v>(g, i, j, k);
  const long long q = g.at(i, j, k);
  const T h = p.H[g.par][C][q] - p.ch * (du - dv);
  gu = h * p.ikh[u][x[u]];
  gv = h * p.ikh[v][x[v]];
  if (pml_h(x[u], p.n[u], p.P)) {
    const T nu = p.bh[u][x[u]] * p.pH[g.par][C][u][q] + p.ah[u][x[u]] * h;
    gu += nu;
    if (own) p.pH[g.par ^ 1][C][u][q] = nu;
  }
  if (pml_h(x[v], p.n[v], p.P)) {
    const T nu = p.bh[v][x[v]] * p.pH[g.par][C][v][q] + p.ah[v][x[v]] * h;
    gv += nu;
    if (own) p.pH[g.par ^ 1][C][v][q] = nu;
  }
  if (own) p.H[g.par ^ 1][C][q] = h;
}

// E_C (or E*_C) update at an owned node given the curl bracket (in units of
// H: the difference of the (graded) H values, plus sources).
template <typename T, bool ADJ, int C>
__device__ void e_update(const G3<T> &g, int n, int i, int j, int k, T curl) {
  const Step3D<T> &p = g.p;
  const long long q = g.at(i, j, k);
  const int di[3] = {i - p.d0[0], j - p.d0[1], k - p.d0[2]};
  const int gi[3] = {i - p.g0[0], j - p.g0[1], k - p.g0[2]};
  const bool des = di[0] >= 0 && di[0] < p.dn[0] && di[1] >= 0 && di[1] < p.dn[1] && di[2] >= 0 && di[2] < p.dn[2];
  const bool gap = gi[0] >= 0 && gi[0] < p.gn[0] && gi[1] >= 0 && gi[1] < p.gn[1] && gi[2] >= 0 && gi[2] < p.gn[2];
  const int nd = p.dn[0] * p.dn[1] * p.dn[2];
  const int d = (di[2] * p.dn[1] + di[1]) * p.dn[0] + di[0];
  const int gg = (gi[2] * p.gn[1] + gi[1]) * p.gn[0] + gi[0];
  if (ADJ && gap) curl += p.asrc[((long long)n * p.ng + gg) * 3 + C];
  const T e0 = p.E[g.par][C][q];
  T e1;
  if (des && !gap) {
    const T r = p.rho[d];
    const T eps2 = p.A0 + r * p.A1;
    const T beta = p.B0 + r * p.B1;
    const T bs = beta * p.dt_ + p.Sg * r * (T(1) - r);
    const T inv = T(2) / (eps2 + bs);
    T *Jc = p.J + (long long)C * nd;
    const T Jo = Jc[d];
    const T dE = inv * (p.dtdx * curl - p.dthJ * Jo - bs * e0);
    e1 = e0 + dE;
    const T Jn = p.kp * Jo + beta * (e0 + e1);
    Jc[d] = Jn;
    if (!ADJ) {
      p.hist[((long long)n * 3 + C) * nd + d] = e1;
    } else {
      const T Em = p.hist[((long long)(n - 1) * 3 + C) * nd + d];
      const T gc = -(T(1) - p.rs) / (T(2) * (p.rs + r * (T(1) - p.rs)));
      const T gb = p.gsm * (T(1) - T(2) * r);
      p.grad[(long long)C * nd + d] += (double)(Em * (p.ga * dE + gb * (e0 + e1) + gc * (Jn + Jo)));
    }
  } else {
    e1 = e0 + (gap ? p.ce_g : p.ce_s) * curl;
    if (!ADJ && des) p.hist[((long long)n * 3 + C) * nd + d] = e1;
  }
  p.E[g.par ^ 1][C][q] = e1;
  if (!ADJ && gap) p.gapE[((long long)(n + 1) * p.ng + gg) * 3 + C] = (double)e1;
}

// Forward curl bracket of E_C at (i,j,k) from new H values hv0/hv1 (H_v at the
// node and one step back along u) and hu0/hu1 (H_u at the node and back
// along v), with the E-side CPML memory and the total-field corrections.
template <typename T, int C>
__device__ T curl_fwd(const G3<T> &g, int n, int i, int j, int k, T hv0, T hv1, T hu0, T hu1) {
  constexpr int u = (C + 1) % 3, v = (C + 2) % 3;
  const Step3D<T> &p = g.p;
  const int x[3] = {i, j, k};
  const long long q = g.at(i, j, k);
  const T du = hv0 - hv1, dv = hu0 - hu1;
  T tu = du * p.ike[u][x[u]], tv = dv * p.ike[v][x[v]];
  if (pml_e(x[u], p.n[u], p.P)) {
    const T ps = p.be[u][x[u]] * p.pE[g.par][C][u][q] + p.ae[u][x[u]] * du;
    tu += ps;
    p.pE[g.par ^ 1][C][u][q] = ps;
  }
  if (pml_e(x[v], p.n[v], p.P)) {
    const T ps = p.be[v][x[v]] * p.pE[g.par][C][v][q] + p.ae[v][x[v]] * dv;
    tv += ps;
    p.pE[g.par ^ 1][C][v][q] = ps;
  }
  T curl = tu - tv;
  if (p.tf_on) {
    if (C == 0 && i >= p.lo[0] && i <= p.hi[0] - 1 && j >= p.lo[1] && j <= p.hi[1]) {
      if (k == p.lo[2]) curl += g.hinc(n, p.lo[2] - 1);
      if (k == p.hi[2]) curl -= g.hinc(n, p.hi[2]);
    }
    if (C == 2 && j >= p.lo[1] && j <= p.hi[1] && k >= p.lo[2] && k <= p.hi[2] - 1) {
      if (i == p.lo[0]) curl -= g.hinc(n, k);
      if (i == p.hi[0]) curl += g.hinc(n, k);
    }
  }
  return curl;
}

// Adjoint: store the new nu of the owned E*_C node along both its axes.
template <typename T, int C>
__device__ void store_nu_e(const G3<T> &g, int i, int j, int k) {
  constexpr int u = (C + 1) % 3, v = (C + 2) % 3;
  const Step3D<T> &p = g.p;
  const int x[3] = {i, j, k};
  const long long q = g.at(i, j, k);
  const T e = p.E[g.par][C][q];
  if (pml_e(x[u], p.n[u], p.P)) p.pE[g.par ^ 1][C][u][q] = p.be[u][x[u]] * p.pE[g.par][C][u][q] + p.ae[u][x[u]] * e;
  if (pml_e(x[v], p.n[v], p.P)) p.pE[g.par ^ 1][C][v][q] = p.be[v][x[v]] * p.pE[g.par][C][v][q] + p.ae[v][x[v]] * e;
}

template <typename T, bool ADJ>
__global__ void __launch_bounds__(NT) step3d_general(const Step3D<T> p, const int n, const int par) {
  const int nbx = (p.n[0] + TX - 1) / TX, nby = (p.n[1] + TY - 1) / TY, nbz = (p.n[2] + R - 1) / R;
  int bx, by, bz;
  block_of(blockIdx.x, nbx, nby, nbz, bx, by, bz);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * R;
  if (block_is_bulk(p, i0, j0, k0)) return;
  const int i = i0 + (threadIdx.x % TX), j = j0 + (threadIdx.x / TX);
  if (i >= p.n[0] || j >= p.n[1]) return;
  const G3<T> g(p, par);
  if (!ADJ) {
    // new H: (i,j) column at k0-1..k0+R-1 for H_x, H_y; neighbours at j-1 / i-1
    T hx00[R + 1], hy00[R + 1], hx0m[R], hym0[R], hz00[R], hz0m[R], hzm0[R];
#pragma unroll
    for (int r = 0; r <= R; ++r) {
      const int k = k0 - 1 + r;
      const bool own = r >= 1 && k < p.n[2];
      hx00[r] = h_fwd<T, 0>(g, n, i, j, k, own);
      hy00[r] = h_fwd<T, 1>(g, n, i, j, k, own);
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = k0 + s;
      hx0m[s] = h_fwd<T, 0>(g, n, i, j - 1, k, false);
      hym0[s] = h_fwd<T, 1>(g, n, i - 1, j, k, false);
      hz00[s] = h_fwd<T, 2>(g, n, i, j, k, k < p.n[2]);
      hz0m[s] = h_fwd<T, 2>(g, n, i, j - 1, k, false);
      hzm0[s] = h_fwd<T, 2>(g, n, i - 1, j, k, false);
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = k0 + s;
      if (g.evalid(0, i, j, k)) e_update<T, false, 0>(g, n, i, j, k, curl_fwd<T, 0>(g, n, i, j, k, hz00[s], hz0m[s], hy00[s + 1], hy00[s]));
      if (g.evalid(1, i, j, k)) e_update<T, false, 1>(g, n, i, j, k, curl_fwd<T, 1>(g, n, i, j, k, hx00[s + 1], hx00[s], hz00[s], hzm0[s]));
      if (g.evalid(2, i, j, k)) e_update<T, false, 2>(g, n, i, j, k, curl_fwd<T, 2>(g, n, i, j, k, hy00[s + 1], hym0[s], hx00[s + 1], hx0m[s]));
    }
  } else {
    // graded new H*: gA_B = H*_A graded along axis B
    T hx_y[R + 1], hx_z[R + 1], hy_z[R + 1], hy_x[R + 1];
    T hx0m_y[R], hym0_x[R], hz_x[R], hz_y[R], hz0m_y[R], hzm0_x[R], tmp;
#pragma unroll
    for (int r = 0; r <= R; ++r) {
      const int k = k0 - 1 + r;
      const bool own = r >= 1 && k < p.n[2];
      h_adj<T, 0>(g, i, j, k, own, hx_y[r], hx_z[r]);   // H_x: u = y, v = z
      h_adj<T, 1>(g, i, j, k, own, hy_z[r], hy_x[r]);   // H_y: u = z, v = x
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = k0 + s;
      h_adj<T, 0>(g, i, j - 1, k, false, hx0m_y[s], tmp);
      h_adj<T, 1>(g, i - 1, j, k, false, tmp, hym0_x[s]);
      h_adj<T, 2>(g, i, j, k, k < p.n[2], hz_x[s], hz_y[s]);  // H_z: u = x, v = y
      h_adj<T, 2>(g, i, j - 1, k, false, tmp, hz0m_y[s]);
      h_adj<T, 2>(g, i - 1, j, k, false, hzm0_x[s], tmp);
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int k = k0 + s;
      if (k >= p.n[2]) continue;
      store_nu_e<T, 0>(g, i, j, k);
      store_nu_e<T, 1>(g, i, j, k);
      store_nu_e<T, 2>(g, i, j, k);
      // (curl H*)_x = d_y G_y(H*_z) - d_z G_z(H*_y), etc.
      if (g.evalid(0, i, j, k)) e_update<T, true, 0>(g, n, i, j, k, (hz_y[s] - hz0m_y[s]) - (hy_z[s + 1] - hy_z[s]));
      if (g.evalid(1, i, j, k)) e_update<T, true, 1>(g, n, i, j, k, (hx_z[s + 1] - hx_z[s]) - (hz_x[s] - hzm0_x[s]));
      if (g.evalid(2, i, j, k)) e_update<T, true, 2>(g, n, i, j, k, (hy_x[s + 1] - hym0_x[s]) - (hx_y[s + 1] - hx0m_y[s]));
    }
  }
}

}  // namespace

template <typename T>
void launch_step3d(const Step3D<T> &p, int n, int par, bool adjoint, hipStream_t s) {
  const int nbx = (p.n[0] + TX - 1) / TX, nby = (p.n[1] + TY - 1) / TY, nbz = (p.n[2] + R - 1) / R;
  const dim3 grid(nbx * nby * nbz);
  hipLaunchKernelGGL(step3d_bulk<T>, grid, dim3(NT), 0, s, p, par);
  if (adjoint)
    hipLaunchKernelGGL((step3d_general<T, true>), grid, dim3(NT), 0, s, p, n, par);
  else
    hipLaunchKernelGGL((step3d_general<T, false>), grid, dim3(NT), 0, s, p, n, par);
}

template void launch_step3d<float>(const Step3D<float> &, int, int, bool, hipStream_t);
template void launch_step3d<double>(const Step3D<double> &, int, int, bool, hipStream_t);

}  // namespace fdtd
