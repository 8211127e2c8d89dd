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
// One thread per node (i, j): it updates H_z(i, j), E_x(i, j) and E_y(i, j),
// recomputing the new H_z of its lower and left neighbours from the read
// copy (every array a halo reads has a read and a write copy).  Workgroups
// of 64 x 4 nodes.  This polarization's workloads are small (the paper's 2D
// designs), so the step is a plain per-step kernel without temporal
// blocking.
//
// Design layout (per edge): the design box of dnx x dny cells holds its E_x
// edges [dny+1][dnx] (density indices 0 .. ndx-1) followed by its E_y edges
// [dny][dnx+1]; the gap box's edges likewise give the monitor order.
#include "fdtd_2d.hpp"

namespace fdtd {
namespace {

constexpr int TEX = 64, TEY = 4;

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
template <typename T, bool ADJ>
__device__ __forceinline__ T te_e(const Step2D<T> &p, int n, int comp, int i, int j, T e0, T curl) {
  const int d = te_design(p, comp, i, j), g = te_gap(p, comp, i, j);
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

// Forward.  Copy 0 read, copy 1 written.  Memories: pex = H_z's x
// difference, pey = H_z's y difference, phx = E_x's (y), phy = E_y's (x).
template <typename T>
__global__ void __launch_bounds__(TEX * TEY) step_te_fwd(const Step2D<T> p, int n) {
  const int i = blockIdx.x * TEX + (threadIdx.x % TEX), j = blockIdx.y * TEY + (threadIdx.x / TEX);
  const int nx = p.nx, ny = p.ny, P = p.P;
  if (i >= nx || j >= ny) return;
  const size_t pitch = p.pitch, q = (size_t)j * pitch + i;
  const T *__restrict__ Ex = p.ez[0];
  const T *__restrict__ Ey = p.hx[0];
  const T *__restrict__ Hz = p.hy[0];
  const T *__restrict__ mhx = p.pex[0];
  const T *__restrict__ mhy = p.pey[0];
  const T *__restrict__ mex = p.phx[0];
  const T *__restrict__ mey = p.phy[0];
  const T *ei = p.einc + (size_t)n * p.L, *hi = p.hinc + (size_t)n * p.L;
  // new H_z at cell (a, b) (a <= nx-2, b <= ny-2) and its memories
  auto hz_new = [&](int a, int b, T &sx, T &sy) {
    const size_t r = (size_t)b * pitch + a;
    const T dEy = Ey[r + 1] - Ey[r];
    const T dEx = Ex[r + pitch] - Ex[r];
    T tx = dEy * p.ikxh[a], ty = dEx * p.ikyh[b];
    sx = T(0);
    sy = T(0);
    if (te_pml_h(a, nx, P)) { sx = p.bxh[a] * mhx[r] + p.axh[a] * dEy; tx += sx; }
    if (te_pml_h(b, ny, P)) { sy = p.byh[b] * mhy[r] + p.ayh[b] * dEx; ty += sy; }
    T h = Hz[r] - p.chx * (tx - ty);
    // the H_z rows just outside the box read E_x on its lower and upper lines
    if (p.tf_on && a >= p.ia && a <= p.ib - 1) {
      if (b == p.ja - 1) h -= p.chx * ei[p.ja - p.jref];
      if (b == p.jb) h += p.chx * ei[p.jb - p.jref];
    }
    return h;
  };
  const bool hin = i <= nx - 2 && j <= ny - 2;
  T h00 = T(0), sx, sy;
  if (hin) {
    h00 = hz_new(i, j, sx, sy);
    p.hy[1][q] = h00;
    if (te_pml_h(i, nx, P)) p.pex[1][q] = sx;
    if (te_pml_h(j, ny, P)) p.pey[1][q] = sy;
  }
  // E_x(i, j): curl = dH_z/dy; incident H_z = -(the line's transverse H)
  if (i <= nx - 2 && j >= 1 && j <= ny - 2) {
    T t0, t1;
    const T d = h00 - hz_new(i, j - 1, t0, t1);
    T c = d * p.ikye[j];
    if (te_pml_e(j, ny, P)) {
      const T s = p.bye[j] * mex[q] + p.aye[j] * d;
      p.phx[1][q] = s;
      c += s;
    }
    if (p.tf_on && i >= p.ia && i <= p.ib - 1) {
      if (j == p.ja) c += hi[p.ja - 1 - p.jref];
      if (j == p.jb) c -= hi[p.jb - p.jref];
    }
    p.ez[1][q] = te_e<T, false>(p, n, 0, i, j, Ex[q], c);
  }
  // E_y(i, j): curl = -dH_z/dx
  if (i >= 1 && i <= nx - 2 && j <= ny - 2) {
    T t0, t1;
    const T d = h00 - hz_new(i - 1, j, t0, t1);
    T g = d * p.ikxe[i];
    if (te_pml_e(i, nx, P)) {
      const T s = p.bxe[i] * mey[q] + p.axe[i] * d;
      p.phy[1][q] = s;
      g += s;
    }
    T c = -g;
    if (p.tf_on && j >= p.ja && j <= p.jb - 1) {
      if (i == p.ia) c -= hi[j - p.jref];
      if (i == p.ib) c += hi[j - p.jref];
    }
    p.hx[1][q] = te_e<T, false>(p, n, 1, i, j, Ey[q], c);
  }
}

// Adjoint step m = n: copy 0 holds E*^{m+1/2}, H_z*^{m+1} and the memories
// (nu), copy 1 receives E*^{m-1/2}, H_z*^m.
template <typename T>
__global__ void __launch_bounds__(TEX * TEY) step_te_adj(const Step2D<T> p, int n) {
  const int i = blockIdx.x * TEX + (threadIdx.x % TEX), j = blockIdx.y * TEY + (threadIdx.x / TEX);
  const int nx = p.nx, ny = p.ny, P = p.P;
  if (i >= nx || j >= ny) return;
  const size_t pitch = p.pitch, q = (size_t)j * pitch + i;
  const T *__restrict__ Ex = p.ez[0];
  const T *__restrict__ Ey = p.hx[0];
  const T *__restrict__ Hz = p.hy[0];
  const T *__restrict__ mhx = p.pex[0];
  const T *__restrict__ mhy = p.pey[0];
  const T *__restrict__ mex = p.phx[0];
  const T *__restrict__ mey = p.phy[0];
  // E* graded by the E update's absorber profile (new memory from E* itself);
  // zero on the walls and the unused slots
  auto gx = [&](int a, int b) {
    if (a > nx - 2 || b < 1 || b > ny - 2) return T(0);
    const size_t r = (size_t)b * pitch + a;
    const T e = Ex[r];
    return e * p.ikye[b] + (te_pml_e(b, ny, P) ? p.bye[b] * mex[r] + p.aye[b] * e : T(0));
  };
  auto gy = [&](int a, int b) {
    if (a < 1 || a > nx - 2 || b > ny - 2) return T(0);
    const size_t r = (size_t)b * pitch + a;
    const T e = Ey[r];
    return e * p.ikxe[a] + (te_pml_e(a, nx, P) ? p.bxe[a] * mey[r] + p.axe[a] * e : T(0));
  };
  // new H_z* at cell (a, b): the forward curl-E update on the graded E*
  auto hz_new = [&](int a, int b) {
    const size_t r = (size_t)b * pitch + a;
    return Hz[r] - p.chx * ((gy(a + 1, b) - gy(a, b)) - (gx(a, b + 1) - gx(a, b)));
  };
  // H_z* graded by the H update's profile along x (for dH/dx) and y (dH/dy)
  auto hxg = [&](int a, int b, T h) {
    return h * p.ikxh[a] + (te_pml_h(a, nx, P) ? p.bxh[a] * mhx[(size_t)b * pitch + a] + p.axh[a] * h : T(0));
  };
  auto hyg = [&](int a, int b, T h) {
    return h * p.ikyh[b] + (te_pml_h(b, ny, P) ? p.byh[b] * mhy[(size_t)b * pitch + a] + p.ayh[b] * h : T(0));
  };
  // own memories of E* (driven by E* of copy 0)
  if (i <= nx - 2 && j >= 1 && j <= ny - 2 && te_pml_e(j, ny, P)) p.phx[1][q] = p.bye[j] * mex[q] + p.aye[j] * Ex[q];
  if (i >= 1 && i <= nx - 2 && j <= ny - 2 && te_pml_e(i, nx, P)) p.phy[1][q] = p.bxe[i] * mey[q] + p.axe[i] * Ey[q];
  T h00 = T(0);
  if (i <= nx - 2 && j <= ny - 2) {
    h00 = hz_new(i, j);
    p.hy[1][q] = h00;
    if (te_pml_h(i, nx, P)) p.pex[1][q] = p.bxh[i] * mhx[q] + p.axh[i] * h00;
    if (te_pml_h(j, ny, P)) p.pey[1][q] = p.byh[j] * mhy[q] + p.ayh[j] * h00;
  }
  if (i <= nx - 2 && j >= 1 && j <= ny - 2) {
    const T c = hyg(i, j, h00) - hyg(i, j - 1, hz_new(i, j - 1));
    p.ez[1][q] = te_e<T, true>(p, n, 0, i, j, Ex[q], c);
  }
  if (i >= 1 && i <= nx - 2 && j <= ny - 2) {
    const T c = -(hxg(i, j, h00) - hxg(i - 1, j, hz_new(i - 1, j)));
    p.hx[1][q] = te_e<T, true>(p, n, 1, i, j, Ey[q], c);
  }
}

}  // namespace

template <typename T>
void launch_step_te(const Step2D<T> &p, int n, bool adjoint, hipStream_t s) {
  const dim3 grid((unsigned)((p.nx + TEX - 1) / TEX), (unsigned)((p.ny + TEY - 1) / TEY));
  if (adjoint) hipLaunchKernelGGL(step_te_adj<T>, grid, dim3(TEX * TEY), 0, s, p, n);
  else hipLaunchKernelGGL(step_te_fwd<T>, grid, dim3(TEX * TEY), 0, s, p, n);
}

template void launch_step_te<float>(const Step2D<float> &, int, bool, hipStream_t);
template void launch_step_te<double>(const Step2D<double> &, int, bool, hipStream_t);

}  // namespace fdtd
