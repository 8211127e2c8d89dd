// fdtd_2d.hip -- fused time step of the 2D TMz Drude-FDTD solve and of its
// adjoint, one launch per time step.
//
// Per step (Sec. 3.2 staggering: E, J at integer steps, H at half steps):
//   H^{n+1/2} = H^{n-1/2} - dt/mu0 curl E^n                 (eq. (10c), CPML, TFSF)
//   E^{n+1}   = E^n + dE,  dE = 2/D [dt curl H^{n+1/2} - dt (1+kp)/2 J^n - (beta+sigma) dt E^n]
//   J^{n+1}   = kp J^n + beta (E^{n+1} + E^n)               (eqs. (10a-b), trapezoidal ADE)
// with the per-edge coefficients of eqs. (4)-(5) evaluated in registers from
// rho (D = 2 eps0 eps_inf_i + (beta_i + sigma_i) dt).  The adjoint step
// (eq. (20)) is the same update on (E*, H*, J*) driven by the gap source, with
// the absorber replaced by its exact transpose: the grading 1/kappa and the
// recursive memory act on the field before the difference, not after it.
// The adjoint also accumulates the sensitivity of eq. (25), folded with the
// chain rule of eq. (27) into one FP64 sum per design edge:
//   g_i += E_i^m [ga dE*_i + gb (E*_i^{m-1/2} + E*_i^{m+1/2}) + gc (J*_i^{m-1/2} + J*_i^{m+1/2})].
//
// Layout: a workgroup owns a 64 x 16 tile of E nodes.  It stages E (or the
// graded E*) of the tile plus a one-node halo in LDS, computes H for the tile
// plus the low-side halo row/column (so no other tile's new H is needed),
// writes the tile's own H, then updates E.  All arrays that a halo reads come
// in two copies so the step needs no grid-wide synchronisation.
#include "fdtd_2d.hpp"

namespace fdtd {
namespace {

constexpr int TX = 64;
constexpr int TY = 16;
constexpr int NT = 256;

__device__ __forceinline__ bool pml_e(int i, int n, int P) { return P > 0 && (i < P || i > n - 1 - P); }
__device__ __forceinline__ bool pml_h(int i, int n, int P) { return P > 0 && (i < P || i >= n - 1 - P); }

template <typename T, bool ADJ>
__global__ void __launch_bounds__(NT) step2d_kernel(Step2D<T> p, int n, int par) {
  __shared__ T sEx[TY + 2][TX + 2];             // E (forward) / x-graded E* (adjoint)
  __shared__ T sEy[ADJ ? TY + 2 : 1][TX + 2];   // y-graded E* (adjoint)
  __shared__ T sHx[TY + 1][TX];                 // new Hx (forward) / graded Hx* (adjoint), rows j0-1 ..
  __shared__ T sHy[TY][TX + 1];                 // new Hy / graded Hy*, columns i0-1 ..
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY, tid = threadIdx.x;
  const int nx = p.nx, ny = p.ny, P = p.P, pitch = p.pitch;
  const int wr = par ^ 1;
  const T *__restrict__ ez = p.ez[par];

  // ---- stage E of the tile plus a one-node halo
  for (int k = tid; k < (TY + 2) * (TX + 2); k += NT) {
    const int ly = k / (TX + 2), lx = k - ly * (TX + 2);
    const int i = i0 - 1 + lx, j = j0 - 1 + ly;
    const bool in = i >= 0 && i < nx && j >= 0 && j < ny;
    const size_t q = (size_t)j * pitch + i;
    const T e = in ? ez[q] : T(0);
    if (!ADJ) {
      sEx[ly][lx] = e;
    } else {
      T gx = e, gy = e;
      if (in) {
        const bool own = lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
        if (pml_e(i, nx, P)) {
          const T nu = p.bxe[i] * p.pex[par][q] + p.axe[i] * e;
          gx = e * p.ikxe[i] + nu;
          if (own) p.pex[wr][q] = nu;
        }
        if (pml_e(j, ny, P)) {
          const T nu = p.bye[j] * p.pey[par][q] + p.aye[j] * e;
          gy = e * p.ikye[j] + nu;
          if (own) p.pey[wr][q] = nu;
        }
      }
      sEx[ly][lx] = gx;
      sEy[ly][lx] = gy;
    }
  }
  __syncthreads();

  // ---- Hx at (i, j+1/2): rows j0-1 .. j0+TY-1 (row j0-1 is the halo)
  for (int k = tid; k < (TY + 1) * TX; k += NT) {
    const int ly = k / TX, lx = k - ly * TX;
    const int i = i0 + lx, j = j0 - 1 + ly;
    T v = T(0);
    if (i >= 1 && i <= nx - 2 && j >= 0 && j <= ny - 2) {
      const size_t q = (size_t)j * pitch + i;
      const bool own = ly >= 1;
      if (!ADJ) {
        const T dE = sEx[ly + 1][lx + 1] - sEx[ly][lx + 1];
        T h = p.hx[par][q];
        if (pml_h(j, ny, P)) {
          const T ps = p.byh[j] * p.phx[par][q] + p.ayh[j] * dE;
          h -= p.chx * (dE * p.ikyh[j] + ps);
          if (own) p.phx[wr][q] = ps;
        } else {
          h -= p.chx * dE;
        }
        if (p.tf_on && i >= p.ia && i <= p.ib) {
          if (j == p.ja - 1) h += p.chx * p.einc[(size_t)n * p.L + (p.ja - p.jref)];
          if (j == p.jb) h -= p.chx * p.einc[(size_t)n * p.L + (p.jb - p.jref)];
        }
        if (own) p.hx[wr][q] = h;
        v = h;
      } else {
        const T dG = sEy[ly + 1][lx + 1] - sEy[ly][lx + 1];
        const T h = p.hx[par][q] - p.chx * dG;
        if (own) p.hx[wr][q] = h;
        v = h;
        if (pml_h(j, ny, P)) {
          const T nu = p.byh[j] * p.phx[par][q] + p.ayh[j] * h;
          v = h * p.ikyh[j] + nu;
          if (own) p.phx[wr][q] = nu;
        }
      }
    }
    sHx[ly][lx] = v;
  }

  // ---- Hy at (i+1/2, j): columns i0-1 .. i0+TX-1 (column i0-1 is the halo)
  for (int k = tid; k < TY * (TX + 1); k += NT) {
    const int ly = k / (TX + 1), lx = k - ly * (TX + 1);
    const int i = i0 - 1 + lx, j = j0 + ly;
    T v = T(0);
    if (i >= 0 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
      const size_t q = (size_t)j * pitch + i;
      const bool own = lx >= 1;
      if (!ADJ) {
        const T dE = sEx[ly + 1][lx + 1] - sEx[ly + 1][lx];
        T h = p.hy[par][q];
        if (pml_h(i, nx, P)) {
          const T ps = p.bxh[i] * p.phy[par][q] + p.axh[i] * dE;
          h += p.chx * (dE * p.ikxh[i] + ps);
          if (own) p.phy[wr][q] = ps;
        } else {
          h += p.chx * dE;
        }
        if (p.tf_on && j >= p.ja && j <= p.jb) {
          if (i == p.ia - 1) h -= p.chx * p.einc[(size_t)n * p.L + (j - p.jref)];
          if (i == p.ib) h += p.chx * p.einc[(size_t)n * p.L + (j - p.jref)];
        }
        if (own) p.hy[wr][q] = h;
        v = h;
      } else {
        const T dG = sEx[ly + 1][lx + 1] - sEx[ly + 1][lx];
        const T h = p.hy[par][q] + p.chx * dG;
        if (own) p.hy[wr][q] = h;
        v = h;
        if (pml_h(i, nx, P)) {
          const T nu = p.bxh[i] * p.phy[par][q] + p.axh[i] * h;
          v = h * p.ikxh[i] + nu;
          if (own) p.phy[wr][q] = nu;
        }
      }
    }
    sHy[ly][lx] = v;
  }
  __syncthreads();

  // ---- E (and J) at the tile's nodes
  const int nd = p.dnx * p.dny;
  for (int k = tid; k < TY * TX; k += NT) {
    const int ly = k / TX, lx = k - ly * TX;
    const int i = i0 + lx, j = j0 + ly;
    if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2) continue;
    const size_t q = (size_t)j * pitch + i;
    const T dHy = sHy[ly][lx + 1] - sHy[ly][lx];
    const T dHx = sHx[ly + 1][lx] - sHx[ly][lx];
    T curl;
    if (!ADJ) {
      T cx = dHy, cy = dHx;
      if (pml_e(i, nx, P)) {
        const T ps = p.bxe[i] * p.pex[par][q] + p.axe[i] * dHy;
        cx = dHy * p.ikxe[i] + ps;
        p.pex[wr][q] = ps;
      }
      if (pml_e(j, ny, P)) {
        const T ps = p.bye[j] * p.pey[par][q] + p.aye[j] * dHx;
        cy = dHx * p.ikye[j] + ps;
        p.pey[wr][q] = ps;
      }
      curl = cx - cy;
      if (p.tf_on && i >= p.ia && i <= p.ib) {
        if (j == p.ja) curl += p.hinc[(size_t)n * p.L + (p.ja - 1 - p.jref)];
        if (j == p.jb) curl -= p.hinc[(size_t)n * p.L + (p.jb - p.jref)];
      }
    } else {
      curl = dHy - dHx;
    }
    const int gi = i - p.gx0, gj = j - p.gy0;
    const bool gap = gi >= 0 && gi < p.gnx && gj >= 0 && gj < p.gny;
    const int g = gj * p.gnx + gi;
    if (ADJ && gap) curl += p.asrc[(size_t)n * p.ng + g];
    const int di = i - p.dx0, dj = j - p.dy0;
    const bool des = di >= 0 && di < p.dnx && dj >= 0 && dj < p.dny;
    const int d = dj * p.dnx + di;
    const T e0 = ez[q];
    T e1;
    if (des && !gap) {
      const T r = p.rho[d];
      const T eps2 = p.A0 + r * p.A1;
      const T beta = p.B0 + r * p.B1;
      const T bs = beta * p.dt_ + p.Sg * r * (T(1) - r);
      const T inv = T(2) / (eps2 + bs);
      const T Jo = p.J[d];
      const T dE = inv * (p.dtdx * curl - p.dthJ * Jo - bs * e0);
      e1 = e0 + dE;
      const T Jn = p.kp * Jo + beta * (e0 + e1);
      p.J[d] = Jn;
      if (!ADJ) {
        p.hist[(size_t)n * nd + d] = e1;
      } else {
        const T Em = p.hist[(size_t)(n - 1) * nd + d];
        const T gc = -(T(1) - p.rs) / (T(2) * (p.rs + r * (T(1) - p.rs)));
        const T gb = p.gsm * (T(1) - T(2) * r);
        p.grad[d] += (double)(Em * (p.ga * dE + gb * (e0 + e1) + gc * (Jn + Jo)));
      }
    } else {
      e1 = e0 + (gap ? p.ce_g : p.ce_s) * curl;
      if (!ADJ && des) p.hist[(size_t)n * nd + d] = e1;
    }
    p.ez[wr][q] = e1;
    if (!ADJ && gap) {
      const double ev = (double)e1;
      p.gapE[(size_t)(n + 1) * p.ng + g] = ev;
      const double *ph = p.phasor + (size_t)(n + 1) * p.K * 2;
      for (int kk = 0; kk < p.K; ++kk) {
        double *a = p.dft + ((size_t)kk * p.ng + g) * 2;
        a[0] += p.dt * ev * ph[2 * kk];
        a[1] -= p.dt * ev * ph[2 * kk + 1];
      }
    }
  }
}

}  // namespace

template <typename T>
void launch_step2d(const Step2D<T> &p, int n, int par, bool adjoint, hipStream_t s) {
  const dim3 grid((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY);
  if (adjoint)
    hipLaunchKernelGGL((step2d_kernel<T, true>), grid, dim3(NT), 0, s, p, n, par);
  else
    hipLaunchKernelGGL((step2d_kernel<T, false>), grid, dim3(NT), 0, s, p, n, par);
}

template void launch_step2d<float>(const Step2D<float> &, int, int, bool, hipStream_t);
template void launch_step2d<double>(const Step2D<double> &, int, int, bool, hipStream_t);

}  // namespace fdtd
