// fdtd_setup.hip -- small per-solve kernels around the time-stepping sweep:
// the incident-field line of the plane-wave injection, DFT phasors, objective
// weights, the objective reduction, the adjoint-source table and density
// validation.  None of them is on the per-step critical path.
#include "fdtd_internal.hpp"

namespace fdtd {
namespace {

constexpr int kRed = 256;  // threads of the single-block reductions

__device__ double block_sum(double v, double *sh) {
  // wavefront (64-lane) shuffle reduction, then across the 4 wavefronts
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
  return r;  // valid in thread 0
}

__device__ double block_max(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, sh[k]);
  return r;
}

// One-dimensional incident-field line (FP64) of the total-field/scattered-
// field injection: nodes 0..n1-1 along the propagation axis in the
// background medium, same dx and dt as the main grid; node 0 is driven by the
// waveform g, the far end is a graded absorber backed by a PEC node.  Emits
// einc[n][p] = E at node p, time n dt (n = 0..N) and hinc[n][p] = H between
// nodes p and p+1 at time (n+1/2) dt (n = 0..N-1), for p < L.
template <typename T>
__global__ void __launch_bounds__(1024) incident_line_kernel(const double *__restrict__ g, int N, int n1, int L,
                                                           const double *__restrict__ prof, double ch, double ce,
                                                           double cmu, double cep, double *__restrict__ sc,
                                                           T *__restrict__ einc, T *__restrict__ hinc) {
  double *e = sc, *h = sc + n1, *pe = sc + 2 * n1, *ph = sc + 3 * n1;
  const double *be = prof, *ae = prof + n1, *ike = prof + 2 * n1;
  const double *bh = prof + 3 * n1, *ah = prof + 4 * n1, *ikh = prof + 5 * n1;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int p = t; p < n1; p += nt) { e[p] = 0.0; h[p] = 0.0; pe[p] = 0.0; ph[p] = 0.0; }
  __syncthreads();
  if (t == 0) e[0] = g[0];
  __syncthreads();
  for (int p = t; p < L; p += nt) einc[p] = T(e[p]);
  for (int n = 0; n < N; ++n) {
    for (int p = t; p < n1 - 1; p += nt) {
      const double de = e[p + 1] - e[p];
      ph[p] = bh[p] * ph[p] + ah[p] * de;
      h[p] -= ch * (de * ikh[p] + ph[p]);
    }
    __syncthreads();
    for (int p = t; p < L; p += nt) hinc[(size_t)n * L + p] = T(h[p]);
    for (int p = t + 1; p < n1 - 1; p += nt) {
      const double dh = h[p] - h[p - 1];
      pe[p] = be[p] * pe[p] + ae[p] * dh;
      e[p] -= ce * (dh * ike[p] + pe[p]);
    }
    __syncthreads();
    if (t == 0) { e[0] = g[n + 1]; e[n1 - 1] = 0.0; }
    __syncthreads();
    for (int p = t; p < L; p += nt) einc[(size_t)(n + 1) * L + p] = T(e[p]);
  }
  (void)cmu; (void)cep;
}

__global__ void phasor_kernel(const double *__restrict__ f, int K, int N, double dt, double *__restrict__ ph) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)(N + 1) * K) return;
  const int n = (int)(idx / K), k = (int)(idx % K);
  double s, c;
  sincos(2.0 * M_PI * f[k] * (double)n * dt, &s, &c);
  ph[2 * idx] = c;
  ph[2 * idx + 1] = s;
}

// w_k = 1/|Ghat(w_k)|^2, Ghat = dt sum_{n=1..N} g(n dt) exp(-j w_k n dt); or 1.
__global__ void weights_kernel(const double *__restrict__ g, const double *__restrict__ f, int N, double dt,
                               int unit, double *__restrict__ w) {
  __shared__ double sh[16];
  const int k = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int n = 1 + threadIdx.x; n <= N; n += blockDim.x) {
    double s, c;
    sincos(2.0 * M_PI * f[k] * (double)n * dt, &s, &c);
    re += dt * g[n] * c;
    im -= dt * g[n] * s;
  }
  const double R = block_sum(re, sh);
  __syncthreads();
  const double I = block_sum(im, sh);
  if (threadIdx.x == 0) w[k] = unit ? 1.0 : 1.0 / (R * R + I * I);
}

// Running DFT of the gap monitors from their time series (one workgroup per
// frequency k and monitor m): dft[k][m] = dt sum_{n=1..N} E_m^n exp(-j w_k n dt).
__global__ void dft_kernel(const double *__restrict__ gapE, const double *__restrict__ ph, int K, int nmon, int N,
                           double dt, double *__restrict__ dft) {
  __shared__ double sh[16];
  const int k = blockIdx.x / nmon, m = blockIdx.x % nmon;
  double re = 0.0, im = 0.0;
  for (int n = 1 + threadIdx.x; n <= N; n += blockDim.x) {
    const double e = gapE[(size_t)n * nmon + m];
    re += e * ph[2 * ((size_t)n * K + k)];
    im -= e * ph[2 * ((size_t)n * K + k) + 1];
  }
  const double R = block_sum(re, sh);
  __syncthreads();
  const double I = block_sum(im, sh);
  if (threadIdx.x == 0) {
    dft[2 * ((size_t)k * nmon + m)] = dt * R;
    dft[2 * ((size_t)k * nmon + m) + 1] = dt * I;
  }
}

// F = sum_k w_k sum_m |dft[k][m]|^2, or te_scale * sum_n sum_m gapE[n][m]^2.
__global__ void objective_kernel(const double *__restrict__ dft, const double *__restrict__ w,
                                 const double *__restrict__ gapE, int K, int nmon, int N, int te,
                                 double te_scale, double *__restrict__ F) {
  __shared__ double sh[16];
  double acc = 0.0;
  if (!te) {
    for (int i = threadIdx.x; i < K * nmon; i += blockDim.x) {
      const double re = dft[2 * i], im = dft[2 * i + 1];
      acc += w[i / nmon] * (re * re + im * im);
    }
  } else {
    for (int64_t i = threadIdx.x; i < (int64_t)(N + 1) * nmon; i += blockDim.x) acc += gapE[i] * gapE[i];
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) F[0] = te ? te_scale * r : r;
}

// Scale S' of the adjoint source: 1 / (dx * max_m bound_m) with bound_m an
// upper bound of |dF/dE_m^n| over n, so that the stored table is O(1).
__global__ void adjoint_scale_kernel(const double *__restrict__ dft, const double *__restrict__ w,
                                     const double *__restrict__ gapE, int K, int nmon, int N, int te,
                                     double te_coef, double dt, double dx, double *__restrict__ scale) {
  __shared__ double sh[16];
  double mx = 0.0;
  if (!te) {
    for (int m = threadIdx.x; m < nmon; m += blockDim.x) {
      double b = 0.0;
      for (int k = 0; k < K; ++k) {
        const double re = dft[2 * (k * nmon + m)], im = dft[2 * (k * nmon + m) + 1];
        b += w[k] * sqrt(re * re + im * im);
      }
      mx = fmax(mx, 2.0 * dt * b);
    }
  } else {
    for (int64_t i = threadIdx.x; i < (int64_t)(N + 1) * nmon; i += blockDim.x) mx = fmax(mx, fabs(te_coef * gapE[i]));
  }
  const double r = block_max(mx, sh);
  if (threadIdx.x == 0) scale[0] = (r > 0.0 && isfinite(r)) ? 1.0 / (dx * r) : 1.0;
}

// table[n][m] = S' dx dF/dE_m^n, the adjoint source of step n folded with dx.
template <typename T>
__global__ void adjoint_source_kernel(const double *__restrict__ dft, const double *__restrict__ w,
                                      const double *__restrict__ ph, const double *__restrict__ gapE, int K,
                                      int nmon, int N, int te, double te_coef, double dt, double dx,
                                      const double *__restrict__ scale, T *__restrict__ table) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)(N + 1) * nmon) return;
  const int n = (int)(idx / nmon), m = (int)(idx % nmon);
  double s;
  if (!te) {
    s = 0.0;
    for (int k = 0; k < K; ++k) {
      const double re = dft[2 * (k * nmon + m)], im = dft[2 * (k * nmon + m) + 1];
      const double c = ph[2 * ((int64_t)n * K + k)], sn = ph[2 * ((int64_t)n * K + k) + 1];
      s += w[k] * (re * c - im * sn);
    }
    s *= 2.0 * dt;
  } else {
    s = te_coef * gapE[idx];
  }
  table[idx] = T(s * dx * scale[0]);
}

// dF/drho_d = (sum over the cell's edges of the folded sensitivity sums) / S';
// gap cells carry no design variable.  (gx0, gy0, gz0) is the gap box in
// design-box coordinates.
template <typename T>
__global__ void grad_finalize_kernel(const double *__restrict__ acc, const double *__restrict__ scale, int ncomp,
                                     int dnx, int dny, int dnz, int gx0, int gy0, int gz0, int gnx, int gny, int gnz,
                                     T *__restrict__ out) {
  const int64_t nd = (int64_t)dnx * dny * dnz;
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nd) return;
  const int x = (int)(d % dnx), y = (int)((d / dnx) % dny), z = (int)(d / ((int64_t)dnx * dny));
  const bool gap = x >= gx0 && x < gx0 + gnx && y >= gy0 && y < gy0 + gny && z >= gz0 && z < gz0 + gnz;
  double v = 0.0;
  if (!gap)
    for (int c = 0; c < ncomp; ++c) v += acc[c * nd + d];
  out[d] = T(v / scale[0]);
}

__global__ void fill_zero_kernel(uint32_t *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0u;
}

template <typename T>
__global__ void check_density_kernel(const T *__restrict__ rho, int64_t n, int *__restrict__ bad) {
  __shared__ double sh[16];
  double cnt = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const T r = rho[i];
    if (!(r >= T(0) && r <= T(1))) cnt += 1.0;
  }
  const double c = block_sum(cnt, sh);
  if (threadIdx.x == 0) bad[0] = (int)c;
}

// Watchdog of a solve: the largest |v| over n values (NaN counts as +inf),
// folded into *slot with an atomic max on the bit pattern (non-negative
// doubles order like their bits).  *slot must start at zero.
template <typename T>
__global__ void __launch_bounds__(256) watch_kernel(const T *__restrict__ p, size_t n,
                                                    unsigned long long *__restrict__ slot) {
  __shared__ double sh[4];
  double m = 0.0;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    double a = fabs((double)p[i]);
    if (!(a == a)) a = HUGE_VAL;
    m = fmax(m, a);
  }
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) atomicMax(slot, (unsigned long long)__double_as_longlong(r));
}

}  // namespace

void launch_watch(hipStream_t s, int precision, const void *p, size_t n, unsigned long long *slot) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (precision == 32)
    hipLaunchKernelGGL(watch_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float *)p, n, slot);
  else
    hipLaunchKernelGGL(watch_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double *)p, n, slot);
  FDTD_HIP(hipGetLastError());
}

void launch_incident_line(hipStream_t s, int precision, const double *g, int N, int n1, int L, const double *prof,
                          double ch, double ce, double cmu, double cep, double *scratch, void *einc, void *hinc) {
  if (precision == 32)
    hipLaunchKernelGGL(incident_line_kernel<float>, dim3(1), dim3(1024), 0, s, g, N, n1, L, prof, ch, ce, cmu, cep,
                       scratch, (float *)einc, (float *)hinc);
  else
    hipLaunchKernelGGL(incident_line_kernel<double>, dim3(1), dim3(1024), 0, s, g, N, n1, L, prof, ch, ce, cmu, cep,
                       scratch, (double *)einc, (double *)hinc);
  FDTD_HIP(hipGetLastError());
}

void launch_phasors(hipStream_t s, const double *freqs, int K, int N, double dt, double *phasor) {
  const int64_t n = (int64_t)(N + 1) * K;
  hipLaunchKernelGGL(phasor_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, freqs, K, N, dt, phasor);
  FDTD_HIP(hipGetLastError());
}

void launch_weights(hipStream_t s, const double *g, const double *freqs, int K, int N, double dt, int unit,
                    double *w) {
  hipLaunchKernelGGL(weights_kernel, dim3(K), dim3(kRed), 0, s, g, freqs, N, dt, unit, w);
  FDTD_HIP(hipGetLastError());
}

void launch_dft(hipStream_t s, const double *gapE, const double *phasor, int K, int nmon, int N, double dt,
                double *dft) {
  hipLaunchKernelGGL(dft_kernel, dim3((unsigned)(K * nmon)), dim3(kRed), 0, s, gapE, phasor, K, nmon, N, dt, dft);
  FDTD_HIP(hipGetLastError());
}

void launch_objective(hipStream_t s, const double *dft, const double *w, const double *gapE, int K, int nmon, int N,
                      int time_energy, double te_scale, double *F_out) {
  hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(kRed), 0, s, dft, w, gapE, K, nmon, N, time_energy, te_scale,
                     F_out);
  FDTD_HIP(hipGetLastError());
}

void launch_adjoint_source(hipStream_t s, int precision, const double *dft, const double *w, const double *phasor,
                           const double *gapE, int K, int nmon, int N, int time_energy, double te_coef, double dt,
                           double dx, double *scale_out, void *table) {
  hipLaunchKernelGGL(adjoint_scale_kernel, dim3(1), dim3(kRed), 0, s, dft, w, gapE, K, nmon, N, time_energy, te_coef,
                     dt, dx, scale_out);
  FDTD_HIP(hipGetLastError());
  const int64_t n = (int64_t)(N + 1) * nmon;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (precision == 32)
    hipLaunchKernelGGL(adjoint_source_kernel<float>, grid, dim3(256), 0, s, dft, w, phasor, gapE, K, nmon, N,
                       time_energy, te_coef, dt, dx, scale_out, (float *)table);
  else
    hipLaunchKernelGGL(adjoint_source_kernel<double>, grid, dim3(256), 0, s, dft, w, phasor, gapE, K, nmon, N,
                       time_energy, te_coef, dt, dx, scale_out, (double *)table);
  FDTD_HIP(hipGetLastError());
}

void launch_grad_finalize(hipStream_t s, int precision, const double *acc, const double *scale, int ncomp, int dnx,
                          int dny, int dnz, int gx0, int gy0, int gz0, int gnx, int gny, int gnz, void *out) {
  const int64_t nd = (int64_t)dnx * dny * dnz;
  const dim3 grid((unsigned)((nd + 255) / 256));
  if (precision == 32)
    hipLaunchKernelGGL(grad_finalize_kernel<float>, grid, dim3(256), 0, s, acc, scale, ncomp, dnx, dny, dnz, gx0, gy0,
                       gz0, gnx, gny, gnz, (float *)out);
  else
    hipLaunchKernelGGL(grad_finalize_kernel<double>, grid, dim3(256), 0, s, acc, scale, ncomp, dnx, dny, dnz, gx0,
                       gy0, gz0, gnx, gny, gnz, (double *)out);
  FDTD_HIP(hipGetLastError());
}

void launch_fill_zero(hipStream_t s, void *p, size_t bytes) {
  const size_t n = bytes / 4;
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, n);
  FDTD_HIP(hipGetLastError());
}

void launch_check_density(hipStream_t s, int precision, const void *rho, int64_t n, int *bad) {
  if (precision == 32)
    hipLaunchKernelGGL(check_density_kernel<float>, dim3(1), dim3(1024), 0, s, (const float *)rho, n, bad);
  else
    hipLaunchKernelGGL(check_density_kernel<double>, dim3(1), dim3(1024), 0, s, (const double *)rho, n, bad);
  FDTD_HIP(hipGetLastError());
}

void launch_copy_density(hipStream_t s, int precision, const void *src, void *dst, int64_t n) {
  FDTD_HIP(hipMemcpyAsync(dst, src, (size_t)n * (precision == 32 ? 4 : 8), hipMemcpyDeviceToDevice, s));
}

}  // namespace fdtd
