// fdtd_design.hip -- per-element kernels of the design-update loop: the
// open-close density filter of eq. (26) with its transposed Jacobian for the
// chain rule of eq. (27), one step of the method of moving asymptotes for a
// box-constrained objective (with the sums of its globally convergent
// variant), and the non-discreteness / optimality statistics.
//
// Sums are deterministic: every reduction writes one FP64 partial per
// workgroup (wavefront shuffles, then the four wavefronts in order) and a
// single workgroup adds the partials in a fixed order.
#include <cmath>
#include <string>
#include <vector>

#include "fdtd_design.h"
#include "fdtd_internal.hpp"

using namespace fdtd;

namespace {

thread_local std::string g_err;

constexpr int BS = 256;  // threads per workgroup (4 wavefronts)

template <typename F>
fdtd_status dguard(F &&f) {
  try {
    f();
    return FDTD_OK;
  } catch (const Error &e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host out of memory";
    return FDTD_ENOMEM;
  }
}

// ---------------------------------------------------------------- reductions
// Sum of v over the workgroup, returned to thread 0 (fixed order).
__device__ __forceinline__ double block_sum(double v, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / 64; ++k) s += lds[k];
  __syncthreads();
  return s;
}

// out[q] = sum over the nb partials part[b * NQ + q] (one workgroup).
template <int NQ>
__global__ void __launch_bounds__(BS) finish_kernel(const double *part, int nb, double *out) {
  __shared__ double lds[BS / 64];
  for (int q = 0; q < NQ; ++q) {
    double v = 0;
    for (int b = threadIdx.x; b < nb; b += BS) v += part[(size_t)b * NQ + q];
    const double s = block_sum(v, lds);
    if (threadIdx.x == 0) out[q] = s;
  }
}

int nblocks(int64_t n) { return (int)((n + BS - 1) / BS); }

template <int NQ>
void finish(hipStream_t s, DevBuf &part, int nb, DevBuf &res, double *host) {
  hipLaunchKernelGGL(finish_kernel<NQ>, dim3(1), dim3(BS), 0, s, part.as<double>(), nb, res.as<double>());
  FDTD_HIP(hipGetLastError());
  FDTD_HIP(hipMemcpyAsync(host, res.p, NQ * sizeof(double), hipMemcpyDeviceToHost, s));
  FDTD_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- filter
// Cell coordinates of linear index i in an nx x ny x nz box (x fastest).
__device__ __forceinline__ void coords(int64_t i, int nx, int ny, int &ix, int &iy, int &iz) {
  ix = (int)(i % nx);
  iy = (int)((i / nx) % ny);
  iz = (int)(i / ((int64_t)nx * ny));
}

// 1 / sum_j w_ij over the box (the weights are symmetric: w_ij = w_ji).
__global__ void __launch_bounds__(BS) winv_kernel(double *winv, int nx, int ny, int nz, double r, int R, int Rz) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= (int64_t)nx * ny * nz) return;
  int ix, iy, iz;
  coords(i, nx, ny, ix, iy, iz);
  double s = 0;
  for (int dz = -Rz; dz <= Rz; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
        if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
        const double w = r - sqrt((double)(dx * dx + dy * dy + dz * dz));
        if (w > 0) s += w;
      }
  winv[i] = 1.0 / s;
}

// One fW-mean stage: e_i = f^-1(sum_j w_ij f(u_j) * winv_i), f(u) = 1/(u+alpha);
// erosion (dual = 0): u = x, y = e; dilation (dual = 1): u = 1-x, y = 1-e.
template <typename TI, typename TO>
__global__ void __launch_bounds__(BS) stage_kernel(const TI *__restrict__ x, TO *__restrict__ y,
                                                  const double *__restrict__ winv, int nx, int ny, int nz, double r,
                                                  int R, int Rz, double alpha, int dual) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= (int64_t)nx * ny * nz) return;
  int ix, iy, iz;
  coords(i, nx, ny, ix, iy, iz);
  double s = 0;
  for (int dz = -Rz; dz <= Rz; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
        if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
        const double w = r - sqrt((double)(dx * dx + dy * dy + dz * dz));
        if (w <= 0) continue;
        const double xj = (double)x[((int64_t)jz * ny + jy) * nx + jx];
        const double u = dual ? 1.0 - xj : xj;
        s += w / (u + alpha);
      }
  const double e = 1.0 / (s * winv[i]) - alpha;
  // an fW-mean of values in [0,1] lies in [0,1]; clamp off the rounding
  // (all-void or all-metal neighbourhoods land within an ulp of the bounds)
  y[i] = (TO)fmin(fmax(dual ? 1.0 - e : e, 0.0), 1.0);
}

// Transpose of one stage at input x, output y: with e = (dual ? 1-y : y),
// u = (dual ? 1-x : x): h_i = gy_i winv_i (e_i+alpha)^2 and
// gx_j = (u_j+alpha)^-2 sum_i w_ij h_i.  (The two sign flips of the dual
// stage cancel.)
template <typename TG, typename TY>
__global__ void __launch_bounds__(BS) stage_h_kernel(const TG *__restrict__ gy, const TY *__restrict__ y,
                                                    const double *__restrict__ winv, int64_t n, double alpha, int dual,
                                                    double *__restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const double yi = (double)y[i];
  const double e = dual ? 1.0 - yi : yi;
  h[i] = (double)gy[i] * winv[i] * (e + alpha) * (e + alpha);
}

template <typename TX, typename TO>
__global__ void __launch_bounds__(BS) stage_gather_kernel(const double *__restrict__ h, const TX *__restrict__ x,
                                                         TO *__restrict__ gx, int nx, int ny, int nz, double r, int R,
                                                         int Rz, double alpha, int dual) {
  const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (j >= (int64_t)nx * ny * nz) return;
  int jx, jy, jz;
  coords(j, nx, ny, jx, jy, jz);
  double s = 0;
  for (int dz = -Rz; dz <= Rz; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int ix = jx + dx, iy = jy + dy, iz = jz + dz;
        if (ix < 0 || ix >= nx || iy < 0 || iy >= ny || iz < 0 || iz >= nz) continue;
        const double w = r - sqrt((double)(dx * dx + dy * dy + dz * dz));
        if (w <= 0) continue;
        s += w * h[((int64_t)iz * ny + iy) * nx + ix];
      }
  const double xj = (double)x[j];
  const double u = dual ? 1.0 - xj : xj;
  gx[j] = (TO)(s / ((u + alpha) * (u + alpha)));
}

// ---------------------------------------------------------------- MMA
struct MmaArgs {
  double xmin, xmax, move, asyinit, asyincr, asydecr;
};

// Asymptotes and move limits of an outer iteration (k = accepted iterations
// so far); partial sums of |df0| for the initial curvature weight.
template <typename T>
__global__ void __launch_bounds__(BS) mma_begin_kernel(const T *__restrict__ xin, const T *__restrict__ dfin, int64_t n,
                                                      int k, MmaArgs a, double *__restrict__ x, double *__restrict__ df,
                                                      const double *__restrict__ xo1, const double *__restrict__ xo2,
                                                      double *__restrict__ L, double *__restrict__ U,
                                                      double *__restrict__ lo, double *__restrict__ hi,
                                                      double *__restrict__ part) {
  __shared__ double lds[BS / 64];
  const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
  double v = 0;
  if (j < n) {
    const double xj = (double)xin[j], dj = (double)dfin[j], dx = a.xmax - a.xmin;
    double l, u;
    if (k < 2) {
      l = xj - a.asyinit * dx;
      u = xj + a.asyinit * dx;
    } else {
      const double s = (xj - xo1[j]) * (xo1[j] - xo2[j]);
      const double g = s < 0 ? a.asydecr : (s > 0 ? a.asyincr : 1.0);
      l = xj - g * (xo1[j] - L[j]);
      u = xj + g * (U[j] - xo1[j]);
      l = fmin(fmax(l, xj - 10.0 * dx), xj - 0.01 * dx);
      u = fmax(fmin(u, xj + 10.0 * dx), xj + 0.01 * dx);
    }
    x[j] = xj;
    df[j] = dj;
    L[j] = l;
    U[j] = u;
    lo[j] = fmax(fmax(a.xmin, l + 0.1 * (xj - l)), xj - a.move * dx);
    hi[j] = fmin(fmin(a.xmax, u - 0.1 * (u - xj)), xj + a.move * dx);
    v = fabs(dj) * dx;
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Minimizer of the separable approximation with curvature weight rho:
// p = (U-x)^2 (1.001 g+ + 0.001 g- + rho/dx), q = (x-L)^2 (0.001 g+ + 1.001 g- + rho/dx),
// x* = clamp((sqrt(p) L + sqrt(q) U) / (sqrt(p) + sqrt(q)), lo, hi); partial sums
// of the change of p/(U-.) + q/(.-L) from x to x* (formed per element as
// (x*-x) [p/((U-x*)(U-x)) - q/((x*-L)(x-L))], so large rho does not cancel)
// and of the distance measure.
template <typename T>
__global__ void __launch_bounds__(BS) mma_solve_kernel(const double *__restrict__ x, const double *__restrict__ df,
                                                      const double *__restrict__ L, const double *__restrict__ U,
                                                      const double *__restrict__ lo, const double *__restrict__ hi,
                                                      int64_t n, double rho, MmaArgs a, T *__restrict__ xnew,
                                                      double *__restrict__ part) {
  __shared__ double lds[BS / 64];
  const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
  double s1 = 0, s3 = 0;
  if (j < n) {
    const double xj = x[j], d = df[j], l = L[j], u = U[j], dx = a.xmax - a.xmin;
    const double gp = fmax(d, 0.0), gm = fmax(-d, 0.0);
    const double p = (u - xj) * (u - xj) * (1.001 * gp + 0.001 * gm + rho / dx);
    const double q = (xj - l) * (xj - l) * (0.001 * gp + 1.001 * gm + rho / dx);
    const double sp = sqrt(p), sq = sqrt(q);
    double xs = (sp * l + sq * u) / (sp + sq);
    xs = fmin(fmax(xs, lo[j]), hi[j]);
    const T xt = (T)xs;
    xnew[j] = xt;
    const double xr = (double)xt;  // the value the caller evaluates
    s1 = (xr - xj) * (p / ((u - xr) * (u - xj)) - q / ((xr - l) * (xj - l)));
    s3 = (u - l) * (xr - xj) * (xr - xj) / ((u - xr) * (xr - l) * dx);
  }
  const double t1 = block_sum(s1, lds);
  const double t3 = block_sum(s3, lds);
  if (threadIdx.x == 0) {
    part[(size_t)blockIdx.x * 2 + 0] = t1;
    part[(size_t)blockIdx.x * 2 + 1] = t3;
  }
}

template <typename T>
__global__ void __launch_bounds__(BS) mma_accept_kernel(const T *__restrict__ xnew, int64_t n, double *__restrict__ x,
                                                       double *__restrict__ xo1, double *__restrict__ xo2) {
  const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (j >= n) return;
  xo2[j] = xo1[j];
  xo1[j] = x[j];
  x[j] = (double)xnew[j];
}

// ---------------------------------------------------------------- stats
template <typename T>
__global__ void __launch_bounds__(BS) stats_kernel(const T *__restrict__ x, const T *__restrict__ g, int64_t n,
                                                  double xmin, double xmax, double *__restrict__ part) {
  __shared__ double lds[BS / 64];
  const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
  double z = 0, r2 = 0;
  if (j < n) {
    const double xj = (double)x[j];
    z = 4.0 * xj * (1.0 - xj);
    if (g) {
      const double r = xj - fmin(fmax(xj - (double)g[j], xmin), xmax);
      r2 = r * r;
    }
  }
  const double a = block_sum(z, lds);
  const double b = block_sum(r2, lds);
  if (threadIdx.x == 0) {
    part[(size_t)blockIdx.x * 2] = a;
    part[(size_t)blockIdx.x * 2 + 1] = b;
  }
}

hipStream_t own_or(void *s, bool &own) {
  if (s) {
    own = false;
    return (hipStream_t)s;
  }
  hipStream_t t;
  FDTD_HIP(hipStreamCreate(&t));
  own = true;
  return t;
}

}  // namespace

struct fdtd_filter {
  int nx = 1, ny = 1, nz = 1, prec = 64, R = 0, Rz = 0;
  int64_t n = 0;
  double r = 0, alpha = 0;
  bool applied = false, own = false;
  hipStream_t s = nullptr;
  DevBuf winv, xs[5], h, g[2];  // stage inputs x0..x3 and output x4; transpose scratch
  ~fdtd_filter() {
    if (s) (void)hipStreamSynchronize(s);
    if (own && s) (void)hipStreamDestroy(s);
  }
};

struct fdtd_mma {
  int64_t n = 0;
  int prec = 64, k = 0;
  bool begun = false, own = false;
  double f0 = 0;
  MmaArgs a{};
  hipStream_t s = nullptr;
  DevBuf x, df, xo1, xo2, L, U, lo, hi, part, res;
  ~fdtd_mma() {
    if (s) (void)hipStreamSynchronize(s);
    if (own && s) (void)hipStreamDestroy(s);
  }
};

namespace {

// Forward stage k of the cascade: erode, dilate, dilate, erode.
constexpr int kDual[4] = {0, 1, 1, 0};

template <typename T>
void filter_apply(fdtd_filter *f, const void *rho, void *out, double alpha) {
  const dim3 g(nblocks(f->n)), b(BS);
  FDTD_HIP(hipMemcpyAsync(f->xs[0].p, rho, f->n * sizeof(T), hipMemcpyDeviceToDevice, f->s));
  for (int k = 0; k < 4; ++k)
    hipLaunchKernelGGL((stage_kernel<T, T>), g, b, 0, f->s, f->xs[k].as<T>(), f->xs[k + 1].as<T>(),
                       f->winv.as<double>(), f->nx, f->ny, f->nz, f->r, f->R, f->Rz, alpha, kDual[k]);
  FDTD_HIP(hipGetLastError());
  FDTD_HIP(hipMemcpyAsync(out, f->xs[4].p, f->n * sizeof(T), hipMemcpyDeviceToDevice, f->s));
}

template <typename T>
void filter_transpose(fdtd_filter *f, const void *gf, void *gout) {
  const dim3 g(nblocks(f->n)), b(BS);
  const double a = f->alpha;
  // stage 3 (erode, x3 -> x4) from the caller's gradient; intermediate
  // gradients in FP64
  hipLaunchKernelGGL((stage_h_kernel<T, T>), g, b, 0, f->s, (const T *)gf, f->xs[4].as<T>(), f->winv.as<double>(),
                     f->n, a, kDual[3], f->h.as<double>());
  int cur = 0;
  for (int k = 3; k >= 0; --k) {
    if (k < 3)
      hipLaunchKernelGGL((stage_h_kernel<double, T>), g, b, 0, f->s, f->g[cur ^ 1].as<double>(), f->xs[k + 1].as<T>(),
                         f->winv.as<double>(), f->n, a, kDual[k], f->h.as<double>());
    if (k > 0)
      hipLaunchKernelGGL((stage_gather_kernel<T, double>), g, b, 0, f->s, f->h.as<double>(), f->xs[k].as<T>(),
                         f->g[cur].as<double>(), f->nx, f->ny, f->nz, f->r, f->R, f->Rz, a, kDual[k]);
    else
      hipLaunchKernelGGL((stage_gather_kernel<T, T>), g, b, 0, f->s, f->h.as<double>(), f->xs[0].as<T>(), (T *)gout,
                         f->nx, f->ny, f->nz, f->r, f->R, f->Rz, a, kDual[0]);
    cur ^= 1;
  }
  FDTD_HIP(hipGetLastError());
}

}  // namespace

extern "C" {

const char *fdtd_design_last_error(void) { return g_err.c_str(); }

fdtd_status fdtd_filter_create(const int32_t n[3], double radius, int32_t precision, void *stream, fdtd_filter **out) {
  if (!out) return FDTD_EINVAL;
  *out = nullptr;
  auto f = new fdtd_filter();
  const fdtd_status st = dguard([&] {
    if (!n || n[0] < 1 || n[1] < 1 || n[2] < 1) throw Error{FDTD_EINVAL, "filter box must have positive size"};
    if (!(radius > 0) || radius > 16) throw Error{FDTD_EINVAL, "filter radius must lie in (0, 16] cells"};
    if (precision != 32 && precision != 64) throw Error{FDTD_EINVAL, "precision must be 32 or 64"};
    f->nx = n[0]; f->ny = n[1]; f->nz = n[2];
    f->n = (int64_t)n[0] * n[1] * n[2];
    f->prec = precision;
    f->r = radius;
    f->R = (int)std::ceil(radius);
    f->Rz = f->nz > 1 ? f->R : 0;
    f->s = own_or(stream, f->own);
    const size_t es = precision == 32 ? 4 : 8;
    f->winv.alloc(f->n * sizeof(double));
    for (auto &x : f->xs) x.alloc(f->n * es);
    f->h.alloc(f->n * sizeof(double));
    for (auto &x : f->g) x.alloc(f->n * sizeof(double));
    hipLaunchKernelGGL(winv_kernel, dim3(nblocks(f->n)), dim3(BS), 0, f->s, f->winv.as<double>(), f->nx, f->ny, f->nz,
                       f->r, f->R, f->Rz);
    FDTD_HIP(hipGetLastError());
    FDTD_HIP(hipStreamSynchronize(f->s));
  });
  if (st != FDTD_OK) {
    delete f;
    return st;
  }
  *out = f;
  return FDTD_OK;
}

fdtd_status fdtd_filter_apply(fdtd_filter *f, const void *rho, void *rho_f, double alpha) {
  if (!f) return FDTD_EINVAL;
  return dguard([&] {
    if (!rho || !rho_f) throw Error{FDTD_EINVAL, "null filter buffer"};
    if (!(alpha > 0)) throw Error{FDTD_EINVAL, "filter alpha must be > 0"};
    if (f->prec == 32) filter_apply<float>(f, rho, rho_f, alpha); else filter_apply<double>(f, rho, rho_f, alpha);
    f->alpha = alpha;
    f->applied = true;
  });
}

fdtd_status fdtd_filter_transpose(fdtd_filter *f, const void *g_f, void *g) {
  if (!f) return FDTD_EINVAL;
  return dguard([&] {
    if (!f->applied) throw Error{FDTD_ESTATE, "filter transpose before apply"};
    if (!g_f || !g) throw Error{FDTD_EINVAL, "null filter buffer"};
    if (f->prec == 32) filter_transpose<float>(f, g_f, g); else filter_transpose<double>(f, g_f, g);
  });
}

fdtd_status fdtd_filter_destroy(fdtd_filter *f) {
  delete f;
  return FDTD_OK;
}

fdtd_status fdtd_mma_create(int64_t n, int32_t precision, double xmin, double xmax, double move, double asyinit,
                            double asyincr, double asydecr, void *stream, fdtd_mma **out) {
  if (!out) return FDTD_EINVAL;
  *out = nullptr;
  auto m = new fdtd_mma();
  const fdtd_status st = dguard([&] {
    if (n < 1) throw Error{FDTD_EINVAL, "mma needs n >= 1"};
    if (precision != 32 && precision != 64) throw Error{FDTD_EINVAL, "precision must be 32 or 64"};
    if (!(xmax > xmin) || !(move > 0) || !(asyinit > 0) || !(asyincr >= 1) || !(asydecr > 0 && asydecr <= 1))
      throw Error{FDTD_EINVAL, "invalid mma parameters"};
    m->n = n;
    m->prec = precision;
    m->a = MmaArgs{xmin, xmax, move, asyinit, asyincr, asydecr};
    m->s = own_or(stream, m->own);
    for (DevBuf *b : {&m->x, &m->df, &m->xo1, &m->xo2, &m->L, &m->U, &m->lo, &m->hi}) b->alloc(n * sizeof(double));
    m->part.alloc((size_t)nblocks(n) * 3 * sizeof(double));
    m->res.alloc(4 * sizeof(double));
  });
  if (st != FDTD_OK) {
    delete m;
    return st;
  }
  *out = m;
  return FDTD_OK;
}

fdtd_status fdtd_mma_begin(fdtd_mma *m, const void *x, double f0, const void *df0, double *rho0) {
  if (!m) return FDTD_EINVAL;
  return dguard([&] {
    if (!x || !df0) throw Error{FDTD_EINVAL, "null mma buffer"};
    const int nb = nblocks(m->n);
    if (m->prec == 32)
      hipLaunchKernelGGL(mma_begin_kernel<float>, dim3(nb), dim3(BS), 0, m->s, (const float *)x, (const float *)df0,
                         m->n, m->k, m->a, m->x.as<double>(), m->df.as<double>(), m->xo1.as<double>(),
                         m->xo2.as<double>(), m->L.as<double>(), m->U.as<double>(), m->lo.as<double>(),
                         m->hi.as<double>(), m->part.as<double>());
    else
      hipLaunchKernelGGL(mma_begin_kernel<double>, dim3(nb), dim3(BS), 0, m->s, (const double *)x, (const double *)df0,
                         m->n, m->k, m->a, m->x.as<double>(), m->df.as<double>(), m->xo1.as<double>(),
                         m->xo2.as<double>(), m->L.as<double>(), m->U.as<double>(), m->lo.as<double>(),
                         m->hi.as<double>(), m->part.as<double>());
    FDTD_HIP(hipGetLastError());
    double sum = 0;
    finish<1>(m->s, m->part, nb, m->res, &sum);
    m->f0 = f0;
    m->begun = true;
    if (rho0) *rho0 = std::max(1e-6, 0.1 * sum / (double)m->n);
  });
}

fdtd_status fdtd_mma_solve(fdtd_mma *m, double rho, void *xnew, double *approx, double *dist) {
  if (!m) return FDTD_EINVAL;
  return dguard([&] {
    if (!m->begun) throw Error{FDTD_ESTATE, "mma solve before begin"};
    if (!xnew) throw Error{FDTD_EINVAL, "null mma buffer"};
    if (!(rho >= 0)) throw Error{FDTD_EINVAL, "mma rho must be >= 0"};
    const int nb = nblocks(m->n);
    if (m->prec == 32)
      hipLaunchKernelGGL(mma_solve_kernel<float>, dim3(nb), dim3(BS), 0, m->s, m->x.as<double>(), m->df.as<double>(),
                         m->L.as<double>(), m->U.as<double>(), m->lo.as<double>(), m->hi.as<double>(), m->n, rho, m->a,
                         (float *)xnew, m->part.as<double>());
    else
      hipLaunchKernelGGL(mma_solve_kernel<double>, dim3(nb), dim3(BS), 0, m->s, m->x.as<double>(), m->df.as<double>(),
                         m->L.as<double>(), m->U.as<double>(), m->lo.as<double>(), m->hi.as<double>(), m->n, rho, m->a,
                         (double *)xnew, m->part.as<double>());
    FDTD_HIP(hipGetLastError());
    double t[2];
    finish<2>(m->s, m->part, nb, m->res, t);
    if (approx) *approx = m->f0 + t[0];
    if (dist) *dist = t[1];
  });
}

fdtd_status fdtd_mma_accept(fdtd_mma *m, const void *xnew) {
  if (!m) return FDTD_EINVAL;
  return dguard([&] {
    if (!m->begun) throw Error{FDTD_ESTATE, "mma accept before begin"};
    if (!xnew) throw Error{FDTD_EINVAL, "null mma buffer"};
    const int nb = nblocks(m->n);
    if (m->prec == 32)
      hipLaunchKernelGGL(mma_accept_kernel<float>, dim3(nb), dim3(BS), 0, m->s, (const float *)xnew, m->n,
                         m->x.as<double>(), m->xo1.as<double>(), m->xo2.as<double>());
    else
      hipLaunchKernelGGL(mma_accept_kernel<double>, dim3(nb), dim3(BS), 0, m->s, (const double *)xnew, m->n,
                         m->x.as<double>(), m->xo1.as<double>(), m->xo2.as<double>());
    FDTD_HIP(hipGetLastError());
    FDTD_HIP(hipStreamSynchronize(m->s));
    m->k += 1;
    m->begun = false;
  });
}

fdtd_status fdtd_mma_destroy(fdtd_mma *m) {
  delete m;
  return FDTD_OK;
}

fdtd_status fdtd_design_stats(int64_t n, int32_t precision, const void *x, const void *g, double xmin, double xmax,
                              void *stream, double out[2]) {
  return dguard([&] {
    if (n < 1 || !x || !out) throw Error{FDTD_EINVAL, "design stats need n >= 1, x and out"};
    if (precision != 32 && precision != 64) throw Error{FDTD_EINVAL, "precision must be 32 or 64"};
    bool own = false;
    hipStream_t s = own_or(stream, own);
    const int nb = nblocks(n);
    DevBuf part, res;
    part.alloc((size_t)nb * 2 * sizeof(double));
    res.alloc(2 * sizeof(double));
    if (precision == 32)
      hipLaunchKernelGGL(stats_kernel<float>, dim3(nb), dim3(BS), 0, s, (const float *)x, (const float *)g, n, xmin,
                         xmax, part.as<double>());
    else
      hipLaunchKernelGGL(stats_kernel<double>, dim3(nb), dim3(BS), 0, s, (const double *)x, (const double *)g, n, xmin,
                         xmax, part.as<double>());
    FDTD_HIP(hipGetLastError());
    double t[2];
    finish<2>(s, part, nb, res, t);
    out[0] = t[0] / (double)n;
    out[1] = std::sqrt(t[1]);
    if (own) (void)hipStreamDestroy(s);
  });
}

}  // extern "C"
