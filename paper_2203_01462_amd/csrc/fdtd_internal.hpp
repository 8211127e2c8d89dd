// fdtd_internal.hpp -- context layout and shared helpers of the HIP library.
//
// Everything here is the product path: the GPU context, its device buffers
// and the small setup kernels (incident-field line, DFT phasors, objective
// weights, objective reduction, adjoint-source table, gradient finalize).
// The time-stepping kernels live in fdtd_2d.hip / fdtd_3d.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "fdtd.h"

namespace fdtd {

constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * M_PI;
constexpr double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

struct Error {
  fdtd_status code;
  std::string msg;
};

#define FDTD_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::fdtd::Error{FDTD_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// A device allocation owned by the context.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{FDTD_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;  // sole owner of its allocation
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
};

// Absorber grading at depth d in (0,1] (1 at the wall): polynomial
// conductivity up to 0.8(m+1)/(eta dx), stretch kappa, shift alpha;
// recursive-convolution coefficients b, a.
struct Grade {
  double b, a, kap;
};

inline Grade pml_grade(const fdtd_config &c, double dt, double d) {
  const double m = c.pml_order;
  const double eta = std::sqrt(kMu0 / (kEps0 * c.eps_s));
  const double smax = c.pml_sigma_scale * 0.8 * (m + 1.0) / (eta * c.dx);
  const double sig = smax * std::pow(d, m);
  const double k = 1.0 + (c.pml_kappa_max - 1.0) * std::pow(d, m);
  const double alp = c.pml_alpha_max * (1.0 - d);
  Grade g;
  g.kap = k;
  g.b = std::exp(-(sig / k + alp) * dt / kEps0);
  g.a = sig > 0.0 ? sig * (g.b - 1.0) / (sig * k + k * k * alp) : 0.0;
  return g;
}

// Depth of coordinate `pos` (cells; half-integers for staggered components)
// on an axis of n nodes with the absorber over the P cells next to each wall.
inline double pml_depth(int n, int P, double pos) {
  if (P <= 0) return 0.0;
  if (pos < P) return (P - pos) / P;
  if (pos > (n - 1) - P) return (pos - ((n - 1) - P)) / P;
  return 0.0;
}

// Excitation waveform samples g(n dt), n = 0..N (see fdtd.h source kinds).
inline double source_wave(const fdtd_config &c, double t) {
  if (c.source_kind == FDTD_SRC_NONE) return 0.0;
  const double fc = 0.5 * (c.f_lo + c.f_hi);
  const double bw = c.f_hi - c.f_lo;
  if (c.source_kind == FDTD_SRC_GAUSS) {
    const double tau = std::sqrt(std::log(2.0)) / (M_PI * 0.5 * bw);
    const double t0 = c.t0_over_tau * tau;
    const double u = (t - t0) / tau;
    return c.amplitude * std::sin(2.0 * M_PI * fc * (t - t0)) * std::exp(-u * u);
  }
  const double half = 4.0 / bw;  // sinc envelope cut after four lobes each side
  const double s = t - half;
  if (std::fabs(s) >= half) return 0.0;
  const double x = M_PI * bw * s;
  const double env = std::fabs(x) < 1e-300 ? 1.0 : std::sin(x) / x;
  const double hann = 0.5 * (1.0 + std::cos(M_PI * s / half));
  return c.amplitude * env * hann * std::cos(2.0 * M_PI * fc * s);
}

// Per-axis grading tables at integer (e) and half-integer (h) positions,
// stored as b, a, 1/kappa in the working precision.
template <typename T>
struct AxisTables {
  std::vector<T> be, ae, ike, bh, ah, ikh;
  void build(const fdtd_config &c, double dt, int n, int P) {
    be.assign(n, T(1)); ae.assign(n, T(0)); ike.assign(n, T(1));
    bh.assign(n, T(1)); ah.assign(n, T(0)); ikh.assign(n, T(1));
    for (int i = 0; i < n; ++i) {
      const double de = pml_depth(n, P, i), dh = pml_depth(n, P, i + 0.5);
      if (de > 0) { Grade g = pml_grade(c, dt, de); be[i] = T(g.b); ae[i] = T(g.a); ike[i] = T(1.0 / g.kap); }
      if (dh > 0) { Grade g = pml_grade(c, dt, dh); bh[i] = T(g.b); ah[i] = T(g.a); ikh[i] = T(1.0 / g.kap); }
    }
  }
};

// Launch helpers implemented in fdtd_setup.hip.
void launch_incident_line(hipStream_t s, int precision, const double *g, int N, int n1, int L,
                          const double *prof, double ch, double ce, double cmu, double cep,
                          double *scratch, void *einc, void *hinc);
void launch_phasors(hipStream_t s, const double *freqs, int K, int N, double dt, double *phasor);
void launch_weights(hipStream_t s, const double *g, const double *freqs, int K, int N, double dt,
                    int unit, double *w);
void launch_dft(hipStream_t s, const double *gapE, const double *phasor, int K, int nmon, int N, double dt,
                double *dft);
void launch_objective(hipStream_t s, const double *dft, const double *w, const double *gapE, int K,
                      int nmon, int N, int time_energy, double te_scale, double *F_out);
void launch_adjoint_source(hipStream_t s, int precision, const double *dft, const double *w,
                           const double *phasor, const double *gapE, int K, int nmon, int N,
                           int time_energy, double te_coef, double dt, double dx, double *scale_out,
                           void *table);
void launch_grad_finalize(hipStream_t s, int precision, const double *acc, const double *scale, int ncomp, int dnx,
                          int dny, int dnz, int gx0, int gy0, int gz0, int gnx, int gny, int gnz, void *out);
void launch_fill_zero(hipStream_t s, void *p, size_t bytes);
void launch_watch(hipStream_t s, int precision, const void *p, size_t n, unsigned long long *slot);
void launch_check_density(hipStream_t s, int precision, const void *rho, int64_t n, int *bad);
void launch_copy_density(hipStream_t s, int precision, const void *src, void *dst, int64_t n);

}  // namespace fdtd
