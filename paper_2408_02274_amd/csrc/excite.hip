// Incident fields of an electric dipole at a complex source point.
//
// Paper, Sec. IV: the waveguide splitter is excited by a source at one end
// face.  A point dipole p at x_s = x_0 + i b d (b real, d a unit vector)
// radiates the exact Maxwell field below, which for k b >> 1 is a Gaussian
// beam of waist w_0 = sqrt(2 b / k) launched along +d from x_0.  With
// R = x - x_s (complex), r = sqrt(R.R) on the principal branch (Re r >= 0),
// G = exp(i k r) / (4 pi r), f1 = G (i k - 1/r) / r and
// f2 = G (-k^2 - 3 i k / r + 3 / r^2) / r^2:
//   E = (1/eps) (k^2 G p + f1 p + f2 (R.p) R)
//   H = -i omega f1 (R x p)
// the fields of the Hertz potential Pi = p G (E = (k^2 Pi + grad div Pi) / eps,
// H = -i omega curl Pi), which satisfy curl E = i omega mu H and
// curl H = -i omega eps E with k^2 = omega^2 eps mu.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/ifgf.h"
#include "util.hpp"

using namespace ifgf;

namespace {

struct Dip {
  double pr[3], pi[3];      // dipole moment (re, im)
  double xs[3], beam[3];    // source x_0 and b d (imaginary part of the source point)
  double k, eps, omega;
};

struct cpx {
  double re, im;
};
__device__ __forceinline__ cpx operator+(cpx a, cpx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cpx operator-(cpx a, cpx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cpx operator*(cpx a, cpx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cpx operator*(double s, cpx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cpx cdiv(cpx a, cpx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
// principal square root (real part >= 0), without cancellation
__device__ __forceinline__ cpx csqrt_p(cpx z) {
  const double m = hypot(z.re, z.im);
  if (m == 0.0) return {0.0, 0.0};
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (m + z.re));
    return {t, z.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (m - z.re));
  return {fabs(z.im) / (2.0 * t), z.im < 0.0 ? -t : t};
}
__device__ __forceinline__ cpx cexp_i(cpx z) {   // exp(i z)
  const double a = exp(-z.im);
  double s, c;
  sincos(z.re, &s, &c);
  return {a * c, a * s};
}

__global__ void __launch_bounds__(256) k_dipole(int64_t n, const double* __restrict__ x, Dip d,
                                                double2* __restrict__ E, double2* __restrict__ H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cpx R[3], p[3];
  for (int c = 0; c < 3; ++c) {
    R[c] = {x[3 * i + c] - d.xs[c], -d.beam[c]};
    p[c] = {d.pr[c], d.pi[c]};
  }
  const cpx rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  const cpx r = csqrt_p(rr);
  const cpx ir = cdiv({1.0, 0.0}, r);
  const cpx ikr = cexp_i(d.k * r);
  const cpx G = 0.07957747154594767 * (ikr * ir);
  const cpx ik = {0.0, d.k};
  const cpx f1 = G * (ik - ir) * ir;
  const cpx ir2 = ir * ir;
  const cpx f2 = G * (cpx{-d.k * d.k, 0.0} - 3.0 * (ik * ir) + 3.0 * ir2) * ir2;
  const cpx Rp = R[0] * p[0] + R[1] * p[1] + R[2] * p[2];
  const double ie = 1.0 / d.eps;
  const cpx kG = (d.k * d.k) * G;
  for (int c = 0; c < 3; ++c) {
    const cpx e = ie * (kG * p[c] + f1 * p[c] + f2 * Rp * R[c]);
    E[3 * i + c] = make_double2(e.re, e.im);
  }
  const cpx rxp[3] = {R[1] * p[2] - R[2] * p[1], R[2] * p[0] - R[0] * p[2], R[0] * p[1] - R[1] * p[0]};
  const cpx mio = {0.0, -d.omega};
  for (int c = 0; c < 3; ++c) {
    const cpx h = mio * f1 * rxp[c];
    H[3 * i + c] = make_double2(h.re, h.im);
  }
}

}  // namespace

extern "C" int ifgf_dipole_field(int64_t n, const void* points, double k, double eps, double omega,
                                 const double* dipole, void* E, void* H, void* stream) {
  clear_error();
  if (n < 0 || (n > 0 && (!points || !E || !H)) || !dipole) return set_error(IFGF_EINVAL, "null argument");
  if (!(k > 0.0) || !(eps > 0.0) || !(omega > 0.0)) return set_error(IFGF_EINVAL, "k, eps and omega must be > 0");
  Dip d;
  for (int c = 0; c < 3; ++c) {
    d.pr[c] = dipole[2 * c];
    d.pi[c] = dipole[2 * c + 1];
    d.xs[c] = dipole[6 + c];
    d.beam[c] = dipole[9 + c];
  }
  for (int j = 0; j < 12; ++j)
    if (!std::isfinite(dipole[j])) return set_error(IFGF_EINVAL, "non-finite dipole parameters");
  d.k = k;
  d.eps = eps;
  d.omega = omega;
  if (n == 0) return IFGF_OK;
  hipLaunchKernelGGL(k_dipole, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                     static_cast<const double*>(points), d, static_cast<double2*>(E), static_cast<double2*>(H));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "dipole field");
}
