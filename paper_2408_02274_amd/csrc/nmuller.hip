// N-Mueller forward map on gfx950: densities, near-field correction product,
// operator assembly and right-hand side (FP64).
//
// Paper: Sec. II eq. n_muller, k_delta, r_delta, t_delta (operator);
// Sec. III intro eq. sl_scalar, dl_scalar (eight densities, S and D = dS/dn,
// derivatives via Chebyshev recurrences); Sec. III-H (local corrections).
#include <hip/hip_runtime.h>

#include <chrono>
#include <memory>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ifgf.h"
#include "corrections.hpp"
#include "device.hpp"
#include "nmuller_host.hpp"
#include "precond.hpp"
#include "util.hpp"

using namespace ifgf;

namespace {

constexpr int kMaxNq = 256;  // nodes per patch handled by one workgroup (Nc <= 16)

struct GeoDev {
  const double* nrm;   // [n][3]
  const double* t1;
  const double* t2;
  const double* gu;
  const double* gv;
  const double* J;     // [n]
  const double* Q;     // [n][4]
  const double* D;     // [nc][nc]
  int nc;
  int64_t n;
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
struct c3 {
  double2 v[3];
};
__device__ __forceinline__ c3 rcross(const double* n, const c3& a) {   // real n x complex a
  c3 o;
  o.v[0] = csub(cscale(n[1], a.v[2]), cscale(n[2], a.v[1]));
  o.v[1] = csub(cscale(n[2], a.v[0]), cscale(n[0], a.v[2]));
  o.v[2] = csub(cscale(n[0], a.v[1]), cscale(n[1], a.v[0]));
  return o;
}
__device__ __forceinline__ double2 rdot(const double* t, const c3& a) {
  return cadd(cadd(cscale(t[0], a.v[0]), cscale(t[1], a.v[1])), cscale(t[2], a.v[2]));
}

// a1: unknowns (m.t1, m.t2, j.t1, j.t2) -> eight densities (m, j, div m, div j)
__global__ void __launch_bounds__(256) k_pre(GeoDev g, const double2* __restrict__ y, double2* __restrict__ phi) {
  __shared__ double2 s[4][kMaxNq];   // J a^u (m), J a^v (m), J a^u (j), J a^v (j)
  const int nq = g.nc * g.nc;
  const int p = blockIdx.x;
  const int r = blockIdx.y;
  const int t = threadIdx.x;
  const int64_t n = g.n;
  const double2* yr = y + (int64_t)r * 4 * n;
  double2* ph = phi + (int64_t)r * 8 * n;
  int64_t l = (int64_t)p * nq + t;
  double2 c[4];
  if (t < nq) {
    for (int k = 0; k < 4; ++k) c[k] = yr[k * n + l];
    const double* Q = g.Q + 4 * l;
    s[0][t] = cadd(cscale(Q[0], c[0]), cscale(Q[1], c[1]));
    s[1][t] = cadd(cscale(Q[2], c[0]), cscale(Q[3], c[1]));
    s[2][t] = cadd(cscale(Q[0], c[2]), cscale(Q[1], c[3]));
    s[3][t] = cadd(cscale(Q[2], c[2]), cscale(Q[3], c[3]));
  }
  __syncthreads();
  if (t >= nq) return;
  const int i = t / g.nc, j = t % g.nc;
  const double* t1 = g.t1 + 3 * l;
  const double* t2 = g.t2 + 3 * l;
  for (int k = 0; k < 3; ++k) {
    ph[k * n + l] = cadd(cscale(t1[k], c[0]), cscale(t2[k], c[1]));
    ph[(3 + k) * n + l] = cadd(cscale(t1[k], c[2]), cscale(t2[k], c[3]));
  }
  for (int a = 0; a < 2; ++a) {
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < g.nc; ++k) {
      acc = cadd(acc, cscale(g.D[i * g.nc + k], s[2 * a][k * g.nc + j]));
      acc = cadd(acc, cscale(g.D[j * g.nc + k], s[2 * a + 1][i * g.nc + k]));
    }
    ph[(6 + a) * n + l] = cscale(1.0 / g.J[l], acc);
  }
}

// a7: out += C phi for the singular patches of every target (one wavefront per
// target).  The lanes run over the (patch, node) pairs of the target's rows
// as one flat range, so every lane has work in every step but the last.
__global__ void __launch_bounds__(256) k_correct(const int64_t* __restrict__ row_off, const int32_t* __restrict__ pair_patch,
                          const double2* __restrict__ vals, int nq, int64_t n,
                          const double2* __restrict__ phi, double2* __restrict__ out, int nrhs) {
  const int lane = threadIdx.x & 63;
  const int64_t l = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int r = blockIdx.y;
  if (l >= n || r >= nrhs) return;
  const double2* ph = phi + (int64_t)r * 8 * n;
  double2 acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = make_double2(0.0, 0.0);
  const int64_t e0 = row_off[l];
  const int tot = (int)(row_off[l + 1] - e0) * nq;
  // flat index f = pair * nq + node, advanced by 64 per step
  int el = lane / nq, q = lane - (lane / nq) * nq;
  for (int f = lane; f < tot; f += 64) {
    {
      const int64_t e = e0 + el;
      const int64_t base = (int64_t)pair_patch[e] * nq;
      const double2* C = vals + e * 4 * nq;
      double2 w0 = C[q], w1 = C[nq + q], w2 = C[2 * nq + q], w3 = C[3 * nq + q];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        double2 v = ph[c * n + base + q];
        acc[c] = cadd(acc[c], cmulc(w0, v));            // S, k_int
        acc[14 + c] = cadd(acc[14 + c], cmulc(w1, v));  // S, k_ext
        if (c < 6) {
          acc[8 + c] = cadd(acc[8 + c], cmulc(w2, v));    // D, k_int
          acc[22 + c] = cadd(acc[22 + c], cmulc(w3, v));  // D, k_ext
        }
      }
    }
    q += 64;
    while (q >= nq) {
      q -= nq;
      ++el;
    }
  }
#pragma unroll
  for (int k = 0; k < 28; ++k) {
    double re = acc[k].x, im = acc[k].y;
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    acc[k] = make_double2(re, im);
  }
  if (lane < 28) {
    double2* o = out + (int64_t)r * 28 * n + (int64_t)lane * n + l;
    double2 v = acc[0];
#pragma unroll
    for (int k = 1; k < 28; ++k)
      if (k == lane) v = acc[k];
    *o = cadd(*o, v);
  }
}

struct Mat {
  double eps_e, eps_i, mu_e, mu_i, omega, ke, ki;
};

// a8: K, R, T from S and D, Delta-combinations and identity terms, projection on t1, t2
__global__ void __launch_bounds__(256) k_post(GeoDev g, Mat mt, const double2* __restrict__ y,
                       const double2* __restrict__ SD, double2* __restrict__ Ay) {
  __shared__ double2 s[16][kMaxNq];   // S_q[phi_c], q = 0,1, c = 0..7
  const int nq = g.nc * g.nc;
  const int p = blockIdx.x;
  const int r = blockIdx.y;
  const int t = threadIdx.x;
  const int64_t n = g.n;
  const double2* sd = SD + (int64_t)r * 28 * n;
  int64_t l = (int64_t)p * nq + t;
  if (t < nq)
    for (int q = 0; q < 2; ++q)
      for (int c = 0; c < 8; ++c) s[q * 8 + c][t] = sd[(q * 14 + c) * n + l];
  __syncthreads();
  if (t >= nq) return;
  const int i = t / g.nc, j = t % g.nc;
  const double* nn = g.nrm + 3 * l;
  const double* gu = g.gu + 3 * l;
  const double* gv = g.gv + 3 * l;
  const double* t1 = g.t1 + 3 * l;
  const double* t2 = g.t2 + 3 * l;
  // surface gradient of field f: f_u gu + f_v gv
  auto sgrad = [&](int f, c3& o) {
    double2 fu = make_double2(0.0, 0.0), fv = make_double2(0.0, 0.0);
    for (int k = 0; k < g.nc; ++k) {
      fu = cadd(fu, cscale(g.D[i * g.nc + k], s[f][k * g.nc + j]));
      fv = cadd(fv, cscale(g.D[j * g.nc + k], s[f][i * g.nc + k]));
    }
    for (int c = 0; c < 3; ++c) o.v[c] = cadd(cscale(gu[c], fu), cscale(gv[c], fv));
  };
  // K, R, T for kernel q and density block (base 0: m, 3: j; div index 6 or 7)
  auto krt = [&](int q, int base, int divi, c3& K, c3& R, c3& T) {
    c3 grad[3];   // grad[c] = grad A_c
    c3 A;
    for (int c = 0; c < 3; ++c) {
      sgrad(q * 8 + base + c, grad[c]);
      double2 Dn = sd[(q * 14 + 8 + base + c) * n + l];
      for (int k = 0; k < 3; ++k) grad[c].v[k] = cadd(grad[c].v[k], cscale(nn[k], Dn));
      A.v[c] = s[q * 8 + base + c][t];
    }
    c3 curl;
    curl.v[0] = csub(grad[2].v[1], grad[1].v[2]);
    curl.v[1] = csub(grad[0].v[2], grad[2].v[0]);
    curl.v[2] = csub(grad[1].v[0], grad[0].v[1]);
    K = rcross(nn, curl);
    R = rcross(nn, A);
    c3 gd;
    sgrad(q * 8 + divi, gd);
    T = rcross(nn, gd);
  };
  c3 Kim, Rim, Tim, Kem, Rem, Tem, Kij, Rij, Tij, Kej, Rej, Tej;
  krt(0, 0, 6, Kim, Rim, Tim);
  krt(1, 0, 6, Kem, Rem, Tem);
  krt(0, 3, 7, Kij, Rij, Tij);
  krt(1, 3, 7, Kej, Rej, Tej);
  const double2* yr = y + (int64_t)r * 4 * n;
  double2 yc[4];
  for (int k = 0; k < 4; ++k) yc[k] = yr[k * n + l];
  c3 m, jv, row1, row2;
  for (int c = 0; c < 3; ++c) {
    m.v[c] = cadd(cscale(t1[c], yc[0]), cscale(t2[c], yc[1]));
    jv.v[c] = cadd(cscale(t1[c], yc[2]), cscale(t2[c], yc[3]));
  }
  const double ke2 = mt.ke * mt.ke, ki2 = mt.ki * mt.ki;
  for (int c = 0; c < 3; ++c) {
    // (R^D + T^D)[a] = (-i/omega)(ke^2 R_e - ki^2 R_i + T_e - T_i)
    double2 sj = cadd(csub(cscale(ke2, Rej.v[c]), cscale(ki2, Rij.v[c])), csub(Tej.v[c], Tij.v[c]));
    double2 sm = cadd(csub(cscale(ke2, Rem.v[c]), cscale(ki2, Rim.v[c])), csub(Tem.v[c], Tim.v[c]));
    double2 RTj = make_double2(sj.y / mt.omega, -sj.x / mt.omega);
    double2 RTm = make_double2(sm.y / mt.omega, -sm.x / mt.omega);
    row1.v[c] = csub(cadd(cscale(0.5 * (mt.mu_e + mt.mu_i), m.v[c]),
                          csub(cscale(mt.mu_e, Kem.v[c]), cscale(mt.mu_i, Kim.v[c]))), RTj);
    row2.v[c] = cadd(RTm, cadd(cscale(0.5 * (mt.eps_e + mt.eps_i), jv.v[c]),
                               csub(cscale(mt.eps_e, Kej.v[c]), cscale(mt.eps_i, Kij.v[c]))));
  }
  double2* o = Ay + (int64_t)r * 4 * n;
  o[0 * n + l] = rdot(t1, row1);
  o[1 * n + l] = rdot(t2, row1);
  o[2 * n + l] = rdot(t1, row2);
  o[3 * n + l] = rdot(t2, row2);
}

// right-hand side of eq. n_muller: omega^-1 (n x E, n x H) on (t1, t2)
__global__ void k_rhs(GeoDev g, double omega, const double2* __restrict__ E,
                      const double2* __restrict__ H, double2* __restrict__ b, int nrhs) {
  int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (l >= g.n || r >= nrhs) return;
  const double* nn = g.nrm + 3 * l;
  const double* t1 = g.t1 + 3 * l;
  const double* t2 = g.t2 + 3 * l;
  c3 e, h;
  for (int c = 0; c < 3; ++c) {
    e.v[c] = cscale(1.0 / omega, E[((int64_t)r * g.n + l) * 3 + c]);
    h.v[c] = cscale(1.0 / omega, H[((int64_t)r * g.n + l) * 3 + c]);
  }
  c3 ne = rcross(nn, e), nh = rcross(nn, h);
  double2* o = b + (int64_t)r * 4 * g.n;
  o[0 * g.n + l] = rdot(t1, ne);
  o[1 * g.n + l] = rdot(t2, ne);
  o[2 * g.n + l] = rdot(t1, nh);
  o[3 * g.n + l] = rdot(t2, nh);
}

}  // namespace

struct nmuller_s {
  nmuller_params prm;
  SurfaceGeo geo;
  Corrections cor;
  ifgf_plan_t ifgf = nullptr;
  int host_only = 0;
  int max_nrhs = 1;
  DeviceArena arena;
  GeoDev gd{};
  int64_t* d_row_off = nullptr;
  int32_t* d_pair_patch = nullptr;
  double2* d_vals = nullptr;
  int cor_on_device = 0;      // corrections built by the device builder
  double cor_seconds = 0.0;   // wall time of the correction build
  double2* d_phi = nullptr;   // [max_nrhs][8][n]
  double2* d_sd = nullptr;    // [max_nrhs][2][14][n]
  Mat mat{};
  std::unique_ptr<ifgf::Precond> pc;   // learned preconditioner (optional)
  ~nmuller_s() {
    if (ifgf) ifgf_destroy(ifgf);
  }
};

ifgf::Precond* nmuller_precond(nmuller_s* nm) { return nm ? nm->pc.get() : nullptr; }
int nmuller_max_rhs(nmuller_s* nm) { return nm ? nm->max_nrhs : 1; }

namespace {
template <class T>
int up(DeviceArena& ar, const std::vector<T>& v, const T** dst) {
  T* p = static_cast<T*>(ar.alloc(v.size() * sizeof(T)));
  if (!p) return set_error(IFGF_ENOMEM, "device allocation failed");
  hipError_t e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return set_hip_error(e, "hipMemcpy");
  *dst = p;
  return 0;
}
}  // namespace

extern "C" {

void nmuller_default_params(nmuller_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->eps_e = 1.0;
  p->eps_i = 1.0;
  p->mu_e = 1.0;
  p->mu_i = 1.0;
  p->omega = 2.0 * 3.141592653589793;
  p->delta_factor = 1.0;
  p->nbeta = 0;
  p->d_cov = 4;
  p->corrections_on_host = 0;
}

int nmuller_plan(nmuller_t* out, const nmuller_params* prm, const double* points,
                 const double* du, const double* dv, double tol, const ifgf_options* opt) {
  clear_error();
  if (!out || !prm || !points || !du || !dv) return set_error(IFGF_EINVAL, "null argument");
  *out = nullptr;
  if (!(prm->eps_e > 0 && prm->eps_i > 0 && prm->mu_e > 0 && prm->mu_i > 0 && prm->omega > 0))
    return set_error(IFGF_EINVAL, "material parameters and omega must be > 0");
  const int64_t n = (int64_t)prm->P * prm->Nc * prm->Nc;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(points[i]) || !std::isfinite(du[i]) || !std::isfinite(dv[i]))
      return set_error(IFGF_EINVAL, "non-finite geometry at entry " + std::to_string(i));
  nmuller_s* nm = new (std::nothrow) nmuller_s();
  if (!nm) return set_error(IFGF_ENOMEM, "host allocation failed");
  nm->prm = *prm;
  std::string err;
  if (build_surface(nm->geo, prm->P, prm->Nc, points, du, dv, err)) {
    delete nm;
    return set_error(IFGF_EINVAL, err);
  }
  const double ke = prm->omega * std::sqrt(prm->eps_e * prm->mu_e);
  const double ki = prm->omega * std::sqrt(prm->eps_i * prm->mu_i);
  nm->mat = Mat{prm->eps_e, prm->eps_i, prm->mu_e, prm->mu_i, prm->omega, ke, ki};
  ifgf_options o;
  ifgf_default_options(&o);
  if (opt) o = *opt;
  nm->host_only = o.host_only;
  nm->max_nrhs = o.max_nrhs > 0 ? o.max_nrhs : 1;
  int rc = ifgf_plan(&nm->ifgf, n, points, nm->geo.nrm.data(), nm->geo.w.data(), ki, ke, tol, &o);
  if (rc) {
    std::string m = ifgf_last_error();
    delete nm;
    return set_error(rc, m);
  }
  SingParams sp;
  if (prm->delta_factor > 0) sp.delta_factor = prm->delta_factor;
  sp.nbeta = prm->nbeta;
  if (prm->d_cov >= 2) sp.d = prm->d_cov;
  const bool on_device = !nm->host_only && !prm->corrections_on_host &&
                         device_corrections_supported(prm->Nc, prm->nbeta);
  const auto t_cor = std::chrono::steady_clock::now();
  if (on_device) {
    DevCorrections dc;
    if ((rc = build_corrections_device(nm->geo, ki, ke, sp, nm->arena, dc, nm->cor, err))) {
      delete nm;
      return set_error(rc, err);
    }
    nm->d_row_off = dc.row_off;
    nm->d_pair_patch = dc.pair_patch;
    nm->d_vals = dc.vals;
    nm->cor_on_device = 1;
  } else {
    try {
      if (build_corrections(nm->geo, ki, ke, sp, nm->cor, err)) {
        delete nm;
        return set_error(IFGF_EINVAL, err);
      }
    } catch (const std::bad_alloc&) {
      delete nm;
      return set_error(IFGF_ENOMEM, "host allocation failed in the singular quadrature");
    }
  }
  nm->cor_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_cor).count();
  if (nm->host_only) {
    *out = nm;
    return IFGF_OK;
  }
  DeviceArena& ar = nm->arena;
  GeoDev& gd = nm->gd;
  gd.nc = prm->Nc;
  gd.n = n;
  if ((rc = up(ar, nm->geo.nrm, &gd.nrm)) || (rc = up(ar, nm->geo.t1, &gd.t1)) ||
      (rc = up(ar, nm->geo.t2, &gd.t2)) || (rc = up(ar, nm->geo.gu, &gd.gu)) ||
      (rc = up(ar, nm->geo.gv, &gd.gv)) || (rc = up(ar, nm->geo.J, &gd.J)) ||
      (rc = up(ar, nm->geo.Q, &gd.Q)) || (rc = up(ar, nm->geo.Dcheb, &gd.D))) {
    delete nm;
    return rc;
  }
  if (!on_device) {
    const int64_t* ro = nullptr;
    const int32_t* pp = nullptr;
    const double* vv = nullptr;
    if ((rc = up(ar, nm->cor.row_off, &ro)) || (rc = up(ar, nm->cor.pair_patch, &pp)) ||
        (rc = up(ar, nm->cor.vals, &vv))) {
      delete nm;
      return rc;
    }
    nm->d_row_off = const_cast<int64_t*>(ro);
    nm->d_pair_patch = const_cast<int32_t*>(pp);
    nm->d_vals = reinterpret_cast<double2*>(const_cast<double*>(vv));
    std::vector<double>().swap(nm->cor.vals);   // device copy is the working one
  }
  nm->d_phi = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)nm->max_nrhs * 8 * n));
  nm->d_sd = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)nm->max_nrhs * 28 * n));
  if (!nm->d_phi || !nm->d_sd) {
    delete nm;
    return set_error(IFGF_ENOMEM, "device workspace allocation failed");
  }
  *out = nm;
  return IFGF_OK;
}

int nmuller_apply(nmuller_t nm, const void* y, int nrhs, void* Ay, void* stream) {
  clear_error();
  if (!nm || !y || !Ay) return set_error(IFGF_EINVAL, "null argument");
  if (nm->host_only) return set_error(IFGF_ENOTPLANNED, "plan was built with host_only");
  if (nrhs < 1 || nrhs > nm->max_nrhs) return set_error(IFGF_EINVAL, "nrhs must lie in [1, max_nrhs]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = nm->gd.n;
  const int nq = nm->gd.nc * nm->gd.nc;
  const int bs = ((nq + 63) / 64) * 64;
  const double2* yy = static_cast<const double2*>(y);
  const int64_t npairs = nm->cor.row_off.back();
  hipEvent_t ev = timer_begin(nm->ifgf, st);
  hipLaunchKernelGGL(k_pre, dim3(nm->prm.P, nrhs), dim3(bs), 0, st, nm->gd, yy, nm->d_phi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_hip_error(e, "nmuller pre");
  timer_end(nm->ifgf, "nm_pre", ev, st, (double)n * nrhs);
  int rc = ifgf_apply(nm->ifgf, nm->d_phi, nrhs, nm->d_sd, stream);
  if (rc) return rc;
  const int wpb = 4;   // wavefronts (targets) per block
  ev = timer_begin(nm->ifgf, st);
  hipLaunchKernelGGL(k_correct, dim3((unsigned)((n + wpb - 1) / wpb), nrhs), dim3(64 * wpb), 0, st,
                     nm->d_row_off, nm->d_pair_patch, nm->d_vals, nq, n, nm->d_phi, nm->d_sd, nrhs);
  if ((e = hipGetLastError()) != hipSuccess) return set_hip_error(e, "nmuller correction");
  timer_end(nm->ifgf, "nm_correct", ev, st, (double)npairs * nq * nrhs);
  ev = timer_begin(nm->ifgf, st);
  hipLaunchKernelGGL(k_post, dim3(nm->prm.P, nrhs), dim3(bs), 0, st, nm->gd, nm->mat, yy, nm->d_sd,
                     static_cast<double2*>(Ay));
  if ((e = hipGetLastError()) != hipSuccess) return set_hip_error(e, "nmuller post");
  timer_end(nm->ifgf, "nm_post", ev, st, (double)n * nrhs);
  return IFGF_OK;
}

int nmuller_rhs(nmuller_t nm, const void* E, const void* H, int nrhs, void* b, void* stream) {
  clear_error();
  if (!nm || !E || !H || !b) return set_error(IFGF_EINVAL, "null argument");
  if (nm->host_only) return set_error(IFGF_ENOTPLANNED, "plan was built with host_only");
  if (nrhs < 1) return set_error(IFGF_EINVAL, "nrhs must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)((nm->gd.n + 255) / 256), nrhs), dim3(256), 0, st, nm->gd,
                     nm->prm.omega, static_cast<const double2*>(E), static_cast<const double2*>(H),
                     static_cast<double2*>(b), nrhs);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "nmuller rhs");
}

int nmuller_geometry(nmuller_t nm, int which, double* buf, int64_t cap) {
  clear_error();
  if (!nm || !buf) return set_error(IFGF_EINVAL, "null argument");
  const std::vector<double>* v = nullptr;
  switch (which) {
    case 0: v = &nm->geo.nrm; break;
    case 1: v = &nm->geo.w; break;
    case 2: v = &nm->geo.t1; break;
    case 3: v = &nm->geo.t2; break;
    case 4: v = &nm->geo.J; break;
    default: return set_error(IFGF_EINVAL, "unknown geometry id");
  }
  if (cap < (int64_t)v->size()) return set_error(IFGF_EINVAL, "buffer too small");
  std::memcpy(buf, v->data(), v->size() * sizeof(double));
  return IFGF_OK;
}

int nmuller_corrections(nmuller_t nm, int64_t* npairs, int64_t* row_off, int32_t* pair_patch,
                        double* vals) {
  clear_error();
  if (!nm || !npairs) return set_error(IFGF_EINVAL, "null argument");
  *npairs = nm->cor.row_off.empty() ? 0 : nm->cor.row_off.back();
  if (row_off) std::memcpy(row_off, nm->cor.row_off.data(), nm->cor.row_off.size() * sizeof(int64_t));
  if (pair_patch)
    std::memcpy(pair_patch, nm->cor.pair_patch.data(), nm->cor.pair_patch.size() * sizeof(int32_t));
  if (vals) {
    if (!nm->cor.vals.empty()) {
      std::memcpy(vals, nm->cor.vals.data(), nm->cor.vals.size() * sizeof(double));
    } else if (nm->d_vals) {
      const size_t nq = (size_t)nm->gd.nc * nm->gd.nc;
      hipError_t e = hipMemcpy(vals, nm->d_vals, sizeof(double2) * 4 * nq * (size_t)*npairs, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return set_hip_error(e, "hipMemcpy");
    } else {
      return set_error(IFGF_ENOTPLANNED, "no correction values");
    }
  }
  return IFGF_OK;
}

int nmuller_plan_info(nmuller_t nm, double* info, int cap) {
  clear_error();
  if (!nm || !info) return set_error(IFGF_EINVAL, "null argument");
  if (cap < 4) return set_error(IFGF_EINVAL, "info needs 4 entries");
  const double npairs = nm->cor.row_off.empty() ? 0.0 : (double)nm->cor.row_off.back();
  info[0] = nm->cor_on_device;
  info[1] = nm->cor_seconds;
  info[2] = npairs;
  info[3] = npairs * 4.0 * nm->geo.nc * nm->geo.nc * 16.0;
  return IFGF_OK;
}

int nmuller_set_preconditioner(nmuller_t nm, const float* params, const int* dims, int nlayers, int dtype) {
  clear_error();
  if (!nm) return set_error(IFGF_EINVAL, "null argument");
  if (nm->host_only) return set_error(IFGF_ENOTPLANNED, "plan was built with host_only");
  nm->pc.reset();
  if (!params) return IFGF_OK;
  std::unique_ptr<ifgf::Precond> pc(new (std::nothrow) ifgf::Precond());
  if (!pc) return set_error(IFGF_ENOMEM, "host allocation failed");
  const nmuller_params& p = nm->prm;
  std::vector<float> feat = ifgf::patch_features(p.P, p.Nc, nm->geo.x.data(), nm->geo.nrm.data(), nm->mat.ke,
                                                 nm->mat.ki, p.eps_i / p.eps_e);
  int rc = ifgf::precond_create(*pc, p.P, p.Nc, feat, 2.0 / (p.mu_e + p.mu_i), 2.0 / (p.eps_e + p.eps_i),
                                params, dims, nlayers, dtype);
  if (rc) return rc;
  nm->pc = std::move(pc);
  return IFGF_OK;
}

int nmuller_precond_apply(nmuller_t nm, const void* v, void* z, int nvec, void* stream) {
  clear_error();
  if (!nm || !v || !z) return set_error(IFGF_EINVAL, "null argument");
  if (!nm->pc) return set_error(IFGF_ENOTPLANNED, "no preconditioner set");
  if (nvec < 1) return set_error(IFGF_EINVAL, "nvec must be >= 1");
  if (v == z) return set_error(IFGF_EINVAL, "z must not alias v");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t m = 4 * nm->gd.n;
  for (int i = 0; i < nvec; ++i) {
    hipError_t e = ifgf::precond_apply(*nm->pc, static_cast<const double2*>(v) + i * m,
                                       static_cast<double2*>(z) + i * m, st);
    if (e != hipSuccess) return set_hip_error(e, "preconditioner apply");
  }
  return IFGF_OK;
}

int nmuller_precond_pairs(nmuller_t nm, const void* R, const void* E, int npairs, float* X, float* T,
                          void* stream) {
  clear_error();
  if (!nm || !R || !E || !X || !T) return set_error(IFGF_EINVAL, "null argument");
  if (!nm->pc) return set_error(IFGF_ENOTPLANNED, "no preconditioner set (it fixes the feature layout)");
  if (npairs < 1) return set_error(IFGF_EINVAL, "npairs must be >= 1");
  hipError_t e = ifgf::precond_pairs(*nm->pc, static_cast<const double2*>(R), static_cast<const double2*>(E),
                                     npairs, X, T, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "preconditioner pairs");
}

int nmuller_patch_features(nmuller_t nm, float* buf, int64_t cap) {
  clear_error();
  if (!nm || !buf) return set_error(IFGF_EINVAL, "null argument");
  const nmuller_params& p = nm->prm;
  std::vector<float> f = ifgf::patch_features(p.P, p.Nc, nm->geo.x.data(), nm->geo.nrm.data(), nm->mat.ke,
                                              nm->mat.ki, p.eps_i / p.eps_e);
  if (cap < (int64_t)f.size()) return set_error(IFGF_EINVAL, "buffer too small");
  std::memcpy(buf, f.data(), f.size() * sizeof(float));
  return IFGF_OK;
}

ifgf_plan_t nmuller_ifgf(nmuller_t nm) { return nm ? nm->ifgf : nullptr; }

void nmuller_destroy(nmuller_t nm) { delete nm; }

}  // extern "C"
