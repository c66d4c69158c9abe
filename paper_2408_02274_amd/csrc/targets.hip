// Sums at points other than the sources: off-surface field evaluation
// through the same IFGF (the paper's near-field maps, Sec. IV).
//
//   out[r][q][c][t]   = sum_m w_m phi_{r,c}(y_m) G_q(x_t, y_m),          c < 8
//   out[r][q][8+c][t] = sum_m w_m phi_{r,c}(y_m) d_t . grad G_q(x_t, y_m), c < 6
// for targets x_t and directions d_t.  The IFGF plan is built over the union
// of sources and targets (targets carry zero density), so every target gets
// the near sums of its neighbour leaves and the interpolated far field of its
// cousins at every level exactly as a source point would; no term is
// excluded, since no target coincides with a source (duplicates are refused).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ifgf.h"
#include "util.hpp"

using namespace ifgf;

struct ifgf_eval_s {
  ifgf_plan_t plan = nullptr;
  int64_t ns = 0, nt = 0;
  int max_nrhs = 1;
  DeviceArena arena;
  double2* udens = nullptr;   // [max_nrhs][8][ns + nt]
  double2* uout = nullptr;    // [max_nrhs][2][14][ns + nt]
  std::vector<double> unrm;   // union normals (sources: z, targets: directions)
  ~ifgf_eval_s() {
    if (plan) ifgf_destroy(plan);
  }
};

namespace {

__global__ void __launch_bounds__(256) k_pad(const double2* __restrict__ dens, int64_t ns, int64_t nu, int nrhs,
                                             double2* __restrict__ ud) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nrhs * 8 * nu) return;
  const int64_t row = i / nu, j = i % nu;
  ud[i] = j < ns ? dens[row * ns + j] : make_double2(0.0, 0.0);
}

__global__ void __launch_bounds__(256) k_extract(const double2* __restrict__ uo, int64_t ns, int64_t nt, int nrhs,
                                                 double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nrhs * 28 * nt) return;
  const int64_t row = i / nt, t = i % nt;
  out[i] = uo[row * (ns + nt) + ns + t];
}

int check_dirs(int64_t nt, const double* d) {
  for (int64_t t = 0; t < nt; ++t) {
    const double a = d[3 * t], b = d[3 * t + 1], c = d[3 * t + 2];
    if (!(std::fabs(std::sqrt(a * a + b * b + c * c) - 1.0) <= 1e-6))
      return set_error(IFGF_EINVAL, "target direction " + std::to_string(t) + " is not a unit vector");
  }
  return 0;
}

}  // namespace

extern "C" int ifgf_eval_plan(ifgf_eval_t* out, int64_t n_src, const double* src, const double* weights,
                              int64_t n_tgt, const double* tgt, const double* dirs, double k_int, double k_ext,
                              double tol, const ifgf_options* opt) {
  clear_error();
  if (!out) return set_error(IFGF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_src < 1 || n_tgt < 1 || !src || !weights || !tgt || !dirs)
    return set_error(IFGF_EINVAL, "need n_src, n_tgt >= 1 and all arrays");
  int rc = check_dirs(n_tgt, dirs);
  if (rc) return rc;
  ifgf_options o;
  ifgf_default_options(&o);
  if (opt) o = *opt;
  if (o.host_only) return set_error(IFGF_EINVAL, "host_only is not supported for evaluation plans");
  const int64_t nu = n_src + n_tgt;
  std::vector<double> x(3 * nu), w(nu, 1.0);
  auto* ev = new (std::nothrow) ifgf_eval_s();
  if (!ev) return set_error(IFGF_ENOMEM, "host allocation failed");
  ev->unrm.assign(3 * nu, 0.0);
  std::memcpy(x.data(), src, sizeof(double) * 3 * n_src);
  std::memcpy(x.data() + 3 * n_src, tgt, sizeof(double) * 3 * n_tgt);
  std::memcpy(w.data(), weights, sizeof(double) * n_src);
  for (int64_t i = 0; i < n_src; ++i) ev->unrm[3 * i + 2] = 1.0;   // source normals enter no output kept
  std::memcpy(ev->unrm.data() + 3 * n_src, dirs, sizeof(double) * 3 * n_tgt);
  if ((rc = ifgf_plan(&ev->plan, nu, x.data(), ev->unrm.data(), w.data(), k_int, k_ext, tol, &o))) {
    delete ev;
    return rc;
  }
  ev->ns = n_src;
  ev->nt = n_tgt;
  ev->max_nrhs = o.max_nrhs > 0 ? o.max_nrhs : 1;
  ev->udens = static_cast<double2*>(ev->arena.alloc(sizeof(double2) * (size_t)ev->max_nrhs * 8 * nu));
  ev->uout = static_cast<double2*>(ev->arena.alloc(sizeof(double2) * (size_t)ev->max_nrhs * 28 * nu));
  if (!ev->udens || !ev->uout) {
    delete ev;
    return set_error(IFGF_ENOMEM, "evaluation workspace allocation failed");
  }
  *out = ev;
  return IFGF_OK;
}

extern "C" int ifgf_eval_apply(ifgf_eval_t ev, const void* densities, int nrhs, void* out, void* stream) {
  clear_error();
  if (!ev || !densities || !out) return set_error(IFGF_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > ev->max_nrhs) return set_error(IFGF_EINVAL, "nrhs must lie in [1, max_nrhs]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nu = ev->ns + ev->nt;
  const int64_t w1 = (int64_t)nrhs * 8 * nu, w2 = (int64_t)nrhs * 28 * ev->nt;
  hipLaunchKernelGGL(k_pad, dim3((unsigned)((w1 + 255) / 256)), dim3(256), 0, st,
                     static_cast<const double2*>(densities), ev->ns, nu, nrhs, ev->udens);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_hip_error(e, "eval pad");
  int rc = ifgf_apply(ev->plan, ev->udens, nrhs, ev->uout, stream);
  if (rc) return rc;
  hipLaunchKernelGGL(k_extract, dim3((unsigned)((w2 + 255) / 256)), dim3(256), 0, st, ev->uout, ev->ns, ev->nt, nrhs,
                     static_cast<double2*>(out));
  e = hipGetLastError();
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "eval extract");
}

extern "C" int ifgf_eval_set_directions(ifgf_eval_t ev, const double* dirs) {
  clear_error();
  if (!ev || !dirs) return set_error(IFGF_EINVAL, "null argument");
  int rc = check_dirs(ev->nt, dirs);
  if (rc) return rc;
  std::memcpy(ev->unrm.data() + 3 * ev->ns, dirs, sizeof(double) * 3 * ev->nt);
  return ifgf_set_normals(ev->plan, ev->unrm.data());
}

extern "C" ifgf_plan_t ifgf_eval_ifgf(ifgf_eval_t ev) { return ev ? ev->plan : nullptr; }

extern "C" void ifgf_eval_destroy(ifgf_eval_t ev) { delete ev; }
