// GMRES on the N-Mueller system A y = b (Sec. III-A eq. lin_system; the
// paper's tolerance is 1e-4, Sec. IV).  Arnoldi in FP64 on the device with
// classical Gram-Schmidt applied twice; the small Hessenberg problem
// (Givens rotations, triangular solve) runs on the host.  Every restart
// cycle begins with the true residual ||b - A y|| / ||b|| from an FP64
// matvec, and only that residual ends the solve, so a plan whose IFGF runs
// in FP32 still converges to an FP64-verified tolerance.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/ifgf.h"
#include "util.hpp"

using namespace ifgf;

namespace {

constexpr int kDotBlocks = 240;
constexpr int kBS = 256;

// part[j * kDotBlocks + b] = sum over block b's strided range of conj(V_j) w
__global__ void __launch_bounds__(256) k_dots(const double2* __restrict__ V, int64_t ld, const double2* __restrict__ w,
                       int64_t m, double2* __restrict__ part) {
  __shared__ double sre[kBS], sim[kBS];
  const int j = blockIdx.y;
  const double2* v = V + (int64_t)j * ld;
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBS) {
    double2 a = v[i], b = w[i];
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int s = kBS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[j * gridDim.x + blockIdx.x] = make_double2(sre[0], sim[0]);
}

// h[j] = sum_b part[j][b]  (fixed order: deterministic)
__global__ void k_dots_final(const double2* __restrict__ part, int nb, int nj, double2* __restrict__ h) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nj) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < nb; ++b) {
    re += part[j * nb + b].x;
    im += part[j * nb + b].y;
  }
  h[j] = make_double2(re, im);
}

// w -= sum_j V_j h_j
__global__ void __launch_bounds__(256) k_orth_update(const double2* __restrict__ V, int64_t ld, const double2* __restrict__ h,
                              int nj, double2* __restrict__ w, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double re = w[i].x, im = w[i].y;
  for (int j = 0; j < nj; ++j) {
    double2 v = V[(int64_t)j * ld + i], c = h[j];
    re -= v.x * c.x - v.y * c.y;
    im -= v.x * c.y + v.y * c.x;
  }
  w[i] = make_double2(re, im);
}

// out = a * x + y (complex a; y may be null)
__global__ void __launch_bounds__(256) k_axpy(double2 a, const double2* __restrict__ x, const double2* __restrict__ y,
                       double2* __restrict__ out, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double2 v = x[i];
  double re = a.x * v.x - a.y * v.y, im = a.x * v.y + a.y * v.x;
  if (y) {
    re += y[i].x;
    im += y[i].y;
  }
  out[i] = make_double2(re, im);
}

// x += sum_j V_j c_j
__global__ void __launch_bounds__(256) k_combine(const double2* __restrict__ V, int64_t ld, const double2* __restrict__ c,
                          int nj, double2* __restrict__ x, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double re = x[i].x, im = x[i].y;
  for (int j = 0; j < nj; ++j) {
    double2 v = V[(int64_t)j * ld + i], a = c[j];
    re += v.x * a.x - v.y * a.y;
    im += v.x * a.y + v.y * a.x;
  }
  x[i] = make_double2(re, im);
}

__global__ void __launch_bounds__(256) k_fill(double2* __restrict__ x, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = make_double2(0.0, 0.0);
}

inline unsigned nblk(int64_t m) { return (unsigned)((m + kBS - 1) / kBS); }

using cd = std::complex<double>;

struct Solver {
  nmuller_t nm;
  int64_t m;       // 4n
  hipStream_t st;
  DeviceArena ar;
  double2 *V = nullptr, *w = nullptr, *part = nullptr, *h = nullptr, *tmp = nullptr;
  int maxbasis = 0;

  int init(int basis) {
    maxbasis = basis;
    V = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m * (basis + 1)));
    w = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m));
    tmp = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m));
    part = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)kDotBlocks * (basis + 2)));
    h = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)(basis + 2)));
    if (!V || !w || !tmp || !part || !h) return set_error(IFGF_ENOMEM, "GMRES workspace allocation failed");
    return 0;
  }
  hipError_t dots(const double2* Vb, int nj, const double2* x, double2* hout) {
    hipLaunchKernelGGL(k_dots, dim3(kDotBlocks, nj), dim3(kBS), 0, st, Vb, m, x, m, part);
    hipLaunchKernelGGL(k_dots_final, dim3((nj + 63) / 64), dim3(64), 0, st, part, kDotBlocks, nj, hout);
    return hipGetLastError();
  }
  int norm(const double2* x, double* out) {
    hipError_t e = dots(x, 1, x, h);
    if (e != hipSuccess) return set_hip_error(e, "gmres norm");
    double2 v;
    if ((e = hipMemcpyAsync(&v, h, sizeof(double2), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return set_hip_error(e, "gmres norm copy");
    *out = std::sqrt(std::max(0.0, v.x));
    return 0;
  }
  // tmp = b - A x with the FP64 form of the operator (a plan running its
  // FP32 form is switched for this one product and switched back)
  int residual(const double2* b, const double2* x) {
    ifgf_plan_t ip = nmuller_ifgf(nm);
    int prev = IFGF_FP64;
    int rc = ifgf_set_precision(ip, IFGF_FP64, &prev);
    if (rc) return rc;
    rc = nmuller_apply(nm, x, 1, tmp, st);
    int rc2 = ifgf_set_precision(ip, prev, nullptr);
    if (rc) return rc;
    if (rc2) return rc2;
    hipLaunchKernelGGL(k_axpy, dim3(nblk(m)), dim3(kBS), 0, st, make_double2(-1.0, 0.0), tmp, b, tmp, m);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : set_hip_error(e, "gmres residual");
  }
};

}  // namespace

extern "C" int nmuller_solve(nmuller_t nm, const void* rhs, int nrhs, void* y, int use_x0, double rtol,
                             int maxit, int restart, ifgf_solve_info* info, void* stream) {
  clear_error();
  if (!nm || !rhs || !y) return set_error(IFGF_EINVAL, "null argument");
  if (nrhs < 1) return set_error(IFGF_EINVAL, "nrhs must be >= 1");
  if (!(rtol > 0.0) || maxit < 1) return set_error(IFGF_EINVAL, "need rtol > 0 and maxit >= 1");
  int64_t n = 0;
  {
    int64_t c[1];
    int rc = ifgf_plan_counts(nmuller_ifgf(nm), c, 1);
    if (rc) return rc;
    n = c[0];
  }
  Solver S;
  S.nm = nm;
  S.m = 4 * n;
  S.st = static_cast<hipStream_t>(stream);
  const int basis = (restart > 0 && restart < maxit) ? restart : maxit;
  int rc = S.init(basis);
  if (rc) return rc;
  int status = IFGF_OK;
  std::vector<cd> H((size_t)(basis + 1) * basis), cs(basis), sn(basis), g(basis + 1), hv(basis + 2);
  for (int r = 0; r < nrhs; ++r) {
    auto t0 = std::chrono::steady_clock::now();
    const double2* b = static_cast<const double2*>(rhs) + (int64_t)r * S.m;
    double2* x = static_cast<double2*>(y) + (int64_t)r * S.m;
    if (!use_x0) hipLaunchKernelGGL(k_fill, dim3(nblk(S.m)), dim3(kBS), 0, S.st, x, S.m);
    double bnorm = 0.0;
    if ((rc = S.norm(b, &bnorm))) return rc;
    int total = 0;
    double est = 1.0, truerel = 0.0;
    if (bnorm == 0.0) {
      hipLaunchKernelGGL(k_fill, dim3(nblk(S.m)), dim3(kBS), 0, S.st, x, S.m);
      est = 0.0;
    }
    // Each cycle starts from the true FP64 residual, which alone decides
    // convergence; the Arnoldi process may run on the FP32 operator.
    while (bnorm > 0.0) {
      if ((rc = S.residual(b, x))) return rc;
      double beta = 0.0;
      if ((rc = S.norm(S.tmp, &beta))) return rc;
      truerel = beta / bnorm;
      if (truerel <= rtol || total >= maxit) break;
      hipLaunchKernelGGL(k_axpy, dim3(nblk(S.m)), dim3(kBS), 0, S.st, make_double2(1.0 / beta, 0.0), S.tmp,
                         (const double2*)nullptr, S.V, S.m);
      std::fill(g.begin(), g.end(), cd(0.0));
      g[0] = beta;
      int k = 0;
      for (; k < basis && total < maxit; ++k, ++total) {
        double2* Vk = S.V + (int64_t)k * S.m;
        if ((rc = nmuller_apply(nm, Vk, 1, S.w, S.st))) return rc;
        // CGS2
        for (int pass = 0; pass < 2; ++pass) {
          hipError_t e = S.dots(S.V, k + 1, S.w, S.h);
          if (e != hipSuccess) return set_hip_error(e, "gmres dots");
          hipLaunchKernelGGL(k_orth_update, dim3(nblk(S.m)), dim3(kBS), 0, S.st, S.V, S.m, S.h, k + 1,
                             S.w, S.m);
          std::vector<double2> hh(k + 1);
          if ((e = hipMemcpyAsync(hh.data(), S.h, sizeof(double2) * (k + 1), hipMemcpyDeviceToHost,
                                  S.st)) != hipSuccess ||
              (e = hipStreamSynchronize(S.st)) != hipSuccess)
            return set_hip_error(e, "gmres copy");
          for (int j = 0; j <= k; ++j) {
            cd v(hh[j].x, hh[j].y);
            hv[j] = pass ? hv[j] + v : v;
          }
        }
        double hn = 0.0;
        if ((rc = S.norm(S.w, &hn))) return rc;
        for (int j = 0; j <= k; ++j) H[(size_t)j * basis + k] = hv[j];
        H[(size_t)(k + 1) * basis + k] = hn;
        for (int i = 0; i < k; ++i) {
          cd a = H[(size_t)i * basis + k], bb = H[(size_t)(i + 1) * basis + k];
          H[(size_t)i * basis + k] = std::conj(cs[i]) * a + std::conj(sn[i]) * bb;
          H[(size_t)(i + 1) * basis + k] = -sn[i] * a + cs[i] * bb;
        }
        cd a = H[(size_t)k * basis + k], bb = H[(size_t)(k + 1) * basis + k];
        double den = std::sqrt(std::norm(a) + std::norm(bb));
        cs[k] = den > 0 ? a / den : cd(1.0);
        sn[k] = den > 0 ? bb / den : cd(0.0);
        H[(size_t)k * basis + k] = den;
        H[(size_t)(k + 1) * basis + k] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = std::conj(cs[k]) * g[k];
        est = std::abs(g[k + 1]) / bnorm;
        if (hn > 0.0)
          hipLaunchKernelGGL(k_axpy, dim3(nblk(S.m)), dim3(kBS), 0, S.st, make_double2(1.0 / hn, 0.0), S.w,
                             (const double2*)nullptr, S.V + (int64_t)(k + 1) * S.m, S.m);
        if (est <= rtol || hn == 0.0) {
          ++k;
          ++total;
          break;
        }
      }
      // x += V y with H y = g (upper triangular)
      std::vector<cd> yy(k);
      for (int i = k - 1; i >= 0; --i) {
        cd s = g[i];
        for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * basis + j] * yy[j];
        yy[i] = s / H[(size_t)i * basis + i];
      }
      std::vector<double2> yd(k);
      for (int i = 0; i < k; ++i) yd[i] = make_double2(yy[i].real(), yy[i].imag());
      hipError_t e;
      if ((e = hipMemcpyAsync(S.h, yd.data(), sizeof(double2) * k, hipMemcpyHostToDevice, S.st)) != hipSuccess)
        return set_hip_error(e, "gmres copy");
      hipLaunchKernelGGL(k_combine, dim3(nblk(S.m)), dim3(kBS), 0, S.st, S.V, S.m, S.h, k, x, S.m);
      if ((e = hipStreamSynchronize(S.st)) != hipSuccess) return set_hip_error(e, "gmres combine");
    }
    const double rn = truerel;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
      info[r].iters = total;
      info[r].true_relres = rn;
      info[r].arnoldi_relres = est;
      info[r].converged = rn <= rtol ? 1 : 0;
      info[r].seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    if (rn > rtol) status = IFGF_WNOCONV;
  }
  return status;
}
