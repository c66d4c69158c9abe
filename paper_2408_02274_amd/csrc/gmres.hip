// GMRES on the N-Mueller system A y = b (Sec. III-A eq. lin_system; the
// paper's tolerance is 1e-4, Sec. IV).  Arnoldi in FP64 on the device with
// classical Gram-Schmidt applied twice; the small Hessenberg problem
// (Givens rotations, triangular solve) runs on the host.  Every restart
// cycle begins with the true residual ||b - A y|| / ||b|| from an FP64
// matvec, and only that residual ends the solve, so a plan whose IFGF runs
// in FP32 still converges to an FP64-verified tolerance.
//
// With a learned preconditioner M = D^-1 + s c(v / s) set on the operator
// the iteration is flexible GMRES (Saad 1993): z_k = M(v_k), the basis of
// the update is kept, x += Z y.  A cycle whose network output is non-finite
// or that stalls (residual estimate down by less than 5% over 20
// iterations) is abandoned at its last good column and the solve goes on
// from that iterate with the network switched off, M = D^-1 (a
// "fallback").
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/ifgf.h"
#include "precond.hpp"
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

constexpr int kStallWindow = 20;
constexpr double kStallRatio = 0.95;

struct Solver {
  nmuller_t nm;
  int64_t m;       // 4n
  hipStream_t st;
  DeviceArena ar;
  double2 *V = nullptr, *Z = nullptr, *w = nullptr, *part = nullptr, *h = nullptr, *tmp = nullptr,
          *coef = nullptr;
  int basis = 0;

  int init(int nbasis, bool flexible) {
    basis = nbasis;
    V = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m * (basis + 1)));
    if (flexible) Z = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m * basis));
    w = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m));
    tmp = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)m));
    part = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)kDotBlocks * (basis + 2)));
    h = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)(basis + 2)));
    coef = static_cast<double2*>(ar.alloc(sizeof(double2) * (size_t)(basis + 2)));
    if (!V || (flexible && !Z) || !w || !tmp || !part || !h || !coef)
      return set_error(IFGF_ENOMEM, "GMRES workspace allocation failed");
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
  // FP32 form is switched for this one product and switched back), or with
  // the working form when fp64 is false
  int residual(const double2* b, const double2* x, bool fp64) {
    ifgf_plan_t ip = nmuller_ifgf(nm);
    int prev = IFGF_FP64;
    int rc = fp64 ? ifgf_set_precision(ip, IFGF_FP64, &prev) : 0;
    if (rc) return rc;
    rc = nmuller_apply(nm, x, 1, tmp, st);
    int rc2 = fp64 ? ifgf_set_precision(ip, prev, nullptr) : 0;
    if (rc) return rc;
    if (rc2) return rc2;
    hipLaunchKernelGGL(k_axpy, dim3(nblk(m)), dim3(kBS), 0, st, make_double2(-1.0, 0.0), tmp, b, tmp, m);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : set_hip_error(e, "gmres residual");
  }
  // out (+)= sum_j B_j c_j for host coefficients c (out zeroed first if init0)
  int combine(const double2* Bb, const std::vector<cd>& c, int nj, double2* out, bool init0) {
    std::vector<double2> cd2(nj);
    for (int i = 0; i < nj; ++i) cd2[i] = make_double2(c[i].real(), c[i].imag());
    hipError_t e;
    if ((e = hipMemcpyAsync(coef, cd2.data(), sizeof(double2) * nj, hipMemcpyHostToDevice, st)) != hipSuccess)
      return set_hip_error(e, "gmres copy");
    if (init0) hipLaunchKernelGGL(k_fill, dim3(nblk(m)), dim3(kBS), 0, st, out, m);
    hipLaunchKernelGGL(k_combine, dim3(nblk(m)), dim3(kBS), 0, st, Bb, m, coef, nj, out, m);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return set_hip_error(e, "gmres combine");
    return 0;
  }
};

// (x_k, r_k) pairs written every `stride` iterations of an unrestarted solve
struct Recorder {
  double2* X = nullptr;
  double2* R = nullptr;
  int cap = 0, stride = 1, count = 0;
};

bool finite(cd a) { return std::isfinite(a.real()) && std::isfinite(a.imag()); }

// One right-hand side.  Returns a status code; fills `inf`.
int solve_one(Solver& S, const double2* b, double2* x, double rtol, int maxit, bool precond, Recorder* rec,
              bool fp64_residual, ifgf_solve_info& inf) {
  auto t0 = std::chrono::steady_clock::now();
  ifgf::Precond* pc = precond ? nmuller_precond(S.nm) : nullptr;
  bool net = pc != nullptr;   // network part of M in use
  const int basis = S.basis;
  std::vector<cd> H((size_t)(basis + 1) * basis), cs(basis), sn(basis), g(basis + 1), hv(basis + 2);
  std::vector<double> hist;
  double bnorm = 0.0;
  int rc;
  if ((rc = S.norm(b, &bnorm))) return rc;
  int total = 0, pc_iters = 0, fallbacks = 0;
  double est = 0.0, truerel = 0.0;
  if (bnorm == 0.0) hipLaunchKernelGGL(k_fill, dim3(nblk(S.m)), dim3(kBS), 0, S.st, x, S.m);
  // Each cycle starts from the true FP64 residual, which alone decides
  // convergence; the Arnoldi process may run on the FP32 operator.
  while (bnorm > 0.0) {
    if ((rc = S.residual(b, x, fp64_residual))) return rc;
    double beta = 0.0;
    if ((rc = S.norm(S.tmp, &beta))) return rc;
    truerel = beta / bnorm;
    est = truerel;
    if (truerel <= rtol || total >= maxit) break;
    hipLaunchKernelGGL(k_axpy, dim3(nblk(S.m)), dim3(kBS), 0, S.st, make_double2(1.0 / beta, 0.0), S.tmp,
                       (const double2*)nullptr, S.V, S.m);
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    hist.assign(1, truerel);
    const bool flex = pc != nullptr;
    bool abandon = false;
    int k = 0;   // columns accepted in this cycle
    while (k < basis && total < maxit) {
      double2* Vk = S.V + (int64_t)k * S.m;
      const double2* src = Vk;
      if (flex) {
        double2* Zk = S.Z + (int64_t)k * S.m;
        hipError_t e = ifgf::precond_apply(*pc, Vk, Zk, S.st, net);
        if (e != hipSuccess) return set_hip_error(e, "preconditioner");
        src = Zk;
      }
      if ((rc = nmuller_apply(S.nm, src, 1, S.w, S.st))) return rc;
      for (int pass = 0; pass < 2; ++pass) {   // CGS2
        hipError_t e = S.dots(S.V, k + 1, S.w, S.h);
        if (e != hipSuccess) return set_hip_error(e, "gmres dots");
        hipLaunchKernelGGL(k_orth_update, dim3(nblk(S.m)), dim3(kBS), 0, S.st, S.V, S.m, S.h, k + 1, S.w, S.m);
        std::vector<double2> hh(k + 1);
        if ((e = hipMemcpyAsync(hh.data(), S.h, sizeof(double2) * (k + 1), hipMemcpyDeviceToHost, S.st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(S.st)) != hipSuccess)
          return set_hip_error(e, "gmres copy");
        for (int j = 0; j <= k; ++j) {
          cd v(hh[j].x, hh[j].y);
          hv[j] = pass ? hv[j] + v : v;
        }
      }
      double hn = 0.0;
      if ((rc = S.norm(S.w, &hn))) return rc;
      bool ok = std::isfinite(hn);
      for (int j = 0; j <= k && ok; ++j) ok = finite(hv[j]);
      if (!ok) {
        if (flex && net) {   // discard this column and switch the network off
          abandon = true;
          break;
        }
        return set_error(IFGF_EINVAL, "non-finite vector in the Arnoldi process");
      }
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
      ++k;
      ++total;
      if (flex && net) ++pc_iters;
      hist.push_back(est);
      if (rec && rec->count < rec->cap && total % rec->stride == 0) {
        // iterate x + B y and its residual V_{k+1} Q^H (0, .., 0, g_k)
        std::vector<cd> yy(k), u(k + 1, cd(0.0));
        for (int i = k - 1; i >= 0; --i) {
          cd s = g[i];
          for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * basis + j] * yy[j];
          yy[i] = s / H[(size_t)i * basis + i];
        }
        u[k] = g[k];
        for (int i = k - 1; i >= 0; --i) {
          cd ui = u[i], ui1 = u[i + 1];
          u[i] = cs[i] * ui - std::conj(sn[i]) * ui1;
          u[i + 1] = sn[i] * ui + std::conj(cs[i]) * ui1;
        }
        double2* Xr = rec->X + (int64_t)rec->count * S.m;
        double2* Rr = rec->R + (int64_t)rec->count * S.m;
        hipLaunchKernelGGL(k_axpy, dim3(nblk(S.m)), dim3(kBS), 0, S.st, make_double2(1.0, 0.0), x,
                           (const double2*)nullptr, Xr, S.m);
        if ((rc = S.combine(flex ? S.Z : S.V, yy, k, Xr, false)) || (rc = S.combine(S.V, u, k + 1, Rr, true)))
          return rc;
        rec->count += 1;
      }
      if (est <= rtol || hn == 0.0) break;
      if (flex && net && k >= kStallWindow && !(est < kStallRatio * hist[k - kStallWindow])) {
        abandon = true;
        break;
      }
    }
    if (k > 0) {
      // x += B y with H y = g (upper triangular)
      std::vector<cd> yy(k);
      for (int i = k - 1; i >= 0; --i) {
        cd s = g[i];
        for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * basis + j] * yy[j];
        yy[i] = s / H[(size_t)i * basis + i];
      }
      if ((rc = S.combine(flex ? S.Z : S.V, yy, k, x, false))) return rc;
    }
    if (abandon) {
      net = false;
      ++fallbacks;
    }
  }
  auto t1 = std::chrono::steady_clock::now();
  inf.iters = total;
  inf.true_relres = truerel;
  inf.arnoldi_relres = est;
  inf.converged = truerel <= rtol ? 1 : 0;
  inf.seconds = std::chrono::duration<double>(t1 - t0).count();
  inf.precond_iters = pc_iters;
  inf.fallbacks = fallbacks;
  return 0;
}

int solver_size(nmuller_t nm, int64_t* n) {
  int64_t c[1];
  int rc = ifgf_plan_counts(nmuller_ifgf(nm), c, 1);
  if (rc) return rc;
  *n = c[0];
  return 0;
}

}  // namespace

extern "C" int nmuller_solve(nmuller_t nm, const void* rhs, int nrhs, void* y, int use_x0, double rtol,
                             int maxit, int restart, ifgf_solve_info* info, void* stream) {
  clear_error();
  if (!nm || !rhs || !y) return set_error(IFGF_EINVAL, "null argument");
  if (nrhs < 1) return set_error(IFGF_EINVAL, "nrhs must be >= 1");
  if (!(rtol > 0.0) || maxit < 1) return set_error(IFGF_EINVAL, "need rtol > 0 and maxit >= 1");
  int64_t n = 0;
  int rc = solver_size(nm, &n);
  if (rc) return rc;
  const bool precond = nmuller_precond(nm) != nullptr;
  Solver S;
  S.nm = nm;
  S.m = 4 * n;
  S.st = static_cast<hipStream_t>(stream);
  if ((rc = S.init((restart > 0 && restart < maxit) ? restart : maxit, precond))) return rc;
  int status = IFGF_OK;
  for (int r = 0; r < nrhs; ++r) {
    const double2* b = static_cast<const double2*>(rhs) + (int64_t)r * S.m;
    double2* x = static_cast<double2*>(y) + (int64_t)r * S.m;
    if (!use_x0) hipLaunchKernelGGL(k_fill, dim3(nblk(S.m)), dim3(kBS), 0, S.st, x, S.m);
    ifgf_solve_info inf{};
    if ((rc = solve_one(S, b, x, rtol, maxit, precond, nullptr, true, inf))) return rc;
    if (info) info[r] = inf;
    if (!inf.converged) status = IFGF_WNOCONV;
  }
  return status;
}

extern "C" int nmuller_solve_trajectory(nmuller_t nm, const void* rhs, void* y, double rtol, int maxit, int stride,
                                        void* X, void* R, int cap, int* nrec, ifgf_solve_info* info,
                                        void* stream) {
  clear_error();
  if (!nm || !rhs || !y || !X || !R || !nrec) return set_error(IFGF_EINVAL, "null argument");
  if (!(rtol > 0.0) || maxit < 1 || stride < 1 || cap < 1)
    return set_error(IFGF_EINVAL, "need rtol > 0, maxit >= 1, stride >= 1, cap >= 1");
  int64_t n = 0;
  int rc = solver_size(nm, &n);
  if (rc) return rc;
  Solver S;
  S.nm = nm;
  S.m = 4 * n;
  S.st = static_cast<hipStream_t>(stream);
  if ((rc = S.init(maxit, false))) return rc;
  double2* x = static_cast<double2*>(y);
  hipLaunchKernelGGL(k_fill, dim3(nblk(S.m)), dim3(kBS), 0, S.st, x, S.m);
  Recorder rec;
  rec.X = static_cast<double2*>(X);
  rec.R = static_cast<double2*>(R);
  rec.cap = cap;
  rec.stride = stride;
  ifgf_solve_info inf{};
  if ((rc = solve_one(S, static_cast<const double2*>(rhs), x, rtol, maxit, false, &rec, false, inf))) return rc;
  *nrec = rec.count;
  if (info) *info = inf;
  return inf.converged ? IFGF_OK : IFGF_WNOCONV;
}
