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
//
// Each right-hand side is a resumable solve that stops at every operator
// product it needs; several right-hand sides advance in lock-step and the
// products of one step are performed as batched applies.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <complex>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/ifgf.h"
#include "device.hpp"
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

  // bytes of the workspaces below for a basis of nbasis vectors, each array
  // starting on a 256-byte boundary
  static size_t workspace_bytes(int64_t m, int nbasis, bool flexible) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t v = sizeof(double2) * (size_t)m;
    return up(v * (nbasis + 1)) + (flexible ? up(v * nbasis) : 0) + 2 * up(v) +
           up(sizeof(double2) * (size_t)kDotBlocks * (nbasis + 2)) + 2 * up(sizeof(double2) * (size_t)(nbasis + 2));
  }
  // the same workspaces carved from caller-provided device memory (no allocation)
  int init_in(char* base, size_t cap, int nbasis, bool flexible) {
    if (workspace_bytes(m, nbasis, flexible) > cap)
      return set_error(IFGF_EINVAL, "GMRES workspace of " + std::to_string(workspace_bytes(m, nbasis, flexible)) +
                                        " bytes exceeds the " + std::to_string(cap) +
                                        "-byte static scratch; lower restart or the problem size");
    basis = nbasis;
    auto take = [&](size_t bytes) {
      double2* p = reinterpret_cast<double2*>(base);
      base += (bytes + 255) & ~(size_t)255;
      return p;
    };
    const size_t v = sizeof(double2) * (size_t)m;
    V = take(v * (basis + 1));
    if (flexible) Z = take(v * basis);
    w = take(v);
    tmp = take(v);
    part = take(sizeof(double2) * (size_t)kDotBlocks * (basis + 2));
    h = take(sizeof(double2) * (size_t)(basis + 2));
    coef = take(sizeof(double2) * (size_t)(basis + 2));
    return 0;
  }
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

// The operator product a solve needs next: dst = A src, with the FP64 form
// of the operator (true residuals) or its working form (Arnoldi).
struct Req {
  const double2* src = nullptr;
  double2* dst = nullptr;
  bool fp64 = false;
};

// One right-hand side as a resumable FGMRES: start() and resume() run the
// solve up to its next operator product and return that product as a
// request; the caller performs it (alone or batched with other solves) and
// calls resume().  Every step of the algorithm lives here, so a lone solve
// and a lock-step batch of solves run the same arithmetic.
class Fgmres {
 public:
  Fgmres(Solver& S, const double2* b, double2* x, double rtol, int maxit, bool precond, Recorder* rec,
         bool fp64_residual)
      : S_(S), b_(b), x_(x), rtol_(rtol), maxit_(maxit), rec_(rec), fp64_res_(fp64_residual),
        basis_(S.basis), H_((size_t)(S.basis + 1) * S.basis), cs_(S.basis), sn_(S.basis), g_(S.basis + 1),
        hv_(S.basis + 2) {
    pc_ = precond ? nmuller_precond(S.nm) : nullptr;
    net_ = pc_ != nullptr;
    verbose_ = plan_verbose(nmuller_ifgf(S.nm));
  }

  int start(Req* req, bool* done) {
    t0_ = std::chrono::steady_clock::now();
    int rc;
    if ((rc = S_.norm(b_, &bnorm_))) return rc;
    if (bnorm_ == 0.0) {
      hipLaunchKernelGGL(k_fill, dim3(nblk(S_.m)), dim3(kBS), 0, S_.st, x_, S_.m);
      return finish(done);
    }
    return request_residual(req, done);
  }

  int resume(Req* req, bool* done) {
    return phase_ == kResidual ? after_residual(req, done) : after_arnoldi(req, done);
  }

  const ifgf_solve_info& info() const { return inf_; }

 private:
  enum Phase { kResidual, kArnoldi };

  // Each cycle starts from the true residual tmp = b - A x (FP64 form when
  // fp64_res_), which alone decides convergence; the Arnoldi process may run
  // on the FP32 operator.
  int request_residual(Req* req, bool* done) {
    phase_ = kResidual;
    *req = Req{x_, S_.tmp, fp64_res_};
    *done = false;
    return 0;
  }

  int after_residual(Req* req, bool* done) {
    hipLaunchKernelGGL(k_axpy, dim3(nblk(S_.m)), dim3(kBS), 0, S_.st, make_double2(-1.0, 0.0), S_.tmp, b_,
                       S_.tmp, S_.m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_hip_error(e, "gmres residual");
    double beta = 0.0;
    int rc;
    if ((rc = S_.norm(S_.tmp, &beta))) return rc;
    truerel_ = beta / bnorm_;
    est_ = truerel_;
    if (truerel_ <= rtol_ || total_ >= maxit_) return finish(done);
    hipLaunchKernelGGL(k_axpy, dim3(nblk(S_.m)), dim3(kBS), 0, S_.st, make_double2(1.0 / beta, 0.0), S_.tmp,
                       (const double2*)nullptr, S_.V, S_.m);
    std::fill(g_.begin(), g_.end(), cd(0.0));
    g_[0] = beta;
    hist_.assign(1, truerel_);
    flex_ = pc_ != nullptr;
    abandon_ = false;
    k_ = 0;
    return request_column(req, done);
  }

  // column k of the cycle: z_k = M(v_k) when flexible, then w = A z_k
  int request_column(Req* req, bool* done) {
    double2* Vk = S_.V + (int64_t)k_ * S_.m;
    const double2* src = Vk;
    if (flex_) {
      double2* Zk = S_.Z + (int64_t)k_ * S_.m;
      hipError_t e = ifgf::precond_apply(*pc_, Vk, Zk, S_.st, net_);
      if (e != hipSuccess) return set_hip_error(e, "preconditioner");
      src = Zk;
    }
    phase_ = kArnoldi;
    *req = Req{src, S_.w, false};
    *done = false;
    return 0;
  }

  int after_arnoldi(Req* req, bool* done) {
    const int k = k_;
    int rc;
    for (int pass = 0; pass < 2; ++pass) {   // CGS2
      hipError_t e = S_.dots(S_.V, k + 1, S_.w, S_.h);
      if (e != hipSuccess) return set_hip_error(e, "gmres dots");
      hipLaunchKernelGGL(k_orth_update, dim3(nblk(S_.m)), dim3(kBS), 0, S_.st, S_.V, S_.m, S_.h, k + 1, S_.w,
                         S_.m);
      std::vector<double2> hh(k + 1);
      if ((e = hipMemcpyAsync(hh.data(), S_.h, sizeof(double2) * (k + 1), hipMemcpyDeviceToHost, S_.st)) !=
              hipSuccess ||
          (e = hipStreamSynchronize(S_.st)) != hipSuccess)
        return set_hip_error(e, "gmres copy");
      for (int j = 0; j <= k; ++j) {
        cd v(hh[j].x, hh[j].y);
        hv_[j] = pass ? hv_[j] + v : v;
      }
    }
    double hn = 0.0;
    if ((rc = S_.norm(S_.w, &hn))) return rc;
    bool ok = std::isfinite(hn);
    for (int j = 0; j <= k && ok; ++j) ok = finite(hv_[j]);
    if (!ok) {
      if (flex_ && net_) {   // discard this column and switch the network off
        abandon_ = true;
        return end_cycle(req, done);
      }
      return set_error(IFGF_EINVAL, "non-finite vector in the Arnoldi process");
    }
    const int basis = basis_;
    for (int j = 0; j <= k; ++j) H_[(size_t)j * basis + k] = hv_[j];
    H_[(size_t)(k + 1) * basis + k] = hn;
    for (int i = 0; i < k; ++i) {
      cd a = H_[(size_t)i * basis + k], bb = H_[(size_t)(i + 1) * basis + k];
      H_[(size_t)i * basis + k] = std::conj(cs_[i]) * a + std::conj(sn_[i]) * bb;
      H_[(size_t)(i + 1) * basis + k] = -sn_[i] * a + cs_[i] * bb;
    }
    cd a = H_[(size_t)k * basis + k], bb = H_[(size_t)(k + 1) * basis + k];
    double den = std::sqrt(std::norm(a) + std::norm(bb));
    cs_[k] = den > 0 ? a / den : cd(1.0);
    sn_[k] = den > 0 ? bb / den : cd(0.0);
    H_[(size_t)k * basis + k] = den;
    H_[(size_t)(k + 1) * basis + k] = 0.0;
    g_[k + 1] = -sn_[k] * g_[k];
    g_[k] = std::conj(cs_[k]) * g_[k];
    est_ = std::abs(g_[k + 1]) / bnorm_;
    if (hn > 0.0)
      hipLaunchKernelGGL(k_axpy, dim3(nblk(S_.m)), dim3(kBS), 0, S_.st, make_double2(1.0 / hn, 0.0), S_.w,
                         (const double2*)nullptr, S_.V + (int64_t)(k + 1) * S_.m, S_.m);
    k_ = k + 1;
    ++total_;
    if (flex_ && net_) ++pc_iters_;
    hist_.push_back(est_);
    if (verbose_ && total_ % 20 == 0) std::fprintf(stderr, "[gmres] %d iterations, residual estimate %.3e\n", total_, est_);
    if (rec_ && rec_->count < rec_->cap && total_ % rec_->stride == 0 && (rc = record())) return rc;
    if (est_ <= rtol_ || hn == 0.0) return end_cycle(req, done);
    if (flex_ && net_ && k_ >= kStallWindow && !(est_ < kStallRatio * hist_[k_ - kStallWindow])) {
      abandon_ = true;
      return end_cycle(req, done);
    }
    if (k_ < basis_ && total_ < maxit_) return request_column(req, done);
    return end_cycle(req, done);
  }

  // y solving H y = g (upper triangular, first nk rows)
  std::vector<cd> hess_solve(int nk) const {
    std::vector<cd> yy(nk);
    for (int i = nk - 1; i >= 0; --i) {
      cd s = g_[i];
      for (int j = i + 1; j < nk; ++j) s -= H_[(size_t)i * basis_ + j] * yy[j];
      yy[i] = s / H_[(size_t)i * basis_ + i];
    }
    return yy;
  }

  // iterate x + B y and its residual V_{k+1} Q^H (0, .., 0, g_k)
  int record() {
    const int k = k_;
    std::vector<cd> yy = hess_solve(k), u(k + 1, cd(0.0));
    u[k] = g_[k];
    for (int i = k - 1; i >= 0; --i) {
      cd ui = u[i], ui1 = u[i + 1];
      u[i] = cs_[i] * ui - std::conj(sn_[i]) * ui1;
      u[i + 1] = sn_[i] * ui + std::conj(cs_[i]) * ui1;
    }
    double2* Xr = rec_->X + (int64_t)rec_->count * S_.m;
    double2* Rr = rec_->R + (int64_t)rec_->count * S_.m;
    hipLaunchKernelGGL(k_axpy, dim3(nblk(S_.m)), dim3(kBS), 0, S_.st, make_double2(1.0, 0.0), x_,
                       (const double2*)nullptr, Xr, S_.m);
    int rc;
    if ((rc = S_.combine(flex_ ? S_.Z : S_.V, yy, k, Xr, false)) || (rc = S_.combine(S_.V, u, k + 1, Rr, true)))
      return rc;
    rec_->count += 1;
    return 0;
  }

  // x += B y; a cycle abandoned by the network goes on with M = D^-1
  int end_cycle(Req* req, bool* done) {
    int rc;
    if (k_ > 0 && (rc = S_.combine(flex_ ? S_.Z : S_.V, hess_solve(k_), k_, x_, false))) return rc;
    if (abandon_) {
      net_ = false;
      ++fallbacks_;
    }
    return request_residual(req, done);
  }

  int finish(bool* done) {
    auto t1 = std::chrono::steady_clock::now();
    inf_.iters = total_;
    inf_.true_relres = truerel_;
    inf_.arnoldi_relres = est_;
    inf_.converged = truerel_ <= rtol_ ? 1 : 0;
    inf_.seconds = std::chrono::duration<double>(t1 - t0_).count();
    inf_.precond_iters = pc_iters_;
    inf_.fallbacks = fallbacks_;
    inf_.residual_fp64 = fp64_res_ ? 1 : 0;
    *done = true;
    return 0;
  }

  Solver& S_;
  const double2* b_;
  double2* x_;
  double rtol_;
  int maxit_;
  Recorder* rec_;
  bool fp64_res_;
  ifgf::Precond* pc_ = nullptr;
  bool net_ = false;   // network part of M in use
  int basis_;
  std::vector<cd> H_, cs_, sn_, g_, hv_;
  std::vector<double> hist_;
  bool verbose_ = false;
  double bnorm_ = 0.0, est_ = 0.0, truerel_ = 0.0;
  int total_ = 0, pc_iters_ = 0, fallbacks_ = 0, k_ = 0;
  bool flex_ = false, abandon_ = false;
  Phase phase_ = kResidual;
  std::chrono::steady_clock::time_point t0_;
  ifgf_solve_info inf_{};
};

// Perform the requests rs (all of one precision) as batched operator
// products: up to `cap` sources packed into P, one apply, results unpacked
// from Q.  A lone request is applied in place.
int apply_requests(nmuller_t nm, const std::vector<Req*>& rs, bool fp64, int cap, double2* P, double2* Q,
                   int64_t m, hipStream_t st) {
  if (rs.empty()) return 0;
  ifgf_plan_t ip = nmuller_ifgf(nm);
  int prev = IFGF_FP64;
  int rc = fp64 ? ifgf_set_precision(ip, IFGF_FP64, &prev) : 0;
  if (rc) return rc;
  const size_t vb = sizeof(double2) * (size_t)m;
  for (size_t c0 = 0; c0 < rs.size() && !rc; c0 += cap) {
    const int nb = (int)std::min<size_t>(cap, rs.size() - c0);
    if (nb == 1) {
      rc = nmuller_apply(nm, rs[c0]->src, 1, rs[c0]->dst, st);
      continue;
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < nb && e == hipSuccess; ++i)
      e = hipMemcpyAsync(P + (int64_t)i * m, rs[c0 + i]->src, vb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
      rc = set_hip_error(e, "gmres pack");
      break;
    }
    if ((rc = nmuller_apply(nm, P, nb, Q, st))) break;
    for (int i = 0; i < nb && e == hipSuccess; ++i)
      e = hipMemcpyAsync(rs[c0 + i]->dst, Q + (int64_t)i * m, vb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) rc = set_hip_error(e, "gmres unpack");
  }
  int rc2 = fp64 ? ifgf_set_precision(ip, prev, nullptr) : 0;
  return rc ? rc : rc2;
}

// A single solve driven to the end.
int run_one(Fgmres& G, nmuller_t nm, int64_t m, hipStream_t st) {
  Req r;
  bool done = false;
  int rc = G.start(&r, &done);
  while (!rc && !done) {
    std::vector<Req*> one{&r};
    if ((rc = apply_requests(nm, one, r.fp64, 1, nullptr, nullptr, m, st))) break;
    rc = G.resume(&r, &done);
  }
  return rc;
}

// Static scratch of nmuller_solve_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (its
// host-side name is not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kScratchBytes];

int scratch_ptr(char** out) {
  static std::mutex mu;
  static char* ptrs[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return set_error(IFGF_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
      return set_hip_error(e, "hipGetSymbolAddress(scratch)");
    ptrs[dev] = static_cast<char*>(p);
  }
  *out = ptrs[dev];
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
  // true residuals on the FP64 form when the plan holds its buffers
  const bool res64 = (ifgf_precisions(nmuller_ifgf(nm)) & 1) != 0;
  const int64_t m = 4 * n;
  const int basis = (restart > 0 && restart < maxit) ? restart : maxit;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Right-hand sides advance in lock-step groups: each step gathers the
  // pending operator products of the group's unconverged solves into
  // batched applies (converged solves drop out).  A group is as large as
  // half the free device memory allows for the solves' Krylov bases.
  const double per_solve = 16.0 * (double)m * ((basis + 1) + (precond ? basis : 0) + 2);
  size_t free_b = 0, total_b = 0;
  hipError_t e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return set_hip_error(e, "gmres memory query");
  const int cap = nmuller_max_rhs(nm);
  int group = (int)std::min<double>(nrhs, std::max(1.0, std::floor(0.5 * (double)free_b / per_solve)));
  int status = IFGF_OK;
  for (int r0 = 0; r0 < nrhs; r0 += group) {
    const int gn = std::min(group, nrhs - r0);
    std::vector<std::unique_ptr<Solver>> Ss(gn);
    std::vector<std::unique_ptr<Fgmres>> Gs(gn);
    for (int i = 0; i < gn; ++i) {
      Ss[i] = std::make_unique<Solver>();
      Ss[i]->nm = nm;
      Ss[i]->m = m;
      Ss[i]->st = st;
      if ((rc = Ss[i]->init(basis, precond))) return rc;
      const double2* b = static_cast<const double2*>(rhs) + (int64_t)(r0 + i) * m;
      double2* x = static_cast<double2*>(y) + (int64_t)(r0 + i) * m;
      if (!use_x0) hipLaunchKernelGGL(k_fill, dim3(nblk(m)), dim3(kBS), 0, st, x, m);
      Gs[i] = std::make_unique<Fgmres>(*Ss[i], b, x, rtol, maxit, precond, nullptr, res64);
    }
    if (gn == 1) {
      if ((rc = run_one(*Gs[0], nm, m, st))) return rc;
    } else {
      DeviceArena pack;
      const int nb = std::min(cap, gn);
      double2 *P = nullptr, *Q = nullptr;
      if (nb > 1) {
        P = static_cast<double2*>(pack.alloc(sizeof(double2) * (size_t)m * nb));
        Q = static_cast<double2*>(pack.alloc(sizeof(double2) * (size_t)m * nb));
        if (!P || !Q) return set_error(IFGF_ENOMEM, "GMRES batch buffers");
      }
      std::vector<Req> reqs(gn);
      std::vector<char> done(gn, 0);
      for (int i = 0; i < gn; ++i) {
        bool d = false;
        if ((rc = Gs[i]->start(&reqs[i], &d))) return rc;
        done[i] = d;
      }
      for (;;) {
        std::vector<Req*> r64, rwk;
        std::vector<int> act;
        for (int i = 0; i < gn; ++i)
          if (!done[i]) {
            act.push_back(i);
            (reqs[i].fp64 ? r64 : rwk).push_back(&reqs[i]);
          }
        if (act.empty()) break;
        if ((rc = apply_requests(nm, r64, true, cap, P, Q, m, st)) ||
            (rc = apply_requests(nm, rwk, false, cap, P, Q, m, st)))
          return rc;
        for (int i : act) {
          bool d = false;
          if ((rc = Gs[i]->resume(&reqs[i], &d))) return rc;
          done[i] = d;
        }
      }
    }
    for (int i = 0; i < gn; ++i) {
      if (info) info[r0 + i] = Gs[i]->info();
      if (!Gs[i]->info().converged) status = IFGF_WNOCONV;
    }
  }
  // a device-side failure of any apply makes the whole solve suspect
  if ((rc = ifgf_check(nmuller_ifgf(nm), stream, nullptr))) return rc;
  return status;
}

extern "C" int nmuller_solve_noalloc(nmuller_t nm, const void* rhs, void* y, int use_x0, double rtol, int maxit,
                                     int restart, ifgf_solve_info* info, void* stream) {
  clear_error();
  if (!nm || !rhs || !y) return set_error(IFGF_EINVAL, "null argument");
  if (!(rtol > 0.0) || maxit < 1) return set_error(IFGF_EINVAL, "need rtol > 0 and maxit >= 1");
  int64_t n = 0;
  int rc = solver_size(nm, &n);
  if (rc) return rc;
  char* base = nullptr;
  if ((rc = scratch_ptr(&base))) return rc;
  const bool precond = nmuller_precond(nm) != nullptr;
  Solver S;
  S.nm = nm;
  S.m = 4 * n;
  S.st = static_cast<hipStream_t>(stream);
  const int basis = (restart > 0 && restart < maxit) ? restart : maxit;
  if ((rc = S.init_in(base, kScratchBytes, basis, precond))) return rc;
  double2* x = static_cast<double2*>(y);
  if (!use_x0) hipLaunchKernelGGL(k_fill, dim3(nblk(S.m)), dim3(kBS), 0, S.st, x, S.m);
  Fgmres G(S, static_cast<const double2*>(rhs), x, rtol, maxit, precond, nullptr,
           (ifgf_precisions(nmuller_ifgf(nm)) & 1) != 0);
  if ((rc = run_one(G, nm, S.m, S.st))) return rc;
  if (info) *info = G.info();
  if ((rc = ifgf_check(nmuller_ifgf(nm), stream, nullptr))) return rc;
  return G.info().converged ? IFGF_OK : IFGF_WNOCONV;
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
  Fgmres G(S, static_cast<const double2*>(rhs), x, rtol, maxit, false, &rec, false);
  if ((rc = run_one(G, nm, S.m, S.st))) return rc;
  *nrec = rec.count;
  if (info) *info = G.info();
  if ((rc = ifgf_check(nmuller_ifgf(nm), stream, nullptr))) return rc;
  return G.info().converged ? IFGF_OK : IFGF_WNOCONV;
}
