// Learned FGMRES preconditioner: per-patch feature packing, the network
// pass and the unpacking into z = D^-1 v + s c(v / s) (project addition).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "precond.hpp"

namespace ifgf {

namespace {

constexpr int kNormBlocks = 240;

// part[b] = sum over block b's strided range of |v_i|^2
__global__ void __launch_bounds__(256) k_sq_part(const double2* __restrict__ v, int64_t m, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    const double2 a = v[i];
    s += a.x * a.x + a.y * a.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// s = sqrt(sum / m), or 1 for a zero vector
__global__ void k_rms(const double* __restrict__ part, int nb, int64_t m, double* __restrict__ s) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[b];
  const double r = sqrt(t / (double)m);
  s[0] = r > 0.0 ? r : 1.0;
}

// X[p][f]: f < 8 nq -> component (f / 2nq), real (f / nq even) or imaginary
// part of v at node p nq + f % nq, divided by s; then the patch features.
__global__ void __launch_bounds__(256) k_pack(const double2* __restrict__ v, int64_t n, int P, int nq,
                                              const double* __restrict__ s, const float* __restrict__ feat,
                                              float* __restrict__ X) {
  const int F = 8 * nq + kPatchFeatures;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)P * F) return;
  const int p = (int)(i / F), f = (int)(i % F);
  if (f >= 8 * nq) {
    X[i] = feat[p * kPatchFeatures + f - 8 * nq];
    return;
  }
  const int c = f / (2 * nq), ri = (f / nq) & 1, t = f % nq;
  const double2 a = v[(int64_t)c * n + (int64_t)p * nq + t];
  X[i] = (float)((ri ? a.y : a.x) / s[0]);
}

// z = D^-1 v + s (Y_re + i Y_im), or D^-1 v when Y is null
__global__ void __launch_bounds__(256) k_unpack(const double2* __restrict__ v, const float* __restrict__ Y, int64_t n,
                                                int nq, const double* __restrict__ s, double dm, double dj,
                                                double2* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * n) return;
  const int c = (int)(i / n);
  const int64_t l = i % n;
  const int64_t p = l / nq;
  const int t = (int)(l % nq);
  const double d = c < 2 ? dm : dj;
  const double2 a = v[i];
  if (!Y) {
    z[i] = make_double2(d * a.x, d * a.y);
    return;
  }
  const float* y = Y + p * 8 * nq + 2 * c * nq + t;
  const double sc = s[0];
  z[i] = make_double2(d * a.x + sc * (double)y[0], d * a.y + sc * (double)y[nq]);
}

// T[p][f] = component of (E - D^-1 R) / s in the layout of k_pack
__global__ void __launch_bounds__(256) k_pack_target(const double2* __restrict__ R, const double2* __restrict__ E,
                                                     int64_t n, int P, int nq, const double* __restrict__ s,
                                                     double dm, double dj, float* __restrict__ T) {
  const int F = 8 * nq;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)P * F) return;
  const int p = (int)(i / F), f = (int)(i % F);
  const int c = f / (2 * nq), ri = (f / nq) & 1, t = f % nq;
  const int64_t k = (int64_t)c * n + (int64_t)p * nq + t;
  const double d = c < 2 ? dm : dj;
  const double2 r = R[k], e = E[k];
  T[i] = (float)((ri ? e.y - d * r.y : e.x - d * r.x) / s[0]);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t rms(Precond& pc, const double2* v, hipStream_t st) {
  hipLaunchKernelGGL(k_sq_part, dim3(kNormBlocks), dim3(256), 0, st, v, 4 * pc.n, pc.part);
  hipLaunchKernelGGL(k_rms, dim3(1), dim3(64), 0, st, pc.part, kNormBlocks, 4 * pc.n, pc.s);
  return hipGetLastError();
}

}  // namespace

std::vector<float> patch_features(int P, int Nc, const double* x, const double* nrm, double ke, double ki,
                                  double eps_ratio) {
  const int nq = Nc * Nc;
  std::vector<float> f((size_t)P * kPatchFeatures);
  for (int p = 0; p < P; ++p) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, mn[3] = {0, 0, 0};
    for (int t = 0; t < nq; ++t) {
      const double* a = x + 3 * ((int64_t)p * nq + t);
      const double* b = nrm + 3 * ((int64_t)p * nq + t);
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], a[c]);
        hi[c] = std::max(hi[c], a[c]);
        mn[c] += b[c];
      }
    }
    const double d = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                               (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const double mnn = std::sqrt(mn[0] * mn[0] + mn[1] * mn[1] + mn[2] * mn[2]);
    double amax = 0.0;
    for (int t = 0; t < nq && mnn > 0.0; ++t) {
      const double* b = nrm + 3 * ((int64_t)p * nq + t);
      const double c = std::max(-1.0, std::min(1.0, (b[0] * mn[0] + b[1] * mn[1] + b[2] * mn[2]) / mnn));
      amax = std::max(amax, std::acos(c));
    }
    const double tp = 2.0 * 3.141592653589793;
    f[(size_t)p * kPatchFeatures + 0] = (float)(ke * d / tp);
    f[(size_t)p * kPatchFeatures + 1] = (float)(ki * d / tp);
    f[(size_t)p * kPatchFeatures + 2] = (float)(2.0 * amax);
    f[(size_t)p * kPatchFeatures + 3] = (float)(eps_ratio / 10.0);
  }
  return f;
}

int precond_create(Precond& pc, int P, int Nc, const std::vector<float>& feat, double dm, double dj,
                   const float* params, const int* dims, int nlayers, int dtype) {
  const int nq = Nc * Nc;
  if (!params || !dims || nlayers < 1) return set_error(IFGF_EINVAL, "preconditioner needs parameters and widths");
  if (dims[0] != 8 * nq + kPatchFeatures || dims[nlayers] != 8 * nq)
    return set_error(IFGF_EINVAL, "preconditioner widths must start at 8 Nc^2 + 4 and end at 8 Nc^2");
  if (dtype != MLP_BF16 && dtype != MLP_FP32) return set_error(IFGF_EINVAL, "dtype must be MLP_BF16 or MLP_FP32");
  int rc = mlp_net_init(pc.net, nlayers, dims, dtype == MLP_BF16, P);
  if (rc) return rc;
  pc.P = P;
  pc.nq = nq;
  pc.n = (int64_t)P * nq;
  pc.dm = dm;
  pc.dj = dj;
  pc.feat = static_cast<float*>(pc.ar.alloc(sizeof(float) * feat.size()));
  pc.X = static_cast<float*>(pc.ar.alloc(sizeof(float) * (size_t)P * dims[0]));
  pc.part = static_cast<double*>(pc.ar.alloc(sizeof(double) * kNormBlocks));
  pc.s = static_cast<double*>(pc.ar.alloc(sizeof(double) * 2));
  if (!pc.feat || !pc.X || !pc.part || !pc.s) return set_error(IFGF_ENOMEM, "preconditioner allocation failed");
  hipError_t e;
  if ((e = hipMemcpy(pc.feat, feat.data(), sizeof(float) * feat.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(pc.net.p32, params, sizeof(float) * pc.net.np, hipMemcpyHostToDevice)) != hipSuccess)
    return set_hip_error(e, "preconditioner upload");
  if (pc.net.bf16) {
    // operand copy of the weights: one pass of the network's own rounding
    std::vector<float> tmp(params, params + pc.net.np);
    std::vector<uint16_t> q(tmp.size());
    for (size_t i = 0; i < tmp.size(); ++i) {
      uint32_t u;
      std::memcpy(&u, &tmp[i], 4);
      u += 0x7FFFu + ((u >> 16) & 1u);
      q[i] = (uint16_t)(u >> 16);
    }
    if ((e = hipMemcpy(pc.net.pq, q.data(), 2 * q.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return set_hip_error(e, "preconditioner upload");
  }
  return 0;
}

hipError_t precond_apply(Precond& pc, const double2* v, double2* z, hipStream_t st, bool net) {
  if (!net) {
    hipLaunchKernelGGL(k_unpack, dim3(nblk(4 * pc.n)), dim3(256), 0, st, v, (const float*)nullptr, pc.n, pc.nq,
                       pc.s, pc.dm, pc.dj, z);
    return hipGetLastError();
  }
  hipError_t e = rms(pc, v, st);
  if (e != hipSuccess) return e;
  const int F = 8 * pc.nq + kPatchFeatures;
  hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)pc.P * F)), dim3(256), 0, st, v, pc.n, pc.P, pc.nq, pc.s, pc.feat,
                     pc.X);
  if ((e = mlp_net_forward(pc.net, pc.X, pc.P, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack, dim3(nblk(4 * pc.n)), dim3(256), 0, st, v, pc.net.out, pc.n, pc.nq, pc.s, pc.dm,
                     pc.dj, z);
  return hipGetLastError();
}

hipError_t precond_pairs(Precond& pc, const double2* R, const double2* E, int npairs, float* X, float* T,
                         hipStream_t st) {
  const int F = 8 * pc.nq + kPatchFeatures, FT = 8 * pc.nq;
  for (int i = 0; i < npairs; ++i) {
    const double2* r = R + (int64_t)i * 4 * pc.n;
    const double2* ee = E + (int64_t)i * 4 * pc.n;
    hipError_t e = rms(pc, r, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)pc.P * F)), dim3(256), 0, st, r, pc.n, pc.P, pc.nq, pc.s,
                       pc.feat, X + (int64_t)i * pc.P * F);
    hipLaunchKernelGGL(k_pack_target, dim3(nblk((int64_t)pc.P * FT)), dim3(256), 0, st, r, ee, pc.n, pc.P, pc.nq,
                       pc.s, pc.dm, pc.dj, T + (int64_t)i * pc.P * FT);
  }
  return hipGetLastError();
}

}  // namespace ifgf
