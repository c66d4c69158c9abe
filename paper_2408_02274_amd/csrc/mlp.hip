// Learned-preconditioner network on the device: matrix products on the
// matrix cores (MFMA 16x16x16 BF16 or 16x16x4 FP32 operands, FP32
// accumulation), ReLU, mean-squared loss, Adam.  Project addition: the
// paper solves with plain GMRES (Sec. III-A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ifgf.h"
#include "mlp.hpp"
#include "util.hpp"

using namespace ifgf;

struct mlp_s {
  MlpNet net;
};

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

// round to nearest even on the upper 16 bits of the FP32 pattern
__device__ __forceinline__ bf16_t to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

template <class T> struct Op;
template <> struct Op<bf16_t> {
  static constexpr int kStep = 16;
  static constexpr int kPad = 8;
  __device__ static bf16_t q(float f) { return to_bf16(f); }
};
template <> struct Op<float> {
  static constexpr int kStep = 4;
  static constexpr int kPad = 4;
  __device__ static float q(float f) { return f; }
};

constexpr int BM = 64, BN = 64, BK = 32;

// C[m][n] = act(sum_k A(m,k) B(k,n) + bias[n]) with A(m,k) = A[m sam + k sak]
// and B(k,n) = B[k sbk + n sbn]; C FP32 with leading dimension ldc, Cq the
// operand-type copy (optional).  256 threads: four waves, each a 32 x 32
// quadrant of the 64 x 64 block as 2 x 2 MFMA tiles.
template <class T>
__global__ void __launch_bounds__(256) k_gemm(const T* __restrict__ A, int64_t sam, int64_t sak,
                                              const T* __restrict__ B, int64_t sbk, int64_t sbn,
                                              int M, int N, int K, const float* __restrict__ bias,
                                              int relu, float* __restrict__ C, int64_t ldc,
                                              T* __restrict__ Cq) {
  constexpr int LD = BK + Op<T>::kPad;
  __shared__ __align__(16) T As[BM * LD];
  __shared__ __align__(16) T Bs[BN * LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int r16 = lane & 15, grp = lane >> 4;
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int j = 0; j < (BM * BK) / 256; ++j) {
      const int e = tid + 256 * j;
      int m, k;
      if (sak == 1) { k = e % BK; m = e / BK; } else { m = e % BM; k = e / BM; }
      const int gm = m0 + m, gk = k0 + k;
      As[m * LD + k] = (gm < M && gk < K) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : T(0);
    }
#pragma unroll
    for (int j = 0; j < (BN * BK) / 256; ++j) {
      const int e = tid + 256 * j;
      int n, k;
      if (sbk == 1) { k = e % BK; n = e / BK; } else { n = e % BN; k = e / BN; }
      const int gn = n0 + n, gk = k0 + k;
      Bs[n * LD + k] = (gn < N && gk < K) ? B[(int64_t)gk * sbk + (int64_t)gn * sbn] : T(0);
    }
    __syncthreads();
    if constexpr (sizeof(T) == 2) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        s4v a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
          a[i] = *reinterpret_cast<const s4v*>(&As[(wm + 16 * i + r16) * LD + kk + 4 * grp]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
          b[j] = *reinterpret_cast<const s4v*>(&Bs[(wn + 16 * j + r16) * LD + kk + 4 * grp]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[(wm + 16 * i + r16) * LD + kk + grp];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[(wn + 16 * j + r16) * LD + kk + grp];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + wm + 16 * i + 4 * grp + t, gn = n0 + wn + 16 * j + r16;
        if (gm < M && gn < N) {
          float v = acc[i][j][t];
          if (bias) v += bias[gn];
          if (relu) v = v > 0.f ? v : 0.f;
          C[(int64_t)gm * ldc + gn] = v;
          if (Cq) Cq[(int64_t)gm * ldc + gn] = Op<T>::q(v);
        }
      }
}

template <class T>
__global__ void __launch_bounds__(256) k_quant(const float* __restrict__ x, int64_t n, T* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = Op<T>::q(x[i]);
}

// out[b][:] = X[idx[b]][:] (FP32), outq its operand copy (optional)
template <class T>
__global__ void __launch_bounds__(256) k_gather_rows(const float* __restrict__ X, const int32_t* __restrict__ idx,
                                                     int B, int d, float* __restrict__ out, T* __restrict__ outq) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * d) return;
  const int b = (int)(i / d), c = (int)(i % d);
  const float v = X[(int64_t)idx[b] * d + c];
  if (out) out[i] = v;
  if (outq) outq[i] = Op<T>::q(v);
}

// g = g * (a > 0) where a is the layer's ReLU output; gq = q(g) (optional)
template <class T>
__global__ void __launch_bounds__(256) k_relu_back(float* __restrict__ g, const float* __restrict__ a, int64_t n,
                                                   T* __restrict__ gq) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = g[i];
  if (a && !(a[i] > 0.f)) v = 0.f;
  g[i] = v;
  if (gq) gq[i] = Op<T>::q(v);
}

// db[c] = sum_b g[b][c]
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ g, int B, int N, float* __restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += g[(int64_t)b * N + c];
  db[c] = s;
}

constexpr int kLossBlocks = 512;

// dY = 2 (Y - T) / n and per-block partial sums of (Y - T)^2
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                                             float* __restrict__ dY, float* __restrict__ part) {
  __shared__ float red[256];
  float s = 0.f;
  const float sc = 2.0f / (float)n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = Y[i] - T[i];
    s += d * d;
    dY[i] = sc * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_loss_final(const float* __restrict__ part, int nb, float inv,
                                                    float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv;
}

// Adam (Kingma & Ba 2015) with bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
template <class T>
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, T* __restrict__ pq, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  if (pq) pq[i] = Op<T>::q(pi);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class T>
hipError_t gemm(const void* A, int64_t sam, int64_t sak, const void* B, int64_t sbk, int64_t sbn, int M,
                int N, int K, const float* bias, int relu, float* C, int64_t ldc, void* Cq, hipStream_t st) {
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM));
  hipLaunchKernelGGL(k_gemm<T>, grid, dim3(256), 0, st, static_cast<const T*>(A), sam, sak,
                     static_cast<const T*>(B), sbk, sbn, M, N, K, bias, relu, C, ldc, static_cast<T*>(Cq));
  return hipGetLastError();
}

hipError_t gemm_any(bool bf16, const void* A, int64_t sam, int64_t sak, const void* B, int64_t sbk,
                    int64_t sbn, int M, int N, int K, const float* bias, int relu, float* C, int64_t ldc,
                    void* Cq, hipStream_t st) {
  return bf16 ? gemm<bf16_t>(A, sam, sak, B, sbk, sbn, M, N, K, bias, relu, C, ldc, Cq, st)
              : gemm<float>(A, sam, sak, B, sbk, sbn, M, N, K, bias, relu, C, ldc, Cq, st);
}

void quant_any(bool bf16, const float* x, int64_t n, void* y, hipStream_t st) {
  if (bf16)
    hipLaunchKernelGGL(k_quant<bf16_t>, dim3(nblk(n)), dim3(256), 0, st, x, n, static_cast<bf16_t*>(y));
  else
    hipLaunchKernelGGL(k_quant<float>, dim3(nblk(n)), dim3(256), 0, st, x, n, static_cast<float*>(y));
}

int maxdim(const MlpNet& net) {
  int d = 0;
  for (int x : net.dims) d = d > x ? d : x;
  return d;
}

// operand pointer of layer l's input (l >= 1)
const void* layer_in(const MlpNet& net, int l) { return net.aq[l]; }

}  // namespace

namespace ifgf {

int mlp_net_init(MlpNet& net, int nl, const int* dims, bool bf16, int max_batch) {
  if (nl < 1 || nl > 16 || !dims) return set_error(IFGF_EINVAL, "need 1..16 layers and their widths");
  for (int i = 0; i <= nl; ++i)
    if (dims[i] < 1 || dims[i] > 65536) return set_error(IFGF_EINVAL, "layer widths must lie in [1, 65536]");
  if (max_batch < 1 || max_batch > (1 << 20)) return set_error(IFGF_EINVAL, "max_batch must lie in [1, 2^20]");
  net.nl = nl;
  net.dims.assign(dims, dims + nl + 1);
  net.bf16 = bf16;
  net.max_batch = max_batch;
  net.woff.assign(nl, 0);
  int64_t o = 0;
  for (int l = 0; l < nl; ++l) {
    net.woff[l] = o;
    o += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
  }
  net.np = o;
  const size_t es = bf16 ? sizeof(bf16_t) : sizeof(float);
  DeviceArena& ar = net.ar;
  net.p32 = static_cast<float*>(ar.alloc(sizeof(float) * o));
  net.grad = static_cast<float*>(ar.alloc(sizeof(float) * o));
  net.m = static_cast<float*>(ar.alloc(sizeof(float) * o));
  net.v = static_cast<float*>(ar.alloc(sizeof(float) * o));
  net.pq = bf16 ? ar.alloc(es * o) : net.p32;
  if (!net.p32 || !net.grad || !net.m || !net.v || !net.pq)
    return set_error(IFGF_ENOMEM, "network parameter allocation failed");
  net.a32.assign(nl + 1, nullptr);
  net.aq.assign(nl + 1, nullptr);
  net.aq[0] = ar.alloc(es * (size_t)max_batch * dims[0]);
  if (!net.aq[0]) return set_error(IFGF_ENOMEM, "network activation allocation failed");
  for (int l = 1; l < nl; ++l) {
    net.a32[l] = static_cast<float*>(ar.alloc(sizeof(float) * (size_t)max_batch * dims[l]));
    net.aq[l] = bf16 ? ar.alloc(es * (size_t)max_batch * dims[l]) : net.a32[l];
    if (!net.a32[l] || !net.aq[l]) return set_error(IFGF_ENOMEM, "network activation allocation failed");
  }
  const size_t big = (size_t)max_batch * maxdim(net);
  net.g0 = static_cast<float*>(ar.alloc(sizeof(float) * big));
  net.g1 = static_cast<float*>(ar.alloc(sizeof(float) * big));
  net.gq = bf16 ? ar.alloc(es * big) : nullptr;
  net.out = static_cast<float*>(ar.alloc(sizeof(float) * (size_t)max_batch * dims[nl]));
  net.tgt = static_cast<float*>(ar.alloc(sizeof(float) * (size_t)max_batch * dims[nl]));
  net.part = static_cast<float*>(ar.alloc(sizeof(float) * (kLossBlocks + 1)));
  if (!net.g0 || !net.g1 || (bf16 && !net.gq) || !net.out || !net.tgt || !net.part)
    return set_error(IFGF_ENOMEM, "network workspace allocation failed");
  hipError_t e;
  if ((e = hipMemset(net.p32, 0, sizeof(float) * o)) != hipSuccess ||
      (e = hipMemset(net.m, 0, sizeof(float) * o)) != hipSuccess ||
      (e = hipMemset(net.v, 0, sizeof(float) * o)) != hipSuccess ||
      (e = hipMemset(net.grad, 0, sizeof(float) * o)) != hipSuccess ||
      (bf16 && (e = hipMemset(net.pq, 0, es * o)) != hipSuccess))
    return set_hip_error(e, "network initialisation");
  return 0;
}

// X == nullptr: the input rows were staged in aq[0] (and, in FP32, are the
// operand there).  Keeps what backward needs.
hipError_t mlp_net_forward(MlpNet& net, const float* X, int B, float* Y, hipStream_t st) {
  const int d0 = net.dims[0];
  const void* in = net.aq[0];
  if (X) {
    if (net.bf16) quant_any(true, X, (int64_t)B * d0, net.aq[0], st);
    else in = X;
  }
  net.in_op = in;
  net.last_B = B;
  for (int l = 0; l < net.nl; ++l) {
    const int K = net.dims[l], N = net.dims[l + 1];
    const bool last = l == net.nl - 1;
    const void* A = l == 0 ? in : layer_in(net, l);
    float* C = last ? (Y ? Y : net.out) : net.a32[l + 1];
    void* Cq = (!last && net.bf16) ? net.aq[l + 1] : nullptr;
    const char* W = static_cast<const char*>(net.pq) + net.woff[l] * (net.bf16 ? 2 : 4);
    hipError_t e = gemm_any(net.bf16, A, K, 1, W, N, 1, B, N, K, net.p32 + net.woff[l] + (int64_t)K * N,
                            last ? 0 : 1, C, N, Cq, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace ifgf

namespace ifgf {

hipError_t mlp_net_backward(MlpNet& net, const float* dY, int B, float* dX, hipStream_t st) {
  const bool bf = net.bf16;
  const size_t es = bf ? 2 : 4;
  float* gb[2] = {net.g0, net.g1};
  // the first input gradient is written to gb[cur ^ 1]: never over dY
  int cur = dY == net.g1 ? 1 : 0;
  for (int l = net.nl - 1; l >= 0; --l) {
    const int K = net.dims[l], N = net.dims[l + 1];
    const int64_t n = (int64_t)B * N;
    const float* g;      // FP32 signal at layer l's output (after the ReLU mask)
    const void* gop;     // its operand copy
    if (l == net.nl - 1) {
      g = dY;
      if (bf) {
        quant_any(true, dY, n, net.gq, st);
        gop = net.gq;
      } else {
        gop = dY;
      }
    } else {
      float* gm = gb[cur];
      if (bf)
        hipLaunchKernelGGL(k_relu_back<bf16_t>, dim3(nblk(n)), dim3(256), 0, st, gm, net.a32[l + 1], n,
                           static_cast<bf16_t*>(net.gq));
      else
        hipLaunchKernelGGL(k_relu_back<float>, dim3(nblk(n)), dim3(256), 0, st, gm, net.a32[l + 1], n,
                           static_cast<float*>(nullptr));
      g = gm;
      gop = bf ? net.gq : gm;
    }
    const void* in = l == 0 ? net.in_op : layer_in(net, l);
    float* gW = net.grad + net.woff[l];
    // dW = in^T g: rows K, columns N, summed over the batch
    hipError_t e = gemm_any(bf, in, 1, K, gop, N, 1, K, N, B, nullptr, 0, gW, N, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, st, g, B, N, gW + (int64_t)K * N);
    if (l > 0 || dX) {
      // dX = g W^T: rows B, columns K
      const char* W = static_cast<const char*>(net.pq) + net.woff[l] * es;
      float* out = l > 0 ? gb[cur ^ 1] : dX;
      if ((e = gemm_any(bf, gop, N, 1, W, 1, N, B, K, N, nullptr, 0, out, K, nullptr, st)) != hipSuccess)
        return e;
      cur ^= 1;
    }
  }
  return hipGetLastError();
}

hipError_t mlp_net_adam(MlpNet& net, float lr, hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  net.step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)net.step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)net.step)));
  if (net.bf16)
    hipLaunchKernelGGL(k_adam<bf16_t>, dim3(nblk(net.np)), dim3(256), 0, st, net.p32,
                       static_cast<bf16_t*>(net.pq), net.grad, net.m, net.v, net.np, lr, (float)b1, (float)b2,
                       1e-8f, c1, c2);
  else
    hipLaunchKernelGGL(k_adam<float>, dim3(nblk(net.np)), dim3(256), 0, st, net.p32, static_cast<float*>(nullptr),
                       net.grad, net.m, net.v, net.np, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

}  // namespace ifgf

extern "C" {

int mlp_create(mlp_t* out, int nlayers, const int* dims, int dtype, int max_batch) {
  clear_error();
  if (!out) return set_error(IFGF_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != MLP_BF16 && dtype != MLP_FP32) return set_error(IFGF_EINVAL, "dtype must be MLP_BF16 or MLP_FP32");
  mlp_s* p = new (std::nothrow) mlp_s();
  if (!p) return set_error(IFGF_ENOMEM, "host allocation failed");
  int rc = mlp_net_init(p->net, nlayers, dims, dtype == MLP_BF16, max_batch);
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return IFGF_OK;
}

int mlp_num_params(mlp_t p, int64_t* n) {
  clear_error();
  if (!p || !n) return set_error(IFGF_EINVAL, "null argument");
  *n = p->net.np;
  return IFGF_OK;
}

int mlp_set_params(mlp_t p, const float* params) {
  clear_error();
  if (!p || !params) return set_error(IFGF_EINVAL, "null argument");
  MlpNet& net = p->net;
  hipError_t e;
  if ((e = hipMemcpy(net.p32, params, sizeof(float) * net.np, hipMemcpyHostToDevice)) != hipSuccess)
    return set_hip_error(e, "mlp_set_params");
  if (net.bf16) quant_any(true, net.p32, net.np, net.pq, nullptr);
  if ((e = hipMemset(net.m, 0, sizeof(float) * net.np)) != hipSuccess ||
      (e = hipMemset(net.v, 0, sizeof(float) * net.np)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return set_hip_error(e, "mlp_set_params");
  net.step = 0;
  return IFGF_OK;
}

int mlp_get_params(mlp_t p, float* params, void* stream) {
  clear_error();
  if (!p || !params) return set_error(IFGF_EINVAL, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if ((e = hipMemcpyAsync(params, p->net.p32, sizeof(float) * p->net.np, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return set_hip_error(e, "mlp_get_params");
  return IFGF_OK;
}

int mlp_get_grad(mlp_t p, float* grad, void* stream) {
  clear_error();
  if (!p || !grad) return set_error(IFGF_EINVAL, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if ((e = hipMemcpyAsync(grad, p->net.grad, sizeof(float) * p->net.np, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return set_hip_error(e, "mlp_get_grad");
  return IFGF_OK;
}

int mlp_forward(mlp_t p, const float* X, int B, float* Y, void* stream) {
  clear_error();
  if (!p || !X || !Y) return set_error(IFGF_EINVAL, "null argument");
  if (B < 1 || B > p->net.max_batch) return set_error(IFGF_EINVAL, "batch must lie in [1, max_batch]");
  hipError_t e = mlp_net_forward(p->net, X, B, Y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "mlp_forward");
}

int mlp_backward(mlp_t p, const float* dY, int B, float* dX, void* stream) {
  clear_error();
  if (!p || !dY) return set_error(IFGF_EINVAL, "null argument");
  if (B != p->net.last_B || !p->net.in_op)
    return set_error(IFGF_EINVAL, "backward needs the batch of the preceding forward pass");
  hipError_t e = mlp_net_backward(p->net, dY, B, dX, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "mlp_backward");
}

int mlp_adam_step(mlp_t p, float lr, void* stream) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "null argument");
  if (!(lr > 0.f) || !std::isfinite(lr)) return set_error(IFGF_EINVAL, "lr must be finite and > 0");
  hipError_t e = mlp_net_adam(p->net, lr, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "mlp_adam_step");
}

int mlp_train_step(mlp_t p, const float* X, const float* T, const int32_t* idx, int B, float lr, float* loss,
                   void* stream) {
  clear_error();
  if (!p || !X || !T || !idx || !loss) return set_error(IFGF_EINVAL, "null argument");
  MlpNet& net = p->net;
  if (B < 1 || B > net.max_batch) return set_error(IFGF_EINVAL, "batch must lie in [1, max_batch]");
  if (!(lr > 0.f) || !std::isfinite(lr)) return set_error(IFGF_EINVAL, "lr must be finite and > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int d0 = net.dims[0], dL = net.dims[net.nl];
  const int64_t n0 = (int64_t)B * d0, nL = (int64_t)B * dL;
  if (net.bf16)
    hipLaunchKernelGGL(k_gather_rows<bf16_t>, dim3(nblk(n0)), dim3(256), 0, st, X, idx, B, d0, (float*)nullptr,
                       static_cast<bf16_t*>(net.aq[0]));
  else
    hipLaunchKernelGGL(k_gather_rows<float>, dim3(nblk(n0)), dim3(256), 0, st, X, idx, B, d0,
                       static_cast<float*>(net.aq[0]), (float*)nullptr);
  hipLaunchKernelGGL(k_gather_rows<float>, dim3(nblk(nL)), dim3(256), 0, st, T, idx, B, dL, net.tgt,
                     (float*)nullptr);
  hipError_t e = mlp_net_forward(net, nullptr, B, net.out, st);
  if (e != hipSuccess) return set_hip_error(e, "mlp_train_step forward");
  const int nb = (int)std::min<int64_t>(kLossBlocks, (nL + 255) / 256);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, net.out, net.tgt, nL, net.g1, net.part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, net.part, nb, 1.0f / (float)nL, loss);
  if ((e = mlp_net_backward(net, net.g1, B, nullptr, st)) != hipSuccess)
    return set_hip_error(e, "mlp_train_step backward");
  if ((e = mlp_net_adam(net, lr, st)) != hipSuccess) return set_hip_error(e, "mlp_train_step adam");
  return IFGF_OK;
}

void mlp_destroy(mlp_t p) { delete p; }

}  // extern "C"
