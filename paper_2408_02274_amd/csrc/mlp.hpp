// Device-resident multilayer perceptron (ReLU hidden layers, affine output)
// used as the learned FGMRES preconditioner.  Matrix products run on the
// matrix cores with BF16 (or FP32) operands and FP32 accumulation; master
// parameters, gradients and Adam moments are FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "util.hpp"

namespace ifgf {

struct MlpNet {
  int nl = 0;                 // layers
  std::vector<int> dims;      // nl + 1 widths
  bool bf16 = true;           // operand type of the matrix products
  int max_batch = 0;
  int64_t np = 0;             // parameters
  std::vector<int64_t> woff;  // offset of W_l in the flat vector (b_l follows)
  int64_t step = 0;           // Adam steps taken
  DeviceArena ar;
  float* p32 = nullptr;       // master parameters [np]
  void* pq = nullptr;         // operand copy of the parameters [np] (bf16 or = p32)
  float* grad = nullptr;      // [np]
  float *m = nullptr, *v = nullptr;
  std::vector<float*> a32;    // a32[l]: FP32 activations entering layer l (l >= 1), [max_batch][dims[l]]
  std::vector<void*> aq;      // aq[l]: operand copy of the activations entering layer l
  float *g0 = nullptr, *g1 = nullptr;  // back-propagated signal, FP32 ping-pong
  void* gq = nullptr;         // its operand copy
  float* tgt = nullptr;       // gathered training targets [max_batch][dims[nl]]
  float* out = nullptr;       // output of the last layer [max_batch][dims[nl]]
  float* part = nullptr;      // loss partial sums
  const void* in_op = nullptr;  // layer-0 operand of the last forward pass
  int last_B = 0;               // its batch size
};

// Create the network; parameters are zero until set.  Returns a status code.
int mlp_net_init(MlpNet& net, int nlayers, const int* dims, bool bf16, int max_batch);

// Y = net(X) for X device FP32 [B][dims[0]], Y device FP32 [B][dims[nl]]
// (Y may be null: the output stays in net.out).  Keeps the activations.
hipError_t mlp_net_forward(MlpNet& net, const float* X, int B, float* Y, hipStream_t st);

// Gradient of a loss with respect to the parameters (into net.grad) and,
// if dX is not null, to the input, given dY [B][dims[nl]] for the batch of
// the last forward pass.  dY is not modified.
hipError_t mlp_net_backward(MlpNet& net, const float* dY, int B, float* dX, hipStream_t st);

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) from net.grad.
hipError_t mlp_net_adam(MlpNet& net, float lr, hipStream_t st);

}  // namespace ifgf
