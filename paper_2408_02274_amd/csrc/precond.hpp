// Learned FGMRES preconditioner of the N-Mueller system (project addition).
//
// z = M(v) acts patch by patch.  For patch p the network sees the 4 Nc^2
// complex entries of v on the patch's nodes (real parts and imaginary parts
// of the four tangential components, scaled by s = rms(v)) and four
// geometry features of the patch, and returns a correction c_p of the same
// layout:  z = D^-1 v + s c(v / s),  D = diag((mu_e+mu_i)/2 I, (eps_e+eps_i)/2 I)
// the identity part of eq. n_muller.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/ifgf.h"
#include "mlp.hpp"
#include "util.hpp"

namespace ifgf {

constexpr int kPatchFeatures = 4;

struct Precond {
  MlpNet net;
  int P = 0, nq = 0;      // patches, nodes per patch
  int64_t n = 0;          // points
  double dm = 1.0, dj = 1.0;
  DeviceArena ar;
  float* feat = nullptr;  // [P][kPatchFeatures]
  float* X = nullptr;     // network input [P][8 nq + kPatchFeatures]
  double* part = nullptr; // norm partial sums
  double* s = nullptr;    // scale of the current vector
};

// Per-patch features: kappa_e d / 2pi, kappa_i d / 2pi, twice the largest
// angle between a node normal and the patch's mean normal, eps_i / eps_e / 10;
// d = diagonal of the patch's node bounding box.  x, nrm [n][3], patch-major.
std::vector<float> patch_features(int P, int Nc, const double* x, const double* nrm, double ke, double ki,
                                  double eps_ratio);

// Build from host parameters (layout of mlp_set_params).
int precond_create(Precond& pc, int P, int Nc, const std::vector<float>& feat, double dm, double dj,
                   const float* params, const int* dims, int nlayers, int dtype);

// z = M(v), v and z device [4][n] complex FP64 (z may not alias v); with
// net = false the network is left out: z = D^-1 v.
hipError_t precond_apply(Precond& pc, const double2* v, double2* z, hipStream_t st, bool net = true);

// Training rows from (residual, error) pairs: X [npairs P][8 nq + 4] and
// T [npairs P][8 nq] with T = pack((E - D^-1 R) / rms(R)).
hipError_t precond_pairs(Precond& pc, const double2* R, const double2* E, int npairs, float* X, float* T,
                         hipStream_t st);

}  // namespace ifgf

struct nmuller_s;
ifgf::Precond* nmuller_precond(nmuller_s* nm);
// right-hand sides one nmuller_apply may take (the operator's max_nrhs)
int nmuller_max_rhs(nmuller_s* nm);
