// Device-side plan layout shared by the HIP kernels and the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ifgf {

constexpr int kNS = 8;          // densities with single-layer sums
constexpr int kND = 6;          // densities with normal-derivative sums
constexpr int kCols = 2 * kNS;  // complex columns per cone point (8 densities x 2 kernels)
constexpr int kOut = 2 * (kNS + kND);  // complex outputs per point

// Interpolation constants: Chebyshev nodes on [-1,1] and Lagrange
// denominators 1 / prod_{m != j} (x_j - x_m).
struct InterpC {
  int Ps, Pa, npts;
  double xs[8], xa[8], ws[8], wa[8];
  float xsf[8], xaf[8], wsf[8], waf[8];   // the same in FP32
};

struct DevLevel {
  int d = 0;
  double h = 0.0;
  int ns = 0, na = 0;
  int64_t nb = 0, nslots = 0;
  double* centers = nullptr;      // [nb][3]
  int32_t* start = nullptr;       // [nb]
  int32_t* end = nullptr;         // [nb]
  int32_t* child_start = nullptr; // [nb] (levels < D)
  int32_t* child_end = nullptr;
  int32_t* nbr_off = nullptr;     // leaf level only
  int32_t* nbr = nullptr;
  int32_t* slot_box = nullptr;    // [nslots]
  int32_t* slot_cone = nullptr;
  int64_t* tp_off = nullptr;      // [n+1]
  int32_t* tp_slot = nullptr;
  int64_t* pp_off = nullptr;      // [nslots+1] (propagation into this level)
  int32_t* pp_slot = nullptr;
};

// Kernel launchers (FP64 path).  All arrays in Morton-sorted point order.
hipError_t launch_gather_weighted(const double2* dens, const int64_t* perm, const double* w,
                                  int64_t n, double2* a, hipStream_t st);
hipError_t launch_near(const DevLevel& leaf, const int32_t* leaf_of_point, const double* xs,
                       const double* nrm, const double2* a, int64_t n, double k0, double k1,
                       double2* out_s, hipStream_t st);
hipError_t launch_leaf(const DevLevel& leaf, const InterpC& ic, const double* xs,
                       const double2* a, double k0, double k1, double2* vals, hipStream_t st);
hipError_t launch_targets(const DevLevel& L, const InterpC& ic, const double* xs,
                          const double* nrm, int64_t n, double k0, double k1,
                          const double2* vals, double2* out_s, hipStream_t st);
hipError_t launch_propagate(const DevLevel& child, const DevLevel& parent, const InterpC& ic,
                            double k0, double k1, const double2* vals_child,
                            double2* vals_parent, hipStream_t st);
hipError_t launch_scatter_out(const double2* out_s, const int64_t* perm, int64_t n,
                              double2* out, hipStream_t st);

}  // namespace ifgf

// Per-kernel timing hooks of a plan (no-ops unless ifgf_set_timing(plan, 1)).
struct ifgf_plan_s;
namespace ifgf {
hipEvent_t timer_begin(ifgf_plan_s* p, hipStream_t st);
void timer_end(ifgf_plan_s* p, const char* name, hipEvent_t ev, hipStream_t st, double units);
bool timing_on(ifgf_plan_s* p);   // per-kernel timing switched on
bool plan_verbose(ifgf_plan_s* p);   // built with the verbose option
}  // namespace ifgf
