// Near-field corrections built on the device (Sec. III-B eq. patch_sing,
// Sec. III-D, Sec. III-H), from the same tables as the host builder.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "nmuller_host.hpp"
#include "util.hpp"

namespace ifgf {

// Device copies of the correction tables, allocated from the plan's arena:
// row_off [n+1], pair_patch [npairs], vals [npairs][4][Nc^2] complex FP64
// (the layout of Corrections).
struct DevCorrections {
  int64_t* row_off = nullptr;
  int32_t* pair_patch = nullptr;
  double2* vals = nullptr;
  int64_t npairs = 0;
};

// Nc and Fejer-point counts the device builder is compiled for.
bool device_corrections_supported(int nc, int nbeta);

// Builds the corrections of eq. patch_sing / Sec. III-H on the device.  The
// (target, patch) pairs and closest points equal the host builder's bit for
// bit; the weights agree to FP64 rounding.  Fills cor.row_off and
// cor.pair_patch on the host as well (cor.vals stays empty).  Temporary
// device buffers are freed before returning.  Synchronous.
int build_corrections_device(const SurfaceGeo& g, double k_int, double k_ext, const SingParams& sp,
                             DeviceArena& ar, DevCorrections& dc, Corrections& cor, std::string& err);

}  // namespace ifgf
