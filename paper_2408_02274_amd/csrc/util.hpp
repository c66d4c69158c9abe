// Error reporting and device-memory ownership helpers for the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace ifgf {

int set_error(int code, const std::string& msg);
int set_hip_error(hipError_t e, const char* where);
void clear_error();
const char* last_error_cstr();

// Owns every device allocation of a plan; frees them on destruction.
class DeviceArena {
 public:
  DeviceArena() = default;
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  ~DeviceArena() {
    for (void* p : ptrs_) (void)hipFree(p);
  }
  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs_.push_back(p);
    bytes_ += bytes;
    return p;
  }
  size_t bytes() const { return bytes_; }

 private:
  std::vector<void*> ptrs_;
  size_t bytes_ = 0;
};

}  // namespace ifgf
