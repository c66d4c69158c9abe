// Thread-local error message of the C-ABI.
#include <hip/hip_runtime.h>

#include <string>

#include "util.hpp"

namespace ifgf {

static thread_local std::string g_err;

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int set_hip_error(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return -3;  // IFGF_EHIP
}

void clear_error() { g_err.clear(); }

const char* last_error_cstr() { return g_err.c_str(); }

}  // namespace ifgf
