// Error handling shared by the host-side sources.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

namespace ftcc {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define FTCC_HIP(expr)                                                                              \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess)                                                                           \
      throw ::ftcc::HipError(std::string(#expr) + ": " + hipGetErrorString(_e) + " at " + __FILE__ + \
                             ":" + std::to_string(__LINE__));                                       \
  } while (0)

}  // namespace ftcc
