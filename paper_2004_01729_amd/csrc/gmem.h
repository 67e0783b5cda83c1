// Global-address-space views of device pointers.
//
// A pointer read out of a problem descriptor is a generic (flat) pointer to the
// compiler, which then emits flat loads and stores.  A flat access counts against
// the LDS / scalar-memory counter as well as the vector-memory one, so every wait
// for an LDS read or a scalar load also waits for the HBM accesses in flight (in a
// GEMM main loop: the next tile's operand loads, issued to overlap the MFMAs, are
// waited for before the first MFMA).  The views below are address space 1, for
// which the compiler emits global_load / global_store, tracked by the vector-memory
// counter only.  Every pointer handed to a kernel here is device (global) memory.
#pragma once
#include <hip/hip_runtime.h>

namespace ftcc {

template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<const T> gview(const T* p) {
  return (gptr<const T>)p;
}
template <class T>
__device__ __forceinline__ gptr<T> gview(T* p) {
  return (gptr<T>)p;
}

}  // namespace ftcc
