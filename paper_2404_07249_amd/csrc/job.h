// Job indexing of batched launches (device side).  One launch can carry up
// to kMaxJobs jobs that share a plan: grid dimension z enumerates them, and
// job j's workspace starts j * wstride bytes after job 0's.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace pb3 {

// Byte-pointer arithmetic (not a round trip through an integer) keeps the
// pointer's provenance, so the compiler still knows it addresses global
// memory and emits global (not flat) loads and stores.
template <typename T> __device__ __forceinline__ T* job_ptr(T* p, size_t wstride) {
  using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<Byte*>(p) + (size_t)blockIdx.z * wstride);
}

}  // namespace pb3
