// Job indexing of batched launches (device side).  One launch can carry up
// to kMaxJobs jobs that share a plan: grid dimension z enumerates them, and
// job j's workspace starts j * wstride bytes after job 0's.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pb3 {

template <typename T> __device__ __forceinline__ T* job_ptr(T* p, size_t wstride) {
  return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + (size_t)blockIdx.z * wstride);
}

}  // namespace pb3
