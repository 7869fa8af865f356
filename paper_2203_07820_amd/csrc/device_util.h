// Device helpers shared by the HIP sources of libchfsi (not by host code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chfsi {

// Problem of work unit `u` in a concatenation whose problems start at units
// off[0..n] (non-decreasing, off[n] = total > u): the last q with
// off[q] <= u.  Each lane of the wave reads one offset and a ballot counts
// those <= u, so the lookup costs one load per 64 problems instead of a
// chain of dependent loads.  All lanes of the wave get the same answer.
__device__ __forceinline__ int problem_of(const int64_t* __restrict__ off, const int n, const int64_t u) {
  const int lane = threadIdx.x % 64;
  int cnt = 0;
  for (int base = 0; base <= n; base += 64) {
    const int i = base + lane;
    const bool le = i <= n && off[i] <= u;
    const int c = __popcll(__ballot(le));
    cnt += c;
    if (c < 64) break;
  }
  return cnt - 1;
}

// A pointer read from device memory (a descriptor table) is a generic
// pointer to the compiler, so its loads, stores and atomics become flat
// instructions, which count in the LDS/scalar counter as well as the vector
// memory one: every wait for an LDS read then also waits for the flat
// operations in flight.  (Pointer kernel arguments are known to be global.)
// Accesses through a gptr are global instructions; only for pointers into
// global memory (or null, never dereferenced).
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)p; }
__device__ __forceinline__ void atomic_add(gptr<double> p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add(gptr<float> p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace chfsi
