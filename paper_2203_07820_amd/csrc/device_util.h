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

}  // namespace chfsi
