// Reads of the level ring by the block kernels (probe GEMM, space sketch).
#pragma once
#include "rtm_internal.h"

namespace rtm {

// level j of the block, s0 - 1 <= j <= s0 + R - 2 (one wrap at most)
template <typename T>
__device__ __forceinline__ const T *ring_level(const ProbeArgs<T> &p, int j) {
  int slot = p.slot0 + (j - p.s0 + 1);
  if (slot >= p.R) slot -= p.R;
  return p.ring + (int64_t)slot * p.ld;
}

// probed value of local step t at cell c
template <typename T>
__device__ __forceinline__ T probed(const ProbeArgs<T> &p, int t, int64_t c) {
  const int s = p.s0 + t;
  if (p.mode == PROBE_UTT) {
    const T un = ring_level(p, s + 1)[c];
    const T u0 = ring_level(p, s)[c];
    const T um = ring_level(p, s - 1)[c];
    return (un - T(2) * u0 + um) * p.inv_dt2;
  }
  return ring_level(p, p.mode == PROBE_NEW ? s + 1 : s)[c];
}

}  // namespace rtm
