// Device helpers shared by the acoustic and TTI step kernels.
#pragma once
#include "rtm_internal.h"

namespace rtm {

// cells into the sponge layer of one axis (0 in the interior)
__device__ __forceinline__ int sponge_depth(int i, int n, int nb) {
  const int a = nb - i;
  const int b = i - (n - 1 - nb);
  const int d = a > b ? a : b;
  return d > 0 ? d : 0;
}

// a = eta dt / 2 at (z, y, x): kd (dz^2 + dy^2 + dx^2)
template <typename T>
__device__ __forceinline__ T sponge_a(const StepArgs<T> &a, int z, int y, int x) {
  if (a.nb <= 0) return T(0);
  const int dz = sponge_depth(z, a.nz, a.nb);
  const int dy = a.ny > 1 ? sponge_depth(y, a.ny, a.nb) : 0;
  const int dx = sponge_depth(x, a.nx, a.nb);
  return a.kd * T(dz * dz + dy * dy + dx * dx);
}

}  // namespace rtm
