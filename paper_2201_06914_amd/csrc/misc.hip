// Imaging condition, residual / misfit and inner products, plus fills and
// copies (kernels rather than hipMemsetAsync so that a captured sweep replays
// correctly).
//
// Reductions are deterministic two-pass sums in double precision: a fixed
// grid of kReduceBlocks workgroups writes one partial each (grid-stride
// accumulation, then a fixed-shape wavefront / workgroup tree), and a single
// workgroup adds the partials in index order.
#include "rtm_internal.h"

namespace rtm {

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(T *__restrict__ d, const T *__restrict__ s,
                                              int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    d[i] = s[i];
}

// Streaming copy by 16-byte vectors: each workgroup moves four consecutive
// runs of 256 vectors (all four loads issued before the stores), one
// workgroup per 1024 vectors, non-temporal loads and stores (each byte is
// touched once).  It is the measured HBM ceiling of a read-once / write-once
// kernel, the reference the roofline figures are set against.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_x4(f32x4 *__restrict__ d, const f32x4 *__restrict__ s,
                                                  int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  f32x4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + 256 * k < n) v[k] = __builtin_nontemporal_load(s + base + 256 * k);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + 256 * k < n) __builtin_nontemporal_store(v[k], d + base + 256 * k);
}

hipError_t launch_copy_x4(void *d, const void *s, int64_t n16, hipStream_t st) {
  if (n16 <= 0) return hipSuccess;
  const int64_t nblk = (n16 + 1023) / 1024;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy_x4, dim3((unsigned)nblk), dim3(256), 0, st, static_cast<f32x4 *>(d),
                     static_cast<const f32x4 *>(s), n16);
  return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_copy(T *d, const T *s, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n)), dim3(256), 0, st, d, s, n);
  return hipGetLastError();
}
// Non-finite watch: any non-finite value among x[0..n) sets status[0] = 1
// (plain stores of the same value; the word is cleared by k_status_clear).
template <typename T>
__global__ __launch_bounds__(256) void k_flag_nonfinite(const T *__restrict__ x, int64_t n,
                                                        uint32_t *status) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    bad |= !isfinite(x[i]);
  if (bad) status[0] = 1u;
}
__global__ void k_status_clear(uint32_t *status) {
  if (threadIdx.x == 0) status[0] = 0u;
}
template <typename T>
hipError_t launch_flag_nonfinite(const T *x, int64_t n, uint32_t *status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_flag_nonfinite<T>), dim3(grid_for(n)), dim3(256), 0, st, x, n, status);
  return hipGetLastError();
}
hipError_t launch_status_clear(uint32_t *status, hipStream_t st) {
  hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, st, status);
  return hipGetLastError();
}
template hipError_t launch_flag_nonfinite<float>(const float *, int64_t, uint32_t *, hipStream_t);
template hipError_t launch_flag_nonfinite<double>(const double *, int64_t, uint32_t *,
                                                  hipStream_t);
template hipError_t launch_fill<float>(float *, int64_t, float, hipStream_t);
template hipError_t launch_fill<double>(double *, int64_t, double, hipStream_t);
template hipError_t launch_copy<float>(float *, const float *, int64_t, hipStream_t);
template hipError_t launch_copy<double>(double *, const double *, int64_t, hipStream_t);

// exact (full-history) imaging, one step at a time (Eq. 2):
//   s = (un - 2 u0 + um) / dt^2            second time derivative of a step
//   g -= s * lam                            zero-lag correlation with lam^n
template <typename T>
__global__ __launch_bounds__(256) void k_second_diff(const T *__restrict__ un,
                                                     const T *__restrict__ u0,
                                                     const T *__restrict__ um, T inv_dt2,
                                                     int64_t n, T *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    out[i] = (un[i] - T(2) * u0[i] + um[i]) * inv_dt2;
}

template <typename T>
__global__ __launch_bounds__(256) void k_correlate(T *__restrict__ g, const T *__restrict__ s,
                                                   const T *__restrict__ lam, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    g[i] -= s[i] * lam[i];
}

template <typename T>
hipError_t launch_second_diff(const T *un, const T *u0, const T *um, T inv_dt2, int64_t n, T *out,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_second_diff<T>), dim3(grid_for(n)), dim3(256), 0, st, un, u0, um, inv_dt2,
                     n, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_correlate(T *g, const T *s, const T *lam, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_correlate<T>), dim3(grid_for(n)), dim3(256), 0, st, g, s, lam, n);
  return hipGetLastError();
}
template hipError_t launch_second_diff<float>(const float *, const float *, const float *, float,
                                              int64_t, float *, hipStream_t);
template hipError_t launch_second_diff<double>(const double *, const double *, const double *,
                                               double, int64_t, double *, hipStream_t);
template hipError_t launch_correlate<float>(float *, const float *, const float *, int64_t,
                                            hipStream_t);
template hipError_t launch_correlate<double>(double *, const double *, const double *, int64_t,
                                             hipStream_t);

// y += x
template <typename T>
__global__ __launch_bounds__(256) void k_axpy(T *__restrict__ y, const T *__restrict__ x,
                                              int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    y[i] += x[i];
}
template <typename T>
hipError_t launch_axpy(T *y, const T *x, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_axpy<T>), dim3(grid_for(n)), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}
template hipError_t launch_axpy<float>(float *, const float *, int64_t, hipStream_t);
template hipError_t launch_axpy<double>(double *, const double *, int64_t, hipStream_t);

// image[x] = scale * sum_i U[i][x] V[i][x]  (Eq. 3), summed in double.
// U, V tile-major: (i, x) at ((x / 32) r + i) 32 + x % 32.
template <typename T>
__global__ __launch_bounds__(256) void k_image(const T *__restrict__ U, const T *__restrict__ V,
                                               int64_t N, int r, double scale,
                                               T *__restrict__ img) {
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < N;
       x += (int64_t)gridDim.x * 256) {
    const int64_t base = (x >> 5) * r * 32 + (x & 31);
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc += (double)U[base + i * 32] * (double)V[base + i * 32];
    img[x] = (T)(scale * acc);
  }
}

template <typename T>
hipError_t launch_image(const T *U, const T *V, int64_t N, int r, double scale, T *img,
                        hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_image<T>), dim3(grid_for(N)), dim3(256), 0, st, U, V, N, r, scale, img);
  return hipGetLastError();
}
template hipError_t launch_image<float>(const float *, const float *, int64_t, int, double,
                                        float *, hipStream_t);
template hipError_t launch_image<double>(const double *, const double *, int64_t, int, double,
                                         double *, hipStream_t);

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((part[0] + part[1]) + part[2]) + part[3];
  __syncthreads();
  return s;
}

template <typename T, bool RESID>
__global__ __launch_bounds__(256) void k_partial(const T *a, const T *b, T *res, int64_t n,
                                                 double *partials) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    if (RESID) {
      const T r = a[i] - b[i];
      res[i] = r;
      acc += (double)r * (double)r;
    } else {
      acc += (double)a[i] * (double)b[i];
    }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_final(const double *partials, int np, double scale,
                                               double *out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += partials[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) out[0] = scale * s;
}

template <typename T>
hipError_t launch_residual_misfit(const T *d, const T *dobs, T *res, int64_t n, double *partials,
                                  double *misfit, hipStream_t st) {
  hipLaunchKernelGGL((k_partial<T, true>), dim3(kReduceBlocks), dim3(256), 0, st, d, dobs, res, n,
                     partials);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, kReduceBlocks, 0.5, misfit);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T *a, const T *b, int64_t n, double *partials, double *out,
                      hipStream_t st) {
  hipLaunchKernelGGL((k_partial<T, false>), dim3(kReduceBlocks), dim3(256), 0, st, a, b,
                     (T *)nullptr, n, partials);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, st, partials, kReduceBlocks, 1.0, out);
  return hipGetLastError();
}

template hipError_t launch_residual_misfit<float>(const float *, const float *, float *, int64_t,
                                                  double *, double *, hipStream_t);
template hipError_t launch_residual_misfit<double>(const double *, const double *, double *,
                                                   int64_t, double *, double *, hipStream_t);
template hipError_t launch_dot<float>(const float *, const float *, int64_t, double *, double *,
                                      hipStream_t);
template hipError_t launch_dot<double>(const double *, const double *, int64_t, double *,
                                       double *, hipStream_t);

}  // namespace rtm
