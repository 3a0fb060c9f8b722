// Subsurface-offset image volume (Eq. 4, horizontal offsets along x):
//   G[h + nh][x] = scale * sum_f sum_i Ubar_f[i][x + h] Vbar_f[i][x - h],
// h = -nh .. nh, x +- h along the grid's x axis (zero where either leaves
// the row).  h = 0 is the image of Eq. 3.
//
// k_offset_gathers: a workgroup owns a 64-cell segment of one x row; probe
// chunks of 16 rows of both compressed fields (segment plus an nh-cell halo
// on each side, tile-major reads) are staged in LDS, and thread (c, g) keeps
// the sums of cell c for offsets h = -nh + g, -nh + g + 4, ... in registers.
#include "rtm_internal.h"

namespace rtm {

namespace {
constexpr int GX = 64;        // cells per segment
constexpr int GIC = 16;       // probe rows per staged chunk
constexpr int GMAXH = 64;     // largest nh
constexpr int GW = GX + 2 * GMAXH;
constexpr int GACC = (2 * GMAXH + 1 + 3) / 4;

__device__ __forceinline__ int64_t gbar_index(int64_t x, int i, int r) {
  return ((x >> 5) * r + i) * 32 + (x & 31);
}
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_offset_gathers(const T *__restrict__ U,
                                                        const T *__restrict__ V, int nfield,
                                                        int64_t fstride, int64_t N, int nx,
                                                        int r, int nh, T scale, int nseg,
                                                        T *__restrict__ G) {
  __shared__ T LU[GIC * GW], LV[GIC * GW];
  const int row = blockIdx.x / nseg, seg = blockIdx.x % nseg;
  const int xs = seg * GX;                       // first x of the segment
  const int64_t rb = (int64_t)row * nx;          // flat index of x = 0
  const int W = GX + 2 * nh;
  const int c = threadIdx.x % GX, g = threadIdx.x / GX;
  const int nout = 2 * nh + 1;
  T acc[GACC];
#pragma unroll
  for (int k = 0; k < GACC; ++k) acc[k] = T(0);
  for (int f = 0; f < nfield; ++f) {
    const T *Uf = U + f * fstride, *Vf = V + f * fstride;
    for (int i0 = 0; i0 < r; i0 += GIC) {
      __syncthreads();
      for (int e = threadIdx.x; e < GIC * W; e += 256) {
        const int ii = e / W, w = e % W;
        const int x = xs - nh + w;
        const int i = i0 + ii;
        const bool ok = i < r && x >= 0 && x < nx;
        const int64_t xf = rb + x;
        LU[ii * GW + w] = ok ? Uf[gbar_index(xf, i, r)] : T(0);
        LV[ii * GW + w] = ok ? Vf[gbar_index(xf, i, r)] : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < GACC; ++k) {
        const int hi = g + 4 * k;  // h + nh
        if (hi < nout) {
          const int h = hi - nh;
          // U at x + h and V at x - h: staged columns c + nh + h and c + nh - h
          const T *pu = LU + c + nh + h, *pv = LV + c + nh - h;
          T s = acc[k];
#pragma unroll
          for (int ii = 0; ii < GIC; ++ii) s += pu[ii * GW] * pv[ii * GW];
          acc[k] = s;
        }
      }
    }
  }
  const int x = xs + c;
  if (x < nx) {
#pragma unroll
    for (int k = 0; k < GACC; ++k) {
      const int hi = g + 4 * k;
      if (hi < nout) G[(int64_t)hi * N + rb + x] = scale * acc[k];
    }
  }
}

template <typename T>
hipError_t launch_offset_gathers(const T *U, const T *V, int nfield, int64_t fstride, int64_t N,
                                 int nx, int r, int nh, double scale, T *G, hipStream_t st) {
  if (nh < 0 || nh > GMAXH) return hipErrorInvalidValue;
  const int64_t rows = N / nx;
  const int nseg = (nx + GX - 1) / GX;
  const int64_t nblk = rows * nseg;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_offset_gathers<T>), dim3((unsigned)nblk), dim3(256), 0, st, U, V, nfield,
                     fstride, N, nx, r, nh, (T)scale, nseg, G);
  return hipGetLastError();
}
template hipError_t launch_offset_gathers<float>(const float *, const float *, int, int64_t,
                                                 int64_t, int, int, int, double, float *,
                                                 hipStream_t);
template hipError_t launch_offset_gathers<double>(const double *, const double *, int, int64_t,
                                                  int64_t, int, int, int, double, double *,
                                                  hipStream_t);

}  // namespace rtm
