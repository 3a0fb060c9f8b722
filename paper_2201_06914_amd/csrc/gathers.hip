// Subsurface-offset image volume (Eq. 4, horizontal offsets along x):
//   G[h + nh][x] = scale * sum_f sum_i Ubar_f[i][x + h] Vbar_f[i][x - h],
// h = -nh .. nh, x +- h along the grid's x axis (zero where either leaves
// the row).  h = 0 is the image of Eq. 3.
//
// k_offset_gathers: a workgroup owns a 64-cell segment of one x row; chunks
// of 16 probe rows of both compressed fields (the segment plus an nh-cell
// halo and a margin on each side, zero outside the row) are staged in LDS.
// Products along a diagonal share an operand (x + h fixed: the same U; x - h
// fixed: the same V), so a thread owning GCX cells x BH offsets reads
// GCX + BH values of each field per probe row (16-byte LDS reads) for
// GCX BH products.  The workgroup's threads form nslice slices over the probe
// rows of each chunk; the slices add up through LDS at the end.  Threads are
// placed in a slice so that the 16-byte reads meet no LDS bank conflicts.
#include "rtm_internal.h"

namespace rtm {

namespace {
constexpr int GX = 64;     // cells per segment
constexpr int GIC = 16;    // probe rows per staged chunk
constexpr int GMAXH = 64;  // largest nh
constexpr int GBH = 12;    // offsets per thread
constexpr int GM = GBH;    // staged margin on each side

__device__ __forceinline__ int64_t gbar_index(int64_t x, int i, int r) {
  return ((x >> 5) * r + i) * 32 + (x & 31);
}

// 4 consecutive LDS values (16-byte aligned) into registers
__device__ __forceinline__ void lds4(const float *p, float *o) {
  const float4 t = *reinterpret_cast<const float4 *>(p);
  o[0] = t.x, o[1] = t.y, o[2] = t.z, o[3] = t.w;
}
__device__ __forceinline__ void lds4(const double *p, double *o) {
  const double2 a = *reinterpret_cast<const double2 *>(p);
  const double2 b = *reinterpret_cast<const double2 *>(p + 2);
  o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
}

// staged row stride: margin + (segment + 2 nh halo) + margin, 4-aligned
__host__ __device__ constexpr int gather_ls(int nh) { return (GX + 2 * nh + 2 * GM + 3) & ~3; }

// cells per thread: 8 in FP32, 4 in FP64 (register budget)
template <typename T> constexpr int gather_cx() { return sizeof(T) == 4 ? 8 : 4; }
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_offset_gathers(const T *__restrict__ U,
                                                        const T *__restrict__ V, int nfield,
                                                        int64_t fstride, int64_t N, int nx,
                                                        int r, int nh, T scale, int nseg,
                                                        int nblk, int nslice, int slice_thr,
                                                        int hgs, T *__restrict__ G) {
  constexpr int GCX = gather_cx<T>(), BH = GBH, CB = GX / GCX, NACC = GCX * BH;
  constexpr int RK = NACC / 3;  // accumulators handed over per reduction round
  extern __shared__ __align__(16) unsigned char gsm[];
  const int LS = gather_ls(nh);
  T *LU = reinterpret_cast<T *>(gsm), *LV = LU + GIC * LS;
  int b = blockIdx.x;
  if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);  // XCD-aware: a row's
  const int row = b / nseg, seg = b % nseg;                      // segments share an L2
  const int xs = seg * GX;
  const int64_t rb = (int64_t)row * nx;
  const int nthr = blockDim.x;
  // slice sl, offset block hg (cells' offsets hg BH - nh ..), cell block cb.
  // A 16-byte LDS read is served in 4 passes of 16 lanes: lane bit 5 and the
  // parity of lane bits 2..4 select the pass, k = (lane bits 3..4, 0..1) the
  // place in it; a bank is a 16-byte chunk mod 16.  Pass gp holds 16 / CB
  // consecutive offset blocks x all cell blocks: in FP32 one even and one odd
  // block, whose chunks (2 cb + 3 hg) differ in parity, so no two lanes of a
  // pass meet in a bank at different addresses.
  const int sl = threadIdx.x / slice_thr, t = threadIdx.x % slice_thr;
  const int l = t & 63, q = (l >> 2) & 7;
  const int gp = 4 * (t >> 6) + 2 * (l >> 5) + (__builtin_popcount(q) & 1);
  const int k = 4 * (q >> 1) + (l & 3);
  const int hg = gp * (16 / CB) + k / CB, cb = k % CB;
  const bool comp = hg < hgs;
  const int nout = 2 * nh + 1;
  // V is staged shifted by sv so that every thread's V reads start 16-byte aligned
  const int sv = (4 - (2 * nh) % 4) % 4;
  const int ubase = GCX * cb + hg * BH + GM;
  const int vbase = GCX * cb - hg * BH - BH + 2 * nh + GM + sv;
  T acc[NACC], keep = T(0);
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = T(0);
  for (int f = 0; f < nfield; ++f) {
    const T *Uf = U + f * fstride, *Vf = V + f * fstride;
    for (int i0 = 0; i0 < r; i0 += GIC) {
      __syncthreads();
      for (int p = threadIdx.x; p < LS; p += nthr) {
        // staged column p holds x = xs - nh + (p - GM) for U, one sv further left for V
        const int xu = xs - nh + p - GM, xv = xu - sv;
        const bool oku = xu >= 0 && xu < nx, okv = xv >= 0 && xv < nx;
        const T *pu = Uf + gbar_index(rb + (oku ? xu : 0), i0, r);
        const T *pv = Vf + gbar_index(rb + (okv ? xv : 0), i0, r);
        T vu[GIC], vw[GIC];
#pragma unroll
        for (int ii = 0; ii < GIC; ++ii) {
          const bool in = i0 + ii < r;
          vu[ii] = (oku && in) ? pu[ii * 32] : T(0);
          vw[ii] = (okv && in) ? pv[ii * 32] : T(0);
        }
#pragma unroll
        for (int ii = 0; ii < GIC; ++ii) {
          LU[ii * LS + p] = vu[ii];
          LV[ii * LS + p] = vw[ii];
        }
      }
      __syncthreads();
      if (comp) {
        const int iend = min(GIC, r - i0);
        for (int ii = sl; ii < iend; ii += nslice) {
          T uu[BH + GCX], vv[BH + GCX];
#pragma unroll
          for (int q = 0; q < BH + GCX; q += 4) {
            lds4(LU + ii * LS + ubase + q, uu + q);
            lds4(LV + ii * LS + vbase + q, vv + q);
          }
          // cell GCX cb + j, offset hg BH + m - nh: U at staged ubase + j + m,
          // V at staged vbase + BH + j - m
#pragma unroll
          for (int j = 0; j < GCX; ++j)
#pragma unroll
            for (int m = 0; m < BH; ++m) acc[j * BH + m] += uu[j + m] * vv[BH + j - m];
          // uu[BH + GCX - 1] and vv[0] are read but not needed; using them
          // keeps the reads whole 16-byte ones (the conflict-free placement
          // above holds for those, not for narrower pieces)
          keep = fma(uu[BH + GCX - 1], vv[0], keep);
        }
      }
    }
  }
  // slices 1 .. nslice - 1 hand their sums to slice 0 through LDS, RK at a time
  T *LR = reinterpret_cast<T *>(gsm);
#pragma unroll
  for (int k0 = 0; k0 < NACC; k0 += RK) {
    for (int s = 1; s < nslice; ++s) {
      __syncthreads();
      if (sl == s) {
#pragma unroll
        for (int k = 0; k < RK; ++k) LR[k * slice_thr + t] = acc[k0 + k];
      }
      __syncthreads();
      if (sl == 0) {
#pragma unroll
        for (int k = 0; k < RK; ++k) acc[k0 + k] += LR[k * slice_thr + t];
      }
    }
  }
  if (nslice < 0) G[0] = keep;  // never: nslice >= 1
  if (sl != 0 || !comp) return;
#pragma unroll
  for (int m = 0; m < BH; ++m) {
    const int hi = hg * BH + m;
    if (hi < nout) {
#pragma unroll
      for (int j = 0; j < GCX; ++j) {
        const int x = xs + GCX * cb + j;
        if (x < nx) G[(int64_t)hi * N + rb + x] = scale * acc[j * BH + m];
      }
    }
  }
}

template <typename T>
hipError_t launch_offset_gathers(const T *U, const T *V, int nfield, int64_t fstride, int64_t N,
                                 int nx, int r, int nh, double scale, T *G, hipStream_t st) {
  if (nh < 0 || nh > GMAXH) return hipErrorInvalidValue;
  constexpr int GCX = gather_cx<T>(), CB = GX / GCX;
  const int nout = 2 * nh + 1;
  const int hgs = (nout + GBH - 1) / GBH;           // offset blocks
  const int slice_thr = 64 * ((hgs * CB + 63) / 64);  // whole waves of (offset, cell) blocks
  const int nslice = 256 / slice_thr;
  const int nthr = nslice * slice_thr;
  const int64_t rows = N / nx;
  const int nseg = (nx + GX - 1) / GX;
  const int64_t nblk = rows * nseg;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t stage = 2 * (size_t)GIC * gather_ls(nh);
  const size_t reduce = (size_t)slice_thr * (GCX * GBH / 3);
  const size_t lds = (stage > reduce ? stage : reduce) * sizeof(T);
  hipLaunchKernelGGL((k_offset_gathers<T>), dim3((unsigned)nblk), dim3(nthr), lds, st, U, V,
                     nfield, fstride, N, nx, r, nh, (T)scale, nseg, (int)nblk, nslice, slice_thr,
                     hgs, G);
  return hipGetLastError();
}
template hipError_t launch_offset_gathers<float>(const float *, const float *, int, int64_t,
                                                 int64_t, int, int, int, double, float *,
                                                 hipStream_t);
template hipError_t launch_offset_gathers<double>(const double *, const double *, int, int64_t,
                                                  int64_t, int, int, int, double, double *,
                                                  hipStream_t);

}  // namespace rtm
