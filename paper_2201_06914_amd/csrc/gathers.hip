// Subsurface-offset image volume (Eq. 4, horizontal offsets along x):
//   G[h + nh][x] = scale * sum_f sum_i Ubar_f[i][x + h] Vbar_f[i][x - h],
// h = -nh .. nh, x +- h along the grid's x axis (zero where either leaves
// the row).  h = 0 is the image of Eq. 3.
//
// A workgroup owns a segment of 64 (or 72) cells of one x row; chunks of 16 probe rows of
// both compressed fields (the segment plus an nh-cell halo and a margin on
// each side, zero outside the row) are staged in LDS.  Products along a
// diagonal share an operand (x + h fixed: the same U; x - h fixed: the same
// V), so a thread owning GCX cells x BH offsets reads GCX + BH values of each
// field per probe row (16-byte LDS reads) for GCX BH products.  The
// workgroup's threads form nslice slices over the probe rows of each chunk;
// the slices add up through LDS at the end.  Threads are placed in a slice so
// that the 16-byte reads meet no LDS bank conflicts.  With 7 offset blocks
// (73 to 84 offsets, e.g. -500 .. 500 m at 12.5 m) FP32 segments are 72 cells:
// 9 cell blocks x 7 offset blocks fill 63 of a wave's 64 lanes (64-cell
// segments fill 56), placed by a table instead of the formula.
//
// k_offset_gathers_f32 stages with direct global -> LDS loads into two
// buffers: chunk c + 1 streams into one while chunk c is multiplied out of
// the other.  The buffers are two distinct LDS arrays and the chunk loop
// alternates them statically, so the compiler can tell the in-flight loads
// from the reads and does not wait for the former before the latter.
// k_offset_gathers (FP64) stages through registers, one chunk at a time.
#include "rtm_internal.h"

namespace rtm {

namespace {
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

// staged row stride: margin + (segment of gx cells + 2 nh halo) + margin, 4-aligned
__host__ __device__ constexpr int gather_ls(int gx, int nh) {
  return (gx + 2 * nh + 2 * GM + 3) & ~3;
}

// 72-cell segments: (cell block | offset block << 4) of place k in pass gp
// (0xFF: idle).  Found by a search under the bank model below: in each pass
// the chunks 2 cb + 3 hg (U) and 2 cb - 3 hg (V) are distinct mod 16 or equal.
__constant__ uint8_t kPlace72[4][16] = {
    {0x02, 0x11, 0x12, 0x17, 0x18, 0x21, 0x22, 0x24, 0x26, 0x31, 0x34, 0x45, 0x48, 0x51, 0x58, 0x67},
    {0x01, 0x04, 0x07, 0x08, 0x10, 0x25, 0x27, 0x30, 0x37, 0x41, 0x44, 0x47, 0x50, 0x53, 0x57, 0x64},
    {0x03, 0x14, 0x16, 0x20, 0x32, 0x33, 0x35, 0x38, 0x42, 0x43, 0x55, 0x60, 0x61, 0x63, 0x65, 0x66},
    {0x00, 0x05, 0x06, 0x13, 0x15, 0x23, 0x28, 0x36, 0x40, 0x46, 0x52, 0x54, 0x56, 0x62, 0x68, 0xFF}};

// cells per thread: 8 in FP32, 4 in FP64 (register budget)
template <typename T> constexpr int gather_cx() { return sizeof(T) == 4 ? 8 : 4; }

struct GatherArgs {
  int64_t fstride, N;
  int nfield, nx, r, nh, nseg, nblk, nslice, slice_thr, hgs;
};

// A thread's place: slice sl, offset block hg (offsets hg BH - nh ..), cell
// block cb.  A 16-byte LDS read is served in 4 passes of 16 lanes: lane bit 5
// and the parity of lane bits 2..4 select the pass, k = (lane bits 3..4,
// 0..1) the place in it; a bank is a 16-byte chunk mod 16.  Pass gp holds
// 16 / CB consecutive offset blocks x all cell blocks: in FP32 one even and
// one odd block, whose chunks (2 cb + 3 hg) differ in parity, so no two lanes
// of a pass meet in a bank at different addresses.
template <typename T, int GX>
struct GatherThread {
  static constexpr int GCX = gather_cx<T>(), BH = GBH, CB = GX / GCX, NACC = GCX * BH;
  int sl, t, hg, cb, ubase, vbase, sv, xs;
  int64_t rb;
  bool comp;
  __device__ explicit GatherThread(const GatherArgs &a) {
    int b = blockIdx.x;
    if ((a.nblk & 7) == 0) b = (b & 7) * (a.nblk >> 3) + (b >> 3);  // XCD-aware: a row's
    const int row = b / a.nseg;                                       // segments share an L2
    xs = (b % a.nseg) * GX;
    rb = (int64_t)row * a.nx;
    sl = threadIdx.x / a.slice_thr;
    t = threadIdx.x % a.slice_thr;
    const int l = t & 63, q = (l >> 2) & 7;
    const int gp = 4 * (t >> 6) + 2 * (l >> 5) + (__builtin_popcount(q) & 1);
    const int k = 4 * (q >> 1) + (l & 3);
    if constexpr (GX == 72) {  // one wave per slice, 7 offset blocks
      const int e = kPlace72[gp & 3][k];
      hg = e == 0xFF ? a.hgs : e >> 4;
      cb = e == 0xFF ? 0 : e & 15;
    } else {
      hg = gp * (16 / CB) + k / CB;
      cb = k % CB;
    }
    comp = hg < a.hgs;
    // V is staged shifted by sv so that every thread's V reads start 16-byte aligned
    sv = (4 - (2 * a.nh) % 4) % 4;
    ubase = GCX * cb + hg * BH + GM;
    vbase = GCX * cb - hg * BH - BH + 2 * a.nh + GM + sv;
  }
};

// multiply out one staged chunk (probe rows i0 .. i0 + 15) from BU / BV
template <typename T, int GX>
__device__ __forceinline__ void gather_chunk(const GatherThread<T, GX> &th, const GatherArgs &a,
                                             const T *BU, const T *BV, int LS, int i0,
                                             T (&acc)[GatherThread<T, GX>::NACC], T &keep) {
  constexpr int GCX = GatherThread<T, GX>::GCX, BH = GBH;
  if (!th.comp) return;
  const int iend = min(GIC, a.r - i0);
  for (int ii = th.sl; ii < iend; ii += a.nslice) {
    T uu[BH + GCX], vv[BH + GCX];
#pragma unroll
    for (int q = 0; q < BH + GCX; q += 4) {
      lds4(BU + ii * LS + th.ubase + q, uu + q);
      lds4(BV + ii * LS + th.vbase + q, vv + q);
    }
    // cell GCX cb + j, offset hg BH + m - nh: U at staged ubase + j + m,
    // V at staged vbase + BH + j - m
#pragma unroll
    for (int j = 0; j < GCX; ++j)
#pragma unroll
      for (int m = 0; m < BH; ++m) acc[j * BH + m] += uu[j + m] * vv[BH + j - m];
    // uu[BH + GCX - 1] and vv[0] are read but not needed; using them keeps the
    // reads whole 16-byte ones (the conflict-free placement holds for those,
    // not for narrower pieces)
    keep = fma(uu[BH + GCX - 1], vv[0], keep);
  }
}

// slices 1 .. nslice - 1 hand their sums to slice 0 through LR (LDS), RK at a
// time; slice 0 writes the volume
template <typename T, int GX>
__device__ __forceinline__ void gather_finish(const GatherThread<T, GX> &th, const GatherArgs &a,
                                              T *LR, T (&acc)[GatherThread<T, GX>::NACC], T keep,
                                              T scale, T *__restrict__ G) {
  constexpr int GCX = GatherThread<T, GX>::GCX, BH = GBH, NACC = GatherThread<T, GX>::NACC;
  constexpr int RK = NACC / 3;
#pragma unroll
  for (int k0 = 0; k0 < NACC; k0 += RK) {
    for (int s = 1; s < a.nslice; ++s) {
      __syncthreads();
      if (th.sl == s) {
#pragma unroll
        for (int k = 0; k < RK; ++k) LR[k * a.slice_thr + th.t] = acc[k0 + k];
      }
      __syncthreads();
      if (th.sl == 0) {
#pragma unroll
        for (int k = 0; k < RK; ++k) acc[k0 + k] += LR[k * a.slice_thr + th.t];
      }
    }
  }
  if (a.nslice < 0) G[0] = keep;  // never: nslice >= 1
  if (th.sl != 0 || !th.comp) return;
  const int nout = 2 * a.nh + 1;
#pragma unroll
  for (int m = 0; m < BH; ++m) {
    const int hi = th.hg * BH + m;
    if (hi < nout) {
#pragma unroll
      for (int j = 0; j < GCX; ++j) {
        const int x = th.xs + GCX * th.cb + j;
        if (x < a.nx) G[(int64_t)hi * a.N + th.rb + x] = scale * acc[j * BH + m];
      }
    }
  }
}
}  // namespace

// FP32, direct global -> LDS staging, two static buffers of row stride <= MAXLS,
// GX-cell segments
template <int MAXLS, int GX>
__global__ __launch_bounds__(256) void k_offset_gathers_f32(const float *__restrict__ U,
                                                            const float *__restrict__ V,
                                                            GatherArgs a, float scale,
                                                            float *__restrict__ G) {
  constexpr int NACC = GatherThread<float, GX>::NACC;
  constexpr int BUFN = 2 * GIC * MAXLS;
  __shared__ __align__(16) float SA[BUFN];
  __shared__ __align__(16) float SB[BUFN];
  const GatherThread<float, GX> th(a);
  const int LS = gather_ls(GX, a.nh);
  // thread p < LS owns staged column p (256 threads >= LS); U rows at S,
  // V rows at S + GIC LS; a wave's loads land at the wave's first column + lane
  const int p = threadIdx.x;
  const int wbase = __builtin_amdgcn_readfirstlane(p & ~63);  // wave-uniform
  const int xu = th.xs - a.nh + p - GM, xv = xu - th.sv;
  const bool stg = p < LS;
  const bool oku = stg && xu >= 0 && xu < a.nx, okv = stg && xv >= 0 && xv < a.nx;
  const int64_t gu = th.rb + (oku ? xu : 0), gv = th.rb + (okv ? xv : 0);
  // columns outside the row are never loaded: zero them once in both buffers
  if (stg) {
    for (int ii = 0; ii < GIC; ++ii) {
      if (!oku) SA[ii * LS + p] = SB[ii * LS + p] = 0.f;
      if (!okv) SA[(GIC + ii) * LS + p] = SB[(GIC + ii) * LS + p] = 0.f;
    }
  }
  const int cpf = (a.r + GIC - 1) / GIC, nch = a.nfield * cpf;  // chunk c = (field, 16 rows)
  auto issue = [&](int c, float *S) {
    const int f = c / cpf, i0 = (c % cpf) * GIC;
    // probe row i0 + ii of a column sits ii * 32 values after row i0
    const float *pu = U + f * a.fstride + gbar_index(gu, i0, a.r);
    const float *pv = V + f * a.fstride + gbar_index(gv, i0, a.r);
    const int nrow = min(GIC, a.r - i0);
#pragma unroll
    for (int ii = 0; ii < GIC; ++ii) {
      if (ii < nrow) {
        if (oku) __builtin_amdgcn_global_load_lds(pu + ii * 32, S + ii * LS + wbase, 4, 0, 0);
        if (okv)
          __builtin_amdgcn_global_load_lds(pv + ii * 32, S + (GIC + ii) * LS + wbase, 4, 0, 0);
      }
    }
  };
  float acc[NACC], keep = 0.f;
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = 0.f;
  issue(0, SA);
  for (int c = 0; c < nch; c += 2) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this thread's loads of chunk c
    __syncthreads();                     // everyone's; and chunk c - 1 is multiplied out
    if (c + 1 < nch) issue(c + 1, SB);
    gather_chunk(th, a, SA, SA + GIC * LS, LS, (c % cpf) * GIC, acc, keep);
    if (c + 1 >= nch) break;
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (c + 2 < nch) issue(c + 2, SA);
    gather_chunk(th, a, SB, SB + GIC * LS, LS, ((c + 1) % cpf) * GIC, acc, keep);
  }
  gather_finish(th, a, SA, acc, keep, scale, G);
}

// any type: register staging, one chunk at a time, dynamic LDS
template <typename T>
__global__ __launch_bounds__(256) void k_offset_gathers(const T *__restrict__ U,
                                                        const T *__restrict__ V, GatherArgs a,
                                                        T scale, T *__restrict__ G) {
  constexpr int GX = 64;
  constexpr int NACC = GatherThread<T, GX>::NACC;
  extern __shared__ __align__(16) unsigned char gsm[];
  const GatherThread<T, GX> th(a);
  const int LS = gather_ls(GX, a.nh);
  T *LU = reinterpret_cast<T *>(gsm), *LV = LU + GIC * LS;
  T acc[NACC], keep = T(0);
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = T(0);
  const int cpf = (a.r + GIC - 1) / GIC, nch = a.nfield * cpf;
  for (int c = 0; c < nch; ++c) {
    const int f = c / cpf, i0 = (c % cpf) * GIC;
    const T *Uf = U + f * a.fstride, *Vf = V + f * a.fstride;
    __syncthreads();
    for (int p = threadIdx.x; p < LS; p += blockDim.x) {
      // staged column p holds x = xs - nh + (p - GM) for U, one sv further left for V
      const int xu = th.xs - a.nh + p - GM, xv = xu - th.sv;
      const bool oku = xu >= 0 && xu < a.nx, okv = xv >= 0 && xv < a.nx;
      const T *pu = Uf + gbar_index(th.rb + (oku ? xu : 0), i0, a.r);
      const T *pv = Vf + gbar_index(th.rb + (okv ? xv : 0), i0, a.r);
      T vu[GIC], vw[GIC];
#pragma unroll
      for (int ii = 0; ii < GIC; ++ii) {
        const bool in = i0 + ii < a.r;
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
    gather_chunk(th, a, LU, LV, LS, i0, acc, keep);
  }
  gather_finish(th, a, LU, acc, keep, scale, G);
}

template <typename T>
hipError_t launch_offset_gathers(const T *U, const T *V, int nfield, int64_t fstride, int64_t N,
                                 int nx, int r, int nh, double scale, T *G, hipStream_t st) {
  if (nh < 0 || nh > GMAXH) return hipErrorInvalidValue;
  constexpr int GCX = gather_cx<T>();
  GatherArgs a;
  a.fstride = fstride;
  a.N = N;
  a.nfield = nfield;
  a.nx = nx;
  a.r = r;
  a.nh = nh;
  const int nout = 2 * nh + 1;
  a.hgs = (nout + GBH - 1) / GBH;  // offset blocks
  // FP32 with 7 offset blocks: 72-cell segments (9 cell blocks, table placement)
  const int gx = (sizeof(T) == 4 && a.hgs == 7) ? 72 : 64;
  const int CB = gx / GCX;
  a.slice_thr = 64 * ((a.hgs * CB + 63) / 64);  // whole waves of (offset, cell) blocks
  a.nslice = 256 / a.slice_thr;
  const int nthr = a.nslice * a.slice_thr;
  const int64_t rows = N / nx;
  a.nseg = (nx + gx - 1) / gx;
  const int64_t nblk = rows * a.nseg;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  a.nblk = (int)nblk;
  const int ls = gather_ls(gx, nh);
  const size_t reduce = (size_t)a.slice_thr * (GCX * GBH / 3);
  if constexpr (sizeof(T) == 4) {
    // 256 threads stage one column each; the reduction fits in one buffer
    constexpr int LS40 = gather_ls(64, 40), LS72 = gather_ls(72, 41), LSMAX = gather_ls(64, GMAXH);
    if (nthr != 256 || ls > 256 || reduce > 2 * (size_t)GIC * LS40) return hipErrorInvalidValue;
    if (gx == 72) {
      if (a.slice_thr != 64 || ls > LS72) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_offset_gathers_f32<LS72, 72>), dim3(a.nblk), dim3(nthr), 0, st, U, V,
                         a, (float)scale, G);
    } else if (ls <= LS40) {
      hipLaunchKernelGGL((k_offset_gathers_f32<LS40, 64>), dim3(a.nblk), dim3(nthr), 0, st, U, V,
                         a, (float)scale, G);
    } else {
      hipLaunchKernelGGL((k_offset_gathers_f32<LSMAX, 64>), dim3(a.nblk), dim3(nthr), 0, st, U,
                         V, a, (float)scale, G);
    }
  } else {
    const size_t stage = 2 * (size_t)GIC * ls;
    const size_t lds = (stage > reduce ? stage : reduce) * sizeof(T);
    hipLaunchKernelGGL((k_offset_gathers<T>), dim3(a.nblk), dim3(nthr), lds, st, U, V, a,
                       (T)scale, G);
  }
  return hipGetLastError();
}
template hipError_t launch_offset_gathers<float>(const float *, const float *, int, int64_t,
                                                 int64_t, int, int, int, double, float *,
                                                 hipStream_t);
template hipError_t launch_offset_gathers<double>(const double *, const double *, int, int64_t,
                                                  int64_t, int, int, int, double, double *,
                                                  hipStream_t);

}  // namespace rtm
