// Subsurface-offset image volume (Eq. 4, horizontal offsets along x):
//   G[h + nh][x] = scale * sum_f sum_i Ubar_f[i][x + h] Vbar_f[i][x - h],
// h = -nh .. nh, x +- h along the grid's x axis (zero where either leaves
// the row).  h = 0 is the image of Eq. 3.
//
// FP32 runs on the matrix cores (k_offset_gathers_mfma, below).  FP64 runs on
// the vector ALUs (k_offset_gathers): a workgroup owns a segment of 64 cells
// of one x row; chunks of 16 probe rows of both compressed fields (the
// segment plus an nh-cell halo and a margin on each side, zero outside the
// row) are staged in LDS.  Products along a diagonal share an operand (x + h
// fixed: the same U; x - h fixed: the same V), so a thread owning GCX cells x
// BH offsets reads GCX + BH values of each field per probe row (16-byte LDS
// reads) for GCX BH products.  The workgroup's threads form nslice slices
// over the probe rows of each chunk; the slices add up through LDS at the
// end.  Threads are placed in a slice so that the 16-byte reads meet no LDS
// bank conflicts.
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

// cells per thread of the vector kernel (register budget; it runs FP64 only)
template <typename T> constexpr int gather_cx() { return sizeof(T) == 4 ? 8 : 4; }

struct GatherArgs {
  int64_t fstride, N;
  int nfield, nx, r, nh, nseg, nblk, nslice, slice_thr, hgs;
};

// A thread's place: slice sl, offset block hg (offsets hg BH - nh ..), cell
// block cb.  A 16-byte LDS read is served in 4 passes of 16 lanes: lane bit 5
// and the parity of lane bits 2..4 select the pass, k = (lane bits 3..4,
// 0..1) the place in it; a bank is a 16-byte chunk mod 16.  Pass gp holds
// 16 / CB consecutive offset blocks x all cell blocks.  In FP64 (CB = 16
// blocks of 4 cells) that is one offset block, whose reads start at chunks
// 2 cb + const: cell blocks 8 apart share a bank (two-way conflicts).
template <typename T, int GX>
struct GatherThread {
  static constexpr int GCX = gather_cx<T>(), BH = GBH, CB = GX / GCX, NACC = GCX * BH;
  int sl, t, hg, cb, ubase, vbase, sv, xs;
  int64_t rb;
  bool comp;
  __device__ explicit GatherThread(const GatherArgs &a) {
    int b = blockIdx.x;
    b = xcd_block(b, a.nblk);  // XCD-aware: a row's
    const int row = b / a.nseg;                                       // segments share an L2
    xs = (b % a.nseg) * GX;
    rb = (int64_t)row * a.nx;
    sl = threadIdx.x / a.slice_thr;
    t = threadIdx.x % a.slice_thr;
    const int l = t & 63, q = (l >> 2) & 7;
    const int gp = 4 * (t >> 6) + 2 * (l >> 5) + (__builtin_popcount(q) & 1);
    const int k = 4 * (q >> 1) + (l & 3);
    hg = gp * (16 / CB) + k / CB;
    cb = k % CB;
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

// FP32 on the matrix cores.  With a = x + h and b = x - h the volume is
// G[h + nh][x] = scale sum_i U[i][a] V[i][b] over the pairs with a - b = 2h:
// a band of the product U^T V whose a and b share a parity.  A wave-tile is
// 16 cells a = a_t + 2m of one parity (32 cells of the row), multiplied by
// NBT tiles of 16 cells b = a_t - 2 nh + 2 (16 bt + n), which hold every b the
// 2 nh + 1 offsets of those a need (1.19 x the needed products at nh = 40), on
// v_mfma_f32_16x16x4f32 (4 probe rows per instruction, FP32 products and
// sums).  A workgroup of 4 waves owns a segment of 32 NT cells (2 NT
// wave-tiles, NT / 2 per wave); a wider segment stages less of the V halo
// (the 4 nh cells around the segment) per cell.  Chunks of GR probe rows
// stream straight from global memory into three LDS buffers by buffer loads,
// two chunks in flight; the buffers are distinct arrays alternated
// statically, so the compiler can tell the loads in flight from the reads
// and does not wait for the former before the latter.  Staged rows keep the
// even cells of each 64-cell group in its first 32 slots and the odd cells in
// the last 32, so a lane group's 16 same-parity cells are 16 consecutive
// words; the row stride is 16 mod 64 words so the 4 probe rows of one
// instruction fall in distinct banks.  The products go out through LDS in
// rounds of TR 32-cell tiles, an array [h + nh][a - a_round] whose rows are
// written as consecutive x for each offset.
typedef float gv4f __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int gm_ug(int nt) { return (nt + 1) / 2; }         // U groups of 64
__host__ __device__ constexpr int gm_vg(int nt, int nbt) { return (nt + nbt + 1) / 2; }  // V groups
__host__ __device__ constexpr int gm_lsu(int nt) { return 64 * gm_ug(nt) + 16; }
__host__ __device__ constexpr int gm_lsv(int nt, int nbt) { return 64 * gm_vg(nt, nbt) + 16; }
__host__ __device__ constexpr int gm_buf(int nt, int nbt, int gr) {
  return gr * (gm_lsu(nt) + gm_lsv(nt, nbt));
}
// staged slot of column c
__device__ __forceinline__ int gm_slot(int c) { return (c & ~63) + 32 * (c & 1) + ((c & 63) >> 1); }

template <int NBT, int NT, int GR>
__global__ __launch_bounds__(256) void k_offset_gathers_mfma(const float *__restrict__ U,
                                                             const float *__restrict__ V,
                                                             GatherArgs a, float scale,
                                                             float *__restrict__ G) {
  constexpr int UG = gm_ug(NT), VG = gm_vg(NT, NBT), LSU = gm_lsu(NT), LSV = gm_lsv(NT, NBT);
  constexpr int BUFN = gm_buf(NT, NBT, GR), NGRP = UG + VG, QG = (NGRP + 3) / 4, NQ = NT / 2;
  constexpr int W = 32 * NT, VL = 32 * (NT + NBT);  // segment cells; V columns read
  constexpr int PER = QG * GR;  // loads per wave per chunk
  constexpr int VMW = 0x0F70 | (PER & 15) | ((PER >> 4) << 14);  // s_waitcnt vmcnt(PER)
  static_assert(NT % 2 == 0 && GR % 4 == 0 && PER < 64, "tile shape");
  __shared__ __align__(16) float SA[BUFN + 64];  // + a spare row for loads past the groups
  __shared__ __align__(16) float SB[BUFN + 64];
  __shared__ __align__(16) float SC[BUFN + 64];
  int blk = blockIdx.x;
  blk = xcd_block(blk, a.nblk);  // XCD-aware
  const int seg = blk % a.nseg;
  const int64_t rb = (int64_t)(blk / a.nseg) * a.nx;
  const int a0 = seg * W;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  // staging: wave w loads groups w + 4 j (U groups first, then V; groups past
  // the last go to a spare row); lane l of a group holds column
  // 2 (l % 32) + l / 32 of it, which lands in slot l.  Buffer loads address
  // this x row's tiles; an offset past them (a cell outside the row, a probe
  // row past r) reads zero, so every wave issues the same loads per chunk.
  const int64_t t0row = rb >> 5;
  const uint32_t nrec = (uint32_t)((((rb + a.nx - 1) >> 5) - t0row + 1) * a.r * 128);
  constexpr uint32_t OOR = 0x80000000u;  // >= nrec
  const int cg = 2 * (lane & 31) + (lane >> 5);
  uint32_t goff[QG];
#pragma unroll
  for (int j = 0; j < QG; ++j) {
    const int g = w + 4 * j;
    const int c = g < UG ? 64 * g + cg : 64 * (g - UG) + cg;
    const int x = g < UG ? a0 + c : a0 - 2 * a.nh + c;
    const bool ok = g < NGRP && x >= 0 && x < a.nx && (g < UG || c < VL);
    const int64_t cell = rb + x;
    goff[j] = ok ? (uint32_t)((((cell >> 5) - t0row) * a.r * 32 + (cell & 31)) * 4) : OOR;
  }
  const int cpf = (a.r + GR - 1) / GR, nch = a.nfield * cpf;
  auto issue = [&](int c, float *S) {
    const int f = c / cpf, i0 = (c % cpf) * GR;
    const int64_t fb = f * a.fstride + t0row * a.r * 32;
    const __amdgpu_buffer_rsrc_t ru =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(U + fb), (short)0, (int)nrec, 0x00020000);
    const __amdgpu_buffer_rsrc_t rv =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(V + fb), (short)0, (int)nrec, 0x00020000);
#pragma unroll
    for (int j = 0; j < QG; ++j) {
      const int g = w + 4 * j;
      float *dst = g < UG ? S + 64 * g : g < NGRP ? S + GR * LSU + 64 * (g - UG) : S + BUFN;
      const int ls = g < UG ? LSU : g < NGRP ? LSV : 0;
#pragma unroll
      for (int ii = 0; ii < GR; ++ii) {
        const uint32_t off = i0 + ii < a.r ? goff[j] + (uint32_t)(i0 + ii) * 128u : OOR;
        if (g < UG) __builtin_amdgcn_raw_ptr_buffer_load_lds(ru, dst + ii * ls, 4, off, 0, 0, 0);
        else __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, dst + ii * ls, 4, off, 0, 0, 0);
      }
    }
  };
  // wave-tile q of this wave: cells a0 + 32 t_q + p + 2 m, t_q = w / 2 + 2 q;
  // lane l holds operand row / column l % 16 and probe row 4 s + l / 16 of
  // each 4-row step
  const int p = w & 1, kq = lane >> 4, ln = lane & 15;
  const int posu = kq * LSU + gm_slot(32 * (w >> 1) + p + 2 * ln);
  int posv[NBT];
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt)
    posv[bt] = GR * LSU + kq * LSV + gm_slot(32 * ((w >> 1) + bt) + p + 2 * ln);
  bool act[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) act[q] = a0 + 32 * ((w >> 1) + 2 * q) + p < a.nx;
  gv4f acc[NQ][NBT];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int bt = 0; bt < NBT; ++bt) acc[q][bt] = gv4f{0.f, 0.f, 0.f, 0.f};
  auto mult = [&](const float *S, int c) {
    const int nst = (min(GR, a.r - (c % cpf) * GR) + 3) >> 2;
    for (int s = 0; s < nst; ++s) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (act[q]) {
          const float av = S[posu + 64 * q + 4 * s * LSU];
#pragma unroll
          for (int bt = 0; bt < NBT; ++bt)
            acc[q][bt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, S[posv[bt] + 64 * q + 4 * s * LSV],
                                                              acc[q][bt], 0, 0, 0);
        }
      }
    }
  };
  // three buffers, two chunks in flight: waiting for chunk k leaves the PER
  // loads of chunk k + 1 outstanding.  The barrier is a bare s_barrier: a
  // workgroup fence would wait for every load in flight.  The loop writes LDS
  // only through those loads, and the reads before it are consumed before it;
  // the empty asm statements keep the compiler from moving memory accesses
  // across it.
  auto wait_chunk = [&](int k) {
    if (k + 1 < nch) __builtin_amdgcn_s_waitcnt(VMW);
    else __builtin_amdgcn_s_waitcnt(0x0F70);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();  // everyone's loads of chunk k; chunk k - 1 is multiplied out
    asm volatile("" ::: "memory");
  };
  issue(0, SA);
  if (1 < nch) issue(1, SB);
  for (int c = 0; c < nch; c += 3) {
    wait_chunk(c);
    if (c + 2 < nch) issue(c + 2, SC);
    mult(SA, c);
    if (c + 1 >= nch) break;
    wait_chunk(c + 1);
    if (c + 3 < nch) issue(c + 3, SA);
    mult(SB, c + 1);
    if (c + 2 >= nch) break;
    wait_chunk(c + 2);
    if (c + 4 < nch) issue(c + 4, SB);
    mult(SC, c + 2);
  }
  // products -> O[H][j] (H = h + nh, j = a - a0 - 32 t0) in rounds of TR tiles,
  // row stride 32 TR + 1, spread over the three buffers
  const int nout = 2 * a.nh + 1, TR = a.hgs, OS = 32 * TR + 1;
  auto oref = [&](int e) -> float & { return e < BUFN ? SA[e] : e < 2 * BUFN ? SB[e - BUFN] : SC[e - 2 * BUFN]; };
  for (int t0 = 0; t0 < NT; t0 += TR) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int tq = (w >> 1) + 2 * q;
      if (act[q] && tq >= t0 && tq < t0 + TR) {
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = 4 * kq + v, H = m - 16 * bt - ln + 2 * a.nh;
            if (H >= 0 && H <= 2 * a.nh) oref(H * OS + 32 * (tq - t0) + p + 2 * m) = acc[q][bt][v];
          }
      }
    }
    __syncthreads();
    const int ar = a0 + 32 * t0, mt = min(TR, NT - t0), wr = 32 * mt;
    if ((mt & (mt - 1)) == 0) {
      // a thread keeps column j and steps over offsets; G[H][x] with
      // x = ar + j + nh - H moves by N - 1 words per offset
      const int lw = 5 + __builtin_ctz(mt), j = tid & (wr - 1), hs = 256 >> lw;
      const bool okj = ar + j < a.nx;
      const int64_t step = (int64_t)hs * (a.N - 1);
      int H = tid >> lw;
      float *gp = G + rb + ar + j + a.nh + (int64_t)H * (a.N - 1);
      for (; H < nout; H += hs, gp += step) {
        const int x = ar + j + a.nh - H;
        if (okj && x >= 0 && x < a.nx) *gp = scale * oref(H * OS + j);
      }
    } else {
      for (int e = tid; e < nout * wr; e += 256) {
        const int H = e / wr, j = e - H * wr, x = ar + j + a.nh - H;
        if (ar + j < a.nx && x >= 0 && x < a.nx) G[(int64_t)H * a.N + rb + x] = scale * oref(H * OS + j);
      }
    }
  }
  // cells with a outside the row are zero: the first segment writes them for
  // h < 0 (x < -h), the last for h > 0 (x >= nx - h)
  const bool first = seg == 0, last = seg == a.nseg - 1;
  if (first || last) {
    for (int e = tid; e < nout * 64; e += 256) {
      const int H = e >> 6, j = e & 63, h = H - a.nh;
      float *Gh = G + (int64_t)H * a.N + rb;
      if (first && h < 0 && j < -h && j < a.nx) Gh[j] = 0.f;
      const int xl = a.nx - 1 - j;
      if (last && h > 0 && j < h && xl >= 0) Gh[xl] = 0.f;
    }
  }
}

// rounds of 32-cell tiles whose products fit the three staging buffers (the
// output rows leave through the same LDS)
template <int NBT, int NT, int GR>
static int gm_rounds(int nh) {
  const int nout = 2 * nh + 1, room = 3 * gm_buf(NT, NBT, GR);
  int tr = NT;
  while (tr > 1 && nout * (32 * tr + 1) > room) --tr;
  return nout * (32 * tr + 1) <= room ? tr : 0;
}

template <int NBT, int NT, int GR>
static hipError_t gm_launch(const float *U, const float *V, GatherArgs a, int64_t rows, double scale,
                            float *G, hipStream_t st) {
  a.nseg = (a.nx + 32 * NT - 1) / (32 * NT);
  // a row's tiles are addressed with 32-bit byte offsets below 2^31
  if (((int64_t)a.nx / 32 + 2) * a.r * 128 >= (int64_t)1 << 31) return hipErrorInvalidValue;
  const int64_t nb = rows * a.nseg;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  a.nblk = (int)nb;
  a.hgs = gm_rounds<NBT, NT, GR>(a.nh);
  if (a.hgs < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_offset_gathers_mfma<NBT, NT, GR>), dim3(a.nblk), dim3(256), 0, st, U, V, a,
                     (float)scale, G);
  return hipGetLastError();
}

template <int NT, int GR>
static hipError_t gm_dispatch(const float *U, const float *V, GatherArgs a, int64_t rows,
                              double scale, float *G, hipStream_t st) {
  switch ((16 + 2 * a.nh + 15) / 16) {
    case 1: return gm_launch<1, NT, GR>(U, V, a, rows, scale, G, st);
    case 2: return gm_launch<2, NT, GR>(U, V, a, rows, scale, G, st);
    case 3: return gm_launch<3, NT, GR>(U, V, a, rows, scale, G, st);
    case 4: return gm_launch<4, NT, GR>(U, V, a, rows, scale, G, st);
    case 5: return gm_launch<5, NT, GR>(U, V, a, rows, scale, G, st);
    case 6: return gm_launch<6, NT, GR>(U, V, a, rows, scale, G, st);
    case 7: return gm_launch<7, NT, GR>(U, V, a, rows, scale, G, st);
    case 8: return gm_launch<8, NT, GR>(U, V, a, rows, scale, G, st);
    case 9: return gm_launch<9, NT, GR>(U, V, a, rows, scale, G, st);
  }
  return hipErrorInvalidValue;
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
  GatherArgs a;
  a.fstride = fstride;
  a.N = N;
  a.nfield = nfield;
  a.nx = nx;
  a.r = r;
  a.nh = nh;
  const int64_t rows = N / nx;
  if (rows <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    // 128-cell segments, chunks of 8 probe rows
    return gm_dispatch<4, 8>(U, V, a, rows, scale, G, st);
  } else {
    constexpr int GCX = gather_cx<T>(), gx = 64, CB = gx / GCX;
    a.hgs = (2 * nh + 1 + GBH - 1) / GBH;          // offset blocks
    a.slice_thr = 64 * ((a.hgs * CB + 63) / 64);  // whole waves of (offset, cell) blocks
    a.nslice = 256 / a.slice_thr;
    const int nthr = a.nslice * a.slice_thr;
    a.nseg = (nx + gx - 1) / gx;
    const int64_t nblk = rows * a.nseg;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    a.nblk = (int)nblk;
    const int ls = gather_ls(gx, nh);
    const size_t reduce = (size_t)a.slice_thr * (GCX * GBH / 3);
    const size_t stage = 2 * (size_t)GIC * ls;
    const size_t lds = (stage > reduce ? stage : reduce) * sizeof(T);
    hipLaunchKernelGGL((k_offset_gathers<T>), dim3(a.nblk), dim3(nthr), lds, st, U, V, a,
                       (T)scale, G);
    return hipGetLastError();
  }
}
template hipError_t launch_offset_gathers<float>(const float *, const float *, int, int64_t,
                                                 int64_t, int, int, int, double, float *,
                                                 hipStream_t);
template hipError_t launch_offset_gathers<double>(const double *, const double *, int, int64_t,
                                                  int64_t, int, int, int, double, double *,
                                                  hipStream_t);

}  // namespace rtm
