// Probe accumulation (Eq. 3: Ubar = Q^T u_tt, Vbar = Q^T v with Q = Z): every
// k_block steps the block of probed levels S (k x N, read from the level ring)
// is contracted with the matching k rows of Z:
//     bar[r][N] += Z_b^T (r x k) * S_b (k x N).
// This is the one dense contraction of the method.
//
// Compressed fields are stored tile-major: element (i, x) at
//     ((x / 32) * r + i) * 32 + x % 32,
// so the r x 32 block of one 32-cell tile is contiguous (16 KB at r = 128).
//
//   k_probe_mfma  +-1 probes on MFMA, FP32 accumulate.  Z (+-1) is exact in
//                 bf16 and float16.  S is rounded to bf16 (plain,
//                 v_mfma_f32_32x32x16_bf16), split into bf16 hi + bf16 lo (two
//                 MFMAs, 16-bit mantissa), or (F16S) scaled by a power of two
//                 per 16-step chunk and rounded to float16 (11-bit mantissa,
//                 v_mfma_f32_32x32x16_f16), the partial product rescaled
//                 exactly between chunks.  One wave owns one 32-cell tile and
//                 up to 128 probe rows at a time; Z sits in LDS in A-operand
//                 order.
//   k_probe_vec   FP64 / FP32 FMA path (any real Z), thread per cell, 32
//                 probe rows per pass; the accumulation order is the per-step
//                 order bar += z_n s^n.
#include "ring.h"

namespace rtm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ int64_t bar_index(int64_t x, int i, int r) {
  return ((x >> 5) * r + i) * 32 + (x & 31);
}

// ---------------------------------------------------------------------------
// vector path
// ---------------------------------------------------------------------------
template <typename T, typename ZT>
__global__ __launch_bounds__(256) void k_probe_vec(ProbeArgs<T> p, const ZT *__restrict__ Z) {
  constexpr int RC = 32;  // probe rows per pass
  extern __shared__ unsigned char smem_raw[];
  T *zs = reinterpret_cast<T *>(smem_raw);  // [kb][RC]
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = c < p.N;
  for (int r0 = 0; r0 < p.r; r0 += RC) {
    const int rc = min(RC, p.r - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < p.kb * RC; e += 256) {
      const int t = e / RC, i = e % RC;
      zs[e] = i < rc ? T(Z[(int64_t)(p.zrow0 + p.zdir * t) * p.r + r0 + i]) : T(0);
    }
    __syncthreads();
    if (!valid) continue;
    T acc[RC];
#pragma unroll
    for (int i = 0; i < RC; ++i) acc[i] = i < rc ? p.bar[bar_index(c, r0 + i, p.r)] : T(0);
    for (int t = 0; t < p.kb; ++t) {
      const T s = probed(p, t, c);
#pragma unroll
      for (int i = 0; i < RC; ++i) acc[i] += zs[t * RC + i] * s;
    }
#pragma unroll
    for (int i = 0; i < RC; ++i)
      if (i < rc) p.bar[bar_index(c, r0 + i, p.r)] = acc[i];
  }
}

template <typename T>
hipError_t launch_probe_vec(const ProbeArgs<T> &p, const void *Z, bool z_is_i8, hipStream_t st) {
  const unsigned nblk = (unsigned)((p.N + 255) / 256);
  const size_t shm = sizeof(T) * (size_t)p.kb * 32;
  if (z_is_i8)
    hipLaunchKernelGGL((k_probe_vec<T, int8_t>), dim3(nblk), dim3(256), shm, st, p,
                       static_cast<const int8_t *>(Z));
  else
    hipLaunchKernelGGL((k_probe_vec<T, T>), dim3(nblk), dim3(256), shm, st, p,
                       static_cast<const T *>(Z));
  return hipGetLastError();
}
template hipError_t launch_probe_vec<float>(const ProbeArgs<float> &, const void *, bool,
                                            hipStream_t);
template hipError_t launch_probe_vec<double>(const ProbeArgs<double> &, const void *, bool,
                                             hipStream_t);

// ---------------------------------------------------------------------------
// MFMA path
// ---------------------------------------------------------------------------
// v_mfma_f32_32x32x16_bf16 operand layout (64 lanes, l = lane):
//   A (32 x 16): lane l holds A[l % 32][8 (l / 32) + v], v = 0..7
//   B (16 x 32): lane l holds B[8 (l / 32) + v][l % 32]
//   C (32 x 32): lane l, register v holds C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]
// In the tile-major layout the C element of lane l, register v of row tile mt
// sits at tile_base + (mt * 32 + 8 (v / 4) + v % 4) * 32 + (4 (l / 32) * 32 + l % 32):
// one wave-uniform base, one per-lane offset, and immediate row offsets.
//
// FUSED (adjoint): instead of bar += W with W = Z_b^T S_b, the block's W is
// contracted with the forward compressed field right away,
//     img[c] += scale * sum_i Uf[i][c] W[i][c],
// which sums to the probed image of Eq. 3 over the blocks (linearity) without
// ever storing Vbar.
// Z_b^T in A-operand order: ldsA[(mt KS + ks) 64 + l] holds A[mt 32 + l % 32][ks 16 + 8 (l / 32) + 0..7]
// with A[i][t] = Z[zrow0 + zdir t][i], zero for t >= kb or i >= r.
// OP_F16S stores the +-1 entries as float16 (exact as well).
template <int OP>
__device__ __forceinline__ void fill_probe_lds(const ProbeArgs<float> &p, const int8_t *Z, int MT,
                                               int KS, bf16x8 *ldsA) {
  for (int e = threadIdx.x; e < MT * KS * 64; e += blockDim.x) {
    const int l = e & 63;
    const int ks = (e >> 6) % KS;
    const int mt = (e >> 6) / KS;
    const int i = mt * 32 + (l & 31);
    bf16x8 v;
    f16x8 vh;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = ks * 16 + 8 * (l >> 5) + q;
      float zv = 0.f;
      if (t < p.kb && i < p.r) zv = (float)Z[(int64_t)(p.zrow0 + p.zdir * t) * p.r + i];
      v[q] = (__bf16)zv;
      vh[q] = (_Float16)zv;
    }
    ldsA[e] = OP == OP_F16S ? __builtin_bit_cast(bf16x8, vh) : v;
  }
  __syncthreads();
}

// Real probes Q (range finder): the same A-operand order, each value split
// into bf16 hi (ldsA[e]) and bf16 lo (ldsA[MT KS 64 + e]).
__device__ __forceinline__ void fill_probe_lds_q(const ProbeArgs<float> &p, const float *Z, int MT,
                                                 int KS, bf16x8 *ldsA) {
  const int n = MT * KS * 64;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int l = e & 63;
    const int ks = (e >> 6) % KS;
    const int mt = (e >> 6) / KS;
    const int i = mt * 32 + (l & 31);
    bf16x8 hi, lo;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = ks * 16 + 8 * (l >> 5) + q;
      float zv = 0.f;
      if (t < p.kb && i < p.r) zv = Z[(int64_t)(p.zrow0 + p.zdir * t) * p.r + i];
      const __bf16 hb = (__bf16)zv;
      hi[q] = hb;
      lo[q] = (__bf16)(zv - (float)hb);
    }
    ldsA[e] = hi;
    ldsA[n + e] = lo;
  }
  __syncthreads();
}

template <bool QF, int OP>
__device__ __forceinline__ void fill_a(const ProbeArgs<float> &p, const void *Z, int MT, int KS,
                                       bf16x8 *ldsA) {
  if constexpr (QF) fill_probe_lds_q(p, static_cast<const float *>(Z), MT, KS, ldsA);
  else fill_probe_lds<OP>(p, static_cast<const int8_t *>(Z), MT, KS, ldsA);
}

// The B operand of step chunk ks for this lane: its 8 probed values (local
// steps tb .. tb+7, tb = 16 ks + 8 half), rounded to bf16 (hi) and, for
// OP_BF16X2, the bf16 rounding of the remainder (lo).  OP_F16S: the chunk's
// 16 x 32 values (the whole wave) share one power-of-two scale 2^-e with e
// from their largest magnitude (below 2^15 after scaling, so every value is
// in float16 range), and hi holds the float16 rounding of the scaled values;
// e is wave-uniform.  FAST: no masking needed.
template <int MODE, int OP, bool FAST>
__device__ __forceinline__ void probe_operand(const ProbeArgs<float> &p, int ks, int half,
                                              int64_t c, bool valid, bf16x8 &bhi, bf16x8 &blo,
                                              int &e) {
  const int tb = ks * 16 + 8 * half;
  float sv[8];
  if (MODE == PROBE_UTT) {
    float lv[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const int t = tb + q - 1;  // level s0 + t, inside [-1, kb] whenever FAST
      const bool ok = FAST || (valid && t >= -1 && t <= p.kb);
      lv[q] = ok ? ring_level(p, p.s0 + t)[c] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float d2 = (lv[q + 2] - 2.f * lv[q + 1] + lv[q]) * p.inv_dt2;
      sv[q] = (FAST || tb + q < p.kb) ? d2 : 0.f;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = tb + q;
      const int lev = p.s0 + t + (MODE == PROBE_NEW ? 1 : 0);
      const bool ok = FAST || (valid && t < p.kb);
      sv[q] = ok ? ring_level(p, lev)[c] : 0.f;
    }
  }
  if constexpr (OP == OP_F16S) {
    float mx = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) mx = fmaxf(mx, fabsf(sv[q]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    // mx < 2^x with x the frexp exponent: scaled by 2^-(x - 15) it stays below 2^15
    e = mx > 0.f ? __builtin_amdgcn_frexp_expf(mx) - 15 : 0;
    f16x8 hv;
#pragma unroll
    for (int q = 0; q < 8; ++q) hv[q] = (_Float16)ldexpf(sv[q], -e);
    bhi = __builtin_bit_cast(bf16x8, hv);
  } else {
    e = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const __bf16 hb = (__bf16)sv[q];
      bhi[q] = hb;
      if (OP == OP_BF16X2) blo[q] = (__bf16)(sv[q] - (float)hb);
    }
  }
}

// acc += A * B for one 16-step chunk, in the operand type of OP (QF: real
// probes split into hi + lo A operands, B hi only)
template <int OP, bool QF>
__device__ __forceinline__ f32x16 chunk_mfma(const bf16x8 &a, const bf16x8 &alo, const bf16x8 &bhi,
                                             const bf16x8 &blo, f32x16 acc) {
  if constexpr (OP == OP_F16S) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, bhi), acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bhi, acc, 0, 0, 0);
    if (OP == OP_BF16X2) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, blo, acc, 0, 0, 0);
    if (QF) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc, 0, 0, 0);
    return acc;
  }
}

// Fast kernel: full 32-cell tiles [0, tile_end), kb == 16 KS, MT % MTC == 0 -
// no load or store is masked.  MTC row tiles (32 probes each) are accumulated
// together, so their 16 x MTC loads per lane are in flight at once.
// NTB: the compressed fields (Ubar / Vbar, the fused adjoint's forward field)
// are read and written with the non-temporal hint (each is touched once per
// block)
template <typename T, bool NT>
__device__ __forceinline__ T ldb(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T, bool NT>
__device__ __forceinline__ void stb(T *p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

constexpr int kQueueChunk = 4;  // tiles per work-queue grab

__global__ void k_queue_reset(int *q) {
  if (threadIdx.x == 0) *q = 0;
}

template <int KS, int OP, int MODE, bool FUSED, int MTC, bool QF, bool NTB = false>
__global__ __launch_bounds__(256) void k_probe_mfma_fast(ProbeArgs<float> p,
                                                         const void *__restrict__ Z, int MT,
                                                         const float *__restrict__ Uf,
                                                         float *__restrict__ img, float scale,
                                                         int64_t tile_end) {
  extern __shared__ bf16x8 ldsA[];
  fill_a<QF, OP>(p, Z, MT, KS, ldsA);
  const int alo_off = MT * KS * 64;  // QF: the lo halves of A
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 31;
  const int half = lane >> 5;
  const int loff = half * 4 * 32 + col;
  // tiles: each wave strides over them, or (p.queue) takes chunks of kQueueChunk
  // consecutive tiles from a counter, so the tiles in flight stay in one band
  // that moves through the field in order; every wave leaves once a chunk
  // starts past tile_end
  auto grab = [&]() -> int64_t {
    int chunk = 0;
    if (lane == 0) chunk = atomicAdd(p.queue, 1);
    return (int64_t)__builtin_amdgcn_readfirstlane(chunk) * kQueueChunk;
  };
  for (int64_t tile = p.queue ? grab() : (int64_t)blockIdx.x * 4 + wave; tile < tile_end;
       tile = p.queue ? (((tile + 1) % kQueueChunk) ? tile + 1 : grab())
                      : tile + (int64_t)gridDim.x * 4) {
    const int64_t c = tile * 32 + col;
    const int64_t tbase = tile * (int64_t)p.r * 32;
    // short blocks: build every step chunk's operand once per tile; long
    // blocks (KS >= 4): build each right before its MFMAs to bound registers
    constexpr bool kEarly = KS <= 2;
    constexpr bool F16 = OP == OP_F16S;
    bf16x8 bhi_e[kEarly ? KS : 1], blo_e[kEarly ? KS : 1];
    int e_e[kEarly ? KS : 1];
    if (kEarly) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        probe_operand<MODE, OP, true>(p, ks, half, c, true, bhi_e[kEarly ? ks : 0],
                                      blo_e[kEarly ? ks : 0], e_e[kEarly ? ks : 0]);
    }
    float part = 0.f;
    for (int mt0 = 0; mt0 < MT; mt0 += MTC) {
      f32x16 acc[MTC];
      // FUSED: the forward field; F16S (not fused): the old Ubar, added once
      // the block's product is back in absolute units
      float uf[(FUSED || F16) ? MTC : 1][16];
      if (FUSED || F16) {  // issue these loads before the MFMAs
        const float *Ut = (FUSED ? Uf : p.bar) + tbase + mt0 * 32 * 32 + loff;
#pragma unroll
        for (int j = 0; j < MTC; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            acc[j][v] = 0.f;
            uf[(FUSED || F16) ? j : 0][v] = ldb<float, NTB>(Ut + (j * 32 + 8 * (v >> 2) + (v & 3)) * 32);
          }
      } else {
        const float *Ut = p.bar + tbase + mt0 * 32 * 32 + loff;
#pragma unroll
        for (int j = 0; j < MTC; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v)
            acc[j][v] = ldb<float, NTB>(Ut + (j * 32 + 8 * (v >> 2) + (v & 3)) * 32);
      }
      int ecur = 0;  // F16S: acc holds the block's partial product in units of 2^ecur
      // step chunks in groups of at most four, the groups in a rolled loop:
      // an 8-chunk block (k = 128) then needs the registers of a 4-chunk one
      constexpr int KSB = KS < 4 ? KS : 4;
#pragma unroll 1
      for (int ks0 = 0; ks0 < KS; ks0 += KSB) {
#pragma unroll
        for (int kk = 0; kk < KSB; ++kk) {
          const int ks = kEarly ? kk : ks0 + kk;
          bf16x8 bhi, blo;
          int eks;
          if (kEarly) {
            bhi = bhi_e[kEarly ? kk : 0];
            blo = blo_e[kEarly ? kk : 0];
            eks = e_e[kEarly ? kk : 0];
          } else {
            __builtin_amdgcn_sched_barrier(0);
            probe_operand<MODE, OP, true>(p, ks, half, c, true, bhi, blo, eks);
          }
          if (F16) {  // move the partial product to this chunk's units (exact)
#pragma unroll
            for (int j = 0; j < MTC; ++j)
#pragma unroll
              for (int v = 0; v < 16; ++v) acc[j][v] = ldexpf(acc[j][v], ecur - eks);
            ecur = eks;
          }
#pragma unroll
          for (int j = 0; j < MTC; ++j) {
            const int ai = ((mt0 + j) * KS + ks) * 64 + lane;
            acc[j] = chunk_mfma<OP, QF>(ldsA[ai], QF ? ldsA[alo_off + ai] : ldsA[ai], bhi, blo,
                                        acc[j]);
          }
        }
      }
      if (F16) {
#pragma unroll
        for (int j = 0; j < MTC; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            acc[j][v] = ldexpf(acc[j][v], ecur);
            if (!FUSED) acc[j][v] += uf[(FUSED || F16) ? j : 0][v];
          }
      }
      if (FUSED) {
#pragma unroll
        for (int j = 0; j < MTC; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) part += uf[(FUSED || F16) ? j : 0][v] * acc[j][v];
      } else {
        float *Uo = p.bar + tbase + mt0 * 32 * 32 + loff;
#pragma unroll
        for (int j = 0; j < MTC; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v)
            stb<float, NTB>(Uo + (j * 32 + 8 * (v >> 2) + (v & 3)) * 32, acc[j][v]);
      }
    }
    if (FUSED) {
      part += __shfl_xor(part, 32, 64);  // the two lanes that share cell c
      if (half == 0) img[c] += scale * part;
    }
  }
}

// Edge kernel: tiles [tile_begin, ntiles) with any masking (ragged last tile,
// a block shorter than 16 KS, r not a multiple of 32).  One row tile at a time.
template <int KS, int OP, int MODE, bool FUSED, bool QF>
__global__ __launch_bounds__(256) void k_probe_mfma_edge(ProbeArgs<float> p,
                                                         const void *__restrict__ Z, int MT,
                                                         const float *__restrict__ Uf,
                                                         float *__restrict__ img, float scale,
                                                         int64_t tile_begin) {
  constexpr bool F16 = OP == OP_F16S;
  extern __shared__ bf16x8 ldsA[];
  fill_a<QF, OP>(p, Z, MT, KS, ldsA);
  const int alo_off = MT * KS * 64;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 31;
  const int half = lane >> 5;
  const int loff = half * 4 * 32 + col;
  const int64_t ntiles = (p.N + 31) / 32;
  for (int64_t tile = tile_begin + (int64_t)blockIdx.x * 4 + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t c = tile * 32 + col;
    const bool valid = c < p.N;
    const int64_t tbase = tile * (int64_t)p.r * 32;
    bf16x8 bhi[KS], blo[KS];
    int eks[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      probe_operand<MODE, OP, false>(p, ks, half, c, valid, bhi[ks], blo[ks], eks[ks]);
    float part = 0.f;
    for (int mt = 0; mt < MT; ++mt) {
      const float *Ut = (FUSED ? Uf : p.bar) + tbase + mt * 32 * 32 + loff;
      f32x16 acc;
      float uf[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rr = 8 * (v >> 2) + (v & 3);
        const bool ok = valid && mt * 32 + rr + 4 * half < p.r;
        const float val = ok ? Ut[rr * 32] : 0.f;
        acc[v] = (FUSED || F16) ? 0.f : val;
        uf[v] = val;
      }
      int ecur = 0;  // F16S: units 2^ecur of the block's partial product
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (F16) {
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[v] = ldexpf(acc[v], ecur - eks[ks]);
          ecur = eks[ks];
        }
        const int ai = (mt * KS + ks) * 64 + lane;
        acc = chunk_mfma<OP, QF>(ldsA[ai], QF ? ldsA[alo_off + ai] : ldsA[ai], bhi[ks], blo[ks],
                                 acc);
      }
      if (F16) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          acc[v] = ldexpf(acc[v], ecur);
          if (!FUSED) acc[v] += uf[v];
        }
      }
      float *Uo = p.bar + tbase + mt * 32 * 32 + loff;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rr = 8 * (v >> 2) + (v & 3);
        if (FUSED)
          part += uf[v] * acc[v];
        else if (valid && mt * 32 + rr + 4 * half < p.r)
          Uo[rr * 32] = acc[v];
      }
    }
    if (FUSED) {
      part += __shfl_xor(part, 32, 64);
      if (half == 0 && valid) img[c] += scale * part;
    }
  }
}

// process wide (rtm_set_probe_nt): non-temporal compressed-field traffic in the
// fast kernels (default on: 11.3 -> 10.3 ms for the fused adjoint block and
// 23.3 -> 22.8 ms for the forward block at 384 x 512 x 512, r = 128, k = 32)
int g_probe_nt = 1;
void set_probe_nt(int on) { g_probe_nt = on ? 1 : 0; }
int get_probe_nt() { return g_probe_nt; }
// process wide (rtm_set_probe_grid): the workgroups of one probe launch, for
// the kernels that update a compressed field in place (forward, unfused
// adjoint) and for the fused adjoint imaging kernel.  -1 (default,
// automatic): the update kernels of +-1 probes and blocks of at most 32 steps
// take one workgroup per four tiles (no stride), those of longer blocks take tiles in
// order from a work queue in the sweep's workspace (2048 workgroups; without
// a queue, as the fused kernel); the fused kernel is sized so that every wave
// takes 48 tiles, with at least 2048 workgroups (or one per four tiles on
// small grids).  -2: work queue; 0: no stride; > 0: at most that many
// workgroups, striding.
// Each workgroup first stages its probe block in LDS, a cost that grows with
// the block length; the in-place update runs faster when the tiles in flight
// form one band that moves through the field in order than when long-lived
// waves drift apart over it.  At 384 x 512 x 512, r = 128, per launch, on the
// two kinds of 51.5 GB allocation seen (the physical placement of the
// compressed field moves the striding kernels by 15 %, see the notes on
// placement):
//   forward, k = 32:  no stride 20.1-20.5 ms on both; work queue 21.1 ms;
//                     12 tiles per wave 21.7 / 18.6 ms; 2048 workgroups
//                     22.9 / 19.9 ms
//   forward, k = 64:  work queue 21.2 ms, 24 tiles per wave 22.9-23.8 ms,
//                     2048 workgroups 24.5 ms, no stride 32.5 ms
//   forward, k = 128: work queue 28.4 ms, 48 tiles per wave 30.2-31.4 ms,
//                     2048 workgroups 31.1 ms, no stride 54.2 ms
//   fused, k = 32 / 128: 48 tiles per wave 10.1 / 20.9-25.0 ms, 2048
//                     workgroups 10.2-10.3 / 22.3 ms, no stride 12.7 / 21.8 ms,
//                     work queue 12.0 / 34.4 ms
// Real probes (range finder), forward, 300^3, r = 64, k = 32: 12 tiles per
// wave (about 17.6K workgroups) 2.78-2.92 ms, no stride 3.2-4.0 ms, work
// queue 3.2 ms.
int g_probe_grid[2] = {-1, -1};
void set_probe_grid(int cap_update, int cap_fused) {
  g_probe_grid[0] = cap_update < -2 ? -1 : cap_update;
  g_probe_grid[1] = cap_fused < -2 ? -1 : cap_fused;
}
int get_probe_grid(int fused) { return g_probe_grid[fused ? 1 : 0]; }

struct FuseArgs {
  const float *Uf = nullptr;
  float *img = nullptr;
  float scale = 0.f;
};

template <int KS, int OP, int MODE, bool FUSED, bool QF>
static void launch_probe_kernels(const ProbeArgs<float> &p, const void *Z, int MT,
                                 const FuseArgs &f, hipStream_t st) {
  const size_t shm = sizeof(bf16x8) * (size_t)MT * KS * 64 * (QF ? 2 : 1);
  const int64_t ntiles = (p.N + 31) / 32;
  const int64_t nfull = p.N / 32;
  const int set = g_probe_grid[FUSED ? 1 : 0];
  // automatic: update kernels of +-1 probes and blocks of at most 32 steps
  // take one workgroup per four tiles (no stride), those of longer blocks a
  // work queue (when the sweep provides a counter); the fused kernel, real
  // probes (whose staging costs twice as much) and longer blocks without a
  // counter a fixed number of tiles per wave, with at least 2048 workgroups
  const bool queue = p.queue && (set == -2 || (set == -1 && !FUSED && !QF && KS > 2));
  auto grid_for = [set, queue](int64_t tiles) -> unsigned {
    const int64_t want = (tiles + 3) / 4;  // one workgroup per four tiles
    int64_t cap = set > 0 ? set : want;
    if (queue) {
      cap = 2048;  // the waves take the tiles in order from the counter
    } else if (set < 0 && (FUSED || QF || KS > 2)) {
      const int64_t tpw = FUSED ? 48 : 6 * KS;
      cap = (tiles + 4 * tpw - 1) / (4 * tpw);
      if (cap < 2048) cap = 2048;  // small grids: fill the chip
    }
    if (cap > want) cap = want;
    return (unsigned)(cap > 0 ? cap : 1);
  };
  // work queue (fast kernel only): reset the counter, then launch
  ProbeArgs<float> pq = p;
  if (queue) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, p.queue);
  } else {
    pq.queue = nullptr;
  }
  // the fast kernel reads and writes whole 32-row tiles and whole 16-step chunks
  const bool fastk = p.kb == 16 * KS && p.r % 32 == 0;
  int64_t done = 0;
  if (fastk && nfull > 0 && MT % 4 == 0 && !FUSED) {
    if (g_probe_nt)
      hipLaunchKernelGGL((k_probe_mfma_fast<KS, OP, MODE, FUSED, 4, QF, true>),
                         dim3(grid_for(nfull)), dim3(256), shm, st, pq, Z, MT, f.Uf, f.img, f.scale,
                         nfull);
    else
      hipLaunchKernelGGL((k_probe_mfma_fast<KS, OP, MODE, FUSED, 4, QF>), dim3(grid_for(nfull)),
                         dim3(256), shm, st, pq, Z, MT, f.Uf, f.img, f.scale, nfull);
    done = nfull;
  } else if (fastk && nfull > 0 && MT % 2 == 0) {
    if (g_probe_nt)
      hipLaunchKernelGGL((k_probe_mfma_fast<KS, OP, MODE, FUSED, 2, QF, true>),
                         dim3(grid_for(nfull)), dim3(256), shm, st, pq, Z, MT, f.Uf, f.img, f.scale,
                         nfull);
    else
      hipLaunchKernelGGL((k_probe_mfma_fast<KS, OP, MODE, FUSED, 2, QF>), dim3(grid_for(nfull)),
                         dim3(256), shm, st, pq, Z, MT, f.Uf, f.img, f.scale, nfull);
    done = nfull;
  }
  if (done < ntiles)
    hipLaunchKernelGGL((k_probe_mfma_edge<KS, OP, MODE, FUSED, QF>), dim3(grid_for(ntiles - done)),
                       dim3(256), shm, st, p, Z, MT, f.Uf, f.img, f.scale, done);
}

template <int KS, int OP, bool QF>
static void launch_mfma_mode(const ProbeArgs<float> &p, const void *Z, int MT,
                             const FuseArgs &f, hipStream_t st) {
  if (f.img) {  // fused imaging: adjoint levels only
    launch_probe_kernels<KS, OP, PROBE_NEW, true, QF>(p, Z, MT, f, st);
    return;
  }
  switch (p.mode) {
    case PROBE_UTT: launch_probe_kernels<KS, OP, PROBE_UTT, false, QF>(p, Z, MT, f, st); break;
    case PROBE_NEW: launch_probe_kernels<KS, OP, PROBE_NEW, false, QF>(p, Z, MT, f, st); break;
    default: launch_probe_kernels<KS, OP, PROBE_CUR, false, QF>(p, Z, MT, f, st);
  }
}

template <int KS>
static void launch_mfma_ks(const ProbeArgs<float> &p, const void *Z, bool zf32, int op,
                           int MT, const FuseArgs &f, hipStream_t st) {
  if (zf32)
    launch_mfma_mode<KS, OP_BF16X2, true>(p, Z, MT, f, st);
  else if (op == OP_BF16X2)
    launch_mfma_mode<KS, OP_BF16X2, false>(p, Z, MT, f, st);
  else if (op == OP_F16S)
    launch_mfma_mode<KS, OP_F16S, false>(p, Z, MT, f, st);
  else
    launch_mfma_mode<KS, OP_BF16, false>(p, Z, MT, f, st);
}

// op: OP_BF16, OP_BF16X2 or OP_F16S; real probes (zf32) need OP_BF16X2
hipError_t launch_probe_mfma(const ProbeArgs<float> &p, const void *Z, bool zf32, int op,
                             const float *Uf, float *img, float scale, hipStream_t st) {
  const FuseArgs f{Uf, img, scale};
  const int MT = (p.r + 31) / 32;
  int KS = (p.kb + 15) / 16;
  KS = KS <= 1 ? 1 : KS <= 2 ? 2 : KS <= 4 ? 4 : 8;
  if (p.kb > 128 || (zf32 && op != OP_BF16X2)) return hipErrorInvalidValue;
  switch (KS) {
    case 1: launch_mfma_ks<1>(p, Z, zf32, op, MT, f, st); break;
    case 2: launch_mfma_ks<2>(p, Z, zf32, op, MT, f, st); break;
    case 4: launch_mfma_ks<4>(p, Z, zf32, op, MT, f, st); break;
    default: launch_mfma_ks<8>(p, Z, zf32, op, MT, f, st); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// layout conversion: tile-major compressed field -> rows [r][N]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_bar_to_rows(const T *__restrict__ bar, int64_t N, int r,
                                                     T *__restrict__ rows) {
  const int64_t total = (int64_t)r * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / N);
    const int64_t x = e - (int64_t)i * N;
    rows[e] = bar[bar_index(x, i, r)];
  }
}

template <typename T>
hipError_t launch_bar_to_rows(const T *bar, int64_t N, int r, T *rows, hipStream_t st) {
  const int64_t total = (int64_t)r * N;
  if (total <= 0) return hipSuccess;
  int64_t b = (total + 255) / 256;
  hipLaunchKernelGGL((k_bar_to_rows<T>), dim3((unsigned)(b < 16384 ? b : 16384)), dim3(256), 0,
                     st, bar, N, r, rows);
  return hipGetLastError();
}
template hipError_t launch_bar_to_rows<float>(const float *, int64_t, int, float *, hipStream_t);
template hipError_t launch_bar_to_rows<double>(const double *, int64_t, int, double *,
                                               hipStream_t);

}  // namespace rtm
