// Probe accumulation (Eq. 3: Ubar = Q^T u_tt, Vbar = Q^T v with Q = Z): every
// k_block steps the block of probed levels S (k x N, read from the level ring)
// is contracted with the matching k rows of Z:
//     bar[r][N] += Z_b^T (r x k) * S_b (k x N).
// This is the one dense contraction of the method.
//
//   k_probe_mfma  +-1 probes on MFMA: v_mfma_f32_32x32x16_bf16, FP32
//                 accumulate.  Z (+-1) is exact in bf16; S is rounded to bf16
//                 (plain) or split into bf16 hi + bf16 lo (two MFMAs, 16-bit
//                 mantissa).  One wave owns 32 cells and all r rows; the
//                 accumulator tile is loaded from / stored to bar directly
//                 (128-byte rows), Z sits in LDS in A-operand order.
//   k_probe_vec   FP64 / FP32 FMA path (any real Z), thread per cell, 32
//                 probe rows per pass; the accumulation order is the per-step
//                 order bar += z_n s^n.
#include "rtm_internal.h"

namespace rtm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

template <typename T>
__device__ __forceinline__ const T *ring_level(const ProbeArgs<T> &p, int j) {
  int slot = (j + 1) % p.R;
  if (slot < 0) slot += p.R;
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
    for (int i = 0; i < RC; ++i) acc[i] = i < rc ? p.bar[(int64_t)(r0 + i) * p.N + c] : T(0);
    for (int t = 0; t < p.kb; ++t) {
      const T s = probed(p, t, c);
#pragma unroll
      for (int i = 0; i < RC; ++i) acc[i] += zs[t * RC + i] * s;
    }
#pragma unroll
    for (int i = 0; i < RC; ++i)
      if (i < rc) p.bar[(int64_t)(r0 + i) * p.N + c] = acc[i];
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
template <int KS, bool SPLIT, int MODE>
__global__ __launch_bounds__(256) void k_probe_mfma(ProbeArgs<float> p,
                                                    const int8_t *__restrict__ Z, int MT) {
  extern __shared__ bf16x8 ldsA[];  // [MT][KS][64]
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // A = Z_b^T: A[i][t] = Z[zrow0 + zdir t][i], zero for t >= kb or i >= r
  for (int e = threadIdx.x; e < MT * KS * 64; e += 256) {
    const int l = e & 63;
    const int ks = (e >> 6) % KS;
    const int mt = (e >> 6) / KS;
    const int i = mt * 32 + (l & 31);
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = ks * 16 + 8 * (l >> 5) + q;
      float zv = 0.f;
      if (t < p.kb && i < p.r) zv = (float)Z[(int64_t)(p.zrow0 + p.zdir * t) * p.r + i];
      v[q] = (__bf16)zv;
    }
    ldsA[e] = v;
  }
  __syncthreads();

  const int64_t ntiles = (p.N + 31) / 32;
  const int col = lane & 31;
  const int half = lane >> 5;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t c = tile * 32 + col;
    const bool valid = c < p.N;
    bf16x8 bhi[KS], blo[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int tb = ks * 16 + 8 * half;  // first local step of this lane's 8
      float sv[8];
      if (MODE == PROBE_UTT) {
        float lv[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) {
          const int t = tb + q - 1;  // level s0 + t
          lv[q] = (valid && t >= -1 && t <= p.kb) ? ring_level(p, p.s0 + t)[c] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          sv[q] = (tb + q < p.kb) ? (lv[q + 2] - 2.f * lv[q + 1] + lv[q]) * p.inv_dt2 : 0.f;
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int t = tb + q;
          const int lev = p.s0 + t + (MODE == PROBE_NEW ? 1 : 0);
          sv[q] = (valid && t < p.kb) ? ring_level(p, lev)[c] : 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const __bf16 hb = (__bf16)sv[q];
        bhi[ks][q] = hb;
        if (SPLIT) blo[ks][q] = (__bf16)(sv[q] - (float)hb);
      }
    }
    for (int mt = 0; mt < MT; ++mt) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = mt * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        acc[v] = (valid && row < p.r) ? p.bar[(int64_t)row * p.N + c] : 0.f;
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 a = ldsA[(mt * KS + ks) * 64 + lane];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bhi[ks], acc, 0, 0, 0);
        if (SPLIT) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, blo[ks], acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = mt * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        if (valid && row < p.r) p.bar[(int64_t)row * p.N + c] = acc[v];
      }
    }
  }
}

template <int KS, bool SPLIT>
static void launch_mfma_mode(const ProbeArgs<float> &p, const int8_t *Z, int MT, unsigned grid,
                             size_t shm, hipStream_t st) {
  switch (p.mode) {
    case PROBE_UTT:
      hipLaunchKernelGGL((k_probe_mfma<KS, SPLIT, PROBE_UTT>), dim3(grid), dim3(256), shm, st, p,
                         Z, MT);
      break;
    case PROBE_NEW:
      hipLaunchKernelGGL((k_probe_mfma<KS, SPLIT, PROBE_NEW>), dim3(grid), dim3(256), shm, st, p,
                         Z, MT);
      break;
    default:
      hipLaunchKernelGGL((k_probe_mfma<KS, SPLIT, PROBE_CUR>), dim3(grid), dim3(256), shm, st, p,
                         Z, MT);
  }
}

template <int KS>
static void launch_mfma_ks(const ProbeArgs<float> &p, const int8_t *Z, bool split, int MT,
                           unsigned grid, size_t shm, hipStream_t st) {
  if (split)
    launch_mfma_mode<KS, true>(p, Z, MT, grid, shm, st);
  else
    launch_mfma_mode<KS, false>(p, Z, MT, grid, shm, st);
}

hipError_t launch_probe_mfma(const ProbeArgs<float> &p, const int8_t *Z, bool split,
                             hipStream_t st) {
  const int MT = (p.r + 31) / 32;
  int KS = (p.kb + 15) / 16;
  KS = KS <= 1 ? 1 : KS <= 2 ? 2 : KS <= 4 ? 4 : 8;
  if (p.kb > 128) return hipErrorInvalidValue;
  const size_t shm = sizeof(bf16x8) * (size_t)MT * KS * 64;
  const int64_t ntiles = (p.N + 31) / 32;
  int64_t want = (ntiles + 3) / 4;
  const unsigned grid = (unsigned)(want < 2048 ? want : 2048);
  switch (KS) {
    case 1: launch_mfma_ks<1>(p, Z, split, MT, grid, shm, st); break;
    case 2: launch_mfma_ks<2>(p, Z, split, MT, grid, shm, st); break;
    case 4: launch_mfma_ks<4>(p, Z, split, MT, grid, shm, st); break;
    default: launch_mfma_ks<8>(p, Z, split, MT, grid, shm, st); break;
  }
  return hipGetLastError();
}

}  // namespace rtm
