// Range-finder probes (Section "Randomized trace estimation": probing vectors
// from a partial QR factorization of A Z, Z a Rademacher +-1 matrix).  A is
// the forward history H [nt][N] of u_tt and Z a sign matrix Omega [N][r] in
// space, so the probes are the orthonormal columns of
//     Y [nt][r] = H Omega,   Q = orth(Y).
// Omega[x][i] = 1 - 2 b, b = bit (i % 64) of word (i / 64) of the
// Philox4x64-10 block with key (seed, 0) at counter (x + 1, 0, 0, 0)
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC 2011), regenerated per cell instead of stored.
//
//   k_sketch_mfma    FP32: every k-step block stages a 64-cell chunk of the
//                    block's levels and the chunk's sign words in LDS; wave w
//                    contracts cells 16 w .. 16 w + 15 on MFMA
//                    (v_mfma_f32_32x32x16_bf16, u_tt as bf16 hi + lo, signs
//                    exact): C[t][i] += sum_x u_tt[t][x] Omega[x][i].  Per-wave
//                    partial sums go to scratch.
//   k_sketch_vec     FP64 (and any shape): the same sum with FMAs, one (t, i)
//                    pair set per thread, per-workgroup partials.
//   k_sketch_reduce  fixed-order FP64 sum of the partials into the block's
//                    rows of Y.
//   k_orthonormalize one workgroup, FP64 classical Gram-Schmidt applied twice
//                    per column; a column whose remainder is below 1e-12 of its
//                    norm (or zero) becomes zero.
#include "ring.h"

namespace rtm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 sk_bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float sk_f32x16;

// Philox4x64-10 block at counter (c0, 0, 0, 0), key (k0, 0)
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t k0, uint64_t w[4]) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = 0, x2 = 0, x3 = 0, k1 = 0;
#pragma unroll
  for (int rd = 0; rd < 10; ++rd) {
    if (rd) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
  }
  w[0] = x0;
  w[1] = x1;
  w[2] = x2;
  w[3] = x3;
}

constexpr int SK_CELLS = 64;   // cells per staged chunk
constexpr int SK_MAXW = 8;     // sign words per cell (r <= 256)

// sign words of cell x (32 bits each, word k = bits 32 k .. 32 k + 31)
__device__ __forceinline__ void sign_words(int64_t x, uint64_t seed, int nw, uint32_t *dst,
                                           int stride) {
  uint64_t w[4];
  philox4x64_10((uint64_t)x + 1, seed, w);
#pragma unroll
  for (int k = 0; k < SK_MAXW; ++k)
    if (k < nw) dst[k * stride] = (uint32_t)(w[k >> 1] >> (32 * (k & 1)));
}

// ---------------------------------------------------------------------------
// MFMA sketch (FP32 levels).  MT = ceil(kb / 32) row tiles (steps), NT =
// ceil(r / 32) column tiles (probes), MT * NT <= 8.
// ---------------------------------------------------------------------------
// CELLS cells per staged chunk (256 for blocks of up to 32 steps, 64 above):
// every thread computes one cell's sign words, every wave CELLS / 64 K steps.
template <int MT, int NT, int CELLS>
__global__ __launch_bounds__(256) void k_sketch_mfma(ProbeArgs<float> p, uint64_t seed,
                                                     int64_t chunk, float *__restrict__ partial) {
  // levels s0 - 1 .. s0 + kb, [lev][c] with an odd row stride: the A operand
  // reads one row per lane, so rows must fall in different banks
  constexpr int LS = CELLS + 1;
  __shared__ float Ll[(MT * 32 + 2) * LS];
  __shared__ uint32_t Lb[SK_MAXW * CELLS];        // sign words, [word][c]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int nw = (p.r + 31) >> 5;
  const int nlev = p.kb + 2;
  sk_f32x16 acc[MT * NT];
#pragma unroll
  for (int a = 0; a < MT * NT; ++a)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[a][v] = 0.f;
  const int64_t xb = (int64_t)blockIdx.x * chunk;
  const int64_t xe = xb + chunk < p.N ? xb + chunk : p.N;
  // staging: thread -> cell c = tid % CELLS, levels lv0, lv0 + LSTEP, ...; all
  // of a thread's loads are issued before any is stored to LDS
  constexpr int LSTEP = 256 / CELLS;
  constexpr int NLV = (MT * 32 + 2 + LSTEP - 1) / LSTEP;
  const int sc = threadIdx.x % CELLS, lv0 = threadIdx.x / CELLS;
  for (int64_t c0 = xb; c0 < xe; c0 += CELLS) {
    {
      const int64_t x = c0 + sc;
      float vals[NLV];
#pragma unroll
      for (int k = 0; k < NLV; ++k) {
        const int lv = lv0 + k * LSTEP;
        vals[k] = (lv < nlev && x < xe) ? ring_level(p, p.s0 - 1 + lv)[x] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < NLV; ++k) {
        const int lv = lv0 + k * LSTEP;
        if (lv < nlev) Ll[lv * LS + sc] = vals[k];
      }
    }
    for (int c = threadIdx.x; c < CELLS; c += 256) sign_words(c0 + c, seed, nw, Lb + c, CELLS);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < CELLS / 64; ++ks) {
    const int cb = 64 * ks + 16 * wave + 8 * half;  // this lane's 8 cells of the K step
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int t = mt * 32 + col;
      sk_bf16x8 ahi, alo;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        float d2 = 0.f;
        if (t < p.kb) {
          const float *L = Ll + t * LS + cb + v;
          d2 = (L[2 * LS] - 2.f * L[LS] + L[0]) * p.inv_dt2;
        }
        const __bf16 hb = (__bf16)d2;
        ahi[v] = hb;
        alo[v] = (__bf16)(d2 - (float)hb);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int i = nt * 32 + col;
        sk_bf16x8 b;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const uint32_t wd = Lb[(i >> 5) * CELLS + cb + v];
          const float s = i < p.r ? (((wd >> (i & 31)) & 1u) ? -1.f : 1.f) : 0.f;
          b[v] = (__bf16)s;
        }
        const int a = mt * NT + nt;
        acc[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, b, acc[a], 0, 0, 0);
        acc[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, b, acc[a], 0, 0, 0);
      }
    }
    }
    __syncthreads();
  }
  // C layout: lane l, register v -> row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
  const int kr = p.kb * p.r;
  float *out = partial + ((int64_t)blockIdx.x * 4 + wave) * kr;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int a = mt * NT + nt;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int t = mt * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        const int i = nt * 32 + col;
        if (t < p.kb && i < p.r) out[t * p.r + i] = acc[a][v];
      }
    }
}

// ---------------------------------------------------------------------------
// vector sketch (FP64 or FP32): thread j-th pair p = tid + 256 j, (t, i) =
// (p / r, p % r), kb * r <= 8192
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sketch_vec(ProbeArgs<T> p, uint64_t seed, int64_t chunk,
                                                    T *__restrict__ partial) {
  constexpr int CW = 32;                        // cells per staged chunk
  __shared__ T Ls[128 * CW];                    // u_tt [t][c] (rows read broadcast)
  __shared__ uint32_t Lb[SK_MAXW * CW];         // [word][c]
  const int kr = p.kb * p.r, nw = (p.r + 31) >> 5;
  T acc[32];
  int tof[32], wof[32], bit[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    acc[j] = T(0);
    const int q = threadIdx.x + 256 * j;
    const int t = q < kr ? q / p.r : 0, i = q < kr ? q - t * p.r : 0;
    tof[j] = t * CW;
    wof[j] = (i >> 5) * CW;
    bit[j] = i & 31;
  }
  const int64_t xb = (int64_t)blockIdx.x * chunk;
  const int64_t xe = xb + chunk < p.N ? xb + chunk : p.N;
  for (int64_t c0 = xb; c0 < xe; c0 += CW) {
    for (int e = threadIdx.x; e < p.kb * CW; e += 256) {
      const int t = e / CW, c = e % CW;
      const int64_t x = c0 + c;
      Ls[e] = x < xe ? probed(p, t, x) : T(0);
    }
    if (threadIdx.x < CW) sign_words(c0 + threadIdx.x, seed, nw, Lb + threadIdx.x, CW);
    __syncthreads();
    for (int c = 0; c < CW; ++c) {
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        if (threadIdx.x + 256 * j < kr) {
          const T v = Ls[tof[j] + c];
          acc[j] += ((Lb[wof[j] + c] >> bit[j]) & 1u) ? -v : v;
        }
      }
    }
    __syncthreads();
  }
  T *out = partial + (int64_t)blockIdx.x * kr;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int q = threadIdx.x + 256 * j;
    if (q < kr) out[q] = acc[j];
  }
}

// Two fixed-order stages: group g (blockIdx.y) sums partials g, g + G, ...
// into stage[g][q]; then Y[row0 + t][i] = sum over g of stage[g][q].
constexpr int SK_GROUPS = 64;
template <typename PT>
__global__ __launch_bounds__(256) void k_sketch_reduce(const PT *__restrict__ partial, int nparts,
                                                       int kr, double *__restrict__ stage) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= kr) return;
  double s = 0.0;
  for (int w = blockIdx.y; w < nparts; w += SK_GROUPS) s += (double)partial[(int64_t)w * kr + q];
  stage[(int64_t)blockIdx.y * kr + q] = s;
}

__global__ __launch_bounds__(256) void k_sketch_final(const double *__restrict__ stage, int kr,
                                                      int r, int row0, double *__restrict__ Y) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= kr) return;
  double s = 0.0;
  for (int g = 0; g < SK_GROUPS; ++g) s += stage[(int64_t)g * kr + q];
  const int t = q / r, i = q - t * r;
  Y[(int64_t)(row0 + t) * r + i] = s;
}

int64_t sketch_grid(int64_t N) {
  const int64_t chunks = (N + SK_CELLS - 1) / SK_CELLS;
  return chunks < 1024 ? (chunks > 0 ? chunks : 1) : 1024;
}

// elements of the partial buffer launch_sketch needs (floats for the MFMA
// path, field elements for the vector path; four per workgroup covers both),
// followed by the FP64 stage of the reduction (SK_GROUPS rows, counted in
// doubles = two floats each, so sized for either element type)
int64_t sketch_partial_elems(int64_t N, int kb, int r) {
  return (sketch_grid(N) * 4 + 2 * SK_GROUPS) * (int64_t)kb * r;
}

template <int MT, int NT>
static void sketch_mfma(const ProbeArgs<float> &p, uint64_t seed, int64_t g, int64_t chunk,
                        float *partial, hipStream_t st) {
  if constexpr (MT == 1)
    hipLaunchKernelGGL((k_sketch_mfma<MT, NT, 256>), dim3((unsigned)g), dim3(256), 0, st, p, seed,
                       chunk, partial);
  else
    hipLaunchKernelGGL((k_sketch_mfma<MT, NT, 64>), dim3((unsigned)g), dim3(256), 0, st, p, seed,
                       chunk, partial);
}

template <typename T>
hipError_t launch_sketch(const ProbeArgs<T> &p, uint64_t seed, void *partial, double *Y,
                         hipStream_t st) {
  if (p.kb > 128 || p.r > 256 || p.kb * p.r > 8192) return hipErrorInvalidValue;
  const int64_t g = sketch_grid(p.N);
  int64_t chunk = (p.N + g - 1) / g;
  chunk = (chunk + 255) / 256 * 256;   // whole chunks of either staging width
  const int kr = p.kb * p.r;
  int nparts;
  if constexpr (sizeof(T) == 4) {
    const int MT = (p.kb + 31) / 32, NT = (p.r + 31) / 32;
    float *pf = static_cast<float *>(partial);
    switch (MT * 16 + NT) {
      case 0x11: sketch_mfma<1, 1>(p, seed, g, chunk, pf, st); break;
      case 0x12: sketch_mfma<1, 2>(p, seed, g, chunk, pf, st); break;
      case 0x13: sketch_mfma<1, 3>(p, seed, g, chunk, pf, st); break;
      case 0x14: sketch_mfma<1, 4>(p, seed, g, chunk, pf, st); break;
      case 0x15: sketch_mfma<1, 5>(p, seed, g, chunk, pf, st); break;
      case 0x16: sketch_mfma<1, 6>(p, seed, g, chunk, pf, st); break;
      case 0x17: sketch_mfma<1, 7>(p, seed, g, chunk, pf, st); break;
      case 0x18: sketch_mfma<1, 8>(p, seed, g, chunk, pf, st); break;
      case 0x21: sketch_mfma<2, 1>(p, seed, g, chunk, pf, st); break;
      case 0x22: sketch_mfma<2, 2>(p, seed, g, chunk, pf, st); break;
      case 0x23: sketch_mfma<2, 3>(p, seed, g, chunk, pf, st); break;
      case 0x24: sketch_mfma<2, 4>(p, seed, g, chunk, pf, st); break;
      case 0x31: sketch_mfma<3, 1>(p, seed, g, chunk, pf, st); break;
      case 0x32: sketch_mfma<3, 2>(p, seed, g, chunk, pf, st); break;
      case 0x41: sketch_mfma<4, 1>(p, seed, g, chunk, pf, st); break;
      case 0x42: sketch_mfma<4, 2>(p, seed, g, chunk, pf, st); break;
      default: return hipErrorInvalidValue;
    }
    nparts = (int)(g * 4);
    double *stage = reinterpret_cast<double *>(pf + (int64_t)nparts * kr);
    hipLaunchKernelGGL((k_sketch_reduce<float>), dim3((kr + 255) / 256, SK_GROUPS), dim3(256), 0,
                       st, static_cast<const float *>(partial), nparts, kr, stage);
    hipLaunchKernelGGL(k_sketch_final, dim3((kr + 255) / 256), dim3(256), 0, st, stage, kr, p.r,
                       p.zrow0, Y);
  } else {
    T *pt = static_cast<T *>(partial);
    hipLaunchKernelGGL((k_sketch_vec<T>), dim3((unsigned)g), dim3(256), 0, st, p, seed, chunk, pt);
    nparts = (int)g;
    // the vector path uses g rows of T; the stage starts after 4 g rows of floats
    double *stage = reinterpret_cast<double *>(static_cast<float *>(partial) +
                                               (int64_t)g * 4 * kr);
    hipLaunchKernelGGL((k_sketch_reduce<T>), dim3((kr + 255) / 256, SK_GROUPS), dim3(256), 0, st,
                       static_cast<const T *>(partial), nparts, kr, stage);
    hipLaunchKernelGGL(k_sketch_final, dim3((kr + 255) / 256), dim3(256), 0, st, stage, kr, p.r,
                       p.zrow0, Y);
  }
  return hipGetLastError();
}
template hipError_t launch_sketch<float>(const ProbeArgs<float> &, uint64_t, void *, double *,
                                         hipStream_t);
template hipError_t launch_sketch<double>(const ProbeArgs<double> &, uint64_t, void *, double *,
                                          hipStream_t);

// ---------------------------------------------------------------------------
// orthonormal columns (classical Gram-Schmidt twice, FP64), one workgroup
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_orthonormalize(const double *__restrict__ Y, int nt, int r,
                                                        double *__restrict__ V, T *__restrict__ Q) {
  __shared__ double c[256];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t e = tid; e < (int64_t)nt * r; e += 256) V[e] = Y[e];
  __syncthreads();
  auto col_norm2 = [&](int j) {
    double s = 0.0;
    for (int n = tid; n < nt; n += 256) s += V[(int64_t)n * r + j] * V[(int64_t)n * r + j];
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return tot;
  };
  for (int j = 0; j < r; ++j) {
    const double n0 = col_norm2(j);
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = wave; i < j; i += 4) {
        double s = 0.0;
        for (int n = lane; n < nt; n += 64) s += V[(int64_t)n * r + i] * V[(int64_t)n * r + j];
        s = wave_sum(s);
        if (lane == 0) c[i] = s;
      }
      __syncthreads();
      for (int n = tid; n < nt; n += 256) {
        double d = V[(int64_t)n * r + j];
        for (int i = 0; i < j; ++i) d -= c[i] * V[(int64_t)n * r + i];
        V[(int64_t)n * r + j] = d;
      }
      __syncthreads();
    }
    const double n1 = col_norm2(j);
    const double inv = (n0 > 0.0 && n1 > 1e-24 * n0) ? 1.0 / sqrt(n1) : 0.0;
    for (int n = tid; n < nt; n += 256) V[(int64_t)n * r + j] *= inv;
    __syncthreads();
  }
  for (int64_t e = tid; e < (int64_t)nt * r; e += 256) Q[e] = (T)V[e];
}

template <typename T>
hipError_t launch_orthonormalize(const double *Y, int nt, int r, double *V, T *Q, hipStream_t st) {
  hipLaunchKernelGGL((k_orthonormalize<T>), dim3(1), dim3(256), 0, st, Y, nt, r, V, Q);
  return hipGetLastError();
}
template hipError_t launch_orthonormalize<float>(const double *, int, int, double *, float *,
                                                 hipStream_t);
template hipError_t launch_orthonormalize<double>(const double *, int, int, double *, double *,
                                                  hipStream_t);

}  // namespace rtm
