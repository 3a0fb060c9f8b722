// Finite-difference time step of the damped acoustic wave equation:
//   next = [2 m cur - (m - a) prev + dt^2 L cur] / (m + a),   a = eta dt / 2,
// L the 8th-order Laplacian with the field taken as zero outside the grid.
// Forward and adjoint sweeps use the same step (the operator is symmetric).
//
// Two kernels share one per-cell arithmetic (cell_lap / cell_update), so their
// results are bitwise identical:
//   k_stencil_simple  one thread per cell, neighbours from global memory
//                     (2D grids, FP64 3D, reference for the tiled kernel)
//   k_stencil3d_tiled 3D: a TX x TY column tile per workgroup marches down a
//                     z-chunk; the current plane (with a 4-cell x/y halo)
//                     sits in LDS, double buffered, and the z neighbours in a
//                     9-deep register queue per column.  Loads of plane z+1
//                     are issued before plane z is computed.
#include <algorithm>

#include "step_common.h"

namespace rtm {

// c1 (p1 + m1) + c2 (p2 + m2) + c3 (p3 + m3) + c4 (p4 + m4), fixed order
template <typename T>
__device__ __forceinline__ T axis_sum(const StepArgs<T> &a, T p1, T m1, T p2, T m2, T p3,
                                      T m3, T p4, T m4) {
  T s = a.c1 * (p1 + m1);
  s += a.c2 * (p2 + m2);
  s += a.c3 * (p3 + m3);
  s += a.c4 * (p4 + m4);
  return s;
}

// n / d; for FP32 a hardware reciprocal refined by one Newton step and one
// residual correction (Markstein's scheme), within an ulp of the IEEE
// quotient for the normal, well-scaled operands of the update (slowness
// squared plus damping), in fewer instructions than the IEEE sequence
template <typename T>
__device__ __forceinline__ T quot(T n, T d) {
  return n / d;
}
template <>
__device__ __forceinline__ float quot<float>(float n, float d) {
  float r = __builtin_amdgcn_rcpf(d);
  r = __builtin_fmaf(__builtin_fmaf(-d, r, 1.0f), r, r);
  const float q = n * r;
  return __builtin_fmaf(__builtin_fmaf(-d, q, n), r, q);
}

template <typename T>
__device__ __forceinline__ T cell_update(const StepArgs<T> &a, T u, T up, T m, T lap, T damp) {
  return quot(T(2) * m * u - (m - damp) * up + a.dt2 * lap, m + damp);
}

// ---------------------------------------------------------------------------
// one thread per cell
// ---------------------------------------------------------------------------
template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_stencil_simple(StepArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.N) return;
  const int x = (int)(i % a.nx);
  const int64_t zy = i / a.nx;
  const int y = (int)(zy % a.ny);
  const int z = (int)(zy / a.ny);
  const T *u = a.cur;
  auto U = [&](int zz, int yy, int xx) -> T {
    return (zz >= 0 && zz < a.nz && yy >= 0 && yy < a.ny && xx >= 0 && xx < a.nx)
               ? u[((int64_t)zz * a.ny + yy) * a.nx + xx]
               : T(0);
  };
  const T c = u[i];
  const T lz = axis_sum(a, U(z + 1, y, x), U(z - 1, y, x), U(z + 2, y, x), U(z - 2, y, x),
                        U(z + 3, y, x), U(z - 3, y, x), U(z + 4, y, x), U(z - 4, y, x));
  const T lx = axis_sum(a, U(z, y, x + 1), U(z, y, x - 1), U(z, y, x + 2), U(z, y, x - 2),
                        U(z, y, x + 3), U(z, y, x - 3), U(z, y, x + 4), U(z, y, x - 4));
  T lap;
  if constexpr (NDIM == 3) {
    const T ly = axis_sum(a, U(z, y + 1, x), U(z, y - 1, x), U(z, y + 2, x), U(z, y - 2, x),
                          U(z, y + 3, x), U(z, y - 3, x), U(z, y + 4, x), U(z, y - 4, x));
    lap = ((a.cc * c + lz) + ly) + lx;
  } else {
    lap = (a.cc * c + lz) + lx;
  }
  a.next[i] = cell_update(a, c, a.prev[i], a.m[i], lap, sponge_a(a, z, y, x));
}

// ---------------------------------------------------------------------------
// 3D LDS tile + z-marching register queue
// ---------------------------------------------------------------------------
// NT: streaming (non-temporal) loads of u^{n-1} and m and stores of u^{n+1};
// each is touched once per step and a level (N x 4 B) exceeds the caches.
template <typename T, bool NT>
__device__ __forceinline__ T ld_stream(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T, bool NT>
__device__ __forceinline__ void st_stream(T *p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
// Raw buffer loads over one level (N values): an offset at or past the end
// returns zero, so a cell outside the grid takes the offset `end` (a select)
// instead of a branch around its load.  NT: the non-temporal hint.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t level_rsrc(const T *f, uint32_t end) {
  // gfx9 buffer descriptor word 3: 32-bit data format, no swizzle
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(f), (short)0, (int)end, 0x00020000);
}
template <bool NT>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t o, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)o, 0, NT ? 2 : 0));
}
template <bool NT>
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t o, double) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, 0, NT ? 2 : 0));
}

// element at a 32-bit byte offset from a base held in scalar registers (the
// tiled kernels run on levels below 4 GiB)
template <typename T>
__device__ __forceinline__ T *at(T *p, uint32_t off) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(p) + off);
}
template <typename T>
__device__ __forceinline__ const T *at(const T *p, uint32_t off) {
  return reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + off);
}

// One column tile (bx, by) over planes [z0, z1) of one level.  EPI adds a
// cell-local epilogue for the exact comparator: EPI_D2 writes the second time
// difference of the step, EPI_CORR subtracts (stored u_tt) x (new level) from
// a gradient.
// EH (early halo): the x/y halo of plane z is loaded together with the
// column fronts of plane z (four planes ahead of its use) and held in a short
// register queue, so that a tile's halo loads and its neighbours' interior
// loads of the same plane are issued close together in time (L2 reuse).
// rev: march the chunk from z1 - 1 down to z0 instead of up (same per-cell
// arithmetic: the z terms pair z + j with z - j in a commutative sum, so the
// levels are bitwise the same either way).  Sweeps alternate the direction
// from step to step, so that a step starts on the planes the previous step
// touched last (still in the memory-side cache).
template <typename T, int TX, int TYT, int RY, bool NT, int EPI = EPI_NONE, bool EH = false>
__device__ __forceinline__ void tiled_body(const StepArgs<T> &a, int bx, int by, int z0, int z1,
                                           const EpiArgs<T> &e = EpiArgs<T>{}, bool rev = false) {
  constexpr int NTH = TX * TYT;
  constexpr int TY = TYT * RY;
  constexpr int LX = TX + 8;
  constexpr int LY = TY + 8;
  constexpr int NHY = (8 + TYT - 1) / TYT;        // y-halo rows per thread
  constexpr int NHX = (8 * TY + NTH - 1) / NTH;   // x-halo cells per thread
  __shared__ T lds[2][LY * LX];

  const int tid = threadIdx.x;
  const int tx = tid % TX;
  const int ty = tid / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int x = x0 + tx;
  const uint32_t sp = (uint32_t)a.ny * (uint32_t)a.nx;
  const T *__restrict__ u = a.cur;
  auto off = [&](int zz, int yy, int xx) -> uint32_t {
    return ((uint32_t)zz * sp + (uint32_t)yy * (uint32_t)a.nx + (uint32_t)xx) * (uint32_t)sizeof(T);
  };

  int yr[RY];
  bool in[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    yr[j] = y0 + ty + j * TYT;
    in[j] = (x < a.nx) && (yr[j] < a.ny);
  }
  const uint32_t end = (uint32_t)a.N * (uint32_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t ru = level_rsrc(u, end), rp = level_rsrc(a.prev, end),
                               rm = level_rsrc(a.m, end);
  // no short circuit: one select per load
  auto ldu = [&](int zz, int yy, int xx) -> T {
    const bool ok = (zz >= 0) & (zz < a.nz) & (yy >= 0) & (yy < a.ny) & (xx >= 0) & (xx < a.nx);
    return bload<false>(ru, ok ? off(zz, yy, xx) : end, T(0));
  };
  // the cell's previous level and model value (m = 1 off the grid, never used)
  auto ldpm = [&](int zz, int j, T &pvo, T &mmo) {
    const uint32_t o = in[j] ? off(zz, yr[j], x) : end;
    pvo = bload<NT>(rp, o, T(0));
    const T mv = bload<NT>(rm, o, T(0));
    mmo = in[j] ? mv : T(1);
  };
  // halo bookkeeping: y-halo rows hy = ty + TYT*k (LDS rows 0..3 and TY+4..TY+7),
  // x-halo cells t = tid + NTH*k over TY rows x 8 columns
  int hyr[NHY], hyg[NHY];
  bool hyon[NHY];
#pragma unroll
  for (int k = 0; k < NHY; ++k) {
    const int hy = ty + TYT * k;
    hyon[k] = hy < 8;
    hyr[k] = hy < 4 ? hy : TY + hy;
    hyg[k] = y0 - 4 + hyr[k];
  }
  int hxr[NHX], hxc[NHX];
  bool hxon[NHX];
#pragma unroll
  for (int k = 0; k < NHX; ++k) {
    const int t = tid + NTH * k;
    hxon[k] = t < 8 * TY;
    const int row = t / 8, col = t % 8;
    hxr[k] = 4 + row;
    hxc[k] = col < 4 ? col : TX + col;
  }

  // queue slot k holds plane z + dz (k - 4); the march starts at zs
  const int dz = rev ? -1 : 1;
  const int zs = rev ? z1 - 1 : z0;
  const int nz_chunk = z1 - z0;
  T q[RY][9];
  T front[RY], pv[RY], mm[RY], hyv[NHY], hxv[NHX];
  T es[RY], eg[RY];  // EPI_CORR operands, fetched with the plane they belong to
#pragma unroll
  for (int j = 0; j < RY; ++j) {
#pragma unroll
    for (int k = 0; k < 8; ++k) q[j][k] = ldu(zs + dz * (k - 4), yr[j], x);
    front[j] = ldu(zs + 4 * dz, yr[j], x);
    const uint32_t o = off(zs, yr[j], x);
    ldpm(zs, j, pv[j], mm[j]);
    if constexpr (EPI == EPI_CORR) {
      es[j] = in[j] ? ld_stream<T, NT>(at(e.s, o)) : T(0);
      eg[j] = in[j] ? *at(e.g, o) : T(0);
    }
  }
  // halo of one plane into hy / hx
  auto ldhalo = [&](int zz, T *hy, T *hx) {
#pragma unroll
    for (int k = 0; k < NHY; ++k) hy[k] = hyon[k] ? ldu(zz, hyg[k], x) : T(0);
#pragma unroll
    for (int k = 0; k < NHX; ++k) hx[k] = hxon[k] ? ldu(zz, y0 - 4 + hxr[k], x0 - 4 + hxc[k]) : T(0);
  };
  constexpr int HQ = EH ? 4 : 1;  // early halo: planes z+1..z+4 queued, z+5 in flight
  T hqy[HQ][NHY], hqx[HQ][NHX];
  if constexpr (EH) {
#pragma unroll
    for (int d = 0; d < 4; ++d) ldhalo(zs + dz * d, hqy[d], hqx[d]);
    ldhalo(zs + 4 * dz, hyv, hxv);
  } else {
    ldhalo(zs, hyv, hxv);
  }

  for (int i = 0; i < nz_chunk; ++i) {
    const int z = zs + dz * i;
    T pvc[RY], mmc[RY], hyc[NHY], hxcv[NHX], esc[RY], egc[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      q[j][8] = front[j];
      pvc[j] = pv[j];
      mmc[j] = mm[j];
      if constexpr (EPI == EPI_CORR) {
        esc[j] = es[j];
        egc[j] = eg[j];
      }
    }
    if constexpr (EH) {
#pragma unroll
      for (int k = 0; k < NHY; ++k) hyc[k] = hqy[0][k];
#pragma unroll
      for (int k = 0; k < NHX; ++k) hxcv[k] = hqx[0][k];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < NHY; ++k) hqy[d][k] = hqy[d + 1][k];
#pragma unroll
        for (int k = 0; k < NHX; ++k) hqx[d][k] = hqx[d + 1][k];
      }
#pragma unroll
      for (int k = 0; k < NHY; ++k) hqy[3][k] = hyv[k];
#pragma unroll
      for (int k = 0; k < NHX; ++k) hqx[3][k] = hxv[k];
    } else {
#pragma unroll
      for (int k = 0; k < NHY; ++k) hyc[k] = hyv[k];
#pragma unroll
      for (int k = 0; k < NHX; ++k) hxcv[k] = hxv[k];
    }
    // prefetch plane z + dz
    if (i + 1 < nz_chunk) {
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        front[j] = ldu(z + 5 * dz, yr[j], x);
        const uint32_t o = off(z + dz, yr[j], x);
        ldpm(z + dz, j, pv[j], mm[j]);
        if constexpr (EPI == EPI_CORR) {
          es[j] = in[j] ? ld_stream<T, NT>(at(e.s, o)) : T(0);
          eg[j] = in[j] ? *at(e.g, o) : T(0);
        }
      }
      ldhalo(EH ? z + 5 * dz : z + dz, hyv, hxv);
    }
    T *L = lds[i & 1];
#pragma unroll
    for (int j = 0; j < RY; ++j) L[(ty + j * TYT + 4) * LX + tx + 4] = q[j][4];
#pragma unroll
    for (int k = 0; k < NHY; ++k)
      if (hyon[k]) L[hyr[k] * LX + tx + 4] = hyc[k];
#pragma unroll
    for (int k = 0; k < NHX; ++k)
      if (hxon[k]) L[hxr[k] * LX + hxc[k]] = hxcv[k];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int ly = ty + j * TYT + 4, lx = tx + 4;
      const T *row = L + ly * LX + lx;
      const T c = q[j][4];
      const T lz = axis_sum(a, q[j][5], q[j][3], q[j][6], q[j][2], q[j][7], q[j][1], q[j][8],
                            q[j][0]);
      const T lyv = axis_sum(a, row[LX], row[-LX], row[2 * LX], row[-2 * LX], row[3 * LX],
                             row[-3 * LX], row[4 * LX], row[-4 * LX]);
      const T lxv = axis_sum(a, row[1], row[-1], row[2], row[-2], row[3], row[-3], row[4],
                             row[-4]);
      const T lap = ((a.cc * c + lz) + lyv) + lxv;
      if (in[j]) {
        const uint32_t o = off(z, yr[j], x);
        const T nv = cell_update(a, c, pvc[j], mmc[j], lap, sponge_a(a, z, yr[j], x));
        st_stream<T, NT>(at(a.next, o), nv);
        if constexpr (EPI == EPI_D2)
          st_stream<T, NT>(at(e.d2, o), (nv - T(2) * c + pvc[j]) * e.inv_dt2);
        if constexpr (EPI == EPI_CORR) *at(e.g, o) = egc[j] - esc[j] * nv;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) q[j][k] = q[j][k + 1];
    }
  }
}

template <typename T, int TX, int TYT, int RY, bool NT, int EPI = EPI_NONE, bool EH = false>
__global__ __launch_bounds__(TX *TYT) void k_stencil3d_tiled(StepArgs<T> a, int ntx, int nty,
                                                             int nzc, int zchunk,
                                                             EpiArgs<T> e = EpiArgs<T>{},
                                                             int rev = 0) {
  // XCD-aware order: consecutive hardware block ids go round-robin over the 8
  // XCDs; give each XCD a contiguous run of tiles so halo re-reads hit its L2.
  const int nblk = ntx * nty * nzc;
  int b = blockIdx.x;
  b = xcd_block(b, nblk);
  const int bx = b % ntx;
  const int by = (b / ntx) % nty;
  const int bz = b / (ntx * nty);
  const int z0 = bz * zchunk;
  tiled_body<T, TX, TYT, RY, NT, EPI, EH>(a, bx, by, z0, min(z0 + zchunk, a.nz), e, rev != 0);
}

// Several shots (independent grids, one ring each) in one launch: entry e of
// the tile table names the shot and the tile; the shot's step arguments come
// from a device table (level pointers rebuilt from the step index s).
template <typename T, int TX, int TYT, int RY, bool NT, bool EH = false>
__global__ __launch_bounds__(TX *TYT) void k_stencil3d_batched(const ShotStep<T> *__restrict__ shots,
                                                               const int4 *__restrict__ tiles,
                                                               int ntiles, int s, int rev) {
  int b = blockIdx.x;
  b = xcd_block(b, ntiles);
  const int4 t = tiles[b];  // (shot, bx | by << 16, z0, z1)
  StepArgs<T> a = shots[t.x].a;
  const ShotStep<T> &sh = shots[t.x];
  a.cur = sh.ring + (int64_t)(((s + 1) % sh.R)) * sh.ld;
  a.prev = sh.ring + (int64_t)(((s + sh.R) % sh.R)) * sh.ld;
  a.next = sh.ring + (int64_t)(((s + 2) % sh.R)) * sh.ld;
  tiled_body<T, TX, TYT, RY, NT, EPI_NONE, EH>(a, t.y & 0xffff, t.y >> 16, t.z, t.w,
                                              EpiArgs<T>{}, rev != 0);
}

template <typename T, int TX, int TYT, int RY, bool NT, int EPI = EPI_NONE, bool EH = false>
static void launch_tiled(const StepArgs<T> &a, int target_blocks, hipStream_t st,
                         const EpiArgs<T> &e = EpiArgs<T>{}, int rev = 0) {
  constexpr int TY = TYT * RY;
  const int ntx = (a.nx + TX - 1) / TX;
  const int nty = (a.ny + TY - 1) / TY;
  // split z so that the launch has at least target_blocks workgroups of 256
  // threads' worth (fewer, larger workgroups for the 512 / 1024 thread shapes)
  const int64_t want = (int64_t)target_blocks * 256 / (TX * TYT);
  const int64_t tiles = (int64_t)ntx * nty;
  int nzc = (int)std::min<int64_t>((want + tiles - 1) / tiles, std::max(1, a.nz / 16));
  if (nzc < 1) nzc = 1;
  const int zchunk = (a.nz + nzc - 1) / nzc;  // chunks of at least 16 planes
  nzc = (a.nz + zchunk - 1) / zchunk;
  hipLaunchKernelGGL((k_stencil3d_tiled<T, TX, TYT, RY, NT, EPI, EH>), dim3(ntx * nty * nzc),
                     dim3(TX * TYT), 0, st, a, ntx, nty, nzc, zchunk, e, rev);
}

// tiled variants: id -> (TX, threads in y, rows per thread, non-temporal)
//   1: 64 x 16 (4 x 4)    2: 64 x 32 (4 x 8)    3: 64 x 16 (8 x 2, 512 thr)
//   4: 64 x 16 (2 x 8, 128 thr)    5: 32 x 32 (8 x 4)    6: 128 x 8 (2 x 4)
//   7: as 1, non-temporal          8: as 2, non-temporal
//   9: 64 x 32 (8 x 4, 512 thr), non-temporal
//  10: 64 x 32 (16 x 2, 1024 thr), non-temporal
//  11: as 3, non-temporal
//  12: as 7 and 13: as 9, with early halo loads
template <typename T>
hipError_t launch_stencil(int ndim, const StepArgs<T> &a, int variant, int target_blocks,
                          hipStream_t st, int rev) {
  const EpiArgs<T> e{};
  // the tiled kernels address a level with 32-bit byte offsets
  const bool fits = a.N * (int64_t)sizeof(T) < (int64_t(1) << 32);
  if (ndim == 3 && fits && variant >= kStencilTiled && variant <= kStencilVariants) {
    if constexpr (sizeof(T) == 4) {
      switch (variant) {
        case 2: launch_tiled<T, 64, 4, 8, false>(a, target_blocks, st, e, rev); break;
        case 3: launch_tiled<T, 64, 8, 2, false>(a, target_blocks, st, e, rev); break;
        case 4: launch_tiled<T, 64, 2, 8, false>(a, target_blocks, st, e, rev); break;
        case 5: launch_tiled<T, 32, 8, 4, false>(a, target_blocks, st, e, rev); break;
        case 6: launch_tiled<T, 128, 2, 4, false>(a, target_blocks, st, e, rev); break;
        case 7: launch_tiled<T, 64, 4, 4, true>(a, target_blocks, st, e, rev); break;
        case 8: launch_tiled<T, 64, 4, 8, true>(a, target_blocks, st, e, rev); break;
        case 9: launch_tiled<T, 64, 8, 4, true>(a, target_blocks, st, e, rev); break;
        case 10: launch_tiled<T, 64, 16, 2, true>(a, target_blocks, st, e, rev); break;
        case 11: launch_tiled<T, 64, 8, 2, true>(a, target_blocks, st, e, rev); break;
        case 12: launch_tiled<T, 64, 4, 4, true, EPI_NONE, true>(a, target_blocks, st, e, rev); break;
        case 13: launch_tiled<T, 64, 8, 4, true, EPI_NONE, true>(a, target_blocks, st, e, rev); break;
        default: launch_tiled<T, 64, 4, 4, false>(a, target_blocks, st, e, rev); break;
      }
    } else {
      launch_tiled<T, 64, 4, 4, false>(a, target_blocks, st, e, rev);
    }
  } else {
    const unsigned nblk = (unsigned)((a.N + 255) / 256);
    if (ndim == 3)
      hipLaunchKernelGGL((k_stencil_simple<T, 3>), dim3(nblk), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_stencil_simple<T, 2>), dim3(nblk), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

template hipError_t launch_stencil<float>(int, const StepArgs<float> &, int, int, hipStream_t, int);
template hipError_t launch_stencil<double>(int, const StepArgs<double> &, int, int, hipStream_t,
                                           int);

// Stencil step with an exact-comparator epilogue (3D F32, tiled variants 1
// and 7; other variants use variant 7).  Returns hipErrorInvalidValue for
// grids the tiled kernel does not serve, so the caller falls back to the
// separate kernels.
template <typename T>
hipError_t launch_stencil_epi(int ndim, const StepArgs<T> &a, int variant, int target_blocks,
                              int epi, const EpiArgs<T> &e, hipStream_t st, int rev) {
  if (ndim != 3 || sizeof(T) != 4 || variant < kStencilTiled ||
      a.N * (int64_t)sizeof(T) >= (int64_t(1) << 32))
    return hipErrorInvalidValue;
  if constexpr (sizeof(T) == 4) {
    const bool nt = variant != 1;
    if (epi == EPI_D2) {
      if (nt) launch_tiled<T, 64, 4, 4, true, EPI_D2>(a, target_blocks, st, e, rev);
      else launch_tiled<T, 64, 4, 4, false, EPI_D2>(a, target_blocks, st, e, rev);
    } else if (epi == EPI_CORR) {
      if (nt) launch_tiled<T, 64, 4, 4, true, EPI_CORR>(a, target_blocks, st, e, rev);
      else launch_tiled<T, 64, 4, 4, false, EPI_CORR>(a, target_blocks, st, e, rev);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}
template hipError_t launch_stencil_epi<float>(int, const StepArgs<float> &, int, int, int,
                                              const EpiArgs<float> &, hipStream_t, int);
template hipError_t launch_stencil_epi<double>(int, const StepArgs<double> &, int, int, int,
                                               const EpiArgs<double> &, hipStream_t, int);

// Injection whose increment d = dt^2 acc / (m + a) also updates an
// exact-comparator epilogue output: EPI_D2 adds d / dt^2 to the stored u_tt,
// EPI_CORR subtracts s * d from the gradient.
template <typename T>
__global__ __launch_bounds__(256) void k_inject_epi(StepArgs<T> a, PointTables<T> pt,
                                                    const T *__restrict__ vals, T *field, int epi,
                                                    EpiArgs<T> e) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= pt.ncell) return;
  T acc = T(0);
  for (int j = pt.ioff[c]; j < pt.ioff[c + 1]; ++j) acc += pt.iw[j] * vals[pt.ipt[j]];
  const int64_t i = pt.icell[c];
  const int x = (int)(i % a.nx);
  const int64_t zy = i / a.nx;
  const int y = (int)(zy % a.ny);
  const int z = (int)(zy / a.ny);
  const T d = a.dt2 * acc / (a.m[i] + sponge_a(a, z, y, x));
  field[i] += d;
  if (epi == EPI_D2) e.d2[i] += d * e.inv_dt2;
  if (epi == EPI_CORR) e.g[i] -= e.s[i] * d;
}

template <typename T>
hipError_t launch_inject_epi(const StepArgs<T> &a, const PointTables<T> &pt, const T *vals,
                             T *field, int epi, const EpiArgs<T> &e, hipStream_t st) {
  if (pt.ncell <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_inject_epi<T>), dim3((pt.ncell + 255) / 256), dim3(256), 0, st, a, pt,
                     vals, field, epi, e);
  return hipGetLastError();
}
template hipError_t launch_inject_epi<float>(const StepArgs<float> &, const PointTables<float> &,
                                             const float *, float *, int, const EpiArgs<float> &,
                                             hipStream_t);
template hipError_t launch_inject_epi<double>(const StepArgs<double> &,
                                              const PointTables<double> &, const double *,
                                              double *, int, const EpiArgs<double> &,
                                              hipStream_t);

// ---------------------------------------------------------------------------
// autotuning helpers: a deterministic test pattern and a bitwise comparison
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_pattern(T *p, int64_t n, uint32_t seed, T scale) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;  // Knuth multiplicative hash
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = scale * (T)((int32_t)(h & 0xffff) - 32768) / T(32768);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_count_diff(const T *a, const T *b, int64_t n,
                                                    unsigned long long *count) {
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    c += (a[i] != b[i]) ? 1ull : 0ull;
  if (c) atomicAdd(count, c);
}

template <typename T>
hipError_t launch_pattern(T *p, int64_t n, uint32_t seed, T scale, hipStream_t st) {
  hipLaunchKernelGGL((k_pattern<T>), dim3(4096), dim3(256), 0, st, p, n, seed, scale);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_count_diff(const T *a, const T *b, int64_t n, unsigned long long *count,
                             hipStream_t st) {
  hipLaunchKernelGGL((k_count_diff<T>), dim3(4096), dim3(256), 0, st, a, b, n, count);
  return hipGetLastError();
}
template hipError_t launch_pattern<float>(float *, int64_t, uint32_t, float, hipStream_t);
template hipError_t launch_pattern<double>(double *, int64_t, uint32_t, double, hipStream_t);
template hipError_t launch_count_diff<float>(const float *, const float *, int64_t,
                                             unsigned long long *, hipStream_t);
template hipError_t launch_count_diff<double>(const double *, const double *, int64_t,
                                              unsigned long long *, hipStream_t);

// ---------------------------------------------------------------------------
// point injection (after the step) and sampling
// ---------------------------------------------------------------------------
// field[cell] += dt^2 * (sum_j w_j vals[pt_j]) / (m + a): the source term of
// the step added once the stencil part of the update is done.
template <typename T>
__global__ __launch_bounds__(256) void k_inject(StepArgs<T> a, PointTables<T> pt,
                                                const T *__restrict__ vals, T *field) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= pt.ncell) return;
  T acc = T(0);
  for (int j = pt.ioff[c]; j < pt.ioff[c + 1]; ++j) acc += pt.iw[j] * vals[pt.ipt[j]];
  const int64_t i = pt.icell[c];
  const int x = (int)(i % a.nx);
  const int64_t zy = i / a.nx;
  const int y = (int)(zy % a.ny);
  const int z = (int)(zy / a.ny);
  field[i] += a.dt2 * acc / (a.m[i] + sponge_a(a, z, y, x));
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample(PointTables<T> pt, const T *__restrict__ field,
                                                T *__restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= pt.npts) return;
  T s = T(0);
  for (int j = pt.soff[p]; j < pt.soff[p + 1]; ++j) s += pt.sw[j] * field[pt.sidx[j]];
  out[p] = s;
}

template <typename T>
hipError_t launch_inject(const StepArgs<T> &a, const PointTables<T> &pt, const T *vals, T *field,
                         hipStream_t st) {
  if (pt.ncell <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_inject<T>), dim3((pt.ncell + 255) / 256), dim3(256), 0, st, a, pt, vals,
                     field);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sample(const PointTables<T> &pt, const T *field, T *out, hipStream_t st) {
  if (pt.npts <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sample<T>), dim3((pt.npts + 255) / 256), dim3(256), 0, st, pt, field,
                     out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched shots
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_stencil_batched(const ShotStep<T> *shots, const int4 *tiles, int ntiles, int s,
                                  int variant, hipStream_t st, int rev) {
  if (ntiles <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    switch (variant) {
      case 3:
        hipLaunchKernelGGL((k_stencil3d_batched<T, 64, 8, 2, false>), dim3(ntiles), dim3(512), 0,
                           st, shots, tiles, ntiles, s, rev);
        break;
      case 11:
        hipLaunchKernelGGL((k_stencil3d_batched<T, 64, 8, 2, true>), dim3(ntiles), dim3(512), 0,
                           st, shots, tiles, ntiles, s, rev);
        break;
      case 12:
      case 13:
        hipLaunchKernelGGL((k_stencil3d_batched<T, 64, 4, 4, true, true>), dim3(ntiles),
                           dim3(256), 0, st, shots, tiles, ntiles, s, rev);
        break;
      case 7:
      case 8:
      case 9:
      case 10:  // 64 x 32 variants run the 64 x 16 tile table with the variant 7 kernel
        hipLaunchKernelGGL((k_stencil3d_batched<T, 64, 4, 4, true>), dim3(ntiles), dim3(256), 0,
                           st, shots, tiles, ntiles, s, rev);
        break;
      default:
        hipLaunchKernelGGL((k_stencil3d_batched<T, 64, 4, 4, false>), dim3(ntiles), dim3(256), 0,
                           st, shots, tiles, ntiles, s, rev);
    }
  } else {
    hipLaunchKernelGGL((k_stencil3d_batched<T, 64, 4, 4, false>), dim3(ntiles), dim3(256), 0, st,
                       shots, tiles, ntiles, s, rev);
  }
  return hipGetLastError();
}

// level s+1 of shot sh
template <typename T>
__device__ __forceinline__ T *next_level(const ShotStep<T> &sh, int s) {
  return sh.ring + (int64_t)((s + 2) % sh.R) * sh.ld;
}

template <typename T>
__global__ __launch_bounds__(256) void k_inject_batched(const ShotStep<T> *__restrict__ shots,
                                                        const ShotIO<T> *__restrict__ io,
                                                        BatchPoints<T> pt, int s, int n) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= pt.ncell) return;
  const int sh = pt.ishot[c];
  const T *vals = io[sh].inj + (int64_t)n * io[sh].n_inj;
  T acc = T(0);
  for (int j = pt.ioff[c]; j < pt.ioff[c + 1]; ++j) acc += pt.iw[j] * vals[pt.ipt[j]];
  const StepArgs<T> &a = shots[sh].a;
  const int64_t i = pt.icell[c];
  const int x = (int)(i % a.nx);
  const int64_t zy = i / a.nx;
  const int y = (int)(zy % a.ny);
  const int z = (int)(zy / a.ny);
  T *field = next_level(shots[sh], s);
  field[i] += a.dt2 * acc / (a.m[i] + sponge_a(a, z, y, x));
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample_batched(const ShotStep<T> *__restrict__ shots,
                                                        const ShotIO<T> *__restrict__ io,
                                                        BatchPoints<T> pt, int s, int n) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= pt.npts) return;
  const int sh = pt.sshot[p];
  if (!io[sh].out) return;
  const T *field = next_level(shots[sh], s);
  T v = T(0);
  for (int j = pt.soff[p]; j < pt.soff[p + 1]; ++j) v += pt.sw[j] * field[pt.sidx[j]];
  io[sh].out[(int64_t)n * io[sh].n_smp + pt.slocal[p]] = v;
}

template <typename T>
hipError_t launch_inject_batched(const ShotStep<T> *shots, const ShotIO<T> *io,
                                 const BatchPoints<T> &pt, int s, int n, hipStream_t st) {
  if (pt.ncell <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_inject_batched<T>), dim3((pt.ncell + 255) / 256), dim3(256), 0, st, shots,
                     io, pt, s, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_sample_batched(const ShotStep<T> *shots, const ShotIO<T> *io,
                                 const BatchPoints<T> &pt, int s, int n, hipStream_t st) {
  if (pt.npts <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sample_batched<T>), dim3((pt.npts + 255) / 256), dim3(256), 0, st, shots,
                     io, pt, s, n);
  return hipGetLastError();
}
template hipError_t launch_stencil_batched<float>(const ShotStep<float> *, const int4 *, int, int,
                                                  int, hipStream_t, int);
template hipError_t launch_inject_batched<float>(const ShotStep<float> *, const ShotIO<float> *,
                                                 const BatchPoints<float> &, int, int,
                                                 hipStream_t);
template hipError_t launch_sample_batched<float>(const ShotStep<float> *, const ShotIO<float> *,
                                                 const BatchPoints<float> &, int, int,
                                                 hipStream_t);

template hipError_t launch_inject<float>(const StepArgs<float> &, const PointTables<float> &,
                                         const float *, float *, hipStream_t);
template hipError_t launch_inject<double>(const StepArgs<double> &, const PointTables<double> &,
                                          const double *, double *, hipStream_t);
template hipError_t launch_sample<float>(const PointTables<float> &, const float *, float *,
                                         hipStream_t);
template hipError_t launch_sample<double>(const PointTables<double> &, const double *, double *,
                                          hipStream_t);

}  // namespace rtm
