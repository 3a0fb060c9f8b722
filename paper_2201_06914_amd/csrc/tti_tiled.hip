// Tiled pseudo-acoustic TTI step: the operator of tti.hip (same symbols),
// restructured so that every pass streams its fields once from HBM.
//
// The mixed terms use the identity D_a D_b = D_b D_a, exact for first
// differences on a box with the field taken as zero outside it (the two
// nested zero-extensions cut the same cells), so each unordered pair {a, b} is
// evaluated once with a factor 2:
//   Hz u  = sum_a n_a^2 D_aa u + 2 [n_x n_y D_x (D_y u) + n_x n_z D_z (D_x u)
//                                   + n_y n_z D_z (D_y u)]
//   HzT w = sum_a D_aa (n_a^2 w) + 2 [D_x E_xy + D_z E_xz],
//           E_xy = D_y (n_x n_y w),  E_xz = D_x (n_x n_z w) + D_y (n_y n_z w).
// Each sweep step is two launches over the same tile geometry:
//   forward  k_tti_fprep  in-plane: G = (D_x p, D_y p, D_x q, D_y q)
//            k_tti_fmarch z-march: D_zz and D_z G from register queues, D_xx,
//                         D_yy and D_x (D_y .) from the LDS plane, update
//   adjoint  k_tti_aprep  in-plane: w1 = c1 lp + c2 lq, w2 = c2 lp + lq,
//                         E_xz and E_xy of w1 and w2
//            k_tti_amarch z-march: D_zz (n_z^2 w) and D_z E_xz from queues,
//                         D_xx, D_yy, D_x E_xy from LDS, update
// A workgroup owns a 64 x 8 column tile (one thread per column) and marches a
// z-chunk; the current plane sits in LDS with a 4-cell halo along x and y
// (double buffered, one barrier per plane) and the next plane's loads are in
// flight while the current one is computed.  Intermediates live in the
// plan's scratch slots g[k] (stride N).
#include "tti_common.h"

namespace rtm {

namespace {

constexpr int TX = 64;

// Tile geometry: 64 x TY columns, one thread each; LDS planes of (TY + 8) x 72
// cells hold the tile with a 4-cell halo along x and y (no corners).
template <int TY>
struct Geo {
  static constexpr int NTHR = TX * TY;
  static constexpr int LX = TX + 8;
  static constexpr int LY = TY + 8;
  static constexpr int PL = LY * LX;  // one LDS plane
  static constexpr int NHY = 8 / TY;  // y-halo cells per thread (8 rows x 64)
  static constexpr int NHX = 8 * TY;  // x-halo cells (8 columns x TY rows), one per thread
};

template <int TY>
struct TtiTile {
  using G = Geo<TY>;
  int x, y, lc;  // own column and its LDS offset
  bool in;
  int hyg[G::NHY], hyl[G::NHY];  // y-halo cells (column x): global row, LDS offset
  bool hyon[G::NHY];
  int hxg_y, hxg_x, hxl;  // x-halo cell (threads < NHX)
  bool hxon;
  int cng_y, cng_x, cnl;  // corner cell (threads NHX .. NHX + 63; 4 corners of 4 x 4)
  bool cnon;
};

template <int TY, typename T>
__device__ __forceinline__ TtiTile<TY> tile_of(const StepArgs<T> &a, int bx, int by) {
  using G = Geo<TY>;
  TtiTile<TY> t;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int x0 = bx * TX, y0 = by * TY;
  t.x = x0 + tx;
  t.y = y0 + ty;
  t.in = t.x < a.nx && t.y < a.ny;
  t.lc = (ty + 4) * G::LX + tx + 4;
#pragma unroll
  for (int k = 0; k < G::NHY; ++k) {
    const int h = ty + TY * k;                 // 0..7
    const int hr = h < 4 ? h : TY + h;         // LDS rows 0..3, TY+4..TY+7
    t.hyg[k] = y0 - 4 + hr;
    t.hyl[k] = hr * G::LX + tx + 4;
    t.hyon[k] = t.x < a.nx && t.hyg[k] >= 0 && t.hyg[k] < a.ny;
  }
  const int r = tid / 8, c = tid % 8;
  const int lcx = c < 4 ? c : TX + c;
  t.hxg_y = y0 + r;
  t.hxg_x = x0 - 4 + lcx;
  t.hxl = (4 + r) * G::LX + lcx;
  t.hxon = tid < G::NHX && t.hxg_y < a.ny && t.hxg_x >= 0 && t.hxg_x < a.nx;
  const int cc = tid - G::NHX, cq = cc / 16, crow = (cc % 16) / 4, ccol = cc % 4;
  const int lrow = cq < 2 ? crow : TY + 4 + crow, lcol = (cq & 1) == 0 ? ccol : TX + 4 + ccol;
  t.cng_y = y0 - 4 + lrow;
  t.cng_x = x0 - 4 + lcol;
  t.cnl = lrow * G::LX + lcol;
  t.cnon = cc >= 0 && cc < 64 && t.cng_y >= 0 && t.cng_y < a.ny && t.cng_x >= 0 &&
           t.cng_x < a.nx;
  return t;
}

template <typename T>
__device__ __forceinline__ uint32_t cidx(const StepArgs<T> &a, int z, int y, int x) {
  return (((uint32_t)z * (uint32_t)a.ny + (uint32_t)y) * (uint32_t)a.nx + (uint32_t)x) *
         (uint32_t)sizeof(T);
}
template <typename T>
__device__ __forceinline__ T ldo(const T *f, uint32_t o) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(f) + o);
}
template <typename T>
__device__ __forceinline__ void sto(T *f, uint32_t o, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(f) + o) = v;
}

// field value at (z, y, x), zero where the cell is off (outside the x-y range or
// a plane outside the grid).  A raw buffer load over the field's N values
// returns zero for an offset past the end, so an off cell takes the offset
// N * sizeof(T) instead of a branch around the load.
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t o, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)o, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t o, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, 0, 0));
}
template <typename T>
__device__ __forceinline__ T ldz(const T *f, const StepArgs<T> &a, bool on, int z, int y, int x) {
  const uint32_t end = (uint32_t)a.N * (uint32_t)sizeof(T);
  // gfx9 buffer descriptor word 3: 32-bit data format, no swizzle
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(f), (short)0, (int)end, 0x00020000);
  const bool ok = on & (z >= 0) & (z < a.nz);  // no short circuit: one select
  const uint32_t o = cidx(a, z, y, x);
  return buf_ld(r, ok ? o : end, T(0));
}

// first difference from a 9-value window centred at w[4] (w[4] unused)
template <typename T>
__device__ __forceinline__ T d1q(const TtiArgs<T> &t, const T *w) {
  T s = t.d1 * (w[5] - w[3]);
  s += t.d2 * (w[6] - w[2]);
  s += t.d3 * (w[7] - w[1]);
  s += t.d4 * (w[8] - w[0]);
  return s;
}
// first difference along an LDS row / column (stride st) centred at c
template <typename T>
__device__ __forceinline__ T d1l(const TtiArgs<T> &t, const T *c, int st) {
  T s = t.d1 * (c[st] - c[-st]);
  s += t.d2 * (c[2 * st] - c[-2 * st]);
  s += t.d3 * (c[3 * st] - c[-3 * st]);
  s += t.d4 * (c[4 * st] - c[-4 * st]);
  return s;
}
// second difference (centre included)
template <typename T>
__device__ __forceinline__ T d2q(const TtiArgs<T> &t, const T *w) {
  T s = t.c0 * w[4];
  s += t.a.c1 * (w[5] + w[3]);
  s += t.a.c2 * (w[6] + w[2]);
  s += t.a.c3 * (w[7] + w[1]);
  s += t.a.c4 * (w[8] + w[0]);
  return s;
}
template <typename T>
__device__ __forceinline__ T d2l(const TtiArgs<T> &t, const T *c, int st) {
  T s = t.c0 * c[0];
  s += t.a.c1 * (c[st] + c[-st]);
  s += t.a.c2 * (c[2 * st] + c[-2 * st]);
  s += t.a.c3 * (c[3 * st] + c[-3 * st]);
  s += t.a.c4 * (c[4 * st] + c[-4 * st]);
  return s;
}

template <typename T>
__device__ __forceinline__ T tti_update(const StepArgs<T> &a, T u, T up, T m, T rhs, T damp) {
  return (T(2) * m * u - (m - damp) * up + a.dt2 * rhs) / (m + damp);
}

// the p and q updates of one cell share the denominator m + damp: one
// division and two products instead of two divisions
template <typename T>
__device__ __forceinline__ void tti_update_pq(const StepArgs<T> &a, T m, T damp, T u, T up,
                                              T rhs_p, T w, T wp, T rhs_q, T &pn, T &qn) {
  const T inv = T(1) / (m + damp);
  const T m2 = T(2) * m, md = m - damp;
  pn = (m2 * u - md * up + a.dt2 * rhs_p) * inv;
  qn = (m2 * w - md * wp + a.dt2 * rhs_q) * inv;
}

// block -> (tile, z-chunk), XCD-aware as in the acoustic kernel
__device__ __forceinline__ void block_of(int ntx, int nty, int nzc, int zchunk, int nz, int &bx,
                                         int &by, int &z0, int &z1) {
  const int nblk = ntx * nty * nzc;
  int b = blockIdx.x;
  b = xcd_block(b, nblk);
  bx = b % ntx;
  by = (b / ntx) % nty;
  z0 = (b / (ntx * nty)) * zchunk;
  z1 = min(z0 + zchunk, nz);
}

}  // namespace

// ---------------------------------------------------------------------------
// forward, in-plane: g0 = D_x p, g1 = D_y p, g2 = D_x q, g3 = D_y q
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_fprep(TtiArgs<T> t, int ntx, int nty,
                                                            int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  __shared__ T L[2][2][G::PL];  // [buffer][p, q]
  const int64_t N = a.N;
  T cp, cq, yp[G::NHY], yq[G::NHY], xp, xq;
  auto fetch = [&](int z) {
    cp = ldz(t.p, a, g.in, z, g.y, g.x);
    cq = ldz(t.q, a, g.in, z, g.y, g.x);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      yp[k] = ldz(t.p, a, g.hyon[k], z, g.hyg[k], g.x);
      yq[k] = ldz(t.q, a, g.hyon[k], z, g.hyg[k], g.x);
    }
    xp = ldz(t.p, a, g.hxon, z, g.hxg_y, g.hxg_x);
    xq = ldz(t.q, a, g.hxon, z, g.hxg_y, g.hxg_x);
  };
  fetch(z0);
  for (int z = z0; z < z1; ++z) {
    T *Lp = L[z & 1][0], *Lq = L[z & 1][1];
    Lp[g.lc] = cp;
    Lq[g.lc] = cq;
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      Lp[g.hyl[k]] = yp[k];
      Lq[g.hyl[k]] = yq[k];
    }
    if (threadIdx.x < G::NHX) {
      Lp[g.hxl] = xp;
      Lq[g.hxl] = xq;
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    if (g.in) {
      const uint32_t o = cidx(a, z, g.y, g.x);
      sto(t.g, o, d1l(t, Lp + g.lc, 1));
      sto(t.g + N, o, d1l(t, Lp + g.lc, G::LX));
      sto(t.g + 2 * N, o, d1l(t, Lq + g.lc, 1));
      sto(t.g + 3 * N, o, d1l(t, Lq + g.lc, G::LX));
    }
  }
}

// ---------------------------------------------------------------------------
// forward, z-march
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_fmarch(TtiArgs<T> t, int ntx, int nty,
                                                             int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  __shared__ T L[2][4][G::PL];  // [buffer][p, q, D_y p, D_y q]
  const int64_t N = a.N;
  const T *Gxp = t.g, *Gyp = t.g + N, *Gxq = t.g + 2 * N, *Gyq = t.g + 3 * N;
  // z queues of the own column: p, q, D_x p, D_y p, D_x q, D_y q
  T Qp[9], Qq[9], Qxp[9], Qyp[9], Qxq[9], Qyq[9];
  T f[6];  // queue fronts (plane z + 4)
  for (int k = 0; k < 8; ++k) {
    const int zz = z0 - 4 + k;
    Qp[k] = ldz(t.p, a, g.in, zz, g.y, g.x);
    Qq[k] = ldz(t.q, a, g.in, zz, g.y, g.x);
    Qxp[k] = ldz(Gxp, a, g.in, zz, g.y, g.x);
    Qyp[k] = ldz(Gyp, a, g.in, zz, g.y, g.x);
    Qxq[k] = ldz(Gxq, a, g.in, zz, g.y, g.x);
    Qyq[k] = ldz(Gyq, a, g.in, zz, g.y, g.x);
  }
  // plane values: previous levels, m, coefficients; halos of p, q, D_y p, D_y q
  T pp, qp, mm, c1, c2, nz, ny, nx, yp[G::NHY], yq[G::NHY], xp, xq, xgp, xgq;
  auto fetch = [&](int z) {
    const int zf = z + 4;
    f[0] = ldz(t.p, a, g.in, zf, g.y, g.x);
    f[1] = ldz(t.q, a, g.in, zf, g.y, g.x);
    f[2] = ldz(Gxp, a, g.in, zf, g.y, g.x);
    f[3] = ldz(Gyp, a, g.in, zf, g.y, g.x);
    f[4] = ldz(Gxq, a, g.in, zf, g.y, g.x);
    f[5] = ldz(Gyq, a, g.in, zf, g.y, g.x);
    pp = ldz(t.pp, a, g.in, z, g.y, g.x);
    qp = ldz(t.qp, a, g.in, z, g.y, g.x);
    mm = ldz(a.m, a, g.in, z, g.y, g.x);
    c1 = ldz(t.coef, a, g.in, z, g.y, g.x);
    c2 = ldz(t.coef + N, a, g.in, z, g.y, g.x);
    nz = ldz(t.coef + 2 * N, a, g.in, z, g.y, g.x);
    ny = ldz(t.coef + 3 * N, a, g.in, z, g.y, g.x);
    nx = ldz(t.coef + 4 * N, a, g.in, z, g.y, g.x);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      yp[k] = ldz(t.p, a, g.hyon[k], z, g.hyg[k], g.x);
      yq[k] = ldz(t.q, a, g.hyon[k], z, g.hyg[k], g.x);
    }
    xp = ldz(t.p, a, g.hxon, z, g.hxg_y, g.hxg_x);
    xq = ldz(t.q, a, g.hxon, z, g.hxg_y, g.hxg_x);
    xgp = ldz(Gyp, a, g.hxon, z, g.hxg_y, g.hxg_x);
    xgq = ldz(Gyq, a, g.hxon, z, g.hxg_y, g.hxg_x);
  };
  fetch(z0);
  for (int z = z0; z < z1; ++z) {
    Qp[8] = f[0];
    Qq[8] = f[1];
    Qxp[8] = f[2];
    Qyp[8] = f[3];
    Qxq[8] = f[4];
    Qyq[8] = f[5];
    const T cpp = pp, cqp = qp, cm = mm, cc1 = c1, cc2 = c2, cnz = nz, cny = ny, cnx = nx;
    T *Lp = L[z & 1][0], *Lq = L[z & 1][1], *Lyp = L[z & 1][2], *Lyq = L[z & 1][3];
    Lp[g.lc] = Qp[4];
    Lq[g.lc] = Qq[4];
    Lyp[g.lc] = Qyp[4];
    Lyq[g.lc] = Qyq[4];
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      Lp[g.hyl[k]] = yp[k];
      Lq[g.hyl[k]] = yq[k];
    }
    if (threadIdx.x < G::NHX) {
      Lp[g.hxl] = xp;
      Lq[g.hxl] = xq;
      Lyp[g.hxl] = xgp;
      Lyq[g.hxl] = xgq;
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    if (g.in) {
      const T pzz = d2q(t, Qp), qzz = d2q(t, Qq);
      const T pxx = d2l(t, Lp + g.lc, 1), qxx = d2l(t, Lq + g.lc, 1);
      const T pyy = d2l(t, Lp + g.lc, G::LX), qyy = d2l(t, Lq + g.lc, G::LX);
      const T pxy = d1l(t, Lyp + g.lc, 1), qxy = d1l(t, Lyq + g.lc, 1);
      const T pxz = d1q(t, Qxp), qxz = d1q(t, Qxq);
      const T pyz = d1q(t, Qyp), qyz = d1q(t, Qyq);
      const T lp = (pzz + pyy) + pxx;
      const T mix_p = (cnx * cny) * pxy + (cnx * cnz) * pxz + (cny * cnz) * pyz;
      const T mix_q = (cnx * cny) * qxy + (cnx * cnz) * qxz + (cny * cnz) * qyz;
      const T hzp = ((cnz * cnz) * pzz + (cny * cny) * pyy + (cnx * cnx) * pxx) + T(2) * mix_p;
      const T hzq = ((cnz * cnz) * qzz + (cny * cny) * qyy + (cnx * cnx) * qxx) + T(2) * mix_q;
      const T h0p = lp - hzp;
      const T damp = sponge_a(a, z, g.y, g.x);
      const uint32_t o = cidx(a, z, g.y, g.x);
      sto(t.pn, o, tti_update(a, Qp[4], cpp, cm, cc1 * h0p + cc2 * hzq, damp));
      sto(t.qn, o, tti_update(a, Qq[4], cqp, cm, cc2 * h0p + hzq, damp));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      Qp[k] = Qp[k + 1];
      Qq[k] = Qq[k + 1];
      Qxp[k] = Qxp[k + 1];
      Qyp[k] = Qyp[k + 1];
      Qxq[k] = Qxq[k + 1];
      Qyq[k] = Qyq[k + 1];
    }
  }
}

// ---------------------------------------------------------------------------
// forward, fused: one kernel per step, no intermediates in HBM.  Iteration z
// stages the lead plane z + 4 (p, q with an x/y halo) and the current plane z
// (with corners); D_x and D_y of the lead plane enter register queues (the z
// first differences of the mixed terms need them four planes ahead);
// D_x (D_y .) of the current plane goes through a second LDS stage.  Eight
// warm-up iterations before the chunk fill the queues.
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_ffused(TtiArgs<T> t, int ntx, int nty,
                                                             int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  __shared__ T Lc[2][2][G::PL];   // current plane p, q (with corners), double buffered
  __shared__ T Ll[2][G::PL];      // lead plane p, q
  __shared__ T H[2][TY * G::LX];  // D_y p, D_y q of the current plane, all 72 columns
  const int64_t N = a.N;
  T Qp[9], Qq[9], Xp[9], Yp[9], Xq[9], Yq[9];  // p, q, D_x p, D_y p, D_x q, D_y q
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Qp[k] = T(0);
    Qq[k] = T(0);
    Xp[k] = Yp[k] = Xq[k] = Yq[k] = T(0);
  }
  // prefetched values of the next iteration
  T fp, fq;                                      // lead interior
  T lyp[G::NHY], lyq[G::NHY], lxp, lxq;          // lead halo
  T cyp[G::NHY], cyq[G::NHY], cxp, cxq, ccp, ccq; // current halo and corners
  T pp, qp, mm, c1, c2, nz, ny, nx;              // current cell
  auto fetch = [&](int z) {  // iteration z: lead plane z + 4, current plane z
    const int zl = z + 4;
    fp = ldz(t.p, a, g.in, zl, g.y, g.x);
    fq = ldz(t.q, a, g.in, zl, g.y, g.x);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      lyp[k] = ldz(t.p, a, g.hyon[k], zl, g.hyg[k], g.x);
      lyq[k] = ldz(t.q, a, g.hyon[k], zl, g.hyg[k], g.x);
    }
    lxp = ldz(t.p, a, g.hxon, zl, g.hxg_y, g.hxg_x);
    lxq = ldz(t.q, a, g.hxon, zl, g.hxg_y, g.hxg_x);
    const bool out = z >= z0;
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      cyp[k] = ldz(t.p, a, out && g.hyon[k], z, g.hyg[k], g.x);
      cyq[k] = ldz(t.q, a, out && g.hyon[k], z, g.hyg[k], g.x);
    }
    cxp = ldz(t.p, a, out && g.hxon, z, g.hxg_y, g.hxg_x);
    cxq = ldz(t.q, a, out && g.hxon, z, g.hxg_y, g.hxg_x);
    ccp = ldz(t.p, a, out && g.cnon, z, g.cng_y, g.cng_x);
    ccq = ldz(t.q, a, out && g.cnon, z, g.cng_y, g.cng_x);
    const bool oc = out && g.in;
    pp = ldz(t.pp, a, oc, z, g.y, g.x);
    qp = ldz(t.qp, a, oc, z, g.y, g.x);
    mm = ldz(a.m, a, oc, z, g.y, g.x);
    c1 = ldz(t.coef, a, oc, z, g.y, g.x);
    c2 = ldz(t.coef + N, a, oc, z, g.y, g.x);
    nz = ldz(t.coef + 2 * N, a, oc, z, g.y, g.x);
    ny = ldz(t.coef + 3 * N, a, oc, z, g.y, g.x);
    nx = ldz(t.coef + 4 * N, a, oc, z, g.y, g.x);
  };
  const int zs = z0 - 8;
  fetch(zs);
  for (int z = zs; z < z1; ++z) {
    const bool out = z >= z0;  // uniform over the workgroup
    Qp[8] = fp;
    Qq[8] = fq;
    const T cpp = pp, cqp = qp, cm = mm, cc1 = c1, cc2 = c2, cnz = nz, cny = ny, cnx = nx;
    T *Lp = Lc[z & 1][0], *Lq = Lc[z & 1][1];
    Ll[0][g.lc] = fp;
    Ll[1][g.lc] = fq;
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      Ll[0][g.hyl[k]] = lyp[k];
      Ll[1][g.hyl[k]] = lyq[k];
    }
    if (threadIdx.x < G::NHX) {
      Ll[0][g.hxl] = lxp;
      Ll[1][g.hxl] = lxq;
    }
    if (out) {
      Lp[g.lc] = Qp[4];
      Lq[g.lc] = Qq[4];
#pragma unroll
      for (int k = 0; k < G::NHY; ++k) {
        Lp[g.hyl[k]] = cyp[k];
        Lq[g.hyl[k]] = cyq[k];
      }
      if (threadIdx.x < G::NHX) {
        Lp[g.hxl] = cxp;
        Lq[g.hxl] = cxq;
      }
      if (threadIdx.x >= G::NHX && threadIdx.x < G::NHX + 64) {
        Lp[g.cnl] = ccp;
        Lq[g.cnl] = ccq;
      }
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    // queue fronts: first differences of the lead plane
    Xp[8] = d1l(t, Ll[0] + g.lc, 1);
    Yp[8] = d1l(t, Ll[0] + g.lc, G::LX);
    Xq[8] = d1l(t, Ll[1] + g.lc, 1);
    Yq[8] = d1l(t, Ll[1] + g.lc, G::LX);
    if (out) {
      const int hr = threadIdx.x / TX, hc = threadIdx.x % TX + 4;
      H[0][hr * G::LX + hc] = d1l(t, Lp + g.lc, G::LX);
      H[1][hr * G::LX + hc] = d1l(t, Lq + g.lc, G::LX);
      if (threadIdx.x < G::NHX) {
        const int r = threadIdx.x / 8, lcx = g.hxl - (4 + r) * G::LX;
        H[0][r * G::LX + lcx] = d1l(t, Lp + g.hxl, G::LX);
        H[1][r * G::LX + lcx] = d1l(t, Lq + g.hxl, G::LX);
      }
    }
    __syncthreads();
    if (out && g.in) {
      const int hrow = (threadIdx.x / TX) * G::LX + threadIdx.x % TX + 4;
      const T pzz = d2q(t, Qp), qzz = d2q(t, Qq);
      const T pxx = d2l(t, Lp + g.lc, 1), qxx = d2l(t, Lq + g.lc, 1);
      const T pyy = d2l(t, Lp + g.lc, G::LX), qyy = d2l(t, Lq + g.lc, G::LX);
      const T pxy = d1l(t, H[0] + hrow, 1), qxy = d1l(t, H[1] + hrow, 1);
      const T pxz = d1q(t, Xp), qxz = d1q(t, Xq);
      const T pyz = d1q(t, Yp), qyz = d1q(t, Yq);
      const T lp = (pzz + pyy) + pxx;
      const T mix_p = (cnx * cny) * pxy + (cnx * cnz) * pxz + (cny * cnz) * pyz;
      const T mix_q = (cnx * cny) * qxy + (cnx * cnz) * qxz + (cny * cnz) * qyz;
      const T hzp = ((cnz * cnz) * pzz + (cny * cny) * pyy + (cnx * cnx) * pxx) + T(2) * mix_p;
      const T hzq = ((cnz * cnz) * qzz + (cny * cny) * qyy + (cnx * cnx) * qxx) + T(2) * mix_q;
      const T h0p = lp - hzp;
      const T damp = sponge_a(a, z, g.y, g.x);
      const uint32_t o = cidx(a, z, g.y, g.x);
      sto(t.pn, o, tti_update(a, Qp[4], cpp, cm, cc1 * h0p + cc2 * hzq, damp));
      sto(t.qn, o, tti_update(a, Qq[4], cqp, cm, cc2 * h0p + hzq, damp));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      Qp[k] = Qp[k + 1];
      Qq[k] = Qq[k + 1];
      Xp[k] = Xp[k + 1];
      Yp[k] = Yp[k + 1];
      Xq[k] = Xq[k + 1];
      Yq[k] = Yq[k + 1];
    }
  }
}

// ---------------------------------------------------------------------------
// forward, fused, with a plane ring in LDS: as k_tti_ffused, but the lead
// plane z + 4 (p, q with its x / y halo and corners) stays in a ring of six
// LDS planes and serves as the current plane four iterations later, so p and
// q leave HBM once per step (k_tti_ffused loads the current plane's halo and
// corners a second time).  Six slots: iteration z writes slot (z + 4) mod 6
// while a slower thread may still read slot z - 1 (its current plane) or
// slot z + 3 (its lead plane); both differ from it.
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW, int U = 1, bool LC = false>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_ffused_ring(TtiArgs<T> t, int ntx, int nty,
                                                                  int nzc, int zchunk) {
  using G = Geo<TY>;
  constexpr int NR = 6;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  __shared__ T Lr[NR][2][G::PL];  // plane ring: p, q with halo and corners
  __shared__ T H[2][TY * G::LX];  // D_y p, D_y q of the current plane, all 72 columns
  const int64_t N = a.N;
  T Qp[9], Qq[9], Xp[9], Yp[9], Xq[9], Yq[9];  // p, q, D_x p, D_y p, D_x q, D_y q
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Qp[k] = T(0);
    Qq[k] = T(0);
    Xp[k] = Yp[k] = Xq[k] = Yq[k] = T(0);
  }
  // prefetched values of the next iteration (LC: the current cell's values
  // are loaded at the start of their own iteration instead, so that one set
  // of them is live rather than two)
  T fp, fq;                                      // lead interior
  T lyp[G::NHY], lyq[G::NHY], lxp, lxq, lcp, lcq; // lead halo and corners
  T pp, qp, mm, c1, c2, nz, ny, nx;              // current cell
  const bool corner = threadIdx.x >= G::NHX && threadIdx.x < G::NHX + 64;
  auto fetch_cur = [&](int z) {  // the current cell at z
    const bool oc = z >= z0 && g.in;
    pp = ldz(t.pp, a, oc, z, g.y, g.x);
    qp = ldz(t.qp, a, oc, z, g.y, g.x);
    mm = ldz(a.m, a, oc, z, g.y, g.x);
    c1 = ldz(t.coef, a, oc, z, g.y, g.x);
    c2 = ldz(t.coef + N, a, oc, z, g.y, g.x);
    nz = ldz(t.coef + 2 * N, a, oc, z, g.y, g.x);
    ny = ldz(t.coef + 3 * N, a, oc, z, g.y, g.x);
    nx = ldz(t.coef + 4 * N, a, oc, z, g.y, g.x);
  };
  auto fetch = [&](int z) {  // iteration z: lead plane z + 4 (and the current cell at z)
    const int zl = z + 4;
    fp = ldz(t.p, a, g.in, zl, g.y, g.x);
    fq = ldz(t.q, a, g.in, zl, g.y, g.x);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      lyp[k] = ldz(t.p, a, g.hyon[k], zl, g.hyg[k], g.x);
      lyq[k] = ldz(t.q, a, g.hyon[k], zl, g.hyg[k], g.x);
    }
    lxp = ldz(t.p, a, g.hxon, zl, g.hxg_y, g.hxg_x);
    lxq = ldz(t.q, a, g.hxon, zl, g.hxg_y, g.hxg_x);
    lcp = ldz(t.p, a, g.cnon, zl, g.cng_y, g.cng_x);
    lcq = ldz(t.q, a, g.cnon, zl, g.cng_y, g.cng_x);
    if constexpr (!LC) fetch_cur(z);
  };
  auto slot = [](int plane) { return (plane + 12 * NR) % NR; };  // plane >= z0 - 4 >= -4
  const int zs = z0 - 8;
  fetch(zs);
  // U planes per trip: the queue shifts of the unrolled planes become
  // register renames (only the shifts across a trip remain moves)
  auto step = [&](int z) {
    const bool out = z >= z0;  // uniform over the workgroup
    if constexpr (LC) fetch_cur(z);
    Qp[8] = fp;
    Qq[8] = fq;
    const T cpp = pp, cqp = qp, cm = mm, cc1 = c1, cc2 = c2, cnz = nz, cny = ny, cnx = nx;
    T *Llp = Lr[slot(z + 4)][0], *Llq = Lr[slot(z + 4)][1];
    Llp[g.lc] = fp;
    Llq[g.lc] = fq;
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      Llp[g.hyl[k]] = lyp[k];
      Llq[g.hyl[k]] = lyq[k];
    }
    if (threadIdx.x < G::NHX) {
      Llp[g.hxl] = lxp;
      Llq[g.hxl] = lxq;
    }
    if (corner) {
      Llp[g.cnl] = lcp;
      Llq[g.cnl] = lcq;
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    // queue fronts: first differences of the lead plane
    Xp[8] = d1l(t, Llp + g.lc, 1);
    Yp[8] = d1l(t, Llp + g.lc, G::LX);
    Xq[8] = d1l(t, Llq + g.lc, 1);
    Yq[8] = d1l(t, Llq + g.lc, G::LX);
    const T *Lp = Lr[slot(z)][0], *Lq = Lr[slot(z)][1];
    if (out) {
      const int hr = threadIdx.x / TX, hc = threadIdx.x % TX + 4;
      H[0][hr * G::LX + hc] = d1l(t, Lp + g.lc, G::LX);
      H[1][hr * G::LX + hc] = d1l(t, Lq + g.lc, G::LX);
      if (threadIdx.x < G::NHX) {
        const int r = threadIdx.x / 8, lcx = g.hxl - (4 + r) * G::LX;
        H[0][r * G::LX + lcx] = d1l(t, Lp + g.hxl, G::LX);
        H[1][r * G::LX + lcx] = d1l(t, Lq + g.hxl, G::LX);
      }
    }
    __syncthreads();
    if (out && g.in) {
      const int hrow = (threadIdx.x / TX) * G::LX + threadIdx.x % TX + 4;
      const T pzz = d2q(t, Qp), qzz = d2q(t, Qq);
      const T pxx = d2l(t, Lp + g.lc, 1), qxx = d2l(t, Lq + g.lc, 1);
      const T pyy = d2l(t, Lp + g.lc, G::LX), qyy = d2l(t, Lq + g.lc, G::LX);
      const T pxy = d1l(t, H[0] + hrow, 1), qxy = d1l(t, H[1] + hrow, 1);
      const T pxz = d1q(t, Xp), qxz = d1q(t, Xq);
      const T pyz = d1q(t, Yp), qyz = d1q(t, Yq);
      const T lp = (pzz + pyy) + pxx;
      const T mix_p = (cnx * cny) * pxy + (cnx * cnz) * pxz + (cny * cnz) * pyz;
      const T mix_q = (cnx * cny) * qxy + (cnx * cnz) * qxz + (cny * cnz) * qyz;
      const T hzp = ((cnz * cnz) * pzz + (cny * cny) * pyy + (cnx * cnx) * pxx) + T(2) * mix_p;
      const T hzq = ((cnz * cnz) * qzz + (cny * cny) * qyy + (cnx * cnx) * qxx) + T(2) * mix_q;
      const T h0p = lp - hzp;
      const T damp = sponge_a(a, z, g.y, g.x);
      const uint32_t o = cidx(a, z, g.y, g.x);
      T pn, qn;
      tti_update_pq(a, cm, damp, Qp[4], cpp, cc1 * h0p + cc2 * hzq, Qq[4], cqp, cc2 * h0p + hzq,
                    pn, qn);
      sto(t.pn, o, pn);
      sto(t.qn, o, qn);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      Qp[k] = Qp[k + 1];
      Qq[k] = Qq[k + 1];
      Xp[k] = Xp[k + 1];
      Yp[k] = Yp[k + 1];
      Xq[k] = Xq[k + 1];
      Yq[k] = Yq[k + 1];
    }
  };
  int z = zs;
  if constexpr (U > 1) {
    for (; z + U <= z1; z += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) step(z + u);
    }
  }
  for (; z < z1; ++z) step(z);
}

// ---------------------------------------------------------------------------
// adjoint, in-plane: g0 = w1, g1 = w2, g2 = E_xz(w1), g3 = E_xz(w2),
// g4 = E_xy(w1), g5 = E_xy(w2)
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_aprep(TtiArgs<T> t, int ntx, int nty,
                                                            int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  // [buffer][X1, X2, Y1, Y2, XY1, XY2]: X = n_x n_z w (x taps), Y = n_y n_z w and
  // XY = n_x n_y w (y taps)
  __shared__ T L[2][6][G::PL];
  const int64_t N = a.N;
  const T *c1f = t.coef, *c2f = t.coef + N, *nzf = t.coef + 2 * N, *nyf = t.coef + 3 * N,
          *nxf = t.coef + 4 * N;
  struct Cell {
    T lp, lq, c1, c2, nz, ny, nx;
  };
  auto load = [&](bool on, int z, int y, int x) {
    Cell c;
    c.lp = ldz(t.p, a, on, z, y, x);
    c.lq = ldz(t.q, a, on, z, y, x);
    c.c1 = ldz(c1f, a, on, z, y, x);
    c.c2 = ldz(c2f, a, on, z, y, x);
    c.nz = ldz(nzf, a, on, z, y, x);
    c.ny = ldz(nyf, a, on, z, y, x);
    c.nx = ldz(nxf, a, on, z, y, x);
    return c;
  };
  Cell cc, cy[G::NHY], cx;
  auto fetch = [&](int z) {
    cc = load(g.in, z, g.y, g.x);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) cy[k] = load(g.hyon[k], z, g.hyg[k], g.x);
    cx = load(g.hxon, z, g.hxg_y, g.hxg_x);
  };
  fetch(z0);
  for (int z = z0; z < z1; ++z) {
    T(*B)[G::PL] = L[z & 1];
    const T w1 = cc.c1 * cc.lp + cc.c2 * cc.lq;
    const T w2 = cc.c2 * cc.lp + cc.lq;
    B[0][g.lc] = (cc.nx * cc.nz) * w1;
    B[1][g.lc] = (cc.nx * cc.nz) * w2;
    B[2][g.lc] = (cc.ny * cc.nz) * w1;
    B[3][g.lc] = (cc.ny * cc.nz) * w2;
    B[4][g.lc] = (cc.nx * cc.ny) * w1;
    B[5][g.lc] = (cc.nx * cc.ny) * w2;
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      const Cell &h = cy[k];
      const T v1 = h.c1 * h.lp + h.c2 * h.lq, v2 = h.c2 * h.lp + h.lq;
      B[2][g.hyl[k]] = (h.ny * h.nz) * v1;
      B[3][g.hyl[k]] = (h.ny * h.nz) * v2;
      B[4][g.hyl[k]] = (h.nx * h.ny) * v1;
      B[5][g.hyl[k]] = (h.nx * h.ny) * v2;
    }
    if (threadIdx.x < G::NHX) {
      const T v1 = cx.c1 * cx.lp + cx.c2 * cx.lq, v2 = cx.c2 * cx.lp + cx.lq;
      B[0][g.hxl] = (cx.nx * cx.nz) * v1;
      B[1][g.hxl] = (cx.nx * cx.nz) * v2;
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    if (g.in) {
      const uint32_t o = cidx(a, z, g.y, g.x);
      sto(t.g, o, w1);
      sto(t.g + N, o, w2);
      sto(t.g + 2 * N, o, d1l(t, B[0] + g.lc, 1) + d1l(t, B[2] + g.lc, G::LX));
      sto(t.g + 3 * N, o, d1l(t, B[1] + g.lc, 1) + d1l(t, B[3] + g.lc, G::LX));
      sto(t.g + 4 * N, o, d1l(t, B[4] + g.lc, G::LX));
      sto(t.g + 5 * N, o, d1l(t, B[5] + g.lc, G::LX));
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint, z-march:
//   rhs_p = L w1 - HzT w1,  rhs_q = HzT w2
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_amarch(TtiArgs<T> t, int ntx, int nty,
                                                             int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  // [buffer][w1, n_x^2 w1, n_y^2 w1, n_x^2 w2, n_y^2 w2, E_xy(w1), E_xy(w2)]
  __shared__ T L[2][7][G::PL];
  const int64_t N = a.N;
  const T *nzf = t.coef + 2 * N, *nyf = t.coef + 3 * N, *nxf = t.coef + 4 * N;
  const T *W1 = t.g, *W2 = t.g + N, *Exz1 = t.g + 2 * N, *Exz2 = t.g + 3 * N,
          *Exy1 = t.g + 4 * N, *Exy2 = t.g + 5 * N;
  // z queues of the own column: w1, n_z^2 w1, n_z^2 w2, E_xz(w1), E_xz(w2)
  T Qw[9], Qz1[9], Qz2[9], Qe1[9], Qe2[9];
  T f[5];
  auto front = [&](int zz, T *o5) {
    const T w1 = ldz(W1, a, g.in, zz, g.y, g.x);
    const T w2 = ldz(W2, a, g.in, zz, g.y, g.x);
    const T n = ldz(nzf, a, g.in, zz, g.y, g.x);
    o5[0] = w1;
    o5[1] = (n * n) * w1;
    o5[2] = (n * n) * w2;
    o5[3] = ldz(Exz1, a, g.in, zz, g.y, g.x);
    o5[4] = ldz(Exz2, a, g.in, zz, g.y, g.x);
  };
  for (int k = 0; k < 8; ++k) {
    T v[5];
    front(z0 - 4 + k, v);
    Qw[k] = v[0];
    Qz1[k] = v[1];
    Qz2[k] = v[2];
    Qe1[k] = v[3];
    Qe2[k] = v[4];
  }
  // plane values of the own cell and the halo cells
  T lp, lq, lpp, lqp, mm, w2c, nxc, nyc, e1c, e2c;
  T hy_w1[G::NHY], hy_w2[G::NHY], hy_ny[G::NHY];  // y-halo
  T hx_w1, hx_w2, hx_nx, hx_e1, hx_e2;        // x-halo
  auto fetch = [&](int z) {
    front(z + 4, f);
    lp = ldz(t.p, a, g.in, z, g.y, g.x);
    lq = ldz(t.q, a, g.in, z, g.y, g.x);
    lpp = ldz(t.pp, a, g.in, z, g.y, g.x);
    lqp = ldz(t.qp, a, g.in, z, g.y, g.x);
    mm = ldz(a.m, a, g.in, z, g.y, g.x);
    w2c = ldz(W2, a, g.in, z, g.y, g.x);
    nxc = ldz(nxf, a, g.in, z, g.y, g.x);
    nyc = ldz(nyf, a, g.in, z, g.y, g.x);
    e1c = ldz(Exy1, a, g.in, z, g.y, g.x);
    e2c = ldz(Exy2, a, g.in, z, g.y, g.x);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      hy_w1[k] = ldz(W1, a, g.hyon[k], z, g.hyg[k], g.x);
      hy_w2[k] = ldz(W2, a, g.hyon[k], z, g.hyg[k], g.x);
      hy_ny[k] = ldz(nyf, a, g.hyon[k], z, g.hyg[k], g.x);
    }
    hx_w1 = ldz(W1, a, g.hxon, z, g.hxg_y, g.hxg_x);
    hx_w2 = ldz(W2, a, g.hxon, z, g.hxg_y, g.hxg_x);
    hx_nx = ldz(nxf, a, g.hxon, z, g.hxg_y, g.hxg_x);
    hx_e1 = ldz(Exy1, a, g.hxon, z, g.hxg_y, g.hxg_x);
    hx_e2 = ldz(Exy2, a, g.hxon, z, g.hxg_y, g.hxg_x);
  };
  fetch(z0);
  for (int z = z0; z < z1; ++z) {
    Qw[8] = f[0];
    Qz1[8] = f[1];
    Qz2[8] = f[2];
    Qe1[8] = f[3];
    Qe2[8] = f[4];
    const T clp = lp, clq = lq, clpp = lpp, clqp = lqp, cm = mm;
    T(*B)[G::PL] = L[z & 1];
    {
      const T w1 = Qw[4];
      B[0][g.lc] = w1;
      B[1][g.lc] = (nxc * nxc) * w1;
      B[2][g.lc] = (nyc * nyc) * w1;
      B[3][g.lc] = (nxc * nxc) * w2c;
      B[4][g.lc] = (nyc * nyc) * w2c;
      B[5][g.lc] = e1c;
      B[6][g.lc] = e2c;
    }
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      B[0][g.hyl[k]] = hy_w1[k];
      B[2][g.hyl[k]] = (hy_ny[k] * hy_ny[k]) * hy_w1[k];
      B[4][g.hyl[k]] = (hy_ny[k] * hy_ny[k]) * hy_w2[k];
    }
    if (threadIdx.x < G::NHX) {
      B[0][g.hxl] = hx_w1;
      B[1][g.hxl] = (hx_nx * hx_nx) * hx_w1;
      B[3][g.hxl] = (hx_nx * hx_nx) * hx_w2;
      B[5][g.hxl] = hx_e1;
      B[6][g.hxl] = hx_e2;
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    if (g.in) {
      const T lw1 = (d2q(t, Qw) + d2l(t, B[0] + g.lc, G::LX)) + d2l(t, B[0] + g.lc, 1);
      const T hz1 = ((d2q(t, Qz1) + d2l(t, B[2] + g.lc, G::LX)) + d2l(t, B[1] + g.lc, 1)) +
                    T(2) * (d1l(t, B[5] + g.lc, 1) + d1q(t, Qe1));
      const T hz2 = ((d2q(t, Qz2) + d2l(t, B[4] + g.lc, G::LX)) + d2l(t, B[3] + g.lc, 1)) +
                    T(2) * (d1l(t, B[6] + g.lc, 1) + d1q(t, Qe2));
      const T damp = sponge_a(a, z, g.y, g.x);
      const uint32_t o = cidx(a, z, g.y, g.x);
      sto(t.pn, o, tti_update(a, clp, clpp, cm, lw1 - hz1, damp));
      sto(t.qn, o, tti_update(a, clq, clqp, cm, hz2, damp));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      Qw[k] = Qw[k + 1];
      Qz1[k] = Qz1[k + 1];
      Qz2[k] = Qz2[k + 1];
      Qe1[k] = Qe1[k + 1];
      Qe2[k] = Qe2[k + 1];
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint, fused: one kernel per step.  The lead plane z + 4 carries n_x n_z w
// and n_y n_z w (x / y halo) for the E_xz queue fronts, and the z-queue fronts
// w1, n_z^2 w1, n_z^2 w2; the current plane z carries w1, n_x^2 w, n_y^2 w and
// n_x n_y w (with corners, for the second LDS stage D_x (D_y .)).  The own
// cell's w2, n_x, n_y, lp, lq reach plane z through 5-deep delay queues.
// Current-plane LDS is double buffered (two barriers per plane) where it fits
// in LDS; FP64 on 64 x 8 tiles keeps one buffer and a third barrier.
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_afused(TtiArgs<T> t, int ntx, int nty,
                                                             int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  // current plane: w1, n_x^2 w1, n_y^2 w1, n_x^2 w2, n_y^2 w2, n_x n_y w1, n_x n_y w2
  // (NB buffers: plane z writes buffer z & 1 while others may still read z - 1's)
  constexpr int NB = (sizeof(T) == 8 && TY == 8) ? 1 : 2;
  __shared__ T LcB[NB][7][G::PL];
  __shared__ T Ll[4][G::PL];      // lead plane: n_x n_z w1, n_x n_z w2, n_y n_z w1, n_y n_z w2
  __shared__ T H[2][TY * G::LX];  // D_y (n_x n_y w1), D_y (n_x n_y w2)
  const int64_t N = a.N;
  const T *c1f = t.coef, *c2f = t.coef + N, *nzf = t.coef + 2 * N, *nyf = t.coef + 3 * N,
          *nxf = t.coef + 4 * N;
  struct In {
    T lp, lq, c1, c2, nz, ny, nx;
  };
  auto load = [&](bool on, int z, int y, int x, bool withz) {
    In c;
    c.lp = ldz(t.p, a, on, z, y, x);
    c.lq = ldz(t.q, a, on, z, y, x);
    c.c1 = ldz(c1f, a, on, z, y, x);
    c.c2 = ldz(c2f, a, on, z, y, x);
    c.nz = withz ? ldz(nzf, a, on, z, y, x) : T(0);
    c.ny = ldz(nyf, a, on, z, y, x);
    c.nx = ldz(nxf, a, on, z, y, x);
    return c;
  };
  T W[9], Z1[9], Z2[9], E1[9], E2[9];               // z queues
  T Dw2[5], Dnx[5], Dny[5], Dlp[5], Dlq[5];         // delays: [4] lead plane, [0] plane z
#pragma unroll
  for (int k = 0; k < 9; ++k) W[k] = Z1[k] = Z2[k] = E1[k] = E2[k] = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) Dw2[k] = Dnx[k] = Dny[k] = Dlp[k] = Dlq[k] = T(0);
  In li, ly[G::NHY], lx, cy[G::NHY], cx, cn;
  T lpp, lqp, mm;
  auto fetch = [&](int z) {
    const int zl = z + 4;
    li = load(g.in, zl, g.y, g.x, true);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) ly[k] = load(g.hyon[k], zl, g.hyg[k], g.x, true);
    lx = load(g.hxon, zl, g.hxg_y, g.hxg_x, true);
    const bool out = z >= z0;
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) cy[k] = load(out && g.hyon[k], z, g.hyg[k], g.x, false);
    cx = load(out && g.hxon, z, g.hxg_y, g.hxg_x, false);
    cn = load(out && g.cnon, z, g.cng_y, g.cng_x, false);
    const bool oc = out && g.in;
    lpp = ldz(t.pp, a, oc, z, g.y, g.x);
    lqp = ldz(t.qp, a, oc, z, g.y, g.x);
    mm = ldz(a.m, a, oc, z, g.y, g.x);
  };
  auto w1of = [](const In &c) { return c.c1 * c.lp + c.c2 * c.lq; };
  auto w2of = [](const In &c) { return c.c2 * c.lp + c.lq; };
  // current-plane LDS values of one cell (halo cells: LDS offset l)
  auto stage_cur = [&](T (*Lc)[G::PL], int l, T w1, T w2, T nx, T ny) {
    Lc[0][l] = w1;
    Lc[1][l] = (nx * nx) * w1;
    Lc[2][l] = (ny * ny) * w1;
    Lc[3][l] = (nx * nx) * w2;
    Lc[4][l] = (ny * ny) * w2;
    Lc[5][l] = (nx * ny) * w1;
    Lc[6][l] = (nx * ny) * w2;
  };
  const int zs = z0 - 8;
  fetch(zs);
  for (int z = zs; z < z1; ++z) {
    const bool out = z >= z0;  // uniform over the workgroup
    T(*Lc)[G::PL] = LcB[NB == 2 ? (z & 1) : 0];
    // lead plane: queue fronts and LDS
    {
      const T w1 = w1of(li), w2 = w2of(li);
      W[8] = w1;
      Z1[8] = (li.nz * li.nz) * w1;
      Z2[8] = (li.nz * li.nz) * w2;
      Dw2[4] = w2;
      Dnx[4] = li.nx;
      Dny[4] = li.ny;
      Dlp[4] = li.lp;
      Dlq[4] = li.lq;
      Ll[0][g.lc] = (li.nx * li.nz) * w1;
      Ll[1][g.lc] = (li.nx * li.nz) * w2;
      Ll[2][g.lc] = (li.ny * li.nz) * w1;
      Ll[3][g.lc] = (li.ny * li.nz) * w2;
    }
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      const T v1 = w1of(ly[k]), v2 = w2of(ly[k]);
      Ll[2][g.hyl[k]] = (ly[k].ny * ly[k].nz) * v1;
      Ll[3][g.hyl[k]] = (ly[k].ny * ly[k].nz) * v2;
    }
    if (threadIdx.x < G::NHX) {
      const T v1 = w1of(lx), v2 = w2of(lx);
      Ll[0][g.hxl] = (lx.nx * lx.nz) * v1;
      Ll[1][g.hxl] = (lx.nx * lx.nz) * v2;
    }
    // current plane
    const T clpp = lpp, clqp = lqp, cm = mm;
    if (out) {
      stage_cur(Lc, g.lc, W[4], Dw2[0], Dnx[0], Dny[0]);
#pragma unroll
      for (int k = 0; k < G::NHY; ++k)
        stage_cur(Lc, g.hyl[k], w1of(cy[k]), w2of(cy[k]), cy[k].nx, cy[k].ny);
      if (threadIdx.x < G::NHX) stage_cur(Lc, g.hxl, w1of(cx), w2of(cx), cx.nx, cx.ny);
      if (threadIdx.x >= G::NHX && threadIdx.x < G::NHX + 64)
        stage_cur(Lc, g.cnl, w1of(cn), w2of(cn), cn.nx, cn.ny);
    }
    if (z + 1 < z1) fetch(z + 1);
    __syncthreads();
    E1[8] = d1l(t, Ll[0] + g.lc, 1) + d1l(t, Ll[2] + g.lc, G::LX);
    E2[8] = d1l(t, Ll[1] + g.lc, 1) + d1l(t, Ll[3] + g.lc, G::LX);
    if (out) {
      const int hr = threadIdx.x / TX, hc = threadIdx.x % TX + 4;
      H[0][hr * G::LX + hc] = d1l(t, Lc[5] + g.lc, G::LX);
      H[1][hr * G::LX + hc] = d1l(t, Lc[6] + g.lc, G::LX);
      if (threadIdx.x < G::NHX) {
        const int r = threadIdx.x / 8, lcx = g.hxl - (4 + r) * G::LX;
        H[0][r * G::LX + lcx] = d1l(t, Lc[5] + g.hxl, G::LX);
        H[1][r * G::LX + lcx] = d1l(t, Lc[6] + g.hxl, G::LX);
      }
    }
    __syncthreads();
    if (out && g.in) {
      const int hrow = (threadIdx.x / TX) * G::LX + threadIdx.x % TX + 4;
      const T lw1 = (d2q(t, W) + d2l(t, Lc[0] + g.lc, G::LX)) + d2l(t, Lc[0] + g.lc, 1);
      const T hz1 = ((d2q(t, Z1) + d2l(t, Lc[2] + g.lc, G::LX)) + d2l(t, Lc[1] + g.lc, 1)) +
                    T(2) * (d1l(t, H[0] + hrow, 1) + d1q(t, E1));
      const T hz2 = ((d2q(t, Z2) + d2l(t, Lc[4] + g.lc, G::LX)) + d2l(t, Lc[3] + g.lc, 1)) +
                    T(2) * (d1l(t, H[1] + hrow, 1) + d1q(t, E2));
      const T damp = sponge_a(a, z, g.y, g.x);
      const uint32_t o = cidx(a, z, g.y, g.x);
      sto(t.pn, o, tti_update(a, Dlp[0], clpp, cm, lw1 - hz1, damp));
      sto(t.qn, o, tti_update(a, Dlq[0], clqp, cm, hz2, damp));
    }
    // one current-plane buffer: it is rewritten next iteration.  Two: the
    // next iteration writes the other one; the lead plane and H are rewritten
    // only after the next iteration's first / this iteration's second barrier
    if constexpr (NB == 1) __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      W[k] = W[k + 1];
      Z1[k] = Z1[k + 1];
      Z2[k] = Z2[k + 1];
      E1[k] = E1[k + 1];
      E2[k] = E2[k + 1];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Dw2[k] = Dw2[k + 1];
      Dnx[k] = Dnx[k + 1];
      Dny[k] = Dny[k + 1];
      Dlp[k] = Dlp[k + 1];
      Dlq[k] = Dlq[k + 1];
    }
  }
}

// adjoint, fused, with delay queues for the halo: as k_tti_afused, but the
// halo and corner cells of the current plane are not loaded again: their w1,
// w2, n_x and n_y are taken at the lead stage (corners are loaded there too)
// and kept in 5-deep register queues until their plane is the current one.
// HLQ (FP32 only): those queues live in a per-thread ring of five LDS planes
// instead of registers; each thread reads back only what it wrote itself, so
// the ring needs no barrier, and the 60 registers it frees let the loop
// carry U planes per trip.
// OBQ (with HLQ, FP32 only): one workgroup barrier per plane instead of two.
// Each wave (one tile row) also forms D_y (n_x n_y w) at its own row's eight
// x-halo columns, so the D_x of that product reads only what the wave itself
// wrote (a wave-level fence, no barrier), and the lead plane's LDS fields are
// double buffered: a wave may write plane z + 1's while another still reads
// plane z's.
// MG: the p equation's right side, Lap w1 - Hz w1, is taken as one sum over
// the axes of D_aa ((1 - n_a^2) w1) (the second differences are linear), so
// each axis needs one second difference of w1 instead of two, and w1 itself
// leaves the LDS plane (six fields) and the z queues (its own cell's w1 waits
// in a five-deep delay instead).  The arithmetic differs from the other forms
// in rounding only.
// ---------------------------------------------------------------------------
template <typename T, int TY, int MINW, int U, bool HLQ, bool OBQ = false, bool MG = false>
__global__ __launch_bounds__(TX *TY, MINW) void k_tti_afused_dq(TtiArgs<T> t, int ntx, int nty,
                                                             int nzc, int zchunk) {
  using G = Geo<TY>;
  const StepArgs<T> &a = t.a;
  int bx, by, z0, z1;
  block_of(ntx, nty, nzc, zchunk, a.nz, bx, by, z0, z1);
  const TtiTile<TY> g = tile_of<TY>(a, bx, by);
  // current plane: w1, n_x^2 w1, n_y^2 w1, n_x^2 w2, n_y^2 w2, n_x n_y w1, n_x n_y w2
  // (NB buffers: plane z writes buffer z & 1 while others may still read z - 1's)
  constexpr int NB = (sizeof(T) == 8 && TY == 8) ? 1 : 2;
  // MG: (1 - n_x^2) w1, (1 - n_y^2) w1, n_x^2 w2, n_y^2 w2, n_x n_y w1, n_x n_y w2
  constexpr int NF = MG ? 6 : 7, FX1 = MG ? 4 : 5, FX2 = MG ? 5 : 6;
  __shared__ T LcB[NB][NF][G::PL];
  constexpr bool HL = HLQ && sizeof(T) == 4;
  constexpr bool OB = OBQ && HL && NB == 2;
  // lead plane: n_x n_z w1, n_x n_z w2, n_y n_z w1, n_y n_z w2
  __shared__ T LlB[OB ? 2 : 1][4][G::PL];
  __shared__ T H[2][TY * G::LX];  // D_y (n_x n_y w1), D_y (n_x n_y w2)
  typedef T V4 __attribute__((ext_vector_type(4)));  // (w1, w2, n_x, n_y) of a halo cell
  constexpr int NHQ = G::NHY * G::NTHR + 128;        // y halo, then x halo or corner
  __shared__ V4 Hq[HL ? 5 : 1][HL ? NHQ : 1];
  auto hslot = [](int plane) { return (plane + 10) % 5; };  // plane >= z0 - 8 >= -8
  const int hxi = G::NHY * G::NTHR + threadIdx.x;  // x-halo (tid < NHX) or corner slot
  const bool corner = threadIdx.x >= G::NHX && threadIdx.x < G::NHX + 64;
  const int64_t N = a.N;
  const T *c1f = t.coef, *c2f = t.coef + N, *nzf = t.coef + 2 * N, *nyf = t.coef + 3 * N,
          *nxf = t.coef + 4 * N;
  struct In {
    T lp, lq, c1, c2, nz, ny, nx;
  };
  auto load = [&](bool on, int z, int y, int x, bool withz) {
    In c;
    c.lp = ldz(t.p, a, on, z, y, x);
    c.lq = ldz(t.q, a, on, z, y, x);
    c.c1 = ldz(c1f, a, on, z, y, x);
    c.c2 = ldz(c2f, a, on, z, y, x);
    c.nz = withz ? ldz(nzf, a, on, z, y, x) : T(0);
    c.ny = ldz(nyf, a, on, z, y, x);
    c.nx = ldz(nxf, a, on, z, y, x);
    return c;
  };
  T W[9], Z1[9], Z2[9], E1[9], E2[9];               // z queues (MG: W = (1 - n_z^2) w1)
  T Dw1[5], Dw2[5], Dnx[5], Dny[5], Dlp[5], Dlq[5];  // delays: [4] lead plane, [0] plane z
  // the halo and corner cells' w1, w2, n_x, n_y, kept from the lead stage
  // until their plane is the current one (no second load of those cells)
  T Hy[G::NHY][4][5], Hx[4][5], Hc[4][5];
#pragma unroll
  for (int k = 0; k < 9; ++k) W[k] = Z1[k] = Z2[k] = E1[k] = E2[k] = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    Dw1[k] = Dw2[k] = Dnx[k] = Dny[k] = Dlp[k] = Dlq[k] = T(0);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int h = 0; h < G::NHY; ++h) Hy[h][f][k] = T(0);
      Hx[f][k] = Hc[f][k] = T(0);
    }
  }
  In li, ly[G::NHY], lx = {}, lc = {};
  T lpp, lqp, mm;
  // the x-halo cells belong to the first NHX threads and the corners to the
  // next 64: whole waves for 64 x 8 tiles, so the other waves skip their loads
  constexpr bool WXH = G::NHX % 64 == 0;
  const bool hasx = threadIdx.x < G::NHX, hasc = corner;
  auto fetch = [&](int z) {
    const int zl = z + 4;
    li = load(g.in, zl, g.y, g.x, true);
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) ly[k] = load(g.hyon[k], zl, g.hyg[k], g.x, true);
    if (!WXH || hasx) lx = load(g.hxon, zl, g.hxg_y, g.hxg_x, true);
    if (!WXH || hasc) lc = load(g.cnon, zl, g.cng_y, g.cng_x, false);
    const bool out = z >= z0;
    const bool oc = out && g.in;
    lpp = ldz(t.pp, a, oc, z, g.y, g.x);
    lqp = ldz(t.qp, a, oc, z, g.y, g.x);
    mm = ldz(a.m, a, oc, z, g.y, g.x);
  };
  auto w1of = [](const In &c) { return c.c1 * c.lp + c.c2 * c.lq; };
  auto w2of = [](const In &c) { return c.c2 * c.lp + c.lq; };
  // current-plane LDS values of one cell (halo cells: LDS offset l)
  auto stage_cur = [&](T (*Lc)[G::PL], int l, T w1, T w2, T nx, T ny) {
    if constexpr (MG) {
      Lc[0][l] = (T(1) - nx * nx) * w1;
      Lc[1][l] = (T(1) - ny * ny) * w1;
      Lc[2][l] = (nx * nx) * w2;
      Lc[3][l] = (ny * ny) * w2;
      Lc[4][l] = (nx * ny) * w1;
      Lc[5][l] = (nx * ny) * w2;
      return;
    }
    Lc[0][l] = w1;
    Lc[1][l] = (nx * nx) * w1;
    Lc[2][l] = (ny * ny) * w1;
    Lc[3][l] = (nx * nx) * w2;
    Lc[4][l] = (ny * ny) * w2;
    Lc[5][l] = (nx * ny) * w1;
    Lc[6][l] = (nx * ny) * w2;
  };
  const int zs = z0 - 8;
  fetch(zs);
  // U planes per trip: the queue shifts of the unrolled planes become
  // register renames (only the shifts across a trip remain moves)
  auto step = [&](int z) {
    const bool out = z >= z0;  // uniform over the workgroup
    T(*Lc)[G::PL] = LcB[NB == 2 ? (z & 1) : 0];
    T(*Ll)[G::PL] = LlB[OB ? (z & 1) : 0];
    // lead plane: queue fronts and LDS
    {
      const T w1 = w1of(li), w2 = w2of(li);
      if constexpr (MG) {
        W[8] = (T(1) - li.nz * li.nz) * w1;
        Dw1[4] = w1;
      } else {
        W[8] = w1;
        Z1[8] = (li.nz * li.nz) * w1;
      }
      Z2[8] = (li.nz * li.nz) * w2;
      Dw2[4] = w2;
      Dnx[4] = li.nx;
      Dny[4] = li.ny;
      Dlp[4] = li.lp;
      Dlq[4] = li.lq;
      Ll[0][g.lc] = (li.nx * li.nz) * w1;
      Ll[1][g.lc] = (li.nx * li.nz) * w2;
      Ll[2][g.lc] = (li.ny * li.nz) * w1;
      Ll[3][g.lc] = (li.ny * li.nz) * w2;
    }
#pragma unroll
    for (int k = 0; k < G::NHY; ++k) {
      const T v1 = w1of(ly[k]), v2 = w2of(ly[k]);
      Ll[2][g.hyl[k]] = (ly[k].ny * ly[k].nz) * v1;
      Ll[3][g.hyl[k]] = (ly[k].ny * ly[k].nz) * v2;
      if constexpr (HL) {
        Hq[hslot(z + 4)][k * G::NTHR + threadIdx.x] = V4{v1, v2, ly[k].nx, ly[k].ny};
      } else {
        Hy[k][0][4] = v1;
        Hy[k][1][4] = v2;
        Hy[k][2][4] = ly[k].nx;
        Hy[k][3][4] = ly[k].ny;
      }
    }
    {
      const T v1 = w1of(lx), v2 = w2of(lx);
      if (threadIdx.x < G::NHX) {
        Ll[0][g.hxl] = (lx.nx * lx.nz) * v1;
        Ll[1][g.hxl] = (lx.nx * lx.nz) * v2;
      }
      if constexpr (HL) {
        if (threadIdx.x < G::NHX) Hq[hslot(z + 4)][hxi] = V4{v1, v2, lx.nx, lx.ny};
        if (corner) Hq[hslot(z + 4)][hxi] = V4{w1of(lc), w2of(lc), lc.nx, lc.ny};
      } else {
        Hx[0][4] = v1;
        Hx[1][4] = v2;
        Hx[2][4] = lx.nx;
        Hx[3][4] = lx.ny;
        Hc[0][4] = w1of(lc);
        Hc[1][4] = w2of(lc);
        Hc[2][4] = lc.nx;
        Hc[3][4] = lc.ny;
      }
    }
    // current plane
    const T clpp = lpp, clqp = lqp, cm = mm;
    // MG: the next plane's loads go out before the current plane is staged
    if constexpr (MG) {
      if (z + 1 < z1) fetch(z + 1);
    }
    if (out) {
      stage_cur(Lc, g.lc, MG ? Dw1[0] : W[4], Dw2[0], Dnx[0], Dny[0]);
      if constexpr (HL) {
#pragma unroll
        for (int k = 0; k < G::NHY; ++k) {
          const V4 h = Hq[hslot(z)][k * G::NTHR + threadIdx.x];
          stage_cur(Lc, g.hyl[k], h.x, h.y, h.z, h.w);
        }
        if (threadIdx.x < G::NHX || corner) {
          const V4 h = Hq[hslot(z)][hxi];
          stage_cur(Lc, threadIdx.x < G::NHX ? g.hxl : g.cnl, h.x, h.y, h.z, h.w);
        }
      } else {
#pragma unroll
        for (int k = 0; k < G::NHY; ++k)
          stage_cur(Lc, g.hyl[k], Hy[k][0][0], Hy[k][1][0], Hy[k][2][0], Hy[k][3][0]);
        if (threadIdx.x < G::NHX) stage_cur(Lc, g.hxl, Hx[0][0], Hx[1][0], Hx[2][0], Hx[3][0]);
        if (corner) stage_cur(Lc, g.cnl, Hc[0][0], Hc[1][0], Hc[2][0], Hc[3][0]);
      }
    }
    if constexpr (!MG) {
      if (z + 1 < z1) fetch(z + 1);
    }
    __syncthreads();
    E1[8] = d1l(t, Ll[0] + g.lc, 1) + d1l(t, Ll[2] + g.lc, G::LX);
    E2[8] = d1l(t, Ll[1] + g.lc, 1) + d1l(t, Ll[3] + g.lc, G::LX);
    if (out) {
      const int hr = threadIdx.x / TX, hc = threadIdx.x % TX + 4;
      H[0][hr * G::LX + hc] = d1l(t, Lc[FX1] + g.lc, G::LX);
      H[1][hr * G::LX + hc] = d1l(t, Lc[FX2] + g.lc, G::LX);
      if constexpr (OB) {
        // lanes 0..7: this row's x-halo columns 0..3 and TX + 4 .. TX + 7
        const int lane = threadIdx.x % TX;
        if (lane < 8) {
          const int lcx = lane < 4 ? lane : TX + lane;
          const int lo = (4 + hr) * G::LX + lcx;
          H[0][hr * G::LX + lcx] = d1l(t, Lc[FX1] + lo, G::LX);
          H[1][hr * G::LX + lcx] = d1l(t, Lc[FX2] + lo, G::LX);
        }
      } else if (threadIdx.x < G::NHX) {
        const int r = threadIdx.x / 8, lcx = g.hxl - (4 + r) * G::LX;
        H[0][r * G::LX + lcx] = d1l(t, Lc[FX1] + g.hxl, G::LX);
        H[1][r * G::LX + lcx] = d1l(t, Lc[FX2] + g.hxl, G::LX);
      }
    }
    if constexpr (OB) {
      // the row of H is written and read by this wave alone
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
    if (out && g.in) {
      const int hrow = (threadIdx.x / TX) * G::LX + threadIdx.x % TX + 4;
      T rp, hz2;
      if constexpr (MG) {
        rp = ((d2q(t, W) + d2l(t, Lc[1] + g.lc, G::LX)) + d2l(t, Lc[0] + g.lc, 1)) -
             T(2) * (d1l(t, H[0] + hrow, 1) + d1q(t, E1));
        hz2 = ((d2q(t, Z2) + d2l(t, Lc[3] + g.lc, G::LX)) + d2l(t, Lc[2] + g.lc, 1)) +
              T(2) * (d1l(t, H[1] + hrow, 1) + d1q(t, E2));
      } else {
        const T lw1 = (d2q(t, W) + d2l(t, Lc[0] + g.lc, G::LX)) + d2l(t, Lc[0] + g.lc, 1);
        const T hz1 = ((d2q(t, Z1) + d2l(t, Lc[2] + g.lc, G::LX)) + d2l(t, Lc[1] + g.lc, 1)) +
                      T(2) * (d1l(t, H[0] + hrow, 1) + d1q(t, E1));
        hz2 = ((d2q(t, Z2) + d2l(t, Lc[4] + g.lc, G::LX)) + d2l(t, Lc[3] + g.lc, 1)) +
              T(2) * (d1l(t, H[1] + hrow, 1) + d1q(t, E2));
        rp = lw1 - hz1;
      }
      const T damp = sponge_a(a, z, g.y, g.x);
      const uint32_t o = cidx(a, z, g.y, g.x);
      T pn, qn;
      tti_update_pq(a, cm, damp, Dlp[0], clpp, rp, Dlq[0], clqp, hz2, pn, qn);
      sto(t.pn, o, pn);
      sto(t.qn, o, qn);
    }
    // one current-plane buffer: it is rewritten next iteration.  Two: the
    // next iteration writes the other one; the lead plane and H are rewritten
    // only after the next iteration's first / this iteration's second barrier
    if constexpr (NB == 1) __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      W[k] = W[k + 1];
      Z1[k] = Z1[k + 1];
      Z2[k] = Z2[k + 1];
      E1[k] = E1[k + 1];
      E2[k] = E2[k + 1];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Dw1[k] = Dw1[k + 1];
      Dw2[k] = Dw2[k + 1];
      Dnx[k] = Dnx[k + 1];
      Dny[k] = Dny[k + 1];
      Dlp[k] = Dlp[k + 1];
      Dlq[k] = Dlq[k + 1];
      if constexpr (!HL) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
#pragma unroll
          for (int h = 0; h < G::NHY; ++h) Hy[h][f][k] = Hy[h][f][k + 1];
          Hx[f][k] = Hx[f][k + 1];
          Hc[f][k] = Hc[f][k + 1];
        }
      }
    }
  };
  int z = zs;
  if constexpr (U > 1) {
    for (; z + U <= z1; z += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) step(z + u);
    }
  }
  for (; z < z1; ++z) step(z);
}

// grid of one tiled launch: (64 x ty) column tiles, z split into the fewest
// chunks (of at least 16 planes) that give target_blocks workgroups
struct TtiGrid {
  int ntx, nty, nzc, zchunk;
};
static TtiGrid tti_grid(int nz, int ny, int nx, int ty, int target_blocks) {
  TtiGrid g;
  g.ntx = (nx + TX - 1) / TX;
  g.nty = (ny + ty - 1) / ty;
  const int tiles = g.ntx * g.nty;
  int nzc = (target_blocks + tiles - 1) / tiles;
  const int most = nz / 16 > 1 ? nz / 16 : 1;
  if (nzc > most) nzc = most;
  if (nzc < 1) nzc = 1;
  g.zchunk = (nz + nzc - 1) / nzc;
  g.nzc = (nz + g.zchunk - 1) / g.zchunk;
  return g;
}

// one TTI step with the tiled kernels (prep with TYP rows, march with TYM
// rows); g needs 4 (forward) / 6 (adjoint) slots of N
// FUSED: 1 = fused forward kernel, 2 = fused forward kernel with the LDS plane ring;
// AFUSED: 1 = fused transpose kernel, 2 = fused transpose kernel with halo delay
// queues in registers, 3 = in LDS; UA / UF: planes per loop trip of the
// delay-queue / ring kernel (UF > 1 caps the FP32 ring kernel at 168 VGPRs,
// three waves per SIMD; at 300 x 400 x 400: one plane per trip 666-672 us;
// two planes 635 us, 1 spilled register; uncapped they need 176 VGPRs and run
// at two waves per SIMD, 802 us); LC: the ring kernel loads each current
// cell's eight values at the start of its own iteration instead of one
// iteration ahead (one set live instead of two): two planes 625 us without
// spills, three planes 610 us with 3 spilled registers (17 without LC, 747
// us), four planes spill 21
template <typename T, int TYP, int TYM, int FUSED = 0, int AFUSED = 0, int UA = 1, int UF = 1,
          bool LC = false>
static hipError_t tti_step_tiled(const TtiArgs<T> &t, bool adjoint, int target_blocks,
                                 hipStream_t st) {
  const StepArgs<T> &a = t.a;
  const TtiGrid gp = tti_grid(a.nz, a.ny, a.nx, TYP, target_blocks);
  const TtiGrid gm = tti_grid(a.nz, a.ny, a.nx, TYM, target_blocks);
  const dim3 bp(TX * TYP), bm(TX * TYM);
  const dim3 np(gp.ntx * gp.nty * gp.nzc), nm(gm.ntx * gm.nty * gm.nzc);
  if constexpr (FUSED == 1) {
    if (!adjoint) {
      hipLaunchKernelGGL((k_tti_ffused<T, TYM, 1>), nm, bm, 0, st, t, gm.ntx, gm.nty, gm.nzc,
                         gm.zchunk);
      return hipGetLastError();
    }
  }
  if constexpr (FUSED == 2) {
    if (!adjoint) {
      constexpr int MINW = (UF > 1 && sizeof(T) == 4) ? 3 : 1;
      hipLaunchKernelGGL((k_tti_ffused_ring<T, TYM, MINW, UF, LC>), nm, bm, 0, st, t, gm.ntx, gm.nty,
                         gm.nzc, gm.zchunk);
      return hipGetLastError();
    }
  }
  if constexpr (AFUSED == 1) {
    if (adjoint) {
      hipLaunchKernelGGL((k_tti_afused<T, TYM, 1>), nm, bm, 0, st, t, gm.ntx, gm.nty, gm.nzc,
                         gm.zchunk);
      return hipGetLastError();
    }
  }
  if constexpr (AFUSED >= 2) {
    if (adjoint) {
      hipLaunchKernelGGL((k_tti_afused_dq<T, TYM, 1, UA, AFUSED >= 3, AFUSED >= 4, AFUSED == 5>),
                         nm, bm, 0, st, t, gm.ntx, gm.nty, gm.nzc, gm.zchunk);
      return hipGetLastError();
    }
  }
  if (!adjoint) {
    hipLaunchKernelGGL((k_tti_fprep<T, TYP, 1>), np, bp, 0, st, t, gp.ntx, gp.nty, gp.nzc,
                       gp.zchunk);
    hipLaunchKernelGGL((k_tti_fmarch<T, TYM, 1>), nm, bm, 0, st, t, gm.ntx, gm.nty, gm.nzc,
                       gm.zchunk);
  } else {
    hipLaunchKernelGGL((k_tti_aprep<T, TYP, 1>), np, bp, 0, st, t, gp.ntx, gp.nty, gp.nzc,
                       gp.zchunk);
    hipLaunchKernelGGL((k_tti_amarch<T, TYM, 1>), nm, bm, 0, st, t, gm.ntx, gm.nty, gm.nzc,
                       gm.zchunk);
  }
  return hipGetLastError();
}

// tile shapes (prep / march rows of 64 columns): 1 = 8 / 8, 2 = 4 / 4,
// 3 = 8 / 4, 4 = as 3 with the fused forward kernel (4 rows), 5 = as 3 with
// the fused forward kernel (8 rows), 6 = both steps fused (4 rows), 7 = both
// fused, forward 4 rows and transpose 8 rows,
// 8 = both fused (8 rows), 9 / 10 = as 7 with the
// forward kernel's LDS plane ring (forward on 4 / 8 rows), 11 / 12 = as 9 with
// the transpose kernel's halo delay queues (transpose on 8 / 4 rows), 13 / 14 /
// 15 = as 11 with the transpose kernel's halo queues in LDS and 1 / 2 / 3
// planes per loop trip, 16 = as 15 with the forward ring kernel carrying two
// planes per loop trip, 17 = as 16 with three planes per trip and each
// current cell's values loaded at the start of its own iteration (the forward
// step of every later shape), 18 = as 17 with one workgroup barrier per plane
// in the transpose, 19 / 20 / 21 (the library's default) = as 18 with the transpose's p equation
// taken as one second difference per axis of (1 - n_a^2) w1 and 3 / 4 / 6
// planes per loop trip in the transpose.  Transpose step at 300 x 400 x 400
// (FP32): 17: 1111 us, 18: 1095 us, 19: 1047 us, 20: 1032 us, 21: 1022 us
// (two and five planes per trip: 1047 and 1039 us); with the waves that hold
// no x-halo or corner cell skipping those loads, 19: 992 us, 21: 967-972 us
template <typename T>
hipError_t launch_tti_step_tiled(const TtiArgs<T> &t, bool adjoint, int shape, int target_blocks,
                                 hipStream_t st) {
  switch (shape) {
    case 1: return tti_step_tiled<T, 8, 8>(t, adjoint, target_blocks, st);
    case 2: return tti_step_tiled<T, 4, 4>(t, adjoint, target_blocks, st);
    case 5: return adjoint ? tti_step_tiled<T, 8, 4>(t, adjoint, target_blocks, st)
                           : tti_step_tiled<T, 8, 8, 1>(t, adjoint, target_blocks, st);
    case 3: return tti_step_tiled<T, 8, 4>(t, adjoint, target_blocks, st);
    case 4: return tti_step_tiled<T, 8, 4, 1>(t, adjoint, target_blocks, st);
    case 7: return adjoint ? tti_step_tiled<T, 8, 8, 1, 1>(t, adjoint, target_blocks, st)
                           : tti_step_tiled<T, 8, 4, 1, 1>(t, adjoint, target_blocks, st);
    case 8: return tti_step_tiled<T, 8, 8, 1, 1>(t, adjoint, target_blocks, st);
    case 9: return adjoint ? tti_step_tiled<T, 8, 8, 1, 1>(t, adjoint, target_blocks, st)
                           : tti_step_tiled<T, 8, 4, 2, 1>(t, adjoint, target_blocks, st);
    case 10: return adjoint ? tti_step_tiled<T, 8, 8, 1, 1>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 8, 2, 1>(t, adjoint, target_blocks, st);
    case 11: return adjoint ? tti_step_tiled<T, 8, 8, 1, 2>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1>(t, adjoint, target_blocks, st);
    case 12: return adjoint ? tti_step_tiled<T, 8, 4, 1, 2>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1>(t, adjoint, target_blocks, st);
    case 13: return adjoint ? tti_step_tiled<T, 8, 8, 1, 3, 1>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1>(t, adjoint, target_blocks, st);
    case 14: return adjoint ? tti_step_tiled<T, 8, 8, 1, 3, 2>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1>(t, adjoint, target_blocks, st);
    case 15: return adjoint ? tti_step_tiled<T, 8, 8, 1, 3, 3>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1>(t, adjoint, target_blocks, st);
    case 16: return adjoint ? tti_step_tiled<T, 8, 8, 1, 3, 3>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1, 1, 2>(t, adjoint, target_blocks, st);
    case 17: return adjoint ? tti_step_tiled<T, 8, 8, 1, 3, 3>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1, 1, 3, true>(t, adjoint, target_blocks, st);
    case 18: return adjoint ? tti_step_tiled<T, 8, 8, 1, 4, 3>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1, 1, 3, true>(t, adjoint, target_blocks, st);
    case 19: return adjoint ? tti_step_tiled<T, 8, 8, 1, 5, 3>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1, 1, 3, true>(t, adjoint, target_blocks, st);
    case 20: return adjoint ? tti_step_tiled<T, 8, 8, 1, 5, 4>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1, 1, 3, true>(t, adjoint, target_blocks, st);
    case 21: return adjoint ? tti_step_tiled<T, 8, 8, 1, 5, 6>(t, adjoint, target_blocks, st)
                            : tti_step_tiled<T, 8, 4, 2, 1, 1, 3, true>(t, adjoint, target_blocks, st);
    default: return tti_step_tiled<T, 8, 4, 1, 1>(t, adjoint, target_blocks, st);  // 6
  }
}

template hipError_t launch_tti_step_tiled<float>(const TtiArgs<float> &, bool, int, int,
                                                 hipStream_t);
template hipError_t launch_tti_step_tiled<double>(const TtiArgs<double> &, bool, int, int,
                                                  hipStream_t);

}  // namespace rtm
