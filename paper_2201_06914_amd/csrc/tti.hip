// Pseudo-acoustic TTI time step (coupled p, q fields) and its exact transpose.
//
//   m p_tt = c1 H0 p + c2 Hz q,   m q_tt = c2 H0 p + Hz q,
//   Hz u = sum_a n_a^2 D_aa u + sum_{a != b} n_a n_b D_a (D_b u),  H0 = L - Hz,
//   c1 = 1 + 2 eps, c2 = sqrt(1 + 2 delta), n = (sin th cos ph, sin th sin ph, cos th)
//   as (x, y, z), D_a / D_aa 8th-order first / second differences, fields zero
//   outside the grid.  The transpose moves coefficients inside the derivatives:
//   lam_p: H0T (c1 lp + c2 lq),  lam_q: HzT (c2 lp + lq),
//   HzT w = sum_a D_aa (n_a^2 w) + sum_{a != b} D_a D_b (n_a n_b w).
// Both use the damped leapfrog of the acoustic step on each field.
//
// Kernels (one thread per cell; three passes per step):
//   k_tti_coef     c1, c2, n_z, n_y, n_x from eps, delta, theta, phi (once)
//   forward:  k_tti_grad   G_b = D_b p, K_b = D_b q (6 fields)
//             k_tti_fwd    second differences, mixed terms D_a G_b, update
//   adjoint:  k_tti_comb   w1 = c1 lp + c2 lq, w2 = c2 lp + lq
//             k_tti_flux   F_a = sum_{b != a} D_b (n_a n_b w) for w1, w2 (6 fields)
//             k_tti_adj    D_aa (n_a^2 w), D_a F_a, L w1, update
#include "tti_common.h"

namespace rtm {

template <typename T>
__device__ __forceinline__ T tti_at(const T *u, const StepArgs<T> &a, int z, int y, int x) {
  return (z >= 0 && z < a.nz && y >= 0 && y < a.ny && x >= 0 && x < a.nx)
             ? u[((int64_t)z * a.ny + y) * a.nx + x]
             : T(0);
}

template <typename T>
__device__ __forceinline__ void tti_cell(const StepArgs<T> &a, int64_t i, int &z, int &y, int &x) {
  x = (int)(i % a.nx);
  const int64_t zy = i / a.nx;
  y = (int)(zy % a.ny);
  z = (int)(zy / a.ny);
}

// D_axis u at (z, y, x); axis 0 = z, 1 = y, 2 = x
template <typename T>
__device__ __forceinline__ T d1_at(const TtiArgs<T> &t, const T *u, int axis, int z, int y,
                                   int x) {
  const int dz = axis == 0, dy = axis == 1, dx = axis == 2;
  const StepArgs<T> &a = t.a;
  T s = t.d1 * (tti_at(u, a, z + dz, y + dy, x + dx) - tti_at(u, a, z - dz, y - dy, x - dx));
  s += t.d2 * (tti_at(u, a, z + 2 * dz, y + 2 * dy, x + 2 * dx) -
               tti_at(u, a, z - 2 * dz, y - 2 * dy, x - 2 * dx));
  s += t.d3 * (tti_at(u, a, z + 3 * dz, y + 3 * dy, x + 3 * dx) -
               tti_at(u, a, z - 3 * dz, y - 3 * dy, x - 3 * dx));
  s += t.d4 * (tti_at(u, a, z + 4 * dz, y + 4 * dy, x + 4 * dx) -
               tti_at(u, a, z - 4 * dz, y - 4 * dy, x - 4 * dx));
  return s;
}

// D_axis,axis of (f * u) at (z, y, x), f = NULL for plain u
template <typename T>
__device__ __forceinline__ T d2_at(const TtiArgs<T> &t, const T *u, const T *f, int axis, int z,
                                   int y, int x) {
  const int dz = axis == 0, dy = axis == 1, dx = axis == 2;
  const StepArgs<T> &a = t.a;
  auto v = [&](int k) -> T {
    const int zz = z + k * dz, yy = y + k * dy, xx = x + k * dx;
    const T uu = tti_at(u, a, zz, yy, xx);
    if (!f) return uu;
    const T ff = tti_at(f, a, zz, yy, xx);
    return ff * ff * uu;
  };
  T s = t.c0 * v(0);
  s += a.c1 * (v(1) + v(-1));
  s += a.c2 * (v(2) + v(-2));
  s += a.c3 * (v(3) + v(-3));
  s += a.c4 * (v(4) + v(-4));
  return s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_tti_coef(const T *__restrict__ aniso, int64_t N,
                                                  T *__restrict__ coef) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    const double eps = aniso[i], del = aniso[N + i], th = aniso[2 * N + i], ph = aniso[3 * N + i];
    coef[i] = (T)(1.0 + 2.0 * eps);
    coef[N + i] = (T)sqrt(1.0 + 2.0 * del);
    coef[2 * N + i] = (T)cos(th);
    coef[3 * N + i] = (T)(sin(th) * sin(ph));
    coef[4 * N + i] = (T)(sin(th) * cos(ph));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tti_grad(TtiArgs<T> t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= t.a.N) return;
  int z, y, x;
  tti_cell(t.a, i, z, y, x);
  const int64_t N = t.a.N;
  for (int b = 0; b < 3; ++b) {
    t.g[b * N + i] = d1_at(t, t.p, b, z, y, x);
    t.g[(3 + b) * N + i] = d1_at(t, t.q, b, z, y, x);
  }
}

template <typename T>
__device__ __forceinline__ T damped_update(const StepArgs<T> &a, T u, T up, T m, T rhs, T damp) {
  return (T(2) * m * u - (m - damp) * up + a.dt2 * rhs) / (m + damp);
}

template <typename T>
__global__ __launch_bounds__(256) void k_tti_fwd(TtiArgs<T> t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const StepArgs<T> &a = t.a;
  if (i >= a.N) return;
  int z, y, x;
  tti_cell(a, i, z, y, x);
  const int64_t N = a.N;
  const T c1 = t.coef[i], c2 = t.coef[N + i];
  const T n[3] = {t.coef[2 * N + i], t.coef[3 * N + i], t.coef[4 * N + i]};
  T lp = T(0), hzp = T(0), hzq = T(0);
  for (int ax = 0; ax < 3; ++ax) {
    const T dp = d2_at(t, t.p, (const T *)nullptr, ax, z, y, x);
    const T dq = d2_at(t, t.q, (const T *)nullptr, ax, z, y, x);
    lp += dp;
    hzp += n[ax] * n[ax] * dp;
    hzq += n[ax] * n[ax] * dq;
  }
  for (int ax = 0; ax < 3; ++ax)
    for (int b = 0; b < 3; ++b) {
      if (b == ax) continue;
      const T nn = n[ax] * n[b];
      hzp += nn * d1_at(t, t.g + b * N, ax, z, y, x);
      hzq += nn * d1_at(t, t.g + (3 + b) * N, ax, z, y, x);
    }
  const T h0p = lp - hzp;
  const T damp = sponge_a(a, z, y, x);
  const T m = a.m[i];
  t.pn[i] = damped_update(a, t.p[i], t.pp[i], m, c1 * h0p + c2 * hzq, damp);
  t.qn[i] = damped_update(a, t.q[i], t.qp[i], m, c2 * h0p + hzq, damp);
}

// adjoint: w1 = c1 lp + c2 lq into g[0], w2 = c2 lp + lq into g[1]
template <typename T>
__global__ __launch_bounds__(256) void k_tti_comb(TtiArgs<T> t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= t.a.N) return;
  const int64_t N = t.a.N;
  const T c1 = t.coef[i], c2 = t.coef[N + i];
  t.g[i] = c1 * t.p[i] + c2 * t.q[i];
  t.g[N + i] = c2 * t.p[i] + t.q[i];
}

// F_a = sum_{b != a} D_b (n_a n_b w) for w = w1 (g[0]) and w2 (g[1]) into g[2..7]
template <typename T>
__global__ __launch_bounds__(256) void k_tti_flux(TtiArgs<T> t, T *__restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const StepArgs<T> &a = t.a;
  if (i >= a.N) return;
  int z, y, x;
  tti_cell(a, i, z, y, x);
  const int64_t N = a.N;
  const T *w1 = t.g, *w2 = t.g + N;
  const T *nax[3] = {t.coef + 2 * N, t.coef + 3 * N, t.coef + 4 * N};
  for (int ax = 0; ax < 3; ++ax) {
    T f1 = T(0), f2 = T(0);
    for (int b = 0; b < 3; ++b) {
      if (b == ax) continue;
      const int dz = b == 0, dy = b == 1, dx = b == 2;
      T s1 = T(0), s2 = T(0);
      for (int j = 4; j >= 1; --j) {
        const T wj = j == 1 ? t.d1 : j == 2 ? t.d2 : j == 3 ? t.d3 : t.d4;
        const int zp = z + j * dz, yp = y + j * dy, xp = x + j * dx;
        const int zm = z - j * dz, ym = y - j * dy, xm = x - j * dx;
        const T np_ = tti_at(nax[ax], a, zp, yp, xp) * tti_at(nax[b], a, zp, yp, xp);
        const T nm_ = tti_at(nax[ax], a, zm, ym, xm) * tti_at(nax[b], a, zm, ym, xm);
        s1 += wj * (np_ * tti_at(w1, a, zp, yp, xp) - nm_ * tti_at(w1, a, zm, ym, xm));
        s2 += wj * (np_ * tti_at(w2, a, zp, yp, xp) - nm_ * tti_at(w2, a, zm, ym, xm));
      }
      f1 += s1;
      f2 += s2;
    }
    F[ax * N + i] = f1;
    F[(3 + ax) * N + i] = f2;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tti_adj(TtiArgs<T> t, const T *__restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const StepArgs<T> &a = t.a;
  if (i >= a.N) return;
  int z, y, x;
  tti_cell(a, i, z, y, x);
  const int64_t N = a.N;
  const T *w1 = t.g, *w2 = t.g + N;
  T lw1 = T(0), hz1 = T(0), hz2 = T(0);
  for (int ax = 0; ax < 3; ++ax) {
    const T *na = t.coef + (2 + ax) * N;
    lw1 += d2_at(t, w1, (const T *)nullptr, ax, z, y, x);
    hz1 += d2_at(t, w1, na, ax, z, y, x);
    hz2 += d2_at(t, w2, na, ax, z, y, x);
    hz1 += d1_at(t, F + ax * N, ax, z, y, x);
    hz2 += d1_at(t, F + (3 + ax) * N, ax, z, y, x);
  }
  const T damp = sponge_a(a, z, y, x);
  const T m = a.m[i];
  t.pn[i] = damped_update(a, t.p[i], t.pp[i], m, lw1 - hz1, damp);
  t.qn[i] = damped_update(a, t.q[i], t.qp[i], m, hz2, damp);
}

// out[n] = Pr (p + q): the adjoint of injecting into both fields
template <typename T>
__global__ __launch_bounds__(256) void k_sample_sum(PointTables<T> pt, const T *__restrict__ f1,
                                                    const T *__restrict__ f2, T *__restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= pt.npts) return;
  T s = T(0);
  for (int j = pt.soff[p]; j < pt.soff[p + 1]; ++j) s += pt.sw[j] * (f1[pt.sidx[j]] + f2[pt.sidx[j]]);
  out[p] = s;
}

static unsigned cells_grid(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
hipError_t launch_tti_coef(const T *aniso, int64_t N, T *coef, hipStream_t st) {
  int64_t b = (N + 255) / 256;
  hipLaunchKernelGGL((k_tti_coef<T>), dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, st,
                     aniso, N, coef);
  return hipGetLastError();
}


template <typename T>
hipError_t launch_tti_step(const StepArgs<T> &a, double h, bool adjoint, const T *coef,
                           const T *p, const T *pp, const T *q, const T *qp, T *pn, T *qn, T *g,
                           int shape, int target_blocks, hipStream_t st) {
  TtiArgs<T> t = tti_args<T>(a, (T)h, coef, p, pp, q, qp, pn, qn, g);
  if (shape > 0) return launch_tti_step_tiled<T>(t, adjoint, shape, target_blocks, st);
  const unsigned nb = cells_grid(a.N);
  if (!adjoint) {
    hipLaunchKernelGGL((k_tti_grad<T>), dim3(nb), dim3(256), 0, st, t);
    hipLaunchKernelGGL((k_tti_fwd<T>), dim3(nb), dim3(256), 0, st, t);
  } else {
    hipLaunchKernelGGL((k_tti_comb<T>), dim3(nb), dim3(256), 0, st, t);
    T *F = g + 2 * a.N;
    hipLaunchKernelGGL((k_tti_flux<T>), dim3(nb), dim3(256), 0, st, t, F);
    hipLaunchKernelGGL((k_tti_adj<T>), dim3(nb), dim3(256), 0, st, t, (const T *)F);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sample_sum(const PointTables<T> &pt, const T *f1, const T *f2, T *out,
                             hipStream_t st) {
  if (pt.npts <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_sample_sum<T>), dim3((pt.npts + 255) / 256), dim3(256), 0, st, pt, f1,
                     f2, out);
  return hipGetLastError();
}

// Stability screen of a TTI model (before a sweep).  With the coefficients
// frozen at a cell, the coupled operator's symbol is C diag(h0, hz), C =
// [[1 + 2 eps, sqrt(1 + 2 delta)], [sqrt(1 + 2 delta), 1]], with h0, hz >= 0
// and h0 + hz the acoustic symbol; for delta <= eps its eigenvalues are real,
// non-negative and at most max(1, 1 + 2 eps)(h0 + hz), so the acoustic CFL
// bound holds with the velocity v sqrt(max(1, 1 + 2 eps)).  Each workgroup
// writes the largest max(1, 1 + 2 eps) / m of its cells and the count of
// cells with delta > eps, eps <= -1/2 or delta <= -1/2 (finite values only:
// a NaN or an infinity is left to the non-finite watch); one workgroup folds
// the partials into out[0] (largest v^2) and out[1] (count).
constexpr int kScreenBlocks = 512;

__device__ __forceinline__ void screen_fold(double &vmax, double &bad) {
  __shared__ double sv[4], sb[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    vmax = fmax(vmax, __shfl_down(vmax, off, 64));
    bad += __shfl_down(bad, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sv[wave] = vmax;
    sb[wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    vmax = fmax(fmax(sv[0], sv[1]), fmax(sv[2], sv[3]));
    bad = ((sb[0] + sb[1]) + sb[2]) + sb[3];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tti_screen(const T *__restrict__ m,
                                                    const T *__restrict__ aniso, int64_t N,
                                                    double *__restrict__ part) {
  double vmax = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    const double mi = m[i], e = aniso[i], d = aniso[N + i];
    const double c1 = 1.0 + 2.0 * e;
    if (isfinite(mi) && mi > 0.0 && isfinite(c1)) vmax = fmax(vmax, (c1 > 1.0 ? c1 : 1.0) / mi);
    if (isfinite(e) && isfinite(d) && (d > e || e <= -0.5 || d <= -0.5)) bad += 1.0;
  }
  screen_fold(vmax, bad);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = vmax;
    part[2 * blockIdx.x + 1] = bad;
  }
}

__global__ __launch_bounds__(256) void k_tti_screen_final(const double *__restrict__ part,
                                                          int np, double *__restrict__ out) {
  double vmax = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
    vmax = fmax(vmax, part[2 * i]);
    bad += part[2 * i + 1];
  }
  screen_fold(vmax, bad);
  if (threadIdx.x == 0) {
    out[0] = vmax;
    out[1] = bad;
  }
}

// Power iteration on m^{-1} A, A the coupled TTI operator without sponge,
// through the forward step with a zero previous level:
//     next = 2 cur + dt^2 m^{-1} A cur,  so  m^{-1} A cur = (next - 2 cur) / dt^2.
// The iterate (p, q) is kept at unit norm; |m^{-1} A cur| of the last
// iteration estimates the spectral radius.  Sums of squares in FP64, fixed
// order (partials per workgroup, then one workgroup).
__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double sv[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sv[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((sv[0] + sv[1]) + sv[2]) + sv[3];
  return s;
}

__device__ __forceinline__ double pi_start_value(uint64_t i, uint32_t seed) {
  uint32_t h = (uint32_t)i * 2654435761u ^ seed;  // Knuth multiplicative hash, then mixing
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  h *= 3266489917u;
  h ^= h >> 16;
  return ((double)(h >> 8) - 8388608.0) / 8388608.0;  // [-1, 1)
}

template <typename T>
__global__ __launch_bounds__(256) void k_pi_start(T *p, T *q, int64_t N, uint32_t seed,
                                                  double *part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    const T vp = (T)pi_start_value((uint64_t)i, seed), vq = (T)pi_start_value((uint64_t)(i + N), seed);
    p[i] = vp;
    q[i] = vq;
    acc += (double)vp * (double)vp + (double)vq * (double)vq;
  }
  const double sum = block_sum_d(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pi_diff(T *pn, T *qn, const T *p, const T *q, int64_t N,
                                                 T inv_dt2, double *part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    const T wp = (pn[i] - T(2) * p[i]) * inv_dt2, wq = (qn[i] - T(2) * q[i]) * inv_dt2;
    pn[i] = wp;
    qn[i] = wq;
    acc += (double)wp * (double)wp + (double)wq * (double)wq;
  }
  const double sum = block_sum_d(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

__global__ __launch_bounds__(256) void k_pi_final(const double *part, int np, double *out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  const double sum = block_sum_d(acc);
  if (threadIdx.x == 0) out[0] = sum;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pi_scale(T *p, T *q, const T *wp, const T *wq, int64_t N,
                                                  const double *sumsq) {
  const double s = 1.0 / sqrt(sumsq[0]);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    p[i] = (T)((double)wp[i] * s);
    q[i] = (T)((double)wq[i] * s);
  }
}

// levels: p, q (iterate), pz, qz (zero previous levels), pn, qn (next); part:
// 1026 doubles, |w|^2 of the last iteration left in part[1024]
template <typename T>
hipError_t tti_power_iteration(const StepArgs<T> &a0, double h, double dt, const T *coef, T *p,
                               T *q, T *pz, T *qz, T *pn, T *qn, T *g, int shape, int target_blocks,
                               int iters, uint32_t seed, double *part, hipStream_t st) {
  StepArgs<T> a = a0;
  a.kd = T(0);  // no sponge: the operator alone
  const int64_t N = a.N;
  constexpr int NB = 512;
  hipError_t e;
  if ((e = launch_fill<T>(pz, N, T(0), st)) != hipSuccess) return e;
  if ((e = launch_fill<T>(qz, N, T(0), st)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_pi_start<T>), dim3(NB), dim3(256), 0, st, p, q, N, seed, part);
  hipLaunchKernelGGL(k_pi_final, dim3(1), dim3(256), 0, st, part, NB, part + 1024);
  hipLaunchKernelGGL((k_pi_scale<T>), dim3(NB), dim3(256), 0, st, p, q, p, q, N, part + 1024);
  const T inv_dt2 = (T)(1.0 / (dt * dt));
  for (int it = 0; it < iters; ++it) {
    if ((e = launch_tti_step<T>(a, h, false, coef, p, pz, q, qz, pn, qn, g, shape, target_blocks,
                                st)) != hipSuccess)
      return e;
    hipLaunchKernelGGL((k_pi_diff<T>), dim3(NB), dim3(256), 0, st, pn, qn, p, q, N, inv_dt2, part);
    hipLaunchKernelGGL(k_pi_final, dim3(1), dim3(256), 0, st, part, NB, part + 1024);
    hipLaunchKernelGGL((k_pi_scale<T>), dim3(NB), dim3(256), 0, st, p, q, pn, qn, N, part + 1024);
  }
  return hipGetLastError();
}
template hipError_t tti_power_iteration<float>(const StepArgs<float> &, double, double,
                                               const float *, float *, float *, float *, float *,
                                               float *, float *, float *, int, int, int, uint32_t,
                                               double *, hipStream_t);
template hipError_t tti_power_iteration<double>(const StepArgs<double> &, double, double,
                                                const double *, double *, double *, double *,
                                                double *, double *, double *, double *, int, int,
                                                int, uint32_t, double *, hipStream_t);

// part: 2 kScreenBlocks + 2 doubles; the result lands in part[2 kScreenBlocks ..]
template <typename T>
hipError_t launch_tti_screen(const T *m, const T *aniso, int64_t N, double *part, hipStream_t st) {
  hipLaunchKernelGGL((k_tti_screen<T>), dim3(kScreenBlocks), dim3(256), 0, st, m, aniso, N, part);
  hipLaunchKernelGGL(k_tti_screen_final, dim3(1), dim3(256), 0, st, part, kScreenBlocks,
                     part + 2 * kScreenBlocks);
  return hipGetLastError();
}
template hipError_t launch_tti_screen<float>(const float *, const float *, int64_t, double *,
                                             hipStream_t);
template hipError_t launch_tti_screen<double>(const double *, const double *, int64_t, double *,
                                              hipStream_t);

template hipError_t launch_tti_coef<float>(const float *, int64_t, float *, hipStream_t);
template hipError_t launch_tti_coef<double>(const double *, int64_t, double *, hipStream_t);
template hipError_t launch_tti_step<float>(const StepArgs<float> &, double, bool, const float *,
                                           const float *, const float *, const float *,
                                           const float *, float *, float *, float *, int, int,
                                           hipStream_t);
template hipError_t launch_tti_step<double>(const StepArgs<double> &, double, bool, const double *,
                                            const double *, const double *, const double *,
                                            const double *, double *, double *, double *, int,
                                            int, hipStream_t);
template hipError_t launch_sample_sum<float>(const PointTables<float> &, const float *,
                                             const float *, float *, hipStream_t);
template hipError_t launch_sample_sum<double>(const PointTables<double> &, const double *,
                                              const double *, double *, hipStream_t);

}  // namespace rtm
