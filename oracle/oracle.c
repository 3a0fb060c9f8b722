/*
 * FP64 CPU oracle for adjoint-state imaging with randomized trace estimation
 * (Louboutin & Herrmann, "Enabling wave-based inversion on GPUs with
 * randomized trace estimation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load, call or
 * link this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library; the two meet only in the seeded inputs they are given.
 *
 * Everything here is plain double precision, written step by step in the
 * order the method states, with no blocking, fusion or reordering:
 *
 *   Operator   L = sum over axes of the 8th-order central second difference
 *              (Fornberg weights), with the field taken as zero outside the
 *              grid, so that L is symmetric.
 *   Damping    eta(z,y,x) = eta_z + eta_y + eta_x, each a quadratic sponge
 *              profile 3 ln(1/R) d^2 / (2 nb h c_ref) over the nb outermost
 *              cells of its axis (d = normalised depth into the layer).
 *   Forward    (Section "Approximate gradient calculations": the forward
 *              wavefield u[t] of the zero-lag imaging condition, Eq. 2)
 *              u^{-1} = u^0 = 0; for n = 0..nt-1:
 *                u^{n+1} = [2 m u^n - (m - eta dt/2) u^{n-1}
 *                           + dt^2 (L u^n + Ps^T q[n])] / (m + eta dt/2)
 *                d[n]    = Pr u^{n+1}
 *                s^n     = (u^{n+1} - 2 u^n + u^{n-1}) / dt^2   (second time
 *                          derivative of Eq. 2)   or   s^n = u^n
 *                Ubar[i] += Z[n][i] s^n          (Eq. 3: Ubar = Q^T s, Q = Z)
 *   Adjoint    (the time-reversed adjoint wavefield v[t] of Eq. 2)
 *              lam^{nt} = lam^{nt+1} = 0; for n = nt-1..0:
 *                lam^n = [2 m lam^{n+1} - (m - eta dt/2) lam^{n+2}
 *                         + dt^2 (L lam^{n+1} + Pr^T res[n])] / (m + eta dt/2)
 *                qadj[n] = Ps lam^n                 (adjoint of q -> d)
 *                Vbar[i] += Z[n][i] lam^n            (Eq. 3: Vbar = Q^T v)
 *                corr    += hist[n] * lam^n          (Eq. 2, full history)
 *
 * With J = 1/2 sum_n |d[n] - d_obs[n]|^2 and res = d - d_obs, the exact
 * gradient of the discrete misfit is -sum_n s^n * lam^n (s = second time
 * derivative), and the probed estimate is -(1/r) sum_i Ubar[i] * Vbar[i].
 *
 * Ps, Pr are multilinear interpolation at positions given in grid units
 * (z, y, x); injection is the exact transpose of sampling.
 *
 * Layout: C order [z][y][x], x fastest; 2D grids use ny = 1 and no y term.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* 8th-order central second-derivative weights, offsets 0..4 (Fornberg). */
static const double W2[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0,
                             -1.0 / 560.0};

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* damping                                                                   */
/* ------------------------------------------------------------------------ */
void orc_damping_profile(long n, int nb, double h, double c_ref, double R, double *eta) {
  for (long i = 0; i < n; ++i) {
    double d = 0.0;
    if (nb > 0) {
      double a = (double)(nb - i);
      double b = (double)(i - (n - 1 - nb));
      d = a > b ? a : b;
      if (d < 0.0) d = 0.0;
      d /= (double)nb;
    }
    eta[i] = nb > 0 ? 3.0 * log(1.0 / R) * d * d / (2.0 * nb * h * c_ref) : 0.0;
  }
}

static double *damping_field(int ndim, long nz, long ny, long nx, int nb, double h,
                             double c_ref, double R) {
  double *ez = malloc(sizeof(double) * nz), *ey = malloc(sizeof(double) * ny),
         *ex = malloc(sizeof(double) * nx);
  double *eta = malloc(sizeof(double) * nz * ny * nx);
  orc_damping_profile(nz, nb, h, c_ref, R, ez);
  orc_damping_profile(nx, nb, h, c_ref, R, ex);
  if (ndim == 3)
    orc_damping_profile(ny, nb, h, c_ref, R, ey);
  else
    for (long y = 0; y < ny; ++y) ey[y] = 0.0;
  for (long z = 0; z < nz; ++z)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) eta[(z * ny + y) * nx + x] = ez[z] + ey[y] + ex[x];
  free(ez);
  free(ey);
  free(ex);
  return eta;
}

/* ------------------------------------------------------------------------ */
/* Laplacian                                                                 */
/* ------------------------------------------------------------------------ */
static inline double at(const double *u, long nz, long ny, long nx, long z, long y, long x) {
  if (z < 0 || z >= nz || y < 0 || y >= ny || x < 0 || x >= nx) return 0.0;
  return u[(z * ny + y) * nx + x];
}

void orc_laplacian(int ndim, long nz, long ny, long nx, double h, const double *u,
                   double *out) {
  const double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        double dzz = W2[0] * at(u, nz, ny, nx, z, y, x);
        double dxx = W2[0] * at(u, nz, ny, nx, z, y, x);
        double dyy = 0.0;
        for (int j = 1; j <= 4; ++j) {
          dzz += W2[j] * (at(u, nz, ny, nx, z + j, y, x) + at(u, nz, ny, nx, z - j, y, x));
          dxx += W2[j] * (at(u, nz, ny, nx, z, y, x + j) + at(u, nz, ny, nx, z, y, x - j));
        }
        if (ndim == 3) {
          dyy = W2[0] * at(u, nz, ny, nx, z, y, x);
          for (int j = 1; j <= 4; ++j)
            dyy += W2[j] * (at(u, nz, ny, nx, z, y + j, x) + at(u, nz, ny, nx, z, y - j, x));
        }
        out[(z * ny + y) * nx + x] = (dzz + dyy + dxx) * ih2;
      }
}

/* ------------------------------------------------------------------------ */
/* multilinear point operators                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nc;           /* corners with their weights (<= 8) */
  long idx[8];
  double w[8];
} pt_t;

/* Returns 0 on success, -1 if the position is outside [0, n-1] on an axis. */
static int point_weights(int ndim, long nz, long ny, long nx, const double *p, pt_t *out) {
  long n[3] = {nz, ny, nx};
  long i0[3];
  double f[3];
  int two[3];
  for (int a = 0; a < 3; ++a) {
    double v = p[a];
    if (a == 1 && ndim == 2) v = 0.0;
    if (!(v >= 0.0 && v <= (double)(n[a] - 1))) return -1;
    double fl = floor(v);
    i0[a] = (long)fl;
    f[a] = v - fl;
    two[a] = f[a] > 0.0;
  }
  out->nc = 0;
  for (int cz = 0; cz <= two[0]; ++cz)
    for (int cy = 0; cy <= two[1]; ++cy)
      for (int cx = 0; cx <= two[2]; ++cx) {
        double w = (cz ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) *
                   (cx ? f[2] : 1.0 - f[2]);
        long id = ((i0[0] + cz) * ny + (i0[1] + cy)) * nx + (i0[2] + cx);
        out->idx[out->nc] = id;
        out->w[out->nc] = w;
        out->nc++;
      }
  return 0;
}

static pt_t *make_points(int ndim, long nz, long ny, long nx, int np, const double *pos,
                         int *err) {
  pt_t *pts = malloc(sizeof(pt_t) * (np > 0 ? np : 1));
  for (int p = 0; p < np; ++p)
    if (point_weights(ndim, nz, ny, nx, pos + 3 * p, &pts[p])) *err = -2;
  return pts;
}

static void inject(const pt_t *pts, int np, const double *val, double *field) {
  for (int p = 0; p < np; ++p)
    for (int c = 0; c < pts[p].nc; ++c) field[pts[p].idx[c]] += pts[p].w[c] * val[p];
}

static void sample(const pt_t *pts, int np, const double *field, double *out) {
  for (int p = 0; p < np; ++p) {
    double s = 0.0;
    for (int c = 0; c < pts[p].nc; ++c) s += pts[p].w[c] * field[pts[p].idx[c]];
    out[p] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* one time step of the damped recursion                                     */
/* ------------------------------------------------------------------------ */
static void update(long N, double dt, const double *m, const double *eta, const double *cur,
                   const double *prev, const double *lap, double *next) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double a = eta[i] * dt * 0.5;
    next[i] = (2.0 * m[i] * cur[i] - (m[i] - a) * prev[i] + dt * dt * lap[i]) / (m[i] + a);
  }
}

/* Ubar[i][j] += z[i] * s[cell j]  for the sampled cells (or all cells). */
static void probe_rank1(long N, int r, const double *z, long ns, const long *sidx,
                        const double *s, double *Ubar) {
  long M = sidx ? ns : N;
  for (int i = 0; i < r; ++i) {
    double *row = Ubar + (long)i * M;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < M; ++j) row[j] += z[i] * s[sidx ? sidx[j] : j];
  }
}

/*
 * Forward sweep.  Returns 0, or a negative code: -1 bad sizes, -2 a position
 * outside the grid.  Output arrays that are NULL are not produced.
 *   q      [nt][nsrc]     injected as is (a point source divides by h^ndim)
 *   d      [nt][nrec]     d[n] = Pr u^{n+1}
 *   Z      [nt][r]        probe rows (any real values); Ubar [r][M] is
 *                         accumulated (the caller zero-fills), M = nsample or N
 *   what   1: probe the second time derivative, 0: probe u^n
 *   hist   [nt][N]        the probed field s^n of every step
 *   fin    [2][N]         u^{nt}, u^{nt-1}
 */
int orc_forward(int ndim, long nz, long ny, long nx, double h, double dt, int nt, int nb,
                double c_ref, double R, const double *m, int nsrc, const double *src_pos,
                const double *q, int nrec, const double *rec_pos, double *d, int r,
                const double *Z, int what, long nsample, const long *sample_idx,
                double *Ubar, double *hist, double *fin) {
  if (ndim != 2 && ndim != 3) return -1;
  if (ndim == 2 && ny != 1) return -1;
  const long N = nz * ny * nx;
  int err = 0;
  pt_t *sp = make_points(ndim, nz, ny, nx, nsrc, src_pos, &err);
  pt_t *rp = make_points(ndim, nz, ny, nx, nrec, rec_pos, &err);
  if (err) {
    free(sp);
    free(rp);
    return err;
  }
  double *eta = damping_field(ndim, nz, ny, nx, nb, h, c_ref, R);
  double *prev = calloc(N, sizeof(double)), *cur = calloc(N, sizeof(double));
  double *next = calloc(N, sizeof(double)), *lap = calloc(N, sizeof(double));
  double *sfield = calloc(N, sizeof(double));
  for (int n = 0; n < nt; ++n) {
    orc_laplacian(ndim, nz, ny, nx, h, cur, lap);
    inject(sp, nsrc, q + (long)n * nsrc, lap);
    update(N, dt, m, eta, cur, prev, lap, next);
    if (d) sample(rp, nrec, next, d + (long)n * nrec);
    if (Ubar || hist) {
      if (what) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i) sfield[i] = (next[i] - 2.0 * cur[i] + prev[i]) / (dt * dt);
      } else {
        memcpy(sfield, cur, sizeof(double) * N);
      }
      if (Ubar) probe_rank1(N, r, Z + (long)n * r, nsample, sample_idx, sfield, Ubar);
      if (hist) memcpy(hist + (long)n * N, sfield, sizeof(double) * N);
    }
    double *t = prev;
    prev = cur;
    cur = next;
    next = t;
  }
  if (fin) {
    memcpy(fin, cur, sizeof(double) * N);
    memcpy(fin + N, prev, sizeof(double) * N);
  }
  free(sp);
  free(rp);
  free(eta);
  free(prev);
  free(cur);
  free(next);
  free(lap);
  free(sfield);
  return 0;
}

/*
 * Adjoint sweep (time reversed).  res [nt][nrec] drives it at the receivers.
 *   qadj  [nt][nsrc]  Ps lam^n (the adjoint of the map q -> d), or NULL
 *   Vbar  [r][M]      accumulated with probe row n paired with lam^n
 *   fhist [nt][N]     if given, corr[N] += fhist[n] * lam^n (zero-lag, Eq. 2)
 *   lhist [nt][N]     if given, receives lam^n
 */
int orc_adjoint(int ndim, long nz, long ny, long nx, double h, double dt, int nt, int nb,
                double c_ref, double R, const double *m, int nrec, const double *rec_pos,
                const double *res, int nsrc, const double *src_pos, double *qadj, int r,
                const double *Z, long nsample, const long *sample_idx, double *Vbar,
                const double *fhist, double *corr, double *lhist) {
  if (ndim != 2 && ndim != 3) return -1;
  if (ndim == 2 && ny != 1) return -1;
  const long N = nz * ny * nx;
  int err = 0;
  pt_t *sp = make_points(ndim, nz, ny, nx, nsrc, src_pos, &err);
  pt_t *rp = make_points(ndim, nz, ny, nx, nrec, rec_pos, &err);
  if (err) {
    free(sp);
    free(rp);
    return err;
  }
  double *eta = damping_field(ndim, nz, ny, nx, nb, h, c_ref, R);
  double *l2 = calloc(N, sizeof(double)), *l1 = calloc(N, sizeof(double));
  double *l0 = calloc(N, sizeof(double)), *lap = calloc(N, sizeof(double));
  for (int n = nt - 1; n >= 0; --n) {
    orc_laplacian(ndim, nz, ny, nx, h, l1, lap);
    inject(rp, nrec, res + (long)n * nrec, lap);
    update(N, dt, m, eta, l1, l2, lap, l0);
    if (qadj) sample(sp, nsrc, l0, qadj + (long)n * nsrc);
    if (Vbar) probe_rank1(N, r, Z + (long)n * r, nsample, sample_idx, l0, Vbar);
    if (fhist && corr) {
      const double *f = fhist + (long)n * N;
#pragma omp parallel for schedule(static)
      for (long i = 0; i < N; ++i) corr[i] += f[i] * l0[i];
    }
    if (lhist) memcpy(lhist + (long)n * N, l0, sizeof(double) * N);
    double *t = l2;
    l2 = l1;
    l1 = l0;
    l0 = t;
  }
  free(sp);
  free(rp);
  free(eta);
  free(l2);
  free(l1);
  free(l0);
  free(lap);
  return 0;
}
