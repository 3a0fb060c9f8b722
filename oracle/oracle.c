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

/* The point operators on their own (Ps^T and Pr of the sweeps), so that the
 * multilinear weights can be checked without a time step:
 *   orc_sample_points: out[p] = sum_c w_c field[c] for each position
 *   orc_inject_points: field[c] += w_c val[p] (field accumulated, not cleared)
 * Return 0, or -2 if a position lies outside the grid (nothing written). */
int orc_sample_points(int ndim, long nz, long ny, long nx, int np, const double *pos,
                      const double *field, double *out) {
  int err = 0;
  pt_t *pts = make_points(ndim, nz, ny, nx, np, pos, &err);
  if (!err) sample(pts, np, field, out);
  free(pts);
  return err;
}

int orc_inject_points(int ndim, long nz, long ny, long nx, int np, const double *pos,
                      const double *val, double *field) {
  int err = 0;
  pt_t *pts = make_points(ndim, nz, ny, nx, np, pos, &err);
  if (!err) inject(pts, np, val, field);
  free(pts);
  return err;
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

/* ------------------------------------------------------------------------ */
/* pseudo-acoustic TTI (coupled p, q system)                                 */
/* ------------------------------------------------------------------------ */
/*
 * Operators (8th order, field zero outside the grid):
 *   D_a   first derivative on axis a, weights +-(4/5, -1/5, 4/105, -1/280)/h
 *   D_aa  second derivative on axis a (the weights above), L = sum_a D_aa
 *   n     symmetry axis (sin th cos ph, sin th sin ph, cos th) as (x, y, z)
 *   Hz u  = sum_a n_a^2 D_aa u + sum_{a != b} n_a n_b D_a (D_b u)
 *   H0 u  = L u - Hz u
 * Forward:  m p_tt = (1+2 eps) H0 p + sqrt(1+2 delta) Hz q
 *           m q_tt = sqrt(1+2 delta) H0 p + Hz q
 * The transpose puts the coefficients inside the derivatives:
 *   HzT w = sum_a D_aa (n_a^2 w) + sum_{a != b} D_a D_b (n_a n_b w)
 *   adjoint p equation:  H0T (c1 lp + c2 lq),   q equation:  HzT (c2 lp + lq)
 * with c1 = 1 + 2 eps, c2 = sqrt(1 + 2 delta), H0T w = L w - HzT w.
 * Sources are injected into p and q; receivers record p.
 */
static const double W1[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

/* out = D_axis u (axis 0 = z, 1 = y, 2 = x) */
static void first_deriv(long nz, long ny, long nx, double h, int axis, const double *u,
                        double *out) {
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        double s = 0.0;
        for (int j = 1; j <= 4; ++j) {
          long dz = axis == 0 ? j : 0, dy = axis == 1 ? j : 0, dx = axis == 2 ? j : 0;
          s += W1[j] * (at(u, nz, ny, nx, z + dz, y + dy, x + dx) -
                        at(u, nz, ny, nx, z - dz, y - dy, x - dx));
        }
        out[(z * ny + y) * nx + x] = s / h;
      }
}

/* out = D_axis,axis u */
static void second_deriv(long nz, long ny, long nx, double h, int axis, const double *u,
                         double *out) {
#pragma omp parallel for schedule(static)
  for (long z = 0; z < nz; ++z)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        double s = W2[0] * at(u, nz, ny, nx, z, y, x);
        for (int j = 1; j <= 4; ++j) {
          long dz = axis == 0 ? j : 0, dy = axis == 1 ? j : 0, dx = axis == 2 ? j : 0;
          s += W2[j] * (at(u, nz, ny, nx, z + dz, y + dy, x + dx) +
                        at(u, nz, ny, nx, z - dz, y - dy, x - dx));
        }
        out[(z * ny + y) * nx + x] = s / (h * h);
      }
}

/* axis components of the symmetry axis per cell: nax[0..2] = (n_z, n_y, n_x) */
static void tti_axis(long N, const double *theta, const double *phi, double *nax) {
  for (long i = 0; i < N; ++i) {
    nax[i] = cos(theta[i]);                       /* z */
    nax[N + i] = sin(theta[i]) * sin(phi[i]);     /* y */
    nax[2 * N + i] = sin(theta[i]) * cos(phi[i]); /* x */
  }
}

/* Hz u (transpose = 0) or HzT u (transpose = 1); work: 2 N doubles */
static void apply_hz(long nz, long ny, long nx, double h, const double *nax, int transpose,
                     const double *u, double *out, double *w1, double *w2) {
  const long N = nz * ny * nx;
  for (long i = 0; i < N; ++i) out[i] = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double *na = nax + a * N;
    if (transpose) {
      for (long i = 0; i < N; ++i) w1[i] = na[i] * na[i] * u[i];
      second_deriv(nz, ny, nx, h, a, w1, w2);
      for (long i = 0; i < N; ++i) out[i] += w2[i];
    } else {
      second_deriv(nz, ny, nx, h, a, u, w2);
      for (long i = 0; i < N; ++i) out[i] += na[i] * na[i] * w2[i];
    }
    for (int b = 0; b < 3; ++b) {
      if (b == a) continue;
      const double *nb = nax + b * N;
      if (transpose) { /* D_a D_b (n_a n_b u) */
        for (long i = 0; i < N; ++i) w1[i] = na[i] * nb[i] * u[i];
        first_deriv(nz, ny, nx, h, b, w1, w2);
        first_deriv(nz, ny, nx, h, a, w2, w1);
        for (long i = 0; i < N; ++i) out[i] += w1[i];
      } else { /* n_a n_b D_a (D_b u) */
        first_deriv(nz, ny, nx, h, b, u, w1);
        first_deriv(nz, ny, nx, h, a, w1, w2);
        for (long i = 0; i < N; ++i) out[i] += na[i] * nb[i] * w2[i];
      }
    }
  }
}

/* The TTI spatial operator (or its transpose) on (p, q): op, oq. */
void orc_tti_apply(long nz, long ny, long nx, double h, const double *eps, const double *delta,
                   const double *theta, const double *phi, int transpose, const double *p,
                   const double *q, double *op, double *oq) {
  const long N = nz * ny * nx;
  double *nax = malloc(sizeof(double) * 3 * N);
  double *w1 = malloc(sizeof(double) * N), *w2 = malloc(sizeof(double) * N);
  double *t1 = malloc(sizeof(double) * N), *t2 = malloc(sizeof(double) * N);
  double *lap = malloc(sizeof(double) * N);
  tti_axis(N, theta, phi, nax);
  if (!transpose) {
    /* op = c1 (L p - Hz p) + c2 Hz q ; oq = c2 (L p - Hz p) + Hz q */
    orc_laplacian(3, nz, ny, nx, h, p, lap);
    apply_hz(nz, ny, nx, h, nax, 0, p, t1, w1, w2); /* Hz p */
    apply_hz(nz, ny, nx, h, nax, 0, q, t2, w1, w2); /* Hz q */
    for (long i = 0; i < N; ++i) {
      const double c1 = 1.0 + 2.0 * eps[i], c2 = sqrt(1.0 + 2.0 * delta[i]);
      const double h0p = lap[i] - t1[i];
      op[i] = c1 * h0p + c2 * t2[i];
      oq[i] = c2 * h0p + t2[i];
    }
  } else {
    /* op = H0T (c1 p + c2 q) ; oq = HzT (c2 p + q) */
    double *a = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N);
    for (long i = 0; i < N; ++i) {
      const double c1 = 1.0 + 2.0 * eps[i], c2 = sqrt(1.0 + 2.0 * delta[i]);
      a[i] = c1 * p[i] + c2 * q[i];
      b[i] = c2 * p[i] + q[i];
    }
    orc_laplacian(3, nz, ny, nx, h, a, lap);
    apply_hz(nz, ny, nx, h, nax, 1, a, t1, w1, w2); /* HzT a */
    apply_hz(nz, ny, nx, h, nax, 1, b, t2, w1, w2); /* HzT b */
    for (long i = 0; i < N; ++i) {
      op[i] = lap[i] - t1[i];
      oq[i] = t2[i];
    }
    free(a);
    free(b);
  }
  free(nax);
  free(w1);
  free(w2);
  free(t1);
  free(t2);
  free(lap);
}

/*
 * TTI sweep, forward (adjoint = 0) or adjoint (adjoint = 1), with the damped
 * leapfrog of the acoustic case applied to p and q.
 *   forward: q_src [nt][ninj] injected into p and q; d[n] = Pr p^{n+1}
 *   adjoint: res [nt][ninj] injected into lam_p only; qadj[n] = Ps (lp + lq)^n
 * Probing (Z, Ubar [2][r][M]): forward probes (p_tt, q_tt); adjoint (lp, lq);
 * M = nsample cells sample_idx[0..nsample-1] when nsample > 0, else all N.
 * fhist [2][nt][N] (forward: written with p_tt, q_tt; adjoint: read) and
 * corr [N]: adjoint only, corr += p_tt lp + q_tt lq.
 */
int orc_tti_sweep(int adjoint, long nz, long ny, long nx, double h, double dt, int nt, int nb,
                  double c_ref, double R, const double *m, const double *eps,
                  const double *delta, const double *theta, const double *phi, int ninj,
                  const double *inj_pos, const double *inj_val, int nsmp, const double *smp_pos,
                  double *smp_out, int r, const double *Z, long nsample,
                  const long *sample_idx, double *Ubar, double *fhist, double *corr) {
  const long N = nz * ny * nx;
  int err = 0;
  pt_t *ip = make_points(3, nz, ny, nx, ninj, inj_pos, &err);
  pt_t *sp = make_points(3, nz, ny, nx, nsmp, smp_pos, &err);
  if (err) {
    free(ip);
    free(sp);
    return err;
  }
  double *eta = damping_field(3, nz, ny, nx, nb, h, c_ref, R);
  double *p0 = calloc(N, 8), *p1 = calloc(N, 8), *p2 = calloc(N, 8);
  double *q0 = calloc(N, 8), *q1 = calloc(N, 8), *q2 = calloc(N, 8);
  double *rp = calloc(N, 8), *rq = calloc(N, 8), *sfp = calloc(N, 8), *sfq = calloc(N, 8);
  double *tmp = calloc(N, 8);
  /* p1, q1: current level; p0, q0: previous; p2, q2: next */
  for (int s = 0; s < nt; ++s) {
    const int n = adjoint ? nt - 1 - s : s;
    orc_tti_apply(nz, ny, nx, h, eps, delta, theta, phi, adjoint, p1, q1, rp, rq);
    if (!adjoint) {
      inject(ip, ninj, inj_val + (long)n * ninj, rp);
      inject(ip, ninj, inj_val + (long)n * ninj, rq);
    } else {
      inject(ip, ninj, inj_val + (long)n * ninj, rp);
    }
    update(N, dt, m, eta, p1, p0, rp, p2);
    update(N, dt, m, eta, q1, q0, rq, q2);
    if (smp_out) {
      if (!adjoint) {
        sample(sp, nsmp, p2, smp_out + (long)n * nsmp);
      } else {
        for (long i = 0; i < N; ++i) tmp[i] = p2[i] + q2[i];
        sample(sp, nsmp, tmp, smp_out + (long)n * nsmp);
      }
    }
    if (!adjoint) {
      for (long i = 0; i < N; ++i) {
        sfp[i] = (p2[i] - 2.0 * p1[i] + p0[i]) / (dt * dt);
        sfq[i] = (q2[i] - 2.0 * q1[i] + q0[i]) / (dt * dt);
      }
      if (fhist) {
        memcpy(fhist + (long)n * N, sfp, 8 * N);
        memcpy(fhist + ((long)nt + n) * N, sfq, 8 * N);
      }
    } else {
      memcpy(sfp, p2, 8 * N);
      memcpy(sfq, q2, 8 * N);
      if (fhist && corr)
        for (long i = 0; i < N; ++i)
          corr[i] += fhist[(long)n * N + i] * sfp[i] + fhist[((long)nt + n) * N + i] * sfq[i];
    }
    if (Ubar) {
      const long M = nsample > 0 ? nsample : N;
      const long *sidx = nsample > 0 ? sample_idx : NULL;
      probe_rank1(N, r, Z + (long)n * r, M, sidx, sfp, Ubar);
      probe_rank1(N, r, Z + (long)n * r, M, sidx, sfq, Ubar + (long)r * M);
    }
    double *t = p0;
    p0 = p1;
    p1 = p2;
    p2 = t;
    t = q0;
    q0 = q1;
    q1 = q2;
    q2 = t;
  }
  free(ip);
  free(sp);
  free(eta);
  free(p0);
  free(p1);
  free(p2);
  free(q0);
  free(q1);
  free(q2);
  free(rp);
  free(rq);
  free(sfp);
  free(sfq);
  free(tmp);
  return 0;
}
