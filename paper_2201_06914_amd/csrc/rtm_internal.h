// Internal interface between the host side of librtm (plan, point tables,
// sweep sequencing) and its HIP kernels.  Not installed; the public ABI is
// include/rtm.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rtm {

// What one stencil step needs.  The 8th-order weights arrive already divided
// by h^2; cc = ndim * c[0] is the centre weight of the full Laplacian.  The
// sponge term a = eta * dt / 2 is rebuilt per cell from integer depths:
// a = kd * (dz^2 + dy^2 + dx^2) with d = cells into the layer, kd = A dt / (2 nb^2)
// and A = 3 ln(1/R) / (2 nb h c_ref).
template <typename T>
struct StepArgs {
  const T *__restrict__ cur;   // level s   (u^n, or lam^{n+1} in the adjoint)
  const T *__restrict__ prev;  // level s-1
  T *__restrict__ next;        // level s+1 (distinct ring slot)
  const T *__restrict__ m;     // slowness squared
  int nz, ny, nx;
  int nb;
  int64_t N;
  T c1, c2, c3, c4;  // off-centre weights / h^2
  T cc;              // ndim * centre weight / h^2
  T dt2;             // dt^2
  T kd;              // sponge coefficient per squared cell depth
};

// One shot of a batched sweep: its step arguments (level pointers are
// rebuilt per step from the ring: level j in slot (j+1) mod R).
template <typename T>
struct ShotStep {
  StepArgs<T> a;
  T *ring;
  int64_t ld;
  int R;
};

// Cell-local epilogue of the exact comparator's stencil steps.
enum { EPI_NONE = 0, EPI_D2 = 1, EPI_CORR = 2 };
template <typename T>
struct EpiArgs {
  T *d2 = nullptr;         // EPI_D2: (next - 2 cur + prev) * inv_dt2
  const T *s = nullptr;    // EPI_CORR: g -= s * next
  T *g = nullptr;
  T inv_dt2 = T(0);
};

// Point tables in CSR form (device pointers into the workspace).
template <typename T>
struct PointTables {
  // sampling: per point p, entries [soff[p], soff[p+1]) of (sidx, sw)
  const int32_t *soff = nullptr;
  const int32_t *sidx = nullptr;
  const T *sw = nullptr;
  // injection: per distinct cell c, entries [ioff[c], ioff[c+1]) of (ipt, iw)
  const int32_t *icell = nullptr;
  const int32_t *ioff = nullptr;
  const int32_t *ipt = nullptr;
  const T *iw = nullptr;
  int32_t npts = 0;
  int32_t ncell = 0;
};

// Point tables of a batch of shots: one CSR across all shots.  Sampling is
// per global point (its shot and local index); injection per distinct
// (shot, cell).  ShotIO gives each shot's value / output arrays of the sweep.
template <typename T>
struct BatchPoints {
  const int32_t *soff = nullptr, *sidx = nullptr, *sshot = nullptr, *slocal = nullptr;
  const T *sw = nullptr;
  const int32_t *icell = nullptr, *ishot = nullptr, *ioff = nullptr, *ipt = nullptr;
  const T *iw = nullptr;
  int32_t npts = 0, ncell = 0;
};
template <typename T>
struct ShotIO {
  const T *inj;   // [nt][n_inj] values injected at this shot's points
  T *out;         // [nt][n_smp] sampled traces, or NULL
  int32_t n_inj, n_smp;
};

// operand type of the MFMA probe path: bf16, bf16 hi + lo, or float16 with a
// power-of-two scale per 16-step chunk and 32-cell tile
enum ProbeOp : int { OP_BF16 = 0, OP_BF16X2 = 1, OP_F16S = 2 };
enum ProbeMode : int {
  PROBE_CUR = 0,  // level s          (forward u^n)
  PROBE_UTT = 1,  // levels s-1, s, s+1, second difference / dt^2
  PROBE_NEW = 2   // level s+1        (adjoint lam^n)
};

// One probe-GEMM block: bar[i][x] += sum_{t < kb} Z[zrow0 + zdir t][i] * S_t[x]
// for the sweep steps s0 .. s0+kb-1, where S_t is read from the level ring.
template <typename T>
struct ProbeArgs {
  const T *ring;     // R slots of ld elements; sweep level j lives in slot (j+1) mod R
  int64_t ld;        // slot stride (elements)
  int R;
  int slot0;         // slot of level s0 - 1, i.e. s0 mod R (levels s0-1 .. s0+R-2 follow)
  int s0, kb;
  int zrow0, zdir;
  int r;
  int64_t N;
  T *bar;            // tile-major [ceil(N/32)][r][32]
  T inv_dt2;
  int mode;
  // optional work-queue counter (device int) for the probe launches that hand
  // out tiles in order; nullptr: each wave strides over the tiles
  int *queue = nullptr;
};

// launchers (stream-ordered; return the launch status)
// rev != 0: the tiled kernels march each z-chunk downwards (same results)
template <typename T>
hipError_t launch_stencil(int ndim, const StepArgs<T> &a, int variant, int target_blocks,
                          hipStream_t st, int rev = 0);
// exact comparator: stencil step with a fused epilogue (hipErrorInvalidValue
// when no tiled kernel serves the grid), and the matching injection
template <typename T>
hipError_t launch_stencil_epi(int ndim, const StepArgs<T> &a, int variant, int target_blocks,
                              int epi, const EpiArgs<T> &e, hipStream_t st, int rev = 0);
template <typename T>
hipError_t launch_inject_epi(const StepArgs<T> &a, const PointTables<T> &pt, const T *vals,
                             T *field, int epi, const EpiArgs<T> &e, hipStream_t st);
// range-finder probes: space sketch of one k-step block into rows zrow0 ..
// zrow0 + kb - 1 of Y [nt][r] (FP64), partial scratch of
// sketch_partial_elems(N, kb, r) elements of T; orthonormal columns of Y into
// Q (V: FP64 scratch of nt x r)
int64_t sketch_grid(int64_t N);
int64_t sketch_partial_elems(int64_t N, int kb, int r);
template <typename T>
hipError_t launch_sketch(const ProbeArgs<T> &p, uint64_t seed, void *partial, double *Y,
                         hipStream_t st);
template <typename T>
hipError_t launch_orthonormalize(const double *Y, int nt, int r, double *V, T *Q, hipStream_t st);
// subsurface-offset image volume along x (Eq. 4): G [2 nh + 1][N], nh <= 64
template <typename T>
hipError_t launch_offset_gathers(const T *U, const T *V, int nfield, int64_t fstride, int64_t N,
                                 int nx, int r, int nh, double scale, T *G, hipStream_t st);
// batched sweep step (all shots, one launch each): stencil over the tile
// table, then injection / sampling of level s+1 for time index n
template <typename T>
hipError_t launch_stencil_batched(const ShotStep<T> *shots, const int4 *tiles, int ntiles, int s,
                                  int variant, hipStream_t st, int rev = 0);
template <typename T>
hipError_t launch_inject_batched(const ShotStep<T> *shots, const ShotIO<T> *io,
                                 const BatchPoints<T> &pt, int s, int n, hipStream_t st);
template <typename T>
hipError_t launch_sample_batched(const ShotStep<T> *shots, const ShotIO<T> *io,
                                 const BatchPoints<T> &pt, int s, int n, hipStream_t st);
// TTI: per-cell coefficients [5][N] = (1 + 2 eps, sqrt(1 + 2 delta), n_z, n_y,
// n_x) from aniso [4][N] = (eps, delta, theta, phi); one step of the coupled
// system (adjoint = exact transpose) with intermediates g [8][N]; sampling of
// p + q (adjoint of injecting into both fields)
template <typename T>
hipError_t launch_tti_coef(const T *aniso, int64_t N, T *coef, hipStream_t st);
// TTI stability screen: writes (largest max(1, 1 + 2 eps) / m, count of cells
// with delta > eps or eps, delta <= -1/2) to part[1024], part[1025]
// power iteration on m^{-1} A (TTI, no sponge); |m^{-1} A v|^2 of the last
// iteration (unit v) left in part[1024]
template <typename T>
hipError_t tti_power_iteration(const StepArgs<T> &a, double h, double dt, const T *coef, T *p,
                               T *q, T *pz, T *qz, T *pn, T *qn, T *g, int shape, int target_blocks,
                               int iters, uint32_t seed, double *part, hipStream_t st);
template <typename T>
hipError_t launch_tti_screen(const T *m, const T *aniso, int64_t N, double *part, hipStream_t st);
// (shape 0: one thread per cell; 1..3: column tiles marching z-chunks, split
// until target_blocks workgroups)
template <typename T>
hipError_t launch_tti_step(const StepArgs<T> &a, double h, bool adjoint, const T *coef,
                           const T *p, const T *pp, const T *q, const T *qp, T *pn, T *qn, T *g,
                           int shape, int target_blocks, hipStream_t st);
template <typename T>
hipError_t launch_sample_sum(const PointTables<T> &pt, const T *f1, const T *f2, T *out,
                             hipStream_t st);
// autotuning: hash pattern fill, count of bitwise-different elements (atomic
// integer add into *count)
template <typename T>
hipError_t launch_pattern(T *p, int64_t n, uint32_t seed, T scale, hipStream_t st);
template <typename T>
hipError_t launch_count_diff(const T *a, const T *b, int64_t n, unsigned long long *count,
                             hipStream_t st);
template <typename T>
hipError_t launch_inject(const StepArgs<T> &a, const PointTables<T> &pt, const T *vals,
                         T *field, hipStream_t st);
template <typename T>
hipError_t launch_sample(const PointTables<T> &pt, const T *field, T *out, hipStream_t st);
template <typename T>
hipError_t launch_probe_vec(const ProbeArgs<T> &p, const void *Z, bool z_is_i8,
                            hipStream_t st);
// Uf / img / scale: non-NULL img selects the fused adjoint imaging variant
// (img[c] += scale * sum_i Uf[i][c] (Z_b^T S_b)[i][c]; p.bar unused).
// Z is int8 +-1, or with zf32 real FP32 probes split into bf16 hi + lo (needs
// split).
void set_probe_nt(int on);
int get_probe_nt();
void set_probe_grid(int cap_update, int cap_fused);
int get_probe_grid(int fused);
hipError_t launch_probe_mfma(const ProbeArgs<float> &p, const void *Z, bool zf32, int op,
                             const float *Uf, float *img, float scale, hipStream_t st);
// exact imaging: out = (un - 2 u0 + um) * inv_dt2 ; g -= s * lam
template <typename T>
hipError_t launch_second_diff(const T *un, const T *u0, const T *um, T inv_dt2, int64_t n, T *out,
                              hipStream_t st);
template <typename T>
hipError_t launch_correlate(T *g, const T *s, const T *lam, int64_t n, hipStream_t st);
// tile-major compressed field -> rows [r][N]
template <typename T>
hipError_t launch_bar_to_rows(const T *bar, int64_t N, int r, T *rows, hipStream_t st);
template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t st);
template <typename T>
hipError_t launch_axpy(T *y, const T *x, int64_t n, hipStream_t st);  // y += x
template <typename T>
hipError_t launch_copy(T *dst, const T *src, int64_t n, hipStream_t st);
hipError_t launch_copy_x4(void *dst, const void *src, int64_t n16, hipStream_t st);
template <typename T>
hipError_t launch_flag_nonfinite(const T *x, int64_t n, uint32_t *status, hipStream_t st);
hipError_t launch_status_clear(uint32_t *status, hipStream_t st);
template <typename T>
hipError_t launch_image(const T *U, const T *V, int64_t N, int r, double scale, T *img,
                        hipStream_t st);
// res = d - d_obs (in place over d when res == d), misfit = 0.5 * sum res^2
template <typename T>
hipError_t launch_residual_misfit(const T *d, const T *dobs, T *res, int64_t n,
                                  double *partials, double *misfit, hipStream_t st);
template <typename T>
hipError_t launch_dot(const T *a, const T *b, int64_t n, double *partials, double *out,
                      hipStream_t st);

constexpr int kReduceBlocks = 1024;  // partial sums of the two-pass reductions

// Stencil variants: 0 = one thread per cell (any ndim, any dtype),
// 1 = LDS-tiled z-marching (3D).  Both share the per-cell arithmetic, so they
// give bitwise-identical levels.
constexpr int kStencilSimple = 0;
constexpr int kStencilTiled = 1;     // first LDS-tiled variant
constexpr int kStencilVariants = 13;  // last variant id

// XCD-aware block order: hardware workgroup ids go round-robin over the 8
// XCDs (id b to XCD b mod 8); XCD x receives ids x, x + 8, ... and this maps
// them to one contiguous run of logical blocks, so that neighbouring tiles
// (which share halo rows) run on the same XCD and meet in its L2.  A
// bijection of [0, nblk) for any nblk.
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int x = b & 7;
  int off = 0;
  for (int j = 0; j < x; ++j) off += (nblk - j + 7) >> 3;
  return off + (b >> 3);
}

}  // namespace rtm
