/*
 * rtm.h - C ABI of librtm, an MI355X (gfx950) library for adjoint-state wave
 * imaging with randomized trace estimation (Louboutin & Herrmann, "Enabling
 * wave-based inversion on GPUs with randomized trace estimation").
 *
 * The method (Section "Methodology"):
 *   - Eq. 1: tr(A) ~ (1/r) tr(Z^T A Z) for r random probe vectors (the
 *     columns of Z, entries +-1).
 *   - Eq. 2: the single-source gradient is the zero-lag correlation over time
 *     of the second time derivative of the forward wavefield with the adjoint
 *     wavefield, sum_t u_tt[t] v[t], cell by cell.
 *   - Eq. 3: per cell this is a trace, so it is estimated from the compressed
 *     fields Ubar = Q^T u_tt and Vbar = Q^T v (r rows instead of nt):
 *     dm[x] ~ (1/r) sum_i Ubar[i][x] Vbar[i][x].  Here Q = Z.
 *
 * Discretisation (the paper prints none; this library fixes it):
 *   2nd order in time, 8th order in space (Fornberg weights, field zero
 *   outside the grid), a quadratic sponge eta over the nb outermost cells of
 *   each face, m = slowness^2 (s^2/m^2).  For n = 0..nt-1:
 *     u^{n+1} = [2 m u^n - (m - eta dt/2) u^{n-1}
 *                + dt^2 (L u^n + Ps^T q[n])] / (m + eta dt/2),
 *     d[n]    = Pr u^{n+1},
 *   with u^{-1} = u^0 = 0.  The adjoint runs the same recursion backwards in
 *   time, driven by Pr^T res[n], giving lam^n (n = nt-1..0) with
 *   lam^{nt} = lam^{nt+1} = 0.  The exact gradient of
 *   J = 1/2 sum_n |d[n] - d_obs[n]|^2 is -sum_n u_tt^n lam^n with
 *   u_tt^n = (u^{n+1} - 2 u^n + u^{n-1}) / dt^2; probe row n of Z pairs with
 *   step n in both sweeps.
 *
 * Conventions for every entry point:
 *   - Arrays are C order; a field is [nz][ny][nx] (x fastest, ny = 1 in 2D),
 *     N = nz*ny*nx cells; traces are [nt][npoints]; Z is [nt][r].
 *   - Compressed fields (Ubar, Vbar: r rows of N cells) are tile-major:
 *     element (i, x) sits at ((x / 32) * r + i) * 32 + x % 32, in a buffer of
 *     r * Npad elements, Npad = N rounded up to a multiple of 32 (padding
 *     cells hold zeros).  One 32-cell tile's r x 32 block is contiguous, which
 *     is what the probe GEMM streams.  rtm_bar_to_rows converts to [r][N].
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory read during the call only.
 *   - Field-typed arrays (m, q, d, res, Ubar, Vbar, image, grad) have the
 *     plan's field dtype: double for RTM_F64 plans, float for RTM_F32 plans.
 *   - Positions are host double [n][3] = (z, y, x) in grid-index units, inside
 *     [0, n_axis - 1]; off-grid points use multilinear weights and injection
 *     is the exact transpose of sampling.  In 2D the y component is ignored.
 *   - Calls are ordered on `stream` and return before the GPU finishes,
 *     except that a call taking positions first uploads its point tables into
 *     `work` and waits for that copy (host memory is then free to reuse).
 *   - The library allocates no device memory: all scratch lives in `work`
 *     (size from rtm_plan_workspace_bytes).  One workspace serves one call at
 *     a time; calls on different streams need different workspaces.
 *   - Errors are returned before any launch; on error nothing is written.
 *     No exception crosses the ABI.
 */
#ifndef RTM_H
#define RTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *rtm_stream; /* a hipStream_t; NULL = default stream */

typedef enum {
  RTM_OK = 0,
  RTM_E_ARG = 1,         /* NULL pointer, non-positive size or bad enum */
  RTM_E_SHAPE = 2,       /* inconsistent or too large grid / counts */
  RTM_E_DTYPE = 3,       /* unsupported dtype combination */
  RTM_E_CFL = 4,         /* dt * c_max / h above the stability bound */
  RTM_E_WORKSPACE = 5,   /* work buffer smaller than required */
  RTM_E_HIP = 6,         /* a HIP runtime call failed */
  RTM_E_UNSUPPORTED = 7, /* valid request the library does not implement */
  RTM_E_POINTS = 8,      /* a source / receiver position outside the grid */
  RTM_E_NONFINITE = 9    /* (rtm_stream_status) a sweep met a non-finite value */
} rtm_status;

typedef enum {
  RTM_F64 = 0,    /* double */
  RTM_F32 = 1,    /* float */
  RTM_BF16 = 2,   /* probe operand: bfloat16, round to nearest even */
  RTM_BF16X2 = 3, /* probe operand: bfloat16 hi + bfloat16 lo split (16-bit mantissa) */
  RTM_I8 = 4,     /* probe matrix entries +-1 stored as int8 */
  RTM_F16S = 5    /* probe operand: float16 after a power-of-two scale shared by
                     each 16-step chunk of a 32-cell tile (its largest magnitude
                     mapped below 2^15), one MFMA per chunk; +-1 probes exact */
} rtm_dtype;

typedef enum {
  RTM_PROBE_U = 0,  /* forward sweep compresses u^n           */
  RTM_PROBE_UTT = 1 /* forward sweep compresses u_tt^n (Eq. 2) */
} rtm_probe_field;

typedef struct {
  int32_t ndim;         /* 2 or 3 */
  int64_t nz, ny, nx;   /* computational grid including damping cells; ny = 1 if ndim = 2 */
  double h;             /* grid spacing (m), equal on every axis */
  double dt;            /* time step (s) */
  int32_t nt;           /* number of time steps */
  int32_t nb;           /* damping cells per face (0 = no sponge) */
  double c_ref;         /* velocity in the sponge formula (m/s) */
  double R;             /* nominal sponge reflection coefficient, 0 < R < 1 */
  double c_max;         /* largest velocity in m, for the CFL check (m/s) */
  rtm_dtype field_dtype;/* RTM_F64 or RTM_F32: fields, model, traces, outputs */
  rtm_dtype probe_dtype;/* GEMM operand type: RTM_F64 (F64 fields), RTM_F32,
                           RTM_BF16 or RTM_F16S (F32 fields; Z RTM_I8) or
                           RTM_BF16X2 (F32 fields; Z RTM_I8, or RTM_F32 for
                           real probes) */
  int32_t r;            /* number of probe vectors, 1..1024 */
  int32_t k_block;      /* time steps per probe-GEMM block, 1..256 */
  int32_t nsrc;         /* number of source points per call (>= 0) */
  int32_t nrec;         /* number of receiver points per call (>= 0) */
} rtm_desc;

typedef struct rtm_plan rtm_plan;

/* Validates `desc` (shapes, dtypes, CFL: dt*c_max/h <= 2/sqrt(ndim*S) with S
 * the Nyquist symbol of the 8th-order weights) and creates a host-only plan.
 * No HIP call is made.  Returns RTM_OK and sets *plan, or an error. */
rtm_status rtm_plan_create(const rtm_desc *desc, rtm_plan **plan);
void rtm_plan_destroy(rtm_plan *plan);
/* Bytes of device workspace the plan's entry points need (256-byte aligned). */
rtm_status rtm_plan_workspace_bytes(const rtm_plan *plan, size_t *bytes);
/* The CFL bound 2/sqrt(ndim*S) the plan was checked against. */
double rtm_cfl_bound(int32_t ndim);
const char *rtm_status_str(rtm_status s);
/* Tuning hooks, process wide: stencil kernel of the sweeps.  -1 automatic
 * (LDS-tiled 64 x 16 for F32 3D grids, else one thread per cell), 0 one
 * thread per cell, 1..13 LDS-tiled z-marching variants (3D; x-width x y-rows):
 * 1: 64x16, 2: 64x32, 3: 64x16 with 512 threads, 4: 64x16 with 128 threads,
 * 5: 32x32, 6: 128x8, 7: as 1 and 8: as 2 with non-temporal streaming loads
 * and stores, 9: 64x32 with 512 threads, 10: 64x32 with 1024 threads,
 * 11: as 3 (all three non-temporal), 12: as 7 and 13: as 9 with the x/y halo
 * of a plane loaded four planes ahead, with the column fronts.  Every choice
 * gives bitwise-identical levels.  Batched shots run the 64x16 variants 3,
 * 11, 7 or 12 (8..10 select 7, 13 selects 12, the others 1).
 * rtm_set_stencil_blocks: the tiled acoustic kernels split z into the fewest
 * chunks (of at least 16 planes) that give a launch this many workgroups of
 * 256 threads' worth (default 2048; a 512 thread shape aims at half as
 * many); a batch's tile table (made by rtm_batch_create) aims at twice as
 * many.  The TTI kernels have their own targets (rtm_set_tti_blocks). */
void rtm_set_stencil_variant(int variant);
void rtm_set_stencil_blocks(int32_t blocks);
/* Tuning hook, process wide: with on != 0 (default) the tiled stencil of the
 * sweeps (single shot and batched) marches each z-chunk upwards on even steps
 * and downwards on odd ones, so a step begins on the planes the previous step
 * touched last; 0 marches upwards always.  Bitwise-identical results. */
void rtm_set_stencil_alternate(int32_t on);
/* Tuning hook, process wide: with on != 0 (default) the fast probe-GEMM
 * kernels read and write the compressed fields with the non-temporal hint
 * (each byte is touched once per block); 0 uses ordinary loads and stores.
 * Same results. */
void rtm_set_probe_nt(int32_t on);
/* Tuning hook, process wide: the workgroups (4 waves, one 32-cell tile per
 * wave at a time) of one probe-GEMM launch, for the kernels that update a
 * compressed field in place (forward, unfused adjoint) and for the fused
 * adjoint imaging kernel.  -1 (default, automatic): update kernels of +-1
 * probes and blocks of at most 32 steps take one workgroup per four tiles
 * (no stride), those of longer blocks in acoustic sweeps take tiles in order
 * from a work-queue counter in the workspace; the fused kernel, real probes
 * and longer blocks elsewhere are sized so that each wave strides over 48
 * tiles (6 per 16 steps of the block for update kernels), with at least 2048
 * workgroups (or one per four tiles on small grids).  -2: work queue where
 * the sweep has a counter; 0: no stride; > 0: at most that many workgroups,
 * striding.  Same results (every tile's arithmetic is the same). */
void rtm_set_probe_grid(int32_t max_workgroups_update, int32_t max_workgroups_fused);
/* Tuning hook, process wide: with on != 0, fwi_gradient captures its launch
 * sequence (everything after the point-table upload) into a HIP graph the
 * first time it sees a set of arguments (plan, pointers, point counts,
 * stream, kernel choices) and replays that graph on later calls with the
 * same set (default 0: launches one by one).  Capture and replay run on an
 * internal non-blocking stream of the device, ordered after `stream`'s
 * earlier work and before its later work by events.  Up to 8 graphs are
 * kept, the oldest dropped; results equal the eager launches bit for bit. */
void rtm_set_graph(int32_t on);
/* Autotuner and race check for the stencil: runs one step of every variant
 * (0..13 in 3D, 0 in 2D) from the same pattern levels in the ring of `work`,
 * counts elements that differ bitwise from variant 0 in either z-marching
 * direction (mismatch[v]), times
 * `steps` launches of each (us[v], microseconds per launch; us and mismatch
 * may be NULL or hold 14 entries) and returns in *best the fastest variant
 * with no mismatch.  It does not change the current variant.  Needs
 * k_block >= 2; synchronises `stream`. */
rtm_status rtm_autotune_stencil(const rtm_plan *plan, const void *m, void *work,
                                size_t work_bytes, int32_t steps, int32_t *best, float *us,
                                int64_t *mismatch, rtm_stream stream);
/* Kernel timing, process wide and off by default.  With stride > 0 the
 * sweeps record HIP events on their own stream around every stride-th
 * stencil launch (every stride-th TTI step, all of its kernels) and around
 * every probe-GEMM and image launch (0 turns it off).
 * rtm_profile_read(kind, ...) waits for the recorded events of one kind
 * (0 stencil, 1 forward probe GEMM, 2 image, 3 adjoint probe GEMM, 4 TTI
 * forward step, 5 TTI transpose step), returns their summed duration in ms
 * and their count, and forgets them. */
void rtm_profile_enable(int32_t stride);
rtm_status rtm_profile_read(int32_t kind, double *total_ms, int64_t *count);
/* Reference for the roofline figures: a streaming device-to-device copy of
 * `bytes` (a multiple of 16; src and dst device, 16-byte aligned, not
 * overlapping) by 16-byte vectors, stream ordered.  Its bytes read + written
 * over its time is the HBM rate a read-once / write-once kernel reaches.
 * NULL or misaligned -> RTM_E_ARG. */
rtm_status rtm_device_copy(const void *src, void *dst, size_t bytes, rtm_stream stream);
/* Message of the last HIP failure seen by this thread (empty if none). */
const char *rtm_last_error(void);

/* Device-side status of the last sweeping call on this workspace (any of the
 * forward / adjoint / gradient / sketch calls, acoustic or TTI, single shot):
 * each such call clears a watch word in `work` once its points are validated,
 * and sets it when the final wavefield level(s) of a sweep, the gradient or
 * image it returns, or the misfit holds a NaN or an infinity (a NaN or Inf in
 * m, the wavelet, the data or the anisotropy, or a blow-up, spreads to
 * these).  Synchronizes `stream`, then returns RTM_OK or RTM_E_NONFINITE;
 * the word is left as it is.  work: the device workspace of the call (256-byte
 * aligned); NULL plan or work -> RTM_E_ARG.  The batched calls have their own
 * watch word (rtm_batch_stream_status). */
rtm_status rtm_stream_status(const rtm_plan *plan, const void *work, rtm_stream stream);

/* Forward sweep with on-the-fly probing (Eq. 3, Ubar = Z^T u_tt or Z^T u).
 *   m        device [N]           slowness squared
 *   src_pos  host   [nsrc][3]
 *   q        device [nt][nsrc]    injected as is (a point source of signature
 *                                 w is q = w / h^ndim)
 *   rec_pos  host   [nrec][3]
 *   d_pred   device [nt][nrec]    d[n] = Pr u^{n+1}; may be NULL
 *   Z        device [nt][r]       dtype z_dtype: RTM_I8 (+-1) on every path;
 *                                 real probes as RTM_F32 on the BF16X2 path
 *                                 (split into bf16 hi + lo) or in the field
 *                                 dtype on the F32 / F64 paths
 *   Ubar     device [r*Npad]      tile-major, overwritten
 *   final_state device [2][N]     u^{nt}, u^{nt-1}; may be NULL
 */
rtm_status rtm_forward_probe(const rtm_plan *plan, const void *m, const double *src_pos,
                             const void *q, const double *rec_pos, void *d_pred,
                             const void *Z, rtm_dtype z_dtype, rtm_probe_field what,
                             void *Ubar, void *final_state, void *work, size_t work_bytes,
                             rtm_stream stream);

/* The forward sweep of rtm_forward_probe over steps n_begin .. n_end - 1 only
 * (checkpoint / resume: the state (u^n, u^{n-1}) plus the partial Ubar is a
 * complete checkpoint, since Ubar is a sum over steps).
 *   0 <= n_begin < n_end <= nt; n_begin a multiple of k_block, n_end a
 *     multiple of k_block or nt (else RTM_E_ARG), so the probe blocks are
 *     those of the whole sweep and a run split into ranges equals the
 *     uninterrupted run bit for bit
 *   state_in  device [2][N]: u^{n_begin}, u^{n_begin - 1} (the state_out of
 *             the previous range); required exactly when n_begin > 0
 *   state_out device [2][N] or NULL: u^{n_end}, u^{n_end - 1}
 *   Ubar      as rtm_forward_probe, overwritten when n_begin = 0 and
 *             accumulated into otherwise
 *   d_pred    rows n_begin .. n_end - 1 of [nt][nrec] written, others kept
 * Other arguments as rtm_forward_probe. */
rtm_status rtm_forward_probe_range(const rtm_plan *plan, const void *m, const double *src_pos,
                                   const void *q, const double *rec_pos, void *d_pred,
                                   const void *Z, rtm_dtype z_dtype, rtm_probe_field what,
                                   void *Ubar, int32_t n_begin, int32_t n_end,
                                   const void *state_in, void *state_out, void *work,
                                   size_t work_bytes, rtm_stream stream);

/* Adjoint (time-reversed) sweep with probing: Vbar = Z^T lam, row n of Z
 * paired with lam^n.
 *   rec_pos host [nrec][3], res device [nt][nrec] (the adjoint source)
 *   src_pos host [nsrc][3] and qadj device [nt][nsrc]: qadj[n] = Ps lam^n,
 *           the adjoint of the map q -> d_pred; both may be NULL
 *   Vbar    device [r*Npad] tile-major, overwritten; may be NULL together with Z
 */
rtm_status rtm_adjoint_probe(const rtm_plan *plan, const void *m, const double *rec_pos,
                             const void *res, const double *src_pos, void *qadj,
                             const void *Z, rtm_dtype z_dtype, void *Vbar, void *work,
                             size_t work_bytes, rtm_stream stream);

/* Adjoint sweep with the probed imaging condition folded into its probe
 * blocks (BF16 / BF16X2 / F16S plans): image[x] = scale * sum_i Ubar[i][x] Vbar[i][x]
 * with Vbar = Z^T lam accumulated block by block and never stored (by
 * linearity the same image as rtm_adjoint_probe + rtm_image, summed in float).
 *   Ubar device [r*Npad] tile-major (from rtm_forward_probe), image device [N]. */
rtm_status rtm_adjoint_image(const rtm_plan *plan, const void *m, const double *rec_pos,
                             const void *res, const void *Z, rtm_dtype z_dtype, const void *Ubar,
                             double scale, void *image, void *work, size_t work_bytes,
                             rtm_stream stream);

/* Probed imaging condition (Eq. 3): image[x] = scale * sum_i Ubar[i][x] Vbar[i][x],
 * summed in double.  scale = 1/r for the image, -1/r for the gradient. */
rtm_status rtm_image(const rtm_plan *plan, const void *Ubar, const void *Vbar, double scale,
                     void *image, rtm_stream stream);

/* Residual and misfit of predicted data (the adjoint source of Eq. 2's
 * gradient): resid = d_pred - d_obs and misfit[0] = 1/2 sum resid^2, the sum
 * in double in a fixed order (deterministic).  d_pred, d_obs, resid device
 * [nt][nrec] field dtype (resid may be d_pred itself); misfit device double
 * [1]; work as for the sweeps (its reduction partials are used). */
rtm_status rtm_residual(const rtm_plan *plan, const void *d_pred, const void *d_obs, void *resid,
                        double *misfit, void *work, size_t work_bytes, rtm_stream stream);

/* Probed FWI gradient of J = 1/2 sum |d_pred - d_obs|^2 (Eq. 2 estimated by
 * Eq. 3): forward probing u_tt, residual, adjoint probing, image with scale
 * -1/r.  Ubar, Vbar device [r*Npad] (tile-major) and resid device [nt][nrec] are outputs
 * (resid = d_pred - d_obs); grad device [N]; misfit device double [1].
 * Vbar may be NULL on the BF16 / BF16X2 / F16S paths: the adjoint sweep then folds
 * the imaging condition into its probe blocks (grad += -1/r sum_i Ubar[i]
 * (Z_b^T Lambda_b)[i], equal to the image of Eq. 3 by linearity) and Vbar is
 * never stored; the sum over blocks is then in float, not double. */
rtm_status fwi_gradient(const rtm_plan *plan, const void *m, const double *src_pos,
                        const void *q, const double *rec_pos, const void *d_obs,
                        const void *Z, rtm_dtype z_dtype, void *Ubar, void *Vbar,
                        void *resid, void *grad, double *misfit, void *work,
                        size_t work_bytes, rtm_stream stream);

/* Subsurface-offset image volume (Eq. 4) for horizontal offsets along x:
 *   gathers[h + nh][x] = scale * sum_f sum_i Ubar_f[i][x + h] Vbar_f[i][x - h],
 * h = -nh .. nh, with x + h and x - h moved along the x axis of the cell's
 * row and zero where either leaves it; h = 0 is the rtm_image sum (here
 * accumulated in the field dtype, in another order, so equal to rounding).
 *   Ubar, Vbar device tile-major, nfield (1, or 2 for the TTI p and q
 *              fields) compressed fields of r * Npad elements each, the
 *              second field right after the first; read only
 *   gathers    device [2 nh + 1][N] field dtype, overwritten; must not
 *              overlap Ubar or Vbar
 *   scale      1/r gives Eq. 4
 * FP32 runs on the matrix cores (v_mfma_f32_16x16x4f32: FP32 products and
 * sums), FP64 on the vector ALUs.
 * Errors: NULL pointer or nfield not 1 / 2 -> RTM_E_ARG; nh outside 0..64,
 * or FP32 fields with (nx / 32 + 2) * r * 128 >= 2^31 (a row's fields are
 * addressed with 32-bit offsets) -> RTM_E_UNSUPPORTED; a failed launch ->
 * RTM_E_HIP.  Stream-ordered; no workspace. */
rtm_status rtm_offset_gathers(const rtm_plan *plan, const void *Ubar, const void *Vbar,
                              int32_t nfield, int32_t nh, double scale, void *gathers,
                              rtm_stream stream);

/* Range-finder probes (Section "Randomized trace estimation": probing vectors
 * Q from a partial QR factorization of A Z with Z a Rademacher +-1 matrix).
 * A is read as the forward history H [nt][N] of u_tt and Z as a sign matrix
 * Omega [N][r] in space:  Y = H Omega  [nt][r],  Q = orthonormal columns of Y,
 * and the gradient is Eq. 3 with Z = Q and scale -1 (Q Q^T is a projector;
 * there is no 1/r).  Omega[x][i] = 1 - 2 b with b the bit i % 64 of word
 * i / 64 of the Philox4x64-10 block (Salmon et al., SC 2011) with key
 * (seed, 0) at counter (x + 1, 0, 0, 0), x the flat cell index; it is
 * regenerated in the kernels, never stored.  Limits: r <= 256,
 * k_block <= 128, k_block * r <= 8192, and for FP32 fields
 * ceil(k_block / 32) * ceil(r / 32) <= 8 (else RTM_E_UNSUPPORTED).  All three
 * calls need `work` of rtm_rf_workspace_bytes (the plan workspace plus sketch
 * scratch).
 * rtm_sketch:         forward sweep (no data, no probing) that writes
 *                     Y  device [nt][r] FP64 (overwritten).
 * rtm_orthonormalize: Q  device [nt][r] field dtype (overwritten) from Y by
 *                     Gram-Schmidt applied twice in FP64; a column whose
 *                     remainder falls below 1e-12 of its norm is zero.
 * fwi_gradient_rf:    sketch, orthonormalize into Q, then the probed gradient
 *                     of fwi_gradient with Z = Q and scale -1 (Ubar, Vbar,
 *                     resid, grad, misfit as there).  The probes are real: the
 *                     plan's probe dtype is BF16X2 (Q split into bf16 hi + lo
 *                     on MFMA; Vbar NULL selects fused imaging) or equals its
 *                     field dtype (F32 / F64 FMA path, Vbar required). */
rtm_status rtm_rf_workspace_bytes(const rtm_plan *plan, size_t *bytes);
rtm_status rtm_sketch(const rtm_plan *plan, const void *m, const double *src_pos, const void *q,
                      uint64_t seed, double *Y, void *work, size_t work_bytes,
                      rtm_stream stream);
rtm_status rtm_orthonormalize(const rtm_plan *plan, const double *Y, void *Q, void *work,
                              size_t work_bytes, rtm_stream stream);
rtm_status fwi_gradient_rf(const rtm_plan *plan, const void *m, const double *src_pos,
                           const void *q, const double *rec_pos, const void *d_obs,
                           uint64_t seed, void *Q, void *Ubar, void *Vbar, void *resid,
                           void *grad, double *misfit, void *work, size_t work_bytes,
                           rtm_stream stream);

/* Exact gradient of the same misfit (Eq. 2, full zero-lag correlation
 * -sum_n u_tt^n lam^n), the comparator of the probed estimate.  The forward
 * history is not stored: uniform checkpointing keeps (u^{jc}, u^{jc-1}) every
 * c = checkpoint_every steps (0: c = ceil(sqrt(2 nt))), and the adjoint sweep
 * recomputes each c-step segment from its checkpoint, keeping that segment's
 * u_tt (c levels) for the correlation.  Cost: two forward sweeps and one
 * adjoint; memory (3 + 2 ceil(nt/c) + c) levels on top of the probed
 * workspace, from rtm_exact_workspace_bytes.  resid [nt][nrec], grad [N],
 * misfit device double [1] as in fwi_gradient. */
rtm_status rtm_exact_workspace_bytes(const rtm_plan *plan, int32_t checkpoint_every,
                                     size_t *bytes);
/* Tuning hook, process wide: 1 (default) lets fwi_gradient_exact fold the
 * u_tt store and the correlation into the stencil (3D F32 tiled grids), 0
 * runs them as separate passes.  Results agree to rounding at the injected
 * cells. */
void rtm_set_exact_fused(int32_t on);
/* Tuning hook, process wide: tile shape of the tiled TTI step kernels, as
 * rows of 64 columns for the in-plane pass / the z-marching pass: 1 = 8 / 8,
 * 2 = 4 / 4, 3 = 8 / 4; 4 and 5: as 3 for the transpose step, and the forward
 * step as one fused kernel of 4 or 8 rows; 6: both steps as one fused
 * kernel each (4 rows); 7: both fused, the forward step on 4 rows and the
 * transpose step on 8 rows; 8: both fused on 8 rows; 9 and 10: as 7 with
 * the forward step keeping its planes in an LDS ring (p and q read once per
 * step), on 4 and 8 rows; 11 and 12: as 9 with the transpose step keeping
 * its halo cells' values from the lead plane in register queues (no second
 * load), on 8 and 4 rows; 13, 14 and 15: as 11 with those queues in a
 * per-thread LDS ring and 1, 2 or 3 planes per loop trip; 16: as 15 with
 * the forward step carrying two planes per loop trip; 17: as 16 with three
 * planes per trip and each cell's own values loaded in its own iteration;
 * 18: as 17 with one workgroup barrier per plane in the transpose step (each
 * wave forms its own row's x-halo of D_y (n_x n_y w), the lead plane's LDS
 * fields double buffered); 19, 20 and 21 (default): as 18 with the
 * transpose's p equation summed as one second difference per axis of
 * (1 - n_a^2) w1 (equal to the other forms up to rounding) and 3, 4 or 6
 * planes per loop trip; other values select 21.
 * rtm_set_stencil_variant(0) forces the one-thread-per-cell TTI kernels
 * instead.  Results agree to rounding. */
void rtm_set_tti_shape(int32_t shape);
/* Tuning hook, process wide: the tiled TTI kernels split z into the fewest
 * chunks (of at least 16 planes) that give a launch this many workgroups,
 * for the forward step and for the transpose step (<= 0: the defaults, 2800
 * and 1750). */
void rtm_set_tti_blocks(int32_t forward, int32_t transpose);
rtm_status fwi_gradient_exact(const rtm_plan *plan, const void *m, const double *src_pos,
                              const void *q, const double *rec_pos, const void *d_obs,
                              int32_t checkpoint_every, void *resid, void *grad, double *misfit,
                              void *work, size_t work_bytes, rtm_stream stream);

/* Pseudo-acoustic TTI (3D plans).  The paper images a TTI model (Section
 * "2007 BP TTI") without printing its equations; this library uses the
 * coupled system
 *   m p_tt = (1+2 eps) H0 p + sqrt(1+2 delta) Hz q
 *   m q_tt = sqrt(1+2 delta) H0 p + Hz q
 *   Hz = sum_a n_a^2 D_aa + sum_{a != b} n_a n_b D_a D_b,  H0 = L - Hz,
 * n = (sin theta cos phi, sin theta sin phi, cos theta) in (x, y, z), D_a and
 * D_aa 8th-order first and second differences, the damped leapfrog of the
 * acoustic case on both fields; the adjoint is its exact transpose (the
 * coefficients move inside the derivatives).  Sources inject into p and q,
 * receivers record p.  The gradient is -sum_n (p_tt lam_p + q_tt lam_q), so
 * both fields are compressed: Ubar / Vbar are [2][r*Npad] (p then q, each
 * tile-major).  aniso: device [4][N] (eps, delta, theta, phi in radians) of
 * the field dtype.
 * Stability screen: before it writes anything, each TTI call reads m, eps and
 * delta once on the device and synchronizes `stream`.  With the coefficients
 * frozen at a cell the operator's symbol is [[c1, c2], [c2, 1]] diag(h0, hz)
 * (c1 = 1 + 2 eps, c2 = sqrt(1 + 2 delta), h0, hz >= 0 the symbols of -H0,
 * -Hz, h0 + hz that of -L); for delta <= eps its eigenvalues are real and at
 * most max(1, c1) (h0 + hz), so the acoustic CFL bound holds with velocity
 * v sqrt(max(1, 1 + 2 eps)).  Hence: a cell with delta > eps, eps <= -1/2
 * or delta <= -1/2 -> RTM_E_ARG (not clipped); a plan c_max below
 * max v sqrt(max(1, 1 + 2 eps)) (1e-6 relative slack) -> RTM_E_CFL.
 * rtm_tti_spectral_radius measures the discrete operator's actual spectral
 * radius on a model.
 *   rtm_tti_adjoint_probe: qadj[n] = Ps (lam_p + lam_q)^n (adjoint of q -> d).
 *   fwi_gradient_tti: Vbar may be NULL on the MFMA probe paths (fused imaging). */
rtm_status rtm_tti_workspace_bytes(const rtm_plan *plan, size_t *bytes);
rtm_status rtm_tti_forward_probe(const rtm_plan *plan, const void *m, const void *aniso,
                                 const double *src_pos, const void *q, const double *rec_pos,
                                 void *d_pred, const void *Z, rtm_dtype z_dtype, void *Ubar,
                                 void *work, size_t work_bytes, rtm_stream stream);
rtm_status rtm_tti_adjoint_probe(const rtm_plan *plan, const void *m, const void *aniso,
                                 const double *rec_pos, const void *res, const double *src_pos,
                                 void *qadj, const void *Z, rtm_dtype z_dtype, void *Vbar,
                                 void *work, size_t work_bytes, rtm_stream stream);
/* Spectral radius of m^{-1} A, A the discrete TTI operator above without the
 * sponge, on this plan's grid and the given model, by power iteration: from a
 * seeded pseudo-random unit vector (p, q), `iters` times w = m^{-1} A v (one
 * forward step with a zero previous level: w = (next - 2 v) / dt^2),
 * v = w / |w|; *rho (host) = |w| of the last iteration, which approaches the
 * spectral radius from below as iters grows (real spectrum for delta <= eps).
 * The leapfrog is stable for dt <= 2 / sqrt(rho).  The screen of the TTI
 * calls is not applied (a rejected model can be measured).  work: as the
 * other TTI calls (rtm_tti_workspace_bytes); overwrites its rings; iters in
 * 1..10^6, else RTM_E_ARG.  Synchronizes `stream`. */
rtm_status rtm_tti_spectral_radius(const rtm_plan *plan, const void *m, const void *aniso,
                                   int32_t iters, uint64_t seed, double *rho, void *work,
                                   size_t work_bytes, rtm_stream stream);
rtm_status fwi_gradient_tti(const rtm_plan *plan, const void *m, const void *aniso,
                            const double *src_pos, const void *q, const double *rec_pos,
                            const void *d_obs, const void *Z, rtm_dtype z_dtype, void *Ubar,
                            void *Vbar, void *resid, void *grad, double *misfit, void *work,
                            size_t work_bytes, rtm_stream stream);

/* Batched shots (3D, F32 fields, BF16 / BF16X2 / F16S probes).  Each descriptor is
 * one shot's sub-domain window (its own nz, ny, nx, nb, c_ref, c_max, nsrc,
 * nrec); nt, dt, h, r, k_block and the probe dtype must agree.  One launch
 * per time step advances every shot (a tile table spans all windows), one
 * launch injects and one samples for all shots; the probe GEMMs run per shot
 * every k_block steps.  fwi_gradient_batched computes every shot's probed
 * gradient (fused imaging, no Vbar) and misfit[i] (device double [nshots]).
 * use_graph != 0 captures the whole launch sequence into a HIP graph on the
 * first call and replays it while the pointers, positions and stencil variant
 * stay the same (the batch object caches it; not thread safe).
 * Stacking (the image / gradient summed over sources, each shot with its own
 * probe matrix Z): shots with the same grid may pass the same `grad`
 * pointer; that buffer then receives the sum of their gradients, added probe
 * block by probe block in shot order (deterministic).  Shots that share a
 * `grad` but not a grid, or a `grad` that is also another array of a shot,
 * -> RTM_E_ARG.  Each call keeps a non-finite watch word in `work` (cleared
 * at its start; set when a shot's last adjoint level, gradient or misfit is a
 * NaN or an infinity), read by rtm_batch_stream_status. */
typedef struct rtm_batch rtm_batch;
typedef struct {
  const void *m;          /* device [N_i] slowness squared */
  const double *src_pos;  /* host [nsrc_i][3] */
  const void *q;          /* device [nt][nsrc_i] */
  const double *rec_pos;  /* host [nrec_i][3] */
  const void *d_obs;      /* device [nt][nrec_i] */
  const void *Z;          /* device [nt][r] int8 +-1 */
  void *Ubar;             /* device [r*Npad_i] tile-major, output */
  void *resid;            /* device [nt][nrec_i], output */
  void *grad;             /* device [N_i], output */
} rtm_shot_io;
rtm_status rtm_batch_create(const rtm_desc *shots, int32_t nshots, rtm_batch **batch);
void rtm_batch_destroy(rtm_batch *batch);
rtm_status rtm_batch_workspace_bytes(const rtm_batch *batch, size_t *bytes);
rtm_status fwi_gradient_batched(rtm_batch *batch, const rtm_shot_io *io, double *misfit,
                                int32_t use_graph, void *work, size_t work_bytes,
                                rtm_stream stream);
/* The batched counterpart of rtm_stream_status: synchronizes `stream`, then
 * returns RTM_E_NONFINITE if the last fwi_gradient_batched call on `work`
 * met a non-finite value, else RTM_OK.  NULL or misaligned -> RTM_E_ARG. */
rtm_status rtm_batch_stream_status(const rtm_batch *batch, const void *work, rtm_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the probed
 * gradient of fwi_gradient, same arguments and results, with the workspace
 * taken from a static device array of RTM_NOALLOC_SCRATCH_BYTES (256 MiB)
 * instead of `work`.  The library holds that array on every GPU it runs on,
 * from the first call there until the process ends; it calls no hipMalloc,
 * hipFree or allocating library routine.
 *   plan  a plan with rtm_plan_workspace_bytes <= RTM_NOALLOC_SCRATCH_BYTES,
 *         else RTM_E_WORKSPACE before any HIP call (the message gives both
 *         sizes)
 *   other arguments and errors as fwi_gradient; the current HIP device is
 *         the one that runs the call
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call initialises what it reads).  Calls that overlap
 * in time on one GPU (different streams or threads) race and give wrong
 * results: order them, e.g. on one stream.  The array holds the call's
 * non-finite watch word, so rtm_stream_status does not apply. */
#define RTM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
rtm_status fwi_gradient_noalloc(const rtm_plan *plan, const void *m, const double *src_pos,
                                const void *q, const double *rec_pos, const void *d_obs,
                                const void *Z, rtm_dtype z_dtype, void *Ubar, void *Vbar,
                                void *resid, void *grad, double *misfit, rtm_stream stream);

/* Converts a tile-major compressed field (device [r*Npad]) to rows (device
 * [r][N], caller-owned): rows[i][x] = bar[((x/32)*r + i)*32 + x%32]. */
rtm_status rtm_bar_to_rows(const rtm_plan *plan, const void *bar, void *rows, rtm_stream stream);

/* Double-precision inner product of two device arrays of the plan's field
 * dtype: out[0] = sum_i a[i] b[i] (device double), deterministic order.
 * Used for the adjoint test and for misfit / gradient norms. */
rtm_status rtm_dot(const rtm_plan *plan, const void *a, const void *b, int64_t n,
                   double *out, void *work, size_t work_bytes, rtm_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* RTM_H */
