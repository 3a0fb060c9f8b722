// Host side of librtm: plan validation, workspace layout, point tables and
// the sequencing of the forward / adjoint sweeps (include/rtm.h).
//
// Sweep structure (both directions).  The wavefield lives in a ring of
// R = k_block + 2 levels in the workspace.  Sweep step s (s = 0..nt-1; the
// time step is n = s forward, n = nt-1-s adjoint) reads levels s and s-1 and
// writes level s+1; level j sits in slot (j+1) mod R, levels -1 and 0 are zero.
// Per step: stencil kernel, injection of the step's point values into level
// s+1, sampling of level s+1.  After every k_block steps (and after the last)
// one probe-GEMM adds the block's k probed levels, weighted by the matching
// rows of Z, into Ubar / Vbar - so the compressed history is built on the fly
// and no level older than the ring is ever needed (Eq. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rtm.h"
#include "rtm_internal.h"

using namespace rtm;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
static int g_stencil_variant = -1;  // -1 auto, else kStencilSimple / a tiled variant id
static int g_stencil_blocks = 2048; // tiled stencil: split z until this many workgroups
// tiled TTI kernels' z-split targets (forward, transpose).  At 300 x 400 x 400
// the forward step (700 tiles, three workgroups per CU) is fastest with 4
// chunks (650 us; 1 chunk 684-691 us), the transpose (350 tiles, one
// workgroup per CU) with 5 (1110 us; 8 chunks 1129-1133 us, 4 chunks 1146 us):
// chunk warm-up (8 planes each) against the last round's idle CUs
static int g_tti_blocks[2] = {2800, 1750};
static int g_exact_fused = 1;       // exact comparator: fused stencil epilogues
static int g_tti_shape = 21;        // tiled TTI tile shape (1..21)
static int g_stencil_alternate = 1; // sweeps: tiled stencil marches z up / down on alternate steps
static int g_graph = 0;             // fwi_gradient: capture and replay HIP graphs

// Opt-in kernel timing: HIP events recorded on the sweep's stream around every
// `stride`-th launch of the stencil and every probe-GEMM / image launch.
enum {
  KT_STENCIL = 0, KT_PROBE = 1, KT_IMAGE = 2, KT_PROBE_ADJ = 3, KT_TTI = 4, KT_TTI_ADJ = 5,
  KT_N = 6
};
struct TimedLaunch {
  int kind;
  hipEvent_t a, b;
};
static int g_prof_stride = 0;  // 0 = off
static std::vector<TimedLaunch> g_prof;

static void prof_begin(int kind, int step, hipStream_t st, TimedLaunch *t) {
  t->kind = -1;
  if (g_prof_stride <= 0) return;
  if ((kind == KT_STENCIL || kind == KT_TTI || kind == KT_TTI_ADJ) && step % g_prof_stride) return;
  if (hipEventCreate(&t->a) != hipSuccess) return;
  if (hipEventCreate(&t->b) != hipSuccess) {
    (void)hipEventDestroy(t->a);
    return;
  }
  t->kind = kind;
  (void)hipEventRecord(t->a, st);
}

static void prof_end(hipStream_t st, TimedLaunch *t) {
  if (t->kind < 0) return;
  (void)hipEventRecord(t->b, st);
  g_prof.push_back(*t);
}

static rtm_status fail(rtm_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

namespace rtm {
// sets the message of rtm_last_error from other translation units of the library
rtm_status note_error(rtm_status s, const char *msg) { return fail(s, "%s", msg); }
}  // namespace rtm

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(RTM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// 8th-order central second-derivative weights (Fornberg), offsets 0..4.
static const double kW[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

static double nyquist_symbol() {  // max over k of the 1D symbol times h^2
  double s = -kW[0];
  for (int j = 1; j <= 4; ++j) s -= 2.0 * kW[j] * ((j & 1) ? -1.0 : 1.0);
  return s;
}

struct Region {
  size_t off = 0, bytes = 0;
};

struct PointRegion {  // device layout of one point set's tables
  Region soff, sidx, sw, icell, ioff, ipt, iw;
  int32_t cap = 0;  // points
};

struct rtm_plan {
  rtm_desc d;
  int64_t N = 0, ld = 0;
  int64_t Npad = 0;  // N rounded up to whole 32-cell tiles (compressed-field layout)
  int R = 0;
  size_t esz = 0;
  Region ring, red, status;  // status: the non-finite watch word (uint32)
  Region queue;              // work-queue counter of the probe launches (int32)
  PointRegion src, rec;
  size_t tab_off = 0, tab_bytes = 0;
  size_t total = 0;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// the probe dtypes that run on the MFMA path, and their operand kind
static bool mfma_probe(rtm_dtype pd) {
  return pd == RTM_BF16 || pd == RTM_BF16X2 || pd == RTM_F16S;
}
static int probe_op(rtm_dtype pd) {
  return pd == RTM_BF16X2 ? OP_BF16X2 : pd == RTM_F16S ? OP_F16S : OP_BF16;
}

static void place(size_t &cur, Region &r, size_t bytes) {
  r.off = cur;
  r.bytes = bytes;
  cur = align256(cur + bytes);
}

static void place_points(size_t &cur, PointRegion &pr, int32_t n, size_t esz) {
  const size_t c = (size_t)8 * n;  // at most 8 corners per point
  pr.cap = n;
  place(cur, pr.soff, 4 * ((size_t)n + 1));
  place(cur, pr.sidx, 4 * c);
  place(cur, pr.sw, esz * c);
  place(cur, pr.icell, 4 * c);
  place(cur, pr.ioff, 4 * (c + 1));
  place(cur, pr.ipt, 4 * c);
  place(cur, pr.iw, esz * c);
}

extern "C" double rtm_cfl_bound(int32_t ndim) {
  if (ndim < 1) return 0.0;
  return 2.0 / std::sqrt((double)ndim * nyquist_symbol());
}

extern "C" const char *rtm_status_str(rtm_status s) {
  switch (s) {
    case RTM_OK: return "ok";
    case RTM_E_ARG: return "invalid argument";
    case RTM_E_SHAPE: return "invalid shape";
    case RTM_E_DTYPE: return "unsupported dtype";
    case RTM_E_CFL: return "time step violates the CFL bound";
    case RTM_E_WORKSPACE: return "workspace too small";
    case RTM_E_HIP: return "HIP runtime error";
    case RTM_E_UNSUPPORTED: return "unsupported request";
    case RTM_E_POINTS: return "point outside the grid";
    case RTM_E_NONFINITE: return "non-finite value in a wavefield or an output";
  }
  return "unknown status";
}

extern "C" const char *rtm_last_error(void) { return g_last_error.c_str(); }

extern "C" rtm_status rtm_stream_status(const rtm_plan *P, const void *work, rtm_stream stream) {
  g_last_error.clear();
  if (!P || !work) return fail(RTM_E_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(RTM_E_ARG, "work must be 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  uint32_t word = 0;
  HIP_TRY(hipMemcpyAsync(&word, static_cast<const char *>(work) + P->status.off, sizeof(word),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (word) return fail(RTM_E_NONFINITE, "a non-finite value reached a wavefield or an output");
  return RTM_OK;
}

extern "C" void rtm_set_stencil_variant(int v) {
  g_stencil_variant = (v >= -1 && v <= kStencilVariants) ? v : -1;
}

extern "C" void rtm_set_exact_fused(int32_t on) { g_exact_fused = on ? 1 : 0; }
extern "C" void rtm_set_stencil_alternate(int32_t on) { g_stencil_alternate = on ? 1 : 0; }
extern "C" void rtm_set_probe_nt(int32_t on) { set_probe_nt(on); }
extern "C" void rtm_set_probe_grid(int32_t max_workgroups_update, int32_t max_workgroups_fused) {
  set_probe_grid(max_workgroups_update, max_workgroups_fused);
}
extern "C" void rtm_set_graph(int32_t on) { g_graph = on ? 1 : 0; }

extern "C" void rtm_set_tti_shape(int32_t shape) {
  g_tti_shape = (shape >= 1 && shape <= 21) ? shape : 21;
}
extern "C" void rtm_set_tti_blocks(int32_t forward, int32_t transpose) {
  g_tti_blocks[0] = forward > 0 ? forward : 2800;
  g_tti_blocks[1] = transpose > 0 ? transpose : 1750;
}

extern "C" void rtm_set_stencil_blocks(int32_t blocks) {
  g_stencil_blocks = blocks > 0 ? blocks : 2048;
}

extern "C" void rtm_profile_enable(int32_t stride) {
  g_prof_stride = stride > 0 ? stride : 0;
}

extern "C" rtm_status rtm_profile_read(int32_t kind, double *total_ms, int64_t *count) {
  if (!total_ms || !count || kind < 0 || kind >= KT_N) return fail(RTM_E_ARG, "bad profile query");
  double tot = 0.0;
  int64_t n = 0;
  std::vector<TimedLaunch> keep;
  for (TimedLaunch &t : g_prof) {
    if (t.kind != kind) {
      keep.push_back(t);
      continue;
    }
    float ms = 0.f;
    HIP_TRY(hipEventSynchronize(t.b));
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    tot += ms;
    ++n;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  g_prof.swap(keep);
  *total_ms = tot;
  *count = n;
  return RTM_OK;
}

extern "C" rtm_status rtm_plan_create(const rtm_desc *desc, rtm_plan **out) {
  g_last_error.clear();
  if (!desc || !out) return fail(RTM_E_ARG, "desc and plan must be non-NULL");
  const rtm_desc &d = *desc;
  if (d.ndim != 2 && d.ndim != 3) return fail(RTM_E_SHAPE, "ndim must be 2 or 3 (got %d)", d.ndim);
  if (d.nz < 1 || d.ny < 1 || d.nx < 1) return fail(RTM_E_SHAPE, "grid sizes must be >= 1");
  if (d.ndim == 2 && d.ny != 1) return fail(RTM_E_SHAPE, "2D grids need ny == 1");
  if (d.nz > (1 << 30) || d.ny > (1 << 30) || d.nx > (1 << 30))
    return fail(RTM_E_SHAPE, "axis too long");
  const int64_t N = d.nz * d.ny * d.nx;
  if (N >= ((int64_t)1 << 31)) return fail(RTM_E_SHAPE, "grid has %lld cells (max 2^31-1)", (long long)N);
  if (!(d.h > 0) || !(d.dt > 0)) return fail(RTM_E_ARG, "h and dt must be positive");
  if (d.nt < 1) return fail(RTM_E_ARG, "nt must be >= 1");
  if (d.nb < 0) return fail(RTM_E_ARG, "nb must be >= 0");
  if (2 * (int64_t)d.nb >= d.nz || 2 * (int64_t)d.nb >= d.nx ||
      (d.ndim == 3 && 2 * (int64_t)d.nb >= d.ny))
    return fail(RTM_E_SHAPE, "damping layers (2 x %d) do not fit the grid", d.nb);
  if (d.nb > 0 && !(d.c_ref > 0)) return fail(RTM_E_ARG, "c_ref must be positive");
  if (d.nb > 0 && !(d.R > 0 && d.R < 1)) return fail(RTM_E_ARG, "R must be in (0, 1)");
  if (!(d.c_max > 0)) return fail(RTM_E_ARG, "c_max must be positive");
  const double courant = d.dt * d.c_max / d.h;
  if (!(courant <= rtm_cfl_bound(d.ndim)))
    return fail(RTM_E_CFL, "dt*c_max/h = %.6f exceeds the bound %.6f", courant,
                rtm_cfl_bound(d.ndim));
  if (d.field_dtype != RTM_F64 && d.field_dtype != RTM_F32)
    return fail(RTM_E_DTYPE, "field dtype must be F64 or F32");
  if (d.field_dtype == RTM_F64 && d.probe_dtype != RTM_F64)
    return fail(RTM_E_DTYPE, "F64 fields need the F64 probe path");
  if (d.field_dtype == RTM_F32 && d.probe_dtype != RTM_F32 && !mfma_probe(d.probe_dtype))
    return fail(RTM_E_DTYPE, "F32 fields need an F32, BF16, BF16X2 or F16S probe path");
  if (d.r < 1 || d.r > 1024) return fail(RTM_E_ARG, "r must be in 1..1024");
  if (d.k_block < 1 || d.k_block > 256) return fail(RTM_E_ARG, "k_block must be in 1..256");
  if (mfma_probe(d.probe_dtype)) {
    const int ks = (d.k_block + 15) / 16;
    const int ksp = ks <= 1 ? 1 : ks <= 2 ? 2 : ks <= 4 ? 4 : 8;
    if (d.k_block > 128 || ((d.r + 31) / 32) * ksp > 64)
      return fail(RTM_E_UNSUPPORTED, "the MFMA probe path needs k_block <= 128 and ceil(r/32)*ceil(k/16) <= 64");
  }
  if (d.nsrc < 0 || d.nrec < 0) return fail(RTM_E_ARG, "point counts must be >= 0");

  rtm_plan *p = new (std::nothrow) rtm_plan();
  if (!p) return fail(RTM_E_ARG, "out of host memory");
  p->d = d;
  p->N = N;
  p->ld = (N + 63) / 64 * 64;
  p->Npad = (N + 31) / 32 * 32;
  p->R = d.k_block + 2;
  p->esz = d.field_dtype == RTM_F64 ? 8 : 4;
  size_t cur = 0;
  place(cur, p->ring, (size_t)p->R * p->ld * p->esz);
  place(cur, p->red, sizeof(double) * (kReduceBlocks + 8));
  place(cur, p->status, sizeof(uint32_t));
  place(cur, p->queue, sizeof(int32_t));
  p->tab_off = cur;
  place_points(cur, p->src, d.nsrc, p->esz);
  place_points(cur, p->rec, d.nrec, p->esz);
  p->tab_bytes = cur - p->tab_off;
  p->total = cur;
  *out = p;
  return RTM_OK;
}

extern "C" void rtm_plan_destroy(rtm_plan *p) { delete p; }

extern "C" rtm_status rtm_plan_workspace_bytes(const rtm_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(RTM_E_ARG, "plan and bytes must be non-NULL");
  *bytes = p->total;
  return RTM_OK;
}

// ---------------------------------------------------------------------------
// point tables
// ---------------------------------------------------------------------------
struct HostPoints {
  std::vector<int32_t> soff, sidx, icell, ioff, ipt;
  std::vector<double> sw, iw;
};

// Multilinear weights of each point; injection entries grouped by cell
// (points in increasing order within a cell) so that the injection kernel
// sums a cell's contributions in a fixed order without atomics.
static rtm_status build_points(const rtm_plan *P, int32_t n, const double *pos, HostPoints &hp) {
  const rtm_desc &d = P->d;
  const int64_t dims[3] = {d.nz, d.ny, d.nx};
  struct Entry {
    int32_t cell, pt;
    double w;
  };
  std::vector<Entry> ent;
  ent.reserve((size_t)n * 8);
  hp.soff.assign(1, 0);
  for (int32_t p = 0; p < n; ++p) {
    int64_t base[3];
    double frac[3];
    int ncor[3];
    for (int a = 0; a < 3; ++a) {
      double v = (a == 1 && d.ndim == 2) ? 0.0 : pos[3 * (size_t)p + a];
      if (!(v >= 0.0 && v <= (double)(dims[a] - 1)))
        return fail(RTM_E_POINTS, "point %d axis %d at %g is outside [0, %lld]", p, a, v,
                    (long long)(dims[a] - 1));
      const double f = std::floor(v);
      base[a] = (int64_t)f;
      frac[a] = v - f;
      ncor[a] = frac[a] > 0.0 ? 2 : 1;
    }
    for (int iz = 0; iz < ncor[0]; ++iz)
      for (int iy = 0; iy < ncor[1]; ++iy)
        for (int ix = 0; ix < ncor[2]; ++ix) {
          const double w = (iz ? frac[0] : 1.0 - frac[0]) * (iy ? frac[1] : 1.0 - frac[1]) *
                           (ix ? frac[2] : 1.0 - frac[2]);
          const int64_t cell = ((base[0] + iz) * d.ny + (base[1] + iy)) * d.nx + (base[2] + ix);
          hp.sidx.push_back((int32_t)cell);
          hp.sw.push_back(w);
          ent.push_back({(int32_t)cell, p, w});
        }
    hp.soff.push_back((int32_t)hp.sidx.size());
  }
  std::stable_sort(ent.begin(), ent.end(),
                   [](const Entry &a, const Entry &b) { return a.cell < b.cell; });
  hp.ioff.assign(1, 0);
  for (size_t e = 0; e < ent.size(); ++e) {
    if (e == 0 || ent[e].cell != ent[e - 1].cell) {
      if (e) hp.ioff.push_back((int32_t)e);
      hp.icell.push_back(ent[e].cell);
    }
    hp.ipt.push_back(ent[e].pt);
    hp.iw.push_back(ent[e].w);
  }
  hp.ioff.push_back((int32_t)ent.size());
  if (ent.empty()) hp.ioff.assign(1, 0);
  return RTM_OK;
}

template <typename T>
static void stage_points(const rtm_plan *P, const PointRegion &pr, const HostPoints &hp,
                         std::vector<unsigned char> &host) {
  auto put = [&](const Region &r, const void *src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + (r.off - P->tab_off), src, bytes);
  };
  put(pr.soff, hp.soff.data(), 4 * hp.soff.size());
  put(pr.sidx, hp.sidx.data(), 4 * hp.sidx.size());
  std::vector<T> sw(hp.sw.begin(), hp.sw.end()), iw(hp.iw.begin(), hp.iw.end());
  put(pr.sw, sw.data(), sizeof(T) * sw.size());
  put(pr.icell, hp.icell.data(), 4 * hp.icell.size());
  put(pr.ioff, hp.ioff.data(), 4 * hp.ioff.size());
  put(pr.ipt, hp.ipt.data(), 4 * hp.ipt.size());
  put(pr.iw, iw.data(), sizeof(T) * iw.size());
}

template <typename T>
static PointTables<T> device_points(const PointRegion &pr, char *work, int32_t npts,
                                    int32_t ncell) {
  PointTables<T> t;
  t.soff = reinterpret_cast<const int32_t *>(work + pr.soff.off);
  t.sidx = reinterpret_cast<const int32_t *>(work + pr.sidx.off);
  t.sw = reinterpret_cast<const T *>(work + pr.sw.off);
  t.icell = reinterpret_cast<const int32_t *>(work + pr.icell.off);
  t.ioff = reinterpret_cast<const int32_t *>(work + pr.ioff.off);
  t.ipt = reinterpret_cast<const int32_t *>(work + pr.ipt.off);
  t.iw = reinterpret_cast<const T *>(work + pr.iw.off);
  t.npts = npts;
  t.ncell = ncell;
  return t;
}

static uint32_t *status_word(const rtm_plan *P, char *work) {
  return reinterpret_cast<uint32_t *>(work + P->status.off);
}

// Builds the tables of the given point sets and copies them into the
// workspace (stream ordered; waits for the copy so host memory can go).  Once
// the points are valid, the call's non-finite watch word is cleared: every
// sweeping call passes through here first.
template <typename T>
static rtm_status upload_points(const rtm_plan *P, char *work, hipStream_t st,
                                const double *src_pos, PointTables<T> *src_t,
                                const double *rec_pos, PointTables<T> *rec_t) {
  std::vector<unsigned char> host(P->tab_bytes, 0);
  HostPoints hs, hr;
  if (src_pos && src_t) {
    rtm_status s = build_points(P, P->d.nsrc, src_pos, hs);
    if (s) return s;
    stage_points<T>(P, P->src, hs, host);
    *src_t = device_points<T>(P->src, work, P->d.nsrc, (int32_t)hs.icell.size());
  }
  if (rec_pos && rec_t) {
    rtm_status s = build_points(P, P->d.nrec, rec_pos, hr);
    if (s) return s;
    stage_points<T>(P, P->rec, hr, host);
    *rec_t = device_points<T>(P->rec, work, P->d.nrec, (int32_t)hr.icell.size());
  }
  HIP_TRY(launch_status_clear(status_word(P, work), st));
  if (P->tab_bytes) {
    HIP_TRY(hipMemcpyAsync(work + P->tab_off, host.data(), P->tab_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return RTM_OK;
}

// ---------------------------------------------------------------------------
// sweeps
// ---------------------------------------------------------------------------
template <typename T>
static StepArgs<T> step_args(const rtm_plan *P, const T *m) {
  const rtm_desc &d = P->d;
  StepArgs<T> a{};
  a.m = m;
  a.nz = (int)d.nz;
  a.ny = (int)d.ny;
  a.nx = (int)d.nx;
  a.nb = d.nb;
  a.N = P->N;
  const double ih2 = 1.0 / (d.h * d.h);
  a.c1 = (T)(kW[1] * ih2);
  a.c2 = (T)(kW[2] * ih2);
  a.c3 = (T)(kW[3] * ih2);
  a.c4 = (T)(kW[4] * ih2);
  a.cc = (T)(d.ndim * kW[0] * ih2);
  a.dt2 = (T)(d.dt * d.dt);
  double kd = 0.0;
  if (d.nb > 0) {
    const double A = 3.0 * std::log(1.0 / d.R) / (2.0 * d.nb * d.h * d.c_ref);
    kd = A * d.dt * 0.5 / ((double)d.nb * d.nb);
  }
  a.kd = (T)kd;
  return a;
}

struct SweepIO {
  bool adjoint = false;
  const void *m = nullptr;
  const void *inj_vals = nullptr;  // [nt][n_inj]
  void *smp_out = nullptr;         // [nt][n_smp] or NULL
  const void *Z = nullptr;
  rtm_dtype zt = RTM_I8;
  int mode = PROBE_UTT;
  void *bar = nullptr;             // [r][N] or NULL
  void *final_state = nullptr;     // [2][N] or NULL: levels n_end, n_end - 1
  // step range (forward only): steps n_begin .. n_end - 1 from state_in
  // (levels n_begin, n_begin - 1; zero when NULL); bar accumulates if n_begin > 0
  int n_begin = 0, n_end = -1;
  const void *state_in = nullptr;
  // fused adjoint imaging (MFMA paths): img += scale * sum_i fuse_U[i] (Z_b^T S_b)[i]
  const void *fuse_U = nullptr;
  void *fuse_img = nullptr;
  double fuse_scale = 0.0;
  // space sketch of u_tt (range-finder probes): Y [nt][r] rows per block
  double *sketch_Y = nullptr;
  void *sketch_partial = nullptr;
  uint64_t sketch_seed = 0;
};

template <typename T>
static rtm_status run_sweep(const rtm_plan *P, const SweepIO &io, const PointTables<T> &inj,
                            const PointTables<T> &smp, char *work, hipStream_t st) {
  const rtm_desc &d = P->d;
  T *ring = reinterpret_cast<T *>(work + P->ring.off);
  auto level = [&](int j) -> T * {
    int slot = (j + 1) % P->R;
    return ring + (int64_t)slot * P->ld;
  };
  const int ndim = d.ndim;
  int variant = kStencilSimple;
  if (ndim == 3 && sizeof(T) == 4) variant = kStencilTiled;
  if (g_stencil_variant >= 0) variant = g_stencil_variant;
  StepArgs<T> a = step_args<T>(P, static_cast<const T *>(io.m));
  const int nb = io.n_begin, ne = io.n_end < 0 ? d.nt : io.n_end;
  if (io.state_in) {
    const T *si = static_cast<const T *>(io.state_in);
    HIP_TRY(launch_copy<T>(level(nb), si, P->N, st));
    HIP_TRY(launch_copy<T>(level(nb - 1), si + P->N, P->N, st));
  } else {
    HIP_TRY(launch_fill<T>(level(nb - 1), P->N, T(0), st));
    HIP_TRY(launch_fill<T>(level(nb), P->N, T(0), st));
  }
  T *bar = static_cast<T *>(io.bar);
  if (bar && nb == 0) HIP_TRY(launch_fill<T>(bar, (int64_t)d.r * P->Npad, T(0), st));
  const T *inj_vals = static_cast<const T *>(io.inj_vals);
  T *smp_out = static_cast<T *>(io.smp_out);
  int s0 = nb;
  for (int s = nb; s < ne; ++s) {
    const int n = io.adjoint ? d.nt - 1 - s : s;
    a.cur = level(s);
    a.prev = level(s - 1);
    a.next = level(s + 1);
    TimedLaunch tl;
    prof_begin(KT_STENCIL, s, st, &tl);
    HIP_TRY(launch_stencil<T>(ndim, a, variant, g_stencil_blocks, st,
                              g_stencil_alternate ? (s & 1) : 0));
    prof_end(st, &tl);
    if (inj.ncell > 0 && inj_vals)
      HIP_TRY(launch_inject<T>(a, inj, inj_vals + (int64_t)n * inj.npts, a.next, st));
    if (smp_out && smp.npts > 0)
      HIP_TRY(launch_sample<T>(smp, a.next, smp_out + (int64_t)n * smp.npts, st));
    if ((bar || io.fuse_img || io.sketch_Y) &&
        (s + 1 - s0 == d.k_block || s == d.nt - 1 || s == ne - 1)) {
      ProbeArgs<T> p{};
      p.ring = ring;
      p.ld = P->ld;
      p.R = P->R;
      p.s0 = s0;
      p.slot0 = s0 % P->R;
      p.kb = s + 1 - s0;
      p.zrow0 = io.adjoint ? d.nt - 1 - s0 : s0;
      p.zdir = io.adjoint ? -1 : 1;
      p.r = d.r;
      p.N = P->N;
      p.bar = bar;
      p.inv_dt2 = (T)(1.0 / (d.dt * d.dt));
      p.mode = io.mode;
      p.queue = reinterpret_cast<int *>(work + P->queue.off);
      if (io.sketch_Y) {
        ProbeArgs<T> ps = p;
        ps.mode = PROBE_UTT;
        HIP_TRY(launch_sketch<T>(ps, io.sketch_seed, io.sketch_partial, io.sketch_Y, st));
      }
      if (!bar && !io.fuse_img) {
        s0 = s + 1;
        continue;
      }
      TimedLaunch tp;
      prof_begin(io.adjoint ? KT_PROBE_ADJ : KT_PROBE, s, st, &tp);
      if constexpr (sizeof(T) == 4) {
        if (mfma_probe(d.probe_dtype)) {
          HIP_TRY(launch_probe_mfma(p, io.Z, io.zt == RTM_F32, probe_op(d.probe_dtype),
                                    static_cast<const float *>(io.fuse_U),
                                    static_cast<float *>(io.fuse_img), (float)io.fuse_scale, st));
        } else {
          HIP_TRY(launch_probe_vec<T>(p, io.Z, io.zt == RTM_I8, st));
        }
      } else {
        HIP_TRY(launch_probe_vec<T>(p, io.Z, io.zt == RTM_I8, st));
      }
      prof_end(st, &tp);
      s0 = s + 1;
    }
  }
  if (io.final_state) {
    T *fs = static_cast<T *>(io.final_state);
    HIP_TRY(launch_copy<T>(fs, level(ne), P->N, st));
    HIP_TRY(launch_copy<T>(fs + P->N, level(ne - 1), P->N, st));
  }
  // a field that went non-finite anywhere stays so: the last level tells
  HIP_TRY(launch_flag_nonfinite<T>(level(ne), P->N, status_word(P, work), st));
  return RTM_OK;
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
static rtm_status check_common(const rtm_plan *P, const void *m, void *work, size_t work_bytes) {
  g_last_error.clear();
  if (!P) return fail(RTM_E_ARG, "plan is NULL");
  if (!m) return fail(RTM_E_ARG, "m is NULL");
  if (!work) return fail(RTM_E_ARG, "work is NULL");
  if (work_bytes < P->total)
    return fail(RTM_E_WORKSPACE, "work has %zu bytes, the plan needs %zu", work_bytes, P->total);
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(RTM_E_ARG, "work must be 256-byte aligned");
  return RTM_OK;
}

static rtm_status check_probe(const rtm_plan *P, const void *Z, rtm_dtype zt, const void *bar) {
  if ((Z == nullptr) != (bar == nullptr))
    return fail(RTM_E_ARG, "Z and the compressed field must both be given or both be NULL");
  if (!Z) return RTM_OK;
  const rtm_dtype pd = P->d.probe_dtype;
  if (pd == RTM_BF16 || pd == RTM_F16S) {
    if (zt != RTM_I8)
      return fail(RTM_E_DTYPE, "the BF16 and F16S probe paths need +-1 probes (RTM_I8)");
  } else if (pd == RTM_BF16X2) {
    if (zt != RTM_I8 && zt != RTM_F32)
      return fail(RTM_E_DTYPE, "the BF16X2 probe path takes RTM_I8 (+-1) or RTM_F32 probes");
  } else if (zt != RTM_I8 && zt != P->d.field_dtype) {
    return fail(RTM_E_DTYPE, "Z must be RTM_I8 or the field dtype");
  }
  return RTM_OK;
}

template <typename T>
static rtm_status forward_impl(const rtm_plan *P, const void *m, const double *src_pos,
                               const void *q, const double *rec_pos, void *d_pred, const void *Z,
                               rtm_dtype zt, rtm_probe_field what, void *Ubar, void *fin,
                               void *work, hipStream_t st, int n_begin = 0, int n_end = -1,
                               const void *state_in = nullptr) {
  PointTables<T> src_t, rec_t;
  rtm_status s = upload_points<T>(P, static_cast<char *>(work), st, src_pos, &src_t,
                                  d_pred ? rec_pos : nullptr, &rec_t);
  if (s) return s;
  SweepIO io;
  io.adjoint = false;
  io.m = m;
  io.inj_vals = q;
  io.smp_out = d_pred;
  io.Z = Z;
  io.zt = zt;
  io.mode = what == RTM_PROBE_U ? PROBE_CUR : PROBE_UTT;
  io.bar = Ubar;
  io.final_state = fin;
  io.n_begin = n_begin;
  io.n_end = n_end;
  io.state_in = state_in;
  return run_sweep<T>(P, io, src_t, rec_t, static_cast<char *>(work), st);
}

extern "C" rtm_status rtm_forward_probe(const rtm_plan *P, const void *m, const double *src_pos,
                                        const void *q, const double *rec_pos, void *d_pred,
                                        const void *Z, rtm_dtype zt, rtm_probe_field what,
                                        void *Ubar, void *final_state, void *work,
                                        size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if (P->d.nsrc > 0 && (!src_pos || !q)) return fail(RTM_E_ARG, "src_pos and q are required");
  if (d_pred && P->d.nrec > 0 && !rec_pos) return fail(RTM_E_ARG, "rec_pos is required with d_pred");
  if (what != RTM_PROBE_U && what != RTM_PROBE_UTT) return fail(RTM_E_ARG, "bad probe field");
  if ((s = check_probe(P, Z, zt, Ubar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    return forward_impl<double>(P, m, src_pos, q, rec_pos, d_pred, Z, zt, what, Ubar,
                                final_state, work, st);
  return forward_impl<float>(P, m, src_pos, q, rec_pos, d_pred, Z, zt, what, Ubar, final_state,
                             work, st);
}

extern "C" rtm_status rtm_forward_probe_range(const rtm_plan *P, const void *m,
                                              const double *src_pos, const void *q,
                                              const double *rec_pos, void *d_pred, const void *Z,
                                              rtm_dtype zt, rtm_probe_field what, void *Ubar,
                                              int32_t n_begin, int32_t n_end,
                                              const void *state_in, void *state_out, void *work,
                                              size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  const int nt = P->d.nt, k = P->d.k_block;
  if (n_begin < 0 || n_end <= n_begin || n_end > nt)
    return fail(RTM_E_ARG, "need 0 <= n_begin < n_end <= nt");
  if (n_begin % k != 0 || (n_end % k != 0 && n_end != nt))
    return fail(RTM_E_ARG, "range ends must fall on probe-block boundaries (multiples of k_block, or nt)");
  if ((n_begin > 0) != (state_in != nullptr))
    return fail(RTM_E_ARG, "state_in is required exactly when n_begin > 0");
  if (P->d.nsrc > 0 && (!src_pos || !q)) return fail(RTM_E_ARG, "src_pos and q are required");
  if (d_pred && P->d.nrec > 0 && !rec_pos) return fail(RTM_E_ARG, "rec_pos is required with d_pred");
  if (what != RTM_PROBE_U && what != RTM_PROBE_UTT) return fail(RTM_E_ARG, "bad probe field");
  if ((s = check_probe(P, Z, zt, Ubar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    return forward_impl<double>(P, m, src_pos, q, rec_pos, d_pred, Z, zt, what, Ubar, state_out,
                                work, st, n_begin, n_end, state_in);
  return forward_impl<float>(P, m, src_pos, q, rec_pos, d_pred, Z, zt, what, Ubar, state_out,
                             work, st, n_begin, n_end, state_in);
}

template <typename T>
static rtm_status adjoint_impl(const rtm_plan *P, const void *m, const double *rec_pos,
                               const void *res, const double *src_pos, void *qadj, const void *Z,
                               rtm_dtype zt, void *Vbar, void *work, hipStream_t st) {
  PointTables<T> src_t, rec_t;
  rtm_status s = upload_points<T>(P, static_cast<char *>(work), st, qadj ? src_pos : nullptr,
                                  &src_t, rec_pos, &rec_t);
  if (s) return s;
  SweepIO io;
  io.adjoint = true;
  io.m = m;
  io.inj_vals = res;
  io.smp_out = qadj;
  io.Z = Z;
  io.zt = zt;
  io.mode = PROBE_NEW;
  io.bar = Vbar;
  return run_sweep<T>(P, io, rec_t, src_t, static_cast<char *>(work), st);
}

extern "C" rtm_status rtm_adjoint_probe(const rtm_plan *P, const void *m, const double *rec_pos,
                                        const void *res, const double *src_pos, void *qadj,
                                        const void *Z, rtm_dtype zt, void *Vbar, void *work,
                                        size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if (P->d.nrec > 0 && (!rec_pos || !res)) return fail(RTM_E_ARG, "rec_pos and res are required");
  if (qadj && P->d.nsrc > 0 && !src_pos) return fail(RTM_E_ARG, "src_pos is required with qadj");
  if ((s = check_probe(P, Z, zt, Vbar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    return adjoint_impl<double>(P, m, rec_pos, res, src_pos, qadj, Z, zt, Vbar, work, st);
  return adjoint_impl<float>(P, m, rec_pos, res, src_pos, qadj, Z, zt, Vbar, work, st);
}

template <typename T>
static rtm_status adjoint_image_impl(const rtm_plan *P, const void *m, const double *rec_pos,
                                     const void *res, const void *Z, rtm_dtype zt,
                                     const void *Ubar, double scale, void *image, void *work,
                                     hipStream_t st) {
  PointTables<T> src_t, rec_t;
  rtm_status s = upload_points<T>(P, static_cast<char *>(work), st, nullptr, &src_t, rec_pos,
                                  &rec_t);
  if (s) return s;
  HIP_TRY(launch_fill<T>(static_cast<T *>(image), P->N, T(0), st));
  SweepIO io;
  io.adjoint = true;
  io.m = m;
  io.inj_vals = res;
  io.Z = Z;
  io.zt = zt;
  io.mode = PROBE_NEW;
  io.fuse_U = Ubar;
  io.fuse_img = image;
  io.fuse_scale = scale;
  PointTables<T> none;
  return run_sweep<T>(P, io, rec_t, none, static_cast<char *>(work), st);
}

extern "C" rtm_status rtm_adjoint_image(const rtm_plan *P, const void *m, const double *rec_pos,
                                        const void *res, const void *Z, rtm_dtype zt,
                                        const void *Ubar, double scale, void *image, void *work,
                                        size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if (P->d.nrec > 0 && (!rec_pos || !res)) return fail(RTM_E_ARG, "rec_pos and res are required");
  if (!Z || !Ubar || !image) return fail(RTM_E_ARG, "Z, Ubar and image are required");
  if (!mfma_probe(P->d.probe_dtype))
    return fail(RTM_E_UNSUPPORTED, "fused adjoint imaging needs a BF16 probe path");
  if ((s = check_probe(P, Z, zt, Ubar))) return s;
  return adjoint_image_impl<float>(P, m, rec_pos, res, Z, zt, Ubar, scale, image, work,
                                   reinterpret_cast<hipStream_t>(stream));
}

extern "C" rtm_status rtm_image(const rtm_plan *P, const void *U, const void *V, double scale,
                                void *image, rtm_stream stream) {
  g_last_error.clear();
  if (!P || !U || !V || !image) return fail(RTM_E_ARG, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_image<double>(static_cast<const double *>(U), static_cast<const double *>(V),
                                 P->N, P->d.r, scale, static_cast<double *>(image), st));
  else
    HIP_TRY(launch_image<float>(static_cast<const float *>(U), static_cast<const float *>(V),
                                P->N, P->d.r, scale, static_cast<float *>(image), st));
  return RTM_OK;
}

extern "C" rtm_status rtm_offset_gathers(const rtm_plan *P, const void *Ubar, const void *Vbar,
                                         int32_t nfield, int32_t nh, double scale, void *gathers,
                                         rtm_stream stream) {
  g_last_error.clear();
  if (!P || !Ubar || !Vbar || !gathers) return fail(RTM_E_ARG, "NULL argument");
  if (nfield != 1 && nfield != 2) return fail(RTM_E_ARG, "nfield must be 1 or 2");
  if (nh < 0 || nh > 64) return fail(RTM_E_UNSUPPORTED, "offsets: 0 <= nh <= 64");
  if (P->d.field_dtype == RTM_F32 && ((int64_t)P->d.nx / 32 + 2) * P->d.r * 128 >= ((int64_t)1 << 31))
    return fail(RTM_E_UNSUPPORTED,
                "FP32 offset gathers need (nx / 32 + 2) * r * 128 < 2^31 (a row's fields "
                "are addressed with 32-bit offsets)");
  {
    // one workgroup of 256 threads per segment of an x row (128 cells in FP32,
    // 64 in FP64); a dispatch holds fewer than 2^32 work items
    const int64_t seg = P->d.field_dtype == RTM_F32 ? 128 : 64;
    const int64_t wgs = (P->N / P->d.nx) * ((P->d.nx + seg - 1) / seg);
    if (wgs * 256 >= ((int64_t)1 << 32))
      return fail(RTM_E_UNSUPPORTED,
                  "offset gathers need rows * ceil(nx / %lld) * 256 < 2^32 work items (got "
                  "%lld workgroups)", (long long)seg, (long long)wgs);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t fs = (int64_t)P->d.r * P->Npad;
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_offset_gathers<double>(static_cast<const double *>(Ubar),
                                          static_cast<const double *>(Vbar), nfield, fs, P->N,
                                          (int)P->d.nx, P->d.r, nh, scale,
                                          static_cast<double *>(gathers), st));
  else
    HIP_TRY(launch_offset_gathers<float>(static_cast<const float *>(Ubar),
                                         static_cast<const float *>(Vbar), nfield, fs, P->N,
                                         (int)P->d.nx, P->d.r, nh, scale,
                                         static_cast<float *>(gathers), st));
  return RTM_OK;
}

extern "C" rtm_status rtm_bar_to_rows(const rtm_plan *P, const void *bar, void *rows,
                                      rtm_stream stream) {
  g_last_error.clear();
  if (!P || !bar || !rows) return fail(RTM_E_ARG, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_bar_to_rows<double>(static_cast<const double *>(bar), P->N, P->d.r,
                                       static_cast<double *>(rows), st));
  else
    HIP_TRY(launch_bar_to_rows<float>(static_cast<const float *>(bar), P->N, P->d.r,
                                      static_cast<float *>(rows), st));
  return RTM_OK;
}

extern "C" rtm_status rtm_residual(const rtm_plan *P, const void *d_pred, const void *d_obs,
                                   void *resid, double *misfit, void *work, size_t work_bytes,
                                   rtm_stream stream) {
  g_last_error.clear();
  if (!P || !d_pred || !d_obs || !resid || !misfit || !work) return fail(RTM_E_ARG, "NULL argument");
  if (work_bytes < P->total) return fail(RTM_E_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(RTM_E_ARG, "work must be 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double *part = reinterpret_cast<double *>(static_cast<char *>(work) + P->red.off);
  const int64_t nd = (int64_t)P->d.nt * P->d.nrec;
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_residual_misfit<double>(static_cast<const double *>(d_pred),
                                           static_cast<const double *>(d_obs),
                                           static_cast<double *>(resid), nd, part, misfit, st));
  else
    HIP_TRY(launch_residual_misfit<float>(static_cast<const float *>(d_pred),
                                          static_cast<const float *>(d_obs),
                                          static_cast<float *>(resid), nd, part, misfit, st));
  return RTM_OK;
}

extern "C" rtm_status rtm_device_copy(const void *src, void *dst, size_t bytes, rtm_stream stream) {
  g_last_error.clear();
  if (!src || !dst) return fail(RTM_E_ARG, "NULL argument");
  if ((bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
    return fail(RTM_E_ARG, "rtm_device_copy needs 16-byte aligned buffers and a size in 16 bytes");
  HIP_TRY(launch_copy_x4(dst, src, (int64_t)(bytes / 16), reinterpret_cast<hipStream_t>(stream)));
  return RTM_OK;
}

extern "C" rtm_status rtm_dot(const rtm_plan *P, const void *a, const void *b, int64_t n,
                              double *out, void *work, size_t work_bytes, rtm_stream stream) {
  g_last_error.clear();
  if (!P || !a || !b || !out || !work) return fail(RTM_E_ARG, "NULL argument");
  if (n < 0) return fail(RTM_E_ARG, "n must be >= 0");
  if (work_bytes < P->total) return fail(RTM_E_WORKSPACE, "workspace too small");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double *part = reinterpret_cast<double *>(static_cast<char *>(work) + P->red.off);
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_dot<double>(static_cast<const double *>(a), static_cast<const double *>(b), n,
                               part, out, st));
  else
    HIP_TRY(launch_dot<float>(static_cast<const float *>(a), static_cast<const float *>(b), n,
                              part, out, st));
  return RTM_OK;
}

// Graphs of single-shot launch sequences (rtm_set_graph): keyed by a hash of
// everything baked into the launches (plan, pointers, point counts, kernel
// choices); at most kGraphCache kept, the oldest dropped.  Shared by all
// threads (a mutex guards the table; a replay itself is a stream launch).
struct GraphEntry {
  uint64_t key;
  hipGraphExec_t exec;
};
static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static const size_t kGraphCache = 8;

static uint64_t key_mix(uint64_t k, uint64_t v) { return (k ^ v) * 1099511628211ull; }

// The graphs are captured and replayed on an internal non-blocking stream of
// the current device (the caller's stream may be the legacy default stream,
// which cannot be captured), ordered after the caller's stream and before its
// later work by two events.
struct GraphStream {
  hipStream_t s = nullptr;
  hipEvent_t in = nullptr, out = nullptr;
};
static GraphStream g_gstream[64];

// runs `body` (stream-ordered launches on the stream it is given) eagerly on
// st, or through a cached graph when graphs are on; capture is thread-local
// and records no timing events
template <typename F>
static rtm_status run_launches(uint64_t key, hipStream_t st, F body) {
  if (!g_graph) return body(st);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(RTM_E_UNSUPPORTED, "graphs: device index above 63");
  key = key_mix(key, (uint64_t)g_stencil_variant + 1000);
  key = key_mix(key, (uint64_t)g_stencil_blocks);
  key = key_mix(key, (uint64_t)g_stencil_alternate + 77);
  key = key_mix(key, (uint64_t)get_probe_nt() + 99);
  key = key_mix(key, (uint64_t)get_probe_grid(0) + 555);
  key = key_mix(key, (uint64_t)get_probe_grid(1) + 556);
  key = key_mix(key, (uint64_t)dev);
  std::lock_guard<std::mutex> lock(g_graph_mu);
  GraphStream &gs = g_gstream[dev];
  if (!gs.s) {
    HIP_TRY(hipStreamCreateWithFlags(&gs.s, hipStreamNonBlocking));  // default priority
    HIP_TRY(hipEventCreateWithFlags(&gs.in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&gs.out, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(gs.in, st));
  HIP_TRY(hipStreamWaitEvent(gs.s, gs.in, 0));
  hipGraphExec_t exec = nullptr;
  for (const GraphEntry &e : g_graphs)
    if (e.key == key) exec = e.exec;
  if (!exec) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(gs.s, hipStreamCaptureModeThreadLocal));
    const int saved = g_prof_stride;
    g_prof_stride = 0;
    rtm_status s = body(gs.s);
    g_prof_stride = saved;
    hipError_t e = hipStreamEndCapture(gs.s, &g);
    if (s) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(RTM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(RTM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    if (g_graphs.size() >= kGraphCache) {
      (void)hipGraphExecDestroy(g_graphs.front().exec);
      g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back({key, exec});
  }
  HIP_TRY(hipGraphLaunch(exec, gs.s));
  HIP_TRY(hipEventRecord(gs.out, gs.s));
  HIP_TRY(hipStreamWaitEvent(st, gs.out, 0));
  return RTM_OK;
}

template <typename T>
static rtm_status gradient_impl(const rtm_plan *P, const void *m, const double *src_pos,
                                const void *q, const double *rec_pos, const void *d_obs,
                                const void *Z, rtm_dtype zt, void *Ubar, void *Vbar, void *resid,
                                void *grad, double *misfit, void *work, hipStream_t st,
                                double scale) {
  PointTables<T> src_t, rec_t;
  char *w = static_cast<char *>(work);
  rtm_status s0 = upload_points<T>(P, w, st, src_pos, &src_t, rec_pos, &rec_t);
  if (s0) return s0;
  uint64_t key = 1469598103934665603ull;
  {  // the plan's parameters (a new plan may reuse an old one's address)
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&P->d);
    for (size_t i = 0; i < sizeof(P->d); ++i) key = key_mix(key, b[i]);
    key = key_mix(key, (uint64_t)P->total);
  }
  for (const void *p : {(const void *)P, m, q, d_obs, Z, (const void *)Ubar, (const void *)Vbar,
                        (const void *)resid, (const void *)grad, (const void *)misfit,
                        (const void *)work})
    key = key_mix(key, (uint64_t)(uintptr_t)p);
  key = key_mix(key, (uint64_t)zt);
  key = key_mix(key, (uint64_t)src_t.ncell * 4096 + (uint64_t)src_t.npts);
  key = key_mix(key, (uint64_t)rec_t.ncell * 4096 + (uint64_t)rec_t.npts);
  key = key_mix(key, (uint64_t)(scale * 1e6));
  return run_launches(key, st, [&](hipStream_t ls) -> rtm_status {
    hipStream_t st = ls;  // the stream the launches go to (caller's, or the capture stream)
    rtm_status s;
    SweepIO f;
    f.adjoint = false;
    f.m = m;
    f.inj_vals = q;
    f.smp_out = resid;  // d_pred first, turned into the residual below
    f.Z = Z;
    f.zt = zt;
    f.mode = PROBE_UTT;
    f.bar = Ubar;
    if ((s = run_sweep<T>(P, f, src_t, rec_t, w, st))) return s;
    double *part = reinterpret_cast<double *>(w + P->red.off);
    const int64_t nd = (int64_t)P->d.nt * P->d.nrec;
    HIP_TRY(launch_residual_misfit<T>(static_cast<const T *>(resid), static_cast<const T *>(d_obs),
                                      static_cast<T *>(resid), nd, part, misfit, st));
    SweepIO b;
    b.adjoint = true;
    b.m = m;
    b.inj_vals = resid;
    b.Z = Z;
    b.zt = zt;
    b.mode = PROBE_NEW;
    b.bar = Vbar;
    PointTables<T> none;
    if (!Vbar) {  // fused imaging: the adjoint blocks add straight into grad
      HIP_TRY(launch_fill<T>(static_cast<T *>(grad), P->N, T(0), st));
      b.fuse_U = Ubar;
      b.fuse_img = grad;
      b.fuse_scale = scale;
      if ((s = run_sweep<T>(P, b, rec_t, none, w, st))) return s;
    } else {
      if ((s = run_sweep<T>(P, b, rec_t, none, w, st))) return s;
      TimedLaunch ti;
      prof_begin(KT_IMAGE, 0, st, &ti);
      HIP_TRY(launch_image<T>(static_cast<const T *>(Ubar), static_cast<const T *>(Vbar), P->N,
                              P->d.r, scale, static_cast<T *>(grad), st));
      prof_end(st, &ti);
    }
    HIP_TRY(launch_flag_nonfinite<T>(static_cast<const T *>(grad), P->N, status_word(P, w), st));
    HIP_TRY(launch_flag_nonfinite<double>(misfit, 1, status_word(P, w), st));
    return RTM_OK;
  });
}

extern "C" rtm_status fwi_gradient(const rtm_plan *P, const void *m, const double *src_pos,
                                   const void *q, const double *rec_pos, const void *d_obs,
                                   const void *Z, rtm_dtype zt, void *Ubar, void *Vbar,
                                   void *resid, void *grad, double *misfit, void *work,
                                   size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if (!src_pos || !q || !rec_pos || !d_obs || !Z || !Ubar || !resid || !grad || !misfit)
    return fail(RTM_E_ARG, "fwi_gradient needs every array except Vbar");
  if (!Vbar && !mfma_probe(P->d.probe_dtype))
    return fail(RTM_E_UNSUPPORTED, "fused imaging (Vbar = NULL) needs an MFMA probe path (BF16, BF16X2 or F16S)");
  if ((s = check_probe(P, Z, zt, Ubar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    return gradient_impl<double>(P, m, src_pos, q, rec_pos, d_obs, Z, zt, Ubar, Vbar, resid, grad,
                                 misfit, work, st, -1.0 / P->d.r);
  return gradient_impl<float>(P, m, src_pos, q, rec_pos, d_obs, Z, zt, Ubar, Vbar, resid, grad,
                              misfit, work, st, -1.0 / P->d.r);
}

// ---------------------------------------------------------------------------
// range-finder probes: space sketch, orthonormal columns, projected gradient
// ---------------------------------------------------------------------------
struct RfLayout {
  size_t partial, Y, V, total;
};
static RfLayout rf_layout(const rtm_plan *P) {
  RfLayout L;
  L.partial = P->total;
  const size_t pe = (size_t)sketch_partial_elems(P->N, P->d.k_block, P->d.r) * P->esz;
  L.Y = align256(L.partial + pe);
  const size_t yb = (size_t)P->d.nt * P->d.r * sizeof(double);
  L.V = align256(L.Y + yb);
  L.total = align256(L.V + yb);
  return L;
}

static rtm_status check_rf(const rtm_plan *P, size_t work_bytes) {
  const rtm_desc &d = P->d;
  if (d.r > 256) return fail(RTM_E_UNSUPPORTED, "the space sketch supports r <= 256");
  if (d.k_block > 128 || (int64_t)d.k_block * d.r > 8192)
    return fail(RTM_E_UNSUPPORTED, "the space sketch needs k_block <= 128 and k_block * r <= 8192");
  if (d.field_dtype == RTM_F32 && ((d.k_block + 31) / 32) * ((d.r + 31) / 32) > 8)
    return fail(RTM_E_UNSUPPORTED, "the FP32 space sketch needs ceil(k/32) * ceil(r/32) <= 8");
  if (work_bytes < rf_layout(P).total)
    return fail(RTM_E_WORKSPACE, "work has %zu bytes, range-finder calls need %zu", work_bytes,
                rf_layout(P).total);
  return RTM_OK;
}

extern "C" rtm_status rtm_rf_workspace_bytes(const rtm_plan *P, size_t *bytes) {
  g_last_error.clear();
  if (!P || !bytes) return fail(RTM_E_ARG, "NULL argument");
  *bytes = rf_layout(P).total;
  return RTM_OK;
}

template <typename T>
static rtm_status sketch_impl(const rtm_plan *P, const void *m, const double *src_pos,
                              const void *q, uint64_t seed, double *Y, char *w, hipStream_t st) {
  PointTables<T> src_t, none;
  rtm_status s = upload_points<T>(P, w, st, src_pos, &src_t, nullptr, &none);
  if (s) return s;
  SweepIO f;
  f.adjoint = false;
  f.m = m;
  f.inj_vals = q;
  f.mode = PROBE_UTT;
  f.sketch_Y = Y;
  f.sketch_partial = w + rf_layout(P).partial;
  f.sketch_seed = seed;
  return run_sweep<T>(P, f, src_t, none, w, st);
}

extern "C" rtm_status rtm_sketch(const rtm_plan *P, const void *m, const double *src_pos,
                                 const void *q, uint64_t seed, double *Y, void *work,
                                 size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if ((s = check_rf(P, work_bytes))) return s;
  if (!Y) return fail(RTM_E_ARG, "Y is NULL");
  if (P->d.nsrc > 0 && (!src_pos || !q)) return fail(RTM_E_ARG, "src_pos and q are required");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(work);
  if (P->d.field_dtype == RTM_F64) return sketch_impl<double>(P, m, src_pos, q, seed, Y, w, st);
  return sketch_impl<float>(P, m, src_pos, q, seed, Y, w, st);
}

extern "C" rtm_status rtm_orthonormalize(const rtm_plan *P, const double *Y, void *Q, void *work,
                                         size_t work_bytes, rtm_stream stream) {
  g_last_error.clear();
  if (!P || !Y || !Q || !work) return fail(RTM_E_ARG, "NULL argument");
  rtm_status s = check_rf(P, work_bytes);
  if (s) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double *V = reinterpret_cast<double *>(static_cast<char *>(work) + rf_layout(P).V);
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_orthonormalize<double>(Y, P->d.nt, P->d.r, V, static_cast<double *>(Q), st));
  else
    HIP_TRY(launch_orthonormalize<float>(Y, P->d.nt, P->d.r, V, static_cast<float *>(Q), st));
  return RTM_OK;
}

extern "C" rtm_status fwi_gradient_rf(const rtm_plan *P, const void *m, const double *src_pos,
                                      const void *q, const double *rec_pos, const void *d_obs,
                                      uint64_t seed, void *Q, void *Ubar, void *Vbar, void *resid,
                                      void *grad, double *misfit, void *work, size_t work_bytes,
                                      rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if ((s = check_rf(P, work_bytes))) return s;
  if (!src_pos || !q || !rec_pos || !d_obs || !Q || !Ubar || !resid || !grad || !misfit)
    return fail(RTM_E_ARG, "fwi_gradient_rf needs every array except Vbar");
  const rtm_dtype pd = P->d.probe_dtype;
  if (pd != P->d.field_dtype && pd != RTM_BF16X2)
    return fail(RTM_E_UNSUPPORTED, "range-finder probes are real: the probe dtype must be "
                                   "BF16X2 or the field dtype");
  if (!Vbar && pd != RTM_BF16X2)
    return fail(RTM_E_UNSUPPORTED, "fused imaging (Vbar = NULL) needs the BF16X2 probe path");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(work);
  double *Y = reinterpret_cast<double *>(w + rf_layout(P).Y);
  if (P->d.field_dtype == RTM_F64) {
    if ((s = sketch_impl<double>(P, m, src_pos, q, seed, Y, w, st))) return s;
    if ((s = rtm_orthonormalize(P, Y, Q, work, work_bytes, stream))) return s;
    return gradient_impl<double>(P, m, src_pos, q, rec_pos, d_obs, Q, RTM_F64, Ubar, Vbar, resid,
                                 grad, misfit, work, st, -1.0);
  }
  if ((s = sketch_impl<float>(P, m, src_pos, q, seed, Y, w, st))) return s;
  if ((s = rtm_orthonormalize(P, Y, Q, work, work_bytes, stream))) return s;
  return gradient_impl<float>(P, m, src_pos, q, rec_pos, d_obs, Q, RTM_F32, Ubar, Vbar, resid,
                              grad, misfit, work, st, -1.0);
}

// ---------------------------------------------------------------------------
// exact gradient with uniform checkpointing (comparator for Eq. 3)
// ---------------------------------------------------------------------------
// Memory beyond the probed workspace: a 3-level ring for the recomputed
// forward field, 2 levels per checkpoint (u^{jc}, u^{jc-1}) for ceil(nt/c)
// checkpoints, and c levels holding one segment's u_tt.
static int default_checkpoint_every(int nt) {
  int c = (int)std::ceil(std::sqrt(2.0 * nt));
  return c < 1 ? 1 : (c > nt ? nt : c);
}

static size_t exact_extra_bytes(const rtm_plan *P, int c) {
  const int ncp = (P->d.nt + c - 1) / c;
  return align256((size_t)(3 + 2 * (size_t)ncp + c) * P->ld * P->esz);
}

extern "C" rtm_status rtm_exact_workspace_bytes(const rtm_plan *P, int32_t checkpoint_every,
                                                size_t *bytes) {
  if (!P || !bytes) return fail(RTM_E_ARG, "plan and bytes must be non-NULL");
  if (checkpoint_every < 0) return fail(RTM_E_ARG, "checkpoint_every must be >= 0");
  const int c = checkpoint_every ? std::min<int>(checkpoint_every, P->d.nt)
                                 : default_checkpoint_every(P->d.nt);
  *bytes = P->total + exact_extra_bytes(P, c);
  return RTM_OK;
}

template <typename T>
static rtm_status exact_impl(const rtm_plan *P, const void *mv, const double *src_pos,
                             const void *qv, const double *rec_pos, const void *dobs, int c,
                             void *residv, void *gradv, double *misfit, void *work,
                             hipStream_t st) {
  const rtm_desc &d = P->d;
  char *w = static_cast<char *>(work);
  PointTables<T> src_t, rec_t;
  rtm_status s = upload_points<T>(P, w, st, src_pos, &src_t, rec_pos, &rec_t);
  if (s) return s;
  const int nt = d.nt, ndim = d.ndim;
  const int64_t N = P->N, ld = P->ld;
  const int ncp = (nt + c - 1) / c;
  T *ringA = reinterpret_cast<T *>(w + P->ring.off);  // main sweep ring (R levels)
  T *F = reinterpret_cast<T *>(w + P->total);         // recompute ring (3 levels)
  T *CP = F + 3 * ld;                                  // checkpoints [ncp][2]
  T *S = CP + 2 * (int64_t)ncp * ld;                   // segment u_tt [c]
  auto lvA = [&](int j) -> T * { return ringA + (int64_t)(((j + 1) % P->R + P->R) % P->R) * ld; };
  auto lvF = [&](int j) -> T * { return F + (int64_t)(((j + 1) % 3 + 3) % 3) * ld; };
  const T *m = static_cast<const T *>(mv);
  const T *q = static_cast<const T *>(qv);
  T *resid = static_cast<T *>(residv);
  T *grad = static_cast<T *>(gradv);
  int variant = kStencilSimple;
  if (ndim == 3 && sizeof(T) == 4) variant = kStencilTiled;
  if (g_stencil_variant >= 0) variant = g_stencil_variant;
  StepArgs<T> a = step_args<T>(P, m);

  // 1. forward sweep, traces, checkpoints (u^{jc}, u^{jc-1}) before step jc
  HIP_TRY(launch_fill<T>(lvA(-1), N, T(0), st));
  HIP_TRY(launch_fill<T>(lvA(0), N, T(0), st));
  for (int n = 0; n < nt; ++n) {
    if (n % c == 0) {
      HIP_TRY(launch_copy<T>(CP + (int64_t)(2 * (n / c)) * ld, lvA(n), N, st));
      HIP_TRY(launch_copy<T>(CP + (int64_t)(2 * (n / c) + 1) * ld, lvA(n - 1), N, st));
    }
    a.cur = lvA(n);
    a.prev = lvA(n - 1);
    a.next = lvA(n + 1);
    TimedLaunch tl;
    prof_begin(KT_STENCIL, n, st, &tl);
    HIP_TRY(launch_stencil<T>(ndim, a, variant, g_stencil_blocks, st,
                              g_stencil_alternate ? (n & 1) : 0));
    prof_end(st, &tl);
    if (src_t.ncell > 0) HIP_TRY(launch_inject<T>(a, src_t, q + (int64_t)n * src_t.npts, a.next, st));
    if (rec_t.npts > 0) HIP_TRY(launch_sample<T>(rec_t, a.next, resid + (int64_t)n * rec_t.npts, st));
  }
  // 2. residual and misfit
  double *part = reinterpret_cast<double *>(w + P->red.off);
  HIP_TRY(launch_residual_misfit<T>(resid, static_cast<const T *>(dobs), resid,
                                    (int64_t)nt * d.nrec, part, misfit, st));
  // 3. adjoint, segment by segment from the last; each segment's forward is
  //    recomputed from its checkpoint and its u_tt kept for the correlation
  HIP_TRY(launch_fill<T>(grad, N, T(0), st));
  HIP_TRY(launch_fill<T>(lvA(-1), N, T(0), st));
  HIP_TRY(launch_fill<T>(lvA(0), N, T(0), st));
  const T inv_dt2 = (T)(1.0 / (d.dt * d.dt));
  // fuse the u_tt store and the correlation into the stencil when a tiled
  // kernel serves the grid (3D F32); else separate passes
  const bool fused = g_exact_fused && ndim == 3 && sizeof(T) == 4 && variant >= kStencilTiled;
  for (int j = ncp - 1; j >= 0; --j) {
    const int n_lo = j * c, n_hi = std::min(nt, (j + 1) * c);
    HIP_TRY(launch_copy<T>(lvF(n_lo), CP + (int64_t)(2 * j) * ld, N, st));
    HIP_TRY(launch_copy<T>(lvF(n_lo - 1), CP + (int64_t)(2 * j + 1) * ld, N, st));
    StepArgs<T> fa = a;
    for (int n = n_lo; n < n_hi; ++n) {
      fa.cur = lvF(n);
      fa.prev = lvF(n - 1);
      fa.next = lvF(n + 1);
      EpiArgs<T> e;
      e.d2 = S + (int64_t)(n - n_lo) * ld;
      e.inv_dt2 = inv_dt2;
      const int rf = g_stencil_alternate ? (n & 1) : 0;
      if (fused && launch_stencil_epi<T>(ndim, fa, variant, g_stencil_blocks, EPI_D2, e, st, rf) ==
                       hipSuccess) {
        // u_tt written by the stencil's epilogue; the injection adds its share
        if (src_t.ncell > 0)
          HIP_TRY(launch_inject_epi<T>(fa, src_t, q + (int64_t)n * src_t.npts, fa.next, EPI_D2,
                                       e, st));
      } else {
        HIP_TRY(launch_stencil<T>(ndim, fa, variant, g_stencil_blocks, st, rf));
        if (src_t.ncell > 0)
          HIP_TRY(launch_inject<T>(fa, src_t, q + (int64_t)n * src_t.npts, fa.next, st));
        HIP_TRY(launch_second_diff<T>(fa.next, fa.cur, fa.prev, inv_dt2, N, e.d2, st));
      }
    }
    for (int n = n_hi - 1; n >= n_lo; --n) {
      const int sa = nt - 1 - n;  // adjoint sweep step: lam^n is level sa + 1
      a.cur = lvA(sa);
      a.prev = lvA(sa - 1);
      a.next = lvA(sa + 1);
      EpiArgs<T> e;
      e.s = S + (int64_t)(n - n_lo) * ld;
      e.g = grad;
      const int ra = g_stencil_alternate ? (sa & 1) : 0;
      if (fused && launch_stencil_epi<T>(ndim, a, variant, g_stencil_blocks, EPI_CORR, e, st, ra) ==
                       hipSuccess) {
        if (rec_t.ncell > 0)
          HIP_TRY(launch_inject_epi<T>(a, rec_t, resid + (int64_t)n * rec_t.npts, a.next,
                                       EPI_CORR, e, st));
      } else {
        HIP_TRY(launch_stencil<T>(ndim, a, variant, g_stencil_blocks, st, ra));
        if (rec_t.ncell > 0)
          HIP_TRY(launch_inject<T>(a, rec_t, resid + (int64_t)n * rec_t.npts, a.next, st));
        HIP_TRY(launch_correlate<T>(grad, e.s, a.next, N, st));
      }
    }
  }
  HIP_TRY(launch_flag_nonfinite<T>(grad, N, status_word(P, w), st));
  HIP_TRY(launch_flag_nonfinite<double>(misfit, 1, status_word(P, w), st));
  return RTM_OK;
}

extern "C" rtm_status fwi_gradient_exact(const rtm_plan *P, const void *m, const double *src_pos,
                                         const void *q, const double *rec_pos, const void *d_obs,
                                         int32_t checkpoint_every, void *resid, void *grad,
                                         double *misfit, void *work, size_t work_bytes,
                                         rtm_stream stream) {
  g_last_error.clear();
  if (!P) return fail(RTM_E_ARG, "plan is NULL");
  if (checkpoint_every < 0) return fail(RTM_E_ARG, "checkpoint_every must be >= 0");
  const int c = checkpoint_every ? std::min<int>(checkpoint_every, P->d.nt)
                                 : default_checkpoint_every(P->d.nt);
  if (!m || !work) return fail(RTM_E_ARG, "m and work are required");
  if (!src_pos || !q || !rec_pos || !d_obs || !resid || !grad || !misfit)
    return fail(RTM_E_ARG, "fwi_gradient_exact needs every array");
  const size_t need = P->total + exact_extra_bytes(P, c);
  if (work_bytes < need)
    return fail(RTM_E_WORKSPACE, "work has %zu bytes, the exact gradient needs %zu", work_bytes,
                need);
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(RTM_E_ARG, "work must be 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    return exact_impl<double>(P, m, src_pos, q, rec_pos, d_obs, c, resid, grad, misfit, work, st);
  return exact_impl<float>(P, m, src_pos, q, rec_pos, d_obs, c, resid, grad, misfit, work, st);
}

// ---------------------------------------------------------------------------
// stencil autotuner and race check
// ---------------------------------------------------------------------------
// Every candidate kernel runs one step from the same hash-pattern levels; its
// output must equal the one-thread-per-cell kernel's bit for bit (the
// per-cell arithmetic is shared, so any difference is a tiling or
// synchronisation bug).  Passing candidates are timed over `steps` launches.
template <typename T>
static rtm_status autotune_impl(const rtm_plan *P, const void *mv, char *w, int steps,
                                int32_t *best, float *us, int64_t *mismatch, hipStream_t st) {
  const int64_t N = P->N, ld = P->ld;
  T *ring = reinterpret_cast<T *>(w + P->ring.off);
  T *s0 = ring, *s1 = ring + ld, *s2 = ring + 2 * ld, *s3 = ring + 3 * ld;
  auto *cnt = reinterpret_cast<unsigned long long *>(w + P->red.off);
  StepArgs<T> a = step_args<T>(P, static_cast<const T *>(mv));
  a.prev = s0;
  a.cur = s1;
  a.next = s2;
  const T amp = (T)1e-3;
  HIP_TRY(launch_pattern<T>(s0, N, 0x1234567u, amp, st));
  HIP_TRY(launch_pattern<T>(s1, N, 0x89abcdefu, amp, st));
  HIP_TRY(launch_stencil<T>(P->d.ndim, a, kStencilSimple, g_stencil_blocks, st));
  HIP_TRY(launch_copy<T>(s3, s2, N, st));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best_t = 0.f;
  bool have_best = false;
  int best_v = kStencilSimple;
  const int last = P->d.ndim == 3 ? kStencilVariants : kStencilSimple;
  rtm_status status = RTM_OK;
  for (int v = kStencilSimple; v <= last && status == RTM_OK; ++v) {
    // both z-marching directions against the one-thread-per-cell step
    unsigned long long diff = 0;
    hipError_t e = launch_fill<double>(reinterpret_cast<double *>(cnt), 1, 0.0, st);
    for (int rev = 0; rev < 2 && e == hipSuccess; ++rev) {
      e = launch_stencil<T>(P->d.ndim, a, v, g_stencil_blocks, st, rev);
      if (e == hipSuccess) e = launch_count_diff<T>(s2, s3, N, cnt, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&diff, cnt, sizeof diff, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < steps && e == hipSuccess; ++i)
      e = launch_stencil<T>(P->d.ndim, a, v, g_stencil_blocks, st,
                            g_stencil_alternate ? (i & 1) : 0);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      status = fail(RTM_E_HIP, "autotune variant %d: %s", v, hipGetErrorString(e));
      break;
    }
    const float t = steps > 0 ? 1e3f * ms / steps : 0.f;
    if (us) us[v] = t;
    if (mismatch) mismatch[v] = (int64_t)diff;
    if (diff == 0 && (!have_best || t < best_t)) {  // fastest bitwise-correct candidate
      have_best = true;
      best_t = t;
      best_v = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == RTM_OK && best) *best = best_v;
  return status;
}

extern "C" rtm_status rtm_autotune_stencil(const rtm_plan *P, const void *m, void *work,
                                           size_t work_bytes, int32_t steps, int32_t *best,
                                           float *us, int64_t *mismatch, rtm_stream stream) {
  rtm_status s = check_common(P, m, work, work_bytes);
  if (s) return s;
  if (P->R < 4) return fail(RTM_E_UNSUPPORTED, "autotuning needs k_block >= 2 (4 ring levels)");
  if (steps < 0) return fail(RTM_E_ARG, "steps must be >= 0");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (P->d.field_dtype == RTM_F64)
    return autotune_impl<double>(P, m, static_cast<char *>(work), steps, best, us, mismatch, st);
  return autotune_impl<float>(P, m, static_cast<char *>(work), steps, best, us, mismatch, st);
}

// ---------------------------------------------------------------------------
// batched shots: one launch per step for all shots, optional hipGraph
// ---------------------------------------------------------------------------
struct BatchPointRegion {
  Region soff, sidx, sw, sshot, slocal, icell, ishot, ioff, ipt, iw;
  int32_t cap = 0;
};

struct rtm_batch {
  int ns = 0;
  std::vector<rtm_plan *> P;
  std::vector<size_t> ring_off;
  Region red, status, shots, io_fwd, io_adj, tiles;
  Region queue;  // work-queue counter of the probe launches (int32)
  BatchPointRegion src, rec;
  size_t tab_off = 0, tab_bytes = 0, total = 0;
  std::vector<int4> tile_host;
  int32_t nsrc_total = 0, nrec_total = 0;
  // cached graph of the last fwi_gradient_batched launch sequence
  hipGraphExec_t gexec = nullptr;
  uint64_t gkey = 0;
};

static void place_batch_points(size_t &cur, BatchPointRegion &pr, int32_t n, size_t esz) {
  const size_t c = (size_t)8 * n;
  pr.cap = n;
  place(cur, pr.soff, 4 * ((size_t)n + 1));
  place(cur, pr.sidx, 4 * c);
  place(cur, pr.sw, esz * c);
  place(cur, pr.sshot, 4 * (size_t)n);
  place(cur, pr.slocal, 4 * (size_t)n);
  place(cur, pr.icell, 4 * c);
  place(cur, pr.ishot, 4 * c);
  place(cur, pr.ioff, 4 * (c + 1));
  place(cur, pr.ipt, 4 * c);
  place(cur, pr.iw, esz * c);
}

extern "C" void rtm_batch_destroy(rtm_batch *b) {
  if (!b) return;
  for (rtm_plan *p : b->P) rtm_plan_destroy(p);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  delete b;
}

extern "C" rtm_status rtm_batch_create(const rtm_desc *shots, int32_t nshots, rtm_batch **out) {
  g_last_error.clear();
  if (!shots || !out || nshots < 1) return fail(RTM_E_ARG, "need nshots >= 1 descriptors");
  const rtm_desc &d0 = shots[0];
  for (int i = 0; i < nshots; ++i) {
    const rtm_desc &d = shots[i];
    if (d.ndim != 3 || d.field_dtype != RTM_F32 ||
        !mfma_probe(d.probe_dtype))
      return fail(RTM_E_UNSUPPORTED, "batched shots are 3D, F32 fields, BF16 / BF16X2 / F16S probes");
    if (d.nt != d0.nt || d.dt != d0.dt || d.h != d0.h || d.r != d0.r ||
        d.k_block != d0.k_block || d.probe_dtype != d0.probe_dtype)
      return fail(RTM_E_ARG, "shot %d: nt, dt, h, r, k_block and probe dtype must agree", i);
  }
  rtm_batch *b = new (std::nothrow) rtm_batch();
  if (!b) return fail(RTM_E_ARG, "out of host memory");
  b->ns = nshots;
  for (int i = 0; i < nshots; ++i) {
    rtm_plan *p = nullptr;
    rtm_status st = rtm_plan_create(&shots[i], &p);
    if (st) {
      rtm_batch_destroy(b);
      return st;
    }
    b->P.push_back(p);
    b->nsrc_total += shots[i].nsrc;
    b->nrec_total += shots[i].nrec;
  }
  // tile table: 64 x 16 column tiles of every shot, z split until the launch
  // has >= 2 x rtm_set_stencil_blocks workgroups (default 4096; each chunk >=
  // 16 planes): the windows are shallow (128-256 planes) and the extra waves
  // in flight outweigh the chunks' warm-up planes (measured: 1024 -> 4096
  // workgroups, 115 -> 121 Gcell-updates/s).  Fixed when the batch is created.
  int nzc = 1;
  auto count = [&](int z) {
    int64_t t = 0;
    for (auto *p : b->P) t += ((p->d.nx + 63) / 64) * ((p->d.ny + 15) / 16) * (int64_t)z;
    return t;
  };
  int minz = INT32_MAX;
  for (auto *p : b->P) minz = std::min<int>(minz, (int)p->d.nz);
  while (count(nzc) < 2 * (int64_t)g_stencil_blocks && minz / (nzc * 2) >= 16) nzc *= 2;
  for (int i = 0; i < nshots; ++i) {
    const rtm_desc &d = b->P[i]->d;
    const int ntx = (int)((d.nx + 63) / 64), nty = (int)((d.ny + 15) / 16);
    const int zc = (int)((d.nz + nzc - 1) / nzc);
    if (ntx > 0xffff || nty > 0x7fff) {
      rtm_batch_destroy(b);
      return fail(RTM_E_SHAPE, "shot %d: too many tiles", i);
    }
    if (b->P[i]->N * 4 >= (int64_t(1) << 32)) {  // tiled kernels use 32-bit offsets
      rtm_batch_destroy(b);
      return fail(RTM_E_SHAPE, "shot %d: a window of 4 GiB or more per level", i);
    }
    for (int z0 = 0; z0 < d.nz; z0 += zc)
      for (int by = 0; by < nty; ++by)
        for (int bx = 0; bx < ntx; ++bx)
          b->tile_host.push_back(make_int4(i, bx | (by << 16), z0, (int)std::min<int64_t>(z0 + zc, d.nz)));
  }
  size_t cur = 0;
  for (auto *p : b->P) {
    b->ring_off.push_back(cur);
    cur = align256(cur + (size_t)p->R * p->ld * 4);
  }
  place(cur, b->red, sizeof(double) * (kReduceBlocks + 8) * nshots);
  place(cur, b->status, sizeof(uint32_t));
  place(cur, b->queue, sizeof(int32_t));
  b->tab_off = cur;
  place(cur, b->shots, sizeof(ShotStep<float>) * nshots);
  place(cur, b->io_fwd, sizeof(ShotIO<float>) * nshots);
  place(cur, b->io_adj, sizeof(ShotIO<float>) * nshots);
  place(cur, b->tiles, sizeof(int4) * b->tile_host.size());
  place_batch_points(cur, b->src, b->nsrc_total, 4);
  place_batch_points(cur, b->rec, b->nrec_total, 4);
  b->tab_bytes = cur - b->tab_off;
  b->total = cur;
  *out = b;
  return RTM_OK;
}

extern "C" rtm_status rtm_batch_workspace_bytes(const rtm_batch *b, size_t *bytes) {
  if (!b || !bytes) return fail(RTM_E_ARG, "batch and bytes must be non-NULL");
  *bytes = b->total;
  return RTM_OK;
}

// merged CSR tables of one point set across shots (host staging)
static rtm_status stage_batch_points(const rtm_batch *b, const BatchPointRegion &pr,
                                     const rtm_shot_io *io, bool rec, std::vector<unsigned char> &host,
                                     int32_t *npts, int32_t *ncell, uint64_t *hash) {
  std::vector<int32_t> soff(1, 0), sidx, sshot, slocal, icell, ishot, ioff(1, 0), ipt;
  std::vector<float> sw, iw;
  for (int i = 0; i < b->ns; ++i) {
    const rtm_plan *P = b->P[i];
    const int32_t n = rec ? P->d.nrec : P->d.nsrc;
    const double *pos = rec ? io[i].rec_pos : io[i].src_pos;
    if (n > 0 && !pos) return fail(RTM_E_ARG, "shot %d: positions missing", i);
    for (int32_t k = 0; k < 3 * n; ++k) {
      uint64_t v;
      std::memcpy(&v, pos + k, 8);
      *hash = (*hash ^ v) * 1099511628211ull;
    }
    HostPoints hp;
    rtm_status st = build_points(P, n, pos, hp);
    if (st) return st;
    for (int32_t p = 0; p < n; ++p) {
      for (int32_t j = hp.soff[p]; j < hp.soff[p + 1]; ++j) {
        sidx.push_back(hp.sidx[j]);
        sw.push_back((float)hp.sw[j]);
      }
      soff.push_back((int32_t)sidx.size());
      sshot.push_back(i);
      slocal.push_back(p);
    }
    for (size_t c = 0; c < hp.icell.size(); ++c) {
      icell.push_back(hp.icell[c]);
      ishot.push_back(i);
      for (int32_t j = hp.ioff[c]; j < hp.ioff[c + 1]; ++j) {
        ipt.push_back(hp.ipt[j]);
        iw.push_back((float)hp.iw[j]);
      }
      ioff.push_back((int32_t)ipt.size());
    }
  }
  auto put = [&](const Region &r, const void *src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + (r.off - b->tab_off), src, bytes);
  };
  put(pr.soff, soff.data(), 4 * soff.size());
  put(pr.sidx, sidx.data(), 4 * sidx.size());
  put(pr.sw, sw.data(), 4 * sw.size());
  put(pr.sshot, sshot.data(), 4 * sshot.size());
  put(pr.slocal, slocal.data(), 4 * slocal.size());
  put(pr.icell, icell.data(), 4 * icell.size());
  put(pr.ishot, ishot.data(), 4 * ishot.size());
  put(pr.ioff, ioff.data(), 4 * ioff.size());
  put(pr.ipt, ipt.data(), 4 * ipt.size());
  put(pr.iw, iw.data(), 4 * iw.size());
  *npts = (int32_t)sshot.size();
  *ncell = (int32_t)icell.size();
  return RTM_OK;
}

static BatchPoints<float> batch_points(const BatchPointRegion &pr, char *w, int32_t npts,
                                       int32_t ncell) {
  BatchPoints<float> t;
  t.soff = reinterpret_cast<const int32_t *>(w + pr.soff.off);
  t.sidx = reinterpret_cast<const int32_t *>(w + pr.sidx.off);
  t.sw = reinterpret_cast<const float *>(w + pr.sw.off);
  t.sshot = reinterpret_cast<const int32_t *>(w + pr.sshot.off);
  t.slocal = reinterpret_cast<const int32_t *>(w + pr.slocal.off);
  t.icell = reinterpret_cast<const int32_t *>(w + pr.icell.off);
  t.ishot = reinterpret_cast<const int32_t *>(w + pr.ishot.off);
  t.ioff = reinterpret_cast<const int32_t *>(w + pr.ioff.off);
  t.ipt = reinterpret_cast<const int32_t *>(w + pr.ipt.off);
  t.iw = reinterpret_cast<const float *>(w + pr.iw.off);
  t.npts = npts;
  t.ncell = ncell;
  return t;
}

// The whole batched gradient as a stream-ordered launch sequence (captured
// into a graph when requested).
static rtm_status batch_enqueue(const rtm_batch *b, const rtm_shot_io *io, double *misfit,
                                char *w, const BatchPoints<float> &src_t,
                                const BatchPoints<float> &rec_t, int variant, hipStream_t st) {
  const rtm_desc &d = b->P[0]->d;
  const int nt = d.nt, k = d.k_block;
  const auto *shots = reinterpret_cast<const ShotStep<float> *>(w + b->shots.off);
  const auto *iof = reinterpret_cast<const ShotIO<float> *>(w + b->io_fwd.off);
  const auto *ioa = reinterpret_cast<const ShotIO<float> *>(w + b->io_adj.off);
  const auto *tiles = reinterpret_cast<const int4 *>(w + b->tiles.off);
  const int ntiles = (int)b->tile_host.size();
  auto ring = [&](int i) { return reinterpret_cast<float *>(w + b->ring_off[i]); };
  auto lvl = [&](int i, int j) {
    const rtm_plan *P = b->P[i];
    return ring(i) + (int64_t)((j + 1) % P->R) * P->ld;
  };
  auto probe = [&](bool adj, int s0, int kb) -> rtm_status {
    for (int i = 0; i < b->ns; ++i) {
      const rtm_plan *P = b->P[i];
      ProbeArgs<float> p{};
      p.ring = ring(i);
      p.ld = P->ld;
      p.R = P->R;
      p.s0 = s0;
      p.slot0 = s0 % P->R;
      p.kb = kb;
      p.zrow0 = adj ? nt - 1 - s0 : s0;
      p.zdir = adj ? -1 : 1;
      p.r = d.r;
      p.N = P->N;
      p.bar = adj ? nullptr : static_cast<float *>(io[i].Ubar);
      p.inv_dt2 = (float)(1.0 / (d.dt * d.dt));
      p.mode = adj ? PROBE_NEW : PROBE_UTT;
      p.queue = reinterpret_cast<int *>(w + b->queue.off);
      HIP_TRY(launch_probe_mfma(p, io[i].Z, false, probe_op(d.probe_dtype),
                                adj ? static_cast<const float *>(io[i].Ubar) : nullptr,
                                adj ? static_cast<float *>(io[i].grad) : nullptr,
                                (float)(-1.0 / d.r), st));
    }
    return RTM_OK;
  };
  rtm_status s_;
  uint32_t *status = reinterpret_cast<uint32_t *>(w + b->status.off);
  HIP_TRY(launch_status_clear(status, st));
  // forward
  for (int i = 0; i < b->ns; ++i) {
    HIP_TRY(launch_fill<float>(lvl(i, -1), b->P[i]->N, 0.f, st));
    HIP_TRY(launch_fill<float>(lvl(i, 0), b->P[i]->N, 0.f, st));
    HIP_TRY(launch_fill<float>(static_cast<float *>(io[i].Ubar), (int64_t)d.r * b->P[i]->Npad, 0.f, st));
  }
  int s0 = 0;
  for (int s = 0; s < nt; ++s) {
    HIP_TRY(launch_stencil_batched<float>(shots, tiles, ntiles, s, variant, st,
                                          g_stencil_alternate ? (s & 1) : 0));
    HIP_TRY(launch_inject_batched<float>(shots, iof, src_t, s, s, st));
    HIP_TRY(launch_sample_batched<float>(shots, iof, rec_t, s, s, st));
    if (s + 1 - s0 == k || s == nt - 1) {
      if ((s_ = probe(false, s0, s + 1 - s0))) return s_;
      s0 = s + 1;
    }
  }
  // residual and misfit per shot
  for (int i = 0; i < b->ns; ++i) {
    double *part = reinterpret_cast<double *>(w + b->red.off) + (size_t)i * (kReduceBlocks + 8);
    float *res = static_cast<float *>(io[i].resid);
    HIP_TRY(launch_residual_misfit<float>(res, static_cast<const float *>(io[i].d_obs), res,
                                          (int64_t)nt * b->P[i]->d.nrec, part, misfit + i, st));
  }
  // adjoint with the imaging condition folded into its probe blocks
  for (int i = 0; i < b->ns; ++i) {
    HIP_TRY(launch_fill<float>(lvl(i, -1), b->P[i]->N, 0.f, st));
    HIP_TRY(launch_fill<float>(lvl(i, 0), b->P[i]->N, 0.f, st));
    HIP_TRY(launch_fill<float>(static_cast<float *>(io[i].grad), b->P[i]->N, 0.f, st));
  }
  s0 = 0;
  for (int s = 0; s < nt; ++s) {
    HIP_TRY(launch_stencil_batched<float>(shots, tiles, ntiles, s, variant, st,
                                          g_stencil_alternate ? (s & 1) : 0));
    HIP_TRY(launch_inject_batched<float>(shots, ioa, rec_t, s, nt - 1 - s, st));
    if (s + 1 - s0 == k || s == nt - 1) {
      if ((s_ = probe(true, s0, s + 1 - s0))) return s_;
      s0 = s + 1;
    }
  }
  // non-finite watch: each shot's last adjoint level, its gradient (a stacked
  // buffer is scanned once per shot that shares it) and its misfit
  for (int i = 0; i < b->ns; ++i) {
    HIP_TRY(launch_flag_nonfinite<float>(lvl(i, nt), b->P[i]->N, status, st));
    HIP_TRY(launch_flag_nonfinite<float>(static_cast<const float *>(io[i].grad), b->P[i]->N,
                                         status, st));
    HIP_TRY(launch_flag_nonfinite<double>(misfit + i, 1, status, st));
  }
  return RTM_OK;
}

extern "C" rtm_status rtm_batch_stream_status(const rtm_batch *b, const void *work,
                                              rtm_stream stream) {
  g_last_error.clear();
  if (!b || !work) return fail(RTM_E_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(RTM_E_ARG, "work must be 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  uint32_t word = 0;
  HIP_TRY(hipMemcpyAsync(&word, static_cast<const char *>(work) + b->status.off, sizeof(word),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (word) return fail(RTM_E_NONFINITE, "a non-finite value reached a shot's wavefield or outputs");
  return RTM_OK;
}

extern "C" rtm_status fwi_gradient_batched(rtm_batch *b, const rtm_shot_io *io, double *misfit,
                                           int32_t use_graph, void *work, size_t work_bytes,
                                           rtm_stream stream) {
  g_last_error.clear();
  if (!b || !io || !misfit || !work) return fail(RTM_E_ARG, "NULL argument");
  if (work_bytes < b->total)
    return fail(RTM_E_WORKSPACE, "work has %zu bytes, the batch needs %zu", work_bytes, b->total);
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(RTM_E_ARG, "work must be 256-byte aligned");
  for (int i = 0; i < b->ns; ++i) {
    const rtm_shot_io &x = io[i];
    if (!x.m || !x.Z || !x.Ubar || !x.grad || !x.d_obs || !x.resid ||
        (b->P[i]->d.nsrc > 0 && (!x.q || !x.src_pos)) || (b->P[i]->d.nrec > 0 && !x.rec_pos))
      return fail(RTM_E_ARG, "shot %d: missing array", i);
    // stacking: shots may share one gradient buffer when their grids agree;
    // no gradient buffer may be another shot's input or output array
    for (int j = 0; j < b->ns; ++j) {
      const rtm_shot_io &y = io[j];
      const rtm_desc &di = b->P[i]->d, &dj = b->P[j]->d;
      if (j != i && x.grad == y.grad &&
          (di.nz != dj.nz || di.ny != dj.ny || di.nx != dj.nx))
        return fail(RTM_E_ARG, "shots %d and %d share a gradient buffer but not a grid", i, j);
      if (x.grad == y.Ubar || x.grad == y.resid || x.grad == y.m || x.grad == y.d_obs ||
          x.grad == y.q)
        return fail(RTM_E_ARG, "shot %d: the gradient buffer is also an input or output of "
                               "shot %d", i, j);
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(work);
  // stage every table (shot steps, io, tiles, points) and upload once
  std::vector<unsigned char> host(b->tab_bytes, 0);
  auto put = [&](const Region &r, const void *src, size_t bytes) {
    std::memcpy(host.data() + (r.off - b->tab_off), src, bytes);
  };
  std::vector<ShotStep<float>> shots(b->ns);
  std::vector<ShotIO<float>> iof(b->ns), ioa(b->ns);
  uint64_t key = 1469598103934665603ull;
  auto mix = [&](const void *p) { key = (key ^ (uint64_t)(uintptr_t)p) * 1099511628211ull; };
  mix(work);
  mix(misfit);
  for (int i = 0; i < b->ns; ++i) {
    const rtm_plan *P = b->P[i];
    shots[i].a = step_args<float>(P, static_cast<const float *>(io[i].m));
    shots[i].ring = reinterpret_cast<float *>(w + b->ring_off[i]);
    shots[i].ld = P->ld;
    shots[i].R = P->R;
    iof[i] = {static_cast<const float *>(io[i].q), static_cast<float *>(io[i].resid), P->d.nsrc,
              P->d.nrec};
    ioa[i] = {static_cast<const float *>(io[i].resid), nullptr, P->d.nrec, 0};
    for (const void *p : {io[i].m, io[i].q, io[i].d_obs, io[i].Z, (const void *)io[i].Ubar,
                          (const void *)io[i].resid, (const void *)io[i].grad})
      mix(p);
  }
  put(b->shots, shots.data(), sizeof(ShotStep<float>) * b->ns);
  put(b->io_fwd, iof.data(), sizeof(ShotIO<float>) * b->ns);
  put(b->io_adj, ioa.data(), sizeof(ShotIO<float>) * b->ns);
  put(b->tiles, b->tile_host.data(), sizeof(int4) * b->tile_host.size());
  int32_t snp = 0, snc = 0, rnp = 0, rnc = 0;
  rtm_status s = stage_batch_points(b, b->src, io, false, host, &snp, &snc, &key);
  if (s) return s;
  if ((s = stage_batch_points(b, b->rec, io, true, host, &rnp, &rnc, &key))) return s;
  int variant = g_stencil_variant >= kStencilTiled ? g_stencil_variant : 7;
  key = (key ^ (uint64_t)variant) * 1099511628211ull;
  key = (key ^ (uint64_t)(g_stencil_alternate + 64)) * 1099511628211ull;
  HIP_TRY(hipMemcpyAsync(w + b->tab_off, host.data(), b->tab_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  BatchPoints<float> src_t = batch_points(b->src, w, snp, snc);
  BatchPoints<float> rec_t = batch_points(b->rec, w, rnp, rnc);
  if (!use_graph) return batch_enqueue(b, io, misfit, w, src_t, rec_t, variant, st);
  if (!b->gexec || b->gkey != key) {
    if (b->gexec) {
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int saved = g_prof_stride;
    g_prof_stride = 0;  // no event records inside a capture
    s = batch_enqueue(b, io, misfit, w, src_t, rec_t, variant, st);
    g_prof_stride = saved;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(RTM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->gexec = nullptr;
      return fail(RTM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->gkey = key;
  }
  HIP_TRY(hipGraphLaunch(b->gexec, st));
  return RTM_OK;
}

// ---------------------------------------------------------------------------
// pseudo-acoustic TTI sweeps
// ---------------------------------------------------------------------------
// Workspace beyond the acoustic plan's: a second ring (q), 5 coefficient
// levels and 8 intermediate levels.  The acoustic ring holds p.
static size_t tti_extra_bytes(const rtm_plan *P) {
  return align256((size_t)(P->R + 5 + 8) * P->ld * P->esz);
}

extern "C" rtm_status rtm_tti_workspace_bytes(const rtm_plan *P, size_t *bytes) {
  if (!P || !bytes) return fail(RTM_E_ARG, "plan and bytes must be non-NULL");
  *bytes = P->total + tti_extra_bytes(P);
  return RTM_OK;
}

struct TtiIO {
  bool adjoint = false;
  const void *m = nullptr, *aniso = nullptr;
  const void *inj_vals = nullptr;  // forward: into p and q; adjoint: into lam_p
  void *smp_out = nullptr;         // forward: Pr p; adjoint: Ps (lam_p + lam_q)
  const void *Z = nullptr;
  rtm_dtype zt = RTM_I8;
  void *bar = nullptr;             // [2][r*Npad]: p then q
  const void *fuse_U = nullptr;    // [2][r*Npad] forward compressed fields (fused imaging)
  void *fuse_img = nullptr;
  double fuse_scale = 0.0;
};

template <typename T>
static rtm_status run_tti_sweep(const rtm_plan *P, const TtiIO &io, const PointTables<T> &inj,
                                const PointTables<T> &smp, char *w, hipStream_t st) {
  const rtm_desc &d = P->d;
  const int64_t N = P->N, ld = P->ld, barn = (int64_t)d.r * P->Npad;
  T *ringP = reinterpret_cast<T *>(w + P->ring.off);
  T *ringQ = reinterpret_cast<T *>(w + P->total);
  T *coef = ringQ + (int64_t)P->R * ld;
  T *g = coef + 5 * ld;
  auto lv = [&](T *ring, int j) { return ring + (int64_t)((j + 1) % P->R) * ld; };
  StepArgs<T> a = step_args<T>(P, static_cast<const T *>(io.m));
  // tiled TTI kernels (32-bit offsets: fields below 4 GiB) unless the simple
  // stencil is forced
  const int shape = (g_stencil_variant == kStencilSimple || ld * (int64_t)sizeof(T) >= (1LL << 32))
                        ? 0 : g_tti_shape;
  // the coefficient levels and intermediates use stride ld (>= N)
  HIP_TRY(launch_tti_coef<T>(static_cast<const T *>(io.aniso), N, coef, st));  // [5][N]
  for (T *ring : {ringP, ringQ}) {
    HIP_TRY(launch_fill<T>(lv(ring, -1), N, T(0), st));
    HIP_TRY(launch_fill<T>(lv(ring, 0), N, T(0), st));
  }
  T *bar = static_cast<T *>(io.bar);
  if (bar) HIP_TRY(launch_fill<T>(bar, 2 * barn, T(0), st));
  const T *vals = static_cast<const T *>(io.inj_vals);
  T *out = static_cast<T *>(io.smp_out);
  int s0 = 0;
  for (int s = 0; s < d.nt; ++s) {
    const int n = io.adjoint ? d.nt - 1 - s : s;
    T *pn = lv(ringP, s + 1), *qn = lv(ringQ, s + 1);
    TimedLaunch tl;
    prof_begin(io.adjoint ? KT_TTI_ADJ : KT_TTI, s, st, &tl);
    HIP_TRY(launch_tti_step<T>(a, d.h, io.adjoint, coef, lv(ringP, s), lv(ringP, s - 1),
                               lv(ringQ, s), lv(ringQ, s - 1), pn, qn, g, shape,
                               g_tti_blocks[io.adjoint ? 1 : 0], st));
    prof_end(st, &tl);
    if (inj.ncell > 0 && vals) {
      HIP_TRY(launch_inject<T>(a, inj, vals + (int64_t)n * inj.npts, pn, st));
      if (!io.adjoint) HIP_TRY(launch_inject<T>(a, inj, vals + (int64_t)n * inj.npts, qn, st));
    }
    if (out && smp.npts > 0) {
      if (!io.adjoint)
        HIP_TRY(launch_sample<T>(smp, pn, out + (int64_t)n * smp.npts, st));
      else
        HIP_TRY(launch_sample_sum<T>(smp, pn, qn, out + (int64_t)n * smp.npts, st));
    }
    if ((bar || io.fuse_img) && (s + 1 - s0 == d.k_block || s == d.nt - 1)) {
      for (int f = 0; f < 2; ++f) {
        ProbeArgs<T> p{};
        p.ring = f == 0 ? ringP : ringQ;
        p.ld = ld;
        p.R = P->R;
        p.s0 = s0;
        p.slot0 = s0 % P->R;
        p.kb = s + 1 - s0;
        p.zrow0 = io.adjoint ? d.nt - 1 - s0 : s0;
        p.zdir = io.adjoint ? -1 : 1;
        p.r = d.r;
        p.N = N;
        p.bar = bar ? bar + f * barn : nullptr;
        p.inv_dt2 = (T)(1.0 / (d.dt * d.dt));
        p.mode = io.adjoint ? PROBE_NEW : PROBE_UTT;
        if constexpr (sizeof(T) == 4) {
          if (mfma_probe(d.probe_dtype)) {
            const float *Uf = io.fuse_img ? static_cast<const float *>(io.fuse_U) + f * barn : nullptr;
            HIP_TRY(launch_probe_mfma(p, io.Z, io.zt == RTM_F32, probe_op(d.probe_dtype), Uf,
                                      static_cast<float *>(io.fuse_img), (float)io.fuse_scale, st));
            continue;
          }
        }
        HIP_TRY(launch_probe_vec<T>(p, io.Z, io.zt == RTM_I8, st));
      }
      s0 = s + 1;
    }
  }
  HIP_TRY(launch_flag_nonfinite<T>(lv(ringP, d.nt), N, status_word(P, w), st));
  HIP_TRY(launch_flag_nonfinite<T>(lv(ringQ, d.nt), N, status_word(P, w), st));
  return RTM_OK;
}

static rtm_status check_tti(const rtm_plan *P, const void *m, const void *aniso, void *work,
                            size_t work_bytes) {
  rtm_status s = check_common(P, m, work, P ? P->total : 0);
  if (s) return s;
  if (P->d.ndim != 3) return fail(RTM_E_UNSUPPORTED, "TTI needs a 3D plan");
  if (!aniso) return fail(RTM_E_ARG, "aniso (eps, delta, theta, phi) is required");
  if (work_bytes < P->total + tti_extra_bytes(P))
    return fail(RTM_E_WORKSPACE, "work has %zu bytes, TTI needs %zu", work_bytes,
                P->total + tti_extra_bytes(P));
  return RTM_OK;
}

// Stability screen of the model before a TTI sweep (one read of m, eps and
// delta into the reduction partials, then a synchronising copy of two
// numbers): the plan's c_max must cover max v sqrt(max(1, 1 + 2 eps)) over
// the cells (the frozen-coefficient bound of the coupled system; see
// k_tti_screen), and every cell needs delta <= eps with eps, delta > -1/2.
// Nothing the caller sees is written before it passes.
static rtm_status screen_tti(const rtm_plan *P, const void *m, const void *aniso, void *work,
                             hipStream_t st) {
  double *part = reinterpret_cast<double *>(static_cast<char *>(work) + P->red.off);
  if (P->d.field_dtype == RTM_F64)
    HIP_TRY(launch_tti_screen<double>(static_cast<const double *>(m),
                                      static_cast<const double *>(aniso), P->N, part, st));
  else
    HIP_TRY(launch_tti_screen<float>(static_cast<const float *>(m),
                                     static_cast<const float *>(aniso), P->N, part, st));
  double out[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(out, part + 1024, sizeof out, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (out[1] > 0.0)
    return fail(RTM_E_ARG, "TTI model: %.0f cells have delta > eps or eps, delta <= -1/2 "
                           "(the coupled system needs delta <= eps)", out[1]);
  const double c = std::sqrt(out[0]);
  if (c > P->d.c_max * (1.0 + 1e-6))
    return fail(RTM_E_CFL, "TTI model: the largest v sqrt(max(1, 1 + 2 eps)) is %.3f m/s, above "
                           "the plan's c_max %.3f m/s (its CFL check used c_max)", c, P->d.c_max);
  return RTM_OK;
}

template <typename T>
static rtm_status tti_fwd_impl(const rtm_plan *P, const void *m, const void *aniso,
                               const double *src_pos, const void *q, const double *rec_pos,
                               void *d_pred, const void *Z, rtm_dtype zt, void *Ubar, void *work,
                               hipStream_t st) {
  PointTables<T> src_t, rec_t;
  char *w = static_cast<char *>(work);
  rtm_status s = upload_points<T>(P, w, st, src_pos, &src_t, d_pred ? rec_pos : nullptr, &rec_t);
  if (s) return s;
  TtiIO io;
  io.m = m;
  io.aniso = aniso;
  io.inj_vals = q;
  io.smp_out = d_pred;
  io.Z = Z;
  io.zt = zt;
  io.bar = Ubar;
  return run_tti_sweep<T>(P, io, src_t, rec_t, w, st);
}

extern "C" rtm_status rtm_tti_forward_probe(const rtm_plan *P, const void *m, const void *aniso,
                                            const double *src_pos, const void *q,
                                            const double *rec_pos, void *d_pred, const void *Z,
                                            rtm_dtype zt, void *Ubar, void *work,
                                            size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_tti(P, m, aniso, work, work_bytes);
  if (s) return s;
  if (P->d.nsrc > 0 && (!src_pos || !q)) return fail(RTM_E_ARG, "src_pos and q are required");
  if (d_pred && P->d.nrec > 0 && !rec_pos) return fail(RTM_E_ARG, "rec_pos is required");
  if ((s = check_probe(P, Z, zt, Ubar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((s = screen_tti(P, m, aniso, work, st))) return s;
  if (P->d.field_dtype == RTM_F64)
    return tti_fwd_impl<double>(P, m, aniso, src_pos, q, rec_pos, d_pred, Z, zt, Ubar, work, st);
  return tti_fwd_impl<float>(P, m, aniso, src_pos, q, rec_pos, d_pred, Z, zt, Ubar, work, st);
}

template <typename T>
static rtm_status tti_adj_impl(const rtm_plan *P, const void *m, const void *aniso,
                               const double *rec_pos, const void *res, const double *src_pos,
                               void *qadj, const void *Z, rtm_dtype zt, void *Vbar, void *work,
                               hipStream_t st) {
  PointTables<T> src_t, rec_t;
  char *w = static_cast<char *>(work);
  rtm_status s = upload_points<T>(P, w, st, qadj ? src_pos : nullptr, &src_t, rec_pos, &rec_t);
  if (s) return s;
  TtiIO io;
  io.adjoint = true;
  io.m = m;
  io.aniso = aniso;
  io.inj_vals = res;
  io.smp_out = qadj;
  io.Z = Z;
  io.zt = zt;
  io.bar = Vbar;
  return run_tti_sweep<T>(P, io, rec_t, src_t, w, st);
}

extern "C" rtm_status rtm_tti_adjoint_probe(const rtm_plan *P, const void *m, const void *aniso,
                                            const double *rec_pos, const void *res,
                                            const double *src_pos, void *qadj, const void *Z,
                                            rtm_dtype zt, void *Vbar, void *work,
                                            size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_tti(P, m, aniso, work, work_bytes);
  if (s) return s;
  if (P->d.nrec > 0 && (!rec_pos || !res)) return fail(RTM_E_ARG, "rec_pos and res are required");
  if (qadj && P->d.nsrc > 0 && !src_pos) return fail(RTM_E_ARG, "src_pos is required with qadj");
  if ((s = check_probe(P, Z, zt, Vbar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((s = screen_tti(P, m, aniso, work, st))) return s;
  if (P->d.field_dtype == RTM_F64)
    return tti_adj_impl<double>(P, m, aniso, rec_pos, res, src_pos, qadj, Z, zt, Vbar, work, st);
  return tti_adj_impl<float>(P, m, aniso, rec_pos, res, src_pos, qadj, Z, zt, Vbar, work, st);
}

template <typename T>
static rtm_status tti_grad_impl(const rtm_plan *P, const void *m, const void *aniso,
                                const double *src_pos, const void *q, const double *rec_pos,
                                const void *d_obs, const void *Z, rtm_dtype zt, void *Ubar,
                                void *Vbar, void *resid, void *grad, double *misfit, void *work,
                                hipStream_t st) {
  PointTables<T> src_t, rec_t;
  char *w = static_cast<char *>(work);
  rtm_status s = upload_points<T>(P, w, st, src_pos, &src_t, rec_pos, &rec_t);
  if (s) return s;
  TtiIO f;
  f.m = m;
  f.aniso = aniso;
  f.inj_vals = q;
  f.smp_out = resid;
  f.Z = Z;
  f.zt = zt;
  f.bar = Ubar;
  if ((s = run_tti_sweep<T>(P, f, src_t, rec_t, w, st))) return s;
  double *part = reinterpret_cast<double *>(w + P->red.off);
  HIP_TRY(launch_residual_misfit<T>(static_cast<const T *>(resid), static_cast<const T *>(d_obs),
                                    static_cast<T *>(resid), (int64_t)P->d.nt * P->d.nrec, part,
                                    misfit, st));
  TtiIO b;
  b.adjoint = true;
  b.m = m;
  b.aniso = aniso;
  b.inj_vals = resid;
  b.Z = Z;
  b.zt = zt;
  PointTables<T> none;
  const int64_t barn = (int64_t)P->d.r * P->Npad;
  if (!Vbar) {
    HIP_TRY(launch_fill<T>(static_cast<T *>(grad), P->N, T(0), st));
    b.fuse_U = Ubar;
    b.fuse_img = grad;
    b.fuse_scale = -1.0 / P->d.r;
    if ((s = run_tti_sweep<T>(P, b, rec_t, none, w, st))) return s;
  } else {
    b.bar = Vbar;
    if ((s = run_tti_sweep<T>(P, b, rec_t, none, w, st))) return s;
    // grad = -(1/r) sum_i (Ubar_p Vbar_p + Ubar_q Vbar_q): two images summed
    T *gq = reinterpret_cast<T *>(w + P->total) + (int64_t)(P->R + 5) * P->ld;  // scratch level
    const T *U = static_cast<const T *>(Ubar), *V = static_cast<const T *>(Vbar);
    HIP_TRY(launch_image<T>(U, V, P->N, P->d.r, -1.0 / P->d.r, static_cast<T *>(grad), st));
    HIP_TRY(launch_image<T>(U + barn, V + barn, P->N, P->d.r, -1.0 / P->d.r, gq, st));
    HIP_TRY(launch_axpy<T>(static_cast<T *>(grad), gq, P->N, st));
  }
  HIP_TRY(launch_flag_nonfinite<T>(static_cast<const T *>(grad), P->N, status_word(P, w), st));
  HIP_TRY(launch_flag_nonfinite<double>(misfit, 1, status_word(P, w), st));
  return RTM_OK;
}

template <typename T>
static rtm_status tti_rho_impl(const rtm_plan *P, const void *m, const void *aniso, int iters,
                               uint64_t seed, double *rho, char *w, hipStream_t st) {
  const int64_t N = P->N, ld = P->ld;
  T *ringP = reinterpret_cast<T *>(w + P->ring.off);
  T *ringQ = reinterpret_cast<T *>(w + P->total);
  T *coef = ringQ + (int64_t)P->R * ld;
  T *g = coef + 5 * ld;
  const int shape = (g_stencil_variant == kStencilSimple || ld * (int64_t)sizeof(T) >= (1LL << 32))
                        ? 0 : g_tti_shape;
  StepArgs<T> a = step_args<T>(P, static_cast<const T *>(m));
  HIP_TRY(launch_tti_coef<T>(static_cast<const T *>(aniso), N, coef, st));
  double *part = reinterpret_cast<double *>(w + P->red.off);
  HIP_TRY(tti_power_iteration<T>(a, P->d.h, P->d.dt, coef, ringP, ringQ, ringP + ld, ringQ + ld,
                                 ringP + 2 * ld, ringQ + 2 * ld, g, shape, g_tti_blocks[0], iters,
                                 (uint32_t)(seed ^ (seed >> 32)), part, st));
  double w2 = 0.0;
  HIP_TRY(hipMemcpyAsync(&w2, part + 1024, sizeof w2, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *rho = std::sqrt(w2);
  return RTM_OK;
}

extern "C" rtm_status rtm_tti_spectral_radius(const rtm_plan *P, const void *m, const void *aniso,
                                              int32_t iters, uint64_t seed, double *rho,
                                              void *work, size_t work_bytes, rtm_stream stream) {
  rtm_status s = check_tti(P, m, aniso, work, work_bytes);
  if (s) return s;
  if (!rho) return fail(RTM_E_ARG, "rho is NULL");
  if (iters < 1 || iters > 1000000) return fail(RTM_E_ARG, "iters must be in 1..10^6");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char *w = static_cast<char *>(work);
  if (P->d.field_dtype == RTM_F64)
    return tti_rho_impl<double>(P, m, aniso, iters, seed, rho, w, st);
  return tti_rho_impl<float>(P, m, aniso, iters, seed, rho, w, st);
}

extern "C" rtm_status fwi_gradient_tti(const rtm_plan *P, const void *m, const void *aniso,
                                       const double *src_pos, const void *q,
                                       const double *rec_pos, const void *d_obs, const void *Z,
                                       rtm_dtype zt, void *Ubar, void *Vbar, void *resid,
                                       void *grad, double *misfit, void *work, size_t work_bytes,
                                       rtm_stream stream) {
  rtm_status s = check_tti(P, m, aniso, work, work_bytes);
  if (s) return s;
  if (!src_pos || !q || !rec_pos || !d_obs || !Z || !Ubar || !resid || !grad || !misfit)
    return fail(RTM_E_ARG, "fwi_gradient_tti needs every array except Vbar");
  if (!Vbar && !mfma_probe(P->d.probe_dtype))
    return fail(RTM_E_UNSUPPORTED, "fused imaging (Vbar = NULL) needs an MFMA probe path (BF16, BF16X2 or F16S)");
  if ((s = check_probe(P, Z, zt, Ubar))) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((s = screen_tti(P, m, aniso, work, st))) return s;
  if (P->d.field_dtype == RTM_F64)
    return tti_grad_impl<double>(P, m, aniso, src_pos, q, rec_pos, d_obs, Z, zt, Ubar, Vbar, resid,
                                 grad, misfit, work, st);
  return tti_grad_impl<float>(P, m, aniso, src_pos, q, rec_pos, d_obs, Z, zt, Ubar, Vbar, resid,
                              grad, misfit, work, st);
}
