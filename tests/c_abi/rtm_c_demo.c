/* A plain C client of librtm: no Python, no torch.  It builds a small 3D
 * layered model, allocates device memory with hipMalloc, runs the probed FWI
 * gradient twice (imaging fused into the adjoint probe blocks, and with Vbar
 * stored and imaged separately), checks that the two agree and that the
 * device status word reports finite values, and exercises a host-side
 * rejection.  Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "rtm.h"

#define HIPCHECK(x)                                                     \
  do {                                                                  \
    hipError_t e_ = (x);                                                \
    if (e_ != hipSuccess) {                                             \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));    \
      return 2;                                                         \
    }                                                                   \
  } while (0)
#define RTMCHECK(x)                                                      \
  do {                                                                   \
    rtm_status s_ = (x);                                                 \
    if (s_ != RTM_OK) {                                                  \
      fprintf(stderr, "%s: %s (%s)\n", #x, rtm_status_str(s_), rtm_last_error()); \
      return 3;                                                          \
    }                                                                    \
  } while (0)

int main(void) {
  const int nz = 40, ny = 36, nx = 70, nt = 64, r = 32, k = 16, nrec = 20;
  const double h = 12.5, dt = 1e-3, f0 = 15.0;
  const int64_t N = (int64_t)nz * ny * nx, Npad = (N + 31) / 32 * 32;

  rtm_desc d = {0};
  d.ndim = 3; d.nz = nz; d.ny = ny; d.nx = nx; d.h = h; d.dt = dt; d.nt = nt; d.nb = 4;
  d.c_ref = 3000.0; d.R = 1e-3; d.c_max = 3000.0;
  d.field_dtype = RTM_F32; d.probe_dtype = RTM_BF16X2;
  d.r = r; d.k_block = k; d.nsrc = 1; d.nrec = nrec;

  /* a host-side rejection first: no time steps */
  rtm_desc bad = d;
  rtm_plan *none = NULL;
  bad.nt = 0;
  if (rtm_plan_create(&bad, &none) == RTM_OK) { fprintf(stderr, "nt = 0 accepted\n"); return 4; }

  rtm_plan *plan = NULL;
  RTMCHECK(rtm_plan_create(&d, &plan));
  size_t wbytes = 0;
  RTMCHECK(rtm_plan_workspace_bytes(plan, &wbytes));

  /* host inputs: two layers (2000 / 3000 m/s), a Ricker point source, a
   * line of receivers, +-1 probes from a fixed linear congruential sequence */
  float *m = malloc(sizeof(float) * N), *q = malloc(sizeof(float) * nt);
  int8_t *Z = malloc((size_t)nt * r);
  double src[3] = {8.0, ny / 2, nx / 2}, rec[3 * 20];
  for (int64_t i = 0; i < N; ++i) {
    const int64_t z = i / ((int64_t)ny * nx);
    const double c = z < nz / 2 ? 2000.0 : 3000.0;
    m[i] = (float)(1.0 / (c * c));
  }
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < nt; ++n) {
    const double t = n * dt - 1.0 / f0, a = pi * pi * f0 * f0 * t * t;
    q[n] = (float)((1.0 - 2.0 * a) * exp(-a) / (h * h * h));
  }
  uint32_t lcg = 12345u;
  for (int i = 0; i < nt * r; ++i) {
    lcg = lcg * 1664525u + 1013904223u;
    Z[i] = (lcg >> 31) ? 1 : -1;
  }
  for (int j = 0; j < nrec; ++j) {
    rec[3 * j] = 8.0; rec[3 * j + 1] = ny / 2; rec[3 * j + 2] = 3.0 * j + 5.0;
  }

  float *dm, *dq, *ddobs, *dU, *dV, *dres, *dg1, *dg2;
  int8_t *dZ;
  double *dJ;
  void *work;
  HIPCHECK(hipMalloc((void **)&dm, sizeof(float) * N));
  HIPCHECK(hipMalloc((void **)&dq, sizeof(float) * nt));
  HIPCHECK(hipMalloc((void **)&ddobs, sizeof(float) * nt * nrec));
  HIPCHECK(hipMalloc((void **)&dZ, (size_t)nt * r));
  HIPCHECK(hipMalloc((void **)&dU, sizeof(float) * r * Npad));
  HIPCHECK(hipMalloc((void **)&dV, sizeof(float) * r * Npad));
  HIPCHECK(hipMalloc((void **)&dres, sizeof(float) * nt * nrec));
  HIPCHECK(hipMalloc((void **)&dg1, sizeof(float) * N));
  HIPCHECK(hipMalloc((void **)&dg2, sizeof(float) * N));
  HIPCHECK(hipMalloc((void **)&dJ, sizeof(double)));
  HIPCHECK(hipMalloc(&work, wbytes));
  HIPCHECK(hipMemcpy(dm, m, sizeof(float) * N, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dq, q, sizeof(float) * nt, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dZ, Z, (size_t)nt * r, hipMemcpyHostToDevice));
  HIPCHECK(hipMemset(ddobs, 0, sizeof(float) * nt * nrec));

  double J1 = 0.0, J2 = 0.0;
  RTMCHECK(fwi_gradient(plan, dm, src, dq, rec, ddobs, dZ, RTM_I8, dU, NULL, dres, dg1, dJ,
                        work, wbytes, NULL));
  RTMCHECK(rtm_stream_status(plan, work, NULL));
  HIPCHECK(hipMemcpy(&J1, dJ, sizeof(double), hipMemcpyDeviceToHost));
  RTMCHECK(fwi_gradient(plan, dm, src, dq, rec, ddobs, dZ, RTM_I8, dU, dV, dres, dg2, dJ,
                        work, wbytes, NULL));
  RTMCHECK(rtm_stream_status(plan, work, NULL));
  HIPCHECK(hipMemcpy(&J2, dJ, sizeof(double), hipMemcpyDeviceToHost));
  HIPCHECK(hipDeviceSynchronize());

  float *g1 = malloc(sizeof(float) * N), *g2 = malloc(sizeof(float) * N);
  HIPCHECK(hipMemcpy(g1, dg1, sizeof(float) * N, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(g2, dg2, sizeof(float) * N, hipMemcpyDeviceToHost));
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    num += ((double)g1[i] - g2[i]) * ((double)g1[i] - g2[i]);
    den += (double)g2[i] * g2[i];
  }
  const double rel = sqrt(num / den);
  printf("misfit %.9e %.9e  |grad| %.6e  fused vs separate imaging rel %.3e\n", J1, J2,
         sqrt(den), rel);

  hipFree(dm); hipFree(dq); hipFree(ddobs); hipFree(dZ); hipFree(dU); hipFree(dV);
  hipFree(dres); hipFree(dg1); hipFree(dg2); hipFree(dJ); hipFree(work);
  free(m); free(q); free(Z); free(g1); free(g2);
  rtm_plan_destroy(plan);
  return (J1 == J2 && den > 0.0 && rel < 1e-4) ? 0 : 1;
}
