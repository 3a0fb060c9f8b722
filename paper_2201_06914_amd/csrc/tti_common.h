// Arguments of the pseudo-acoustic TTI step kernels (simple and tiled).
#pragma once
#include "step_common.h"

namespace rtm {

template <typename T>
struct TtiArgs {
  StepArgs<T> a;            // grid, damping, second-difference weights, dt^2
  T d1, d2, d3, d4;         // first-difference weights / h
  T c0;                     // centre weight of one axis' second difference / h^2
  const T *coef;            // [5][N]: c1, c2, n_z, n_y, n_x
  const T *p, *pp, *q, *qp; // current and previous levels
  T *pn, *qn;               // next levels
  T *g;                     // [8][N] intermediates
};

template <typename T>
inline TtiArgs<T> tti_args(const StepArgs<T> &a, T h, const T *coef, const T *p, const T *pp,
                           const T *q, const T *qp, T *pn, T *qn, T *g) {
  TtiArgs<T> t;
  t.a = a;
  t.d1 = (T)(4.0 / 5.0 / (double)h);
  t.d2 = (T)(-1.0 / 5.0 / (double)h);
  t.d3 = (T)(4.0 / 105.0 / (double)h);
  t.d4 = (T)(-1.0 / 280.0 / (double)h);
  t.c0 = (T)(-205.0 / 72.0 / ((double)h * (double)h));
  t.coef = coef;
  t.p = p;
  t.pp = pp;
  t.q = q;
  t.qp = qp;
  t.pn = pn;
  t.qn = qn;
  t.g = g;
  return t;
}

// one step with the tiled kernels (tti_tiled.hip), tile shape 1..3; g needs 6
// slots of N
template <typename T>
hipError_t launch_tti_step_tiled(const TtiArgs<T> &t, bool adjoint, int shape, int target_blocks,
                                 hipStream_t st);

}  // namespace rtm
