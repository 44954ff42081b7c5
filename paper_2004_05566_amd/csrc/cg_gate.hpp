// Convergence test of the preconditioned CG (Algorithm 1), shared by the stand-alone test kernel
// and the first stage of a preconditioner apply that runs the test itself.
#pragma once
#include "kernels.hpp"

namespace hifcn {

// Sum of nb per-block partial sums in one fixed order, computed by one wave (result in lane 0):
// virtual lanes t = 0..255 add part[t], part[t + 256], ... in turn; each run of 64 of them is
// reduced by a shuffle tree and the four run sums are added in order.  This is the order in
// which a 256-lane block reduces the same partials, so the total is the same bits in every
// kernel that tests convergence.  load() issues the loads of the first 512 partials early.
struct CgTotal {
  double v[8];
  __device__ void load(const double* __restrict__ part, int nb) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = lane + 64 * (k & 3) + 256 * (k >> 2);
      v[k] = i < nb ? part[i] : 0.0;
    }
  }
  __device__ double sum(const double* __restrict__ part, int nb) const {
    const int lane = threadIdx.x & 63;
    double s = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      double acc = 0;
      acc += v[w];
      if (lane + 64 * w + 256 < nb) acc += v[w + 4];
      for (int i = lane + 64 * w + 512; i < nb; i += 256) acc += part[i];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
      s += acc;
    }
    return s;
  }
};

// Whether a total of squares is unusable (NaN, or large enough that later products overflow).
__device__ inline bool cg_bad_total(double total) { return !(total == total) || total > 1.7e308; }

// The test once the total is known: init (the right-hand side g just formed): total = ||g||^2,
// the solve ends at once when g = 0 (u = 0, no iteration) or when ||g||^2 is not finite
// (HIF_ERR_NO_CONV after no iteration, u left as it was); otherwise total = ||r||^2 after the
// update of iteration it0 (0-based), tested against rtol^2 ||g||^2, the iteration cap and
// overflow / NaN.
// tol2 and maxit are the state's (read by the caller, possibly ahead of time); for init, maxit is
// the new step's cap.  Returns whether the iteration stops; `publish` (one lane of one block)
// writes the scalars.
__device__ inline bool cg_verdict(CgState* st, int init, int it0, double rtol, double total,
                                  double tol2, int maxit, bool publish) {
  if (init) {  // a new step: its scalars (maxit is the step's cap)
    const bool bad = cg_bad_total(total);
    const bool stop = bad || total == 0.0;
    if (publish) {
      st->gg = total;
      st->tol2 = rtol * rtol * total;
      st->rr = total;
      st->iters = 0;
      st->status = bad ? HIF_ERR_NO_CONV : 0;
      st->maxit = maxit;
      st->done = stop ? 1 : 0;
    }
    return stop;
  }
  const int it = it0 + 1;
  const bool bad = cg_bad_total(total);
  const bool conv = !bad && total <= tol2;
  const bool cap = !bad && !conv && it >= maxit;
  const bool stop = bad || conv || cap;
  if (publish) {
    st->rr = total;
    st->iters = it;
    st->done = stop ? 1 : 0;
    st->status = (bad || cap) ? HIF_ERR_NO_CONV : 0;
  }
  return stop;
}

// The test of a warm-started step (x0 = u^k): gtot = ||g||^2 sets the tolerance, rtot =
// ||r0||^2 = ||g - A u^k||^2 is tested against it; the step ends at once when g = 0 (u = 0),
// when r0 already meets it (u = u^k, no iteration) or when either total is not finite.
__device__ inline bool cg_verdict_warm(CgState* st, double rtol, double gtot, double rtot,
                                       int maxit, bool publish) {
  const bool bad = cg_bad_total(gtot) || cg_bad_total(rtot);
  const double tol2 = rtol * rtol * gtot;
  const bool stop = bad || gtot == 0.0 || rtot <= tol2;
  if (publish) {
    st->gg = gtot;
    st->tol2 = tol2;
    st->rr = rtot;
    st->iters = 0;
    st->status = bad ? HIF_ERR_NO_CONV : 0;
    st->maxit = maxit;
    st->done = stop ? 1 : 0;
  }
  return stop;
}

}  // namespace hifcn
