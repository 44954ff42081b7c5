// The stencil operator's pieces shared by the PCG kernels and the first stage of the apply
// (Sec. 2): the sum over the links of a node and the explicit reaction term (eq1, eq_nr).
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hifcn {

// Sum over links of w (p_j - p_nbr) at node i.  P(k) returns the value at node k.
template <int DIM, typename P>
__device__ __forceinline__ double link_sum(int64_t i, int n, const double* __restrict__ w,
                                           double pi, P pv) {
  const int64_t n1 = n + 1;
  const int64_t nn = (int64_t)n * n;
  int ix = (int)(i % n);
  int64_t rest = i / n;
  int iy = (int)(rest % n);
  int iz = DIM == 3 ? (int)(rest / n) : 0;
  double acc = 0;
  // x links: array (.., n+1) with link k between nodes k-1 and k
  {
    const int64_t row = DIM == 3 ? ((int64_t)iz * n + iy) : iy;
    const double* wx = w + row * n1;
    const double wl = wx[ix], wr = wx[ix + 1];
    const double pl = ix > 0 ? pv(i - 1) : 0.0;
    const double pr = ix < n - 1 ? pv(i + 1) : 0.0;
    acc += wl * (pi - pl) + wr * (pi - pr);
  }
  {
    const int64_t lx = (DIM == 3 ? nn : (int64_t)n) * n1;  // size of the x-link array
    const double* wy = w + lx;
    const int64_t b = DIM == 3 ? ((int64_t)iz * n1 + iy) * n + ix : (int64_t)iy * n + ix;
    const double wl = wy[b], wr = wy[b + n];
    const double pl = iy > 0 ? pv(i - n) : 0.0;
    const double pr = iy < n - 1 ? pv(i + n) : 0.0;
    acc += wl * (pi - pl) + wr * (pi - pr);
  }
  if (DIM == 3) {
    const int64_t lx = nn * n1;
    const double* wz = w + 2 * lx;
    const int64_t b = ((int64_t)iz * n + iy) * n + ix;
    const double wl = wz[b], wr = wz[b + nn];
    const double pl = iz > 0 ? pv(i - nn) : 0.0;
    const double pr = iz < n - 1 ? pv(i + nn) : 0.0;
    acc += wl * (pi - pl) + wr * (pi - pr);
  }
  return acc;
}

// The reaction r(u): kind 1 is logistic, k1 u (1 - u / k2); kind 0 none.
__device__ __forceinline__ double react(double u, int kind, double k1, double k2) {
  return kind == 1 ? k1 * u * (1.0 - u / k2) : 0.0;
}

}  // namespace hifcn
