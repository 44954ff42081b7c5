// The stencil operator's pieces shared by the PCG kernels and the first stage of the apply
// (Sec. 2): the sum over the links of a node and the explicit reaction term (eq1, eq_nr).
//
// Link weights (w = dt / (2 h^2) a_link) are stored per axis: x links n^(DIM-1) rows of n+1
// (link k of a row between nodes k-1 and k), then y links, then (3D) z links, each as
// (n+1) planes/rows of n^(DIM-1) indexed like the nodes (link plane k between node planes k-1
// and k).  Node coordinates come from the kernels' row structure, so no division is needed on
// the hot paths; link_sum() for an arbitrary node derives them in 32-bit arithmetic.
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hifcn {

// Sum over the links of node i = (ix, iy, iz) of w (p_i - p_nbr).  P(k) returns the value at
// node k; neighbours beyond the boundary are the Dirichlet zeros.
// Contraction into fused multiply-adds is off here and in cn_rhs_value: the value of a node must
// not depend on the kernel it is inlined into (the first apply stage and the right-hand-side
// launch form the same g bit for bit).
template <int DIM, typename P>
__device__ __forceinline__ double link_sum_at(int64_t i, int ix, int iy, int iz, int n,
                                              const double* __restrict__ w, double pi, P pv) {
#pragma clang fp contract(off)
  const int64_t n1 = n + 1;
  const int64_t nn = (int64_t)n * n;
  double acc = 0;
  {  // x links
    const int64_t row = DIM == 3 ? (int64_t)iz * n + iy : iy;
    const double* wx = w + row * n1 + ix;
    const double pl = ix > 0 ? pv(i - 1) : 0.0;
    const double pr = ix < n - 1 ? pv(i + 1) : 0.0;
    acc += wx[0] * (pi - pl) + wx[1] * (pi - pr);
  }
  {  // y links
    const int64_t lx = (DIM == 3 ? nn : (int64_t)n) * n1;
    const int64_t b = DIM == 3 ? ((int64_t)iz * n1 + iy) * n + ix : (int64_t)iy * n + ix;
    const double* wy = w + lx + b;
    const double pl = iy > 0 ? pv(i - n) : 0.0;
    const double pr = iy < n - 1 ? pv(i + n) : 0.0;
    acc += wy[0] * (pi - pl) + wy[n] * (pi - pr);
  }
  if (DIM == 3) {  // z links
    const double* wz = w + 2 * nn * n1 + i;
    const double pl = iz > 0 ? pv(i - nn) : 0.0;
    const double pr = iz < n - 1 ? pv(i + nn) : 0.0;
    acc += wz[0] * (pi - pl) + wz[nn] * (pi - pr);
  }
  return acc;
}

// link_sum_at for a node given only by its index (N < 2^31: 32-bit division).
template <int DIM, typename P>
__device__ __forceinline__ double link_sum(int64_t i, int n, const double* __restrict__ w,
                                           double pi, P pv) {
  const int i32 = (int)i;
  const int ix = i32 % n, rest = i32 / n;
  const int iy = DIM == 3 ? rest % n : rest, iz = DIM == 3 ? rest / n : 0;
  return link_sum_at<DIM>(i, ix, iy, iz, n, w, pi, pv);
}

// The coordinates of node i and of the nodes i + stride, i + 2 stride, ... of a grid-stride loop,
// advanced by mixed-radix addition (two divisions at the start, none per node).
template <int DIM>
struct NodeWalk {
  int64_t i;
  int ix, iy, iz;
  int dx, dy, dz;
  int64_t di;
  // start and stride below 2^31 (the grid holds fewer than 2^31 nodes and the launches fewer
  // than 2^31 lanes)
  __device__ __forceinline__ NodeWalk(int64_t start, int64_t stride, int n) : i(start), di(stride) {
    const int s = (int)start, d = (int)stride;
    ix = s % n;
    dx = d % n;
    if (DIM == 2) {
      iy = s / n;
      dy = d / n;
      iz = dz = 0;
    } else {
      iy = s / n % n;
      dy = d / n % n;
      iz = s / n / n;
      dz = d / n / n;
    }
  }
  __device__ __forceinline__ void next(int n) {
    i += di;
    ix += dx;
    int c = ix >= n;
    ix -= c ? n : 0;
    iy += dy + c;
    if (DIM == 3) {
      c = iy >= n;
      iy -= c ? n : 0;
      iz += dz + c;
    }
  }
};

// The reaction r(u): kind 1 is logistic, k1 u (1 - u / k2); kind 0 none.
__device__ __forceinline__ double react(double u, int kind, double k1, double k2) {
#pragma clang fp contract(off)
  return kind == 1 ? k1 * u * (1.0 - u / k2) : 0.0;
}

// g at a node: (I + dt/2 M) u + dt r(u) = u - sum of w (u - u_nbr) + dt r(u)  (eq_CN).
__device__ __forceinline__ double cn_rhs_value(double u, double links, double dt, int kind,
                                               double k1, double k2) {
#pragma clang fp contract(off)
  return u - links + dt * react(u, kind, k1, k2);
}

}  // namespace hifcn
