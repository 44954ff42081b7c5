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

// Sum over the links of a node of w (p_i - p_nbr) from the values at hand: the x links (l, r),
// the y links (d, u) and, in 3D, the z links (b, f), in that order.
template <int DIM>
__device__ __forceinline__ double link_sum_vals(double pi, double pl, double pr, double wl,
                                                double wr, double pd, double pu, double wd,
                                                double wu, double pb = 0, double pf = 0,
                                                double wb = 0, double wf = 0) {
#pragma clang fp contract(off)
  double acc = 0;
  acc += wl * (pi - pl) + wr * (pi - pr);
  acc += wd * (pi - pd) + wu * (pi - pu);
  if (DIM == 3) acc += wb * (pi - pb) + wf * (pi - pf);
  return acc;
}

// Sum over the links of node i = (ix, iy, iz) of w (p_i - p_nbr).  P(k) returns the value at
// node k; neighbours beyond the boundary are the Dirichlet zeros.
// Contraction into fused multiply-adds is off here and in cn_rhs_value: the value of a node must
// not depend on the kernel it is inlined into (the first apply stage and the right-hand-side
// launch form the same g bit for bit).
template <int DIM, typename P>
__device__ __forceinline__ double link_sum_at(int64_t i, int ix, int iy, int iz, int n,
                                              const double* __restrict__ w, double pi, P pv) {
  const int64_t n1 = n + 1;
  const int64_t nn = (int64_t)n * n;
  const int64_t row = DIM == 3 ? (int64_t)iz * n + iy : iy;
  const double* wx = w + row * n1 + ix;
  const double pl = ix > 0 ? pv(i - 1) : 0.0;
  const double pr = ix < n - 1 ? pv(i + 1) : 0.0;
  const int64_t lx = (DIM == 3 ? nn : (int64_t)n) * n1;
  const int64_t b = DIM == 3 ? ((int64_t)iz * n1 + iy) * n + ix : (int64_t)iy * n + ix;
  const double* wy = w + lx + b;
  const double pd = iy > 0 ? pv(i - n) : 0.0;
  const double pu = iy < n - 1 ? pv(i + n) : 0.0;
  if (DIM == 3) {
    const double* wz = w + 2 * nn * n1 + i;
    const double pb = iz > 0 ? pv(i - nn) : 0.0;
    const double pf = iz < n - 1 ? pv(i + nn) : 0.0;
    return link_sum_vals<3>(pi, pl, pr, wx[0], wx[1], pd, pu, wy[0], wy[n], pb, pf, wz[0],
                            wz[nn]);
  }
  return link_sum_vals<2>(pi, pl, pr, wx[0], wx[1], pd, pu, wy[0], wy[n]);
}

// The link sums of the two nodes i, i + 1 of an x-pair (n even, i and ix even, so the pair is
// in one row and every pair-wide load is 16-byte aligned): (s0, s1), each as link_sum_at forms
// it.  v = (p_i, p_{i+1}); P(k) and P2(k) return the value at node k and the pair at k, k + 1.
template <int DIM, typename P, typename P2>
__device__ __forceinline__ void link_sum_pair(int64_t i, int ix, int iy, int iz, int n,
                                              const double* __restrict__ w, double2 v, P pv,
                                              P2 pv2, double& s0, double& s1) {
  const int64_t n1 = n + 1;
  const int64_t nn = (int64_t)n * n;
  const double2 zero{0.0, 0.0};
  const int64_t row = DIM == 3 ? (int64_t)iz * n + iy : iy;
  const double* wx = w + row * n1 + ix;
  const double wx0 = wx[0], wx1 = wx[1], wx2 = wx[2];
  const double pl = ix > 0 ? pv(i - 1) : 0.0;
  const double pr = ix + 2 < n ? pv(i + 2) : 0.0;
  const int64_t lx = (DIM == 3 ? nn : (int64_t)n) * n1;
  const int64_t b = DIM == 3 ? ((int64_t)iz * n1 + iy) * n + ix : (int64_t)iy * n + ix;
  const double2 wd = *reinterpret_cast<const double2*>(w + lx + b);
  const double2 wu = *reinterpret_cast<const double2*>(w + lx + b + n);
  const double2 pd = iy > 0 ? pv2(i - n) : zero;
  const double2 pu = iy < n - 1 ? pv2(i + n) : zero;
  if (DIM == 3) {
    const double2 wb = *reinterpret_cast<const double2*>(w + 2 * nn * n1 + i);
    const double2 wf = *reinterpret_cast<const double2*>(w + 2 * nn * n1 + i + nn);
    const double2 pb = iz > 0 ? pv2(i - nn) : zero;
    const double2 pf = iz < n - 1 ? pv2(i + nn) : zero;
    s0 = link_sum_vals<3>(v.x, pl, v.y, wx0, wx1, pd.x, pu.x, wd.x, wu.x, pb.x, pf.x, wb.x,
                          wf.x);
    s1 = link_sum_vals<3>(v.y, v.x, pr, wx1, wx2, pd.y, pu.y, wd.y, wu.y, pb.y, pf.y, wb.y,
                          wf.y);
  } else {
    s0 = link_sum_vals<2>(v.x, pl, v.y, wx0, wx1, pd.x, pu.x, wd.x, wu.x);
    s1 = link_sum_vals<2>(v.y, v.x, pr, wx1, wx2, pd.y, pu.y, wd.y, wu.y);
  }
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
