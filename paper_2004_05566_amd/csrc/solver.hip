// Stencil operator and preconditioned CG kernels (Sec. 2, Sec. 2.1, Algorithm 1).
//
// A = I - dt/2 M with M the five/seven-point variable-coefficient stencil: with link weights
// w = dt/(2 h^2) a_link, (A p)_j = p_j + sum_links w (p_j - p_nbr) and (I + dt/2 M) u =
// u - sum_links w (u_j - u_nbr) (Dirichlet: p = 0 beyond the boundary).
//
// PCG keeps every scalar on the device (CgState), so a whole iteration is queued without a
// host round trip.  The iteration is arranged with one reduction phase between the
// preconditioner and the update (the single-reduction form of Chronopoulos and Gear): the SpMV
// is applied to z (w = A z) together with the partial sums of r.z, z.w and z.q (q = A p of the
// previous direction); the update then forms beta = rho / rho_prev, p.Ap = z.w + 2 beta z.q +
// beta^2 p_prev.A p_prev (A is symmetric), alpha = rho / p.Ap, p = z + beta p, q = w + beta q,
// x += alpha p, r -= alpha q: the iterates of Algorithm 1 in exact arithmetic.  Reductions are
// deterministic two-level sums (per-block partials, re-added in a fixed order by the kernel that
// consumes them), and the convergence test ||r|| <= rtol ||g|| sets a device flag that makes
// every later kernel of the step return.
#include "common.hpp"
#include "kernels.hpp"
#include "cg_gate.hpp"
#include "stencil.hpp"

#include <cstdint>
#include <cstdlib>
#include <initializer_list>

namespace hifcn {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Per-block partial sums: every reduction kernel writes one partial per block; the kernel that
// needs the total re-adds all partials in the same fixed order in every block, so the result is
// deterministic and no inter-block synchronisation (fences, atomics) is needed inside a kernel.
__device__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  return s;
}

__device__ void put_partial(double v, double* part) {
  const double s = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ double total(const double* part, int nb) {
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += part[i];
  return block_sum(acc);
}

// ---- link weights from cell values: mean of the 2 (2D) / 4 (3D) cells sharing the link ------
__global__ void k_links2d(const double* __restrict__ a, int n, double scale, double* __restrict__ w) {
  const int64_t n1 = n + 1;
  const int64_t per = (int64_t)n * n1;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 2 * per;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t < per) {  // x link k at node row iy: cells (cy in {iy, iy+1}, cx = k)
      const int64_t iy = t / n1, k = t % n1;
      w[t] = scale * 0.5 * (a[iy * n1 + k] + a[(iy + 1) * n1 + k]);
    } else {        // y link k at node column ix: cells (cy = k, cx in {ix, ix+1})
      const int64_t u = t - per, k = u / n, ix = u % n;
      w[t] = scale * 0.5 * (a[k * n1 + ix] + a[k * n1 + ix + 1]);
    }
  }
}

__global__ void k_links3d(const double* __restrict__ a, int n, double scale, double* __restrict__ w) {
  const int64_t n1 = n + 1;
  const int64_t per = (int64_t)n * n * n1;
  auto A = [&](int64_t cz, int64_t cy, int64_t cx) { return a[(cz * n1 + cy) * n1 + cx]; };
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 3 * per;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int axis = (int)(t / per);
    const int64_t u = t - axis * per;
    double s;
    if (axis == 0) {         // (iz, iy, k)
      const int64_t k = u % n1, r = u / n1, iy = r % n, iz = r / n;
      s = A(iz, iy, k) + A(iz, iy + 1, k) + A(iz + 1, iy, k) + A(iz + 1, iy + 1, k);
    } else if (axis == 1) {  // (iz, k, ix)
      const int64_t ix = u % n, r = u / n, k = r % n1, iz = r / n1;
      s = A(iz, k, ix) + A(iz, k, ix + 1) + A(iz + 1, k, ix) + A(iz + 1, k, ix + 1);
    } else {                 // (k, iy, ix)
      const int64_t ix = u % n, r = u / n, iy = r % n, k = r / n;
      s = A(k, iy, ix) + A(k, iy, ix + 1) + A(k, iy + 1, ix) + A(k, iy + 1, ix + 1);
    }
    w[t] = scale * 0.25 * s;
  }
}

// y = A x, two nodes per lane per turn (i and i + stride) so that both nodes' loads are in
// flight together; node coordinates by NodeWalk (no division per node).
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_spmv(int n, int64_t N, const double* __restrict__ w,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  NodeWalk<DIM> a(blockIdx.x * (int64_t)kThreads + threadIdx.x, 2 * stride, n);
  NodeWalk<DIM> b(a.i + stride, 2 * stride, n);
  auto X = [&](int64_t k) { return x[k]; };
  for (; b.i < N; a.next(n), b.next(n)) {
    const double xa = x[a.i], xb = x[b.i];
    const double la = link_sum_at<DIM>(a.i, a.ix, a.iy, a.iz, n, w, xa, X);
    const double lb = link_sum_at<DIM>(b.i, b.ix, b.iy, b.iz, n, w, xb, X);
    y[a.i] = xa + la;
    y[b.i] = xb + lb;
  }
  if (a.i < N) {
    const double xa = x[a.i];
    y[a.i] = xa + link_sum_at<DIM>(a.i, a.ix, a.iy, a.iz, n, w, xa, X);
  }
}


// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD b mod 8), each XCD
// with its own L2.  The stencil kernels give each XCD a contiguous run of chunks instead, so the
// rows above and below a chunk are mostly read through the same L2 (a bijection of [0, nb)).
__device__ __forceinline__ int xcd_chunk(int b, int nb) {
  const int per = nb / 8;
  return b < 8 * per ? (b % 8) * per + b / 8 : b;
}

// y = A x over x-pairs of nodes (n even): one 16-byte load of the pair, of each neighbouring
// pair across y (and z) and of the pair's y (z) link weights, instead of one load per node and
// neighbour.  Each node's value is the arithmetic of link_sum_at.
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_spmv_pairs(int n, int64_t N,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const double2* x2 = reinterpret_cast<const double2*>(x);
  double2* y2 = reinterpret_cast<double2*>(y);
  auto X = [&](int64_t k) { return x[k]; };
  auto X2 = [&](int64_t k) { return x2[k >> 1]; };
  for (NodeWalk<DIM> a(2 * (xcd_chunk(blockIdx.x, gridDim.x) * (int64_t)kThreads + threadIdx.x),
                          2 * stride, n);
       a.i < N; a.next(n)) {
    const double2 v = x2[a.i >> 1];
    double s0, s1;
    link_sum_pair<DIM>(a.i, a.ix, a.iy, a.iz, n, w, v, X, X2, s0, s1);
    y2[a.i >> 1] = double2{v.x + s0, v.y + s1};
  }
}

// Partial-sum slots (each nblk long): ||g||^2, ||r||^2, and the direction kernel's r.z, z.w, z.q.
enum { P_GG = 0, P_RR = 1, P_RZ = 2, P_ZW = 3, P_ZQ = 4, P_SLOTS = 5 };

// Three block sums at once (one pair of barriers); valid in every lane.
__device__ void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  __syncthreads();
  if (lane == 0) {
    red[0][wid] = a;
    red[1][wid] = b;
    red[2][wid] = c;
  }
  __syncthreads();
  a = b = c = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    a += red[0][w];
    b += red[1][w];
    c += red[2][w];
  }
}

// g = (I + dt/2 M) u + dt r(u) -> r; x = 0; partials of ||g||^2 (the test of g that follows
// resets the step's scalars).
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_cg_rhs(int n, int64_t N, const double* __restrict__ w,
                                                     const double* __restrict__ u,
                                                     double* __restrict__ r, double* __restrict__ x,
                                                     int kind, double k1, double k2, double dt,
                                                     int ahead, int warm, CgState* st,
                                                     double* part) {
  // queued ahead of the previous step's outcome: nothing to do unless that step ended well
  // (every block reads the same two fields, which no block writes here)
  const bool held = ahead && (!st->done || st->status);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->hold = held ? 1 : 0;
  if (held) return;
  double acc = 0, accr = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (NodeWalk<DIM> a(blockIdx.x * (int64_t)kThreads + threadIdx.x, stride, n); a.i < N;
       a.next(n)) {
    const int64_t i = a.i;
    const double ui = u[i];
    const double sl = link_sum_at<DIM>(i, a.ix, a.iy, a.iz, n, w, ui,
                                       [&](int64_t k) { return u[k]; });
    const double g = cn_rhs_value(ui, sl, dt, kind, k1, k2);
    // warm start: r0 = g - A u (A u = u + the link sum), x0 = 0 for the correction
    const double r0 = warm ? g - (ui + sl) : g;
    r[i] = r0;
    x[i] = 0.0;
    acc += g * g;
    accr += r0 * r0;
  }
  put_partial(acc, part + P_GG * (int64_t)gridDim.x);
  if (warm) put_partial(accr, part + P_RR * (int64_t)gridDim.x);
}

// k_cg_rhs over x-pairs of nodes (n even; see k_spmv_pairs): the same g at every node.
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_cg_rhs_pairs(int n, int64_t N,
                                                           const double* __restrict__ w,
                                                           const double* __restrict__ u,
                                                           double* __restrict__ r,
                                                           double* __restrict__ x, int kind,
                                                           double k1, double k2, double dt,
                                                           int ahead, int warm, CgState* st,
                                                           double* part) {
  const bool held = ahead && (!st->done || st->status);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->hold = held ? 1 : 0;
  if (held) return;
  double acc = 0, accr = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const double2* u2 = reinterpret_cast<const double2*>(u);
  auto U = [&](int64_t k) { return u[k]; };
  auto U2 = [&](int64_t k) { return u2[k >> 1]; };
  for (NodeWalk<DIM> a(2 * (xcd_chunk(blockIdx.x, gridDim.x) * (int64_t)kThreads + threadIdx.x),
                          2 * stride, n);
       a.i < N; a.next(n)) {
    const double2 v = u2[a.i >> 1];
    double s0, s1;
    link_sum_pair<DIM>(a.i, a.ix, a.iy, a.iz, n, w, v, U, U2, s0, s1);
    const double g0 = cn_rhs_value(v.x, s0, dt, kind, k1, k2);
    const double g1 = cn_rhs_value(v.y, s1, dt, kind, k1, k2);
    const double r0 = warm ? g0 - (v.x + s0) : g0, r1 = warm ? g1 - (v.y + s1) : g1;
    reinterpret_cast<double2*>(r)[a.i >> 1] = double2{r0, r1};
    reinterpret_cast<double2*>(x)[a.i >> 1] = double2{0.0, 0.0};
    acc += g0 * g0;
    acc += g1 * g1;
    accr += r0 * r0;
    accr += r1 * r1;
  }
  put_partial(acc, part + P_GG * (int64_t)gridDim.x);
  if (warm) put_partial(accr, part + P_RR * (int64_t)gridDim.x);
}

__global__ void k_cg_resume(CgState* st) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->hold = 0;
  }
}

// Convergence test, then z = r if the iteration goes on.  init: ||g||^2 is finalised (g = 0
// ends the solve at once); otherwise ||r||^2 of the update just made is finalised and the
// iteration count advanced.  Block 0 publishes the scalars; every block reaches the same verdict.
// `it` is the 0-based index of the iteration whose update was just made (ignored for init);
// it comes from the host so that no block reads a scalar that block 0 rewrites in this launch.
// With hflag, block 0 also posts the outcome to the host as one aligned 64-bit store (seen
// whole or not at all): seq in the high word, iters | done << 24 | status << 28 in the low one.
// The word of sequence number seq is hflag[8 + 2 (seq & 1)].
__device__ void post_flag(int32_t* hflag, int seq, int iters, int done, int status) {
  const uint64_t lo = (uint32_t)iters | (uint32_t)done << 24 | (uint32_t)status << 28;
  *reinterpret_cast<volatile uint64_t*>(hflag + 8 + 2 * (seq & 1)) =
      (uint64_t)(uint32_t)seq << 32 | lo;
}

// The end of a CN step: u = x, and the iteration count and relative residual ||r|| / ||g|| of
// step `step` recorded (block 0).  x0: the lane's first element of x, loaded already.  keep_u:
// the step failed before its first iteration (a non-finite right-hand side), so u stays.  warm:
// x is the correction of a step started from u^k, so u = u^k + x (u = 0 when g = 0).
__device__ void finish_step(int64_t N, const double* __restrict__ x, double* __restrict__ u,
                            int iters, double rr, double gg, int32_t* it_out, double* rel_out,
                            int step, double x0, bool keep_u = false, bool warm = false) {
  const int64_t i0 = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (!keep_u && !warm)
    for (int64_t i = i0; i < N; i += (int64_t)gridDim.x * kThreads) u[i] = i == i0 ? x0 : x[i];
  if (!keep_u && warm)  // u^k + the correction, or 0 when g = 0
    for (int64_t i = i0; i < N; i += (int64_t)gridDim.x * kThreads)
      u[i] = gg == 0.0 ? 0.0 : u[i] + (i == i0 ? x0 : x[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    it_out[step] = iters;
    rel_out[step] = gg > 0 ? sqrt(rr / gg) : 0.0;
  }
}

// The convergence test closing a queued batch of iterations (fin != nullptr) also ends the step
// when the iteration stops, here or at an earlier test of the batch: finish_step, then the post
// to the host (block 0).  A closing test that finds hold set belongs to a step queued ahead of
// one that did not end well, and does nothing.  warm: the step started from x0 = u^k (its
// initial test takes ||g||^2 and ||r0||^2; its end adds the correction to u).
struct CgFinish {
  int32_t* hflag;
  int seq;
  const double* x;
  double* u;
  int32_t* it_out;
  double* rel_out;
  int step;
};

__global__ __launch_bounds__(kThreads) void k_cg_check_copy(int64_t N, int init, int it0,
                                                            double rtol, int maxit,
                                                            const double* __restrict__ r,
                                                            double* __restrict__ z, CgState* st,
                                                            const double* __restrict__ part,
                                                            CgFinish fin, int warm) {
  __shared__ int stop;
  const bool post = fin.hflag && blockIdx.x == 0 && threadIdx.x == 0;
  // the lane's first elements of r (z = r, as a 16-byte pair) and x (u = x) load with the flags
  // and partials
  const int64_t i0 = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int64_t N2 = N / 2;
  const double2* __restrict__ r2 = reinterpret_cast<const double2*>(r);
  double x0 = 0;
  double2 rp{0, 0};
  if (i0 < N2) rp = r2[i0];
  if (i0 < N && fin.hflag) x0 = fin.x[i0];
  if (fin.hflag && st->hold) return;  // queued ahead of a step that did not end well
  if (init) {  // the test of the right-hand side publishes the state of the new step
    if (st->hold) {  // (queued ahead, see k_cg_rhs): later kernels of the step do nothing
      if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 1;
      return;
    }
  } else if (st->done) {  // stopped by an earlier test of the batch
    if (fin.hflag) {
      finish_step(N, fin.x, fin.u, st->iters, st->rr, st->gg, fin.it_out, fin.rel_out, fin.step,
                  x0, st->status != 0 && st->iters == 0, warm != 0);
      if (post) {
        st->ok_next = st->status == 0;
        post_flag(fin.hflag, fin.seq, st->iters, 1, st->status);
      }
    }
    return;
  }
  const int nb = gridDim.x;
  if (threadIdx.x < 64) {
    CgTotal ct;
    const double* p = part + (init ? P_GG : P_RR) * (int64_t)nb;
    ct.load(p, nb);
    const double t = ct.sum(p, nb);
    if (init && warm) {  // the test of r0 = g - A u^k against rtol ||g|| (g's total above)
      CgTotal cr;
      const double* q = part + P_RR * (int64_t)nb;
      cr.load(q, nb);
      const double tr = cr.sum(q, nb);
      if (threadIdx.x == 0) stop = cg_verdict_warm(st, rtol, t, tr, maxit, blockIdx.x == 0);
    } else if (threadIdx.x == 0) {
      stop = cg_verdict(st, init, it0, rtol, t, st->tol2, init ? maxit : st->maxit,
                        blockIdx.x == 0);
    }
  }
  __syncthreads();
  if (stop) {
    if (fin.hflag) {
      // block 0 wrote the scalars it reads here; other blocks only copy x
      finish_step(N, fin.x, fin.u, it0 + 1, st->rr, st->gg, fin.it_out, fin.rel_out, fin.step,
                  x0, false, warm != 0);
      if (post) {
        st->ok_next = st->status == 0;
        post_flag(fin.hflag, fin.seq, st->iters, 1, st->status);
      }
    }
    return;
  }
  if (post) {
    st->ok_next = 0;
    post_flag(fin.hflag, fin.seq, it0 + 1, 0, 0);
  }
  // z = r in 16-byte pairs, four in flight per lane (r and z are 16-byte aligned)
  double2* __restrict__ z2 = reinterpret_cast<double2*>(z);
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  if (i0 < N2) z2[i0] = rp;
  int64_t i = i0 + stride;
  for (; i + 3 * stride < N2; i += 4 * stride) {
    const double2 a = r2[i], b = r2[i + stride], c = r2[i + 2 * stride], d = r2[i + 3 * stride];
    z2[i] = a;
    z2[i + stride] = b;
    z2[i + 2 * stride] = c;
    z2[i + 3 * stride] = d;
  }
  for (; i < N2; i += stride) z2[i] = r2[i];
  if ((N & 1) && i0 == 0) z[N - 1] = r[N - 1];
}

// w = A z and the partial sums of r.z, z.w and (after the first iteration) z.q.  Runs whether
// or not the iteration has stopped: its outputs are scratch that nothing reads once it has, and
// not waiting for the flag lets the first loads go out at once.
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_cg_dir_dots(int n, int64_t N, int it,
                                                          const double* __restrict__ lw,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ r,
                                                          const double* __restrict__ q,
                                                          double* __restrict__ w,
                                                          double* part) {
  const int nb = gridDim.x;
  double rz = 0, zw = 0, zq = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  auto Z = [&](int64_t k) { return z[k]; };
  NodeWalk<DIM> a(blockIdx.x * (int64_t)kThreads + threadIdx.x, 2 * stride, n);
  NodeWalk<DIM> b(a.i + stride, 2 * stride, n);
  auto one = [&](const NodeWalk<DIM>& c, double zi, double ri, double qi) {
    const double wi = zi + link_sum_at<DIM>(c.i, c.ix, c.iy, c.iz, n, lw, zi, Z);
    w[c.i] = wi;
    rz += ri * zi;
    zw += zi * wi;
    if (it > 0) zq += zi * qi;
  };
  // nodes in the order i, i + stride, i + 2 stride, ... as a one-node loop would take them
  for (; b.i < N; a.next(n), b.next(n)) {
    const double za = z[a.i], zb = z[b.i], ra = r[a.i], rb = r[b.i];
    const double qa = it > 0 ? q[a.i] : 0.0, qb = it > 0 ? q[b.i] : 0.0;
    one(a, za, ra, qa);
    one(b, zb, rb, qb);
  }
  if (a.i < N) one(a, z[a.i], r[a.i], it > 0 ? q[a.i] : 0.0);
  block_sum3(rz, zw, zq);
  if (threadIdx.x == 0) {
    part[P_RZ * (int64_t)nb + blockIdx.x] = rz;
    part[P_ZW * (int64_t)nb + blockIdx.x] = zw;
    part[P_ZQ * (int64_t)nb + blockIdx.x] = zq;
  }
}

// k_cg_dir_dots over x-pairs of nodes (n even; see k_spmv_pairs), two pairs per lane and turn
// (their loads in flight together).
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_cg_dir_dots_pairs(int n, int64_t N, int it,
                                                                const double* __restrict__ lw,
                                                                const double* __restrict__ z,
                                                                const double* __restrict__ r,
                                                                const double* __restrict__ q,
                                                                double* __restrict__ w,
                                                                double* part) {
  const int nb = gridDim.x;
  double rz = 0, zw = 0, zq = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const double2* z2 = reinterpret_cast<const double2*>(z);
  auto Z = [&](int64_t k) { return z[k]; };
  auto Z2 = [&](int64_t k) { return z2[k >> 1]; };
  auto one = [&](const NodeWalk<DIM>& c) {
    const int64_t h = c.i >> 1;
    const double2 zv = z2[h];
    const double2 rv = reinterpret_cast<const double2*>(r)[h];
    const double2 qv = it > 0 ? reinterpret_cast<const double2*>(q)[h] : double2{0.0, 0.0};
    double s0, s1;
    link_sum_pair<DIM>(c.i, c.ix, c.iy, c.iz, n, lw, zv, Z, Z2, s0, s1);
    const double w0 = zv.x + s0, w1 = zv.y + s1;
    reinterpret_cast<double2*>(w)[h] = double2{w0, w1};
    rz += rv.x * zv.x;
    rz += rv.y * zv.y;
    zw += zv.x * w0;
    zw += zv.y * w1;
    zq += zv.x * qv.x;
    zq += zv.y * qv.y;
  };
  // pairs in the order t, t + stride, t + 2 stride, ... (t: this lane's first pair)
  NodeWalk<DIM> a(2 * (xcd_chunk(blockIdx.x, gridDim.x) * (int64_t)kThreads + threadIdx.x),
                  4 * stride, n);
  NodeWalk<DIM> b(a.i + 2 * stride, 4 * stride, n);
  for (; b.i < N; a.next(n), b.next(n)) {
    one(a);
    one(b);
  }
  if (a.i < N) one(a);
  block_sum3(rz, zw, zq);
  if (threadIdx.x == 0) {
    part[P_RZ * (int64_t)nb + blockIdx.x] = rz;
    part[P_ZW * (int64_t)nb + blockIdx.x] = zw;
    part[P_ZQ * (int64_t)nb + blockIdx.x] = zq;
  }
}

// The update's scalars from this iteration's partial sums (every block adds them up in the same
// order): beta, alpha; with gpart, the test of g first (it may stop the step: dn).  Block 0
// records rho and p.Ap for the next direction and, with gpart, the step's ||g||^2 and tolerance.
struct CgCoef {
  double alpha, beta;
  int dn;
};
__device__ CgCoef cg_coef(int it, CgState* st, const double* part, const double* gpart, int ngp,
                          double rtol, int dn) {
  const int nb = gridDim.x;
  const bool first = it == 0;
  double rz = 0, zw = 0, zq = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    rz += part[P_RZ * (int64_t)nb + i];
    zw += part[P_ZW * (int64_t)nb + i];
    zq += part[P_ZQ * (int64_t)nb + i];
  }
  double gg = 0, unused = 0, unused2 = 0;
  if (gpart)  // the test of g of a step whose right-hand side the apply made
    for (int i = threadIdx.x; i < ngp; i += kThreads) gg += gpart[i];
  block_sum3(rz, zw, zq);
  if (gpart) {
    block_sum3(gg, unused, unused2);
    // g = 0: u = 0 after no iteration; ||g||^2 not finite: HIF_ERR_NO_CONV after none
    const bool bad = cg_bad_total(gg);
    if (blockIdx.x == 0 && threadIdx.x == 0 && !dn) {
      st->gg = gg;
      st->tol2 = rtol * rtol * gg;
      st->rr = gg;
      if (bad || gg == 0.0) st->done = 1;
      if (bad) st->status = HIF_ERR_NO_CONV;
    }
    if (bad || gg == 0.0) dn = 1;
  }
  const double beta = first ? 0.0 : rz / st->rzv[(it + 1) & 1];
  const double pq = first ? zw : zw + beta * (2.0 * zq + beta * st->pqv[(it + 1) & 1]);
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0 && !dn) {
    st->rzv[it & 1] = rz;
    st->pqv[it & 1] = pq;
  }
  return CgCoef{alpha, beta, dn};
}

__global__ __launch_bounds__(kThreads) void k_cg_update(int64_t N, int it,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ p,
                                                        double* __restrict__ q,
                                                        double* __restrict__ x,
                                                        double* __restrict__ r, CgState* st,
                                                        double* part,
                                                        const double* __restrict__ gpart, int ngp,
                                                        double rtol) {
  const int dn0 = st->done;
  const int nb = gridDim.x;
  const bool first = it == 0;
  // the lane's first element is loaded before the totals, so its latency overlaps theirs
  const int64_t i0 = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  double z0 = 0, w0 = 0, p0 = 0, q0 = 0, x0 = 0, r0 = 0;
  if (i0 < N) {
    z0 = z[i0];
    w0 = w[i0];
    if (!first) {
      p0 = p[i0];
      q0 = q[i0];
    }
    x0 = x[i0];
    r0 = r[i0];
  }
  const CgCoef c = cg_coef(it, st, part, gpart, ngp, rtol, dn0);
  const double alpha = c.alpha, beta = c.beta;
  const int dn = c.dn;
  double acc = 0;
  for (int64_t i = i0; i < N; i += (int64_t)gridDim.x * kThreads) {
    const bool pre = i == i0;
    const double zi = pre ? z0 : z[i], wi = pre ? w0 : w[i];
    const double pi = first ? zi : zi + beta * (pre ? p0 : p[i]);
    const double qi = first ? wi : wi + beta * (pre ? q0 : q[i]);
    const double xi = (pre ? x0 : x[i]) + alpha * pi;
    const double ri = (pre ? r0 : r[i]) - alpha * qi;
    acc += ri * ri;
    if (!dn) {
      p[i] = pi;
      q[i] = qi;
      x[i] = xi;
      r[i] = ri;
    }
  }
  put_partial(acc, part + P_RR * (int64_t)nb);
}

// k_cg_update over pairs of elements (N even, 16-byte aligned vectors): two pairs per lane and
// turn, every load of both issued before the first store, so twice the bytes are in flight.
__global__ __launch_bounds__(kThreads) void k_cg_update_pairs(int64_t N, int it,
                                                              const double* __restrict__ z,
                                                              const double* __restrict__ w,
                                                              double* __restrict__ p,
                                                              double* __restrict__ q,
                                                              double* __restrict__ x,
                                                              double* __restrict__ r,
                                                              CgState* st, double* part,
                                                              const double* __restrict__ gpart,
                                                              int ngp, double rtol) {
  const int dn0 = st->done;
  const int nb = gridDim.x;
  const bool first = it == 0;
  const int64_t H = N / 2, S = (int64_t)gridDim.x * kThreads;
  const double2* z2 = reinterpret_cast<const double2*>(z);
  const double2* w2 = reinterpret_cast<const double2*>(w);
  double2* p2 = reinterpret_cast<double2*>(p);
  double2* q2 = reinterpret_cast<double2*>(q);
  double2* x2 = reinterpret_cast<double2*>(x);
  double2* r2 = reinterpret_cast<double2*>(r);
  const double2 zero{0.0, 0.0};
  // the lane's first two pairs are loaded before the totals, so their latency overlaps theirs
  const int64_t h0 = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  double2 zv[2], wv[2], pv[2], qv[2], xv[2], rv[2];
  auto load = [&](int64_t h0_, int u) {
    const int64_t h = h0_ + u * S;
    if (h < H) {
      zv[u] = z2[h];
      wv[u] = w2[h];
      pv[u] = first ? zero : p2[h];
      qv[u] = first ? zero : q2[h];
      xv[u] = x2[h];
      rv[u] = r2[h];
    }
  };
  load(h0, 0);
  load(h0, 1);
  const CgCoef c = cg_coef(it, st, part, gpart, ngp, rtol, dn0);
  const double alpha = c.alpha, beta = c.beta;
  const int dn = c.dn;
  double acc = 0;
  for (int64_t hb = h0; hb < H; hb += 2 * S) {
    if (hb != h0) {
      load(hb, 0);
      load(hb, 1);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t h = hb + u * S;
      if (h >= H) break;
      double2 pi, qi, xi, ri;
      pi.x = first ? zv[u].x : zv[u].x + beta * pv[u].x;
      pi.y = first ? zv[u].y : zv[u].y + beta * pv[u].y;
      qi.x = first ? wv[u].x : wv[u].x + beta * qv[u].x;
      qi.y = first ? wv[u].y : wv[u].y + beta * qv[u].y;
      xi.x = xv[u].x + alpha * pi.x;
      xi.y = xv[u].y + alpha * pi.y;
      ri.x = rv[u].x - alpha * qi.x;
      ri.y = rv[u].y - alpha * qi.y;
      acc += ri.x * ri.x;
      acc += ri.y * ri.y;
      if (!dn) {
        p2[h] = pi;
        q2[h] = qi;
        x2[h] = xi;
        r2[h] = ri;
      }
    }
  }
  put_partial(acc, part + P_RR * (int64_t)nb);
}

// ------------------------------------------------------------------- batched PCG kernels --
// The kernels above over several solves at once (continuous batching): each solve keeps its own
// block count, so its partial sums, and with them its iterates, are those it makes alone.
__device__ __forceinline__ const BatchCg* bcg_arg(const BatchCg* __restrict__ args, int nslot,
                                                  int* vb) {
  int lo = 0, hi = nslot - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (args[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  *vb = b - args[lo].first;
  return args + lo;
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_bcg_rhs(const BatchCg* __restrict__ args,
                                                      int nslot) {
  int vb;
  const BatchCg& a = *bcg_arg(args, nslot, &vb);
  if (vb == 0 && threadIdx.x == 0) {  // a new step (no block reads these here)
    CgState* st = a.st;
    st->iters = 0;
    st->status = 0;
    st->done = 0;
    st->hold = 0;
    st->maxit = a.maxit;
  }
  double acc = 0;
  const int64_t stride = (int64_t)a.nb * kThreads;
  for (NodeWalk<DIM> c(vb * (int64_t)kThreads + threadIdx.x, stride, a.n); c.i < a.N;
       c.next(a.n)) {
    const double ui = a.u[c.i];
    const double g = cn_rhs_value(ui, link_sum_at<DIM>(c.i, c.ix, c.iy, c.iz, a.n, a.links, ui,
                                                       [&](int64_t k) { return a.u[k]; }),
                                  a.dt, a.kind, a.k1, a.k2);
    a.r[c.i] = g;
    a.x[c.i] = 0.0;
    acc += g * g;
  }
  const double sblk = block_sum(acc);
  if (threadIdx.x == 0) a.part[P_GG * (int64_t)a.nb + vb] = sblk;
}

__global__ __launch_bounds__(kThreads) void k_bcg_check(const BatchCg* __restrict__ args,
                                                        int nslot, int init, int it0, int fin,
                                                        int seq) {
  __shared__ int stop;
  int vb;
  const BatchCg& a = *bcg_arg(args, nslot, &vb);
  CgState* st = a.st;
  const int nb = a.nb;
  const bool lead = vb == 0 && threadIdx.x == 0;
  const int64_t stride = (int64_t)nb * kThreads, i0 = vb * (int64_t)kThreads + threadIdx.x;
  // the step's records (lead lane): iteration count and relative residual on the device and,
  // for the host, the residual in the mapped flag block ahead of the posted word
  auto record = [&](int iters) {
    const double rel = st->gg > 0 ? sqrt(st->rr / st->gg) : 0.0;
    a.it_out[0] = iters;
    a.rel_out[0] = rel;
    *reinterpret_cast<volatile double*>(a.hflag + 4) = rel;
    __threadfence_system();
    post_flag(a.hflag, seq, iters, 1, st->status);
  };
  auto finish = [&](int iters, bool keep_u) {  // u = x; the step's records
    if (!keep_u)
      for (int64_t i = i0; i < a.N; i += stride) a.u[i] = a.x[i];
    if (lead) record(iters);
  };
  if (!init && st->done) {  // stopped by an earlier test of this step
    if (fin) finish(st->iters, st->status != 0 && st->iters == 0);
    return;
  }
  if (threadIdx.x < 64) {
    CgTotal ct;
    const double* part = a.part + (init ? P_GG : P_RR) * (int64_t)nb;
    ct.load(part, nb);
    const double t = ct.sum(part, nb);
    if (threadIdx.x == 0)
      stop = cg_verdict(st, init, it0, a.rtol, t, st->tol2, init ? a.maxit : st->maxit, vb == 0);
  }
  __syncthreads();
  if (stop) {
    // block 0 published the scalars; the other blocks only copy x (init stops copy nothing)
    if (fin && !init) finish(it0 + 1, false);
    return;
  }
  if (fin && lead) post_flag(a.hflag, seq, it0 + 1, 0, 0);
  for (int64_t i = i0; i < a.N; i += stride) a.z[i] = a.r[i];
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_bcg_dir_dots(const BatchCg* __restrict__ args,
                                                           int nslot, int it) {
  int vb;
  const BatchCg& a = *bcg_arg(args, nslot, &vb);
  if (a.st->done) return;
  const int nb = a.nb;
  double rz = 0, zw = 0, zq = 0;
  const int64_t stride = (int64_t)nb * kThreads;
  auto Z = [&](int64_t k) { return a.z[k]; };
  for (NodeWalk<DIM> c(vb * (int64_t)kThreads + threadIdx.x, stride, a.n); c.i < a.N;
       c.next(a.n)) {
    const double zi = a.z[c.i];
    const double wi = zi + link_sum_at<DIM>(c.i, c.ix, c.iy, c.iz, a.n, a.links, zi, Z);
    a.w[c.i] = wi;
    rz += a.r[c.i] * zi;
    zw += zi * wi;
    if (it > 0) zq += zi * a.q[c.i];
  }
  block_sum3(rz, zw, zq);
  if (threadIdx.x == 0) {
    a.part[P_RZ * (int64_t)nb + vb] = rz;
    a.part[P_ZW * (int64_t)nb + vb] = zw;
    a.part[P_ZQ * (int64_t)nb + vb] = zq;
  }
}

__global__ __launch_bounds__(kThreads) void k_bcg_update(const BatchCg* __restrict__ args,
                                                         int nslot, int it) {
  int vb;
  const BatchCg& a = *bcg_arg(args, nslot, &vb);
  CgState* st = a.st;
  if (st->done) return;
  const int nb = a.nb;
  const bool first = it == 0;
  double rz = 0, zw = 0, zq = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    rz += a.part[P_RZ * (int64_t)nb + i];
    zw += a.part[P_ZW * (int64_t)nb + i];
    zq += a.part[P_ZQ * (int64_t)nb + i];
  }
  block_sum3(rz, zw, zq);
  const double beta = first ? 0.0 : rz / st->rzv[(it + 1) & 1];
  const double pq = first ? zw : zw + beta * (2.0 * zq + beta * st->pqv[(it + 1) & 1]);
  const double alpha = rz / pq;
  if (vb == 0 && threadIdx.x == 0) {
    st->rzv[it & 1] = rz;
    st->pqv[it & 1] = pq;
  }
  double acc = 0;
  const int64_t stride = (int64_t)nb * kThreads;
  for (int64_t i = vb * (int64_t)kThreads + threadIdx.x; i < a.N; i += stride) {
    const double zi = a.z[i], wi = a.w[i];
    const double pi = first ? zi : zi + beta * a.p[i];
    const double qi = first ? wi : wi + beta * a.q[i];
    const double ri = a.r[i] - alpha * qi;
    a.x[i] += alpha * pi;
    a.p[i] = pi;
    a.q[i] = qi;
    a.r[i] = ri;
    acc += ri * ri;
  }
  const double sblk = block_sum(acc);
  if (threadIdx.x == 0) a.part[P_RR * (int64_t)nb + vb] = sblk;
}

}  // namespace

void launch_bcg_rhs(const BatchCg* args, int nslot, int blocks, int dim, hipStream_t s) {
  auto k = dim == 2 ? k_bcg_rhs<2> : k_bcg_rhs<3>;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(kThreads), 0, s, args, nslot);
}

void launch_bcg_check(const BatchCg* args, int nslot, int blocks, int init, int it0, int fin,
                      int seq, hipStream_t s) {
  hipLaunchKernelGGL(k_bcg_check, dim3(blocks), dim3(kThreads), 0, s, args, nslot, init, it0,
                     fin, seq);
}

void launch_bcg_dir_dots(const BatchCg* args, int nslot, int blocks, int dim, int it,
                         hipStream_t s) {
  auto k = dim == 2 ? k_bcg_dir_dots<2> : k_bcg_dir_dots<3>;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(kThreads), 0, s, args, nslot, it);
}

void launch_bcg_update(const BatchCg* args, int nslot, int blocks, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_bcg_update, dim3(blocks), dim3(kThreads), 0, s, args, nslot, it);
}

int vec_blocks(int64_t N) {
  int64_t b = (N + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 512));
}

int cg_partial_slots() { return P_SLOTS; }

void launch_links(const double* a_cells, int dim, int n, double scale, double* links,
                  hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_links2d, dim3(1024), dim3(kThreads), 0, s, a_cells, n, scale, links);
  else
    hipLaunchKernelGGL(k_links3d, dim3(1024), dim3(kThreads), 0, s, a_cells, n, scale, links);
  HIF_CHECK(hipGetLastError());
}

// The stencil kernels take x-pairs of nodes where n is even and the vectors are 16-byte aligned
// (HIFCN_NO_PAIRS=1: one node per lane everywhere).
bool use_pairs_ptrs(std::initializer_list<const void*> vecs) {
  static const bool off = std::getenv("HIFCN_NO_PAIRS") != nullptr;
  if (off) return false;
  for (const void* p : vecs)
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return false;
  return true;
}
bool use_pairs(const Handle& h, std::initializer_list<const void*> vecs) {
  return h.n % 2 == 0 && use_pairs_ptrs(vecs);
}

void launch_spmv(const Handle& h, const double* x, double* y, hipStream_t s) {
  if (use_pairs(h, {x, y})) {
    const int nb = (int)std::min<int64_t>((h.N / 2 + kThreads - 1) / kThreads, 4096);
    auto k = h.dim == 2 ? k_spmv_pairs<2> : k_spmv_pairs<3>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(kThreads), 0, s, h.n, h.N, h.links.p, x, y);
    HIF_CHECK(hipGetLastError());
    return;
  }
  const int nb = (int)std::min<int64_t>((h.N + kThreads - 1) / kThreads, 4096);
  if (h.dim == 2)
    hipLaunchKernelGGL(k_spmv<2>, dim3(nb), dim3(kThreads), 0, s, h.n, h.N, h.links.p, x, y);
  else
    hipLaunchKernelGGL(k_spmv<3>, dim3(nb), dim3(kThreads), 0, s, h.n, h.N, h.links.p, x, y);
  HIF_CHECK(hipGetLastError());
}

void launch_cg_rhs(Handle& h, const double* u, int kind, double k1, double k2, bool ahead,
                   hipStream_t s, bool warm) {
  auto k = use_pairs(h, {u, h.r.p, h.x.p}) ? (h.dim == 2 ? k_cg_rhs_pairs<2> : k_cg_rhs_pairs<3>)
                        : (h.dim == 2 ? k_cg_rhs<2> : k_cg_rhs<3>);
  hipLaunchKernelGGL(k, dim3(h.nblk), dim3(kThreads), 0, s, h.n, h.N, h.links.p, u, h.r.p, h.x.p,
                     kind, k1, k2, h.dt, ahead ? 1 : 0, warm ? 1 : 0, h.st.p, h.partials.p);
}

void launch_cg_resume(Handle& h, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_resume, dim3(1), dim3(64), 0, s, h.st.p);
}

void launch_cg_check_copy(Handle& h, int it, double rtol, int maxit, hipStream_t s,
                          bool warm) {
  hipLaunchKernelGGL(k_cg_check_copy, dim3(h.nblk), dim3(kThreads), 0, s, h.N, it < 0 ? 1 : 0, it,
                     rtol, maxit, h.r.p, h.z.p, h.st.p, h.partials.p, CgFinish{}, warm ? 1 : 0);
}

void launch_cg_check_finish(Handle& h, int it, double rtol, double* u, int step, int seq,
                            hipStream_t s, bool warm) {
  const CgFinish fin{h.flag_dev, seq, h.x.p, u, h.step_iters.p, h.step_relres.p, step};
  hipLaunchKernelGGL(k_cg_check_copy, dim3(h.nblk), dim3(kThreads), 0, s, h.N, 0, it, rtol, 0,
                     h.r.p, h.z.p, h.st.p, h.partials.p, fin, warm ? 1 : 0);
}

CgGate cg_gate_args(Handle& h, int it, double rtol, int maxit) {
  CgGate g;
  g.maxit = maxit;
  g.st = h.st.p;
  g.nb = h.nblk;
  g.init = it < 0 ? 1 : 0;
  g.it0 = it;
  g.rtol = rtol;
  g.part = h.partials.p + (it < 0 ? P_GG : P_RR) * (int64_t)h.nblk;
  g.src = h.r.p;
  return g;
}

void launch_cg_dir_dots(Handle& h, int it, hipStream_t s) {
  auto k = use_pairs(h, {h.z.p, h.r.p, h.q.p, h.w.p})
               ? (h.dim == 2 ? k_cg_dir_dots_pairs<2> : k_cg_dir_dots_pairs<3>)
                        : (h.dim == 2 ? k_cg_dir_dots<2> : k_cg_dir_dots<3>);
  hipLaunchKernelGGL(k, dim3(h.nblk), dim3(kThreads), 0, s, h.n, h.N, it, h.links.p, h.z.p, h.r.p,
                     h.q.p, h.w.p, h.partials.p);
}

void launch_cg_update(Handle& h, int it, double rtol, hipStream_t s, bool fused_g) {
  const bool g = it == 0 && fused_g;
  const bool pairs = h.N % 2 == 0 && use_pairs_ptrs({h.z.p, h.w.p, h.p.p, h.q.p, h.x.p, h.r.p});
  hipLaunchKernelGGL(pairs ? k_cg_update_pairs : k_cg_update, dim3(h.nblk), dim3(kThreads), 0, s,
                     h.N, it, h.z.p, h.w.p,
                     h.p.p, h.q.p, h.x.p, h.r.p, h.st.p, h.partials.p,
                     g ? (const double*)h.gpart.p : (const double*)nullptr, (int)h.gpart.n, rtol);
}

}  // namespace hifcn
