// PHIF factor build on the GPU, FP64 (Sec. 2.2).
//
// The active matrix of a level is held as a table of dense blocks A_gh between the level's
// groups (cell interiors, edges/faces, corners, 3D edges) for every pair of groups that share a
// cell closure.  Per level l = 0..L-1 (every stage is one batched launch over independent
// blocks):
//   (1) k_build_cells  : per cell, L = chol(A_II), L^-1, G = L^-1 A_IB, Schur S = G^T G, and the
//                        apply blocks L^-1 and H = G^T L^-1 (eq2_3).
//       k_schur_add    : per separator block, A_gh -= sum of the S pieces of the cells sharing
//                        it, in a fixed cell order (deterministic, no atomics) (eq3_1).
//   (2) k_jacobi_chol  : per separator group, L_g = chol(A_gg), L_g^-1, A_gg <- I.
//       k_jacobi_scale : per separator block, A_gh <- L_g^-1 A_gh L_h^-T (jacobi-precond, eq3_2).
//   (3) k_id           : per edge (3D face), column-pivoted Householder QR of the coupling to all
//                        other active DOFs, rank k at relative precision eps, T = R11^-1 R12,
//                        L_s = chol(I + T^T T), X = I - T (I + T^T T)^-1 T^T (eq2_5, eq_T, eq2_9).
//       k_regroup      : blocks of level l+1 gathered from the surviving rows/columns (eq3_3).
// Root: chol of the last remaining block (eq3_4).  The host plans the index structure between
// launches; only ranks and pivot orders come back from the device once per level.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <list>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "front.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace hifcn {

namespace {

constexpr int kBT = 256;  // threads per build workgroup

struct SubBlk { int64_t off; int32_t width, pad; };
struct CellTask {
  int32_t nI, nB, nsub, offSub;
  int64_t offAII, offW, offS, offV;
  int32_t mode, offIb;  // mode 1: keep A_IB(ib_b, b) per boundary DOF instead of H
  int32_t symE, pad;    // mode 2: elements of the storage type per 16 bytes (storage order)
};
struct Contrib { int64_t offS; int32_t ld, r0, c0, pad; };
struct SchurTask { int64_t dst; int32_t rows, cols, ncontrib, offC; };
struct GroupTask { int32_t n, pad; int64_t offBlk, offW, offLD, offV; };
struct ScaleTask { int64_t offBlk, offTmp, offLg, offLh; int32_t rows, cols; };
struct IdTask { int32_t n, m, nrs, offRS; int64_t offW, offV, offX; int32_t offPerm, kslot; };
struct SrcEnt { int64_t off; int32_t ld, g; };
struct RegroupTask { int64_t dst; int32_t nG, nH, offRowsG, offRowsH, nsubH, offSrc; };
struct FillTask { int64_t off; int32_t rows, cols, offRowIds, offColIds; };

// ------------------------------------------------------------- workgroup dense FP64 helpers --
// In-place Cholesky (lower) of the n x n row-major matrix W (leading dimension ld).  A
// non-positive or non-finite pivot raises *err and is replaced by 1 so the kernel completes.
__device__ void wg_potrf(double* W, int n, int ld, int* err) {
  __shared__ double piv;
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = W[(int64_t)j * ld + j];
      if (!(d > 0.0) || !(d < 1.0e300)) {
        atomicOr(err, 1);
        d = 1.0;
      }
      piv = sqrt(d);
      W[(int64_t)j * ld + j] = piv;
    }
    __syncthreads();
    const double p = piv;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) W[(int64_t)i * ld + j] /= p;
    __syncthreads();
    const int m = n - j - 1;
    const int64_t tot = (int64_t)m * m;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
      const int r = (int)(t / m), c = (int)(t - (int64_t)r * m);
      if (c <= r) {
        const int i = j + 1 + r, k = j + 1 + c;
        W[(int64_t)i * ld + k] -= W[(int64_t)i * ld + j] * W[(int64_t)k * ld + j];
      }
    }
    __syncthreads();
  }
}

// B <- L^-1 B by right-looking forward substitution; L lower n x n (ld_l), B n x nc (ld_b).
// tri: B is lower triangular (the identity), so step k only touches columns <= k.
__device__ void wg_trsm_lower(const double* L, int n, int ldl, double* B, int nc, int ldb,
                              bool tri) {
  for (int k = 0; k < n; ++k) {
    const double d = L[(int64_t)k * ldl + k];
    const int cols = tri ? k + 1 : nc;
    for (int c = threadIdx.x; c < cols; c += blockDim.x) B[(int64_t)k * ldb + c] /= d;
    __syncthreads();
    const int rows = n - k - 1;
    const int64_t tot = (int64_t)rows * cols;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
      const int r = (int)(t / cols), c = (int)(t - (int64_t)r * cols);
      const int i = k + 1 + r;
      B[(int64_t)i * ldb + c] -= L[(int64_t)i * ldl + k] * B[(int64_t)k * ldb + c];
    }
    __syncthreads();
  }
}

__device__ void wg_identity(double* X, int n, int ld) {
  for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) {
    const int i = (int)(t / n), j = (int)(t - (int64_t)i * n);
    X[(int64_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
}

// packed column-major lower triangle of the row-major lower matrix X
__device__ void wg_store_packed(double* dst, const double* X, int n, int ld) {
  const int64_t tot = (int64_t)n * n;
  for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
    const int j = (int)(t / n), i = (int)(t - (int64_t)j * n);
    if (i >= j) dst[colstart(j, n) + (i - j)] = X[(int64_t)i * ld + j];
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return __shfl(v, 0, 64);
}

// ---------------------------------------------------------------------------- stencil fill --
// Entry (i, j) of A = I - dt/2 M from the scaled link weights (see solver.hip for the layout).
__device__ double a_entry(int n, int dim, const double* w, int32_t i, int32_t j) {
  const int64_t n1 = n + 1, nn = (int64_t)n * n;
  const int ix = i % n, iy = (i / n) % n, iz = dim == 3 ? i / (int)nn : 0;
  const int64_t lx = (dim == 3 ? nn : (int64_t)n) * n1;
  const int64_t xrow = dim == 3 ? ((int64_t)iz * n + iy) * n1 : (int64_t)iy * n1;
  const int64_t yb = dim == 3 ? ((int64_t)iz * n1 + iy) * n + ix : (int64_t)iy * n + ix;
  const int64_t zb = ((int64_t)iz * n + iy) * n + ix;
  if (i == j) {
    double d = 1.0 + w[xrow + ix] + w[xrow + ix + 1] + w[lx + yb] + w[lx + yb + n];
    if (dim == 3) d += w[2 * lx + zb] + w[2 * lx + zb + nn];
    return d;
  }
  const int jx = j % n, jy = (j / n) % n, jz = dim == 3 ? j / (int)nn : 0;
  const int dx = jx - ix, dy = jy - iy, dz = jz - iz;
  if (dy == 0 && dz == 0) {
    if (dx == 1) return -w[xrow + ix + 1];
    if (dx == -1) return -w[xrow + ix];
  } else if (dx == 0 && dz == 0) {
    if (dy == 1) return -w[lx + yb + n];
    if (dy == -1) return -w[lx + yb];
  } else if (dim == 3 && dx == 0 && dy == 0) {
    if (dz == 1) return -w[2 * lx + zb + nn];
    if (dz == -1) return -w[2 * lx + zb];
  }
  return 0.0;
}

__global__ __launch_bounds__(kBT) void k_fill(const FillTask* __restrict__ tasks,
                                              const int32_t* __restrict__ ids, int n, int dim,
                                              const double* __restrict__ w, double* __restrict__ A) {
  const FillTask t = tasks[blockIdx.x];
  const int64_t tot = (int64_t)t.rows * t.cols;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e / t.cols), c = (int)(e - (int64_t)r * t.cols);
    A[t.off + e] = a_entry(n, dim, w, ids[t.offRowIds + r], ids[t.offColIds + c]);
  }
}

// ------------------------------------------------------------------- (1) cell elimination --
__global__ __launch_bounds__(kBT) void k_build_cells(const CellTask* __restrict__ tasks,
                                                     const SubBlk* __restrict__ subs,
                                                     const int32_t* __restrict__ ibl,
                                                     const double* __restrict__ A,
                                                     double* __restrict__ work,
                                                     double* __restrict__ schur,
                                                     double* __restrict__ fv, int* err) {
  const CellTask t = tasks[blockIdx.x];
  const int nI = t.nI, nB = t.nB;
  double* W = work + t.offW;                    // nI x nI : A_II -> L
  double* X = W + (int64_t)nI * nI;             // nI x nI : L^-1
  double* G = X + (int64_t)nI * nI;             // nI x nB : A_IB -> G
  for (int64_t e = threadIdx.x; e < (int64_t)nI * nI; e += blockDim.x) W[e] = A[t.offAII + e];
  int c0 = 0;
  for (int s = 0; s < t.nsub; ++s) {
    const SubBlk sb = subs[t.offSub + s];
    for (int64_t e = threadIdx.x; e < (int64_t)nI * sb.width; e += blockDim.x) {
      const int i = (int)(e / sb.width), j = (int)(e - (int64_t)i * sb.width);
      G[(int64_t)i * nB + c0 + j] = A[sb.off + e];
    }
    c0 += sb.width;
  }
  wg_identity(X, nI, nI);
  __syncthreads();
  double* V = fv + t.offV;
  const int64_t coff = t.mode == 2 ? sym_coff(tri_count(nI)) : tri_count(nI);
  if (t.mode)   // the single coupling of each boundary DOF, before G overwrites A_IB
    for (int b = threadIdx.x; b < nB; b += blockDim.x)
      V[coff + b] = G[(int64_t)ibl[t.offIb + b] * nB + b];
  wg_potrf(W, nI, nI, err);
  wg_trsm_lower(W, nI, nI, X, nI, nI, true);
  if (nB) wg_trsm_lower(W, nI, nI, G, nB, nB, false);
  __syncthreads();
  // Schur contribution S = G^T G
  for (int64_t e = threadIdx.x; e < (int64_t)nB * nB; e += blockDim.x) {
    const int a = (int)(e / nB), b = (int)(e - (int64_t)a * nB);
    double acc = 0;
    for (int i = 0; i < nI; ++i) acc += G[(int64_t)i * nB + a] * G[(int64_t)i * nB + b];
    schur[t.offS + e] = acc;
  }
  // apply blocks: packed L^-1 (mode 2: packed A_II^-1 = L^-T L^-1), then (mode 0)
  // H = G^T L^-1 column-major (H[j*nB + b])
  if (t.mode == 2) {
    // (A_II^-1)_ij = sum over k >= max(i, j) of (L^-1)_ki (L^-1)_kj; packed column-major lower,
    // in the storage order of sym_store_index (padding slots up to sym_coff: zero)
    const int tl = (int)tri_count(nI);
    for (int s = threadIdx.x; s < (int)coff; s += blockDim.x) {
      const int e = sym_packed_index(s, tl, t.symE);
      double acc = 0;
      if (s < (tl + t.symE - 1) / t.symE * t.symE && e < tl) {
        int j = 0, c = e;
        while (c >= nI - j) c -= nI - j++;
        const int i = j + c;
        for (int k = i; k < nI; ++k) acc += X[(int64_t)k * nI + i] * X[(int64_t)k * nI + j];
      }
      V[s] = acc;
    }
    return;
  }
  wg_store_packed(V, X, nI, nI);
  if (t.mode) return;
  double* H = V + tri_count(nI);
  for (int64_t e = threadIdx.x; e < (int64_t)nB * nI; e += blockDim.x) {
    const int j = (int)(e / nB), b = (int)(e - (int64_t)j * nB);
    double acc = 0;
    for (int i = j; i < nI; ++i) acc += G[(int64_t)i * nB + b] * X[(int64_t)i * nI + j];
    H[e] = acc;
  }
}

__global__ __launch_bounds__(kBT) void k_schur_add(const SchurTask* __restrict__ tasks,
                                                   const Contrib* __restrict__ con,
                                                   const double* __restrict__ schur,
                                                   double* __restrict__ A) {
  const SchurTask t = tasks[blockIdx.x];
  const int64_t tot = (int64_t)t.rows * t.cols;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int i = (int)(e / t.cols), j = (int)(e - (int64_t)i * t.cols);
    double acc = A[t.dst + e];
    for (int c = 0; c < t.ncontrib; ++c) {
      const Contrib q = con[t.offC + c];
      acc -= schur[q.offS + (int64_t)(q.r0 + i) * q.ld + q.c0 + j];
    }
    A[t.dst + e] = acc;
  }
}

// --------------------------------------------------------------------- (2) block Jacobi --
__global__ __launch_bounds__(kBT) void k_jacobi_chol(const GroupTask* __restrict__ tasks,
                                                     double* __restrict__ A,
                                                     double* __restrict__ work,
                                                     double* __restrict__ LD,
                                                     double* __restrict__ fv, int* err) {
  const GroupTask t = tasks[blockIdx.x];
  const int n = t.n;
  double* W = work + t.offW;
  double* X = LD + t.offLD;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) W[e] = A[t.offBlk + e];
  wg_identity(X, n, n);
  __syncthreads();
  wg_potrf(W, n, n, err);
  wg_trsm_lower(W, n, n, X, n, n, true);
  __syncthreads();
  wg_store_packed(fv + t.offV, X, n, n);
  wg_identity(A + t.offBlk, n, n);  // the rescaled diagonal block is the identity
}

// A_gh <- L_g^-1 A_gh L_h^-T via Y = A L_h^-T (scratch), then A = L_g^-1 Y.
__global__ __launch_bounds__(kBT) void k_jacobi_scale(const ScaleTask* __restrict__ tasks,
                                                      double* __restrict__ A,
                                                      double* __restrict__ tmp,
                                                      const double* __restrict__ LD) {
  const ScaleTask t = tasks[blockIdx.x];
  const int R = t.rows, C = t.cols;
  double* Ab = A + t.offBlk;
  double* Y = tmp + t.offTmp;
  const double* Lg = LD + t.offLg;
  const double* Lh = LD + t.offLh;
  const int64_t tot = (int64_t)R * C;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int i = (int)(e / C), j = (int)(e - (int64_t)i * C);
    double acc = 0;
    for (int q = 0; q <= j; ++q) acc += Ab[(int64_t)i * C + q] * Lh[(int64_t)j * C + q];
    Y[e] = acc;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int i = (int)(e / C), j = (int)(e - (int64_t)i * C);
    double acc = 0;
    for (int p = 0; p <= i; ++p) acc += Lg[(int64_t)i * R + p] * Y[(int64_t)p * C + j];
    Ab[e] = acc;
  }
}

// Large groups after their Cholesky on the matrix cores: dense L_g^-1 (row-major, for the
// rescaling) from the packed copy, and A_gg <- I.
__global__ __launch_bounds__(kBT) void k_jacobi_unpack(const GroupTask* __restrict__ tasks,
                                                       double* __restrict__ A,
                                                       double* __restrict__ LD,
                                                       const double* __restrict__ fv) {
  const GroupTask t = tasks[blockIdx.x];
  const int n = t.n;
  const double* pk = fv + t.offV;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    LD[t.offLD + e] = j <= i ? pk[colstart(j, n) + (i - j)] : 0.0;
    A[t.offBlk + e] = i == j ? 1.0 : 0.0;
  }
}

// blocks with both sides at least this large are rescaled by products on the matrix cores
constexpr int kScaleMfma = 48;

// ------------------------------------------------------------------ (3) skeletonization --
// T = R11^-1 R12, L_s, X and the outputs of one ID, once the first k steps of the pivoted QR are
// in M (R in its upper triangle) and perm holds the column order.  Work layout after M: norms
// (n), v (m), T (k x nr col-major), S/Ls (nr x nr), Ls^-1 (nr x nr), Wm (k x nr).
__device__ void id_finish(const IdTask& t, double* M, int k, const int* perm,
                          double* __restrict__ fv, double* __restrict__ Xbuf,
                          int32_t* __restrict__ permout, int32_t* __restrict__ kout, int* err) {
  const int n = t.n, m = t.m;
  double* v = M + (int64_t)m * n + n;
  const int nr = n - k;
  double* T = v + m;                     // k x nr, column-major
  double* S = T + (int64_t)k * nr;       // nr x nr -> L_s
  double* Li = S + (int64_t)nr * nr;     // nr x nr -> L_s^-1
  double* Wm = Li + (int64_t)nr * nr;    // k x nr row-major: T L_s^-T
  // T = R11^-1 R12 by back substitution, one column per thread
  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    double* tc = T + (int64_t)j * k;
    for (int s = k - 1; s >= 0; --s) {
      double acc = M[(int64_t)(k + j) * m + s];
      for (int q = s + 1; q < k; ++q) acc -= M[(int64_t)q * m + s] * tc[q];
      tc[s] = acc / M[(int64_t)s * m + s];
    }
  }
  __syncthreads();
  // S = I + T^T T
  for (int64_t e = threadIdx.x; e < (int64_t)nr * nr; e += blockDim.x) {
    const int a = (int)(e / nr), b = (int)(e - (int64_t)a * nr);
    double acc = (a == b) ? 1.0 : 0.0;
    for (int s = 0; s < k; ++s) acc += T[(int64_t)a * k + s] * T[(int64_t)b * k + s];
    S[e] = acc;
  }
  wg_identity(Li, nr, nr);
  __syncthreads();
  wg_potrf(S, nr, nr, err);
  wg_trsm_lower(S, nr, nr, Li, nr, nr, true);
  __syncthreads();
  // factor values: T (column-major k x nr) and packed L_s^-1 after the group's packed L_g^-1
  double* V = fv + t.offV + tri_count(n);
  for (int64_t e = threadIdx.x; e < (int64_t)k * nr; e += blockDim.x) V[e] = T[e];
  wg_store_packed(V + (int64_t)k * nr, Li, nr, nr);
  // Wm = T L_s^-T,  X = I - Wm Wm^T (k x k)
  for (int64_t e = threadIdx.x; e < (int64_t)k * nr; e += blockDim.x) {
    const int s = (int)(e / nr), i = (int)(e - (int64_t)s * nr);
    double acc = 0;
    for (int j = 0; j <= i; ++j) acc += T[(int64_t)j * k + s] * Li[(int64_t)i * nr + j];
    Wm[e] = acc;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) {
    const int a = (int)(e / k), b = (int)(e - (int64_t)a * k);
    double acc = (a == b) ? 1.0 : 0.0;
    for (int i = 0; i < nr; ++i) acc -= Wm[(int64_t)a * nr + i] * Wm[(int64_t)b * nr + i];
    Xbuf[t.offX + e] = acc;
  }
  // pivot order: redundant first, then skeletons
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    permout[t.offPerm + i] = (i < nr) ? perm[k + i] : perm[i - nr];
  if (threadIdx.x == 0) kout[t.kslot] = k;
}

// One ID per workgroup (small edges): gather M (m x n column-major), column-pivoted Householder
// QR until the rank test stops it, then id_finish.
__global__ __launch_bounds__(kBT) void k_id(const IdTask* __restrict__ tasks,
                                            const SubBlk* __restrict__ rs,
                                            const double* __restrict__ A,
                                            double* __restrict__ work, double* __restrict__ fv,
                                            double* __restrict__ Xbuf, int32_t* __restrict__ permout,
                                            int32_t* __restrict__ kout, double eps, int* err) {
  const IdTask t = tasks[blockIdx.x];
  const int n = t.n, m = t.m;
  double* M = work + t.offW;
  double* nrm = M + (int64_t)m * n;
  double* v = nrm + n;
  __shared__ int perm_s[1024];
  __shared__ int piv_s, kstop_s;
  __shared__ double r00_s, pnorm_s;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // gather M: rows = the coupling blocks (h, g) of every other group h, stacked
  {
    int r0 = 0;
    for (int s = 0; s < t.nrs; ++s) {
      const SubBlk sb = rs[t.offRS + s];  // block (h, g): width = |h| rows, n columns
      for (int64_t e = threadIdx.x; e < (int64_t)sb.width * n; e += blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        M[(int64_t)j * m + r0 + i] = A[sb.off + e];
      }
      r0 += sb.width;
    }
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x) perm_s[j] = j;
  if (threadIdx.x == 0) { kstop_s = -1; r00_s = 0; }
  __syncthreads();
  const int kk = min(m, n);
  int k = kk;
  for (int st = 0; st < kk; ++st) {
    for (int j = st + wid; j < n; j += nw) {   // squared norms of the remaining columns
      double acc = 0;
      for (int i = st + lane; i < m; i += 64) acc += M[(int64_t)j * m + i] * M[(int64_t)j * m + i];
      acc = wave_sum(acc);
      if (lane == 0) nrm[j] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int p = st;
      double best = nrm[st];
      for (int j = st + 1; j < n; ++j)
        if (nrm[j] > best) { best = nrm[j]; p = j; }   // ties: lowest position
      const double pn = sqrt(best);
      if (st == 0) r00_s = pn;
      kstop_s = (pn <= eps * r00_s || pn == 0.0) ? st : -1;
      piv_s = p;
      pnorm_s = pn;
      if (kstop_s < 0 && p != st) {
        const int tmpi = perm_s[st];
        perm_s[st] = perm_s[p];
        perm_s[p] = tmpi;
      }
    }
    __syncthreads();
    if (kstop_s >= 0) { k = st; break; }
    const int p = piv_s;
    if (p != st)
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double a = M[(int64_t)st * m + i];
        M[(int64_t)st * m + i] = M[(int64_t)p * m + i];
        M[(int64_t)p * m + i] = a;
      }
    __syncthreads();
    // Householder reflector for column st, rows st..m-1
    const double pn = pnorm_s;
    const double x0 = M[(int64_t)st * m + st];
    const double alpha = x0 >= 0 ? -pn : pn;
    const double v0 = x0 - alpha;
    const double vtv = pn * pn - x0 * x0 + v0 * v0;
    for (int i = st + threadIdx.x; i < m; i += blockDim.x) v[i] = (i == st) ? v0 : M[(int64_t)st * m + i];
    __syncthreads();
    if (threadIdx.x == 0) M[(int64_t)st * m + st] = alpha;
    if (vtv > 0) {
      const double tau = 2.0 / vtv;
      for (int j = st + 1 + wid; j < n; j += nw) {
        double acc = 0;
        for (int i = st + lane; i < m; i += 64) acc += v[i] * M[(int64_t)j * m + i];
        acc = wave_sum(acc) * tau;
        for (int i = st + lane; i < m; i += 64) M[(int64_t)j * m + i] -= acc * v[i];
      }
    }
    __syncthreads();
  }
  id_finish(t, M, k, perm_s, fv, Xbuf, permout, kout, err);
}

// Large IDs (3D faces): the same pivoted QR, one launch pair per step over all of a level's
// large IDs, so each step's reflector is applied by many workgroups (one wavefront per column)
// instead of one.  Per step: k_qr_pivot (one workgroup per ID) picks the column of largest
// remaining norm (ties: lowest position), applies the rank test, swaps it into place and forms
// the reflector; k_qr_apply updates every later column and recomputes its norm over the rows
// below the step.  The arithmetic and the order of the steps are those of k_id.
struct QrState {
  int32_t k, stopped;
  double r00, tau, v0;
};

__global__ __launch_bounds__(kBT) void k_qr_init(const IdTask* __restrict__ tasks,
                                                 const SubBlk* __restrict__ rs,
                                                 const double* __restrict__ A,
                                                 double* __restrict__ work,
                                                 int32_t* __restrict__ perm,
                                                 QrState* __restrict__ qs) {
  const IdTask t = tasks[blockIdx.x];
  const int n = t.n, m = t.m;
  double* M = work + t.offW;
  double* nrm = M + (int64_t)m * n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int r0 = 0;
  for (int q = 0; q < t.nrs; ++q) {
    const SubBlk sb = rs[t.offRS + q];
    for (int64_t e = threadIdx.x; e < (int64_t)sb.width * n; e += blockDim.x) {
      const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
      M[(int64_t)j * m + r0 + i] = A[sb.off + e];
    }
    r0 += sb.width;
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x) perm[t.offPerm + j] = j;
  __syncthreads();
  for (int j = wid; j < n; j += nw) {
    double acc = 0;
    for (int i = lane; i < m; i += 64) acc += M[(int64_t)j * m + i] * M[(int64_t)j * m + i];
    acc = wave_sum(acc);
    if (lane == 0) nrm[j] = acc;
  }
  if (threadIdx.x == 0) qs[blockIdx.x] = QrState{-1, 0, 0.0, 0.0, 0.0};
}

__global__ __launch_bounds__(kBT) void k_qr_pivot(const IdTask* __restrict__ tasks, int st,
                                                  double* __restrict__ work,
                                                  int32_t* __restrict__ perm,
                                                  QrState* __restrict__ qs, double eps) {
  __shared__ double bv[kBT];
  __shared__ int bi[kBT];
  __shared__ int stop_s;
  QrState q = qs[blockIdx.x];
  if (q.stopped) return;
  const IdTask t = tasks[blockIdx.x];
  const int n = t.n, m = t.m;
  double* M = work + t.offW;
  double* nrm = M + (int64_t)m * n;
  if (st >= min(m, n)) {
    if (threadIdx.x == 0) {
      q.k = st;
      q.stopped = 1;
      qs[blockIdx.x] = q;
    }
    return;
  }
  double best = -1.0;
  int p = n;
  for (int j = st + threadIdx.x; j < n; j += blockDim.x)
    if (nrm[j] > best) { best = nrm[j]; p = j; }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = p;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double ob = bv[threadIdx.x + w];
      const int oi = bi[threadIdx.x + w];
      if (ob > bv[threadIdx.x] || (ob == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ob;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  p = bi[0];
  double pb = bv[0];
  if (p >= n) {  // no comparable norm (NaN): keep the column in place, as the one-workgroup QR
    p = st;
    pb = nrm[st];
  }
  const double pn = sqrt(pb);
  const double r00 = st == 0 ? pn : q.r00;
  if (threadIdx.x == 0) stop_s = (pn <= eps * r00 || pn == 0.0) ? 1 : 0;
  __syncthreads();
  if (stop_s) {
    if (threadIdx.x == 0) {
      q.k = st;
      q.stopped = 1;
      q.r00 = r00;
      qs[blockIdx.x] = q;
    }
    return;
  }
  if (p != st) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      const double a = M[(int64_t)st * m + i];
      M[(int64_t)st * m + i] = M[(int64_t)p * m + i];
      M[(int64_t)p * m + i] = a;
    }
    if (threadIdx.x == 0) {
      const int32_t a = perm[t.offPerm + st];
      perm[t.offPerm + st] = perm[t.offPerm + p];
      perm[t.offPerm + p] = a;
      nrm[p] = nrm[st];
    }
  }
  __syncthreads();
  const double x0 = M[(int64_t)st * m + st];
  __syncthreads();
  if (threadIdx.x == 0) {
    const double alpha = x0 >= 0 ? -pn : pn;
    const double v0 = x0 - alpha;
    const double vtv = pn * pn - x0 * x0 + v0 * v0;
    M[(int64_t)st * m + st] = alpha;
    q.r00 = r00;
    q.v0 = v0;
    q.tau = vtv > 0 ? 2.0 / vtv : 0.0;
    qs[blockIdx.x] = q;
  }
}

// One wavefront per column j > st: apply the step's reflector, then the squared norm over the
// rows below st (the next step's pivot test).
__global__ __launch_bounds__(kBT) void k_qr_apply(const IdTask* __restrict__ tasks, int st,
                                                  double* __restrict__ work,
                                                  const QrState* __restrict__ qs) {
  const QrState q = qs[blockIdx.y];
  if (q.stopped) return;
  const IdTask t = tasks[blockIdx.y];
  const int n = t.n, m = t.m;
  const int lane = threadIdx.x & 63;
  const int j = st + 1 + (int)blockIdx.x * (kBT / 64) + ((int)threadIdx.x >> 6);
  if (j >= n) return;
  double* M = work + t.offW;
  const double* vc = M + (int64_t)st * m;  // the reflector below the diagonal
  double* c = M + (int64_t)j * m;
  if (q.tau > 0) {  // same lane split as k_id, so both give identical results
    double acc = 0;
    for (int i = st + lane; i < m; i += 64) acc += (i == st ? q.v0 : vc[i]) * c[i];
    const double d = wave_sum(acc) * q.tau;
    for (int i = st + lane; i < m; i += 64) c[i] -= d * (i == st ? q.v0 : vc[i]);
  }
  double nn = 0;
  for (int i = st + 1 + lane; i < m; i += 64) nn += c[i] * c[i];
  nn = wave_sum(nn);
  if (lane == 0) M[(int64_t)m * n + j] = nn;
}

// Large IDs after the QR, the first part of id_finish: T = R11^-1 R12 (one column per lane),
// its copy into the factor values, the pivot order and the rank.  The products that follow
// (S = I + T^T T, X = I - Wm Wm^T with Wm = T L_s^-T) and chol(S) run on the matrix cores.
__global__ __launch_bounds__(kBT) void k_qr_t(const IdTask* __restrict__ tasks,
                                              double* __restrict__ work,
                                              const int32_t* __restrict__ perm,
                                              const QrState* __restrict__ qs,
                                              double* __restrict__ fv,
                                              int32_t* __restrict__ permout,
                                              int32_t* __restrict__ kout) {
  const IdTask t = tasks[blockIdx.x];
  const int n = t.n, m = t.m, k = qs[blockIdx.x].k, nr = n - k;
  const double* M = work + t.offW;
  double* T = work + t.offW + (int64_t)m * n + n + m;
  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    double* tc = T + (int64_t)j * k;
    for (int s = k - 1; s >= 0; --s) {
      double acc = M[(int64_t)(k + j) * m + s];
      for (int q = s + 1; q < k; ++q) acc -= M[(int64_t)q * m + s] * tc[q];
      tc[s] = acc / M[(int64_t)s * m + s];
    }
  }
  __syncthreads();
  double* V = fv + t.offV + tri_count(n);
  for (int64_t e = threadIdx.x; e < (int64_t)k * nr; e += blockDim.x) V[e] = T[e];
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    permout[t.offPerm + i] = (i < nr) ? perm[t.offPerm + k + i] : perm[t.offPerm + i - nr];
  if (threadIdx.x == 0) kout[t.kslot] = k;
}

// Dense row-major copy (zeros above the diagonal) of packed column-major lower triangles.
struct UnpackTask { int64_t src, dst; int32_t n, pad; };
__global__ __launch_bounds__(kBT) void k_unpack_tri(const UnpackTask* __restrict__ tasks,
                                                    const double* __restrict__ src,
                                                    double* __restrict__ dst) {
  const UnpackTask t = tasks[blockIdx.x];
  const int n = t.n;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    dst[t.dst + e] = j <= i ? src[t.src + colstart(j, n) + (i - j)] : 0.0;
  }
}

// ------------------------------------------------------------------------------- regroup --
__global__ __launch_bounds__(kBT) void k_regroup(const RegroupTask* __restrict__ tasks,
                                                 const RowSrc* __restrict__ rows,
                                                 const SrcEnt* __restrict__ src,
                                                 const double* __restrict__ Aold,
                                                 const double* __restrict__ Xbuf,
                                                 const int64_t* __restrict__ xoff,
                                                 const int32_t* __restrict__ gk,
                                                 double* __restrict__ Anew) {
  const RegroupTask t = tasks[blockIdx.x];
  const int64_t tot = (int64_t)t.nG * t.nH;
  // gridDim.y workgroups share a block (large blocks would otherwise run on one CU)
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.y * blockDim.x) {
    const int i = (int)(e / t.nH), j = (int)(e - (int64_t)i * t.nH);
    const RowSrc ri = rows[t.offRowsG + i], rj = rows[t.offRowsH + j];
    const SrcEnt s = src[t.offSrc + (int64_t)ri.sub * t.nsubH + rj.sub];
    double v = 0.0;
    if (s.off >= 0) {
      v = Aold[s.off + (int64_t)ri.pos * s.ld + rj.pos];
    } else if (s.off == -2) {  // the same previous group: X (skeletonized) or the identity
      const int64_t xo = xoff[s.g];
      v = xo >= 0 ? Xbuf[xo + (int64_t)ri.spos * gk[s.g] + rj.spos] : (ri.pos == rj.pos ? 1.0 : 0.0);
    }
    Anew[t.dst + e] = v;
  }
}

__global__ void k_to_store_f64(const double* src, double* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_to_store_f32(const double* src, float* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
__global__ void k_to_store_bf16(const double* src, bf16_t* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i].bits = f32_to_bf16_bits((float)src[i]);
}

template <typename T>
void upload(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc_on(std::max<size_t>(1, h.size()), s);
  if (!h.empty())
    HIF_CHECK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

int64_t tri64(int64_t n) { return n * (n + 1) / 2; }

// Level-0 plans by grid.  A level-0 plan depends on the geometry only, so factors of one grid
// (the requests of one size on a server, the rebuilds of a drifting coefficient) share it.
// The most recently used plans are kept, up to 8M DOFs of grids in all.
std::shared_ptr<const LevelPlan> level0_plan(const Geometry& geo) {
  using Key = std::array<int, 5>;
  static std::mutex mu;
  static std::list<std::pair<Key, std::shared_ptr<const LevelPlan>>> kept;  // most recent first
  const Key key{geo.dim, geo.n, geo.m, geo.L, geo.skel_edges ? 1 : 0};
  auto dofs = [](const Key& k) {
    int64_t N = 1;
    for (int d = 0; d < k[0]; ++d) N *= k[1];
    return N;
  };
  {
    std::lock_guard<std::mutex> lock(mu);
    for (auto it = kept.begin(); it != kept.end(); ++it)
      if (it->first == key) {
        kept.splice(kept.begin(), kept, it);
        return kept.front().second;
      }
  }
  auto plan = std::make_shared<const LevelPlan>(plan_level0(geo));
  constexpr int64_t kKeepDofs = int64_t(1) << 23;
  if (dofs(key) > kKeepDofs) return plan;
  std::lock_guard<std::mutex> lock(mu);
  kept.emplace_front(key, plan);
  int64_t total = 0;
  for (auto it = kept.begin(); it != kept.end();) {
    total += dofs(it->first);
    if (total > kKeepDofs) it = kept.erase(it);
    else ++it;
  }
  return plan;
}

}  // namespace

// Build the factor of the handle's operator on the device and lay it out for the apply.
void gpu_build(Handle& hd, const double* a_cells, hif_store_t store, hipStream_t s) {
  (void)a_cells;  // the link weights were already derived from it
  const Geometry geo{hd.dim, hd.n, hd.leaf, hd.L, hd.f.skel_edges};
  DevBuf<int> err(1, s);
  HIF_CHECK(hipMemsetAsync(err.p, 0, sizeof(int), s));
  // cells with at least this many interior DOFs (and the root) use the blocked front path;
  // HIFCN_FRONT_MIN overrides it (tests force either path on small grids)
  int front_min = 128;
  if (const char* e = std::getenv("HIFCN_FRONT_MIN")) front_min = std::max(1, std::atoi(e));
  FrontStats fstats;
  const int scale_min = std::min(kScaleMfma, front_min);  // forcing the front path forces this too
  const bool build_log = std::getenv("HIFCN_BUILD_LOG") != nullptr;
  // with the log on, each phase's wall time (the stream is synchronised at every mark)
  auto t_last = std::chrono::steady_clock::now();
  auto mark = [&](const char* what, int lev) {
    if (!build_log) return;
    HIF_CHECK(hipStreamSynchronize(s));
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[hifcn build] level %d %-14s %8.3f ms\n", lev, what,
                 std::chrono::duration<double, std::milli>(now - t_last).count());
    t_last = now;
  };
  // IDs with at least this many columns use the multi-workgroup QR; HIFCN_QR_MULTI_MIN
  // overrides it (tests force either path on small grids)
  int qr_multi = 96;
  if (const char* e = std::getenv("HIFCN_QR_MULTI_MIN")) qr_multi = std::max(1, std::atoi(e));
  // the one-workgroup ID (k_id) keeps the pivot order of at most 1024 columns in LDS; every
  // larger ID takes the multi-workgroup QR
  qr_multi = std::min(qr_multi, 1024);
  auto check_err = [&](const char* where) {
    int e = 0;
    HIF_CHECK(hipMemcpyAsync(&e, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIF_CHECK(hipStreamSynchronize(s));
    HIF_REQUIRE(e == 0, HIF_ERR_NOT_SPD,
                std::string("non-positive Cholesky pivot during ") + where);
  };

  const std::shared_ptr<const LevelPlan> plan0 = hd.plan0 ? hd.plan0 : level0_plan(geo);
  LevelPlan P(*plan0);
  if (hd.keep_plan0 && !hd.plan0) hd.plan0 = plan0;
  mark("plan", 0);
  DevBuf<double> A(std::max<int64_t>(1, P.nvals), s);
  {  // level-0 blocks straight from the stencil
    std::vector<int32_t> ids;
    std::vector<int32_t> goff(P.groups.size());
    for (size_t g = 0; g < P.groups.size(); ++g) {
      goff[g] = (int32_t)ids.size();
      ids.insert(ids.end(), P.groups[g].dofs.begin(), P.groups[g].dofs.end());
    }
    std::vector<FillTask> ft(P.blocks.size());
    for (size_t b = 0; b < P.blocks.size(); ++b) {
      const int g = P.blocks[b].first, h = P.blocks[b].second;
      ft[b] = {P.block_off[b], (int32_t)P.groups[g].dofs.size(), (int32_t)P.groups[h].dofs.size(),
               goff[g], goff[h]};
    }
    DevBuf<int32_t> dids;
    DevBuf<FillTask> dft;
    upload(dids, ids, s);
    upload(dft, ft, s);
    hipLaunchKernelGGL(k_fill, dim3(ft.size()), dim3(kBT), 0, s, dft.p, dids.p, hd.n, hd.dim,
                       hd.links.p, A.p);
    HIF_CHECK(hipGetLastError());
    HIF_CHECK(hipStreamSynchronize(s));
  }

  // Host record of the factor layout (offsets relative to each level's value chunk).
  struct LevelOut {
    std::vector<CellDesc> cells;
    std::vector<std::vector<int32_t>> cellI, cellB, cellIb;
    std::vector<GroupDesc> groups;
    std::vector<std::vector<int32_t>> gids, gperm, gslots_ptr, gslots;
    int64_t base = 0;
    int maxI = 0, maxB = 0, maxG = 0, maxK = 0, maxR = 0, maxCV = 0, maxGV = 0;
    int64_t cbn = 0;
  };
  std::vector<LevelOut> outs;
  std::vector<DevBuf<double>> chunks;
  int64_t nvals_actual = 0;
  int64_t total_chunk = 0;

  for (int lev = 0; lev < hd.L; ++lev) {
    LevelOut lo;
    const int G = (int)P.groups.size();
    auto gsz = [&](int g) { return (int)P.groups[g].dofs.size(); };
    // ---- value chunk layout: cells then separator groups
    int64_t voff = 0;
    std::vector<int64_t> cell_voff(P.cells.size()), grp_voff(G, -1);
    std::vector<int> cell_nB(P.cells.size());
    // level 0: A_IB is the stencil, one link per boundary DOF; keep that link instead of H.
    // Where every level-0 interior fits one wavefront (at most 64 DOFs) and none goes through
    // the front elimination, the cell block is A_II^-1 itself (mode 2, applied as one symmetric
    // product per sweep), else L^-1 (mode 1, two triangular products).  BF16 keeps L^-1: with
    // 8-bit significands the rounded A_II^-1 of a stiff cell (kappa(A_II) ~ 1e7 at dt = 0.1 and
    // contrast 1e4) is no longer positive definite, while L~^-T L~^-1 always is.
    int maxI_lev = 0;
    for (int c : P.cells) maxI_lev = std::max(maxI_lev, gsz(c));
    const bool sym_ok = maxI_lev <= kSymMaxCell && maxI_lev < front_min &&
                        store != HIF_STORE_BF16 && !sym_cells_off();
    const int cmode = lev != 0 ? 0 : sym_ok ? 2 : 1;
    std::vector<std::vector<int32_t>> cell_ib(P.cells.size());
    // position of a DOF in the interior of the cell at hand (-1 elsewhere), reset after each cell
    std::vector<int32_t> pos(cmode ? hd.N : 0, -1);
    for (size_t ci = 0; ci < P.cells.size(); ++ci) {
      int nB = 0;
      for (int b : P.cellB[ci]) nB += gsz(b);
      cell_nB[ci] = nB;
      voff = align_vals(voff);
      cell_voff[ci] = voff;
      const int nI = gsz(P.cells[ci]);
      voff += (cmode == 2 ? sym_coff(tri64(nI)) : tri64(nI)) +
              (cmode ? (int64_t)nB : (int64_t)nB * nI);
      if (cmode) {
        const std::vector<int32_t>& I = P.groups[P.cells[ci]].dofs;
        for (int i = 0; i < nI; ++i) pos[I[i]] = i;
        const int64_t nn = (int64_t)hd.n * hd.n;
        cell_ib[ci].reserve(nB);
        for (int b : P.cellB[ci])
          for (int32_t id : P.groups[b].dofs) {
            int found = -1;
            const int64_t cand[6] = {id - 1, id + 1, id - hd.n, id + hd.n, id - nn, id + nn};
            for (int q = 0; q < (hd.dim == 3 ? 6 : 4) && found < 0; ++q)
              if (cand[q] >= 0 && cand[q] < hd.N) found = pos[cand[q]];
            HIF_REQUIRE(found >= 0, HIF_ERR_ARG, "internal: boundary DOF without a stencil link");
            cell_ib[ci].push_back(found);
          }
        for (int i = 0; i < nI; ++i) pos[I[i]] = -1;
      }
    }
    for (int g : P.seps) {
      voff = align_vals(voff);
      grp_voff[g] = voff;
      // twice the packed triangle: room for T and L_s^-1 after an ID, or for the dense form
      // of the group step (n^2 <= n (n + 1))
      voff += 2 * tri64(gsz(g));
    }
    voff = align_vals(voff);
    DevBuf<double> fv(std::max<int64_t>(1, voff), s);

    // ---- (1) cell elimination
    std::vector<CellTask> ct(P.cells.size());
    std::vector<SubBlk> subs;
    std::vector<int32_t> ibl;
    int64_t woff = 0, soff = 0;
    std::vector<int64_t> cell_soff(P.cells.size());
    for (size_t ci = 0; ci < P.cells.size(); ++ci) {
      const int c = P.cells[ci];
      const int nI = gsz(c), nB = cell_nB[ci];
      CellTask& t = ct[ci];
      t.nI = nI;
      t.nB = nB;
      t.nsub = (int)P.cellB[ci].size();
      t.offSub = (int32_t)subs.size();
      for (int b : P.cellB[ci]) {
        const int blk = P.find_block(c, b);
        HIF_REQUIRE(blk >= 0, HIF_ERR_ARG, "internal: missing cell-boundary block");
        subs.push_back({P.block_off[blk], gsz(b), 0});
      }
      t.offAII = P.block_off[P.find_block(c, c)];
      t.offW = woff;
      woff += 2 * (int64_t)nI * nI + (int64_t)nI * nB;
      t.offS = soff;
      cell_soff[ci] = soff;
      soff += (int64_t)nB * nB;
      t.offV = cell_voff[ci];
      t.mode = cmode;
      t.symE = (int32_t)(16 / store_elem_bytes(store));
      t.offIb = (int32_t)ibl.size();
      ibl.insert(ibl.end(), cell_ib[ci].begin(), cell_ib[ci].end());
    }
    // large cells (dense H) go through the blocked front elimination on the matrix cores
    std::vector<CellTask> small;
    std::vector<FrontTask> fronts;
    std::vector<FrontSub> fsubs;
    woff = 0;
    for (CellTask t : ct) {
      if (t.nI >= front_min) {
        fronts.push_back({t.nI, t.nB, t.nsub, (int32_t)fsubs.size(), t.offAII, t.offV, t.offS,
                          0, 0, t.mode, t.offIb});
        for (int q = 0; q < t.nsub; ++q) fsubs.push_back({subs[t.offSub + q].off,
                                                          subs[t.offSub + q].width, 0});
      } else {
        t.offW = woff;
        woff += 2 * (int64_t)t.nI * t.nI + (int64_t)t.nI * t.nB;
        small.push_back(t);
      }
    }
    {
      DevBuf<CellTask> dct;
      DevBuf<SubBlk> dsub;
      DevBuf<int32_t> dibl;
      DevBuf<double> work(std::max<int64_t>(1, woff), s);
      DevBuf<double> schur(std::max<int64_t>(1, soff), s);
      upload(dct, small, s);
      upload(dsub, subs, s);
      upload(dibl, ibl, s);
      if (!small.empty())
        hipLaunchKernelGGL(k_build_cells, dim3(small.size()), dim3(kBT), 0, s, dct.p, dsub.p,
                           dibl.p, A.p, work.p, schur.p, fv.p, err.p);
      HIF_CHECK(hipGetLastError());
      build_fronts(fronts, fsubs, A.p, schur.p, fv.p, err.p, s, &fstats, dibl.p);
      // Schur assembly into every separator block touched by some cell
      // contributions grouped by block (counting sort: per block in cell order)
      std::vector<int32_t> hit;      // block of each contribution, in visiting order
      std::vector<Contrib> visit;
      for (size_t ci = 0; ci < P.cells.size(); ++ci) {
        const std::vector<int>& B = P.cellB[ci];
        std::vector<int> boff(B.size());
        int acc = 0;
        for (size_t q = 0; q < B.size(); ++q) { boff[q] = acc; acc += gsz(B[q]); }
        for (size_t a = 0; a < B.size(); ++a)
          for (size_t b = 0; b < B.size(); ++b) {
            const int blk = P.find_block(B[a], B[b]);
            HIF_REQUIRE(blk >= 0, HIF_ERR_ARG, "internal: missing separator block");
            hit.push_back(blk);
            visit.push_back({cell_soff[ci], cell_nB[ci], boff[a], boff[b], 0});
          }
      }
      std::vector<int32_t> start(P.blocks.size() + 1, 0);
      for (int32_t blk : hit) ++start[blk + 1];
      for (size_t b = 0; b < P.blocks.size(); ++b) start[b + 1] += start[b];
      std::vector<Contrib> con(visit.size());
      {
        std::vector<int32_t> fillp(start.begin(), start.end() - 1);
        for (size_t e = 0; e < visit.size(); ++e) con[fillp[hit[e]]++] = visit[e];
      }
      std::vector<SchurTask> stk;
      for (size_t b = 0; b < P.blocks.size(); ++b) {
        const int32_t cnt = start[b + 1] - start[b];
        if (!cnt) continue;
        const int g = P.blocks[b].first, h = P.blocks[b].second;
        stk.push_back({P.block_off[b], gsz(g), gsz(h), cnt, start[b]});
      }
      DevBuf<SchurTask> dst;
      DevBuf<Contrib> dcon;
      upload(dst, stk, s);
      upload(dcon, con, s);
      if (!stk.empty())
        hipLaunchKernelGGL(k_schur_add, dim3(stk.size()), dim3(kBT), 0, s, dst.p, dcon.p, schur.p,
                           A.p);
      HIF_CHECK(hipGetLastError());
      check_err("cell elimination");
    }

    mark("cells", lev);
    // ---- (2) block Jacobi on every separator group
    std::vector<int64_t> ld_off(G, -1);
    {
      // large groups: Cholesky and inverse as fronts without boundary on the matrix cores
      std::vector<GroupTask> gt, gbig;
      std::vector<FrontTask> gf;
      int64_t wo = 0, lo2 = 0;
      for (int g : P.seps) {
        const int n = gsz(g);
        ld_off[g] = lo2;
        const GroupTask t{n, 0, P.block_off[P.find_block(g, g)], wo, lo2, grp_voff[g]};
        if (n >= front_min) {
          gbig.push_back(t);
          gf.push_back({n, 0, 0, 0, t.offBlk, t.offV, -1, 0, 0});
        } else {
          gt.push_back(t);
          wo += (int64_t)n * n;
        }
        lo2 += (int64_t)n * n;
      }
      DevBuf<GroupTask> dgt, dgb;
      DevBuf<double> work(std::max<int64_t>(1, wo), s);
      DevBuf<double> LD(std::max<int64_t>(1, lo2), s);
      upload(dgt, gt, s);
      upload(dgb, gbig, s);
      if (!gt.empty())
        hipLaunchKernelGGL(k_jacobi_chol, dim3(gt.size()), dim3(kBT), 0, s, dgt.p, A.p, work.p,
                           LD.p, fv.p, err.p);
      if (!gf.empty()) {
        build_fronts(gf, {}, A.p, nullptr, fv.p, err.p, s, &fstats);
        hipLaunchKernelGGL(k_jacobi_unpack, dim3(gbig.size()), dim3(kBT), 0, s, dgb.p, A.p, LD.p,
                           (const double*)fv.p);
      }
      HIF_CHECK(hipGetLastError());
      std::vector<ScaleTask> sc, scb;
      int64_t to = 0;
      for (size_t b = 0; b < P.blocks.size(); ++b) {
        const int g = P.blocks[b].first, h = P.blocks[b].second;
        if (g == h || P.groups[g].kind == 0 || P.groups[h].kind == 0) continue;
        const ScaleTask t{P.block_off[b], to, ld_off[g], ld_off[h], gsz(g), gsz(h)};
        // large blocks: two batched products on the matrix cores
        (gsz(g) >= scale_min && gsz(h) >= scale_min ? scb : sc).push_back(t);
        to += (int64_t)gsz(g) * gsz(h);
      }
      DevBuf<ScaleTask> dsc;
      DevBuf<double> tmp(std::max<int64_t>(1, to), s);
      upload(dsc, sc, s);
      if (!scb.empty()) {
        std::vector<GemmTask> y_of, a_of;
        for (const ScaleTask& t : scb) {
          double* Ab = A.p + t.offBlk;
          double* Y = tmp.p + t.offTmp;
          // Y = A_gh L_h^-T, then A_gh = L_g^-1 Y
          y_of.push_back({Ab, LD.p + t.offLh, Y, t.cols, t.cols, t.cols, t.rows, t.cols, t.cols,
                          1, 1, 0, 1.0, 0, 0});
          a_of.push_back({LD.p + t.offLg, Y, Ab, t.rows, t.cols, t.cols, t.rows, t.cols, t.rows,
                          0, 2, 0, 1.0, 0, 0});
        }
        gemm_batched(y_of, s, &fstats);
        gemm_batched(a_of, s, &fstats);
      }
      if (!sc.empty())
        hipLaunchKernelGGL(k_jacobi_scale, dim3(sc.size()), dim3(kBT), 0, s, dsc.p, A.p, tmp.p,
                           LD.p);
      HIF_CHECK(hipGetLastError());
      check_err("block Jacobi");
    }

    mark("jacobi", lev);
    // ---- (3) skeletonization of every edge (3D: face, and edge with skel_edges)
    std::vector<int32_t> kval(P.skel.size());
    std::vector<int32_t> permv;
    std::vector<int32_t> perm_off(G, -1);
    DevBuf<double> Xbuf;
    std::vector<int64_t> xoff(G, -1);
    {
      // rows of every edge's ID: the blocks (h, g) of all other separator groups h
      std::vector<std::vector<int>> rows_of(G);
      for (size_t b = 0; b < P.blocks.size(); ++b) {
        const int h = P.blocks[b].first, g = P.blocks[b].second;
        if (h != g && P.groups[h].kind > 0 && geo.skeletonized(P.groups[g].kind))
          rows_of[g].push_back((int)b);
      }
      std::vector<IdTask> it;
      std::vector<SubBlk> rs;
      int64_t wo = 0, xo = 0;
      int32_t po = 0;
      for (size_t q = 0; q < P.skel.size(); ++q) {
        const int g = P.skel[q];
        const int n = gsz(g);
        IdTask t{};
        t.n = n;
        t.offRS = (int32_t)rs.size();
        int m = 0;
        for (int blk : rows_of[g]) {   // blocks sorted by (h, g): h in group order
          const int h = P.blocks[blk].first;
          rs.push_back({P.block_off[blk], gsz(h), 0});
          m += gsz(h);
        }
        t.m = m;
        t.nrs = (int32_t)(rs.size() - t.offRS);
        t.offW = wo;
        wo += (int64_t)m * n + n + m + (int64_t)n * n * 3 + 16;
        t.offV = grp_voff[g];
        t.offX = xo;
        xoff[g] = xo;
        xo += (int64_t)n * n;
        t.offPerm = po;
        perm_off[g] = po;
        po += n;
        t.kslot = (int32_t)q;
        it.push_back(t);
      }
      if (build_log) {
        int mx_n = 0, mx_m = 0;
        double mn = 0;
        for (const IdTask& t : it) {
          mx_n = std::max(mx_n, t.n);
          mx_m = std::max(mx_m, t.m);
          mn += (double)t.m * t.n;
        }
        int mx_i = 0, mx_b = 0, mx_g = 0;
        for (const CellTask& t : ct) { mx_i = std::max(mx_i, t.nI); mx_b = std::max(mx_b, t.nB); }
        for (int g : P.seps) mx_g = std::max(mx_g, gsz(g));
        std::fprintf(stderr,
                     "[hifcn build] level %d: %zu cells (max nI %d, nB %d), %zu separator groups "
                     "(max %d), %zu IDs (max n %d, max m %d, sum m*n %.3g)\n",
                     lev, ct.size(), mx_i, mx_b, P.seps.size(), mx_g, it.size(), mx_n, mx_m, mn);
      }
      // IDs of at least qr_multi columns take the multi-workgroup QR
      std::vector<IdTask> small, big;
      int big_steps = 0, big_cols = 0;
      for (const IdTask& t : it) {
        if (t.n >= qr_multi) {
          big.push_back(t);
          big_steps = std::max(big_steps, std::min(t.m, t.n));
          big_cols = std::max(big_cols, t.n);
        } else {
          small.push_back(t);
        }
      }
      DevBuf<IdTask> dit, dbig;
      DevBuf<SubBlk> drs;
      DevBuf<double> work(std::max<int64_t>(1, wo), s);
      Xbuf.alloc_on(std::max<int64_t>(1, xo), s);
      DevBuf<int32_t> dperm(std::max<int32_t>(1, po), s);
      DevBuf<int32_t> dk(std::max<size_t>(1, P.skel.size()), s);
      upload(dit, small, s);
      upload(dbig, big, s);
      upload(drs, rs, s);
      if (!small.empty())
        hipLaunchKernelGGL(k_id, dim3(small.size()), dim3(kBT), 0, s, dit.p, drs.p, A.p, work.p,
                           fv.p, Xbuf.p, dperm.p, dk.p, hd.eps, err.p);
      if (!big.empty()) {
        const int nb = (int)big.size();
        DevBuf<int32_t> pw(std::max<int32_t>(1, po), s);
        DevBuf<QrState> qs(nb, s);
        hipLaunchKernelGGL(k_qr_init, dim3(nb), dim3(kBT), 0, s, dbig.p, drs.p, A.p, work.p, pw.p,
                           qs.p);
        for (int st = 0; st <= big_steps; ++st) {
          hipLaunchKernelGGL(k_qr_pivot, dim3(nb), dim3(kBT), 0, s, dbig.p, st, work.p, pw.p,
                             qs.p, hd.eps);
          const int cols = big_cols - st - 1;
          if (st < big_steps && cols > 0)
            hipLaunchKernelGGL(k_qr_apply, dim3((cols + kBT / 64 - 1) / (kBT / 64), nb),
                               dim3(kBT), 0, s, dbig.p, st, work.p, (const QrState*)qs.p);
        }
        // ranks back to the host: the rest is sized by them
        std::vector<QrState> qh(nb);
        HIF_CHECK(hipMemcpyAsync(qh.data(), qs.p, nb * sizeof(QrState), hipMemcpyDeviceToHost,
                                 s));
        HIF_CHECK(hipStreamSynchronize(s));
        hipLaunchKernelGGL(k_qr_t, dim3(nb), dim3(kBT), 0, s, dbig.p, work.p,
                           (const int32_t*)pw.p, (const QrState*)qs.p, fv.p, dperm.p, dk.p);
        std::vector<GemmTask> g_s, g_w, g_x;
        std::vector<FrontTask> f_s;
        std::vector<UnpackTask> u_s;
        for (int q = 0; q < nb; ++q) {
          const IdTask& t = big[q];
          const int n = t.n, m = t.m, k = qh[q].k, nr = n - k;
          double* T = work.p + t.offW + (int64_t)m * n + n + m;  // k x nr col-major
          double* S = T + (int64_t)k * nr;
          double* Li = S + (int64_t)nr * nr;
          double* Wm = Li + (int64_t)nr * nr;
          // X = I - Wm Wm^T (k x k); with nothing redundant (nr = 0) that is the identity
          g_x.push_back({Wm, Wm, Xbuf.p + t.offX, nr, nr, k, k, k, nr, 1, 0, 0, -1.0, 1, 0});
          if (nr == 0) continue;
          g_s.push_back({T, T, S, k, k, nr, nr, nr, k, 1, 0, 0, 1.0, 1, 0});
          f_s.push_back({nr, 0, 0, 0, S - work.p, t.offV + tri64(n) + (int64_t)k * nr, -1, 0, 0});
          u_s.push_back({t.offV + tri64(n) + (int64_t)k * nr, Li - work.p, nr, 0});
          g_w.push_back({T, Li, Wm, k, nr, nr, k, nr, nr, 1, 1, 1, 1.0, 0, 0});
        }
        gemm_batched(g_s, s, &fstats);                                    // S = I + T^T T
        build_fronts(f_s, {}, work.p, nullptr, fv.p, err.p, s, &fstats);  // packed L_s^-1
        if (!u_s.empty()) {
          DevBuf<UnpackTask> du;
          upload(du, u_s, s);
          hipLaunchKernelGGL(k_unpack_tri, dim3(u_s.size()), dim3(kBT), 0, s,
                             (const UnpackTask*)du.p, (const double*)fv.p, work.p);
          HIF_CHECK(hipGetLastError());
          gemm_batched(g_w, s, &fstats);  // Wm = T L_s^-T (also synchronises before du goes)
        }
        gemm_batched(g_x, s, &fstats);    // X = I - Wm Wm^T
        HIF_CHECK(hipGetLastError());
        check_err("skeletonization");  // synchronises: pw and qs are released after their use
      }
      HIF_CHECK(hipGetLastError());
      permv.resize(po);
      if (po)
        HIF_CHECK(hipMemcpyAsync(permv.data(), dperm.p, po * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, s));
      if (!kval.empty())
        HIF_CHECK(hipMemcpyAsync(kval.data(), dk.p, kval.size() * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, s));
      check_err("skeletonization");
    }

    mark("skeletons", lev);
    // ---- record this level's apply layout
    std::vector<int> gk(G, -1);
    for (size_t q = 0; q < P.skel.size(); ++q) gk[P.skel[q]] = kval[q];
    int64_t cbn = 0;
    std::vector<int64_t> cell_cb(P.cells.size());
    for (size_t ci = 0; ci < P.cells.size(); ++ci) {
      const int c = P.cells[ci];
      CellDesc d{};
      d.nI = gsz(c);
      d.nB = cell_nB[ci];
      d.offV = (int32_t)cell_voff[ci];  // chunk-relative for now
      d.offCB = (int32_t)cbn;
      d.mode = cmode;
      lo.cellIb.push_back(cell_ib[ci]);
      cell_cb[ci] = cbn;
      cbn += d.nB;
      lo.cells.push_back(d);
      lo.cellI.push_back(P.groups[c].dofs);
      std::vector<int32_t> B;
      for (int b : P.cellB[ci]) B.insert(B.end(), P.groups[b].dofs.begin(), P.groups[b].dofs.end());
      lo.cellB.push_back(std::move(B));
      lo.maxI = std::max(lo.maxI, d.nI);
      lo.maxB = std::max(lo.maxB, d.nB);
      const int64_t cv = tri64(d.nI) + (cmode ? (int64_t)d.nB : (int64_t)d.nI * d.nB);
      lo.maxCV = std::max<int>(lo.maxCV, (int)cv);
      nvals_actual += cv;
    }
    lo.cbn = cbn;
    // gather map of boundary contributions, in cell order
    std::vector<int> sep_index(G, -1);
    for (size_t q = 0; q < P.seps.size(); ++q) sep_index[P.seps[q]] = (int)q;
    // slots of separator DOF p of group q: sstart[sbase[q] + p] .. (counting sort, cell order)
    std::vector<int64_t> sbase(P.seps.size() + 1, 0);
    for (size_t q = 0; q < P.seps.size(); ++q) sbase[q + 1] = sbase[q] + gsz(P.seps[q]);
    std::vector<int32_t> sstart(sbase.back() + 1, 0);
    for (size_t ci = 0; ci < P.cells.size(); ++ci)
      for (int b : P.cellB[ci]) {
        const int64_t s0 = sbase[sep_index[b]];
        for (int p = 0; p < gsz(b); ++p) ++sstart[s0 + p + 1];
      }
    for (int64_t e = 0; e < sbase.back(); ++e) sstart[e + 1] += sstart[e];
    std::vector<int32_t> sval(sstart.back());
    {
      std::vector<int32_t> fillp(sstart.begin(), sstart.end() - 1);
      for (size_t ci = 0; ci < P.cells.size(); ++ci) {
        int64_t o = cell_cb[ci];
        for (int b : P.cellB[ci]) {
          const int64_t s0 = sbase[sep_index[b]];
          for (int p = 0; p < gsz(b); ++p) sval[fillp[s0 + p]++] = (int32_t)(o + p);
          o += gsz(b);
        }
      }
    }
    std::vector<std::vector<int32_t>> surv(G);
    for (size_t q = 0; q < P.seps.size(); ++q) {
      const int g = P.seps[q];
      const int n = gsz(g);
      GroupDesc d{};
      d.n = n;
      d.nr = gk[g] >= 0 ? n - gk[g] : 0;
      d.offV = (int32_t)grp_voff[g];
      d.cap = (int32_t)(2 * tri64(n));
      lo.gids.push_back(P.groups[g].dofs);
      std::vector<int32_t> pm;
      if (gk[g] >= 0) {
        pm.assign(permv.begin() + perm_off[g], permv.begin() + perm_off[g] + n);
        surv[g].assign(pm.begin() + d.nr, pm.end());
      } else {
        surv[g].resize(n);
        for (int i = 0; i < n; ++i) surv[g][i] = i;
      }
      lo.gperm.push_back(pm);
      const int32_t* sp = sstart.data() + sbase[q];
      std::vector<int32_t> ptr(n + 1);
      for (int p = 0; p <= n; ++p) ptr[p] = sp[p] - sp[0];
      std::vector<int32_t> sl(sval.begin() + sp[0], sval.begin() + sp[n]);
      lo.gslots_ptr.push_back(std::move(ptr));
      lo.gslots.push_back(std::move(sl));
      lo.groups.push_back(d);
      lo.maxG = std::max(lo.maxG, n);
      lo.maxR = std::max(lo.maxR, d.nr);
      lo.maxK = std::max(lo.maxK, n - d.nr);
      const int64_t kk = n - d.nr;
      nvals_actual += tri64(n) + (d.nr ? kk * d.nr + tri64(d.nr) : 0);
      lo.maxGV = std::max<int>(lo.maxGV, (int)(tri64(n) + kk * d.nr + tri64(d.nr)));
    }
    lo.base = total_chunk;
    total_chunk += voff;
    outs.push_back(std::move(lo));
    chunks.push_back(std::move(fv));

    // ---- regroup into level l+1
    mark("layout", lev);
    LevelPlan Pn = plan_next(geo, P, surv);
    mark("plan next", lev);
    DevBuf<double> An(std::max<int64_t>(1, Pn.nvals), s);
    {
      std::vector<RegroupTask> rt;
      std::vector<RowSrc> rows;
      std::vector<SrcEnt> src;
      std::vector<int32_t> rows_off(Pn.groups.size());
      for (size_t g = 0; g < Pn.groups.size(); ++g) {
        rows_off[g] = (int32_t)rows.size();
        rows.insert(rows.end(), Pn.rows[g].begin(), Pn.rows[g].end());
      }
      for (size_t b = 0; b < Pn.blocks.size(); ++b) {
        const int Gi = Pn.blocks[b].first, Hi = Pn.blocks[b].second;
        const std::vector<int>& sg = Pn.subs[Gi];
        const std::vector<int>& sh = Pn.subs[Hi];
        RegroupTask t{};
        t.dst = Pn.block_off[b];
        t.nG = (int32_t)Pn.groups[Gi].dofs.size();
        t.nH = (int32_t)Pn.groups[Hi].dofs.size();
        t.offRowsG = rows_off[Gi];
        t.offRowsH = rows_off[Hi];
        t.nsubH = (int32_t)sh.size();
        t.offSrc = (int32_t)src.size();
        for (int ga : sg)
          for (int hb : sh) {
            if (ga == hb) {
              src.push_back({-2, 0, ga});
            } else {
              const int blk = P.find_block(ga, hb);
              src.push_back(blk >= 0 ? SrcEnt{P.block_off[blk], gsz(hb), 0} : SrcEnt{-1, 0, 0});
            }
          }
        rt.push_back(t);
      }
      std::vector<int32_t> gkv(G, 0);
      for (int g = 0; g < G; ++g) gkv[g] = gk[g] >= 0 ? gk[g] : 0;
      DevBuf<RegroupTask> drt;
      DevBuf<RowSrc> drows;
      DevBuf<SrcEnt> dsrc;
      DevBuf<int64_t> dxoff;
      DevBuf<int32_t> dgk;
      upload(drt, rt, s);
      upload(drows, rows, s);
      upload(dsrc, src, s);
      upload(dxoff, xoff, s);
      upload(dgk, gkv, s);
      int64_t maxtot = 0;
      for (const RegroupTask& t : rt) maxtot = std::max<int64_t>(maxtot, (int64_t)t.nG * t.nH);
      const int slices = (int)std::min<int64_t>(64, std::max<int64_t>(1, maxtot / (1 << 16)));
      if (!rt.empty())
        hipLaunchKernelGGL(k_regroup, dim3(rt.size(), slices), dim3(kBT), 0, s, drt.p, drows.p,
                           dsrc.p, A.p, Xbuf.p, dxoff.p, dgk.p, An.p);
      HIF_CHECK(hipGetLastError());
      HIF_CHECK(hipStreamSynchronize(s));
    }
    A = std::move(An);
    P = std::move(Pn);
    mark("regroup", lev);
  }

  // ---- root: the single group left at level L
  mark("(levels done)", hd.L);
  HIF_REQUIRE(P.cells.size() == 1 && P.seps.empty(), HIF_ERR_ARG, "internal: root is not one cell");
  const int rg = P.cells[0];
  const int nroot = (int)P.groups[rg].dofs.size();
  DevBuf<double> rchunk(std::max<int64_t>(1, tri64(nroot)), s);
  if (nroot >= front_min) {
    build_fronts({FrontTask{nroot, 0, 0, 0, P.block_off[P.find_block(rg, rg)], 0, -1, 0, 0}}, {},
                 A.p, nullptr, rchunk.p, err.p, s, &fstats);
    check_err("root factorization");
  } else {
    std::vector<CellTask> ct(1);
    ct[0] = {nroot, 0, 0, 0, P.block_off[P.find_block(rg, rg)], 0, 0, 0, 0, 0};
    DevBuf<CellTask> dct;
    DevBuf<SubBlk> dsub(1, s);
    DevBuf<int32_t> dibl(1, s);
    DevBuf<double> work(std::max<int64_t>(1, 2 * (int64_t)nroot * nroot), s);
    DevBuf<double> schur(1, s);
    upload(dct, ct, s);
    hipLaunchKernelGGL(k_build_cells, dim3(1), dim3(kBT), 0, s, dct.p, dsub.p, dibl.p, A.p,
                       work.p, schur.p, rchunk.p, err.p);
    HIF_CHECK(hipGetLastError());
    check_err("root factorization");
  }
  nvals_actual += tri64(nroot);
  const int64_t root_base = total_chunk;
  total_chunk += align_vals(tri64(nroot));

  // ---- final layout: descriptors and indices on the host, values converted on the device
  FactorDev& f = hd.f;
  f.store = store;
  f.lv.clear();
  f.lv.resize(outs.size());
  std::vector<int32_t> idx;
  int64_t cbmax = 0;
  for (size_t l = 0; l < outs.size(); ++l) {
    LevelOut& lo = outs[l];
    LevelDev& ld = f.lv[l];
    for (size_t c = 0; c < lo.cells.size(); ++c) {
      CellDesc& d = lo.cells[c];
      d.offV = (int32_t)(lo.base + d.offV);
      d.offI = (int32_t)idx.size();
      idx.insert(idx.end(), lo.cellI[c].begin(), lo.cellI[c].end());
      d.offB = (int32_t)idx.size();
      idx.insert(idx.end(), lo.cellB[c].begin(), lo.cellB[c].end());
      d.offC = (int32_t)idx.size();
      idx.insert(idx.end(), lo.cellIb[c].begin(), lo.cellIb[c].end());
      if (d.mode >= 1) {  // links grouped by interior DOF: rowptr[nI + 1], blist[nB]
        const std::vector<int32_t>& ib = lo.cellIb[c];
        std::vector<int32_t> rp(d.nI + 1, 0), bl(ib.size());
        for (int32_t i : ib) ++rp[i + 1];
        for (int i = 0; i < d.nI; ++i) rp[i + 1] += rp[i];
        std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
        for (size_t b = 0; b < ib.size(); ++b) bl[fill[ib[b]]++] = (int32_t)b;
        idx.insert(idx.end(), rp.begin(), rp.end());
        idx.insert(idx.end(), bl.begin(), bl.end());
      }
    }
    for (size_t q = 0; q < lo.groups.size(); ++q) {
      GroupDesc& d = lo.groups[q];
      d.offV = (int32_t)(lo.base + d.offV);
      d.offIdx = (int32_t)idx.size();
      idx.insert(idx.end(), lo.gids[q].begin(), lo.gids[q].end());
      d.offPerm = (int32_t)idx.size();
      idx.insert(idx.end(), lo.gperm[q].begin(), lo.gperm[q].end());
      d.offGP = (int32_t)idx.size();
      idx.insert(idx.end(), lo.gslots_ptr[q].begin(), lo.gslots_ptr[q].end());
      idx.insert(idx.end(), lo.gslots[q].begin(), lo.gslots[q].end());
    }
    ld.ncell = (int)lo.cells.size();
    ld.ngroup = (int)lo.groups.size();
    ld.maxI = lo.maxI;
    ld.maxB = lo.maxB;
    ld.maxG = lo.maxG;
    ld.maxK = lo.maxK;
    ld.maxR = lo.maxR;
    ld.maxCV = lo.maxCV;
    ld.maxGV = lo.maxGV;
    ld.cmode = lo.cells.empty() ? 0 : lo.cells[0].mode;
    if (ld.cmode == 2) build_sym_table(f, lo.cells, s);
    {
      std::vector<int64_t> nsl(lo.groups.size());
      for (size_t q = 0; q < lo.groups.size(); ++q) nsl[q] = (int64_t)lo.gslots[q].size();
      level_stage_bytes(lo.cells, lo.groups, nsl, store_elem_bytes(store), ld);
    }
    ld.cells.upload(lo.cells, s);
    ld.groups.upload(lo.groups, s);
    cbmax = std::max(cbmax, lo.cbn);
  }
  f.nroot = nroot;
  f.mfma_flops = fstats.flops;
  f.mfma_ms = fstats.ms;
  f.root_bytes = (int64_t)store_elem_bytes(store) * tri64(nroot) + 20 * (int64_t)nroot;
  f.offRootIdx = (int32_t)idx.size();
  idx.insert(idx.end(), P.groups[rg].dofs.begin(), P.groups[rg].dofs.end());
  f.offRootV = root_base;
  HIF_REQUIRE(total_chunk < (int64_t)INT32_MAX && idx.size() < (size_t)INT32_MAX, HIF_ERR_ARG,
              "factor too large for 32-bit offsets");
  f.idx.upload(idx, s);
  f.nvals = nvals_actual;
  const size_t eb = store_elem_bytes(store);
  f.vals.alloc((total_chunk + kValAlign) * eb);
  HIF_CHECK(hipMemsetAsync(f.vals.p, 0, (total_chunk + kValAlign) * eb, s));
  auto convert = [&](const double* src, int64_t base, int64_t n) {
    if (n == 0) return;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (store == HIF_STORE_F64)
      hipLaunchKernelGGL(k_to_store_f64, dim3(blocks), dim3(256), 0, s, src,
                         reinterpret_cast<double*>(f.vals.p) + base, n);
    else if (store == HIF_STORE_F32)
      hipLaunchKernelGGL(k_to_store_f32, dim3(blocks), dim3(256), 0, s, src,
                         reinterpret_cast<float*>(f.vals.p) + base, n);
    else
      hipLaunchKernelGGL(k_to_store_bf16, dim3(blocks), dim3(256), 0, s, src,
                         reinterpret_cast<bf16_t*>(f.vals.p) + base, n);
  };
  for (size_t l = 0; l < outs.size(); ++l) {
    const int64_t n = (l + 1 < outs.size() ? outs[l + 1].base : root_base) - outs[l].base;
    convert(chunks[l].p, outs[l].base, n);
  }
  mark("root", hd.L);
  convert(rchunk.p, root_base, tri64(nroot));
  HIF_CHECK(hipGetLastError());
  mark("store", hd.L);
  f.cbstride = std::max<int64_t>(1, cbmax);
  f.cb.alloc(2 * f.cbstride);
  {
    std::vector<std::vector<CellDesc>> cells;
    std::vector<std::vector<GroupDesc>> groups;
    for (const LevelOut& lo : outs) {
      cells.push_back(lo.cells);
      groups.push_back(lo.groups);
    }
    setup_tiling(f, cells, groups, idx, s);
    setup_dense_groups(f, groups, idx, dense_top_level(f, cells, groups), s);
    setup_fusion(f, cells, groups, idx, hd.N, s);
    setup_dense_top(f, cells, groups, idx, hd.N, s);
    setup_cg_gate(f, cells, idx, hd.N, s);
  }
  size_t worst = 0;
  apply_smem_need(f, &worst);
  f.smem_max = worst;
  HIF_REQUIRE(worst <= 160 * 1024, HIF_ERR_ARG, "factor blocks too large for the apply kernels");
  if (worst > 64 * 1024) set_apply_smem_limits(worst);
  HIF_CHECK(hipStreamSynchronize(s));
  mark("apply setup", hd.L);
}

}  // namespace hifcn
