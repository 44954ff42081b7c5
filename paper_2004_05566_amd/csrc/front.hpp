// Dense FP64 elimination of large cells and of the root on the matrix cores (Sec. 2.2, eq2_3,
// eq3_4).  Used by the factor build for cells too large for one workgroup.
#pragma once

#include <vector>

#include "common.hpp"

namespace hifcn {

// One cell to eliminate.  Inputs live in the build's block table A (row-major blocks): A_II
// (nI x nI at offAII) and A_IB as nsub column blocks (nI x width at FrontSub.off).  Outputs:
// packed column-major L^-1 (nI(nI+1)/2) at fv + offV followed, if nB > 0, by H = A_BI A_II^-1
// column-major (nB x nI), and the Schur complement S = A_BI A_II^-1 A_IB (nB x nB row-major) at
// schur + offS.
struct FrontTask {
  int32_t nI, nB, nsub, offSub;
  int64_t offAII, offV, offS;
  int64_t offF, offD;  // internal: the front and the diagonal-block inverse (set by the driver)
  // mode 1 (stencil links): instead of H, store the single coupling A_IB(ib_b, b) of each
  // boundary DOF b, with ib_b = ibl[offIb + b]
  int32_t mode = 0, offIb = 0;
};
struct FrontSub {
  int64_t off;
  int32_t width, pad;
};

// Work done on the matrix cores: algorithmic FP64 flops of the panel, trailing-update and H
// products, and the summed durations of those kernels (HIP events around each launch).
struct FrontStats {
  int64_t flops = 0;
  double ms = 0;
  int64_t launches = 0;
};

// One product C = alpha op(A) op(B) (+ I if addI) of row-major FP64 matrices (m x n result,
// inner dimension k): op(B) = B^T if nt = 1, else B; op(A) = A, or with ta = 1 A is given as
// its transpose (k x m).  tri = 1: column j of the result needs only inner indices <= j (op(B)
// = L^T with L lower); tri = 2: row i needs only inner indices <= i (op(A) lower triangular);
// tri = 3: entry (i, j) needs only inner indices >= max(i, j) (op(A) = L^T, op(B) = L, square).
struct GemmTask {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int32_t m, n, k, nt, tri, ta;
  double alpha;
  int32_t addI, pad;
};

// Run every product (batched: one launch over the 64 x 64 tiles of all of them).  C must not
// overlap A or B.
void gemm_batched(const std::vector<GemmTask>& tasks, hipStream_t s, FrontStats* stats = nullptr);

// Factor every task (batched: each kernel covers all tasks).  A non-positive pivot raises *err.
// Synchronises the stream when `stats` is given (to read the kernel timings).
// Fronts are processed in batches of at most about 2 GiB of front storage.  ibl: device copy
// of the interior positions of mode-1 tasks (may be NULL when there are none).
void build_fronts(std::vector<FrontTask> tasks, const std::vector<FrontSub>& subs,
                  const double* A, double* schur, double* fv, int* err, hipStream_t s,
                  FrontStats* stats = nullptr, const int32_t* ibl = nullptr);

}  // namespace hifcn
