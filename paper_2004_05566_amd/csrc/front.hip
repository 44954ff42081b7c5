// Dense FP64 work of the factor build on the matrix cores (Sec. 2.2): the elimination of large
// cells and of the root (eq2_3, eq3_4), and batched products (the block-Jacobi rescaling).
//
// A cell with interior I and boundary B is eliminated through the augmented front
//
//          [ A_II  A_IB ]      rows I (nI), B (nB), E (nI); columns I, B; only the lower
//     F =  [ A_BI   0   ]      triangle is used (F is symmetric)
//          [  I         ]
//
// by a blocked right-looking Cholesky over the nI interior columns.  Afterwards its lower
// triangle holds
//     I rows : L = chol(A_II)
//     B rows : A_BI L^-T = G^T              with G = L^-1 A_IB
//     E rows : L^-T                         (row j of E is column j of L^-1)
//     B x B  : -G^T G = -S                  (minus the Schur complement)
// so one pass yields every block the apply and the next level need; H = G^T L^-1 is one more
// product.  Per panel of 64 columns: the diagonal block is factored and inverted by one
// workgroup, the panel rows are multiplied by that inverse, and the trailing update runs as
// 64 x 64 tiles of v_mfma_f64_16x16x4f64.  The update is restricted to what the results above
// read: E rows only against interior columns, and only the E rows that are nonzero so far
// (L^-T is upper triangular, so E row j is zero left of column j).
#include <hip/hip_ext.h>

#include <algorithm>

#include "front.hpp"

namespace hifcn {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kT = 64;         // output tile and panel width
constexpr int kKc = 32;        // K chunk staged in LDS
constexpr int kLd = kKc + 1;   // LDS row stride of a staged chunk (doubles)
constexpr int kThreads = 256;  // 4 wavefronts; wave w owns the 32 x 32 quadrant (w / 2, w % 2)

__device__ __forceinline__ int64_t front_ld(const FrontTask& t) { return t.nI + t.nB; }

// A 64 x kKc chunk of an operand on its way to LDS: each thread holds 8 of its elements, so a
// chunk's global loads can be issued while the matrix cores work on the previous chunk.
struct Chunk {
  double v[kT * kKc / kThreads];
};
constexpr int kChunkPer = kT * kKc / kThreads;

// Rows [0, rows) x columns [0, kv) of src (leading dimension ld), zero elsewhere; thread t holds
// row t / kKc + 8 u, column t % kKc (32 consecutive lanes read one row segment).
__device__ __forceinline__ void load_chunk(Chunk& R, const double* src, int64_t ld, int rows,
                                           int kv) {
  const int c = threadIdx.x % kKc, r0 = threadIdx.x / kKc;
#pragma unroll
  for (int u = 0; u < kChunkPer; ++u) {
    const int r = r0 + (kThreads / kKc) * u;
    R.v[u] = (r < rows && c < kv) ? src[(int64_t)r * ld + c] : 0.0;
  }
}
// Rows [0, kv) x columns [0, cols) of src, to be stored transposed; thread t holds row
// t / kT + 4 u, column t % kT.
__device__ __forceinline__ void load_chunk_t(Chunk& R, const double* src, int64_t ld, int kv,
                                             int cols) {
  const int j = threadIdx.x % kT, k0 = threadIdx.x / kT;
#pragma unroll
  for (int u = 0; u < kChunkPer; ++u) {
    const int k = k0 + (kThreads / kT) * u;
    R.v[u] = (k < kv && j < cols) ? src[(int64_t)k * ld + j] : 0.0;
  }
}
// The chunk into S (64 x kKc, stride kLd): as loaded, or transposed (S[j][k] = src[k][j]).
__device__ __forceinline__ void store_chunk(double* S, const Chunk& R) {
  const int c = threadIdx.x % kKc, r0 = threadIdx.x / kKc;
#pragma unroll
  for (int u = 0; u < kChunkPer; ++u) S[(r0 + (kThreads / kKc) * u) * kLd + c] = R.v[u];
}
__device__ __forceinline__ void store_chunk_t(double* S, const Chunk& R) {
  const int j = threadIdx.x % kT, k0 = threadIdx.x / kT;
#pragma unroll
  for (int u = 0; u < kChunkPer; ++u) S[j * kLd + k0 + (kThreads / kT) * u] = R.v[u];
}

// acc += As (64 x kKc) * Bs (64 x kKc)^T.  MFMA 16x16x4 FP64 operands: lane l holds A[l%16][l/16]
// and B^T[l%16][l/16]; accumulator element r of lane l is row 4r + l/16, column l%16 (the FP64
// form interleaves the rows, unlike the 4(l/16) + r of the FP16/BF16 forms).
__device__ __forceinline__ void mfma_chunk(const double* As, const double* Bs, d4 acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int ra = 32 * (w >> 1), cb = 32 * (w & 1);
#pragma unroll
  for (int k0 = 0; k0 < kKc; k0 += 4) {
    const double a0 = As[(ra + i) * kLd + k0 + kk];
    const double a1 = As[(ra + 16 + i) * kLd + k0 + kk];
    const double b0 = Bs[(cb + i) * kLd + k0 + kk];
    const double b1 = Bs[(cb + 16 + i) * kLd + k0 + kk];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// Tile position of accumulator element (a, b, r) of this lane.
__device__ __forceinline__ void acc_pos(int a, int b, int r, int* row, int* col) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  *row = 32 * (w >> 1) + 16 * a + 4 * r + (lane >> 4);
  *col = 32 * (w & 1) + 16 * b + (lane & 15);
}

// acc = A (rows x K) * B (cols x K)^T over k in [k_begin, k_end), both row-major with ld.  The
// next chunk's loads are in flight while the matrix cores multiply the current one.
__device__ void tile_nt(const double* A, const double* B, int64_t ld, int rows, int cols,
                        int k_begin, int k_end, d4 acc[2][2]) {
  __shared__ double As[kT * kLd], Bs[kT * kLd];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  Chunk ra, rb;
  if (k_begin < k_end) {
    const int kv = min(kKc, k_end - k_begin);
    load_chunk(ra, A + k_begin, ld, rows, kv);
    load_chunk(rb, B + k_begin, ld, cols, kv);
  }
  for (int k0 = k_begin; k0 < k_end; k0 += kKc) {
    store_chunk(As, ra);
    store_chunk(Bs, rb);
    __syncthreads();
    const int k1 = k0 + kKc;
    if (k1 < k_end) {
      const int kv = min(kKc, k_end - k1);
      load_chunk(ra, A + k1, ld, rows, kv);
      load_chunk(rb, B + k1, ld, cols, kv);
    }
    mfma_chunk(As, Bs, acc);
    __syncthreads();
  }
}

// Row segments of a panel step at column k (width w): interior rows below the panel, all
// boundary rows, and the E rows that are nonzero so far.  Block index -> (first row, rows).
__device__ bool panel_rows(const FrontTask& t, int k, int w, int blk, int* r0, int* rows,
                           int* seg) {
  const int s1 = t.nI - k - w, s2 = t.nB, s3 = min(k + w, t.nI);
  const int b1 = (s1 + kT - 1) / kT, b2 = (s2 + kT - 1) / kT, b3 = (s3 + kT - 1) / kT;
  if (blk < b1) {
    *seg = 0;
    *r0 = k + w + blk * kT;
    *rows = min(kT, t.nI - *r0);
  } else if (blk < b1 + b2) {
    *seg = 1;
    *r0 = t.nI + (blk - b1) * kT;
    *rows = min(kT, t.nI + t.nB - *r0);
  } else if (blk < b1 + b2 + b3) {
    *seg = 2;
    const int j0 = (blk - b1 - b2) * kT;
    *r0 = t.nI + t.nB + j0;
    *rows = min(kT, s3 - j0);
  } else {
    return false;
  }
  return true;
}

__global__ __launch_bounds__(kThreads) void k_front_init(const FrontTask* __restrict__ tasks,
                                                         const FrontSub* __restrict__ subs,
                                                         const double* __restrict__ A,
                                                         double* __restrict__ F,
                                                         const int32_t* __restrict__ ibl,
                                                         double* __restrict__ fv) {
  const FrontTask t = tasks[blockIdx.y];
  const int64_t ld = front_ld(t);
  const int R = 2 * t.nI + t.nB;
  for (int r = blockIdx.x * 4; r < min(R, (int)blockIdx.x * 4 + 4); ++r) {
    double* row = F + t.offF + (int64_t)r * ld;
    if (r < t.nI) {
      for (int c = threadIdx.x; c < ld; c += kThreads)
        row[c] = c < t.nI ? A[t.offAII + (int64_t)r * t.nI + c] : 0.0;
    } else if (r < t.nI + t.nB) {
      // boundary DOF b lies in column block q at local column b - c0
      const int b = r - t.nI;
      int q = 0, c0 = 0;
      while (q + 1 < t.nsub && b >= c0 + subs[t.offSub + q].width) c0 += subs[t.offSub + q++].width;
      const FrontSub sb = subs[t.offSub + q];
      for (int c = threadIdx.x; c < ld; c += kThreads)
        row[c] = c < t.nI ? A[sb.off + (int64_t)c * sb.width + (b - c0)] : 0.0;
      if (t.mode == 1 && threadIdx.x == 0)  // the boundary DOF's one coupling, kept for the apply
        fv[t.offV + tri_count(t.nI) + b] = A[sb.off + (int64_t)ibl[t.offIb + b] * sb.width + (b - c0)];
    } else {
      const int j = r - t.nI - t.nB;
      for (int c = threadIdx.x; c < ld; c += kThreads) row[c] = (c == j) ? 1.0 : 0.0;
    }
  }
}

// Factor the diagonal block of the panel at column k in LDS, write L11 back and L11^-1 to D.
__global__ __launch_bounds__(kThreads) void k_front_diag(const FrontTask* __restrict__ tasks,
                                                         int k, double* __restrict__ F,
                                                         double* __restrict__ D, int* err) {
  __shared__ double Ls[kT * (kT + 1)], Ys[kT * (kT + 1)];
  constexpr int ls = kT + 1;
  const FrontTask t = tasks[blockIdx.x];
  const int w = min(kT, t.nI - k);
  if (w <= 0) return;
  const int64_t ld = front_ld(t);
  double* Fk = F + t.offF + (int64_t)k * ld + k;
  for (int e = threadIdx.x; e < kT * kT; e += kThreads) {
    const int i = e / kT, j = e - i * kT;
    Ls[i * ls + j] = (i < w && j <= i) ? Fk[(int64_t)i * ld + j] : 0.0;
    Ys[i * ls + j] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (threadIdx.x == 0) {
      double d = Ls[j * ls + j];
      if (!(d > 0.0) || !(d < 1.0e300)) {
        *err = 1;
        d = 1.0;
      }
      Ls[j * ls + j] = sqrt(d);
    }
    __syncthreads();
    const double p = Ls[j * ls + j];
    for (int i = j + 1 + threadIdx.x; i < w; i += kThreads) Ls[i * ls + j] /= p;
    __syncthreads();
    const int m = w - j - 1;
    for (int e = threadIdx.x; e < m * m; e += kThreads) {
      const int r = e / m, c = e - r * m;
      if (c <= r) Ls[(j + 1 + r) * ls + j + 1 + c] -= Ls[(j + 1 + r) * ls + j] * Ls[(j + 1 + c) * ls + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < w * w; e += kThreads) {
    const int i = e / w, j = e - i * w;
    if (j <= i) Fk[(int64_t)i * ld + j] = Ls[i * ls + j];
  }
  // column c of L11^-1 by forward substitution, one thread per column
  if (threadIdx.x < w) {
    const int c = threadIdx.x;
    Ys[c * ls + c] = 1.0 / Ls[c * ls + c];
    for (int i = c + 1; i < w; ++i) {
      double acc = 0.0;
      for (int q = c; q < i; ++q) acc += Ls[i * ls + q] * Ys[q * ls + c];
      Ys[i * ls + c] = -acc / Ls[i * ls + i];
    }
  }
  __syncthreads();
  double* Dt = D + t.offD;
  for (int e = threadIdx.x; e < kT * kT; e += kThreads) {
    const int i = e / kT, j = e - i * kT;
    Dt[e] = Ys[i * ls + j];
  }
}

// Panel rows times L11^-T: X[r][:] = F[r][k:k+w] L11^-T.
__global__ __launch_bounds__(kThreads) void k_front_panel(const FrontTask* __restrict__ tasks,
                                                          int k, double* __restrict__ F,
                                                          const double* __restrict__ D) {
  const FrontTask t = tasks[blockIdx.y];
  const int w = min(kT, t.nI - k);
  if (w <= 0) return;
  int r0, rows, seg;
  if (!panel_rows(t, k, w, blockIdx.x, &r0, &rows, &seg)) return;
  const int64_t ld = front_ld(t);
  double* Fr = F + t.offF + (int64_t)r0 * ld + k;
  d4 acc[2][2];
  // B operand: D (64 x 64, ld 64) staged in the same chunks
  __shared__ double As[kT * kLd], Bs[kT * kLd];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  Chunk ra, rb;
  load_chunk(ra, Fr, ld, rows, min(kKc, w));
  load_chunk(rb, D + t.offD, kT, kT, min(kKc, w));
  for (int k0 = 0; k0 < w; k0 += kKc) {
    store_chunk(As, ra);
    store_chunk(Bs, rb);
    __syncthreads();
    const int k1 = k0 + kKc;
    if (k1 < w) {
      load_chunk(ra, Fr + k1, ld, rows, min(kKc, w - k1));
      load_chunk(rb, D + t.offD + k1, kT, kT, min(kKc, w - k1));
    }
    mfma_chunk(As, Bs, acc);
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(a, b, r, &row, &col);
        if (row < rows && col < w) Fr[(int64_t)row * ld + col] = acc[a][b][r];
      }
}

// Trailing update F[r][c] -= sum_t X[r][t] X[c][t] over the columns right of the panel.
__global__ __launch_bounds__(kThreads) void k_front_update(const FrontTask* __restrict__ tasks,
                                                           int k, double* __restrict__ F) {
  const FrontTask t = tasks[blockIdx.z];
  const int w = min(kT, t.nI - k);
  if (w <= 0) return;
  int r0, rows, seg;
  if (!panel_rows(t, k, w, blockIdx.y, &r0, &rows, &seg)) return;
  const int c0 = k + w + blockIdx.x * kT;
  const int cmax = seg == 2 ? t.nI - 1 : r0 + rows - 1;  // E rows: interior columns only
  if (c0 > cmax) return;
  const int cols = min(kT, cmax - c0 + 1);
  const int64_t ld = front_ld(t);
  double* base = F + t.offF;
  d4 acc[2][2];
  tile_nt(base + (int64_t)r0 * ld + k, base + (int64_t)c0 * ld + k, ld, rows, cols, 0, w, acc);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(a, b, r, &row, &col);
        if (row < rows && col < cols && (seg == 2 || c0 + col <= r0 + row))
          base[(int64_t)(r0 + row) * ld + c0 + col] -= acc[a][b][r];
      }
}

// Packed column-major L^-1 from the E rows and S = -(B x B block), symmetric, row-major.
__global__ __launch_bounds__(kThreads) void k_front_out(const FrontTask* __restrict__ tasks,
                                                        const double* __restrict__ F,
                                                        double* __restrict__ fv,
                                                        double* __restrict__ schur) {
  const FrontTask t = tasks[blockIdx.y];
  const int64_t ld = front_ld(t);
  const int j = blockIdx.x;
  const double* Fb = F + t.offF;
  if (j < t.nI) {
    const double* e = Fb + (int64_t)(t.nI + t.nB + j) * ld;
    double* v = fv + t.offV + colstart(j, t.nI) - j;
    for (int i = j + threadIdx.x; i < t.nI; i += kThreads) v[i] = e[i];
  }
  if (j < t.nB && t.offS >= 0) {
    double* srow = schur + t.offS + (int64_t)j * t.nB;
    for (int b = threadIdx.x; b < t.nB; b += kThreads) {
      const int hi = max(j, b), lo = min(j, b);
      srow[b] = -Fb[(int64_t)(t.nI + hi) * ld + t.nI + lo];
    }
  }
}

// H = G^T L^-1 (nB x nI, stored column-major): H[b][j] = sum_{i >= j} G^T[b][i] E[j][i].
__global__ __launch_bounds__(kThreads) void k_front_h(const FrontTask* __restrict__ tasks,
                                                      const double* __restrict__ F,
                                                      double* __restrict__ fv) {
  const FrontTask t = tasks[blockIdx.z];
  const int b0 = blockIdx.y * kT, j0 = blockIdx.x * kT;
  if (t.mode == 1 || b0 >= t.nB || j0 >= t.nI) return;
  const int64_t ld = front_ld(t);
  const double* Fb = F + t.offF;
  const int rows = min(kT, t.nB - b0), cols = min(kT, t.nI - j0);
  d4 acc[2][2];
  tile_nt(Fb + (int64_t)(t.nI + b0) * ld, Fb + (int64_t)(t.nI + t.nB + j0) * ld, ld, rows, cols,
          j0, t.nI, acc);
  double* H = fv + t.offV + tri_count(t.nI);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(a, b, r, &row, &col);
        if (row < rows && col < cols) H[(int64_t)(j0 + col) * t.nB + b0 + row] = acc[a][b][r];
      }
}


// One 64 x 64 tile (task, first row, first column) of a batched product.
__global__ __launch_bounds__(kThreads) void k_gemm_tiles(const GemmTask* __restrict__ tasks,
                                                         const int4* __restrict__ tiles) {
  __shared__ double As[kT * kLd], Bs[kT * kLd];
  const int4 tl = tiles[blockIdx.x];
  const GemmTask t = tasks[tl.x];
  const int r0 = tl.y, c0 = tl.z;
  const int rows = min(kT, t.m - r0), cols = min(kT, t.n - c0);
  int kend = t.k, kbeg = 0;
  if (t.tri == 1) kend = min(kend, c0 + cols);
  if (t.tri == 2) kend = min(kend, r0 + rows);
  if (t.tri == 3) kbeg = max(r0, c0);
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // the operands of chunk k0 into registers (A transposed when ta, B when not nt)
  Chunk ra, rb;
  auto load = [&](int k0) {
    const int kv = min(kKc, kend - k0);
    if (t.ta) load_chunk_t(ra, t.A + (int64_t)k0 * t.lda + r0, t.lda, kv, rows);
    else load_chunk(ra, t.A + (int64_t)r0 * t.lda + k0, t.lda, rows, kv);
    if (t.nt) load_chunk(rb, t.B + (int64_t)c0 * t.ldb + k0, t.ldb, cols, kv);
    else load_chunk_t(rb, t.B + (int64_t)k0 * t.ldb + c0, t.ldb, kv, cols);
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kKc) {
    if (t.ta) store_chunk_t(As, ra);
    else store_chunk(As, ra);
    if (t.nt) store_chunk(Bs, rb);
    else store_chunk_t(Bs, rb);
    __syncthreads();
    if (k0 + kKc < kend) load(k0 + kKc);  // in flight during the products below
    mfma_chunk(As, Bs, acc);
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        int row, col;
        acc_pos(a, b, r, &row, &col);
        if (row < rows && col < cols)
          t.C[(int64_t)(r0 + row) * t.ldc + c0 + col] =
              t.alpha * acc[a][b][r] + ((t.addI && r0 + row == c0 + col) ? 1.0 : 0.0);
      }
}

int cdiv(int64_t a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

void gemm_batched(const std::vector<GemmTask>& tasks, hipStream_t s, FrontStats* stats) {
  if (tasks.empty()) return;
  std::vector<int4> tiles;
  for (size_t q = 0; q < tasks.size(); ++q) {
    const GemmTask& t = tasks[q];
    for (int r0 = 0; r0 < t.m; r0 += kT)
      for (int c0 = 0; c0 < t.n; c0 += kT) tiles.push_back({(int)q, r0, c0, 0});
    if (stats) {  // algorithmic flops (triangular operands count their nonzero part)
      if (t.tri == 1) stats->flops += (int64_t)t.m * t.n * (t.n + 1);
      else if (t.tri == 2) stats->flops += (int64_t)t.n * t.m * (t.m + 1);
      else if (t.tri == 3)  // entries (i, j) with max(i, j) = d: 2d + 1 of them, k - d terms
        for (int64_t d = 0; d < std::min<int64_t>(std::min(t.m, t.n), t.k); ++d)
          stats->flops += 2 * (2 * d + 1) * (t.k - d);
      else stats->flops += 2 * (int64_t)t.m * t.n * t.k;
    }
  }
  if (tiles.empty()) return;
  DevBuf<GemmTask> dt(tasks.size(), s);
  DevBuf<int4> dtl(tiles.size(), s);
  dt.upload(tasks, s);
  dtl.upload(tiles, s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIF_CHECK(hipEventCreate(&e0));
    HIF_CHECK(hipEventCreate(&e1));
    hipExtLaunchKernelGGL(k_gemm_tiles, dim3(tiles.size()), dim3(kThreads), 0, s, e0, e1, 0,
                          (const GemmTask*)dt.p, (const int4*)dtl.p);
  } else {
    hipLaunchKernelGGL(k_gemm_tiles, dim3(tiles.size()), dim3(kThreads), 0, s,
                       (const GemmTask*)dt.p, (const int4*)dtl.p);
  }
  HIF_CHECK(hipGetLastError());
  if (stats) {
    HIF_CHECK(hipStreamSynchronize(s));
    float ms = 0;
    HIF_CHECK(hipEventElapsedTime(&ms, e0, e1));
    stats->ms += ms;
    ++stats->launches;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  // the task and tile lists are released when this returns; hipFree waits for the kernel
}

void build_fronts(std::vector<FrontTask> tasks, const std::vector<FrontSub>& subs,
                  const double* A, double* schur, double* fv, int* err, hipStream_t s,
                  FrontStats* stats, const int32_t* ibl) {
  if (tasks.empty()) return;
  // batches of at most kFrontBatch doubles of front storage
  constexpr int64_t kFrontBatch = int64_t(1) << 28;
  {
    size_t b0 = 0;
    int64_t acc = 0;
    bool split = false;
    for (size_t q = 0; q < tasks.size(); ++q) {
      const int64_t f = (int64_t)(2 * tasks[q].nI + tasks[q].nB) * (tasks[q].nI + tasks[q].nB);
      if (q > b0 && acc + f > kFrontBatch) {
        build_fronts(std::vector<FrontTask>(tasks.begin() + b0, tasks.begin() + q), subs, A,
                     schur, fv, err, s, stats, ibl);
        b0 = q;
        acc = 0;
        split = true;
      }
      acc += f;
    }
    if (split) {
      build_fronts(std::vector<FrontTask>(tasks.begin() + b0, tasks.end()), subs, A, schur, fv,
                   err, s, stats, ibl);
      return;
    }
  }
  // event pairs around every matrix-core launch (only when statistics are wanted)
  std::vector<hipEvent_t> ev;
  auto timed = [&](auto kernel, dim3 grid, auto... args) {
    if (!stats) {
      hipLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, s, args...);
      return;
    }
    hipEvent_t e0, e1;
    HIF_CHECK(hipEventCreate(&e0));
    HIF_CHECK(hipEventCreate(&e1));
    ev.push_back(e0);
    ev.push_back(e1);
    hipExtLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, s, e0, e1, 0, args...);
  };
  int64_t foff = 0;
  int maxR = 0, maxI = 0, maxB = 0, maxLd = 0;
  for (size_t q = 0; q < tasks.size(); ++q) {
    FrontTask& t = tasks[q];
    t.offF = foff;
    t.offD = (int64_t)q * kT * kT;
    foff += (int64_t)(2 * t.nI + t.nB) * (t.nI + t.nB);
    maxR = std::max(maxR, 2 * t.nI + t.nB);
    maxI = std::max(maxI, t.nI);
    maxB = std::max(maxB, t.nB);
    maxLd = std::max(maxLd, t.nI + t.nB);
  }
  const int nt = (int)tasks.size();
  DevBuf<double> F(foff, s), D((size_t)nt * kT * kT, s);
  DevBuf<FrontTask> dt(tasks.size(), s);
  std::vector<FrontSub> sv = subs.empty() ? std::vector<FrontSub>(1) : subs;
  DevBuf<FrontSub> ds(sv.size(), s);
  dt.upload(tasks, s);
  ds.upload(sv, s);
  hipLaunchKernelGGL(k_front_init, dim3(cdiv(maxR, 4), nt), dim3(kThreads), 0, s, dt.p, ds.p, A,
                     F.p, ibl, fv);
  for (int k = 0; k < maxI; k += kT) {
    // grid extents: the largest task at this panel (smaller ones exit at once)
    int prow = 0, pcol = 0;
    for (const FrontTask& t : tasks) {
      const int w = std::min(kT, t.nI - k);
      if (w <= 0) continue;
      prow = std::max(prow, cdiv(t.nI - k - w, kT) + cdiv(t.nB, kT) +
                                cdiv(std::min(k + w, t.nI), kT));
      pcol = std::max(pcol, cdiv(t.nI + t.nB - k - w, kT));
    }
    hipLaunchKernelGGL(k_front_diag, dim3(nt), dim3(kThreads), 0, s, dt.p, k, F.p, D.p, err);
    timed(k_front_panel, dim3(prow, nt), (const FrontTask*)dt.p, k, F.p, (const double*)D.p);
    if (pcol > 0) timed(k_front_update, dim3(pcol, prow, nt), (const FrontTask*)dt.p, k, F.p);
  }
  hipLaunchKernelGGL(k_front_out, dim3(std::max(maxI, maxB), nt), dim3(kThreads), 0, s, dt.p,
                     F.p, fv, schur);
  if (maxB > 0)
    timed(k_front_h, dim3(cdiv(maxI, kT), cdiv(maxB, kT), nt), (const FrontTask*)dt.p,
          (const double*)F.p, fv);
  HIF_CHECK(hipGetLastError());
  if (stats) {
    // algorithmic flops: panel X = F L11^-T (w(w+1) per row), the trailing update over the
    // rows and columns the results read (2w per entry), H = G^T L^-1 (triangular)
    for (const FrontTask& t : tasks) {
      for (int k = 0; k < t.nI; k += kT) {
        const int64_t w = std::min(kT, t.nI - k), m = t.nI - k - w, e = std::min<int64_t>(k + w, t.nI);
        stats->flops += w * (w + 1) * (m + t.nB + e);
        stats->flops += 2 * w * (m * (m + 1) / 2 + (int64_t)t.nB * m +
                                 (int64_t)t.nB * (t.nB + 1) / 2 + e * m);
      }
      if (t.mode == 0) stats->flops += (int64_t)t.nB * t.nI * (t.nI + 1);
    }
    HIF_CHECK(hipStreamSynchronize(s));
    for (size_t q = 0; q < ev.size(); q += 2) {
      float ms = 0;
      HIF_CHECK(hipEventElapsedTime(&ms, ev[q], ev[q + 1]));
      stats->ms += ms;
      ++stats->launches;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  // F and D are released when this returns: the caller's next check synchronises the stream,
  // and hipFree waits for the kernels that use them.
}

}  // namespace hifcn
