// Dense forms of the factor blocks that the apply spreads over many workgroups.
//
// Where one workgroup cannot hold a block, applying it as stored takes several passes (a packed
// triangle read once for L^-1 and once more for L^-T, or the five products of a group step),
// each pass a launch of its own.  For the apply such a block is replaced by the one dense matrix
// the passes multiply out to, applied in a single pass:
//   cell interiors coupled by stencil links, and the root:  M = L^-T L^-1 = A^-1 of the block
//     (eq2_3, eq3_4; symmetric)
//   a group: its whole step G = P^T K P L_g^-1 (block Jacobi, then the skeletonization of
//     eq2_5 / eq2_9), with, in the order (redundant r, skeleton s) given by the pivots P,
//       K = [[L_s^-1, -L_s^-1 T^T], [T L_s^-T L_s^-1, I - T L_s^-T L_s^-1 T^T]];
//     the forward sweep applies G and the backward sweep G^T (eqAinv).
// The products are formed in FP64 on the matrix cores from the stored blocks and rounded once to
// the storage precision.  They are stored column-major with a leading dimension that is a
// multiple of 32 elements, so that every 64-row segment of a column is whole cache lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "front.hpp"
#include "kernels.hpp"

namespace hifcn {
namespace {

constexpr int kB = 256;

template <typename S> __device__ __forceinline__ double ld_s(const S* p) { return (double)*p; }
template <> __device__ __forceinline__ double ld_s<bf16_t>(const bf16_t* p) {
  return (double)__uint_as_float(((uint32_t)p->bits) << 16);
}
template <typename S> __device__ __forceinline__ void st_s(S* p, double v) { *p = (S)v; }
template <> __device__ __forceinline__ void st_s<bf16_t>(bf16_t* p, double v) {
  p->bits = f32_to_bf16_bits((float)v);
}

// FP64 operands of one job (offsets into the batch's scratch).
struct Prep {
  int32_t kind, n, nr, pad;
  int64_t src;      // value block in vals
  int32_t offPerm;  // groups: pivot order in idx (redundant first)
  int32_t pad2;
  int64_t a, x1, ls, tr;  // kind 0: a = L^-1 (n x n);  kind 1: a = P L_g^-1, X1 = [I, -T^T],
                          // L_s^-1 (nr x nr), T^T (nr x k); all dense row-major
};

// Unpack the stored blocks of every job into dense row-major FP64.
template <typename S>
__global__ __launch_bounds__(kB) void k_dense_unpack(const Prep* __restrict__ jobs,
                                                     const int32_t* __restrict__ idx,
                                                     const S* __restrict__ vals,
                                                     double* __restrict__ w) {
  const Prep t = jobs[blockIdx.y];
  const int n = t.n, nr = t.nr, k = n - nr;
  const S* Lg = vals + t.src;
  const int32_t* perm = idx + t.offPerm;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = e0; e < (int64_t)n * n; e += step) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const int p = (t.kind == 1 && nr > 0) ? perm[i] : i;
    w[t.a + e] = j <= p ? ld_s(Lg + colstart(j, n) + (p - j)) : 0.0;
  }
  if (t.kind != 1 || nr == 0) return;
  const S* T = Lg + tri_count(n);       // T[j * k + s]: row j of T^T
  const S* Ls = T + (int64_t)k * nr;    // packed L_s^-1
  for (int64_t e = e0; e < (int64_t)nr * n; e += step) {
    const int i = (int)(e / n), c = (int)(e - (int64_t)i * n);
    w[t.x1 + e] = c < nr ? (c == i ? 1.0 : 0.0) : -ld_s(T + (int64_t)i * k + (c - nr));
  }
  for (int64_t e = e0; e < (int64_t)nr * nr; e += step) {
    const int i = (int)(e / nr), j = (int)(e - (int64_t)i * nr);
    w[t.ls + e] = j <= i ? ld_s(Ls + colstart(j, nr) + (i - j)) : 0.0;
  }
  for (int64_t e = e0; e < (int64_t)nr * k; e += step) w[t.tr + e] = ld_s(T + e);
}

// dvals[dst + j * ld + row(i)] = src[i * n + j], row(i) = perm[i] for skeletonized groups.
struct Store {
  int64_t src, dst;
  int32_t n, ld, offPerm, pad;  // offPerm < 0: rows in order
};
template <typename S>
__global__ __launch_bounds__(kB) void k_dense_store(const Store* __restrict__ jobs,
                                                    const int32_t* __restrict__ idx,
                                                    const double* __restrict__ w,
                                                    S* __restrict__ dv) {
  const Store t = jobs[blockIdx.y];
  const int n = t.n;
  const int32_t* perm = t.offPerm >= 0 ? idx + t.offPerm : nullptr;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += step) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const int row = perm ? perm[i] : i;
    st_s(dv + t.dst + (int64_t)j * t.ld + row, w[t.src + e]);
  }
}

int64_t job_scratch(const DenseJob& j) {
  const int64_t n = j.n, nr = j.nr, k = n - nr;
  if (j.kind == 0) return 2 * n * n;                     // L^-1, M
  if (nr == 0) return n * n;                             // L_g^-1 is the whole step
  return 3 * n * n + 2 * nr * n + nr * nr + nr * k + nr * n;  // Zp, K, G'; X1, V; L_s^-1; T^T
}

// S: storage type of the stored blocks; O: type of the dense forms written to `out`.
template <typename S, typename O>
void run_batch(FactorDev& f, const std::vector<DenseJob>& jobs, size_t b0, size_t b1,
               int64_t wtot, O* out, hipStream_t s, FrontStats* st) {
  DevBuf<double> w(std::max<int64_t>(1, wtot), s);
  std::vector<Prep> prep;
  std::vector<Store> store;
  std::vector<GemmTask> g1, g2, g3, g4;
  int64_t o = 0;
  int64_t maxn2 = 1;
  for (size_t q = b0; q < b1; ++q) {
    const DenseJob& j = jobs[q];
    const int n = j.n, nr = j.kind == 1 ? j.nr : 0, k = n - nr;
    maxn2 = std::max<int64_t>(maxn2, (int64_t)n * n);
    Prep p{};
    p.kind = j.kind;
    p.n = n;
    p.nr = nr;
    p.src = j.src;
    p.offPerm = j.offPerm;
    p.a = o;
    o += (int64_t)n * n;
    if (j.kind == 0) {  // M = (L^-1)^T L^-1: entry (i, j) needs inner indices >= max(i, j)
      const int64_t m = o;
      o += (int64_t)n * n;
      g1.push_back({w.p + p.a, w.p + p.a, w.p + m, n, n, n, n, n, n, 0, 3, 1, 1.0, 0, 0});
      store.push_back({m, j.dst, n, j.ld, -1, 0});
    } else if (nr == 0) {
      store.push_back({p.a, j.dst, n, j.ld, -1, 0});
    } else {
      p.x1 = o; o += (int64_t)nr * n;
      p.ls = o; o += (int64_t)nr * nr;
      p.tr = o; o += (int64_t)nr * k;
      const int64_t K = o; o += (int64_t)n * n;
      const int64_t V = o; o += (int64_t)nr * n;
      const int64_t G = o; o += (int64_t)n * n;
      double* b = w.p;
      // K_top = L_s^-1 [I, -T^T]
      g1.push_back({b + p.ls, b + p.x1, b + K, nr, n, n, nr, n, nr, 0, 2, 0, 1.0, 0, 0});
      // V = L_s^-T K_top
      g2.push_back({b + p.ls, b + K, b + V, nr, n, n, nr, n, nr, 0, 0, 1, 1.0, 0, 0});
      // K_bottom = [0, I] + T V
      g3.push_back({b + p.tr, b + V, b + K + (int64_t)nr * n, k, n, n, k, nr, nr, 0, 0, 1, 1.0,
                    0, 0});
      g3.push_back({b + p.tr, b + V + nr, b + K + (int64_t)nr * n + nr, k, n, n, k, k, nr, 0, 0,
                    1, 1.0, 1, 0});
      // G' = K P L_g^-1 (rows in the order (r, s))
      g4.push_back({b + K, b + p.a, b + G, n, n, n, n, n, n, 0, 0, 0, 1.0, 0, 0});
      store.push_back({G, j.dst, n, j.ld, j.offPerm, 0});
    }
    prep.push_back(p);
  }
  HIF_REQUIRE(o <= wtot, HIF_ERR_ARG, "dense form scratch");
  DevBuf<Prep> dp(prep.size(), s);
  DevBuf<Store> ds(store.size(), s);
  dp.upload(prep, s);
  ds.upload(store, s);
  const int gx = (int)std::min<int64_t>(64, (maxn2 + kB - 1) / kB);
  hipLaunchKernelGGL(k_dense_unpack<S>, dim3(gx, prep.size()), dim3(kB), 0, s,
                     (const Prep*)dp.p, (const int32_t*)f.idx.p,
                     reinterpret_cast<const S*>(f.vals.p), w.p);
  HIF_CHECK(hipGetLastError());
  gemm_batched(g1, s, st);
  gemm_batched(g2, s, st);
  gemm_batched(g3, s, st);
  gemm_batched(g4, s, st);
  hipLaunchKernelGGL(k_dense_store<O>, dim3(gx, store.size()), dim3(kB), 0, s,
                     (const Store*)ds.p, (const int32_t*)f.idx.p, (const double*)w.p, out);
  HIF_CHECK(hipGetLastError());
  HIF_CHECK(hipStreamSynchronize(s));  // the job lists go out of scope
}

template <typename S, typename O>
void build_dense_t(FactorDev& f, const std::vector<DenseJob>& jobs, O* out, hipStream_t s) {
  constexpr int64_t kBatch = int64_t(1) << 28;  // FP64 scratch per batch (2 GiB)
  FrontStats st;
  size_t b0 = 0;
  int64_t acc = 0;
  for (size_t q = 0; q < jobs.size(); ++q) {
    const int64_t need = job_scratch(jobs[q]);
    if (q > b0 && (acc + need > kBatch || q - b0 == 65535)) {  // grid.y counts the jobs
      run_batch<S, O>(f, jobs, b0, q, acc, out, s, &st);
      b0 = q;
      acc = 0;
    }
    acc += need;
  }
  if (b0 < jobs.size()) run_batch<S, O>(f, jobs, b0, jobs.size(), acc, out, s, &st);
  f.mfma_flops += st.flops;
  f.mfma_ms += st.ms;
}

}  // namespace

void build_dense_forms(FactorDev& f, const std::vector<DenseJob>& jobs, hipStream_t s) {
  if (jobs.empty()) return;
  switch (f.store) {
    case HIF_STORE_F64:
      build_dense_t<double>(f, jobs, reinterpret_cast<double*>(f.dvals.p), s);
      break;
    case HIF_STORE_F32:
      build_dense_t<float>(f, jobs, reinterpret_cast<float*>(f.dvals.p), s);
      break;
    case HIF_STORE_BF16:
      build_dense_t<bf16_t>(f, jobs, reinterpret_cast<bf16_t*>(f.dvals.p), s);
      break;
  }
}

void build_dense_forms_f64(FactorDev& f, const std::vector<DenseJob>& jobs, double* out,
                           hipStream_t s) {
  if (jobs.empty()) return;
  switch (f.store) {
    case HIF_STORE_F64: build_dense_t<double>(f, jobs, out, s); break;
    case HIF_STORE_F32: build_dense_t<float>(f, jobs, out, s); break;
    case HIF_STORE_BF16: build_dense_t<bf16_t>(f, jobs, out, s); break;
  }
}

}  // namespace hifcn
