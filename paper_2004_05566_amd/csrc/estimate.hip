// Estimate of the inverse error ||I - A F^-1||_2 (Sec. 3, Example 1: the paper judges how close
// the factor is to A^-1 by this norm, estimated by a randomized power iteration).
//
// With E = I - A F^-1 and A, F^-1 symmetric, E^T = I - F^-1 A.  From a caller's start vector
// x0, x_0 = x0 / ||x0||, and for k = 1..iters: y = E x_{k-1}, z = E^T y, lambda_k = ||z||,
// x_k = z / lambda_k; the estimate is sqrt(lambda_iters), a lower bound of ||E||_2 that rises
// towards it.  Everything stays on the device: the norms are per-block partial sums re-added
// in a fixed order by the kernel that scales, so the result is deterministic and no step waits
// for the host.
#include <mutex>
#include <string>

#include "common.hpp"
#include "kernels.hpp"

namespace hifcn {

namespace {

constexpr int kEstThreads = 256;
constexpr int kEstBlocks = 512;

__device__ double est_block_sum(double v) {
  __shared__ double red[kEstThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < kEstThreads / 64; ++w) s += red[w];
  return s;
}

// out = a - b (b may be null: out = a), and this block's share of ||out||^2 in part.
__global__ __launch_bounds__(kEstThreads) void k_est_sub(int64_t N, const double* __restrict__ a,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ out,
                                                         double* __restrict__ part) {
  double acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)kEstThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kEstThreads) {
    const double v = b ? a[i] - b[i] : a[i];
    out[i] = v;
    acc += v * v;
  }
  const double s = est_block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// lambda = sqrt(sum of the nb partials) (same order in every block); dst = src / lambda
// (dst = 0 when lambda = 0: E vanished); block 0 stores lambda.
__global__ __launch_bounds__(kEstThreads) void k_est_scale(int64_t N, const double* __restrict__ src,
                                                           const double* __restrict__ part, int nb,
                                                           double* __restrict__ dst,
                                                           double* __restrict__ lam) {
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += kEstThreads) acc += part[i];
  const double l = sqrt(est_block_sum(acc));
  const double inv = l > 0 ? 1.0 / l : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kEstThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kEstThreads)
    dst[i] = src[i] * inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) *lam = l;
}

int est_blocks(int64_t N) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((N + kEstThreads - 1) / kEstThreads,
                                                     kEstBlocks));
}

// Scratch one estimate needs: four N-vectors (x, t, s, y), the partial sums and lambda.
int64_t est_scratch_doubles(int64_t N) { return 4 * N + kEstBlocks + 8; }

// The power iteration on the scratch at `work` (est_scratch_doubles(N) doubles); leaves lambda
// in work[4N + kEstBlocks] and copies sqrt(lambda) to *est_host (synchronising the stream).
void est_run(Handle& h, const double* x0, int iters, double* work, double* est_host,
             hipStream_t s) {
  const int64_t N = h.N;
  double* x = work;
  double* t = x + N;
  double* sv = t + N;
  double* y = sv + N;
  double* part = y + N;
  double* lam = part + kEstBlocks;
  const int nb = est_blocks(N);
  const dim3 g(nb), b(kEstThreads);
  hipLaunchKernelGGL(k_est_sub, g, b, 0, s, N, x0, (const double*)nullptr, y, part);
  hipLaunchKernelGGL(k_est_scale, g, b, 0, s, N, (const double*)y, (const double*)part, nb, x,
                     lam);
  for (int k = 0; k < iters; ++k) {
    HIF_CHECK(hipMemcpyAsync(t, x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    hif_apply_inplace(h.f, t, nullptr, s);                      // t = F^-1 x
    launch_spmv(h, t, sv, s);                                    // s = A F^-1 x
    hipLaunchKernelGGL(k_est_sub, g, b, 0, s, N, (const double*)x, (const double*)sv, y,
                       part);                                    // y = E x
    launch_spmv(h, y, t, s);                                     // t = A y
    hif_apply_inplace(h.f, t, nullptr, s);                      // t = F^-1 A y
    hipLaunchKernelGGL(k_est_sub, g, b, 0, s, N, (const double*)y, (const double*)t, y,
                       part);                                    // y = E^T E x
    hipLaunchKernelGGL(k_est_scale, g, b, 0, s, N, (const double*)y, (const double*)part, nb, x,
                       lam);                                     // x = y / ||y||
  }
  HIF_CHECK(hipGetLastError());
  double l = 0;
  HIF_CHECK(hipMemcpyAsync(&l, lam, sizeof(double), hipMemcpyDeviceToHost, s));
  HIF_CHECK(hipStreamSynchronize(s));
  *est_host = iters > 0 ? std::sqrt(l) : 0.0;
}

// Scratch of the allocation-free estimate: est_scratch_doubles(N) values for N up to
// kNoAllocMaxN, at file scope so that each GPU the library runs on holds one copy until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the host it is only a
// stand-in for the symbol): it uses the device address looked up by scratch_ptr().
constexpr int64_t kNoAllocMaxN = 262144;
static __device__ __align__(256) double scratch[4 * kNoAllocMaxN + kEstBlocks + 8];

// The device address of `scratch` on the current GPU, looked up once per device with that
// device current and kept.
double* scratch_ptr() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* ptrs[kMaxDevices] = {};
  int dev = 0;
  HIF_CHECK(hipGetDevice(&dev));
  HIF_REQUIRE(dev >= 0 && dev < kMaxDevices, HIF_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    HIF_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HIF_REQUIRE(p != nullptr, HIF_ERR_HIP, "no device address for the estimate's scratch");
    ptrs[dev] = static_cast<double*>(p);
  }
  return ptrs[dev];
}

}  // namespace

hif_status_t inverse_error_impl(Handle& h, const double* x0, int iters, double* est_host,
                                hipStream_t s) {
  DevBuf<double> work(est_scratch_doubles(h.N), s);
  est_run(h, x0, iters, work.p, est_host, s);
  return HIF_OK;
}

// Every value est_run reads from the scratch is written by it first in the same call (x from
// x0, the partial sums and lambda by the kernels before the ones that read them), so nothing
// needs clearing between calls.
hif_status_t inverse_error_noalloc_impl(Handle& h, const double* x0, int iters,
                                        double* est_host, hipStream_t s) {
  HIF_REQUIRE(h.N <= kNoAllocMaxN, HIF_ERR_ARG,
              "hif_inverse_error_noalloc: N = " + std::to_string(h.N) +
                  " exceeds the fixed scratch of N <= " + std::to_string(kNoAllocMaxN));
  est_run(h, x0, iters, scratch_ptr(), est_host, s);
  return HIF_OK;
}

}  // namespace hifcn
