// Shared host/device helpers of the hifcn library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hifcn.h"
#include "errors.hpp"

namespace hifcn {

// ---------------------------------------------------------------------------------------------
// Errors of HIP calls become HifError (errors.hpp) with HIF_ERR_OOM or HIF_ERR_HIP.
#define HIF_CHECK(expr)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::hifcn::HifError(e_ == hipErrorOutOfMemory ? HIF_ERR_OOM : HIF_ERR_HIP,          \
                              std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

// ---------------------------------------------------------------------------------------------
// The stream on which long-lived buffers are taken from the device's stream-ordered pool (one
// per device, default priority, created on first use).  Each allocation waits for it, so the
// memory is ready for every stream as soon as alloc() returns.
inline hipStream_t pool_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  HIF_CHECK(hipGetDevice(&dev));
  HIF_REQUIRE(dev >= 0 && dev < 64, HIF_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev]) HIF_CHECK(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}

// The library's stream-ordered memory pool of the current device (created on first use).  It
// keeps up to 4 GiB of released memory for later allocations instead of handing it back to the
// driver at every synchronisation, so the temporaries of one factor build reuse those of the
// last one.
inline hipMemPool_t lib_pool() {
  static std::mutex mu;
  static hipMemPool_t pools[64] = {};
  int dev = 0;
  HIF_CHECK(hipGetDevice(&dev));
  HIF_REQUIRE(dev >= 0 && dev < 64, HIF_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!pools[dev]) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    HIF_CHECK(hipMemPoolCreate(&pool, &props));
    uint64_t keep = uint64_t(4) << 30;
    HIF_CHECK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    pools[dev] = pool;
  }
  return pools[dev];
}

// Set on a thread while every stream of the device is known to be idle (DeviceIdle): long-lived
// buffers released meanwhile skip the device synchronisation each release otherwise makes.
inline bool& device_idle_flag() {
  thread_local bool idle = false;
  return idle;
}
struct DeviceIdle {  // synchronise the device once, then release any number of buffers
  DeviceIdle() {
    (void)hipDeviceSynchronize();
    device_idle_flag() = true;
  }
  ~DeviceIdle() { device_idle_flag() = false; }
  DeviceIdle(const DeviceIdle&) = delete;
  DeviceIdle& operator=(const DeviceIdle&) = delete;
};

// Owning device buffer.  Both kinds of allocation come from the library's pool, so that
// releasing them never waits for other streams the way hipFree does (it synchronises the
// device):
//   alloc()     long-lived buffers (a factor, a solve's vectors): taken on pool_stream(); a
//               release first waits for the device's queued work, as hipFree would, unless the
//               device is known idle (DeviceIdle: a handle's whole set after one synchronisation);
//   alloc_on()  the many short-lived buffers of a factor build: taken and released in the order
//               of their own stream.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t so = nullptr;  // the stream it was allocated on
  bool ordered = false;      // alloc_on: released in the order of so
  bool pooled = false;       // alloc: released after the device's queued work
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(size_t count, hipStream_t s) { alloc_on(count, s); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept
      : p(o.p), n(o.n), so(o.so), ordered(o.ordered), pooled(o.pooled) {
    o.p = nullptr;
    o.n = 0;
    o.ordered = o.pooled = false;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; so = o.so; ordered = o.ordered; pooled = o.pooled;
      o.p = nullptr; o.n = 0; o.ordered = o.pooled = false;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) {
      so = pool_stream();
      HIF_CHECK(hipMallocFromPoolAsync(reinterpret_cast<void**>(&p), count * sizeof(T),
                                       lib_pool(), so));
      pooled = true;
      HIF_CHECK(hipStreamSynchronize(so));
    }
  }
  void alloc_on(size_t count, hipStream_t s) {
    release();
    n = count;
    so = s;
    ordered = true;
    if (count)
      HIF_CHECK(hipMallocFromPoolAsync(reinterpret_cast<void**>(&p), count * sizeof(T),
                                       lib_pool(), s));
  }
  void release() {
    if (p) {
      if (pooled && !device_idle_flag()) (void)hipDeviceSynchronize();
      (void)hipFreeAsync(p, so);
    }
    p = nullptr;
    n = 0;
    ordered = pooled = false;
    so = nullptr;
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    if (h.size() != n) alloc(h.size());
    if (n) HIF_CHECK(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// A small table uploaded again and again between launches (the batched step's per-solve
// arguments): device storage that only grows (by doubling, so a growing hipFree, which waits for
// the device, is rare) filled from pinned host memory that is written again only once the copy
// out of it has ended (an event).  A refill thus leaves the device running.
template <typename T>
struct StagedBuf {
  T* p = nullptr;  // device
  size_t n = 0;    // elements of the last upload
  size_t cap = 0;
  T* h = nullptr;  // pinned host staging, cap elements
  hipEvent_t copied = nullptr;
  StagedBuf() = default;
  StagedBuf(const StagedBuf&) = delete;
  StagedBuf& operator=(const StagedBuf&) = delete;
  ~StagedBuf() {
    if (copied) {
      (void)hipEventSynchronize(copied);
      (void)hipEventDestroy(copied);
    }
    if (p) (void)hipFree(p);
    if (h) (void)hipHostFree(h);
  }
  void upload(const std::vector<T>& v, hipStream_t s) {
    if (!copied) HIF_CHECK(hipEventCreateWithFlags(&copied, hipEventDisableTiming));
    HIF_CHECK(hipEventSynchronize(copied));  // the previous copy out of h has ended
    if (v.size() > cap) {
      const size_t c = std::max(v.size(), 2 * cap);
      if (p) HIF_CHECK(hipFree(p));
      p = nullptr;
      if (h) HIF_CHECK(hipHostFree(h));
      h = nullptr;
      cap = 0;
      HIF_CHECK(hipMalloc(reinterpret_cast<void**>(&p), c * sizeof(T)));
      HIF_CHECK(hipHostMalloc(reinterpret_cast<void**>(&h), c * sizeof(T), hipHostMallocDefault));
      cap = c;
    }
    n = v.size();
    if (!n) return;
    std::memcpy(h, v.data(), n * sizeof(T));
    HIF_CHECK(hipMemcpyAsync(p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    HIF_CHECK(hipEventRecord(copied, s));
  }
};

// ---------------------------------------------------------------------------------------------
// Storage element types of the factor blocks.
struct bf16_t { uint16_t bits; };

template <typename C> __device__ __forceinline__ C load_as(const double* p) { return (C)(*p); }
template <typename C> __device__ __forceinline__ C load_as(const float* p) { return (C)(*p); }
template <typename C> __device__ __forceinline__ C load_as(const bf16_t* p) {
  return (C)__uint_as_float(((uint32_t)p->bits) << 16);
}

// Round-to-nearest-even FP32 -> BF16 (host and device).
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16 | ((u & 0xffff) ? 0x40 : 0));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

inline size_t store_elem_bytes(hif_store_t s) {
  return s == HIF_STORE_F64 ? 8 : (s == HIF_STORE_F32 ? 4 : 2);
}

// ---------------------------------------------------------------------------------------------
// Descriptors of one level of the factor, as read by the apply kernels.  Offsets are element
// offsets into the handle's index array (int32) and value array (storage type).
struct CellDesc {
  int32_t nI, nB;      // interior and boundary sizes
  int32_t offI, offB;  // index lists (global DOF ids)
  int32_t offV;        // values: packed column-major lower L^-1 (nI(nI+1)/2), then
                       //   mode 0: H = A_BI A_II^-1 column-major (nB x nI, H[j*nB + b])
                       //   mode 1: the coupling A_IB(ib_b, b) of each boundary DOF b (nB)
  int32_t offCB;       // first slot of this cell's boundary contributions
  int32_t mode;        // 0: dense H; 1: A_IB has one entry per column (stencil links, level 0)
  int32_t offC;        // mode 1: interior position ib_b of each boundary DOF's link (nB)
};

struct GroupDesc {
  int32_t n, nr;       // group size, number of redundant DOFs (0: not skeletonized)
  int32_t offIdx;      // DOF ids, group order (the order of L_g)
  int32_t offPerm;     // positions in group order: redundant first (nr), then skeleton
  int32_t offV;        // values: packed L_g^-1 (n(n+1)/2), T column-major (k x nr, T[j*k + s]),
                       //         packed L_s^-1 (nr(nr+1)/2), with k = n - nr
  int32_t offGP;       // gather map: ptr[n+1] (relative), then slots[] into the contributions
  int32_t pad0;
  int32_t cap;         // elements the storage at offV holds (room for a dense n x n form)
};

__host__ __device__ inline int64_t tri_count(int64_t n) { return n * (n + 1) / 2; }

// Storage order of a symmetric level-0 cell block (A_II^-1 of a cell held as one matrix): its
// tl packed elements (column-major lower triangle) go in chunks of 64 E, E being the elements of
// the storage type in 16 bytes.  In a chunk of m elements, with q = ceil(m / E), the E stored
// elements E L .. E L + E - 1 hold the packed elements L, L + q, ..., L + (E - 1) q, so a
// wavefront that loads one 16-byte vector per lane stores consecutive packed elements across
// its lanes with each of its E stores.  The block's couplings follow at sym_coff(tl).
__host__ __device__ inline int sym_chunk_q(int c, int tl, int E) {
  const int m = tl - 64 * E * c;
  return ((m < 64 * E ? m : 64 * E) + E - 1) / E;
}
__host__ __device__ inline int sym_store_index(int p, int tl, int E) {
  const int c = p / (64 * E), w = p - 64 * E * c, q = sym_chunk_q(c, tl, E);
  const int k = w / q, L = w - k * q;
  return 64 * E * c + E * L + k;
}
// The packed element at stored position s (tl or more: a padding slot of the last chunk).
__host__ __device__ inline int sym_packed_index(int s, int tl, int E) {
  const int c = s / (64 * E), w = s - 64 * E * c, q = sym_chunk_q(c, tl, E);
  return 64 * E * c + w / E + q * (w % E);
}
__host__ __device__ inline int64_t sym_coff(int64_t tl) { return (tl + 7) / 8 * 8; }
// start of column j of a packed column-major lower triangle of order n
__host__ __device__ inline int colstart(int j, int n) { return j * n - (j * (j - 1)) / 2; }

}  // namespace hifcn
