// Shared host/device helpers of the hifcn library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hifcn.h"

namespace hifcn {

// ---------------------------------------------------------------------------------------------
// Errors: internal code throws HifError; the C entry points translate it to a status code.
struct HifError : std::runtime_error {
  hif_status_t status;
  HifError(hif_status_t s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define HIF_CHECK(expr)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::hifcn::HifError(e_ == hipErrorOutOfMemory ? HIF_ERR_OOM : HIF_ERR_HIP,          \
                              std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

#define HIF_REQUIRE(cond, status, msg)                                                        \
  do {                                                                                        \
    if (!(cond)) throw ::hifcn::HifError((status), (msg));                                    \
  } while (0)

// ---------------------------------------------------------------------------------------------
// Owning device buffer.  alloc() uses hipMalloc (long-lived buffers); alloc_on() uses the
// stream-ordered allocator, so that the many short-lived buffers of a factor build neither take
// a device-wide lock nor wait for other streams when they are freed (hipFree synchronises the
// device; hipFreeAsync only orders the release on the buffer's stream).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t so = nullptr;  // stream-ordered: the stream it was allocated on
  bool ordered = false;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(size_t count, hipStream_t s) { alloc_on(count, s); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), so(o.so), ordered(o.ordered) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; so = o.so; ordered = o.ordered;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) HIF_CHECK(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
  }
  void alloc_on(size_t count, hipStream_t s) {
    release();
    n = count;
    so = s;
    ordered = true;
    if (count) HIF_CHECK(hipMallocAsync(reinterpret_cast<void**>(&p), count * sizeof(T), s));
  }
  void release() {
    if (p) {
      if (ordered) (void)hipFreeAsync(p, so);
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    ordered = false;
    so = nullptr;
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    if (h.size() != n) alloc(h.size());
    if (n) HIF_CHECK(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
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
