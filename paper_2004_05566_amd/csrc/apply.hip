// HIF apply z = F^-1 r (eqAinv): level-by-level batched small dense work.
//
// Forward sweep, level l (R_l^T = K_l^T C_l^T E_l^T):
//   cell stage  (E_l^T, eq2_3):  w = L^-1 y_I;  contribution c_B = H y_I with H = A_BI A_II^-1
//                                (= G^T L^-1); y_I <- w.  Cells are disjoint, but several cells
//                                share a boundary DOF, so each writes its c_B to its own slots.
//   group stage (C_l^T, K_l^T):  y_g -= sum of the contributions aimed at g (fixed order:
//                                deterministic, no atomics); y_g <- L_g^-1 y_g (jacobi-precond);
//                                edges/faces: t = L_s^-1 (y_I~ - T^T y_I^), y_I^ += T L_s^-T t,
//                                y_I~ <- t (eq_T, eq2_9).
// Root: y_r <- L_r^-T L_r^-1 y_r.
// Backward sweep, level l (R_l = E_l C_l K_l):
//   group stage (K_l, C_l):      u = L_s^-T (x_I~ + L_s^-1 T^T x_I^), x_I^ -= T u, x_I~ <- u;
//                                x_g <- L_g^-T x_g.
//   cell stage  (E_l):           x_I <- L^-T x_I - H^T x_B (gather only).
//
// Every block of a stage is independent (the factors are block diagonal up to a permutation,
// Sec. 2.2), so each stage is one launch with one workgroup per cell or group.  Blocks are
// staged into LDS with coalesced loads (padded square layouts keep both the row and the column
// walks free of bank conflicts), converted to the compute type C on the way.  Every kernel
// returns at once when the device flag `done` is set, so PCG iterations can be queued ahead.
#include "common.hpp"
#include "kernels.hpp"

namespace hifcn {

namespace {

constexpr int kRootThreads = 256;

__host__ __device__ inline int odd_stride(int n) { return (n & 1) ? n : n + 1; }

// Stage packed column-major lower triangle (order n) into LDS as a row-major square with odd
// row stride `ld` (entries above the diagonal are left unset and never read).
template <typename S, typename C>
__device__ __forceinline__ void stage_tri(C* dst, const S* src, int n, int ld) {
  int base = 0;
  for (int j = 0; j < n; ++j) {
    for (int i = j + (int)threadIdx.x; i < n; i += blockDim.x)
      dst[i * ld + j] = load_as<C>(src + base + (i - j));
    base += n - j;
  }
}

// Stage a column-major rows x cols block into LDS, column stride `ld` (ld >= rows).
template <typename S, typename C>
__device__ __forceinline__ void stage_cols(C* dst, const S* src, int rows, int cols, int ld) {
  const int tot = rows * cols;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int j = t / rows, r = t - j * rows;
    dst[j * ld + r] = load_as<C>(src + t);
  }
}

// Read-only views of the factor blocks: staged in LDS (ST) or read straight from global memory.
// Tri: lower triangle of order n, element (i, j), i >= j; packed column-major in global memory,
//      row-major with odd stride `ld` in LDS.
// Col: column-major rows x cols block, element (r, c); column stride `ld` in LDS.
template <typename S, typename C, bool ST>
struct Tri {
  const C* l;
  const S* g;
  int n, ld;
  __device__ __forceinline__ C operator()(int i, int j) const {
    if constexpr (ST) return l[i * ld + j];
    else return load_as<C>(g + colstart(j, n) + (i - j));
  }
};
template <typename S, typename C, bool ST>
struct Col {
  const C* l;
  const S* g;
  int rows, ld;
  __device__ __forceinline__ C operator()(int r, int c) const {
    if constexpr (ST) return l[c * ld + r];
    else return load_as<C>(g + (int64_t)c * rows + r);
  }
};

// ------------------------------------------------------------------------------ cell stages --
template <typename S, typename C, bool ST>
__global__ __launch_bounds__(256) void k_cell_fwd(const CellDesc* __restrict__ cd,
                                                  const int32_t* __restrict__ idx,
                                                  const S* __restrict__ vals,
                                                  double* __restrict__ y, double* __restrict__ cb,
                                                  const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const CellDesc d = cd[blockIdx.x];
  const int nI = d.nI, nB = d.nB;
  const int ldL = odd_stride(nI), ldH = odd_stride(nB);
  const S* v = vals + d.offV;
  C* Ls = sm;
  C* Hs = ST ? Ls + nI * ldL : Ls;
  C* ys = ST ? Hs + nI * ldH : sm;
  if constexpr (ST) {
    stage_tri(Ls, v, nI, ldL);
    stage_cols(Hs, v + tri_count(nI), nB, nI, ldH);
  }
  const Tri<S, C, ST> Li{Ls, v, nI, ldL};
  const Col<S, C, ST> H{Hs, v + tri_count(nI), nB, ldH};
  for (int i = threadIdx.x; i < nI; i += blockDim.x) ys[i] = (C)y[idx[d.offI + i]];
  __syncthreads();
  for (int i = threadIdx.x; i < nI; i += blockDim.x) {
    C acc = 0;
    for (int j = 0; j <= i; ++j) acc += Li(i, j) * ys[j];
    y[idx[d.offI + i]] = (double)acc;
  }
  for (int b = threadIdx.x; b < nB; b += blockDim.x) {
    C acc = 0;
    for (int j = 0; j < nI; ++j) acc += H(b, j) * ys[j];
    cb[d.offCB + b] = (double)acc;
  }
}

template <typename S, typename C, bool ST>
__global__ __launch_bounds__(256) void k_cell_bwd(const CellDesc* __restrict__ cd,
                                                  const int32_t* __restrict__ idx,
                                                  const S* __restrict__ vals,
                                                  double* __restrict__ x,
                                                  const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const CellDesc d = cd[blockIdx.x];
  const int nI = d.nI, nB = d.nB;
  const int ldL = odd_stride(nI), ldH = odd_stride(nB);
  const S* v = vals + d.offV;
  C* Ls = sm;
  C* Hs = ST ? Ls + nI * ldL : Ls;
  C* xs = ST ? Hs + nI * ldH : sm;
  C* xb = xs + nI;
  if constexpr (ST) {
    stage_tri(Ls, v, nI, ldL);
    stage_cols(Hs, v + tri_count(nI), nB, nI, ldH);
  }
  const Tri<S, C, ST> Li{Ls, v, nI, ldL};
  const Col<S, C, ST> H{Hs, v + tri_count(nI), nB, ldH};
  for (int i = threadIdx.x; i < nI; i += blockDim.x) xs[i] = (C)x[idx[d.offI + i]];
  for (int b = threadIdx.x; b < nB; b += blockDim.x) xb[b] = (C)x[idx[d.offB + b]];
  __syncthreads();
  for (int i = threadIdx.x; i < nI; i += blockDim.x) {
    C acc = 0;
    for (int j = i; j < nI; ++j) acc += Li(j, i) * xs[j];
    C hb = 0;
    for (int b = 0; b < nB; ++b) hb += H(b, i) * xb[b];
    x[idx[d.offI + i]] = (double)(acc - hb);
  }
}

// ----------------------------------------------------------------------------- group stages --
// LDS: Lg (n x ldG), T (nr cols of stride ldT >= k), Ls (nr x ldR) when staged; then vectors.
template <typename S, typename C, bool ST>
__global__ __launch_bounds__(256) void k_group_fwd(const GroupDesc* __restrict__ gd,
                                                   const int32_t* __restrict__ idx,
                                                   const S* __restrict__ vals,
                                                   double* __restrict__ y,
                                                   const double* __restrict__ cb,
                                                   const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const GroupDesc d = gd[blockIdx.x];
  const int n = d.n, nr = d.nr, k = n - nr;
  const int ldG = odd_stride(n), ldT = odd_stride(k), ldR = odd_stride(nr);
  const S* v = vals + d.offV;
  const S* vT = v + tri_count(n);
  const S* vR = vT + (int64_t)k * nr;
  C* Lgs = sm;
  C* Tss = ST ? Lgs + n * ldG : sm;
  C* Lrs = ST ? Tss + nr * ldT : sm;
  C* yg = ST ? Lrs + nr * ldR : sm;
  C* zg = yg + n;
  C* tv = zg + n;   // nr
  C* uv = tv + nr;  // nr
  if constexpr (ST) {
    stage_tri(Lgs, v, n, ldG);
    if (nr > 0) {
      stage_cols(Tss, vT, k, nr, ldT);
      stage_tri(Lrs, vR, nr, ldR);
    }
  }
  const Tri<S, C, ST> Lg{Lgs, v, n, ldG};
  const Col<S, C, ST> T{Tss, vT, k, ldT};
  const Tri<S, C, ST> Lr{Lrs, vR, nr, ldR};
  const int32_t* gp = idx + d.offGP;
  const int32_t* slots = gp + n + 1;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc = y[idx[d.offIdx + i]];
    for (int s = gp[i]; s < gp[i + 1]; ++s) acc -= cb[slots[s]];
    yg[i] = (C)acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {   // C^T: z = L_g^-1 y_g
    C acc = 0;
    for (int j = 0; j <= i; ++j) acc += Lg(i, j) * yg[j];
    zg[i] = acc;
  }
  __syncthreads();
  const int32_t* perm = idx + d.offPerm;
  if (nr > 0) {   // K^T
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {     // y_I~ - T^T y_I^
      C acc = zg[perm[i]];
      for (int s = 0; s < k; ++s) acc -= T(s, i) * zg[perm[nr + s]];
      tv[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {     // t = L_s^-1 (...)
      C acc = 0;
      for (int j = 0; j <= i; ++j) acc += Lr(i, j) * tv[j];
      uv[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {     // L_s^-T t
      C acc = 0;
      for (int j = i; j < nr; ++j) acc += Lr(j, i) * uv[j];
      tv[i] = acc;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < k; s += blockDim.x) {      // y_I^ += T L_s^-T t
      C acc = zg[perm[nr + s]];
      for (int i = 0; i < nr; ++i) acc += T(s, i) * tv[i];
      y[idx[d.offIdx + perm[nr + s]]] = (double)acc;
    }
    for (int i = threadIdx.x; i < nr; i += blockDim.x) y[idx[d.offIdx + perm[i]]] = (double)uv[i];
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) y[idx[d.offIdx + i]] = (double)zg[i];
  }
}

template <typename S, typename C, bool ST>
__global__ __launch_bounds__(256) void k_group_bwd(const GroupDesc* __restrict__ gd,
                                                   const int32_t* __restrict__ idx,
                                                   const S* __restrict__ vals,
                                                   double* __restrict__ x,
                                                   const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  const GroupDesc d = gd[blockIdx.x];
  const int n = d.n, nr = d.nr, k = n - nr;
  const int ldG = odd_stride(n), ldT = odd_stride(k), ldR = odd_stride(nr);
  const S* v = vals + d.offV;
  const S* vT = v + tri_count(n);
  const S* vR = vT + (int64_t)k * nr;
  C* Lgs = sm;
  C* Tss = ST ? Lgs + n * ldG : sm;
  C* Lrs = ST ? Tss + nr * ldT : sm;
  C* xg = ST ? Lrs + nr * ldR : sm;
  C* zg = xg + n;
  C* tv = zg + n;
  C* uv = tv + nr;
  if constexpr (ST) {
    stage_tri(Lgs, v, n, ldG);
    if (nr > 0) {
      stage_cols(Tss, vT, k, nr, ldT);
      stage_tri(Lrs, vR, nr, ldR);
    }
  }
  const Tri<S, C, ST> Lg{Lgs, v, n, ldG};
  const Col<S, C, ST> T{Tss, vT, k, ldT};
  const Tri<S, C, ST> Lr{Lrs, vR, nr, ldR};
  for (int i = threadIdx.x; i < n; i += blockDim.x) xg[i] = (C)x[idx[d.offIdx + i]];
  __syncthreads();
  const int32_t* perm = idx + d.offPerm;
  if (nr > 0) {   // K
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {     // a = T^T x_I^
      C acc = 0;
      for (int s = 0; s < k; ++s) acc += T(s, i) * xg[perm[nr + s]];
      tv[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {     // x_I~ + L_s^-1 a
      C acc = xg[perm[i]];
      for (int j = 0; j <= i; ++j) acc += Lr(i, j) * tv[j];
      uv[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nr; i += blockDim.x) {     // u = L_s^-T (...)
      C acc = 0;
      for (int j = i; j < nr; ++j) acc += Lr(j, i) * uv[j];
      tv[i] = acc;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < k; s += blockDim.x) {      // x_I^ -= T u
      C acc = xg[perm[nr + s]];
      for (int i = 0; i < nr; ++i) acc -= T(s, i) * tv[i];
      zg[perm[nr + s]] = acc;
    }
    for (int i = threadIdx.x; i < nr; i += blockDim.x) zg[perm[i]] = tv[i];
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) zg[i] = xg[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {        // C: x_g = L_g^-T x_g
    C acc = 0;
    for (int j = i; j < n; ++j) acc += Lg(j, i) * zg[j];
    x[idx[d.offIdx + i]] = (double)acc;
  }
}

// ------------------------------------------------------------------------------------ root --
// y_r <- L_r^-T (L_r^-1 y_r), L_r^-1 packed column-major, read straight from global memory.
template <typename S, typename C>
__global__ __launch_bounds__(kRootThreads) void k_root(int nr, const int32_t* __restrict__ ridx,
                                                       const S* __restrict__ Lv,
                                                       double* __restrict__ y,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* ys = reinterpret_cast<C*>(smem_raw);
  C* ws = ys + nr;
  for (int i = threadIdx.x; i < nr; i += blockDim.x) ys[i] = (C)y[ridx[i]];
  __syncthreads();
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    C acc = 0;
    int base = 0;
    for (int j = 0; j <= i; ++j) { acc += load_as<C>(Lv + base + (i - j)) * ys[j]; base += nr - j; }
    ws[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    C acc = 0;
    const int base = colstart(i, nr);
    for (int j = i; j < nr; ++j) acc += load_as<C>(Lv + base + (j - i)) * ws[j];
    y[ridx[i]] = (double)acc;
  }
}

template <typename C>
size_t cell_smem(int maxI, int maxB, bool staged) {
  const size_t vec = (size_t)maxI + maxB;
  if (!staged) return sizeof(C) * vec;
  return sizeof(C) * ((size_t)maxI * odd_stride(maxI) + (size_t)maxI * odd_stride(maxB) + vec);
}
template <typename C>
size_t group_smem(int maxN, int maxK, int maxR, bool staged) {
  const size_t vec = 2 * (size_t)maxN + 2 * (size_t)maxR;
  if (!staged) return sizeof(C) * vec;
  return sizeof(C) * ((size_t)maxN * odd_stride(maxN) + (size_t)maxR * odd_stride(maxK) +
                      (size_t)maxR * odd_stride(maxR) + vec);
}

// Blocks are staged in LDS when a level's largest block fits this budget (keeps several
// workgroups resident per CU); larger blocks are read straight from global memory.
constexpr size_t kStageBudget = 48 * 1024;

template <typename C>
bool cell_staged(const LevelDev& L) { return cell_smem<C>(L.maxI, L.maxB, true) <= kStageBudget; }
template <typename C>
bool group_staged(const LevelDev& L) {
  return group_smem<C>(L.maxG, L.maxK, L.maxR, true) <= kStageBudget;
}

int cell_threads(const LevelDev& L, bool st) { return (st && L.maxI <= 64) ? 64 : (L.maxI <= 128 ? 128 : 256); }
int group_threads(const LevelDev& L) { return L.maxG <= 64 ? 64 : (L.maxG <= 128 ? 128 : 256); }

template <typename S, typename C>
void apply_impl(const FactorDev& f, double* y, const int* done, hipStream_t s) {
  const S* vals = reinterpret_cast<const S*>(f.vals.p);
  const int32_t* idx = f.idx.p;
  for (size_t l = 0; l < f.lv.size(); ++l) {
    const LevelDev& L = f.lv[l];
    if (L.ncell) {
      const bool st = cell_staged<C>(L);
      auto k = st ? k_cell_fwd<S, C, true> : k_cell_fwd<S, C, false>;
      hipLaunchKernelGGL(k, dim3(L.ncell), dim3(cell_threads(L, st)),
                         cell_smem<C>(L.maxI, L.maxB, st), s, L.cells.p, idx, vals, y, f.cb.p,
                         done);
    }
    if (L.ngroup) {
      const bool st = group_staged<C>(L);
      auto k = st ? k_group_fwd<S, C, true> : k_group_fwd<S, C, false>;
      hipLaunchKernelGGL(k, dim3(L.ngroup), dim3(group_threads(L)),
                         group_smem<C>(L.maxG, L.maxK, L.maxR, st), s, L.groups.p, idx, vals, y,
                         f.cb.p, done);
    }
  }
  if (f.nroot)
    hipLaunchKernelGGL((k_root<S, C>), dim3(1), dim3(kRootThreads), 2 * sizeof(C) * f.nroot, s,
                       f.nroot, idx + f.offRootIdx, vals + f.offRootV, y, done);
  for (size_t l = f.lv.size(); l-- > 0;) {
    const LevelDev& L = f.lv[l];
    if (L.ngroup) {
      const bool st = group_staged<C>(L);
      auto k = st ? k_group_bwd<S, C, true> : k_group_bwd<S, C, false>;
      hipLaunchKernelGGL(k, dim3(L.ngroup), dim3(group_threads(L)),
                         group_smem<C>(L.maxG, L.maxK, L.maxR, st), s, L.groups.p, idx, vals, y,
                         done);
    }
    if (L.ncell) {
      const bool st = cell_staged<C>(L);
      auto k = st ? k_cell_bwd<S, C, true> : k_cell_bwd<S, C, false>;
      hipLaunchKernelGGL(k, dim3(L.ncell), dim3(cell_threads(L, st)),
                         cell_smem<C>(L.maxI, L.maxB, st), s, L.cells.p, idx, vals, y, done);
    }
  }
  HIF_CHECK(hipGetLastError());
}

}  // namespace

size_t apply_smem_need(const FactorDev& f, size_t* worst) {
  size_t w = 0;
  const bool f64 = f.store == HIF_STORE_F64;
  for (const LevelDev& L : f.lv) {
    size_t c, g;
    if (f64) {
      c = cell_smem<double>(L.maxI, L.maxB, cell_staged<double>(L));
      g = group_smem<double>(L.maxG, L.maxK, L.maxR, group_staged<double>(L));
    } else {
      c = cell_smem<float>(L.maxI, L.maxB, cell_staged<float>(L));
      g = group_smem<float>(L.maxG, L.maxK, L.maxR, group_staged<float>(L));
    }
    w = std::max(w, std::max(c, g));
  }
  w = std::max(w, (size_t)(f64 ? 16 : 8) * f.nroot);
  if (worst) *worst = w;
  return w;
}

void hif_apply_inplace(const FactorDev& f, double* y, const int* done, hipStream_t s) {
  switch (f.store) {
    case HIF_STORE_F64: apply_impl<double, double>(f, y, done, s); break;
    case HIF_STORE_F32: apply_impl<float, float>(f, y, done, s); break;
    case HIF_STORE_BF16: apply_impl<bf16_t, float>(f, y, done, s); break;
  }
}

}  // namespace hifcn

namespace hifcn {

// Allow the apply kernels to use up to `bytes` of dynamic LDS (gfx950: 160 KiB per CU).
void set_apply_smem_limits(size_t bytes) {
  const int b = (int)bytes;
#define HIF_SMEM(K) HIF_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(K),           \
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, b))
#define HIF_SMEM_ALL(S, C)                                                                    \
  HIF_SMEM((k_cell_fwd<S, C, false>));                                                        \
  HIF_SMEM((k_cell_bwd<S, C, false>));                                                        \
  HIF_SMEM((k_group_fwd<S, C, false>));                                                       \
  HIF_SMEM((k_group_bwd<S, C, false>));                                                       \
  HIF_SMEM((k_root<S, C>))
  HIF_SMEM_ALL(double, double);
  HIF_SMEM_ALL(float, float);
  HIF_SMEM_ALL(bf16_t, float);
#undef HIF_SMEM_ALL
#undef HIF_SMEM
}

}  // namespace hifcn
