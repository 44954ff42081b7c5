// Dense top of the apply.
//
// Above some level k every stage of the apply moves little data, and its time is the latency of
// its launches.  All of them — the group step of level k (block Jacobi and skeletonization, Sec.
// 2.2), the cell elimination and group step of every level above it, and the root (eq3_4), in
// the forward sweep and back — act only on the DOFs of level k's groups once level k's cells
// have been eliminated, so together they are one linear map
//     x_k = M_k (y_k - c_k)
// of the group DOFs y_k of level k less the contributions c_k of level k's cells.  M_k is
// symmetric (the forward steps' transposes in reverse order, around the root's A_r^-1) and is
// formed at factor time, top down, in FP64 on the matrix cores:
//   level t (the last):  M_t = G_t^T S G_t,  S = A_r^-1 on the root DOFs, I on the redundant ones;
//   level l < t:         M_l = G_l^T C_l G_l, with, in the order (interiors I of the level l+1
//                        cells, separators S of level l+1, redundant DOFs R of level l),
//     C_l = [[A_II^-1 + H^T M_{l+1} H, -H^T M_{l+1}, 0], [-M_{l+1} H, M_{l+1}, 0], [0, 0, I]],
//   H = A_SI A_II^-1 (the level l+1 cells' dense couplings) and G_l the level l group steps
//   (the dense group forms of dense_form.hip).
// The apply then runs the sweeps up to level k's cells, one pass of M_k (row tiles over column
// ranges, partial sums added up by a write-back launch) and the backward sweep from level k's
// cells down.  k is the lowest level whose M_k stays within an element budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "common.hpp"
#include "front.hpp"
#include "kernels.hpp"

namespace hifcn {
namespace {

constexpr int kB = 256;

template <typename S> __device__ __forceinline__ double ld_v(const S* p) { return (double)*p; }
template <> __device__ __forceinline__ double ld_v<bf16_t>(const bf16_t* p) {
  return (double)__uint_as_float(((uint32_t)p->bits) << 16);
}
template <typename S> __device__ __forceinline__ void st_v(S* p, double v) { *p = (S)v; }
template <> __device__ __forceinline__ void st_v<bf16_t>(bf16_t* p, double v) {
  p->bits = f32_to_bf16_bits((float)v);
}

// Cn[p][q] = C[cls(p)][cls(q)]: from the order (first, S, R) back to the natural one.
__global__ __launch_bounds__(kB) void k_top_to_natural(int nl, const int32_t* __restrict__ cls,
                                                       const double* __restrict__ C,
                                                       double* __restrict__ Cn) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)nl * nl;
       e += step) {
    const int p = (int)(e / nl), q = (int)(e - (int64_t)p * nl);
    Cn[e] = C[(int64_t)cls[p] * nl + cls[q]];
  }
}

// Hg[bpos[b]][ibase + j] = H_c(b, j) for every cell (H column-major nB x nI after the packed L^-1).
struct HScatter { int64_t offV; int32_t nI, nB, ibase, boff; };
template <typename S>
__global__ __launch_bounds__(kB) void k_top_scatter_h(const HScatter* __restrict__ t,
                                                      const int32_t* __restrict__ bpos,
                                                      const S* __restrict__ vals, int nI_all,
                                                      double* __restrict__ Hg) {
  const HScatter c = t[blockIdx.y];
  const S* H = vals + c.offV + tri_count(c.nI);
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)c.nI * c.nB;
       e += step) {
    const int j = (int)(e / c.nB), b = (int)(e - (int64_t)j * c.nB);
    Hg[(int64_t)bpos[c.boff + b] * nI_all + c.ibase + j] = ld_v(H + e);
  }
}

// C[r0 + i][c0 + j] (+)= src(i, j) for the cells' A_II^-1 blocks (column-major, symmetric).
struct BAdd { int64_t src; int32_t n, base; };
__global__ __launch_bounds__(kB) void k_top_add_blocks(const BAdd* __restrict__ t,
                                                       const double* __restrict__ af, int ldc,
                                                       double* __restrict__ C) {
  const BAdd a = t[blockIdx.y];
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)a.n * a.n;
       e += step) {
    const int j = (int)(e / a.n), i = (int)(e - (int64_t)j * a.n);
    C[(int64_t)(a.base + i) * ldc + a.base + j] += af[a.src + e];
  }
}

// The blocks of C around C_II: C_SI = -T1, C_IS = -T1^T, C_SS = M (all n_S x n_S / n_S x n_I
// row-major), C_RR = I.
__global__ __launch_bounds__(kB) void k_top_fill(int nI, int nS, int nR, const double* __restrict__ T1,
                                                 const double* __restrict__ M,
                                                 double* __restrict__ C) {
  const int nl = nI + nS + nR;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = e0; e < (int64_t)nS * nI; e += step) {
    const int i = (int)(e / nI), j = (int)(e - (int64_t)i * nI);
    const double v = -T1[e];
    C[(int64_t)(nI + i) * nl + j] = v;
    C[(int64_t)j * nl + nI + i] = v;
  }
  for (int64_t e = e0; e < (int64_t)nS * nS; e += step) {
    const int i = (int)(e / nS), j = (int)(e - (int64_t)i * nS);
    C[(int64_t)(nI + i) * nl + nI + j] = M[e];
  }
  for (int64_t e = e0; e < nR; e += step) {
    const int64_t q = nI + nS + e;
    C[q * nl + q] = 1.0;
  }
}

// Top level: C = [[A_r^-1, 0], [0, I]] (A_r^-1 column-major, symmetric).
__global__ __launch_bounds__(kB) void k_top_fill_root(int nr, int nR, const double* __restrict__ Ar,
                                                      double* __restrict__ C) {
  const int nl = nr + nR;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = e0; e < (int64_t)nr * nr; e += step) {
    const int j = (int)(e / nr), i = (int)(e - (int64_t)j * nr);
    C[(int64_t)i * nl + j] = Ar[e];
  }
  for (int64_t e = e0; e < nR; e += step) {
    const int64_t q = nr + e;
    C[q * nl + q] = 1.0;
  }
}

// tv[j * ld + i] = M[i * n + j] in the storage precision.
template <typename S>
__global__ __launch_bounds__(kB) void k_top_store(int n, int ld, const double* __restrict__ M,
                                                  S* __restrict__ tv) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += step) {
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    st_v(tv + (int64_t)j * ld + i, M[e]);
  }
}

int grid_for(int64_t elems) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (elems + kB - 1) / kB)); }

template <typename T>
void upload_vec(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc_on(std::max<size_t>(1, h.size()), s);
  if (!h.empty())
    HIF_CHECK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// DOF ids of a level's groups in group order, and the first position of each group.
std::vector<int32_t> group_dofs(const std::vector<GroupDesc>& gs, const std::vector<int32_t>& idx,
                                std::vector<int32_t>* base) {
  std::vector<int32_t> ids;
  base->clear();
  for (const GroupDesc& g : gs) {
    base->push_back((int32_t)ids.size());
    for (int i = 0; i < g.n; ++i) ids.push_back(idx[g.offIdx + i]);
  }
  return ids;
}

// Classification of one level's group DOFs (natural order: groups in order, each in its own
// order) into the order (first, S, R) of C_l: `first` = the root DOFs (top level) or the
// interiors of the next level's cells, S = the next level's group DOFs, R = redundant DOFs.
struct LevelSplit {
  std::vector<int32_t> ids, gbase, cls;
  int nl = 0, nfirst = 0, nS = 0;
};

LevelSplit split_level(const FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                       const std::vector<std::vector<GroupDesc>>& groups,
                       const std::vector<int32_t>& idx, int l, std::vector<int32_t>& where) {
  const int t = (int)f.lv.size() - 1;
  const std::vector<GroupDesc>& gs = groups[l];
  LevelSplit sp;
  sp.ids = group_dofs(gs, idx, &sp.gbase);
  sp.nl = (int)sp.ids.size();
  std::vector<char> red(sp.nl, 0);
  for (size_t q = 0; q < gs.size(); ++q)
    for (int i = 0; i < gs[q].nr; ++i) red[sp.gbase[q] + idx[gs[q].offPerm + i]] = 1;
  sp.cls.assign(sp.nl, -1);
  std::vector<int32_t> marked;
  auto mark = [&](int32_t id, int32_t v) {
    where[id] = v;
    marked.push_back(id);
  };
  if (l == t) {
    sp.nfirst = f.nroot;
    for (int i = 0; i < f.nroot; ++i) mark(idx[f.offRootIdx + i], i);
  } else {
    for (const CellDesc& c : cells[l + 1])
      for (int i = 0; i < c.nI; ++i) mark(idx[c.offI + i], sp.nfirst++);
    std::vector<int32_t> nb;
    const std::vector<int32_t> sids = group_dofs(groups[l + 1], idx, &nb);
    sp.nS = (int)sids.size();
    for (int q = 0; q < sp.nS; ++q) mark(sids[q], sp.nfirst + q);
  }
  int kept = 0;
  for (int p = 0; p < sp.nl; ++p) {
    if (red[p]) continue;
    const int32_t w = where[sp.ids[p]];
    HIF_REQUIRE(w >= 0, HIF_ERR_ARG, "dense top: a skeleton DOF is missing one level up");
    sp.cls[p] = w;
    ++kept;
  }
  for (int32_t id : marked) where[id] = -1;
  HIF_REQUIRE(kept == sp.nfirst + sp.nS, HIF_ERR_ARG, "dense top: level structure mismatch");
  int r = sp.nfirst + sp.nS;
  for (int p = 0; p < sp.nl; ++p)
    if (red[p]) sp.cls[p] = r++;
  return sp;
}

// C_l (row-major nl x nl, order (first, S, R)) for l < t, from M_{l+1}.
template <typename S>
void assemble_c(FactorDev& f, const std::vector<CellDesc>& pc, const std::vector<int32_t>& idx,
                const LevelSplit& sp, const double* Mnext, std::vector<int32_t>& where,
                double* C, hipStream_t s, FrontStats* st) {
  const int nl = sp.nl, nI = sp.nfirst, nS = sp.nS;
  // boundary positions (in S order) of every next-level cell
  std::vector<int32_t> bpos;
  std::vector<HScatter> hs;
  std::vector<DenseJob> aj;
  std::vector<BAdd> ba;
  {
    std::vector<int32_t> marked;
    for (int p = 0; p < nl; ++p)  // S DOFs: cls in [nI, nI + nS)
      if (sp.cls[p] >= nI && sp.cls[p] < nI + nS) {
        where[sp.ids[p]] = sp.cls[p] - nI;
        marked.push_back(sp.ids[p]);
      }
    int ib = 0;
    int64_t ao = 0;
    for (const CellDesc& c : pc) {
      HIF_REQUIRE(c.mode == 0, HIF_ERR_ARG, "dense top: link-mode cell above level 0");
      hs.push_back({(int64_t)c.offV, c.nI, c.nB, ib, (int32_t)bpos.size()});
      for (int b = 0; b < c.nB; ++b) {
        const int32_t w = where[idx[c.offB + b]];
        HIF_REQUIRE(w >= 0, HIF_ERR_ARG, "dense top: cell boundary outside the separators");
        bpos.push_back(w);
      }
      aj.push_back({0, c.nI, 0, c.nI, (int64_t)c.offV, ao, 0, 0});
      ba.push_back({ao, c.nI, ib});
      ao += (int64_t)c.nI * c.nI;
      ib += c.nI;
    }
    for (int32_t id : marked) where[id] = -1;
  }
  int64_t maxc = 1, maxa = 1, ao = 0;
  for (const CellDesc& c : pc) {
    maxc = std::max<int64_t>(maxc, (int64_t)c.nI * c.nB);
    maxa = std::max<int64_t>(maxa, (int64_t)c.nI * c.nI);
    ao += (int64_t)c.nI * c.nI;
  }
  DevBuf<double> Hg((size_t)std::max<int64_t>(1, (int64_t)nS * nI), s);
  HIF_CHECK(hipMemsetAsync(Hg.p, 0, sizeof(double) * (size_t)nS * nI, s));
  DevBuf<int32_t> dbpos;
  DevBuf<HScatter> dhs;
  DevBuf<BAdd> dba;
  upload_vec(dbpos, bpos, s);
  upload_vec(dhs, hs, s);
  upload_vec(dba, ba, s);
  hipLaunchKernelGGL(k_top_scatter_h<S>, dim3(grid_for(maxc), hs.size()), dim3(kB), 0, s,
                     (const HScatter*)dhs.p, (const int32_t*)dbpos.p,
                     reinterpret_cast<const S*>(f.vals.p), nI, Hg.p);
  DevBuf<double> af((size_t)std::max<int64_t>(1, ao), s);
  build_dense_forms_f64(f, aj, af.p, s);  // the cells' A_II^-1 (column-major, symmetric)
  DevBuf<double> T1((size_t)std::max<int64_t>(1, (int64_t)nS * nI), s);
  // T1 = M_{l+1} H;  C_II = H^T T1 (+ A_II^-1 below)
  gemm_batched({{Mnext, Hg.p, T1.p, nS, nI, nI, nS, nI, nS, 0, 0, 0, 1.0, 0, 0}}, s, st);
  gemm_batched({{Hg.p, T1.p, C, nI, nI, nl, nI, nI, nS, 0, 0, 1, 1.0, 0, 0}}, s, st);
  hipLaunchKernelGGL(k_top_add_blocks, dim3(grid_for(maxa), ba.size()), dim3(kB), 0, s,
                     (const BAdd*)dba.p, (const double*)af.p, nl, C);
  hipLaunchKernelGGL(k_top_fill, dim3(grid_for((int64_t)nS * std::max(nS, nI))), dim3(kB), 0, s,
                     nI, nS, nl - nI - nS, (const double*)T1.p, Mnext, C);
  HIF_CHECK(hipGetLastError());
  HIF_CHECK(hipStreamSynchronize(s));  // the lists and temporaries go out of scope
}

// M_k for k <= l <= t, top down; returns M_k (row-major n_k x n_k, FP64).
template <typename S>
DevBuf<double> build_top(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                         const std::vector<std::vector<GroupDesc>>& groups,
                         const std::vector<int32_t>& idx, int k, int64_t N, hipStream_t s) {
  const int t = (int)f.lv.size() - 1;
  FrontStats st;
  std::vector<int32_t> where(N, -1);
  DevBuf<double> Mnext;
  for (int l = t; l >= k; --l) {
    const LevelSplit sp = split_level(f, cells, groups, idx, l, where);
    const int nl = sp.nl;
    DevBuf<double> C((size_t)nl * nl, s);
    HIF_CHECK(hipMemsetAsync(C.p, 0, sizeof(double) * (size_t)nl * nl, s));
    if (l == t) {
      DevBuf<double> ar((size_t)std::max(1, f.nroot) * std::max(1, f.nroot), s);
      build_dense_forms_f64(f, {{0, f.nroot, 0, f.nroot, f.offRootV, 0, 0, 0}}, ar.p, s);
      hipLaunchKernelGGL(k_top_fill_root, dim3(grid_for((int64_t)f.nroot * f.nroot)), dim3(kB),
                         0, s, f.nroot, nl - f.nroot, (const double*)ar.p, C.p);
      HIF_CHECK(hipGetLastError());
      HIF_CHECK(hipStreamSynchronize(s));
    } else {
      assemble_c<S>(f, cells[l + 1], idx, sp, Mnext.p, where, C.p, s, &st);
    }
    // C back in the natural order, then M_l = G^T Cn G one group block at a time (G is
    // block diagonal: group q's block sits at rows and columns gbase[q] ..)
    DevBuf<int32_t> dcls;
    upload_vec(dcls, sp.cls, s);
    DevBuf<double> Cn((size_t)nl * nl, s);
    hipLaunchKernelGGL(k_top_to_natural, dim3(grid_for((int64_t)nl * nl)), dim3(kB), 0, s, nl,
                       (const int32_t*)dcls.p, (const double*)C.p, Cn.p);
    HIF_CHECK(hipGetLastError());
    const std::vector<GroupDesc>& gs = groups[l];
    std::vector<DenseJob> gj;
    std::vector<GemmTask> tw, tm;
    int64_t go = 0;
    for (size_t q = 0; q < gs.size(); ++q) {
      gj.push_back({1, gs[q].n, gs[q].nr, gs[q].n, (int64_t)gs[q].offV, go, gs[q].offPerm, 0});
      go += (int64_t)gs[q].n * gs[q].n;
    }
    DevBuf<double> gf((size_t)std::max<int64_t>(1, go), s);
    build_dense_forms_f64(f, gj, gf.p, s);  // column-major G_g = row-major G_g^T
    DevBuf<double> W((size_t)nl * nl, s), Ml((size_t)nl * nl, s);
    go = 0;
    for (size_t q = 0; q < gs.size(); ++q) {
      const int ng = gs[q].n, b = sp.gbase[q];
      // W[:, g] = Cn[:, g] G_g  (op(B) = (G_g^T)^T)
      tw.push_back({Cn.p + b, gf.p + go, W.p + b, nl, ng, nl, nl, ng, ng, 1, 0, 0, 1.0, 0, 0});
      // M[g, :] = G_g^T W[g, :]
      tm.push_back({gf.p + go, W.p + (int64_t)b * nl, Ml.p + (int64_t)b * nl, ng, nl, nl, ng, nl,
                    ng, 0, 0, 0, 1.0, 0, 0});
      go += (int64_t)ng * ng;
    }
    gemm_batched(tw, s, &st);
    gemm_batched(tm, s, &st);
    HIF_CHECK(hipStreamSynchronize(s));
    Mnext = std::move(Ml);
  }
  f.mfma_flops += st.flops;
  f.mfma_ms += st.ms;
  return Mnext;
}

}  // namespace

int dense_top_level(const FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                    const std::vector<std::vector<GroupDesc>>& groups) {
  const int nlev = (int)f.lv.size();
  // entries of M_k: up to 40M (160 MiB in FP32, within the 256 MiB Infinity Cache) one pass
  // over M_k costs less than the launches it replaces (1024^2 grid: level 4 instead of 5, -7%
  // apply time; 256^2 and 64^3 keep the level a 10M budget gives them).  The serving scheduler
  // builds without it (forming it costs more than a 50-step request wins back).
  int64_t budget = int64_t(40) << 20;
  if (const char* e = std::getenv("HIFCN_DENSE_TOP")) budget = std::atoll(e);
  if (f.top_budget >= 0) budget = f.top_budget;
  if (budget <= 0 || nlev == 0 || f.nroot == 0) return -1;
  // the lowest level whose M_k fits, with every level from it up to the top eligible
  int k = -1;
  for (int l = nlev - 1; l >= 0; --l) {
    int64_t n = 0;
    for (const GroupDesc& g : groups[l]) n += g.n;
    if (groups[l].empty() || cells[l].empty() || n * n > budget) break;
    if (l + 1 < nlev) {
      bool mode0 = true;
      for (const CellDesc& c : cells[l + 1]) mode0 = mode0 && c.mode == 0;
      if (!mode0) break;
    }
    k = l;
  }
  return k;
}

void setup_dense_top(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                     const std::vector<std::vector<GroupDesc>>& groups,
                     const std::vector<int32_t>& idx, int64_t N, hipStream_t s) {
  f.top = -1;
  const int k = dense_top_level(f, cells, groups);
  if (k < 0) return;
  DevBuf<double> M;
  switch (f.store) {
    case HIF_STORE_F64: M = build_top<double>(f, cells, groups, idx, k, N, s); break;
    case HIF_STORE_F32: M = build_top<float>(f, cells, groups, idx, k, N, s); break;
    case HIF_STORE_BF16: M = build_top<bf16_t>(f, cells, groups, idx, k, N, s); break;
  }
  // apply layout: M_k in the storage precision, its inputs, tiles and write-back list
  std::vector<int32_t> gbase;
  const std::vector<int32_t> ids = group_dofs(groups[k], idx, &gbase);
  const int n = (int)ids.size();
  const int ld = (n + 31) & ~31;
  const size_t eb = store_elem_bytes(f.store);
  f.tvals.alloc((size_t)n * ld * eb);
  HIF_CHECK(hipMemsetAsync(f.tvals.p, 0, (size_t)n * ld * eb, s));
  const int g = grid_for((int64_t)n * n);
  switch (f.store) {
    case HIF_STORE_F64:
      hipLaunchKernelGGL(k_top_store<double>, dim3(g), dim3(kB), 0, s, n, ld, (const double*)M.p,
                         reinterpret_cast<double*>(f.tvals.p));
      break;
    case HIF_STORE_F32:
      hipLaunchKernelGGL(k_top_store<float>, dim3(g), dim3(kB), 0, s, n, ld, (const double*)M.p,
                         reinterpret_cast<float*>(f.tvals.p));
      break;
    case HIF_STORE_BF16:
      hipLaunchKernelGGL(k_top_store<bf16_t>, dim3(g), dim3(kB), 0, s, n, ld,
                         (const double*)M.p, reinterpret_cast<bf16_t*>(f.tvals.p));
      break;
  }
  HIF_CHECK(hipGetLastError());
  // the contribution slots of each top DOF, padded to the largest count (-1)
  int kslot = 1;
  for (const GroupDesc& gd : groups[k]) {
    const int32_t* gp = idx.data() + gd.offGP;
    for (int i = 0; i < gd.n; ++i) kslot = std::max(kslot, gp[i + 1] - gp[i]);
  }
  std::vector<int32_t> slots((size_t)n * kslot, -1);
  int64_t ns = 0;
  {
    int i0 = 0;
    for (const GroupDesc& gd : groups[k]) {
      const int32_t* gp = idx.data() + gd.offGP;
      const int32_t* sl = gp + gd.n + 1;
      for (int i = 0; i < gd.n; ++i, ++i0)
        for (int e = gp[i]; e < gp[i + 1]; ++e, ++ns)
          slots[(size_t)i0 * kslot + (e - gp[i])] = sl[e];
    }
  }
  // row tiles of 64 16-byte vectors (256 rows in FP32) times column chunks, chunk-major (the
  // kernel derives its tile from the workgroup index); enough chunks for ~256 workgroups, at
  // most 16 (each DOF's result is the sum of one partial per chunk)
  const int rows = 64 * (16 / (int)eb);
  const int nrt = (n + rows - 1) / rows;
  int want = std::max(1, std::min(16, (256 + nrt - 1) / nrt));
  if (const char* e = std::getenv("HIFCN_TOP_CHUNKS")) want = std::max(1, std::atoi(e));
  // (a multiple of the 256 columns one batch of the kernel covers)
  f.tspan = std::max(256, ((n + want - 1) / want + 255) / 256 * 256);
  const int nch = (n + f.tspan - 1) / f.tspan;
  std::vector<int4> scat;
  for (int i = 0; i < n; ++i) scat.push_back({ids[i], i, nch, n});
  f.tgid.upload(ids, s);
  f.tkslot = kslot;
  f.tgslot.upload(slots, s);
  f.tscat.upload(scat, s);
  f.twsc.alloc((size_t)nch * n);
  f.top = k;
  f.ntop = n;
  f.ntdt = nch * nrt;
  f.ntsc = (int)scat.size();
  f.top_bytes = (int64_t)eb * n * n + 8 * (2 * (int64_t)n + ns + 2 * (int64_t)nch * n) +
                4 * (3 * (int64_t)n + (int64_t)n * kslot);
  f.root_fused = false;
  // When the level's cells run one workgroup each and their boundaries cover every top DOF, the
  // backward cell stage adds up the partial sums itself and writes them to y.
  f.tfold = false;
  const LevelDev& Lk = f.lv[k];
  if (!Lk.tiled && !Lk.cdense && !std::getenv("HIFCN_NO_TOP_FOLD")) {
    std::vector<int32_t> at(N, -1);
    for (int i = 0; i < n; ++i) at[ids[i]] = i;
    const size_t nc = cells[k].size();
    int maxB = 1;
    for (const CellDesc& c : cells[k]) maxB = std::max(maxB, c.nB);
    std::vector<char> hit(n, 0);
    bool ok = true;
    for (size_t c = 0; c < nc && ok; ++c)
      for (int b = 0; b < cells[k][c].nB && ok; ++b) {
        const int i = at[idx[cells[k][c].offB + b]];
        ok = i >= 0;
        if (ok) hit[i] = 1;
      }
    // top DOFs on no cell's boundary (where separators cross): dealt out over the cells
    std::vector<std::vector<int32_t>> ext(nc);
    for (int i = 0, e = 0; i < n && ok; ++i)
      if (!hit[i]) ext[e++ % nc].push_back(i);
    size_t maxE = 0;
    for (const auto& v : ext) maxE = std::max(maxE, v.size());
    // record per cell: ne, (position, id) x maxE, positions of the boundary DOFs at the end
    const int stride = 1 + 2 * (int)maxE + maxB;
    std::vector<int32_t> pos(nc * (size_t)stride, 0);
    for (size_t c = 0; c < nc && ok; ++c) {
      int32_t* r = pos.data() + c * stride;
      r[0] = (int32_t)ext[c].size();
      for (size_t e = 0; e < ext[c].size(); ++e) {
        r[1 + 2 * e] = ext[c][e];
        r[2 + 2 * e] = ids[ext[c][e]];
      }
      const CellDesc& d = cells[k][c];
      for (int b = 0; b < d.nB; ++b) r[stride - d.nB + b] = at[idx[d.offB + b]];
    }
    if (ok) {
      f.tpos.upload(pos, s);
      f.tpstride = stride;
      f.tfold = true;
      f.top_bytes += 4 * (int64_t)pos.size();
    }
  }
  HIF_CHECK(hipStreamSynchronize(s));
  if (std::getenv("HIFCN_BUILD_LOG"))
    std::fprintf(stderr, "[hifcn build] dense top from level %d: %d DOFs, %d row tiles%s\n", k,
                 n, f.ntdt, f.tfold ? ", write-back in the cell stage" : "");
}

}  // namespace hifcn
