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
// Sec. 2.2), so each stage is one launch.  Each block's values are contiguous and 16-byte
// aligned; a workgroup (or, for small groups, a lane segment of a wavefront) copies its block
// into LDS with vector loads that are all in flight together, converting to the compute type C,
// then works from LDS.  Loops that walk a block across rows and across columns start each lane
// at a skewed position so that lanes hit different LDS banks.  Blocks too large for LDS are read
// straight from global memory instead.  Every kernel returns at once when the device flag
// `done` is set, so PCG iterations can be queued ahead.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <queue>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "cg_gate.hpp"
#include "stencil.hpp"

namespace hifcn {

namespace {

constexpr int kRootThreads = 256;
constexpr size_t kStageBudget = 48 * 1024;   // LDS per workgroup when many are in flight
constexpr size_t kStageMax = 150 * 1024;     // LDS per workgroup for few, large blocks

// ---------------------------------------------------------------------- vector staging --
template <typename S> struct VecOf;
template <> struct VecOf<float> { using T = float4; static constexpr int W = 4; };
template <> struct VecOf<double> { using T = double2; static constexpr int W = 2; };
template <> struct VecOf<bf16_t> { using T = uint4; static constexpr int W = 8; };

template <typename C>
__device__ __forceinline__ void unpack(const float4& v, C* d) {
  d[0] = (C)v.x; d[1] = (C)v.y; d[2] = (C)v.z; d[3] = (C)v.w;
}
template <typename C>
__device__ __forceinline__ void unpack(const double2& v, C* d) {
  d[0] = (C)v.x; d[1] = (C)v.y;
}
template <typename C>
__device__ __forceinline__ void unpack(const uint4& v, C* d) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    d[2 * q] = (C)__uint_as_float(w[q] << 16);
    d[2 * q + 1] = (C)__uint_as_float(w[q] & 0xffff0000u);
  }
}

// Copy `tot` elements starting at the (16-byte aligned) `src` into LDS `dst`, using `nthr`
// threads numbered `lt`; kStageUnroll vector loads per thread are issued before any is consumed
// (few lanes staging a large block need many loads in flight to cover the memory latency).
// `dst` must hold `tot` rounded up to the vector width.  (Measured side by side: 6 loads is 1%
// faster than 8 on 256^2 and no slower on 1024^2; 16 is 4% slower.)
constexpr int kStageUnroll = 6;
template <typename S, typename C>
__device__ __forceinline__ void stage_flat(C* dst, const S* src, int tot, int lt, int nthr) {
  using V = typename VecOf<S>::T;
  constexpr int W = VecOf<S>::W;
  constexpr int U = kStageUnroll;
  const V* sv = reinterpret_cast<const V*>(src);
  const int nv = (tot + W - 1) / W;
  for (int b = lt; b < nv; b += U * nthr) {
    V r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = b + u * nthr;
      if (q < nv) r[u] = sv[q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = b + u * nthr;
      if (q < nv) unpack<C>(r[u], dst + q * W);
    }
  }
}

// stage_flat of a block together with the gather of up to two index lists from an FP64 vector
// (list a: na values into da, list b: nb values into db).  The index loads are issued first,
// then the block's first round of vector loads, then the value loads, which wait only for the
// indices; the block reaches LDS after that.  So the dependent index -> value loads overlap the
// block copy instead of following it.
template <typename S, typename C>
__device__ __forceinline__ void stage_gather(C* dst, const S* src, int tot,
                                             const double* __restrict__ vec,
                                             const int32_t* __restrict__ ia, int na, C* da,
                                             const int32_t* __restrict__ ibx, int nb, C* db,
                                             int lt, int nthr) {
  using V = typename VecOf<S>::T;
  constexpr int W = VecOf<S>::W;
  constexpr int U = kStageUnroll;
  const int ga = lt < na ? ia[lt] : -1;
  const int gb = lt < nb ? ibx[lt] : -1;
  const V* sv = reinterpret_cast<const V*>(src);
  const int nv = (tot + W - 1) / W;
  V r[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = lt + u * nthr;
    if (q < nv) r[u] = sv[q];
  }
  const double va = ga >= 0 ? vec[ga] : 0.0;
  const double vb = gb >= 0 ? vec[gb] : 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = lt + u * nthr;
    if (q < nv) unpack<C>(r[u], dst + q * W);
  }
  for (int b = lt + U * nthr; b < nv; b += U * nthr) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = b + u * nthr;
      if (q < nv) r[u] = sv[q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = b + u * nthr;
      if (q < nv) unpack<C>(r[u], dst + q * W);
    }
  }
  if (ga >= 0) da[lt] = (C)va;
  if (gb >= 0) db[lt] = (C)vb;
  for (int i = lt + nthr; i < na; i += nthr) da[i] = (C)vec[ia[i]];
  for (int i = lt + nthr; i < nb; i += nthr) db[i] = (C)vec[ibx[i]];
}

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Per-block records: a block's descriptor followed by its index lists, with the descriptor's
// offsets relative to the record, so that one coalesced copy into LDS brings everything a
// stage needs before any of its data loads (instead of a descriptor load, then index loads,
// then data loads).  `n` int32 (a multiple of 4), 16-byte aligned on both sides.
__device__ __forceinline__ void load_record(int32_t* dst, const int32_t* __restrict__ src, int n,
                                            int lt, int nthr) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
  int4* d4 = reinterpret_cast<int4*>(dst);
  for (int q = lt; q < n / 4; q += nthr) d4[q] = s4[q];
}

// Dot products along a line of a factor block: sum over j = j0, j0 + step, ... < j1 of
// e(o_j) x(j), where the element offsets advance by d, d + dd, d + 2 dd, ... (a packed triangle's
// rows advance quadratically, everything else linearly), so no term needs a multiply.  Up to U
// elements and inputs are loaded before their products are added; the additions keep the order
// of a plain loop.
template <int U, typename C, typename E, typename X>
__device__ __forceinline__ C dot_walk(E e, int o, int d, int dd, int j0, int j1, int step, X x) {
  C acc = 0;
  int j = j0;
  for (; j + (U - 1) * step < j1; j += U * step) {
    C ev[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ev[u] = e(o);
      xv[u] = x(j + u * step);
      o += d;
      d += dd;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += ev[u] * xv[u];
  }
  for (; j < j1; j += step) {
    acc += e(o) * x(j);
    o += d;
    d += dd;
  }
  return acc;
}
// terms per batch of the LDS line walks (measured side by side: 2 is 2.8% faster than 4 on 256^2
// and no slower in FP32 on 1024^2 and 64^3; choosing per wave by line length was slower still)
constexpr int kLineUnroll = 2;

// Read-only views of the factor blocks: from LDS (packed layouts, ST) or global memory.
// Tri: packed column-major lower triangle of order n; Col: column-major rows x cols block.
template <typename S, typename C, bool ST>
struct Tri {
  const C* l;
  const S* g;
  int n;
  __device__ __forceinline__ C at(int o) const {
    if constexpr (ST) return l[o];
    else return load_as<C>(g + o);
  }
  __device__ __forceinline__ C operator()(int i, int j) const { return at(colstart(j, n) + (i - j)); }
  // sum over j = j0, j0 + step, ... <= i of (i, j) x(j)
  template <typename X>
  __device__ __forceinline__ C row_dot(int i, int j0, int step, X x) const {
    return dot_walk<kLineUnroll, C>([&](int o) { return at(o); }, colstart(j0, n) + (i - j0),
                                    step * (n - 1 - j0) - step * (step - 1) / 2, -step * step,
                                    j0, i + 1, step, x);
  }
  // sum over j = j0, j0 + step, ... < n of (j, c) x(j), j0 >= c (column c is contiguous)
  template <typename X>
  __device__ __forceinline__ C col_dot(int c, int j0, int step, X x) const {
    return dot_walk<kLineUnroll, C>([&](int o) { return at(o); }, colstart(c, n) + (j0 - c),
                                    step, 0, j0, n, step, x);
  }
};
template <typename S, typename C, bool ST>
struct Col {
  const C* l;
  const S* g;
  int rows;
  __device__ __forceinline__ C at(int o) const {
    if constexpr (ST) return l[o];
    else return load_as<C>(g + o);
  }
  __device__ __forceinline__ C operator()(int r, int c) const { return at(c * rows + r); }
  // sum over r = r0, r0 + step, ... < r1 of (r, c) x(r)
  template <typename X>
  __device__ __forceinline__ C col_dot(int c, int r0, int r1, int step, X x) const {
    return dot_walk<kLineUnroll, C>([&](int o) { return at(o); }, c * rows + r0, step, 0, r0, r1,
                                    step, x);
  }
  // sum over c = c0, c0 + step, ... < c1 of (r, c) x(c)
  template <typename X>
  __device__ __forceinline__ C row_dot(int r, int c0, int c1, int step, X x) const {
    return dot_walk<kLineUnroll, C>([&](int o) { return at(o); }, c0 * rows + r, step * rows, 0,
                                    c0, c1, step, x);
  }
};

// Results of the dense top read by the backward cell stage of its level in place of the
// boundary values in y (the write-back launch is then not needed).  Per cell: the position among
// the top's DOFs of each boundary DOF (pos) and `ne` further top DOFs that lie on no cell's
// boundary (crossings of separators), as (position, DOF id) pairs that this cell writes to y;
// part: the top's partial sums (nch ranges of n).
struct TopIn {
  const int32_t* pos = nullptr;
  const int32_t* ext = nullptr;
  int ne = 0;
  const double* part = nullptr;
  int nch = 0, n = 0;
  __device__ double sum(int i) const {
    double s = 0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * n + i];
    return s;
  }
};

// ------------------------------------------------------------------------------ cell stages --
// Sum over the `team` adjacent lanes that share one output (team a power of two <= 64).
template <typename C>
__device__ __forceinline__ C team_sum(C v, int team) {
  for (int off = team >> 1; off > 0; off >>= 1) v += __shfl_down(v, off, team);
  return v;
}

// LDS (staged): block (blk_elems) | 3 nI + 2 nB vector elements.  Outputs are computed by teams
// of `team` lanes splitting the inner dot product.
//   mode 0 (dense H):  w = L^-1 y_I and c = H y_I as nI + nB independent dot products.
//   mode 1 (links):    w = L^-1 y_I, v = L^-T w (= A_II^-1 y_I), c_b = A_BI(b, ib_b) v_ib_b.
struct NoHook {
  template <typename C>
  __device__ void operator()(C*) const {}
};

// prestaged: the block is already in LDS (a fused launch loads it while its groups run).
// hook(ys): run by every lane once the block and inputs are on their way to LDS, before the
// barrier that publishes them (ys: the LDS vector of the interior inputs); stop (LDS): looked at
// after that barrier, nothing is written if set.  own_ys: the hook writes ys itself.
template <typename S, typename C, bool ST, int MODE, typename Hook = NoHook>
__device__ __forceinline__ void cell_fwd_body(const CellDesc& d, const int32_t* __restrict__ idx,
                                              const S* __restrict__ vals, double* __restrict__ y,
                                              double* __restrict__ cb, int blk_elems, int team,
                                              bool prestaged, unsigned char* smem_raw,
                                              const double* __restrict__ in = nullptr,
                                              Hook hook = Hook{},
                                              const int* stop = nullptr, bool own_ys = false) {
  // in: where the interior values are read (y unless the input vector is another one)
  const double* src = in ? in : y;
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int nI = d.nI, nB = d.nB;
  constexpr int mode = MODE;
  const int tl = tri_count(nI);
  const S* v = vals + d.offV;
  C* blk = sm;
  C* ys = ST ? sm + blk_elems : sm;
  C* ws = ys + nI;
  C* vs = ws + nI;
  int* ib = reinterpret_cast<int*>(vs + nI);
  const int32_t* gI = idx + d.offI;
  const int nIy = own_ys ? 0 : nI;  // interior inputs gathered here
  if (ST && !prestaged) {
    stage_gather(blk, v, tl + (mode ? nB : nB * nI), src, gI, nIy, ys, gI, 0, ys, threadIdx.x,
                 blockDim.x);
  } else {
    for (int i = threadIdx.x; i < nIy; i += blockDim.x) ys[i] = (C)src[gI[i]];
  }
  const Tri<S, C, ST> Li{blk, v, nI};
  const Col<S, C, ST> H{blk + tl, v + tl, nB};
  if constexpr (MODE == 1)
    for (int b = threadIdx.x; b < nB; b += blockDim.x) ib[b] = idx[d.offC + b];
  hook(ys);
  __syncthreads();
  if (stop && *stop) return;
  const int part = threadIdx.x % team, per = blockDim.x / team;
  const int nout = mode ? nI : nI + nB;
  for (int ob = 0; ob < nout; ob += per) {
    const int o = ob + (int)threadIdx.x / team;
    C acc = 0;
    if (o < nI) {
      acc = Li.row_dot(o, part, team, [&](int j) { return ys[j]; });
    } else if (o < nout) {
      acc = H.row_dot(o - nI, part, nI, team, [&](int j) { return ys[j]; });
    }
    acc = team_sum(acc, team);
    if (part == 0 && o < nout) {
      if (o < nI) {
        y[gI[o]] = (double)acc;
        ws[o] = acc;
      } else {
        cb[d.offCB + o - nI] = (double)acc;
      }
    }
  }
  if constexpr (MODE == 1) {
    __syncthreads();
    for (int ob = 0; ob < nI; ob += per) {   // v = L^-T w
      const int o = ob + (int)threadIdx.x / team;
      C acc = 0;
      if (o < nI)
        acc = Li.col_dot(o, o + part, team, [&](int j) { return ws[j]; });
      acc = team_sum(acc, team);
      if (part == 0 && o < nI) vs[o] = acc;
    }
    __syncthreads();
    const S* cw = v + tl;
    for (int b = threadIdx.x; b < nB; b += blockDim.x)
      cb[d.offCB + b] = (double)((C)(ST ? blk[tl + b] : load_as<C>(cw + b)) * vs[ib[b]]);
  }
}

// A stop flag that is never set: symmetric cell stages read their flag through a pointer to it
// when none is given, so that the flag, the descriptor and the ids load without a branch
// between them.
__device__ const int kNeverStop = 0;

// ------------------------------------------------------------ symmetric-inverse cells (mode 2) --
// A level-0 cell stored as M = A_II^-1 (= L^-T L^-1, packed column-major lower triangle) and the
// single stencil coupling of each boundary DOF.  Forward: c_b = A_BI(b, ib_b) (M y_I)_{ib_b},
// with y_I left as it is; backward: x_I = M (y_I - A_IB x_B).  In exact arithmetic this is the
// pair of triangular passes of each sweep (E^T: y_I <- L^-1 y_I, c_B = A_BI L^-T (L^-1 y_I);
// E: x_I <- L^-T (L^-1 y_I - L^-1 A_IB x_B)), since nothing between the two sweeps reads the
// interior values.  One wavefront per cell (interiors of at most 64 DOFs), lane i forming
// (M t)_i.  A cell of at most the level's square order (SymCfg::n, the usual interior size) is
// copied into an LDS square with both halves filled (a table gives the two positions of every
// element), then lane i walks row i.  The leading dimension is odd, so the mirrored stores of
// consecutive packed elements and the row walks of consecutive lanes meet no bank conflicts.
// The block is stored in the order of sym_store_index: each lane loads 16-byte vectors and the
// wavefront's k-th store of a vector covers consecutive packed elements.  A larger cell (the
// few of the last row and column of cells) stays a packed triangle in LDS and lane i walks its
// row i (consecutive lanes, consecutive words) and then its column i.  The LDS of a launch is
// sized for the usual cell, so more wavefronts stay resident.

// LDS elements of the compute type a symmetric cell stage needs besides its record: the matrix,
// t, and (M t) forward or the boundary values and their couplings backward.
__host__ __device__ inline int sym_smem_elems(int mat, int maxB) {
  const int b2 = 2 * round_up(maxB, 4);
  return mat + kSymMaxCell + (b2 > kSymMaxCell ? b2 : kSymMaxCell);
}

// Every element of the cell block into LDS: to both of its square positions (tab: this order's
// entries, in storage order) or to its packed position.  sym_load issues the loads (so that a
// stage can issue its other loads before it waits for them) and sym_store makes the stores.
// Every lane issues every load, the vector index clamped to the block's last vector and the
// table index to the table's last (a cell in the packed form reads the square's order's table
// and ignores it): loads under a lane condition would make the compiler wait for every
// outstanding load where the paths join, and move the gathers of the inputs behind the
// block's loads.  A block starts 16-byte aligned and its storage runs to sym_coff(tl), so every
// vector lies inside it; the spare slots of the last chunk land on the spare word (tab) or
// below the packed triangle's padded end (packed), where nothing reads them.
template <typename S>
struct SymRegs {
  static constexpr int E = 16 / sizeof(S);  // elements per vector
  static constexpr int P =                  // vectors per lane (chunks)
      (kSymMaxCell * (kSymMaxCell + 1) / 2 + 64 * E - 1) / (64 * E);
  int4 e[P];
  int32_t t[P][E];
};

template <typename S>
__device__ __forceinline__ void sym_load(SymRegs<S>& R, const S* __restrict__ v, int tl,
                                         const int32_t* __restrict__ tab, int ttl, int lane) {
  constexpr int E = SymRegs<S>::E, P = SymRegs<S>::P;
  const int4* vv = reinterpret_cast<const int4*>(v);
  const int last = max((tl + E - 1) / E - 1, 0), tlast = max((ttl + E - 1) / E - 1, 0);
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int q = lane + 64 * u;
    R.e[u] = vv[min(q, last)];
    const int tq = min(q, tlast);
    if constexpr (E == 2) {
      const int2 w = reinterpret_cast<const int2*>(tab)[tq];
      R.t[u][0] = w.x;
      R.t[u][1] = w.y;
    } else {
#pragma unroll
      for (int h = 0; h < E / 4; ++h) {
        const int4 w = reinterpret_cast<const int4*>(tab)[tq * (E / 4) + h];
        R.t[u][4 * h] = w.x;
        R.t[u][4 * h + 1] = w.y;
        R.t[u][4 * h + 2] = w.z;
        R.t[u][4 * h + 3] = w.w;
      }
    }
  }
}

template <typename S, typename C>
__device__ __forceinline__ void sym_store(C* sq, const SymRegs<S>& R, int tl, bool tab, int lane) {
  constexpr int E = SymRegs<S>::E, P = SymRegs<S>::P;
  const int nv = (tl + E - 1) / E;
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int q = lane + 64 * u;
    if (q < nv) {
      S ev[E];
      __builtin_memcpy(ev, &R.e[u], 16);
      if (tab) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const C x = load_as<C>(ev + k);
          sq[R.t[u][k] & 0xffff] = x;
          sq[R.t[u][k] >> 16] = x;
        }
      } else {
        const int qc = sym_chunk_q(u, tl, E);  // packed element lane + qc k of chunk u
#pragma unroll
        for (int k = 0; k < E; ++k) sq[64 * E * u + lane + qc * k] = load_as<C>(ev + k);
      }
    }
  }
}

// (M t)_lane for lane < n from the square (leading dimension ld): row `lane` against t
// (broadcast from LDS), eight terms per batch into four running sums, added in a fixed order.
template <typename C>
__device__ __forceinline__ C sym_row(const C* sq, const C* ts, int n, int ld, int lane) {
  const C* row = sq + lane * ld;
  C a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int c = 0;
  for (; c + 8 <= n; c += 8) {
    C m[8], t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m[u] = row[c + u];
      t[u] = ts[c + u];
    }
    a0 += m[0] * t[0];
    a1 += m[1] * t[1];
    a2 += m[2] * t[2];
    a3 += m[3] * t[3];
    a0 += m[4] * t[4];
    a1 += m[5] * t[5];
    a2 += m[6] * t[6];
    a3 += m[7] * t[7];
  }
  for (; c < n; ++c) a0 += row[c] * ts[c];
  return (a0 + a1) + (a2 + a3);
}

// (M t)_lane for lane < n from the packed column-major lower triangle P: row `lane` left of
// the diagonal (entry (lane, j) at colstart(j) + lane - j, consecutive across lanes), then
// column `lane` from the diagonal down (contiguous).
template <typename C>
__device__ __forceinline__ C sym_packed(const C* P, const C* ts, int n, int lane) {
  C a = 0;
  int o = lane;  // colstart(j) + lane - j for j = 0
  for (int j = 0; j < lane; ++j) {
    a += P[o] * ts[j];
    o += n - j - 1;
  }
  const C* col = P + o;  // o = colstart(lane): the diagonal entry
  C b = 0;
  for (int j = lane; j < n; ++j) b += col[j - lane] * ts[j];
  return a + b;
}

// (M t)_lane: the square or the packed form, as the cell's size decided.
template <typename C>
__device__ __forceinline__ C sym_apply(const C* sq, const C* ts, int nI, const SymCfg& cfg,
                                       int lane) {
  return nI <= cfg.n ? sym_row(sq, ts, nI, cfg.ld, lane) : sym_packed(sq, ts, nI, lane);
}

// Forward stage of a symmetric cell (one wavefront).  idx: the cell's record (LDS).  in: where
// the interior inputs are read (y unless another vector; the output y then receives them at the
// interiors).  hook(ts) runs while the block loads, before the barrier that publishes ts; with
// own_ys the hook writes ts (and y_I) itself.  stop: looked at after that barrier.
template <typename S, typename C, typename Hook = NoHook>
__device__ __forceinline__ void cell_fwd_sym(const CellDesc& d, const int32_t* __restrict__ idx,
                                             const S* __restrict__ vals, double* __restrict__ y,
                                             double* __restrict__ cb, const SymCfg& cfg,
                                             unsigned char* smem_raw,
                                             const double* __restrict__ in = nullptr,
                                             Hook hook = Hook{}, const int* stop = nullptr,
                                             bool own_ys = false, int pre_gi = 0,
                                             bool pre = false) {
  const double* src = in ? in : y;
  C* sq = reinterpret_cast<C*>(smem_raw);
  C* ts = sq + cfg.mat;
  C* zs = ts + kSymMaxCell;
  const int lane = threadIdx.x;
  const int nI = d.nI, nB = d.nB, tl = tri_count(nI);
  const S* v = vals + d.offV;
  const int32_t* gI = idx + d.offI;
  const int32_t* ibp = idx + d.offC;
  const S* cw = v + sym_coff(tl);  // the couplings
  // loads in order of need: the interior ids (pre: already loaded with the descriptor, so the
  // gathers go out first, idle lanes at the first interior DOF), the block, the inputs, the
  // first couplings
  int gi = -1;
  double yv = 0;
  if (!own_ys && pre) {
    const int g0 = __builtin_amdgcn_readfirstlane(pre_gi);
    gi = lane < nI ? pre_gi : -1;
    yv = src[lane < nI ? pre_gi : g0];
    if (lane >= nI) yv = 0;
  } else if (!own_ys && lane < nI) {
    gi = gI[lane];
  }
  // the record's mode word: where the cell's order's table entries start (-1: packed form)
  const bool square = d.mode >= 0;
  SymRegs<S> R;
  sym_load<S>(R, v, tl, cfg.tab + (square ? d.mode : cfg.sqoff),
              square ? tl : (int)tri_count(cfg.n), lane);
  if (!own_ys && !pre && lane < nI) yv = src[gi];
  const int lb = min(lane, max(nB - 1, 0));  // (clamped: no load under a lane condition)
  int ib0 = ibp[lb];
  C a0 = load_as<C>(cw + lb);
  if (!own_ys && pre) ts[lane] = (C)yv;
  sym_store<S, C>(sq, R, tl, square, lane);
  if (!own_ys && !pre) ts[lane] = (C)yv;
  hook(ts);
  __syncthreads();
  if (stop && *stop) return;
  if (lane < nI) zs[lane] = sym_apply(sq, ts, nI, cfg, lane);
  __syncthreads();
  if (lane < nB) cb[d.offCB + lane] = (double)(a0 * zs[ib0]);
  for (int b = lane + 64; b < nB; b += 64)
    cb[d.offCB + b] = (double)(load_as<C>(cw + b) * zs[ibp[b]]);
  if (in && in != y && lane < nI) y[gi] = yv;  // the output takes the inputs at the interiors
}

// Backward stage of a symmetric cell (one wavefront): x_I = M (x_I - A_IB x_B), the boundary
// values read from x or, with a dense top folded into this level, added up from its partial
// sums (and written to x, as every cell on that boundary does).
template <typename S, typename C>
__device__ __forceinline__ void cell_bwd_sym(const CellDesc& d, const int32_t* __restrict__ idx,
                                             const S* __restrict__ vals, double* __restrict__ x,
                                             const SymCfg& cfg, unsigned char* smem_raw,
                                             const TopIn& top, int r0 = 0, int r1 = 0,
                                             bool pre = false) {
  C* sq = reinterpret_cast<C*>(smem_raw);
  C* ts = sq + cfg.mat;
  C* xbs = ts + kSymMaxCell;
  const int lane = threadIdx.x;
  const int nI = d.nI, nB = d.nB, tl = tri_count(nI);
  C* abs_ = xbs + round_up(nB, 4);
  const S* v = vals + d.offV;
  const int32_t* gI = idx + d.offI;
  const int32_t* gB = idx + d.offB;
  const int32_t* lw = idx + d.offC + nB;  // per interior DOF: link count, boundary positions
  // pre: the record's first 128 words after the descriptor (r0: word 8 + lane, r1: word
  // 72 + lane) came with the descriptor and hold both id lists, so the gathers go out at once
  // (idle lanes at the first interior DOF), then the link words, couplings and the block
  const bool fast = pre && !top.pos && nI + nB <= 128 && nB <= 64;
  int gi = -1, w = 0;
  double xi = 0, xv = 0;
  C ab = 0;
  if (fast) {
    const int k = (nI + lane) & 63;  // boundary DOF lane is word 8 + nI + lane
    const int blo = __shfl(r0, k, 64), bhi = __shfl(r1, k, 64);
    const int gb = nI + lane < 64 ? blo : bhi;
    const int g0 = __builtin_amdgcn_readfirstlane(r0);
    gi = lane < nI ? r0 : -1;
    xi = x[lane < nI ? r0 : g0];
    xv = x[lane < nB ? gb : g0];
    if (lane >= nI) xi = 0;
    w = lw[min(lane, nI - 1)];  // (clamped: no load under a lane condition)
    ab = load_as<C>(v + sym_coff(tl) + min(lane, nB - 1));
    if (lane >= nI) w = 0;
  } else if (lane < nI) {
    gi = gI[lane];
    w = lw[lane];
    xi = x[gi];
  }
  for (int b = fast ? nB : lane; b < nB; b += 64) {
    double xv;
    if (top.pos) {
      xv = top.sum(top.pos[b]);
      x[gB[b]] = xv;
    } else {
      xv = x[gB[b]];
    }
    xbs[b] = (C)xv;
    abs_[b] = load_as<C>(v + sym_coff(tl) + b);
  }
  if (top.pos)
    for (int e = lane; e < top.ne; e += 64) x[top.ext[2 * e + 1]] = top.sum(top.ext[2 * e]);
  const bool square = d.mode >= 0;  // see cell_fwd_sym
  SymRegs<S> R;
  sym_load<S>(R, v, tl, cfg.tab + (square ? d.mode : cfg.sqoff),
              square ? tl : (int)tri_count(cfg.n), lane);
  if (fast && lane < nB) {
    xbs[lane] = (C)xv;
    abs_[lane] = ab;
  }
  sym_store<S, C>(sq, R, tl, square, lane);
  __syncthreads();
  if (lane < nI) {
    C t = (C)xi;
    const int cnt = w & 255;
    for (int q = 0; q < cnt; ++q) {
      const int b = (w >> (8 * (q + 1))) & 255;
      t -= abs_[b] * xbs[b];
    }
    ts[lane] = t;
  }
  __syncthreads();
  if (lane < nI) x[gi] = (double)sym_apply(sq, ts, nI, cfg, lane);
}

// The first stage of a step's first apply, making the step's right-hand side on the way: the
// cell's workgroup forms g = (I + dt/2 M) u + dt r(u) (Sec. 2.1) at its interiors, which are the
// stage's inputs (z = g is the initial residual), and at the DOFs of its copy list (outside every
// interior, z = r = g there); r = g and x = 0 at all of them, and the cell's share of ||g||^2 in
// part[cell].  Block 0 starts the step's scalars (the test of g is made by the first update).
// Queued ahead of the previous step's outcome (ahead), it does nothing unless that step ended
// well (ok_next, written by its closing test and read only here): hold and done are set instead,
// so the rest of the step does nothing.
template <typename S, typename C, bool ST, int MODE>
__device__ __forceinline__ void cell_rhs(const int32_t* __restrict__ recs, int stride,
                                         const S* __restrict__ vals, double* __restrict__ y,
                                         double* __restrict__ cb, int blk_elems, int team,
                                         const int32_t* __restrict__ gcopy, int gcstride,
                                         const CgRhs& rhs, unsigned char* smem_raw,
                                         double* gred, SymCfg sym, int flen) {
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  const bool held = rhs.ahead && !rhs.st->ok_next;  // (the same in every block)
  load_record(rec, recs + (int64_t)blockIdx.x * stride, flen, threadIdx.x, blockDim.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CgState* st = rhs.st;
    st->hold = held ? 1 : 0;
    st->done = held ? 1 : 0;
    if (!held) {
      st->iters = 0;
      st->status = 0;
      st->maxit = rhs.maxit;
    }
  }
  if (held) return;
  __syncthreads();
  const CellDesc d = *reinterpret_cast<const CellDesc*>(rec);
  auto g_at = [&](int64_t i) {
    const double ui = rhs.u[i];
    const double l = rhs.dim == 2
                         ? link_sum<2>(i, rhs.n, rhs.links, ui, [&](int64_t k) { return rhs.u[k]; })
                         : link_sum<3>(i, rhs.n, rhs.links, ui, [&](int64_t k) { return rhs.u[k]; });
    return cn_rhs_value(ui, l, rhs.dt, rhs.kind, rhs.k1, rhs.k2);
  };
  double acc = 0;
  auto make = [&](C* ys) {
    const int32_t* gI = rec + d.offI;
    for (int i = threadIdx.x; i < d.nI; i += blockDim.x) {
      const double g = g_at(gI[i]);
      ys[i] = (C)g;
      rhs.r[gI[i]] = g;
      rhs.x[gI[i]] = 0.0;
      if constexpr (MODE == 2) y[gI[i]] = g;  // (the symmetric stage keeps y_I = its input)
      acc += g * g;
    }
    const int32_t* cp = gcopy + (int64_t)blockIdx.x * gcstride;
    for (int e = threadIdx.x; e < cp[0]; e += blockDim.x) {
      const int32_t id = cp[1 + e];
      const double g = g_at(id);
      rhs.r[id] = g;
      rhs.x[id] = 0.0;
      y[id] = g;
      acc += g * g;
    }
  };
  if constexpr (MODE == 2)
    cell_fwd_sym<S, C>(d, rec, vals, y, cb, sym, smem_raw + 4 * stride, nullptr, make, nullptr,
                       true);
  else
    cell_fwd_body<S, C, ST, MODE>(d, rec, vals, y, cb, blk_elems, team, false,
                                  smem_raw + 4 * stride, nullptr, make, nullptr, true);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) gred[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += gred[w];
    rhs.part[blockIdx.x] = s;
  }
}

template <typename S, typename C, bool ST, int MODE>
// One workgroup per cell; its record (stride int32) goes to the front of LDS.
__global__ __launch_bounds__(256) void k_cell_fwd(const int32_t* __restrict__ recs, int stride,
                                                  const S* __restrict__ vals,
                                                  double* __restrict__ y, double* __restrict__ cb,
                                                  const int* __restrict__ done, int blk_elems,
                                                  int team, CgGate gate,
                                                  const int32_t* __restrict__ gcopy, int gcstride,
                                                  CgRhs rhs, SymCfg sym, int flen) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int gstop;
  __shared__ double gred[4];
  if (rhs.u) {  // the step's right-hand side made here (see cell_rhs)
    cell_rhs<S, C, ST, MODE>(recs, stride, vals, y, cb, blk_elems, team, gcopy, gcstride, rhs,
                             smem_raw, gred, sym, flen);
    return;
  }
  // symmetric cells read their record in place (global memory) and keep all of LDS for the
  // block; the other modes copy it to the front of LDS first
  const int32_t* grec = recs + (int64_t)blockIdx.x * stride;
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  // with a gate, the PCG convergence test comes first: its partials, the state and this
  // cell's copy list load ahead of the record
  const bool gated = gate.st != nullptr;
  CgTotal ct;
  int g_done = 0, g_maxit = 0, cid = -1, ccnt = 0;
  double g_tol2 = 0, cval = 0;
  const int32_t* cp = gcopy + (int64_t)blockIdx.x * gcstride;
  if (gated) {
    if (threadIdx.x < 64) ct.load(gate.part, gate.nb);
    // the test of g (init) looks at hold only (the right-hand side just set it; done is the
    // previous step's); later tests at done (set by an earlier test of the step)
    g_done = gate.init ? gate.st->hold : gate.st->done;
    g_tol2 = gate.st->tol2;
    g_maxit = gate.init ? gate.maxit : gate.st->maxit;
    ccnt = cp[0];
    if ((int)threadIdx.x < gcstride - 1) cid = cp[1 + threadIdx.x];
  }
  if constexpr (MODE != 2) load_record(rec, grec, flen, threadIdx.x, blockDim.x);
  // symmetric cells: the descriptor and (records of 72 words or more) the interior ids load
  // together with the stop flag
  const bool pre = MODE == 2 && stride >= 72;
  CellDesc dsym{};
  int pre_gi = 0;
  if constexpr (MODE == 2) {
    dsym = *reinterpret_cast<const CellDesc*>(grec);
    if (pre) pre_gi = grec[8 + threadIdx.x];
  }
  const int dn = gated ? 0 : MODE == 2 ? *(done ? done : &kNeverStop) : (done ? *done : 0);
  if (gated && cid >= 0) cval = gate.src[cid];  // (padding entries read DOF 0; never stored)
  if constexpr (MODE != 2) __syncthreads();
  if (dn || (MODE == 2 && dsym.nI < 0)) return;  // (the descriptor's load stays ahead of this)
  const CellDesc d = MODE == 2 ? dsym : *reinterpret_cast<const CellDesc*>(rec);
  // the test's verdict is reached while the cell's block and inputs load (they are only read
  // before it is known)
  auto verdict = [&](C*) {
    if (!gated || threadIdx.x >= 64) return;
    const double t = ct.sum(gate.part, gate.nb);
    if (threadIdx.x != 0) return;
    if (g_done) {  // stopped by an earlier test: nothing to publish (a held step: stop it)
      if (gate.init && blockIdx.x == 0) gate.st->done = 1;
      gstop = 1;
    } else {
      gstop = cg_verdict(gate.st, gate.init, gate.it0, gate.rtol, t, g_tol2, g_maxit,
                         blockIdx.x == 0);
    }
  };
  if constexpr (MODE == 2)
    cell_fwd_sym<S, C>(d, grec, vals, y, cb, sym, smem_raw, gate.src, verdict,
                       gated ? &gstop : nullptr, false, pre_gi, pre);
  else
    cell_fwd_body<S, C, ST, MODE>(d, rec, vals, y, cb, blk_elems, team, false,
                                  smem_raw + 4 * stride, gate.src, verdict,
                                  gated ? &gstop : nullptr);
  if (gated && gstop) return;
  if (gated) {  // the DOFs outside every interior that this cell hands over unchanged
    if ((int)threadIdx.x < ccnt) y[cid] = cval;
    for (int e = threadIdx.x + blockDim.x; e < ccnt; e += blockDim.x)
      y[cp[1 + e]] = gate.src[cp[1 + e]];
  }
}

//   mode 0: x_I <- L^-T x_I - H^T x_B as nI dot products over [L^-1 column | H column].
//   mode 1: t = A_IB x_B (one link per boundary DOF), x_I <- L^-T (x_I - L^-1 t).
template <typename S, typename C, bool ST, int MODE>
__device__ __forceinline__ void cell_bwd_body(const CellDesc& d, const int32_t* __restrict__ idx,
                                              const S* __restrict__ vals, double* __restrict__ x,
                                              int blk_elems, int team, unsigned char* smem_raw,
                                              const TopIn& top = TopIn{}) {
  C* sm = reinterpret_cast<C*>(smem_raw);
  const int nI = d.nI, nB = d.nB;
  constexpr int mode = MODE;
  const int tl = tri_count(nI);
  const S* v = vals + d.offV;
  C* blk = sm;
  C* xs = ST ? sm + blk_elems : sm;
  C* xb = xs + nI;
  C* ts = xb + nB;
  C* us = ts + nI;
  int* ib = reinterpret_cast<int*>(us + nI);
  const int32_t* gI = idx + d.offI;
  const int nBy = top.pos ? 0 : nB;  // boundary values read from y
  // the first boundary DOF of each lane: its partial sums are loaded before the block is staged
  constexpr int kTopPre = 16;
  double tp[kTopPre];
  const bool pre = top.pos && top.nch <= kTopPre && (int)threadIdx.x < nB;
  if (pre) {
    const int i = top.pos[threadIdx.x];
#pragma unroll
    for (int c = 0; c < kTopPre; ++c) tp[c] = c < top.nch ? top.part[(int64_t)c * top.n + i] : 0.0;
  }
  if constexpr (ST) {
    stage_gather(blk, v, tl + (mode ? nB : nB * nI), x, gI, nI, xs, idx + d.offB, nBy, xb,
                 threadIdx.x, blockDim.x);
  } else {
    for (int i = threadIdx.x; i < nI; i += blockDim.x) xs[i] = (C)x[gI[i]];
    for (int b = threadIdx.x; b < nBy; b += blockDim.x) xb[b] = (C)x[idx[d.offB + b]];
  }
  if (top.pos) {  // the boundary values are the dense top's results: add up its partial sums
    for (int b = threadIdx.x; b < nB; b += blockDim.x) {
      double s = 0;
      if (pre && b == (int)threadIdx.x) {
#pragma unroll
        for (int c = 0; c < kTopPre; ++c)
          if (c < top.nch) s += tp[c];  // the order of TopIn::sum
      } else {
        s = top.sum(top.pos[b]);
      }
      xb[b] = (C)s;
      x[idx[d.offB + b]] = s;  // every cell on a separator writes the same sum
    }
    for (int e = threadIdx.x; e < top.ne; e += blockDim.x)
      x[top.ext[2 * e + 1]] = top.sum(top.ext[2 * e]);
  }
  const Tri<S, C, ST> Li{blk, v, nI};
  const Col<S, C, ST> H{blk + tl, v + tl, nB};
  if constexpr (MODE == 1)
    for (int b = threadIdx.x; b < nB; b += blockDim.x) ib[b] = idx[d.offC + b];
  __syncthreads();
  const int part = threadIdx.x % team, per = blockDim.x / team;
  if constexpr (MODE == 0) {
    for (int ob = 0; ob < nI; ob += per) {
      const int o = ob + (int)threadIdx.x / team;
      C acc = 0;
      if (o < nI) {
        acc = Li.col_dot(o, o + part, team, [&](int j) { return xs[j]; });
        acc -= H.col_dot(o, part, nB, team, [&](int b) { return xb[b]; });
      }
      acc = team_sum(acc, team);
      if (part == 0 && o < nI) x[gI[o]] = (double)acc;
    }
    return;
  }
  const S* cw = v + tl;
  // the links of each interior DOF: rowptr (nI + 1) and boundary positions (nB) after ib
  const int32_t* rp = idx + d.offC + nB;
  const int32_t* bl = rp + nI + 1;
  for (int i = threadIdx.x; i < nI; i += blockDim.x) {   // t = A_IB x_B
    C acc = 0;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
      const int b = bl[q];
      acc += (C)(ST ? blk[tl + b] : load_as<C>(cw + b)) * xb[b];
    }
    ts[i] = acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nI; ob += per) {                 // u = x_I - L^-1 t
    const int o = ob + (int)threadIdx.x / team;
    C acc = 0;
    if (o < nI)
      acc = Li.row_dot(o, part, team, [&](int j) { return ts[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && o < nI) us[o] = xs[o] - acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nI; ob += per) {                 // x_I = L^-T u
    const int o = ob + (int)threadIdx.x / team;
    C acc = 0;
    if (o < nI)
      acc = Li.col_dot(o, o + part, team, [&](int j) { return us[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && o < nI) x[gI[o]] = (double)acc;
  }
}

template <typename S, typename C, bool ST, int MODE>
__global__ __launch_bounds__(256) void k_cell_bwd(const int32_t* __restrict__ recs, int stride,
                                                  const S* __restrict__ vals,
                                                  double* __restrict__ x,
                                                  const int* __restrict__ done, int blk_elems,
                                                  int team, const int32_t* __restrict__ tpos,
                                                  int tstride, const double* __restrict__ tpart,
                                                  int tnch, int tn, SymCfg sym) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // symmetric cells read their record in place (see k_cell_fwd)
  const int32_t* grec = recs + (int64_t)blockIdx.x * stride;
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  if constexpr (MODE != 2) load_record(rec, grec, stride, threadIdx.x, blockDim.x);
  // symmetric cells: the descriptor and (records of 136 words or more, no dense top folded in)
  // the 128 words after it, which hold both id lists, load together with the stop flag
  const bool pre = MODE == 2 && stride >= 136 && !tpos;
  CellDesc dsym{};
  int r0 = 0, r1 = 0;
  if constexpr (MODE == 2) {
    dsym = *reinterpret_cast<const CellDesc*>(grec);
    if (pre) {
      r0 = grec[8 + threadIdx.x];
      r1 = grec[72 + threadIdx.x];
    }
  }
  const int dn = MODE == 2 ? *(done ? done : &kNeverStop) : (done ? *done : 0);
  if constexpr (MODE != 2) __syncthreads();
  if (dn || (MODE == 2 && dsym.nI < 0)) return;  // (the descriptor's load stays ahead of this)
  const CellDesc d = MODE == 2 ? dsym : *reinterpret_cast<const CellDesc*>(rec);
  TopIn top;
  if (tpos) {  // per cell: ne, (position, id) x ne, then one position per boundary DOF
    const int32_t* r = tpos + (int64_t)blockIdx.x * tstride;
    top = TopIn{r + tstride - d.nB, r + 1, r[0], tpart, tnch, tn};
  }
  if constexpr (MODE == 2)
    cell_bwd_sym<S, C>(d, grec, vals, x, sym, smem_raw, top, r0, r1, pre);
  else
    cell_bwd_body<S, C, ST, MODE>(d, rec, vals, x, blk_elems, team, smem_raw + 4 * stride, top);
}

// ----------------------------------------------------------------------------- group stages --
// A workgroup handles blockDim/seg groups, `seg` lanes each.  Every phase runs on all lanes
// (empty loops where a group has nothing to do) so the barriers are uniform.
// LDS per group (staged): block (blk_elems) then yg/zg (n each) and tv/uv (nr each).
// A lane segment without a group gets an empty descriptor (n = 0) and still takes part in every
// barrier.
template <typename S, typename C, bool ST>
__device__ __forceinline__ void group_fwd_body(const GroupDesc& d, int seg, int per_group,
                                               int blk_elems, int team,
                                               const int32_t* __restrict__ idx,
                                               const S* __restrict__ vals,
                                               double* __restrict__ y,
                                               const double* __restrict__ cb,
                                               unsigned char* smem_raw, bool dense = false) {
  const int gsel = threadIdx.x / seg, lt = threadIdx.x - gsel * seg;
  const int n = d.n, nr = dense ? 0 : d.nr, k = n - nr;
  C* base = reinterpret_cast<C*>(smem_raw) + (int64_t)gsel * per_group;
  const S* v = vals + d.offV;
  const int tg = dense ? n * n : tri_count(n), tt = k * nr, tr = tri_count(nr);
  C* blk = base;
  C* yg = ST ? base + blk_elems : base;
  C* zg = yg + n;
  C* tv = zg + n;
  C* uv = tv + nr;
  if constexpr (ST) stage_flat(blk, v, tg + tt + tr, lt, seg);
  const Tri<S, C, ST> Lg{blk, v, n};
  const Col<S, C, ST> T{blk + tg, v + tg, k};
  const Tri<S, C, ST> Lr{blk + tg + tt, v + tg + tt, nr};
  const int32_t* gi_idx = idx + d.offIdx;
  const int32_t* gp = idx + d.offGP;
  const int32_t* slots = gp + n + 1;
  const int32_t* perm = idx + d.offPerm;
  for (int i = lt; i < n; i += seg) {  // contributions loaded two at a time
    double acc = y[gi_idx[i]];
    int s = gp[i];
    const int s1 = gp[i + 1];
    for (; s + 1 < s1; s += 2) {
      const double c0 = cb[slots[s]], c1 = cb[slots[s + 1]];
      acc -= c0;
      acc -= c1;
    }
    if (s < s1) acc -= cb[slots[s]];
    yg[i] = (C)acc;
  }
  __syncthreads();
  // Every product is split over `team` adjacent lanes per output.
  const int part = lt % team, per_t = seg / team;
  if (dense) {  // the whole step at once: y_g = G (y_g - contributions)
    const Col<S, C, ST> G{blk, v, n};
    for (int ob = 0; ob < n; ob += per_t) {
      const int i = ob + lt / team;
      C acc = 0;
      if (i < n) acc = G.row_dot(i, part, n, team, [&](int j) { return yg[j]; });
      acc = team_sum(acc, team);
      if (part == 0 && i < n) y[gi_idx[i]] = (double)acc;
    }
    return;
  }
  for (int ob = 0; ob < n; ob += per_t) {    // C^T: z = L_g^-1 y_g
    const int i = ob + lt / team;
    C acc = 0;
    if (i < n)
      acc = Lg.row_dot(i, part, team, [&](int j) { return yg[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < n) zg[i] = acc;
  }
  __syncthreads();
  // K^T (no-op when nr == 0)
  for (int ob = 0; ob < nr; ob += per_t) {   // y_I~ - T^T y_I^
    const int i = ob + lt / team;
    C acc = 0;
    if (i < nr)
      acc = T.col_dot(i, part, k, team, [&](int s) { return zg[perm[nr + s]]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < nr) tv[i] = zg[perm[i]] - acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nr; ob += per_t) {   // t = L_s^-1 (...)
    const int i = ob + lt / team;
    C acc = 0;
    if (i < nr)
      acc = Lr.row_dot(i, part, team, [&](int j) { return tv[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < nr) uv[i] = acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nr; ob += per_t) {   // L_s^-T t
    const int i = ob + lt / team;
    C acc = 0;
    if (i < nr)
      acc = Lr.col_dot(i, i + part, team, [&](int j) { return uv[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < nr) tv[i] = acc;
  }
  __syncthreads();
  if (nr > 0) {
    for (int ob = 0; ob < k; ob += per_t) {  // y_I^ += T L_s^-T t
      const int s = ob + lt / team;
      C acc = 0;
      if (s < k)
        acc = T.row_dot(s, part, nr, team, [&](int i) { return tv[i]; });
      acc = team_sum(acc, team);
      if (part == 0 && s < k) y[gi_idx[perm[nr + s]]] = (double)(zg[perm[nr + s]] + acc);
    }
    for (int i = lt; i < nr; i += seg) y[gi_idx[perm[i]]] = (double)uv[i];
  } else {
    for (int i = lt; i < n; i += seg) y[gi_idx[i]] = (double)zg[i];
  }
}

template <typename S, typename C, bool ST>
// blockDim/seg groups per workgroup, consecutive, so their records are one contiguous copy.
__global__ __launch_bounds__(256) void k_group_fwd(const int32_t* __restrict__ recs, int stride,
                                                   int ngroup, int seg, int per_group,
                                                   int blk_elems, int team,
                                                   const S* __restrict__ vals,
                                                   double* __restrict__ y,
                                                   const double* __restrict__ cb,
                                                   const int* __restrict__ done, int gdense) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int per = blockDim.x / seg, g0 = blockIdx.x * per, cnt = min(per, ngroup - g0);
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  load_record(rec, recs + (int64_t)g0 * stride, cnt * stride, threadIdx.x, blockDim.x);
  const int dn = done ? *done : 0;
  __syncthreads();
  if (dn) return;
  const int gsel = threadIdx.x / seg;
  const int32_t* rb = rec + gsel * stride;
  GroupDesc d{};
  if (gsel < cnt) d = *reinterpret_cast<const GroupDesc*>(rb);
  group_fwd_body<S, C, ST>(d, seg, per_group, blk_elems, team, rb, vals, y, cb,
                           smem_raw + 4 * per * stride, gdense != 0);
}

template <typename S, typename C, bool ST>
__device__ __forceinline__ void group_bwd_body(const GroupDesc& d, int seg, int per_group,
                                               int blk_elems, int team,
                                               const int32_t* __restrict__ idx,
                                               const S* __restrict__ vals,
                                               double* __restrict__ x, unsigned char* smem_raw,
                                               bool dense = false) {
  const int gsel = threadIdx.x / seg, lt = threadIdx.x - gsel * seg;
  const int n = d.n, nr = dense ? 0 : d.nr, k = n - nr;
  C* base = reinterpret_cast<C*>(smem_raw) + (int64_t)gsel * per_group;
  const S* v = vals + d.offV;
  const int tg = dense ? n * n : tri_count(n), tt = k * nr, tr = tri_count(nr);
  C* blk = base;
  C* xg = ST ? base + blk_elems : base;
  C* zg = xg + n;
  C* tv = zg + n;
  C* uv = tv + nr;
  if constexpr (ST) stage_flat(blk, v, tg + tt + tr, lt, seg);
  const Tri<S, C, ST> Lg{blk, v, n};
  const Col<S, C, ST> T{blk + tg, v + tg, k};
  const Tri<S, C, ST> Lr{blk + tg + tt, v + tg + tt, nr};
  const int32_t* gi_idx = idx + d.offIdx;
  const int32_t* perm = idx + d.offPerm;
  for (int i = lt; i < n; i += seg) xg[i] = (C)x[gi_idx[i]];
  __syncthreads();
  const int part = lt % team, per_t = seg / team;
  if (dense) {  // the whole step at once: x_g = G^T x_g
    const Col<S, C, ST> G{blk, v, n};
    for (int ob = 0; ob < n; ob += per_t) {
      const int i = ob + lt / team;
      C acc = 0;
      if (i < n) acc = G.col_dot(i, part, n, team, [&](int j) { return xg[j]; });
      acc = team_sum(acc, team);
      if (part == 0 && i < n) x[gi_idx[i]] = (double)acc;
    }
    return;
  }
  for (int ob = 0; ob < nr; ob += per_t) {   // a = T^T x_I^
    const int i = ob + lt / team;
    C acc = 0;
    if (i < nr)
      acc = T.col_dot(i, part, k, team, [&](int s) { return xg[perm[nr + s]]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < nr) tv[i] = acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nr; ob += per_t) {   // x_I~ + L_s^-1 a
    const int i = ob + lt / team;
    C acc = 0;
    if (i < nr)
      acc = Lr.row_dot(i, part, team, [&](int j) { return tv[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < nr) uv[i] = xg[perm[i]] + acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nr; ob += per_t) {   // u = L_s^-T (...)
    const int i = ob + lt / team;
    C acc = 0;
    if (i < nr)
      acc = Lr.col_dot(i, i + part, team, [&](int j) { return uv[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < nr) tv[i] = acc;
  }
  __syncthreads();
  if (nr > 0) {
    for (int ob = 0; ob < k; ob += per_t) {  // x_I^ -= T u
      const int s = ob + lt / team;
      C acc = 0;
      if (s < k)
        acc = T.row_dot(s, part, nr, team, [&](int i) { return tv[i]; });
      acc = team_sum(acc, team);
      if (part == 0 && s < k) zg[perm[nr + s]] = xg[perm[nr + s]] - acc;
    }
    for (int i = lt; i < nr; i += seg) zg[perm[i]] = tv[i];
  } else {
    for (int i = lt; i < n; i += seg) zg[i] = xg[i];
  }
  __syncthreads();
  for (int ob = 0; ob < n; ob += per_t) {    // C: x_g = L_g^-T x_g
    const int i = ob + lt / team;
    C acc = 0;
    if (i < n)
      acc = Lg.col_dot(i, i + part, team, [&](int j) { return zg[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && i < n) x[gi_idx[i]] = (double)acc;
  }
}

template <typename S, typename C, bool ST>
__global__ __launch_bounds__(256) void k_group_bwd(const int32_t* __restrict__ recs, int stride,
                                                   int ngroup, int seg, int per_group,
                                                   int blk_elems, int team,
                                                   const S* __restrict__ vals,
                                                   double* __restrict__ x,
                                                   const int* __restrict__ done, int gdense) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int per = blockDim.x / seg, g0 = blockIdx.x * per, cnt = min(per, ngroup - g0);
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  load_record(rec, recs + (int64_t)g0 * stride, cnt * stride, threadIdx.x, blockDim.x);
  const int dn = done ? *done : 0;
  __syncthreads();
  if (dn) return;
  const int gsel = threadIdx.x / seg;
  const int32_t* rb = rec + gsel * stride;
  GroupDesc d{};
  if (gsel < cnt) d = *reinterpret_cast<const GroupDesc*>(rb);
  group_bwd_body<S, C, ST>(d, seg, per_group, blk_elems, team, rb, vals, x,
                           smem_raw + 4 * per * stride, gdense != 0);
}

// ------------------------------------------------------------------------------------ root --
// y_r <- L_r^-T (L_r^-1 y_r), L_r^-1 packed column-major, read straight from global memory.
template <typename S, typename C>
__device__ __forceinline__ void root_body(int nr, const int32_t* __restrict__ ridx,
                                          const S* __restrict__ Lv, double* __restrict__ y,
                                          bool staged, unsigned char* smem_raw) {
  // staged: packed L^-1 copied into LDS first (tri(nr) rounded up to the vector width)
  C* Ls = reinterpret_cast<C*>(smem_raw);
  C* ys = Ls + (staged ? round_up((int)tri_count(nr), 8) : 0);
  C* ws = ys + nr;
  if (staged) stage_flat(Ls, Lv, (int)tri_count(nr), threadIdx.x, blockDim.x);
  const Tri<S, C, true> Lst{Ls, Lv, nr};
  const Tri<S, C, false> Lgl{Ls, Lv, nr};
  for (int i = threadIdx.x; i < nr; i += blockDim.x) ys[i] = (C)y[ridx[i]];
  __syncthreads();
  // `team` lanes share each output's dot product
  int team = 1;
  while (team < 16 && team * 2 * nr <= (int)blockDim.x) team <<= 1;
  const int part = threadIdx.x % team, per = blockDim.x / team;
  for (int ob = 0; ob < nr; ob += per) {   // w = L^-1 y
    const int o = ob + (int)threadIdx.x / team;
    C acc = 0;
    if (o < nr)
      acc = staged ? Lst.row_dot(o, part, team, [&](int j) { return ys[j]; })
                   : Lgl.row_dot(o, part, team, [&](int j) { return ys[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && o < nr) ws[o] = acc;
  }
  __syncthreads();
  for (int ob = 0; ob < nr; ob += per) {   // y = L^-T w (column o is contiguous)
    const int o = ob + (int)threadIdx.x / team;
    C acc = 0;
    if (o < nr)
      acc = staged ? Lst.col_dot(o, o + part, team, [&](int j) { return ws[j]; })
                   : Lgl.col_dot(o, o + part, team, [&](int j) { return ws[j]; });
    acc = team_sum(acc, team);
    if (part == 0 && o < nr) y[ridx[o]] = (double)acc;
  }
}

// LDS of the root stage: staged when the packed block fits next to the two vectors.
template <typename C>
size_t root_smem(int nr, bool* staged) {
  const size_t st = sizeof(C) * ((size_t)round_up((int)tri_count(nr), 8) + 2 * (size_t)nr);
  *staged = st <= kStageMax;
  return *staged ? st : 2 * sizeof(C) * (size_t)nr;
}

template <typename S, typename C>
__global__ __launch_bounds__(kRootThreads) void k_root(int nr, const int32_t* __restrict__ ridx,
                                                       const S* __restrict__ Lv,
                                                       double* __restrict__ y,
                                                       int staged,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  root_body<S, C>(nr, ridx, Lv, y, staged != 0, smem_raw);
}

// --------------------------------------------------------------------------- fused stages --
// The group stage of level l and the forward cell stage of level l+1 in one launch.  Workgroup
// p runs the level-l groups it owns (every group with a DOF in the interior of the level l+1
// cell p, plus a share of the groups on level l+1 cell boundaries) at once, `seg` lanes each,
// then the cell stage of cell p.  Cell p reads only its own interior, which only its own groups
// write; groups read only their own DOFs and the contributions of the level-l cells (the
// previous launch); so no workgroup needs another one's result.  The contributions of
// consecutive levels live in the two halves of the contribution buffer (cb_in: level l,
// cb_out: level l+1).  The owned groups' descriptors are stored padded to `maxown` per cell, so
// one load finds them.  With `prestage`, the cell's block is loaded into LDS (below `goff`)
// while the groups run.
template <typename S, typename C, bool CST>
__global__ __launch_bounds__(1024) void k_fuse_fwd(const int32_t* __restrict__ frec, int fstride,
                                                   int cstride, int gstride, int maxown, int seg,
                                                   int team_g, int per_group, int blk_g, int goff,
                                                   int blk_c, int team_c, int prestage,
                                                   const S* __restrict__ vals,
                                                   double* __restrict__ y,
                                                   const double* __restrict__ cb_in,
                                                   double* __restrict__ cb_out,
                                                   const int* __restrict__ done, int gdense) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the record of cell p, then those of the groups it owns (padded to maxown)
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  load_record(rec, frec + (int64_t)blockIdx.x * fstride, fstride, threadIdx.x, blockDim.x);
  const int dn = done ? *done : 0;
  __syncthreads();
  if (dn) return;
  unsigned char* work = smem_raw + 4 * fstride;
  const CellDesc d = *reinterpret_cast<const CellDesc*>(rec);
  const int gsel = threadIdx.x / seg;
  const int32_t* rb = rec + cstride + gsel * gstride;
  GroupDesc g{};
  if (gsel < maxown) g = *reinterpret_cast<const GroupDesc*>(rb);
  if constexpr (CST)
    if (prestage)
      stage_flat(reinterpret_cast<C*>(work), vals + d.offV, tri_count(d.nI) + d.nB * d.nI,
                 threadIdx.x, blockDim.x);
  group_fwd_body<S, C, true>(g, seg, per_group, blk_g, team_g, rb, vals, y, cb_in, work + goff,
                             gdense != 0);
  __syncthreads();
  cell_fwd_body<S, C, CST, 0>(d, rec, vals, y, cb_out, blk_c, team_c, prestage != 0, work);
}

// The last level's groups (forward), the root, and the same groups (backward) in one
// workgroup: the root is the only cell above them, so barriers order everything.  Groups run
// `per` at a time.
template <typename S, typename C>
__global__ __launch_bounds__(1024) void k_fuse_root(const GroupDesc* __restrict__ gd, int ngroup,
                                                    int seg, int team, int per, int per_group,
                                                    int blk_g,
                                                    int nr, const int32_t* __restrict__ ridx,
                                                    const S* __restrict__ Lv,
                                                    const int32_t* __restrict__ idx,
                                                    const S* __restrict__ vals,
                                                    double* __restrict__ y,
                                                    const double* __restrict__ cb_in,
                                                    int rstaged, const int* __restrict__ done,
                                                    int gdense) {
  const int gsel = threadIdx.x / seg;
  GroupDesc g{};
  if (gsel < per && gsel < ngroup) g = gd[gsel];
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  for (int b = 0; b < ngroup; b += per) {
    if (b > 0) {
      g = GroupDesc{};
      if (gsel < per && b + gsel < ngroup) g = gd[b + gsel];
    }
    group_fwd_body<S, C, true>(g, seg, per_group, blk_g, team, idx, vals, y, cb_in, smem_raw,
                               gdense != 0);
    __syncthreads();
  }
  root_body<S, C>(nr, ridx, Lv, y, rstaged != 0, smem_raw);
  __syncthreads();
  for (int b = 0; b < ngroup; b += per) {
    g = GroupDesc{};
    if (gsel < per && b + gsel < ngroup) g = gd[b + gsel];
    group_bwd_body<S, C, true>(g, seg, per_group, blk_g, team, idx, vals, y, smem_raw,
                               gdense != 0);
    __syncthreads();
  }
}

// -------------------------------------------------------------------------- tiled cells --
// Cells with a dense coupling H = A_BI A_II^-1 whose blocks do not fit one workgroup's LDS
// are spread over many workgroups (link-mode cells of that size use the dense form below).
// The forward sweep writes the new interior values into a scratch vector (not into y), so
// that every tile of a cell still reads the old y_I; the backward sweep reads them back from
// there and writes the final interior values into y.
//   row tiles:    64 consecutive rows of [L^-1; H] (packed columns are contiguous over rows,
//                 so each load of a wavefront is coalesced); the wavefronts of the workgroup
//                 split the columns and add up through LDS.
//   column tiles: 32 consecutive columns; each wavefront reduces whole columns (contiguous in
//                 memory).
constexpr int kRowTile = 64;
constexpr int kColTile = 32;
constexpr int kDotUnroll = 8;   // matrix loads in flight per lane in the dot products

// Workgroup b of a launch runs on XCD b % 8, and each XCD has its own L2.  Tile b' = xcd_tile(b)
// gives every XCD one contiguous run of the tile list, so neighbouring tiles of one block, which
// share the cache lines at their edges, are fetched into the same L2.
__device__ __forceinline__ int xcd_tile(int b, int g) {
  const int q = g >> 3, rem = g & 7, x = b & 7;
  return x * q + min(x, rem) + (b >> 3);
}

// sum of elem(j) x_j over j = j0, j0 + step, ... < j1, in that order, with up to U loads of
// the matrix in flight (the loads of U terms are issued before their products are added)
template <int U, typename C, typename F>
__device__ __forceinline__ C strided_dot(int j0, int j1, int step, F elem, const C* x) {
  C acc = 0;
  int j = j0;
  for (; j + (U - 1) * step < j1; j += U * step) {
    C e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) e[u] = elem(j + u * step);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += e[u] * x[j + u * step];
  }
  for (; j < j1; j += step) acc += elem(j) * x[j];
  return acc;
}

// Forward: w = L^-1 y_I -> scratch, c_B = H w -> cb.
template <typename S, typename C, int TT>
__global__ __launch_bounds__(TT) void k_tfwd_rows(const CellDesc* __restrict__ cd,
                                                   const int4* __restrict__ tiles,
                                                   const int32_t* __restrict__ idx,
                                                   const S* __restrict__ vals,
                                                   const double* __restrict__ y,
                                                   double* __restrict__ wsc,
                                                   double* __restrict__ cb,
                                                   const int* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* ys = reinterpret_cast<C*>(smem_raw);
  __shared__ C red[(TT / 64)][kRowTile];
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  if (done && *done) return;
  const CellDesc d = cd[t.x];
  const int nI = d.nI, nB = d.nB;
  const int nrows = nI + nB;
  const int r0 = t.y;
  const int32_t* gI = idx + d.offI;
  for (int j = threadIdx.x; j < nI; j += blockDim.x) ys[j] = (C)y[gI[j]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = r0 + lane;
  const S* v = vals + d.offV;
  const int tl = tri_count(nI);
  C acc = 0;
  if (r < nI) {
    acc = strided_dot<kDotUnroll>(
        wave, r + 1, (TT / 64), [&](int j) { return load_as<C>(v + colstart(j, nI) + (r - j)); },
        ys);
  } else if (r < nrows) {
    const S* H = v + tl + (r - nI);
    acc = strided_dot<kDotUnroll>(
        wave, nI, (TT / 64), [&](int j) { return load_as<C>(H + (int64_t)j * nB); }, ys);
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && r < nrows) {
    C tot = 0;
#pragma unroll
    for (int w = 0; w < (TT / 64); ++w) tot += red[w][lane];
    if (r < nI) wsc[t.z + r] = (double)tot;
    else cb[d.offCB + r - nI] = (double)tot;
  }
}

__device__ __forceinline__ double wave_reduce(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_reduce(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Backward: x_I = L^-T w - H^T x_B -> y, with w from the scratch vector.
template <typename S, typename C, int TT>
__global__ __launch_bounds__(TT) void k_tcols(const CellDesc* __restrict__ cd,
                                               const int4* __restrict__ tiles,
                                               const int32_t* __restrict__ idx,
                                               const S* __restrict__ vals,
                                               double* __restrict__ y,
                                               const double* __restrict__ wsc,
                                               const int* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* xs = reinterpret_cast<C*>(smem_raw);
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  if (done && *done) return;
  const CellDesc d = cd[t.x];
  const int nI = d.nI, nB = d.nB;
  C* xb = xs + nI;
  const int c0 = t.y;
  for (int j = c0 + (int)threadIdx.x; j < nI; j += blockDim.x) xs[j] = (C)wsc[t.z + j];
  for (int b = threadIdx.x; b < nB; b += blockDim.x) xb[b] = (C)y[idx[d.offB + b]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const S* v = vals + d.offV;
  const int tl = tri_count(nI);
  for (int q = wave; q < kColTile; q += (TT / 64)) {
    const int i = c0 + q;
    if (i >= nI) break;
    const S* col = v + colstart(i, nI);
    C acc = strided_dot<kDotUnroll>(
        i + lane, nI, 64, [&](int j) { return load_as<C>(col + (j - i)); }, xs);
    const S* hc = v + tl + (int64_t)i * nB;
    acc -= strided_dot<kDotUnroll>(lane, nB, 64, [&](int b) { return load_as<C>(hc + b); }, xb);
    acc = wave_reduce(acc);
    if (lane == 0) y[idx[d.offI + i]] = (double)acc;
  }
}

// --------------------------------------------------------------------------- dense forms --
// Blocks in dense form (column-major, leading dimension ld = n rounded up to 32 elements) are
// applied in one pass over many workgroups:
//   row tiles:    64 rows; the wavefronts split the columns of the tile's column range
//                 [c0, c0 + span) and add up through LDS.  Every 64-row segment of a column is
//                 whole, aligned cache lines.
//   column tiles: consecutive columns, each reduced by one wavefront over its whole length.
// Tile: (block, first row or column, first column of the range, scratch offset).
//   DR_CELL_FWD   cell interior in link mode: v = A_II^-1 y_I; the couplings of the tile's rows
//                 go to cb, y_I is kept in the scratch vector for the backward sweep (the
//                 level's interiors are not touched in between)
//   DR_CELL_BWD   x_I = A_II^-1 (y_I - A_IB x_B) -> y
//   DR_GROUP_FWD  the group step G (y_g less the cell contributions) -> scratch
//   DR_ROOT       partial sums of A_r^-1 y_r over one column range -> scratch
//   column tiles: the backward group step G^T x_g -> scratch
// Dense group and root results go back to y by a scatter list once every tile has read its
// inputs.  (The dense top has a kernel of its own, k_top_rows.)
enum { DR_CELL_FWD = 0, DR_CELL_BWD, DR_GROUP_FWD, DR_ROOT };
constexpr int kDenseColsPerTile = 32;

__host__ __device__ inline int dense_ld(int n) { return (n + 31) & ~31; }

template <typename S, typename C, int KIND, int TT>
__global__ __launch_bounds__(TT) void k_dense_rows(const CellDesc* __restrict__ cd,
                                                   const GroupDesc* __restrict__ gd,
                                                   const int64_t* __restrict__ ddoff,
                                                   const int4* __restrict__ tiles, int span,
                                                   int nroot, const int32_t* __restrict__ ridx,
                                                   const int32_t* __restrict__ idx,
                                                   const S* __restrict__ vals,
                                                   const S* __restrict__ dv,
                                                   double* __restrict__ y,
                                                   double* __restrict__ cb,
                                                   double* __restrict__ wsc,
                                                   const int* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* xs = reinterpret_cast<C*>(smem_raw);
  __shared__ C red[TT / 64][kRowTile];
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  if (done && *done) return;
  int n;
  CellDesc c{};
  GroupDesc g{};
  if constexpr (KIND == DR_CELL_FWD || KIND == DR_CELL_BWD) {
    c = cd[t.x];
    n = c.nI;
  } else if constexpr (KIND == DR_GROUP_FWD) {
    g = gd[t.x];
    n = g.n;
  } else {
    n = nroot;
  }
  const int r0 = t.y, c0 = t.z;
  const int c1 = min(n, c0 + span);
  const S* M = dv + ddoff[t.x];
  const int ld = dense_ld(n);
  double* w = wsc + t.w;
  // the inputs of the tile's column range
  if constexpr (KIND == DR_CELL_FWD) {
    const int32_t* gI = idx + c.offI;
    for (int j = c0 + (int)threadIdx.x; j < c1; j += TT) xs[j - c0] = (C)y[gI[j]];
  } else if constexpr (KIND == DR_CELL_BWD) {
    // idx layout after offC: ib[nB], rowptr[nI + 1], blist[nB] (links grouped by interior DOF)
    const int32_t* rp = idx + c.offC + c.nB;
    const int32_t* bl = rp + n + 1;
    const int32_t* gB = idx + c.offB;
    const S* cw = vals + c.offV + tri_count(n);
    for (int j = c0 + (int)threadIdx.x; j < c1; j += TT) {
      C tj = 0;
      for (int q = rp[j]; q < rp[j + 1]; ++q) {
        const int b = bl[q];
        tj += load_as<C>(cw + b) * (C)y[gB[b]];
      }
      xs[j - c0] = (C)w[j] - tj;
    }
  } else if constexpr (KIND == DR_GROUP_FWD) {
    const int32_t* gi = idx + g.offIdx;
    const int32_t* gp = idx + g.offGP;
    const int32_t* slots = gp + n + 1;
    for (int j = c0 + (int)threadIdx.x; j < c1; j += TT) {
      double a = y[gi[j]];
      for (int q = gp[j]; q < gp[j + 1]; ++q) a -= cb[slots[q]];
      xs[j - c0] = (C)a;
    }
  } else {
    for (int j = c0 + (int)threadIdx.x; j < c1; j += TT) xs[j - c0] = (C)y[ridx[j]];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = r0 + lane;
  C acc = 0;
  if (r < n) {
    const S* col = M + r;
    acc = strided_dot<kDotUnroll>(
        wave, c1 - c0, TT / 64, [&](int j) { return load_as<C>(col + (int64_t)(c0 + j) * ld); },
        xs);
  }
  red[wave][lane] = acc;
  __syncthreads();
  if constexpr (KIND == DR_CELL_FWD) {
    __shared__ C vt[kRowTile];
    if (wave == 0 && r < n) {
      C tot = 0;
#pragma unroll
      for (int q = 0; q < TT / 64; ++q) tot += red[q][lane];
      vt[lane] = tot;
      w[r] = y[idx[c.offI + r]];
    }
    __syncthreads();
    const int32_t* ib = idx + c.offC;
    const S* cw = vals + c.offV + tri_count(n);
    for (int b = threadIdx.x; b < c.nB; b += TT) {
      const int i = ib[b];
      if (i >= r0 && i < r0 + kRowTile) cb[c.offCB + b] = (double)(load_as<C>(cw + b) * vt[i - r0]);
    }
  } else {
    if (wave == 0 && r < n) {
      C tot = 0;
#pragma unroll
      for (int q = 0; q < TT / 64; ++q) tot += red[q][lane];
      if constexpr (KIND == DR_CELL_BWD) y[idx[c.offI + r]] = (double)tot;
      else w[r] = (double)tot;
    }
  }
}

// Backward group step: x_g <- G^T x_g, column c of G (contiguous) by one wavefront.
template <typename S, typename C, int TT>
__global__ __launch_bounds__(TT) void k_dense_gcols(const GroupDesc* __restrict__ gd,
                                                    const int64_t* __restrict__ ddoff,
                                                    const int4* __restrict__ tiles,
                                                    const int32_t* __restrict__ idx,
                                                    const S* __restrict__ dv,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ wsc,
                                                    const int* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* xs = reinterpret_cast<C*>(smem_raw);
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  if (done && *done) return;
  const GroupDesc g = gd[t.x];
  const int n = g.n, ld = dense_ld(n);
  const int32_t* gi = idx + g.offIdx;
  for (int j = threadIdx.x; j < n; j += TT) xs[j] = (C)y[gi[j]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const S* M = dv + ddoff[t.x];
  for (int q = wave; q < kDenseColsPerTile; q += TT / 64) {
    const int i = t.y + q;
    if (i >= n) break;
    const S* col = M + (int64_t)i * ld;
    C acc = strided_dot<kDotUnroll>(lane, n, 64, [&](int j) { return load_as<C>(col + j); }, xs);
    acc = wave_reduce(acc);
    if (lane == 0) wsc[t.w + i] = (double)acc;
  }
}

// y[id] = sum over p < parts of wsc[src + p * stride], entries (id, src, parts, stride).
__global__ __launch_bounds__(256) void k_dense_scatter(const int4* __restrict__ e, int count,
                                                       const double* __restrict__ wsc,
                                                       double* __restrict__ y,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const int4 q = e[i];
    double a = 0;
    for (int p = 0; p < q.z; ++p) a += wsc[q.y + (int64_t)p * q.w];
    y[q.x] = a;
  }
}

// Dense top: the partial sums w[chunk][r] = sum over the chunk's columns c of M_k[r, c]
// (y_k - c_k)[c].  One workgroup per (row tile, column chunk), chunk-major; each lane covers
// VecOf<S>::W consecutive rows, read as one 16-byte vector per column (M_k is column-major), so
// a wave streams 1 KiB per load; the waves split the chunk's columns (wave w takes w, w + NW,
// ...).  The first U vectors of every lane are loaded before the inputs are gathered and the
// early-exit flag is looked at, so their latencies overlap.  Same summation order as the
// 64-row form of k_dense_rows.
constexpr int kTopThreads = 1024;
constexpr int kTopUnroll = 16;

template <typename S, typename C>
__global__ __launch_bounds__(kTopThreads) void k_top_rows(int nrt, int span, int n, int ld,
                                                          const int32_t* __restrict__ ridx,
                                                          int kslot,
                                                          const int32_t* __restrict__ gslot,
                                                          const S* __restrict__ M,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ cb,
                                                          double* __restrict__ wsc,
                                                          const int* __restrict__ done) {
  using V = typename VecOf<S>::T;
  constexpr int W = VecOf<S>::W, RT = 64 * W, NW = kTopThreads / 64, U = kTopUnroll;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* xs = reinterpret_cast<C*>(smem_raw);
  __shared__ C red[NW][RT];
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int ch = b / nrt, r0 = (b - ch * nrt) * RT, c0 = ch * span;
  const int nc = min(n, c0 + span) - c0;
  const int dn = done ? *done : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // lanes past the column read its last vector (ld is a multiple of W; their sums are dropped),
  // and columns past the chunk read its last column with a zero input: no branch separates the
  // loads of a batch from their use
  const int rl = min(r0 + lane * W, ld - W);
  const int64_t ldv = ld / W;
  const V* col = reinterpret_cast<const V*>(M + rl) + (int64_t)c0 * ldv;
  V v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = col[(int64_t)min(wave + u * NW, nc - 1) * ldv];
  // inputs: y less the contributions of level k's cells (kslot slots per DOF, -1 = none)
  for (int j = threadIdx.x; j < nc; j += kTopThreads) {
    const int32_t* sl = gslot + (int64_t)(c0 + j) * kslot;
    double s = y[ridx[c0 + j]];
    for (int q = 0; q < kslot; ++q)
      if (sl[q] >= 0) s -= cb[sl[q]];
    xs[j] = (C)s;
  }
  if (dn) return;  // (uniform)
  __syncthreads();
  C acc[W];
#pragma unroll
  for (int e = 0; e < W; ++e) acc[e] = 0;
  for (int j = wave; j < nc; j += U * NW) {
    if (j > wave) {  // the next batch (the first one is in flight already)
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = col[(int64_t)min(j + u * NW, nc - 1) * ldv];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      C e[W];
      unpack<C>(v[u], e);
      const C x = j + u * NW < nc ? xs[j + u * NW] : (C)0;
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += e[k] * x;
    }
  }
#pragma unroll
  for (int e = 0; e < W; ++e) red[wave][lane * W + e] = acc[e];
  __syncthreads();
  for (int q = threadIdx.x; q < RT; q += kTopThreads) {
    if (r0 + q >= n) continue;
    C tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += red[w][q];
    wsc[(int64_t)ch * n + r0 + q] = (double)tot;
  }
}

// --------------------------------------------------------------------------- launch plans --
struct StagePlan {
  bool staged;
  size_t rec;     // bytes of the block records at the front of LDS
  int threads;
  int seg;        // lanes per group (group stages)
  int per;        // groups per workgroup
  int blk_elems;  // LDS elements reserved for one block
  int per_group;  // LDS elements per group (blocks + vectors)
  size_t smem;    // bytes
  int grid;
  int team;       // lanes sharing one column walk (group stages)
};

// Cells: one workgroup each.  Few, large cells (upper levels) get 256 lanes and may use most of
// the LDS; many small cells (level 0) keep the footprint small so that many stay resident.
template <typename C>
StagePlan cell_plan(const LevelDev& L) {
  StagePlan p{};
  if (L.cmode == 2) {  // symmetric-inverse cells: one wavefront each, the square in LDS
    p.staged = true;
    p.threads = 64;
    p.seg = 1;
    p.blk_elems = 0;
    p.rec = 4 * (size_t)L.cstride;
    p.smem = sizeof(C) * (size_t)sym_smem_elems(L.sqmat, L.maxB);
    p.grid = L.ncell;
    return p;
  }
  p.blk_elems = round_up(L.maxCV, 8);
  const size_t vec = 3 * (size_t)L.maxI + 2 * (size_t)L.maxB + 4;
  const size_t budget = L.ncell >= 2048 ? kStageBudget : kStageMax;
  p.staged = sizeof(C) * (p.blk_elems + vec) <= budget;
  const int outs = L.maxI + L.maxB;
  // many cells (2048 or more): one wave each keeps the most cells in flight (measured on 1024^2:
  // 128 or 256 lanes are 3-15% slower); fewer cells: 256 lanes split the dot products further
  // (256^2: 0.3-0.5 us per launch faster than 128)
  p.threads = (L.ncell >= 2048 || outs <= 64) ? 64 : 256;
  // lanes per output: spread the dot products over the workgroup
  int team = 1;
  while (team < 8 && (team * 2) * L.maxI <= p.threads) team <<= 1;
  p.seg = team;
  if (!p.staged) p.blk_elems = 0;
  p.rec = 4 * (size_t)L.cstride;
  p.smem = sizeof(C) * (p.blk_elems + vec);
  p.grid = L.ncell;
  return p;
}

template <typename C>
StagePlan group_plan(const LevelDev& L) {
  StagePlan p{};
  int seg = 8;
  while (seg < L.maxG && seg < 256) seg <<= 1;
  // lanes per output of the staged form: two where the level has few groups (measured side by
  // side: +1% CN steps/s on 256^2 and 64^3; on 1024^2, with 32K level-0 groups, one lane is best)
  int team = L.ngroup < 4096 ? 2 : 1;
  while (team > 1 && seg * team > 256) team >>= 1;
  p.seg = seg * team;
  p.threads = std::max(p.seg, 64);
  p.per = p.threads / p.seg;
  p.blk_elems = round_up(L.maxGV, 8);
  const int vec = round_up(2 * L.maxG + 2 * L.maxR, 4);
  p.per_group = p.blk_elems + vec;
  p.staged = sizeof(C) * (size_t)p.per * p.per_group <= kStageBudget;
  if (!p.staged) {  // global-memory blocks: one group per workgroup, vectors only in LDS
    p.seg = p.threads = L.maxG <= 64 ? 64 : (L.maxG <= 128 ? 128 : 256);
    p.per = 1;
    p.per_group = vec;
    p.blk_elems = 0;
  }
  p.rec = 4 * (size_t)p.per * L.gstride;
  p.smem = sizeof(C) * (size_t)p.per * p.per_group;
  p.grid = (L.ngroup + p.per - 1) / p.per;
  // column walks: lanes of one group read a column together when it is in global memory
  p.team = p.staged ? team : 64;
  return p;
}

// Fused launches: the owned groups all run at once (the block size is the smallest of 256, 512
// and 1024 lanes that holds them; a level whose cells own more is not fused), then the cell
// (team re-derived for that block size); or, for the root, groups `per` at a time.
struct FusePlan {
  bool ok = false;
  int team_g = 1;  // lanes per output in the group stage (segments of g.seg x team_g lanes)
  size_t rec = 0;  // bytes of the record (cell + owned groups) at the front of LDS
  int threads = 256, per = 0, team_c = 1, goff = 0;
  bool cst = false, prestage = false;
  int blk_c = 0;
  size_t smem = 0;
  StagePlan g{};
};

template <typename C>
FusePlan fuse_plan(const LevelDev& G, const LevelDev* Cl, int nroot) {
  FusePlan f;
  if (!G.ngroup) return f;
  f.g = group_plan<C>(G);
  if (!f.g.staged) return f;
  f.g.seg /= f.g.team;  // (fused launches set their own lanes per output)
  f.g.team = 1;
  const size_t pg = sizeof(C) * (size_t)f.g.per_group;
  if (Cl) {
    if (!Cl->ncell || Cl->tiled || Cl->cmode != 0 || G.maxown < 1) return f;
    // lanes per group output: four when the next level's cells fit in one round of workgroups
    // (measured side by side: +1.1% CN steps/s on 256^2), one otherwise (1024^2: four on every
    // level is 11% slower); HIFCN_FUSE_TEAM overrides
    f.team_g = Cl->ncell <= 256 ? 4 : 1;
    if (const char* e = std::getenv("HIFCN_FUSE_TEAM")) f.team_g = std::max(1, std::atoi(e));
    while (f.team_g > 1 && f.g.seg * f.team_g * G.maxown > 1024) f.team_g >>= 1;
    const int gl = f.g.seg * f.team_g;  // lanes per group
    f.threads = 256;
    while (f.threads < 1024 && f.threads / gl < G.maxown) f.threads *= 2;
    if (f.threads / gl < G.maxown) return f;
    f.per = G.maxown;
    const size_t gsm = (size_t)f.per * pg;
    const StagePlan cp = cell_plan<C>(*Cl);
    int team = 1;
    while (team < 8 && (team * 2) * Cl->maxI <= f.threads) team <<= 1;
    f.team_c = team;
    f.cst = cp.staged;
    f.blk_c = cp.blk_elems;
    const size_t csm = (cp.smem + 15) / 16 * 16;
    f.rec = 4 * (size_t)G.fstride;
    f.prestage = f.cst && f.rec + csm + gsm <= kStageMax;
    f.goff = f.prestage ? (int)csm : 0;
    f.smem = f.prestage ? csm + gsm : std::max(gsm, cp.smem);
  } else {
    f.threads = 1024;
    f.per = (int)std::min<size_t>(f.threads / f.g.seg, std::max<size_t>(1, kStageMax / pg));
    f.per = std::min(f.per, G.ngroup);
    // spare lanes share each group's products: `team_g` lanes per output
    while (f.team_g < 8 && (size_t)f.per * f.g.seg * f.team_g * 2 <= (size_t)f.threads)
      f.team_g *= 2;
    bool rs;
    const size_t rsm = root_smem<C>(nroot, &rs);
    f.prestage = rs;  // the root block is staged in LDS
    f.smem = std::max((size_t)f.per * pg, rsm);
  }
  f.ok = f.rec + f.smem <= kStageMax;
  return f;
}

// Optional timing of the launches of one (level, stage): the kernel is launched with a start
// and a stop event that the runtime records around its execution on the same stream.
// A tiny follow-up kernel records whether the timed launch did work (the early-exit flag cannot
// change during an apply), so that launches that returned at once are left out of the average.
__global__ void k_record_live(const int* __restrict__ done, int32_t* __restrict__ live) {
  if (threadIdx.x == 0) *live = (done && *done) ? 0 : 1;
}

struct StageTimer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  StageProfiler* p = nullptr;
  const int* done;
  hipStream_t s;
  StageTimer() : done(nullptr), s(nullptr) {}
  StageTimer(StageProfiler* prof, int level, int stage, const int* dn, hipStream_t st)
      : done(dn), s(st) {
    if (prof && prof->enabled && prof->level == level && prof->stage == stage) {
      p = prof;
      e0 = p->next_event();
      e1 = p->next_event();
      p->pending.push_back({e0, e1});
      if (p->live.n < p->pending.size()) {  // grow (only between timed runs in practice)
        HIF_CHECK(hipStreamSynchronize(s));
        DevBuf<int32_t> nl(std::max<size_t>(256, 2 * p->pending.size()));
        if (p->live.n)
          HIF_CHECK(hipMemcpy(nl.p, p->live.p, p->live.n * sizeof(int32_t),
                              hipMemcpyDeviceToDevice));
        p->live = std::move(nl);
      }
    }
  }
  ~StageTimer() {
    if (p)
      hipLaunchKernelGGL(k_record_live, dim3(1), dim3(64), 0, s, done,
                         p->live.p + (p->pending.size() - 1));
  }
};

// A stage of several launches: its start event goes with the first, its stop event with the
// last.
struct TimedSeq {
  const StageTimer& t;
  int n, i = 0;
  TimedSeq(const StageTimer& st, int count) : t(st), n(count) {}
  StageTimer next() {
    StageTimer x;
    if (i == 0) x.e0 = t.e0;
    if (i == n - 1) x.e1 = t.e1;
    ++i;
    return x;
  }
};

template <typename K, typename... Args>
void launch(K kernel, dim3 grid, dim3 block, size_t smem, hipStream_t s, const StageTimer& t,
            Args... args) {
  if (t.e0 || t.e1)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)smem, s, t.e0, t.e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, smem, s, args...);
}

SymCfg sym_cfg(const FactorDev& f, const LevelDev& L) {
  return SymCfg{f.sqtab.p, L.sqn, L.sqld, L.sqmat, L.sqoff};
}

template <typename S, typename C, int MODE>
void launch_cell(const FactorDev& f, const LevelDev& L, bool fwd, const S* vals, double* y,
                 double* cb, const int* done, hipStream_t s, const StageTimer& t,
                 const CgGate* gate = nullptr, const CgRhs* rhs = nullptr) {
  const StagePlan p = cell_plan<C>(L);
  if (t.p) t.p->kernel = fwd ? "k_cell_fwd" : "k_cell_bwd";
  // symmetric cells keep their record out of LDS, except where the first stage makes the
  // right-hand side
  const size_t lds = p.smem + (MODE == 2 && !(fwd && rhs) ? 0 : p.rec);
  if (fwd) {
    auto k = p.staged ? k_cell_fwd<S, C, true, MODE> : k_cell_fwd<S, C, false, MODE>;
    launch(k, dim3(p.grid), dim3(p.threads), lds, s, t, (const int32_t*)L.crec.p,
           L.cstride, vals, y, cb, done, p.blk_elems, p.seg, gate ? *gate : CgGate{},
           (gate || rhs) ? (const int32_t*)f.gcopy.p : (const int32_t*)nullptr, f.gcstride,
           rhs ? *rhs : CgRhs{}, sym_cfg(f, L), L.cfwd);
  } else {
    auto k = p.staged ? k_cell_bwd<S, C, true, MODE> : k_cell_bwd<S, C, false, MODE>;
    const bool fold = &L == &f.lv[std::max(0, f.top)] && f.top >= 0 && f.tfold;
    launch(k, dim3(p.grid), dim3(p.threads), lds, s, t, (const int32_t*)L.crec.p,
           L.cstride, vals, y, done, p.blk_elems, p.seg,
           fold ? (const int32_t*)f.tpos.p : (const int32_t*)nullptr, f.tpstride,
           (const double*)f.twsc.p, (f.ntop + f.tspan - 1) / std::max(1, f.tspan), f.ntop,
           sym_cfg(f, L));
  }
}

// One sweep of a tiled level (dense H): row tiles forward, column tiles backward.
template <typename S, typename C, int TT>
void launch_tiled_tt(const FactorDev& f, const LevelDev& L, bool fwd, const S* vals, double* y,
                     double* cb, const int* done, hipStream_t s, const StageTimer& t) {
  const int32_t* idx = f.idx.p;
  if (fwd)
    launch(k_tfwd_rows<S, C, TT>, dim3(L.nrt), dim3(TT), sizeof(C) * (size_t)std::max(1, L.maxI),
           s, t, (const CellDesc*)L.cells.p, (const int4*)L.rtiles.p, idx, vals,
           (const double*)y, f.wsc.p, cb, done);
  else
    launch(k_tcols<S, C, TT>, dim3(L.nct), dim3(TT),
           sizeof(C) * (size_t)std::max(1, L.maxI + L.maxB), s, t, (const CellDesc*)L.cells.p,
           (const int4*)L.ctiles.p, idx, vals, y, (const double*)f.wsc.p, done);
}

template <typename S, typename C>
void launch_tiled(const FactorDev& f, const LevelDev& L, bool fwd, const S* vals, double* y,
                  double* cb, const int* done, hipStream_t s, const StageTimer& t) {
  switch (L.tthreads) {
    case 256: launch_tiled_tt<S, C, 256>(f, L, fwd, vals, y, cb, done, s, t); break;
    case 512: launch_tiled_tt<S, C, 512>(f, L, fwd, vals, y, cb, done, s, t); break;
    default: launch_tiled_tt<S, C, 1024>(f, L, fwd, vals, y, cb, done, s, t); break;
  }
}

constexpr int kDenseSpanAll = 1 << 30;   // row tiles over all columns of their block

template <typename S, typename C, int TT>
void launch_dense_cells_tt(const FactorDev& f, const LevelDev& L, bool fwd, const S* vals,
                           double* y, double* cb, const int* done, hipStream_t s,
                           const StageTimer& t) {
  const size_t sm = sizeof(C) * (size_t)std::max(1, L.maxI);
  auto k = fwd ? k_dense_rows<S, C, DR_CELL_FWD, TT> : k_dense_rows<S, C, DR_CELL_BWD, TT>;
  launch(k, dim3(L.ncdt), dim3(TT), sm, s, t, (const CellDesc*)L.cells.p,
         (const GroupDesc*)nullptr, (const int64_t*)L.cddoff.p, (const int4*)L.cdtiles.p,
         kDenseSpanAll, 0, (const int32_t*)nullptr, (const int32_t*)f.idx.p, vals,
         reinterpret_cast<const S*>(f.dvals.p), y, cb, f.wsc.p, done);
}

template <typename S, typename C>
void launch_dense_cells(const FactorDev& f, const LevelDev& L, bool fwd, const S* vals,
                        double* y, double* cb, const int* done, hipStream_t s,
                        const StageTimer& t) {
  switch (L.tthreads) {
    case 256: launch_dense_cells_tt<S, C, 256>(f, L, fwd, vals, y, cb, done, s, t); break;
    case 512: launch_dense_cells_tt<S, C, 512>(f, L, fwd, vals, y, cb, done, s, t); break;
    default: launch_dense_cells_tt<S, C, 1024>(f, L, fwd, vals, y, cb, done, s, t); break;
  }
}

constexpr int kDenseThreads = 512;

void launch_scatter(const DevBuf<int4>& e, int count, const FactorDev& f, double* y,
                    const int* done, hipStream_t s, const StageTimer& t) {
  const int grid = std::max(1, std::min(1024, (count + 255) / 256));
  launch(k_dense_scatter, dim3(grid), dim3(256), 0, s, t, (const int4*)e.p, count,
         (const double*)f.wsc.p, y, done);
}

template <typename S, typename C>
void launch_dense_groups(const FactorDev& f, const LevelDev& L, bool fwd, double* y,
                         const double* cb, const int* done, hipStream_t s, const StageTimer& t) {
  TimedSeq ts(t, 2);
  const size_t sm = sizeof(C) * (size_t)std::max(1, L.maxG);
  const S* dv = reinterpret_cast<const S*>(f.dvals.p);
  if (fwd)
    launch(k_dense_rows<S, C, DR_GROUP_FWD, kDenseThreads>, dim3(L.ngrt), dim3(kDenseThreads),
           sm, s, ts.next(), (const CellDesc*)nullptr, (const GroupDesc*)L.groups.p,
           (const int64_t*)L.gddoff.p, (const int4*)L.grtiles.p, kDenseSpanAll, 0,
           (const int32_t*)nullptr, (const int32_t*)f.idx.p, (const S*)nullptr, dv, y,
           const_cast<double*>(cb), f.wsc.p, done);
  else
    launch(k_dense_gcols<S, C, kDenseThreads>, dim3(L.ngct), dim3(kDenseThreads), sm, s,
           ts.next(), (const GroupDesc*)L.groups.p, (const int64_t*)L.gddoff.p,
           (const int4*)L.gctiles.p, (const int32_t*)f.idx.p, dv, (const double*)y, f.wsc.p,
           done);
  launch_scatter(L.gscat, L.ngsc, f, y, done, s, ts.next());
}

template <typename S, typename C>
void launch_dense_root(const FactorDev& f, double* y, const int* done, hipStream_t s,
                       const StageTimer& t) {
  TimedSeq ts(t, 2);
  const size_t sm = sizeof(C) * (size_t)std::max(1, std::min(f.nroot, f.rspan));
  launch(k_dense_rows<S, C, DR_ROOT, kDenseThreads>, dim3(f.nrdt), dim3(kDenseThreads), sm, s,
         ts.next(), (const CellDesc*)nullptr, (const GroupDesc*)nullptr,
         (const int64_t*)f.rddoff.p, (const int4*)f.rdtiles.p, f.rspan, f.nroot,
         (const int32_t*)f.idx.p + f.offRootIdx, (const int32_t*)f.idx.p, (const S*)nullptr,
         reinterpret_cast<const S*>(f.dvals.p), y, (double*)nullptr, f.wsc.p, done);
  launch_scatter(f.rscat, f.nrsc, f, y, done, s, ts.next());
}

template <typename S, typename C>
void launch_dense_top(const FactorDev& f, double* y, const double* cb, const int* done,
                      hipStream_t s, const StageTimer& t) {
  TimedSeq ts(t, f.tfold ? 1 : 2);
  const size_t sm = sizeof(C) * (size_t)std::max(1, std::min(f.ntop, f.tspan));
  const int nrt = (f.ntop + 64 * VecOf<S>::W - 1) / (64 * VecOf<S>::W);
  launch(k_top_rows<S, C>, dim3(f.ntdt), dim3(kTopThreads), sm, s, ts.next(), nrt, f.tspan,
         f.ntop, (f.ntop + 31) & ~31, (const int32_t*)f.tgid.p, f.tkslot,
         (const int32_t*)f.tgslot.p,
         reinterpret_cast<const S*>(f.tvals.p), (const double*)y, cb, f.twsc.p, done);
  if (f.tfold) return;  // the backward cell stage of the level reads the partial sums
  const int grid = std::max(1, std::min(1024, (f.ntsc + 255) / 256));
  launch(k_dense_scatter, dim3(grid), dim3(256), 0, s, ts.next(), (const int4*)f.tscat.p, f.ntsc,
         (const double*)f.twsc.p, y, done);
}

template <typename S, typename C>
void apply_impl(const FactorDev& f, double* y, const int* done, hipStream_t s,
                const CgGate* gate = nullptr, const CgRhs* rhs = nullptr) {
  const S* vals = reinterpret_cast<const S*>(f.vals.p);
  const int32_t* idx = f.idx.p;
  StageProfiler* prof = f.prof.get();
  const int nlev = (int)f.lv.size();
  auto cbl = [&](int l) { return f.cb.p + (int64_t)(l & 1) * f.cbstride; };
  for (int l = 0; l < nlev; ++l) {
    const LevelDev& L = f.lv[l];
    if (L.ncell && !(l > 0 && f.lv[l - 1].fuse)) {
      const StageTimer t(prof, l, STAGE_CELL_FWD, done, s);
      if (L.cdense) launch_dense_cells<S, C>(f, L, true, vals, y, cbl(l), done, s, t);
      else if (L.tiled) launch_tiled<S, C>(f, L, true, vals, y, cbl(l), done, s, t);
      else if (L.cmode == 2) launch_cell<S, C, 2>(f, L, true, vals, y, cbl(l), done, s, t,
                                                  l == 0 ? gate : nullptr, l == 0 ? rhs : nullptr);
      else if (L.cmode) launch_cell<S, C, 1>(f, L, true, vals, y, cbl(l), done, s, t,
                                             l == 0 ? gate : nullptr, l == 0 ? rhs : nullptr);
      else launch_cell<S, C, 0>(f, L, true, vals, y, cbl(l), done, s, t, l == 0 ? gate : nullptr,
                                l == 0 ? rhs : nullptr);
    }
    if (!L.ngroup) continue;
    if (l == f.top) {  // this level's groups, every level above and the root: one matrix
      const StageTimer t(prof, nlev, STAGE_ROOT, done, s);
      launch_dense_top<S, C>(f, y, cbl(l), done, s, t);
      break;
    }
    if (L.fuse) {  // + the cell stage of level l+1
      const LevelDev& P = f.lv[l + 1];
      const FusePlan fp = fuse_plan<C>(L, &P, 0);
      const StageTimer t(prof, l, STAGE_GROUP_FWD, done, s);
      auto k = fp.cst ? k_fuse_fwd<S, C, true> : k_fuse_fwd<S, C, false>;
      launch(k, dim3(P.ncell), dim3(fp.threads), fp.rec + fp.smem, s, t,
             (const int32_t*)L.frec.p, L.fstride, P.cstride, L.gstride, L.maxown,
             fp.g.seg * fp.team_g, fp.team_g, fp.g.per_group, fp.g.blk_elems, fp.goff, fp.blk_c,
             fp.team_c, (int)fp.prestage, vals, y, (const double*)cbl(l), cbl(l + 1), done,
             L.gdense);
    } else if (l == nlev - 1 && f.root_fused) {  // + root + this level's backward groups
      const FusePlan fp = fuse_plan<C>(L, nullptr, f.nroot);
      const StageTimer t(prof, nlev, STAGE_ROOT, done, s);
      launch(k_fuse_root<S, C>, dim3(1), dim3(fp.threads), fp.smem, s, t,
             (const GroupDesc*)L.groups.p, L.ngroup, fp.g.seg * fp.team_g, fp.team_g, fp.per,
             fp.g.per_group,
             fp.g.blk_elems, f.nroot, idx + f.offRootIdx, vals + f.offRootV, idx, vals, y,
             (const double*)cbl(l), (int)fp.prestage, done, L.gdense);
    } else if (L.gtiled) {
      const StageTimer t(prof, l, STAGE_GROUP_FWD, done, s);
      launch_dense_groups<S, C>(f, L, true, y, cbl(l), done, s, t);
    } else {
      const StageTimer t(prof, l, STAGE_GROUP_FWD, done, s);
      const StagePlan p = group_plan<C>(L);
      launch(k_group_fwd<S, C, true>, dim3(p.grid), dim3(p.threads), p.rec + p.smem, s, t,
             (const int32_t*)L.grec.p, L.gstride, L.ngroup, p.seg, p.per_group, p.blk_elems,
             p.team, vals, y, (const double*)cbl(l), done, L.gdense);
    }
  }
  if (f.nroot && !f.root_fused && f.top < 0) {
    const StageTimer t(prof, nlev, STAGE_ROOT, done, s);
    if (f.root_tiled) {
      launch_dense_root<S, C>(f, y, done, s, t);
    } else {
      bool rs;
      const size_t rsm = root_smem<C>(f.nroot, &rs);
      launch(k_root<S, C>, dim3(1), dim3(kRootThreads), rsm, s, t, f.nroot, idx + f.offRootIdx,
             vals + f.offRootV, y, (int)rs, done);
    }
  }
  for (int l = f.top >= 0 ? f.top : nlev - 1; l >= 0; --l) {
    const LevelDev& L = f.lv[l];
    if (L.ngroup && l != f.top && !(l == nlev - 1 && f.root_fused)) {
      const StageTimer t(prof, l, STAGE_GROUP_BWD, done, s);
      if (L.gtiled) {
        launch_dense_groups<S, C>(f, L, false, y, cbl(l), done, s, t);
      } else {
        const StagePlan p = group_plan<C>(L);
        launch(k_group_bwd<S, C, true>, dim3(p.grid), dim3(p.threads), p.rec + p.smem, s, t,
               (const int32_t*)L.grec.p, L.gstride, L.ngroup, p.seg, p.per_group, p.blk_elems,
               p.team, vals, y, done, L.gdense);
      }
    }
    if (L.ncell) {
      const StageTimer t(prof, l, STAGE_CELL_BWD, done, s);
      if (L.cdense) launch_dense_cells<S, C>(f, L, false, vals, y, cbl(l), done, s, t);
      else if (L.tiled) launch_tiled<S, C>(f, L, false, vals, y, cbl(l), done, s, t);
      else if (L.cmode == 2) launch_cell<S, C, 2>(f, L, false, vals, y, cbl(l), done, s, t);
      else if (L.cmode) launch_cell<S, C, 1>(f, L, false, vals, y, cbl(l), done, s, t);
      else launch_cell<S, C, 0>(f, L, false, vals, y, cbl(l), done, s, t);
    }
  }
  HIF_CHECK(hipGetLastError());
}


// ------------------------------------------------------------------- batched stage launches --
// Continuous batching: one launch runs a stage of several independent solves.  Every solve's
// blocks form a contiguous range of the launch's blocks; a workgroup finds its solve by a
// binary search over the first blocks (every lane the same, so the loads are uniform) and runs
// that solve's stage exactly as a launch of its own would, with its own records, values,
// vectors and stop flag.  A solve's arithmetic therefore does not depend on its companions.
__device__ __forceinline__ BatchArg batch_arg(const BatchArg* __restrict__ args, int nslot,
                                              int* vb) {
  int lo = 0, hi = nslot - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (args[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  *vb = b - args[lo].first;
  return args[lo];
}

template <typename S, typename C, int MODE>
__global__ __launch_bounds__(256) void k_bcell_fwd(const BatchArg* __restrict__ args, int nslot,
                                                   int recmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int vb;
  const BatchArg a = batch_arg(args, nslot, &vb);
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  load_record(rec, a.recs + (int64_t)vb * a.stride, a.len, threadIdx.x, blockDim.x);
  const int dn = a.done ? *a.done : 0;
  __syncthreads();
  if (dn) return;
  const CellDesc d = *reinterpret_cast<const CellDesc*>(rec);
  const S* vals = reinterpret_cast<const S*>(a.vals);
  unsigned char* sm = smem_raw + 4 * recmax;
  if constexpr (MODE == 2)
    cell_fwd_sym<S, C>(d, rec, vals, a.y, a.cb,
                       SymCfg{a.sqtab, a.sqn, a.sqld, a.sqmat, a.sqoff}, sm);
  else if (a.staged)
    cell_fwd_body<S, C, true, 0>(d, rec, vals, a.y, a.cb, a.blk_elems, a.team, false, sm);
  else
    cell_fwd_body<S, C, false, 0>(d, rec, vals, a.y, a.cb, a.blk_elems, a.team, false, sm);
}

template <typename S, typename C, int MODE>
__global__ __launch_bounds__(256) void k_bcell_bwd(const BatchArg* __restrict__ args, int nslot,
                                                   int recmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int vb;
  const BatchArg a = batch_arg(args, nslot, &vb);
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  load_record(rec, a.recs + (int64_t)vb * a.stride, a.len, threadIdx.x, blockDim.x);
  const int dn = a.done ? *a.done : 0;
  __syncthreads();
  if (dn) return;
  const CellDesc d = *reinterpret_cast<const CellDesc*>(rec);
  const S* vals = reinterpret_cast<const S*>(a.vals);
  unsigned char* sm = smem_raw + 4 * recmax;
  if constexpr (MODE == 2)
    cell_bwd_sym<S, C>(d, rec, vals, a.y, SymCfg{a.sqtab, a.sqn, a.sqld, a.sqmat, a.sqoff}, sm,
                       TopIn{});
  else if (a.staged)
    cell_bwd_body<S, C, true, 0>(d, rec, vals, a.y, a.blk_elems, a.team, sm);
  else
    cell_bwd_body<S, C, false, 0>(d, rec, vals, a.y, a.blk_elems, a.team, sm);
}

// Group stages: blockDim / seg groups per workgroup (seg: the solve's lanes per group).
template <typename S, typename C, bool FWD>
__global__ __launch_bounds__(256) void k_bgroup(const BatchArg* __restrict__ args, int nslot,
                                                int recmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int vb;
  const BatchArg a = batch_arg(args, nslot, &vb);
  const int per = blockDim.x / a.seg, g0 = vb * per, cnt = min(per, a.count - g0);
  int32_t* rec = reinterpret_cast<int32_t*>(smem_raw);
  load_record(rec, a.recs + (int64_t)g0 * a.stride, cnt * a.stride, threadIdx.x, blockDim.x);
  const int dn = a.done ? *a.done : 0;
  __syncthreads();
  if (dn) return;
  const int gsel = threadIdx.x / a.seg;
  const int32_t* rb = rec + gsel * a.stride;
  GroupDesc d{};
  if (gsel < cnt) d = *reinterpret_cast<const GroupDesc*>(rb);
  const S* vals = reinterpret_cast<const S*>(a.vals);
  if constexpr (FWD)
    group_fwd_body<S, C, true>(d, a.seg, a.per_group, a.blk_elems, a.team, rb, vals, a.y, a.cb,
                               smem_raw + 4 * recmax, a.gdense != 0);
  else
    group_bwd_body<S, C, true>(d, a.seg, a.per_group, a.blk_elems, a.team, rb, vals, a.y,
                               smem_raw + 4 * recmax, a.gdense != 0);
}

// Roots: one workgroup per solve.
template <typename S, typename C>
__global__ __launch_bounds__(kRootThreads) void k_broot(const BatchArg* __restrict__ args,
                                                        int nslot) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BatchArg a = args[blockIdx.x];
  if (a.done && *a.done) return;
  root_body<S, C>(a.count, a.recs, reinterpret_cast<const S*>(a.vals), a.y, a.staged != 0,
                  smem_raw);
}

template <typename S, typename C>
void batch_launch(const BatchApplyPlan& plan, const BatchLaunch& l, hipStream_t s) {
  const BatchArg* a = plan.args.p + l.off;
  const dim3 g(l.blocks), b(l.threads);
  switch (l.kind) {
    case BK_CELL_FWD_SYM:
      hipLaunchKernelGGL((k_bcell_fwd<S, C, 2>), g, b, l.smem, s, a, l.nslot, l.recmax); break;
    case BK_CELL_FWD:
      hipLaunchKernelGGL((k_bcell_fwd<S, C, 0>), g, b, l.smem, s, a, l.nslot, l.recmax); break;
    case BK_GROUP_FWD:
      hipLaunchKernelGGL((k_bgroup<S, C, true>), g, b, l.smem, s, a, l.nslot, l.recmax); break;
    case BK_ROOT:
      hipLaunchKernelGGL((k_broot<S, C>), g, b, l.smem, s, a, l.nslot); break;
    case BK_GROUP_BWD:
      hipLaunchKernelGGL((k_bgroup<S, C, false>), g, b, l.smem, s, a, l.nslot, l.recmax); break;
    case BK_CELL_BWD_SYM:
      hipLaunchKernelGGL((k_bcell_bwd<S, C, 2>), g, b, l.smem, s, a, l.nslot, l.recmax); break;
    default:
      hipLaunchKernelGGL((k_bcell_bwd<S, C, 0>), g, b, l.smem, s, a, l.nslot, l.recmax); break;
  }
}

}  // namespace

size_t apply_smem_need(const FactorDev& f, size_t* worst) {
  size_t w = 0;
  const size_t cs = f.store == HIF_STORE_F64 ? 8 : 4;
  for (const LevelDev& L : f.lv) {
    size_t c, g;
    if (f.store == HIF_STORE_F64) {
      c = cell_plan<double>(L).rec + cell_plan<double>(L).smem;
      g = group_plan<double>(L).rec + group_plan<double>(L).smem;
    } else {
      c = cell_plan<float>(L).rec + cell_plan<float>(L).smem;
      g = group_plan<float>(L).rec + group_plan<float>(L).smem;
    }
    if (L.tiled) c = cs * (size_t)(L.maxI + L.maxB);
    if (L.gtiled) g = cs * (size_t)std::max(1, L.maxG);
    w = std::max(w, std::max(c, g));
  }
  bool rs;
  w = std::max(w, f.root_tiled ? cs * (size_t)f.nroot
                               : (f.store == HIF_STORE_F64 ? root_smem<double>(f.nroot, &rs)
                                                           : root_smem<float>(f.nroot, &rs)));
  const int nlev = (int)f.lv.size();
  for (int l = 0; l < nlev; ++l) {
    const LevelDev* P = l + 1 < nlev ? &f.lv[l + 1] : nullptr;
    if (!(f.lv[l].fuse || (!P && f.root_fused))) continue;
    const FusePlan fp = f.store == HIF_STORE_F64 ? fuse_plan<double>(f.lv[l], P, f.nroot)
                                                 : fuse_plan<float>(f.lv[l], P, f.nroot);
    w = std::max(w, fp.rec + fp.smem);
  }
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

void hif_apply_gated(const FactorDev& f, double* y, const CgGate& g, hipStream_t s) {
  HIF_REQUIRE(f.gate && !f.lv.empty() && f.lv[0].ncell && !f.lv[0].tiled && !f.lv[0].cdense,
              HIF_ERR_ARG, "factor has no gated apply");
  const int* done = &g.st->done;
  switch (f.store) {
    case HIF_STORE_F64: apply_impl<double, double>(f, y, done, s, &g); break;
    case HIF_STORE_F32: apply_impl<float, float>(f, y, done, s, &g); break;
    case HIF_STORE_BF16: apply_impl<bf16_t, float>(f, y, done, s, &g); break;
  }
}

void hif_apply_rhs(const FactorDev& f, double* y, const CgRhs& r, hipStream_t s) {
  HIF_REQUIRE(f.gate && !f.lv.empty() && f.lv[0].ncell && !f.lv[0].tiled && !f.lv[0].cdense,
              HIF_ERR_ARG, "factor has no first stage that makes the right-hand side");
  const int* done = &r.st->done;
  switch (f.store) {
    case HIF_STORE_F64: apply_impl<double, double>(f, y, done, s, nullptr, &r); break;
    case HIF_STORE_F32: apply_impl<float, float>(f, y, done, s, nullptr, &r); break;
    case HIF_STORE_BF16: apply_impl<bf16_t, float>(f, y, done, s, nullptr, &r); break;
  }
}

void setup_cg_gate(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                   const std::vector<int32_t>& idx, int64_t N, hipStream_t s) {
  f.gate = false;
  if (f.lv.empty() || cells.empty() || cells[0].empty() || f.lv[0].tiled || f.lv[0].cdense ||
      std::getenv("HIFCN_NO_CG_GATE"))
    return;
  const std::vector<CellDesc>& cs = cells[0];
  // owner of each DOF outside the interiors: the first cell with it on its boundary, the
  // rest (no cell's boundary) dealt out in turn
  std::vector<int32_t> owner(N, -1);
  for (const CellDesc& c : cs)
    for (int i = 0; i < c.nI; ++i) owner[idx[c.offI + i]] = -2;
  for (size_t c = 0; c < cs.size(); ++c)
    for (int b = 0; b < cs[c].nB; ++b) {
      int32_t& o = owner[idx[cs[c].offB + b]];
      if (o == -1) o = (int32_t)c;
    }
  std::vector<std::vector<int32_t>> lists(cs.size());
  int64_t spare = 0;
  for (int64_t i = 0; i < N; ++i) {
    if (owner[i] == -2) continue;
    const size_t c = owner[i] >= 0 ? (size_t)owner[i] : (size_t)(spare++ % (int64_t)cs.size());
    lists[c].push_back((int32_t)i);
  }
  size_t maxc = 0;
  for (const auto& v : lists) maxc = std::max(maxc, v.size());
  f.gcstride = 1 + (int)maxc;
  std::vector<int32_t> rec(cs.size() * (size_t)f.gcstride, 0);
  for (size_t c = 0; c < cs.size(); ++c) {
    rec[c * f.gcstride] = (int32_t)lists[c].size();
    std::copy(lists[c].begin(), lists[c].end(), rec.begin() + c * f.gcstride + 1);
  }
  f.gcopy.upload(rec, s);
  f.gate_n = N;
  f.gate = true;
}

// Allow the apply kernels to use up to `bytes` of dynamic LDS (gfx950: 160 KiB per CU).  The
// attribute is shared by every handle, so it only ever grows (a smaller factor built later must
// not take LDS away from a larger one), under a lock since factors may be built concurrently.
void set_apply_smem_limits(size_t bytes) {
  static std::mutex mu;
  static size_t granted = 64 * 1024;
  std::lock_guard<std::mutex> lock(mu);
  if (bytes <= granted) return;
  const int b = (int)bytes;
#define HIF_SMEM(K) HIF_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(K),           \
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, b))
#define HIF_SMEM_TILES(S, C, TT)                                                              \
  HIF_SMEM((k_tfwd_rows<S, C, TT>));                                                          \
  HIF_SMEM((k_tcols<S, C, TT>))
#define HIF_SMEM_ALL(S, C)                                                                    \
  HIF_SMEM((k_cell_fwd<S, C, false, 0>));                                                     \
  HIF_SMEM((k_cell_bwd<S, C, false, 0>));                                                     \
  HIF_SMEM((k_cell_fwd<S, C, true, 0>));                                                      \
  HIF_SMEM((k_cell_bwd<S, C, true, 0>));                                                      \
  HIF_SMEM((k_cell_fwd<S, C, false, 1>));                                                     \
  HIF_SMEM((k_cell_bwd<S, C, false, 1>));                                                     \
  HIF_SMEM((k_cell_fwd<S, C, true, 1>));                                                      \
  HIF_SMEM((k_cell_bwd<S, C, true, 1>));                                                      \
  HIF_SMEM((k_group_fwd<S, C, true>));                                                        \
  HIF_SMEM((k_group_bwd<S, C, true>));                                                        \
  HIF_SMEM((k_group_fwd<S, C, false>));                                                       \
  HIF_SMEM((k_group_bwd<S, C, false>));                                                       \
  HIF_SMEM_TILES(S, C, 256);                                                                  \
  HIF_SMEM_TILES(S, C, 512);                                                                  \
  HIF_SMEM_TILES(S, C, 1024);                                                                 \
  HIF_SMEM((k_root<S, C>));                                                                   \
  HIF_SMEM((k_fuse_fwd<S, C, true>));                                                         \
  HIF_SMEM((k_fuse_fwd<S, C, false>));                                                        \
  HIF_SMEM((k_fuse_root<S, C>))
#define HIF_SMEM_BATCH(S, C)                                                                  \
  HIF_SMEM((k_bcell_fwd<S, C, 0>));                                                           \
  HIF_SMEM((k_bcell_bwd<S, C, 0>));                                                           \
  HIF_SMEM((k_bcell_fwd<S, C, 2>));                                                           \
  HIF_SMEM((k_bcell_bwd<S, C, 2>));                                                           \
  HIF_SMEM((k_bgroup<S, C, true>));                                                           \
  HIF_SMEM((k_bgroup<S, C, false>));                                                          \
  HIF_SMEM((k_broot<S, C>))
  HIF_SMEM_ALL(double, double);
  HIF_SMEM_ALL(float, float);
  HIF_SMEM_ALL(bf16_t, float);
  HIF_SMEM_BATCH(double, double);
  HIF_SMEM_BATCH(float, float);
#undef HIF_SMEM_BATCH
#undef HIF_SMEM_ALL
#undef HIF_SMEM_TILES
#undef HIF_SMEM
  granted = bytes;
}

bool batchable(const FactorDev& f) {
  if (f.store == HIF_STORE_BF16 || f.top >= 0 || f.root_tiled) return false;
  for (size_t l = 0; l < f.lv.size(); ++l) {
    const LevelDev& L = f.lv[l];
    if (L.tiled || L.cdense || L.gtiled) return false;
    if (L.ncell && L.cmode != (l == 0 ? 2 : 0)) return false;
    if (L.ngroup && !(f.store == HIF_STORE_F64 ? group_plan<double>(L).staged
                                               : group_plan<float>(L).staged))
      return false;
  }
  return true;
}

namespace {

constexpr int kBatchThreads = 256;

// The launch plan of one solve's stage inside a batched launch (the solve's own plan with the
// launch's block size).
template <typename C>
void batch_cell(const FactorDev& f, int l, double* y, const int* done, BatchArg& a,
                BatchLaunch& bl, bool fwd) {
  const LevelDev& L = f.lv[l];
  a.recs = L.crec.p;
  a.vals = f.vals.p;
  a.y = y;
  a.cb = f.cb.p + (int64_t)(l & 1) * f.cbstride;
  a.done = done;
  a.sqtab = f.sqtab.p;
  a.sqn = L.sqn;
  a.sqld = L.sqld;
  a.sqmat = L.sqmat;
  a.sqoff = L.sqoff;
  a.stride = L.cstride;
  a.len = fwd ? L.cfwd : L.cstride;
  a.count = L.ncell;
  if (L.cmode == 2) {
    bl.threads = 64;
    bl.smem = std::max(bl.smem, sizeof(C) * (size_t)sym_smem_elems(L.sqmat, L.maxB));
  } else {
    const size_t vec = 3 * (size_t)L.maxI + 2 * (size_t)L.maxB + 4;
    a.blk_elems = round_up(L.maxCV, 8);
    a.staged = sizeof(C) * (a.blk_elems + vec) <= kStageMax ? 1 : 0;
    if (!a.staged) a.blk_elems = 0;
    int team = 1;
    while (team < 8 && (team * 2) * L.maxI <= kBatchThreads) team <<= 1;
    a.team = team;
    bl.threads = kBatchThreads;
    bl.smem = std::max(bl.smem, sizeof(C) * (a.blk_elems + vec));
  }
  bl.recmax = std::max(bl.recmax, L.cstride);
  a.first = bl.blocks;
  bl.blocks += L.ncell;
}

template <typename C>
void batch_group(const FactorDev& f, int l, double* y, const int* done, BatchArg& a,
                 BatchLaunch& bl) {
  const LevelDev& L = f.lv[l];
  const StagePlan p = group_plan<C>(L);
  a.recs = L.grec.p;
  a.vals = f.vals.p;
  a.y = y;
  a.cb = f.cb.p + (int64_t)(l & 1) * f.cbstride;
  a.done = done;
  a.stride = L.gstride;
  a.count = L.ngroup;
  a.gdense = L.gdense;
  a.seg = p.seg;
  a.team = p.team;
  a.blk_elems = p.blk_elems;
  a.per_group = p.per_group;
  // as many groups per workgroup as fit the block size and the LDS budget
  int per = kBatchThreads / p.seg;
  while (per > 1 && sizeof(C) * (size_t)per * p.per_group > kStageBudget) per >>= 1;
  a.seg = kBatchThreads / per;  // lanes per group (the extra ones idle in the body's loops)
  bl.threads = kBatchThreads;
  bl.smem = std::max(bl.smem, sizeof(C) * (size_t)per * p.per_group);
  bl.recmax = std::max(bl.recmax, per * L.gstride);
  a.first = bl.blocks;
  bl.blocks += (L.ngroup + per - 1) / per;
}

template <typename C>
void build_batch_impl(const std::vector<const FactorDev*>& fs, const std::vector<double*>& y,
                      const std::vector<const int*>& done, BatchApplyPlan& plan, hipStream_t s) {
  const int ns = (int)fs.size();
  int lmax = 0;
  for (const FactorDev* f : fs) lmax = std::max(lmax, (int)f->lv.size());
  std::vector<BatchArg> args;
  plan.launches.clear();
  auto close = [&](BatchLaunch& bl, std::vector<BatchArg>& part) {
    if (part.empty()) return;
    bl.off = (int)args.size();
    bl.nslot = (int)part.size();
    args.insert(args.end(), part.begin(), part.end());
    plan.launches.push_back(bl);
  };
  auto stage = [&](int l, int kind) {
    BatchLaunch bl;
    std::vector<BatchArg> part;
    for (int i = 0; i < ns; ++i) {
      const FactorDev& f = *fs[i];
      if (l >= (int)f.lv.size()) continue;
      const LevelDev& L = f.lv[l];
      BatchArg a{};
      if (kind == BK_CELL_FWD || kind == BK_CELL_BWD) {
        if (!L.ncell) continue;
        batch_cell<C>(f, l, y[i], done[i], a, bl, kind == BK_CELL_FWD);
        bl.kind = L.cmode == 2 ? (kind == BK_CELL_FWD ? BK_CELL_FWD_SYM : BK_CELL_BWD_SYM) : kind;
      } else {
        if (!L.ngroup) continue;
        batch_group<C>(f, l, y[i], done[i], a, bl);
        bl.kind = kind;
      }
      part.push_back(a);
    }
    bl.smem += 4 * (size_t)bl.recmax;
    close(bl, part);
  };
  for (int l = 0; l < lmax; ++l) {
    stage(l, BK_CELL_FWD);
    stage(l, BK_GROUP_FWD);
  }
  {
    BatchLaunch bl;
    bl.kind = BK_ROOT;
    bl.threads = kRootThreads;
    std::vector<BatchArg> part;
    for (int i = 0; i < ns; ++i) {
      const FactorDev& f = *fs[i];
      if (!f.nroot) continue;
      BatchArg a{};
      bool rs;
      bl.smem = std::max(bl.smem, root_smem<C>(f.nroot, &rs));
      a.recs = f.idx.p + f.offRootIdx;
      a.vals = reinterpret_cast<const unsigned char*>(f.vals.p) +
               (size_t)f.offRootV * store_elem_bytes(f.store);
      a.y = y[i];
      a.done = done[i];
      a.count = f.nroot;
      a.staged = rs ? 1 : 0;
      a.first = bl.blocks++;
      part.push_back(a);
    }
    close(bl, part);
  }
  for (int l = lmax - 1; l >= 0; --l) {
    stage(l, BK_GROUP_BWD);
    stage(l, BK_CELL_BWD);
  }
  size_t need = 0;
  for (const BatchLaunch& bl : plan.launches) need = std::max(need, bl.smem);
  set_apply_smem_limits(need);
  plan.args.upload(args, s);
}

}  // namespace

void build_batch_apply(const std::vector<const FactorDev*>& fs, const std::vector<double*>& y,
                       const std::vector<const int*>& done, BatchApplyPlan& plan,
                       hipStream_t s) {
  HIF_REQUIRE(!fs.empty() && fs.size() == y.size() && fs.size() == done.size(), HIF_ERR_ARG,
              "internal: batch apply lists");
  plan.store = fs[0]->store;
  for (const FactorDev* f : fs)
    HIF_REQUIRE(f->store == plan.store && batchable(*f), HIF_ERR_ARG,
                "internal: factor not batchable");
  if (plan.store == HIF_STORE_F64) build_batch_impl<double>(fs, y, done, plan, s);
  else build_batch_impl<float>(fs, y, done, plan, s);
}

void run_batch_apply(const BatchApplyPlan& plan, hipStream_t s) {
  for (const BatchLaunch& l : plan.launches) {
    if (plan.store == HIF_STORE_F64) batch_launch<double, double>(plan, l, s);
    else batch_launch<float, float>(plan, l, s);
  }
  HIF_CHECK(hipGetLastError());
}

namespace {
// Tiles of one level; its cells' interiors take scratch [*base, *base + sum nI): every level
// keeps its own region because all forward stages run before any backward stage.
void tile_level(LevelDev& L, const std::vector<CellDesc>& cells, int64_t* base, hipStream_t s) {
  std::vector<int4> rt, ct;
  int64_t woff = *base;
  for (size_t c = 0; c < cells.size(); ++c) {
    const CellDesc& d = cells[c];
    const int nrows = d.mode ? d.nI : d.nI + d.nB;
    for (int r0 = 0; r0 < nrows; r0 += kRowTile) rt.push_back({(int)c, r0, (int)woff, 0});
    for (int c0 = 0; c0 < d.nI; c0 += kColTile) ct.push_back({(int)c, c0, (int)woff, 0});
    woff += d.nI;
  }
  L.nrt = (int)rt.size();
  L.nct = (int)ct.size();
  L.rtiles.upload(rt, s);
  L.ctiles.upload(ct, s);
  HIF_REQUIRE(woff < (int64_t)INT32_MAX, HIF_ERR_ARG, "tiled scratch too large");
  *base = woff;
}

}  // namespace

namespace {
// Record of one cell: the descriptor with record-relative index offsets, then its index lists.
// Modes 0 and 1: interior ids, then (mode 1) ib[nB] and the links grouped by interior DOF
// (rowptr[nI + 1], blist[nB]), then the boundary ids; the forward stage reads only the prefix
// up to the coupling positions (cell_fwd_len), the backward stage the whole record.  Symmetric cells (mode 2): interior ids, boundary ids, ib[nB], then one word
// per interior DOF: its link count and up to three boundary positions of 8 bits each (a 5- or
// 7-point stencil gives an interior node at most three boundary neighbours, and boundaries stay
// below 256 DOFs), so the backward stage needs one load per DOF where the lists need two
// dependent ones.  Both id lists then lie in the 128 words after the descriptor, which a stage
// loads together with the descriptor itself (their positions need only nI).
int cell_record_len(const CellDesc& d) {
  if (d.mode == 2) return round_up(8 + 2 * d.nI + 2 * d.nB, 4);
  return round_up(8 + d.nI + d.nB + (d.mode ? 2 * d.nB + d.nI + 1 : 0), 4);
}
int cell_fwd_len(const CellDesc& d) {
  return round_up(8 + d.nI + (d.mode == 2 ? 2 * d.nB : d.mode ? d.nB : 0), 4);
}
void put_cell_record(int32_t* r, const CellDesc& d, const std::vector<int32_t>& idx,
                     const LevelDev* sym = nullptr) {
  CellDesc e = d;
  e.offI = 8;
  for (int i = 0; i < d.nI; ++i) r[8 + i] = idx[d.offI + i];
  if (d.mode == 2) {
    HIF_REQUIRE(sym && (int)sym->sqhead.size() == kSymTabHead, HIF_ERR_ARG,
                "internal: symmetric cell record without its table");
    e.mode = d.nI <= sym->sqn ? sym->sqhead[d.nI] : -1;  // see SymCfg
    e.offB = 8 + d.nI;
    e.offC = 8 + d.nI + d.nB;
    for (int b = 0; b < d.nB; ++b) r[e.offB + b] = idx[d.offB + b];
    for (int b = 0; b < d.nB; ++b) r[e.offC + b] = idx[d.offC + b];
    const int32_t* rp = idx.data() + d.offC + d.nB;
    const int32_t* bl = rp + d.nI + 1;
    for (int i = 0; i < d.nI; ++i) {
      const int cnt = rp[i + 1] - rp[i];
      HIF_REQUIRE(cnt <= 3 && d.nB < 256, HIF_ERR_ARG, "internal: level-0 link count");
      int32_t w = cnt;
      for (int q = 0; q < cnt; ++q) w |= bl[rp[i] + q] << (8 * (q + 1));
      r[e.offC + d.nB + i] = w;
    }
  } else {
    const int nc = d.mode ? 2 * d.nB + d.nI + 1 : 0;
    e.offC = d.mode ? 8 + d.nI : 0;
    e.offB = 8 + d.nI + nc;
    for (int q = 0; q < nc; ++q) r[8 + d.nI + q] = idx[d.offC + q];
    for (int b = 0; b < d.nB; ++b) r[e.offB + b] = idx[d.offB + b];
  }
  std::memcpy(r, &e, sizeof(CellDesc));
}
// Record of one group: the descriptor, then DOF ids, pivot order, gather pointers and slots.
int group_record_len(const GroupDesc& g, const std::vector<int32_t>& idx) {
  return round_up(8 + 2 * g.n + g.n + 1 + idx[g.offGP + g.n], 4);
}
void put_group_record(int32_t* r, const GroupDesc& g, const std::vector<int32_t>& idx) {
  const int n = g.n, ns = idx[g.offGP + n];
  GroupDesc e = g;
  e.offIdx = 8;
  e.offPerm = 8 + n;
  e.offGP = 8 + 2 * n;
  std::memcpy(r, &e, sizeof(GroupDesc));
  for (int i = 0; i < n; ++i) r[8 + i] = idx[g.offIdx + i];
  for (int i = 0; i < n; ++i)
    r[8 + n + i] = g.offPerm + i < (int64_t)idx.size() ? idx[g.offPerm + i] : i;
  for (int i = 0; i < n + 1 + ns; ++i) r[8 + 2 * n + i] = idx[g.offGP + i];
}
}  // namespace

void setup_fusion(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                  const std::vector<std::vector<GroupDesc>>& groups,
                  const std::vector<int32_t>& idx, int64_t N, hipStream_t s) {
  const bool f64 = f.store == HIF_STORE_F64;
  const int nlev = (int)f.lv.size();
  const bool off = std::getenv("HIFCN_NO_FUSE") != nullptr;
  // block records of every level
  for (int l = 0; l < nlev; ++l) {
    LevelDev& L = f.lv[l];
    L.cstride = 4;
    L.cfwd = 4;
    for (const CellDesc& d : cells[l]) {
      L.cstride = std::max(L.cstride, cell_record_len(d));
      L.cfwd = std::max(L.cfwd, cell_fwd_len(d));
    }
    std::vector<int32_t> cr((size_t)cells[l].size() * L.cstride, 0);
    for (size_t c = 0; c < cells[l].size(); ++c)
      put_cell_record(cr.data() + c * L.cstride, cells[l][c], idx, &L);
    L.crec.upload(cr, s);
    L.gstride = 8;
    for (const GroupDesc& g : groups[l]) L.gstride = std::max(L.gstride, group_record_len(g, idx));
    std::vector<int32_t> gr((size_t)groups[l].size() * L.gstride, 0);
    for (size_t g = 0; g < groups[l].size(); ++g)
      put_group_record(gr.data() + g * L.gstride, groups[l][g], idx);
    L.grec.upload(gr, s);
  }
  std::vector<int32_t> parent(N, -1);
  for (int l = 0; l + 1 < nlev; ++l) {
    LevelDev& L = f.lv[l];
    const LevelDev& P = f.lv[l + 1];
    L.fuse = false;
    if (off || !L.ngroup || L.gtiled || !P.ncell || P.tiled || P.cmode != 0) continue;
    // owner of each level-l group: the level l+1 cell holding one of its DOFs in its interior
    const std::vector<CellDesc>& pc = cells[l + 1];
    for (size_t p = 0; p < pc.size(); ++p)
      for (int i = 0; i < pc[p].nI; ++i) parent[idx[pc[p].offI + i]] = (int32_t)p;
    const std::vector<GroupDesc>& gs = groups[l];
    std::vector<int32_t> owner(gs.size(), -1);
    bool split = false;
    for (size_t g = 0; g < gs.size() && !split; ++g)
      for (int i = 0; i < gs[g].n; ++i) {
        const int32_t q = parent[idx[gs[g].offIdx + i]];
        if (q < 0) continue;
        if (owner[g] < 0) owner[g] = q;
        else if (owner[g] != q) { split = true; break; }
      }
    for (size_t p = 0; p < pc.size(); ++p)
      for (int i = 0; i < pc[p].nI; ++i) parent[idx[pc[p].offI + i]] = -1;
    if (split) continue;
    // groups on level l+1 cell boundaries go to the least loaded cell
    std::vector<int32_t> load(pc.size(), 0);
    for (int32_t o : owner) if (o >= 0) ++load[o];
    std::priority_queue<std::pair<int32_t, int32_t>, std::vector<std::pair<int32_t, int32_t>>,
                        std::greater<>> least;  // (load, cell)
    for (size_t p = 0; p < pc.size(); ++p) least.push({load[p], (int32_t)p});
    for (int32_t& o : owner)
      if (o < 0) {
        const auto top = least.top();
        least.pop();
        o = top.second;
        least.push({++load[o], o});
      }
    int maxown = 0;
    for (int32_t c : load) maxown = std::max(maxown, c);
    L.maxown = maxown;
    L.fstride = P.cstride + maxown * L.gstride;
    if (!(f64 ? fuse_plan<double>(L, &P, 0).ok : fuse_plan<float>(L, &P, 0).ok)) continue;
    // per next-level cell: its record, then the records of the groups it owns
    std::vector<int32_t> fr((size_t)pc.size() * L.fstride, 0);
    for (size_t p = 0; p < pc.size(); ++p) put_cell_record(fr.data() + p * L.fstride, pc[p], idx);
    std::vector<int32_t> fill(pc.size(), 0);
    for (size_t g = 0; g < gs.size(); ++g) {
      const int32_t o = owner[g];
      put_group_record(fr.data() + (size_t)o * L.fstride + P.cstride +
                           (size_t)fill[o]++ * L.gstride, gs[g], idx);
    }
    L.frec.upload(fr, s);
    L.fuse = true;
  }
  f.root_fused = false;
  if (!off && nlev > 0 && f.nroot && !f.root_tiled && f.lv[nlev - 1].ngroup &&
      !f.lv[nlev - 1].gtiled)
    f.root_fused = f64 ? fuse_plan<double>(f.lv[nlev - 1], nullptr, f.nroot).ok
                       : fuse_plan<float>(f.lv[nlev - 1], nullptr, f.nroot).ok;
}

namespace {
// Workgroup size of a tiled level: small cells (few columns per row tile) run more, smaller
// workgroups per CU.  HIFCN_TILE_SMALL_THREADS / HIFCN_TILE_SMALL_MAX override the choice.
int tile_threads(int maxI) {
  int small_threads = 512, small_max = 512;
  if (const char* e = std::getenv("HIFCN_TILE_SMALL_THREADS")) small_threads = std::atoi(e);
  if (const char* e = std::getenv("HIFCN_TILE_SMALL_MAX")) small_max = std::atoi(e);
  if (small_threads != 256 && small_threads != 512) small_threads = 1024;
  return maxI <= small_max ? small_threads : 1024;
}
}  // namespace

// ------------------------------------------------------------------------ dense groups --
struct DenseGroupTask {
  int64_t offV, offW;  // the group's storage in vals; its work area (doubles)
  int32_t n, nr, offPerm, pad;
};

// One workgroup per group: column c of G = (the forward group step applied to e_c), in FP64
// from the stored blocks (packed L_g^-1, T, packed L_s^-1; see group_fwd_body), then G over
// the blocks (column-major, storage precision) once every column is formed.
template <typename S>
__global__ __launch_bounds__(256) void k_group_dense(const DenseGroupTask* __restrict__ tasks,
                                                     S* __restrict__ vals,
                                                     const int32_t* __restrict__ idx,
                                                     double* __restrict__ work) {
  const DenseGroupTask t = tasks[blockIdx.x];
  const int n = t.n, nr = t.nr, k = n - nr;
  const S* v = vals + t.offV;
  const S* T = v + tri_count(n);            // k x nr, T[i k + s]
  const S* Ls = T + (int64_t)k * nr;         // packed L_s^-1
  const int32_t* perm = idx + t.offPerm;
  double* G = work + t.offW;                 // n x n, column-major
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double* z = work + t.offW + (int64_t)n * n + (int64_t)c * (n + 3 * nr);
    double* tv = z + n;
    double* uv = tv + nr;
    double* wv = uv + nr;
    double* out = G + (int64_t)c * n;
    for (int i = 0; i < n; ++i)  // z = L_g^-1 e_c
      z[i] = i >= c ? load_as<double>(v + colstart(c, n) + (i - c)) : 0.0;
    if (nr == 0) {
      for (int i = 0; i < n; ++i) out[i] = z[i];
      continue;
    }
    for (int i = 0; i < nr; ++i) {  // z_I~ - T^T z_I^
      double a = 0;
      for (int q = 0; q < k; ++q) a += load_as<double>(T + (int64_t)i * k + q) * z[perm[nr + q]];
      tv[i] = z[perm[i]] - a;
    }
    for (int i = 0; i < nr; ++i) {  // u = L_s^-1 (...)
      double a = 0;
      for (int j = 0; j <= i; ++j) a += load_as<double>(Ls + colstart(j, nr) + (i - j)) * tv[j];
      uv[i] = a;
    }
    for (int i = 0; i < nr; ++i) {  // w = L_s^-T u
      double a = 0;
      for (int j = i; j < nr; ++j) a += load_as<double>(Ls + colstart(i, nr) + (j - i)) * uv[j];
      wv[i] = a;
    }
    for (int q = 0; q < k; ++q) {  // z_I^ + T w, and u at the redundant DOFs
      double a = 0;
      for (int i = 0; i < nr; ++i) a += load_as<double>(T + (int64_t)i * k + q) * wv[i];
      out[perm[nr + q]] = z[perm[nr + q]] + a;
    }
    for (int i = 0; i < nr; ++i) out[perm[i]] = uv[i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) vals[t.offV + e] = (S)G[e];
}

void setup_dense_groups(FactorDev& f, const std::vector<std::vector<GroupDesc>>& groups,
                        const std::vector<int32_t>& idx, int top, hipStream_t s) {
  if (std::getenv("HIFCN_NO_DENSE_GROUPS") || f.store == HIF_STORE_BF16) return;
  const bool f64 = f.store == HIF_STORE_F64;
  const int64_t eb = (int64_t)store_elem_bytes(f.store);
  for (size_t l = 0; l < f.lv.size(); ++l) {
    LevelDev& L = f.lv[l];
    if (!L.ngroup || L.gtiled || (top >= 0 && (int)l >= top)) continue;
    int64_t dense = 0, packed = 0;
    int maxsq = 0;
    bool fits = true;
    for (const GroupDesc& d : groups[l]) {
      const int64_t n = d.n, nr = d.nr;
      dense += n * n;
      packed += tri_count(n) + (n - nr) * nr + tri_count(nr);
      maxsq = std::max<int>(maxsq, (int)(n * n));
      fits = fits && d.cap >= n * n;
    }
    if (!fits || dense > 2 * packed) continue;
    // the level must stay staged (one workgroup's LDS holds its blocks) with G in them
    const int gv0 = L.maxGV, r0 = L.maxR;
    L.maxGV = maxsq;
    L.maxR = 0;
    const bool staged = f64 ? group_plan<double>(L).staged : group_plan<float>(L).staged;
    L.maxGV = gv0;
    L.maxR = r0;
    if (!staged) continue;
    // form G in every group of the level, over its blocks
    std::vector<DenseGroupTask> tasks;
    int64_t wo = 0;
    for (const GroupDesc& d : groups[l]) {
      tasks.push_back({d.offV, wo, d.n, d.nr, d.offPerm, 0});
      wo += (int64_t)d.n * d.n + (int64_t)d.n * (d.n + 3 * d.nr);
    }
    DevBuf<DenseGroupTask> dt(tasks.size(), s);
    dt.upload(tasks, s);
    DevBuf<double> work(std::max<int64_t>(1, wo), s);
    switch (f.store) {
      case HIF_STORE_F64:
        hipLaunchKernelGGL(k_group_dense<double>, dim3(tasks.size()), dim3(256), 0, s,
                           (const DenseGroupTask*)dt.p, reinterpret_cast<double*>(f.vals.p),
                           (const int32_t*)f.idx.p, work.p);
        break;
      default:
        hipLaunchKernelGGL(k_group_dense<float>, dim3(tasks.size()), dim3(256), 0, s,
                           (const DenseGroupTask*)dt.p, reinterpret_cast<float*>(f.vals.p),
                           (const int32_t*)f.idx.p, work.p);
    }
    HIF_CHECK(hipGetLastError());
    L.gdense = 1;
    L.maxGV = maxsq;
    L.maxR = 0;
    // bytes per sweep: G, the group's vectors and indices (forward: also the gathered slots)
    int64_t gf = 0, gb = 0;
    for (const GroupDesc& d : groups[l]) {
      const int64_t n = d.n, nsl = idx[d.offGP + n];
      gf += eb * n * n + 16 * n + 12 * nsl + 4 * n + 4 * (n + 1) + (int64_t)sizeof(GroupDesc);
      gb += eb * n * n + 16 * n + 4 * n + (int64_t)sizeof(GroupDesc);
    }
    L.group_bytes[0] = gf;
    L.group_bytes[1] = gb;
  }
}

void setup_tiling(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                  const std::vector<std::vector<GroupDesc>>& groups,
                  const std::vector<int32_t>& idx, hipStream_t s) {
  const bool f64 = f.store == HIF_STORE_F64;
  const int64_t eb = (int64_t)store_elem_bytes(f.store);
  std::vector<DenseJob> jobs;
  int64_t dtot = 0;
  auto dense_job = [&](int kind, int n, int nr, int64_t src, int32_t perm) {
    const DenseJob j{kind, n, nr, dense_ld(n), src, dtot, perm, 0};
    jobs.push_back(j);
    dtot += (int64_t)n * dense_ld(n);
    return j.dst;
  };
  // cells: link-mode blocks too large for one workgroup in dense form; the scratch keeps the
  // interiors of tiled cells from the forward to the backward sweep ([0, wtot))
  int64_t wtot = 0;
  for (size_t l = 0; l < f.lv.size(); ++l) {
    LevelDev& L = f.lv[l];
    L.tiled = L.ncell > 0 && !(f64 ? cell_plan<double>(L).staged : cell_plan<float>(L).staged);
    L.cdense = L.tiled && L.cmode == 1;
    if (!L.tiled) continue;
    L.tthreads = tile_threads(L.maxI);
    if (!L.cdense) {
      tile_level(L, cells[l], &wtot, s);
      continue;
    }
    std::vector<int4> tl;
    std::vector<int64_t> off;
    int64_t fb = 0, bb = 0;
    for (size_t c = 0; c < cells[l].size(); ++c) {
      const CellDesc& d = cells[l][c];
      off.push_back(dense_job(0, d.nI, 0, d.offV, 0));
      for (int r0 = 0; r0 < d.nI; r0 += kRowTile) tl.push_back({(int)c, r0, 0, (int)wtot});
      wtot += d.nI;
      const int64_t nI = d.nI, nB = d.nB;
      fb += eb * (nI * nI + nB) + 8 * (3 * nI + nB) + 4 * (nI + 2 * nB) + (int64_t)sizeof(CellDesc);
      bb += eb * (nI * nI + nB) + 8 * (2 * nI + nB) + 4 * (2 * nI + 1 + 3 * nB) +
            (int64_t)sizeof(CellDesc);
    }
    L.ncdt = (int)tl.size();
    L.cdtiles.upload(tl, s);
    L.cddoff.upload(off, s);
    L.cell_bytes[0] = fb;
    L.cell_bytes[1] = bb;
  }
  // groups that do not fit one workgroup (HIFCN_GROUP_TILES=1: every level's groups, for tests)
  // in dense form; their results, and the root's partial sums, take the scratch from wtot on
  // (one stage at a time)
  const char* ge = std::getenv("HIFCN_GROUP_TILES");
  const bool all_groups = ge && std::atoi(ge) != 0;
  int64_t dneed = 0;
  for (size_t l = 0; l < f.lv.size(); ++l) {
    LevelDev& L = f.lv[l];
    L.gtiled = L.ngroup > 0 && (all_groups || !(f64 ? group_plan<double>(L).staged
                                                     : group_plan<float>(L).staged));
    if (!L.gtiled) continue;
    std::vector<int4> rt, ct, sc;
    std::vector<int64_t> off;
    int64_t zo = wtot, fb = 0, bb = 0;
    for (size_t g = 0; g < groups[l].size(); ++g) {
      const GroupDesc& d = groups[l][g];
      const int n = d.n;
      off.push_back(dense_job(1, n, d.nr, d.offV, d.offPerm));
      for (int r0 = 0; r0 < n; r0 += kRowTile) rt.push_back({(int)g, r0, 0, (int)zo});
      for (int c0 = 0; c0 < n; c0 += kDenseColsPerTile) ct.push_back({(int)g, c0, 0, (int)zo});
      for (int r = 0; r < n; ++r) sc.push_back({idx[d.offIdx + r], (int)(zo + r), 1, 0});
      zo += n;
      const int64_t ns = idx[d.offGP + n];
      fb += eb * (int64_t)n * n + 8 * (4 * (int64_t)n + ns) + 4 * (3 * (int64_t)n + 1 + ns) +
            (int64_t)sizeof(GroupDesc);
      bb += eb * (int64_t)n * n + 8 * 4 * (int64_t)n + 4 * 2 * (int64_t)n +
            (int64_t)sizeof(GroupDesc);
    }
    dneed = std::max(dneed, zo - wtot);
    L.ngrt = (int)rt.size();
    L.ngct = (int)ct.size();
    L.ngsc = (int)sc.size();
    L.grtiles.upload(rt, s);
    L.gctiles.upload(ct, s);
    L.gscat.upload(sc, s);
    L.gddoff.upload(off, s);
    L.group_bytes[0] = fb;
    L.group_bytes[1] = bb;
  }
  // a root of more than 256 KiB of factor: dense A_r^-1, row tiles over column ranges
  f.root_tiled = tri_count(f.nroot) * eb > 256 * 1024;
  if (f.root_tiled) {
    const int n = f.nroot;
    f.rspan = 512;
    const int nch = (n + f.rspan - 1) / f.rspan;
    f.rddoff.upload(std::vector<int64_t>{dense_job(0, n, 0, f.offRootV, 0)}, s);
    std::vector<int4> rt, sc;
    for (int c = 0; c < nch; ++c)
      for (int r0 = 0; r0 < n; r0 += kRowTile)
        rt.push_back({0, r0, c * f.rspan, (int)(wtot + (int64_t)c * n)});
    for (int r = 0; r < n; ++r) sc.push_back({idx[f.offRootIdx + r], (int)(wtot + r), nch, n});
    f.nrdt = (int)rt.size();
    f.nrsc = (int)sc.size();
    f.rdtiles.upload(rt, s);
    f.rscat.upload(sc, s);
    dneed = std::max(dneed, (int64_t)nch * n);
    f.root_bytes = eb * (int64_t)n * n + 8 * (2 * (int64_t)n + 2 * (int64_t)nch * n) +
                   4 * 2 * (int64_t)n;
  }
  HIF_REQUIRE(wtot + dneed < (int64_t)INT32_MAX, HIF_ERR_ARG, "tiled scratch too large");
  f.wsc.alloc(std::max<int64_t>(1, wtot + dneed));
  f.ndvals = dtot;
  f.dvals.alloc((size_t)std::max<int64_t>(1, dtot) * eb);
  if (dtot) HIF_CHECK(hipMemsetAsync(f.dvals.p, 0, (size_t)dtot * eb, s));
  build_dense_forms(f, jobs, s);
}

}  // namespace hifcn
