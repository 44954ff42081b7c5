// Factor layout on the device: reading the HIFB test blob and uploading a factor.
//
// The apply kernels read, per level, one descriptor per cell and per separator group and the
// blocks of the factors E_l, C_l, K_l (Sec. 2.2) in explicit-inverse form:
//   cell  : packed L^-1 and H = A_BI A_II^-1 = G^T L^-1  (E_l of eq2_3)
//   group : packed L_g^-1                                  (C_l of jacobi-precond)
//   edge  : T and packed L_s^-1, L_s = chol(I + T^T T)     (K_l of eq_T, eq2_9)
//   root  : packed L_r^-1                                  (A_L of eq3_4)
// Explicit triangular inverses turn every sweep stage into small matrix-vector products with
// no serial triangular-solve chain.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <unordered_map>

#include "kernels.hpp"

namespace hifcn {

namespace {

struct Reader {
  const unsigned char* p;
  size_t n, pos = 0;
  int32_t i32() {
    HIF_REQUIRE(pos + 4 <= n, HIF_ERR_ARG, "HIFB blob truncated");
    int32_t v;
    std::memcpy(&v, p + pos, 4);
    pos += 4;
    return v;
  }
  void i32s(std::vector<int32_t>& v, size_t k) {
    v.resize(k);
    HIF_REQUIRE(pos + 4 * k <= n, HIF_ERR_ARG, "HIFB blob truncated");
    if (k) std::memcpy(v.data(), p + pos, 4 * k);
    pos += 4 * k;
  }
  void f64s(std::vector<double>& v, size_t k) {
    v.resize(k);
    HIF_REQUIRE(pos + 8 * k <= n, HIF_ERR_ARG, "HIFB blob truncated");
    if (k) std::memcpy(v.data(), p + pos, 8 * k);
    pos += 8 * k;
  }
};

// Inverse of a row-major lower-triangular matrix (host, FP64, forward substitution by rows:
// row i of X = (e_i - sum_{k<i} L_ik X_k) / L_ii, with contiguous row operations).
std::vector<double> tri_inverse(const std::vector<double>& L, int n) {
  std::vector<double> X((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const double d = L[(size_t)i * n + i];
    HIF_REQUIRE(d > 0.0, HIF_ERR_NOT_SPD, "non-positive Cholesky pivot in blob");
    double* xi = &X[(size_t)i * n];
    xi[i] = 1.0;
    for (int k = 0; k < i; ++k) {
      const double l = L[(size_t)i * n + k];
      if (l == 0.0) continue;
      const double* xk = &X[(size_t)k * n];
      for (int j = 0; j <= k; ++j) xi[j] -= l * xk[j];
    }
    for (int j = 0; j <= i; ++j) xi[j] /= d;
  }
  return X;
}

void push_packed(std::vector<double>& out, const std::vector<double>& M, int n) {
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) out.push_back(M[(size_t)i * n + j]);
}

}  // namespace

void level_stage_bytes(const std::vector<CellDesc>& cells, const std::vector<GroupDesc>& groups,
                       const std::vector<int64_t>& group_slots, size_t eb, LevelDev& ld) {
  int64_t cf = 0, cbk = 0, gf = 0, gbk = 0;
  for (const CellDesc& d : cells) {
    const int64_t nI = d.nI, nB = d.nB;
    const int64_t blk = (int64_t)eb * (tri_count(nI) + (d.mode ? nB : nB * nI));
    const int64_t ib = d.mode ? 4 * nB : 0;
    // mode 2 leaves the interior values in place in the forward sweep (reads y_I, writes c_B);
    // link modes read the links grouped by interior DOF in the backward sweep
    const int64_t fvec = d.mode == 2 ? 8 * (nI + nB) : 8 * (2 * nI + nB);
    const int64_t links = d.mode ? 4 * (nI + 1 + nB) : 0;
    cf += blk + fvec + 4 * nI + ib + (int64_t)sizeof(CellDesc);
    cbk += blk + 8 * (2 * nI + nB) + 4 * (nI + nB) + ib + links + (int64_t)sizeof(CellDesc);
  }
  for (size_t q = 0; q < groups.size(); ++q) {
    const GroupDesc& d = groups[q];
    const int64_t n = d.n, nr = d.nr, k = n - nr;
    const int64_t blk = (int64_t)eb * (tri_count(n) + (nr ? k * nr + tri_count(nr) : 0));
    const int64_t perm = nr ? 4 * n : 0;
    const int64_t sl = q < group_slots.size() ? group_slots[q] : 0;
    gf += blk + 16 * n + 12 * sl + 4 * n + 4 * (n + 1) + perm + (int64_t)sizeof(GroupDesc);
    gbk += blk + 16 * n + 4 * n + perm + (int64_t)sizeof(GroupDesc);
  }
  ld.cell_bytes[0] = cf;
  ld.cell_bytes[1] = cbk;
  ld.group_bytes[0] = gf;
  ld.group_bytes[1] = gbk;
}

bool sym_cells_off() { return std::getenv("HIFCN_NO_SYM_CELLS") != nullptr; }

void build_sym_table(FactorDev& f, const std::vector<CellDesc>& cells, hipStream_t s) {
  HIF_REQUIRE(!cells.empty() && !f.lv.empty(), HIF_ERR_ARG, "internal: symmetric cells");
  HIF_REQUIRE(f.store == HIF_STORE_F32 || f.store == HIF_STORE_F64, HIF_ERR_ARG,
              "internal: symmetric cells need FP32 or FP64 storage");
  std::vector<int> sizes;
  for (const CellDesc& d : cells) sizes.push_back(d.nI);
  std::sort(sizes.begin(), sizes.end());
  const int maxI = sizes.back();
  HIF_REQUIRE(maxI <= kSymMaxCell, HIF_ERR_ARG, "internal: symmetric cell size");
  LevelDev& L = f.lv[0];
  // With 2048 cells or more the launch runs many waves of workgroups and the LDS footprint sets
  // how many cells are in flight, so the square fits the median cell and the few larger cells
  // (the last cell of each axis absorbs the extra nodes) read the packed triangle.  With fewer
  // cells every workgroup is resident at once and the launch lasts as long as its slowest cell,
  // so every cell gets the square.
  L.sqn = cells.size() >= 2048 ? sizes[sizes.size() / 2] : maxI;
  // odd leading dimension: the mirrored stores of consecutive packed elements (consecutive rows
  // of one column) and the row walks of consecutive lanes fall in different banks
  L.sqld = L.sqn | 1;
  // the square or the packed triangle (padded to its storage length), then one spare word that
  // takes the stores of the storage order's padding slots
  const int E = (int)(16 / store_elem_bytes(f.store));
  L.sqmat = (int)((std::max<int64_t>((int64_t)L.sqn * L.sqld, sym_coff(tri_count(maxI))) + 3) /
                  4 * 4) + 4;
  const int32_t dump = L.sqmat - 1;
  // header: the start of each order's entries (16-byte aligned); entries in storage order
  std::vector<int32_t> tab(kSymTabHead, 0);
  for (int n = 1; n <= L.sqn; ++n) {
    tab[n] = (int32_t)tab.size();
    const int tl = (int)tri_count(n), ns = (tl + E - 1) / E * E;
    for (int sidx = 0; sidx < ns; ++sidx) {
      int p = sym_packed_index(sidx, tl, E);
      if (p >= tl) {
        tab.push_back(dump | dump << 16);
        continue;
      }
      int j = 0;
      while (p >= n - j) p -= n - j++;
      const int i = j + p;
      tab.push_back((j * L.sqld + i) | (i * L.sqld + j) << 16);
    }
    tab.resize((tab.size() + 3) / 4 * 4, 0);
  }
  L.sqoff = tab[L.sqn];
  L.sqhead.assign(tab.begin(), tab.begin() + kSymTabHead);
  f.sqtab.upload(tab, s);
}

FactorHost import_blob(const void* blob, size_t nbytes, int dim, int n, int leaf) {
  HIF_REQUIRE(blob != nullptr, HIF_ERR_ARG, "NULL blob");
  Reader rd{static_cast<const unsigned char*>(blob), nbytes};
  HIF_REQUIRE(rd.i32() == 0x42464948, HIF_ERR_ARG, "bad HIFB magic");
  HIF_REQUIRE(rd.i32() == 1, HIF_ERR_ARG, "unsupported HIFB version");
  HIF_REQUIRE(rd.i32() == dim && rd.i32() == n && rd.i32() == leaf, HIF_ERR_ARG,
              "HIFB grid does not match the grid argument");
  const int nlev = rd.i32();
  HIF_REQUIRE(nlev >= 0 && nlev < 32, HIF_ERR_ARG, "bad level count");
  const int64_t N = (int64_t)std::pow((double)n, dim);
  FactorHost fh;
  auto check_ids = [&](const std::vector<int32_t>& v) {
    for (int32_t d : v) HIF_REQUIRE(d >= 0 && d < N, HIF_ERR_ARG, "DOF id out of range");
  };
  std::vector<int32_t> I, B, ids, red, skel;
  std::vector<double> Lm, Gm, Tm;
  for (int l = 0; l < nlev; ++l) {
    LevelHost lh;
    // ---- cells
    const int ncell = rd.i32();
    HIF_REQUIRE(ncell >= 0, HIF_ERR_ARG, "bad cell count");
    int64_t cb = 0;
    struct CellB { std::vector<int32_t> B; int64_t off; };
    std::vector<CellB> cellB;
    for (int c = 0; c < ncell; ++c) {
      const int nI = rd.i32(), nB = rd.i32();
      HIF_REQUIRE(nI > 0 && nB >= 0, HIF_ERR_ARG, "bad cell sizes");
      rd.i32s(I, nI);
      rd.i32s(B, nB);
      check_ids(I);
      check_ids(B);
      rd.f64s(Lm, (size_t)nI * nI);
      rd.f64s(Gm, (size_t)nI * nB);
      const std::vector<double> Li = tri_inverse(Lm, nI);
      std::vector<int> keep;
      for (int b = 0; b < nB; ++b) {
        bool nz = false;
        for (int i = 0; i < nI && !nz; ++i) nz = Gm[(size_t)i * nB + b] != 0.0;
        if (nz) keep.push_back(b);
      }
      CellDesc d{};
      d.nI = nI;
      d.nB = (int)keep.size();
      d.offI = (int32_t)fh.idx.size();
      fh.idx.insert(fh.idx.end(), I.begin(), I.end());
      d.offB = (int32_t)fh.idx.size();
      std::vector<int32_t> Bk;
      for (int b : keep) Bk.push_back(B[b]);
      fh.idx.insert(fh.idx.end(), Bk.begin(), Bk.end());
      fh.vals.resize(align_vals((int64_t)fh.vals.size()), 0.0);
      d.offV = (int32_t)fh.vals.size();
      push_packed(fh.vals, Li, nI);
      {  // H[q][j] = sum_i G[i][keep_q] Linv[i][j] (row operations), stored column-major
        const int nk = (int)keep.size();
        std::vector<double> H((size_t)nk * nI, 0.0);
        for (int i = 0; i < nI; ++i) {
          const double* li = &Li[(size_t)i * nI];
          for (int q = 0; q < nk; ++q) {
            const double g = Gm[(size_t)i * nB + keep[q]];
            if (g == 0.0) continue;
            double* hq = &H[(size_t)q * nI];
            for (int j = 0; j <= i; ++j) hq[j] += g * li[j];
          }
        }
        for (int j = 0; j < nI; ++j)
          for (int q = 0; q < nk; ++q) fh.vals.push_back(H[(size_t)q * nI + j]);
      }
      d.offCB = (int32_t)cb;
      fh.nvals_used += tri_count(nI) + (int64_t)nI * d.nB;
      cellB.push_back({Bk, cb});
      cb += d.nB;
      lh.maxI = std::max(lh.maxI, nI);
      lh.maxB = std::max(lh.maxB, d.nB);
      lh.maxCV = std::max<int>(lh.maxCV, (int)(tri_count(nI) + (int64_t)d.nB * nI));
      lh.cells.push_back(d);
    }
    fh.cbmax = std::max(fh.cbmax, cb);
    // ---- groups
    const int ngroup = rd.i32();
    HIF_REQUIRE(ngroup >= 0, HIF_ERR_ARG, "bad group count");
    struct G { std::vector<int32_t> ids; std::vector<double> Linv; };
    std::vector<G> groups(ngroup);
    std::unordered_map<int32_t, std::pair<int, int>> where;  // dof -> (group, position)
    for (int g = 0; g < ngroup; ++g) {
      const int gn = rd.i32();
      HIF_REQUIRE(gn > 0, HIF_ERR_ARG, "bad group size");
      rd.i32s(groups[g].ids, gn);
      check_ids(groups[g].ids);
      rd.f64s(Lm, (size_t)gn * gn);
      groups[g].Linv = tri_inverse(Lm, gn);
      for (int i = 0; i < gn; ++i) where[groups[g].ids[i]] = {g, i};
    }
    // ---- skeletonized edges
    const int nskel = rd.i32();
    struct Sk { int nr = 0, k = 0; std::vector<int32_t> perm; std::vector<double> T, Lsinv; };
    std::vector<Sk> sk(ngroup);
    for (int e = 0; e < nskel; ++e) {
      const int nr = rd.i32(), k = rd.i32();
      HIF_REQUIRE(nr >= 0 && k >= 0 && nr + k > 0, HIF_ERR_ARG, "bad edge sizes");
      rd.i32s(red, nr);
      rd.i32s(skel, k);
      rd.f64s(Tm, (size_t)k * nr);
      rd.f64s(Lm, (size_t)nr * nr);
      const int32_t any = nr ? red[0] : skel[0];
      auto it = where.find(any);
      HIF_REQUIRE(it != where.end(), HIF_ERR_ARG, "skeletonized edge is not a group");
      const int g = it->second.first;
      HIF_REQUIRE((int)groups[g].ids.size() == nr + k, HIF_ERR_ARG, "edge/group size mismatch");
      Sk s;
      s.nr = nr;
      s.k = k;
      for (int32_t d : red) {
        auto w = where.find(d);
        HIF_REQUIRE(w != where.end() && w->second.first == g, HIF_ERR_ARG, "edge DOF mismatch");
        s.perm.push_back(w->second.second);
      }
      for (int32_t d : skel) {
        auto w = where.find(d);
        HIF_REQUIRE(w != where.end() && w->second.first == g, HIF_ERR_ARG, "edge DOF mismatch");
        s.perm.push_back(w->second.second);
      }
      s.T.resize((size_t)k * nr);
      for (int j = 0; j < nr; ++j)
        for (int r = 0; r < k; ++r) s.T[(size_t)j * k + r] = Tm[(size_t)r * nr + j];
      if (nr) s.Lsinv = tri_inverse(Lm, nr);
      sk[g] = std::move(s);
    }
    // gather map: contributions aimed at every group DOF, in cell order
    std::vector<std::vector<std::vector<int32_t>>> slots(ngroup);
    for (int g = 0; g < ngroup; ++g) slots[g].resize(groups[g].ids.size());
    for (const CellB& c : cellB)
      for (size_t b = 0; b < c.B.size(); ++b) {
        auto w = where.find(c.B[b]);
        HIF_REQUIRE(w != where.end(), HIF_ERR_ARG, "cell boundary DOF is not in a group");
        slots[w->second.first][w->second.second].push_back((int32_t)(c.off + b));
      }
    for (int g = 0; g < ngroup; ++g) {
      const int gn = (int)groups[g].ids.size();
      int64_t nsl = 0;
      for (int i = 0; i < gn; ++i) nsl += (int64_t)slots[g][i].size();
      lh.group_slots.push_back(nsl);
      GroupDesc d{};
      d.n = gn;
      d.nr = sk[g].nr;
      d.offIdx = (int32_t)fh.idx.size();
      fh.idx.insert(fh.idx.end(), groups[g].ids.begin(), groups[g].ids.end());
      d.offPerm = (int32_t)fh.idx.size();
      if (d.nr) {
        fh.idx.insert(fh.idx.end(), sk[g].perm.begin(), sk[g].perm.end());
      }
      d.offGP = (int32_t)fh.idx.size();
      int32_t acc = 0;
      fh.idx.push_back(0);
      for (int i = 0; i < gn; ++i) {
        acc += (int32_t)slots[g][i].size();
        fh.idx.push_back(acc);
      }
      for (int i = 0; i < gn; ++i)
        fh.idx.insert(fh.idx.end(), slots[g][i].begin(), slots[g][i].end());
      fh.vals.resize(align_vals((int64_t)fh.vals.size()), 0.0);
      d.offV = (int32_t)fh.vals.size();
      push_packed(fh.vals, groups[g].Linv, gn);
      if (d.nr) {
        fh.vals.insert(fh.vals.end(), sk[g].T.begin(), sk[g].T.end());
        push_packed(fh.vals, sk[g].Lsinv, d.nr);
      }
      fh.nvals_used += tri_count(gn) + (int64_t)(gn - d.nr) * d.nr + tri_count(d.nr);
      d.cap = (int32_t)(tri_count(gn) + (int64_t)(gn - d.nr) * d.nr + tri_count(d.nr));
      lh.maxG = std::max(lh.maxG, gn);
      lh.maxR = std::max(lh.maxR, d.nr);
      lh.maxK = std::max(lh.maxK, gn - d.nr);
      lh.maxGV = std::max<int>(lh.maxGV, (int)(tri_count(gn) + (int64_t)(gn - d.nr) * d.nr +
                                               tri_count(d.nr)));
      lh.groups.push_back(d);
    }
    fh.lv.push_back(std::move(lh));
  }
  const int nroot = rd.i32();
  HIF_REQUIRE(nroot >= 0, HIF_ERR_ARG, "bad root size");
  rd.i32s(ids, nroot);
  check_ids(ids);
  rd.f64s(Lm, (size_t)nroot * nroot);
  fh.nroot = nroot;
  fh.offRootIdx = (int32_t)fh.idx.size();
  fh.idx.insert(fh.idx.end(), ids.begin(), ids.end());
  fh.vals.resize(align_vals((int64_t)fh.vals.size()), 0.0);
  fh.offRootV = (int64_t)fh.vals.size();
  if (nroot) push_packed(fh.vals, tri_inverse(Lm, nroot), nroot);
  fh.nvals_used += tri_count(nroot);
  HIF_REQUIRE(rd.pos == rd.n, HIF_ERR_ARG, "trailing bytes in HIFB blob");
  HIF_REQUIRE(fh.vals.size() < (size_t)INT32_MAX && fh.idx.size() < (size_t)INT32_MAX,
              HIF_ERR_ARG, "factor too large for 32-bit offsets");
  return fh;
}

void upload_factor(const FactorHost& fh, hif_store_t store, FactorDev& fd, hipStream_t s) {
  fd.store = store;
  fd.lv.clear();
  fd.lv.resize(fh.lv.size());
  for (size_t l = 0; l < fh.lv.size(); ++l) {
    const LevelHost& lh = fh.lv[l];
    LevelDev& ld = fd.lv[l];
    ld.ncell = (int)lh.cells.size();
    ld.ngroup = (int)lh.groups.size();
    ld.maxI = lh.maxI;
    ld.maxB = lh.maxB;
    ld.maxG = lh.maxG;
    ld.maxK = lh.maxK;
    ld.maxR = lh.maxR;
    ld.maxCV = lh.maxCV;
    ld.maxGV = lh.maxGV;
    ld.cmode = 0;
    level_stage_bytes(lh.cells, lh.groups, lh.group_slots, store_elem_bytes(store), ld);
    ld.cells.upload(lh.cells, s);
    ld.groups.upload(lh.groups, s);
  }
  fd.idx.upload(fh.idx, s);
  fd.nvals = fh.nvals_used;
  const size_t eb = store_elem_bytes(store);
  std::vector<unsigned char> raw((fh.vals.size() + kValAlign) * eb, 0);
  for (size_t i = 0; i < fh.vals.size(); ++i) {
    if (store == HIF_STORE_F64) {
      std::memcpy(&raw[i * 8], &fh.vals[i], 8);
    } else if (store == HIF_STORE_F32) {
      const float f = (float)fh.vals[i];
      std::memcpy(&raw[i * 4], &f, 4);
    } else {
      const uint16_t b = f32_to_bf16_bits((float)fh.vals[i]);
      std::memcpy(&raw[i * 2], &b, 2);
    }
  }
  fd.vals.upload(raw, s);
  fd.nroot = fh.nroot;
  fd.root_bytes = (int64_t)eb * tri_count(fh.nroot) + 20 * (int64_t)fh.nroot;
  fd.offRootIdx = fh.offRootIdx;
  fd.offRootV = fh.offRootV;
  fd.cbstride = std::max<int64_t>(1, fh.cbmax);
  fd.cb.alloc(2 * fd.cbstride);
  {
    std::vector<std::vector<CellDesc>> cells;
    std::vector<std::vector<GroupDesc>> groups;
    int64_t N = 0;  // one past the largest DOF id
    for (const LevelHost& lh : fh.lv) {
      cells.push_back(lh.cells);
      groups.push_back(lh.groups);
      for (const CellDesc& c : lh.cells)
        for (int i = 0; i < c.nI + c.nB; ++i)
          N = std::max<int64_t>(N, fh.idx[(i < c.nI ? c.offI + i : c.offB + i - c.nI)] + 1);
      for (const GroupDesc& g : lh.groups)
        for (int i = 0; i < g.n; ++i) N = std::max<int64_t>(N, fh.idx[g.offIdx + i] + 1);
    }
    for (int i = 0; i < fh.nroot; ++i) N = std::max<int64_t>(N, fh.idx[fh.offRootIdx + i] + 1);
    setup_tiling(fd, cells, groups, fh.idx, s);
    setup_dense_groups(fd, groups, fh.idx, dense_top_level(fd, cells, groups), s);
    setup_fusion(fd, cells, groups, fh.idx, N, s);
    setup_dense_top(fd, cells, groups, fh.idx, N, s);
    setup_cg_gate(fd, cells, fh.idx, N, s);
  }
  size_t worst = 0;
  apply_smem_need(fd, &worst);
  fd.smem_max = worst;
  HIF_REQUIRE(worst <= 160 * 1024, HIF_ERR_ARG, "factor blocks too large for the LDS-staged apply");
  if (worst > 64 * 1024) set_apply_smem_limits(worst);
  HIF_CHECK(hipStreamSynchronize(s));
}

}  // namespace hifcn
