// Host-side level structure of the PHIF build (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <numeric>

#include "errors.hpp"

namespace hifcn {

uint64_t Geometry::key(int32_t id, int lev, int* kind) const {
  int c[3];
  coords(id, c);
  const int st = step(lev), ns = nsep(lev);
  uint64_t k = 0;
  int kd = 0;
  for (int a = 0; a < dim; ++a) {
    const int x = c[a];
    const bool on = ns > 0 && x % st == 0 && x / st >= 1 && x / st <= ns;
    uint64_t v;
    if (on) {
      v = (1ull << 20) | (uint64_t)x;
      ++kd;
    } else {
      v = (uint64_t)std::min((x - 1) / st, ns);  // number of separators below x
    }
    // the slowest axis goes to the high bits so that keys sort like grid positions
    k |= v << (21 * a);
  }
  *kind = kd;
  return k;
}

int64_t Geometry::slot(uint64_t key, int lev) const {
  const int st = step(lev), ns = nsep(lev), R = 2 * ns + 1;
  int64_t sl = 0, mul = 1;
  for (int a = 0; a < dim; ++a) {
    const uint64_t v = (key >> (21 * a)) & ((1ull << 21) - 1);
    const int on = (int)(v >> 20), val = (int)(v & ((1ull << 20) - 1));
    sl += mul * (on ? ns + val / st : val);
    mul *= R;
  }
  return sl;
}

int64_t Geometry::nslots(int lev) const {
  const int64_t R = 2 * nsep(lev) + 1;
  int64_t t = 1;
  for (int a = 0; a < dim; ++a) t *= R;
  return t;
}

namespace {

void decode(uint64_t key, int dim, int on[3], int val[3]) {
  for (int a = 0; a < dim; ++a) {
    const uint64_t v = (key >> (21 * a)) & ((1ull << 21) - 1);
    on[a] = (int)(v >> 20);
    val[a] = (int)(v & ((1ull << 20) - 1));
  }
}

uint64_t encode(int dim, const int on[3], const int val[3]) {
  uint64_t k = 0;
  for (int a = 0; a < dim; ++a)
    k |= ((uint64_t)on[a] << 20 | (uint64_t)val[a]) << (21 * a);
  return k;
}

// Sort groups by key (carrying provenance), then derive cells, separators, boundaries, blocks.
void finish_plan(const Geometry& geo, LevelPlan& P) {
  const int G = (int)P.groups.size();
  std::vector<int> order(G);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return P.groups[a].key < P.groups[b].key; });
  {
    std::vector<PGroup> g2(G);
    std::vector<std::vector<int>> s2;
    std::vector<std::vector<RowSrc>> r2;
    const bool prov = !P.subs.empty();
    if (prov) {
      s2.resize(G);
      r2.resize(G);
    }
    for (int i = 0; i < G; ++i) {
      g2[i] = std::move(P.groups[order[i]]);
      if (prov) {
        s2[i] = std::move(P.subs[order[i]]);
        r2[i] = std::move(P.rows[order[i]]);
      }
    }
    P.groups = std::move(g2);
    if (prov) {
      P.subs = std::move(s2);
      P.rows = std::move(r2);
    }
  }
  std::vector<int> gid(geo.nslots(P.level), -1);  // slot -> group
  for (int i = 0; i < G; ++i) gid[geo.slot(P.groups[i].key, P.level)] = i;
  P.cells.clear();
  P.seps.clear();
  P.skel.clear();
  for (int i = 0; i < G; ++i) {
    if (P.groups[i].kind == 0) P.cells.push_back(i);
    else P.seps.push_back(i);
    if (geo.skeletonized(P.groups[i].kind)) P.skel.push_back(i);
  }
  const int st = geo.step(P.level), ns = geo.nsep(P.level);
  P.cellB.assign(P.cells.size(), {});
  // partners of each group: every group sharing a cell closure with it
  std::vector<std::vector<int>> nbr(G);
  for (size_t ci = 0; ci < P.cells.size(); ++ci) {
    const int c = P.cells[ci];
    int on[3], val[3];
    decode(P.groups[c].key, geo.dim, on, val);
    // per axis: own interval, separator below, separator above
    int opts_on[3][3], opts_val[3][3], nopt[3];
    for (int a = 0; a < geo.dim; ++a) {
      nopt[a] = 0;
      opts_on[a][nopt[a]] = 0;
      opts_val[a][nopt[a]++] = val[a];
      if (val[a] >= 1) {
        opts_on[a][nopt[a]] = 1;
        opts_val[a][nopt[a]++] = val[a] * st;
      }
      if (val[a] < ns) {
        opts_on[a][nopt[a]] = 1;
        opts_val[a][nopt[a]++] = (val[a] + 1) * st;
      }
    }
    std::vector<int> closure{c};
    int idx[3] = {0, 0, 0};
    while (true) {
      int o[3] = {0, 0, 0}, v[3] = {0, 0, 0}, kd = 0;
      for (int a = 0; a < geo.dim; ++a) {
        o[a] = opts_on[a][idx[a]];
        v[a] = opts_val[a][idx[a]];
        kd += o[a];
      }
      if (kd > 0) {
        const int h = gid[geo.slot(encode(geo.dim, o, v), P.level)];
        if (h >= 0) {
          closure.push_back(h);
          // at level 0 a cell interior couples (through the stencil) only to faces/edges with a
          // single separator coordinate
          if (P.level > 0 || kd == 1) P.cellB[ci].push_back(h);
        }
      }
      int a = 0;
      while (a < geo.dim && ++idx[a] == nopt[a]) idx[a++] = 0;
      if (a == geo.dim) break;
    }
    std::sort(P.cellB[ci].begin(), P.cellB[ci].end());
    for (int g : closure) nbr[g].insert(nbr[g].end(), closure.begin(), closure.end());
  }
  // blocks in (g, h) order: per g its partners sorted and unique
  std::vector<uint64_t> pairs;
  for (int g = 0; g < G; ++g) {
    std::vector<int>& v = nbr[g];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    for (int h : v) pairs.push_back(((uint64_t)(uint32_t)g << 32) | (uint32_t)h);
  }
  P.blocks.resize(pairs.size());
  P.block_off.resize(pairs.size());
  int64_t off = 0;
  for (size_t b = 0; b < pairs.size(); ++b) {
    const int g = (int)(pairs[b] >> 32), h = (int)(pairs[b] & 0xffffffffu);
    P.blocks[b] = {g, h};
    P.block_off[b] = off;
    off += (int64_t)P.groups[g].dofs.size() * (int64_t)P.groups[h].dofs.size();
  }
  P.block_keys = std::move(pairs);
  P.block_row.assign(G + 1, 0);
  for (const auto& b : P.blocks) ++P.block_row[b.first + 1];
  for (int g = 0; g < G; ++g) P.block_row[g + 1] += P.block_row[g];
  P.nvals = off;
}

}  // namespace

LevelPlan plan_level0(const Geometry& geo) {
  LevelPlan P;
  P.level = 0;
  int64_t N = 1;
  for (int d = 0; d < geo.dim; ++d) N *= geo.n;
  std::vector<int> gid(geo.nslots(0), -1);  // slot -> group
  // per coordinate x = 1..n: its field of the key, its term of the slot, whether it lies on a
  // separator (Geometry::key and Geometry::slot, one axis at a time)
  const int n = geo.n, st = geo.step(0), ns = geo.nsep(0);
  const int64_t R = 2 * ns + 1;
  std::vector<uint64_t> kv(n + 1);
  std::vector<int64_t> sv(n + 1);
  std::vector<int> onv(n + 1);
  for (int x = 1; x <= n; ++x) {
    const bool on = ns > 0 && x % st == 0 && x / st >= 1 && x / st <= ns;
    kv[x] = on ? ((1ull << 20) | (uint64_t)x) : (uint64_t)std::min((x - 1) / st, ns);
    sv[x] = on ? ns + x / st : (int64_t)kv[x];
    onv[x] = on ? 1 : 0;
  }
  const int nz = geo.dim == 3 ? n : 1;
  int32_t id = 0;
  for (int z = 1; z <= nz; ++z) {
    const uint64_t kz = geo.dim == 3 ? kv[z] << 42 : 0;
    const int64_t sz = geo.dim == 3 ? sv[z] * R * R : 0;
    const int oz = geo.dim == 3 ? onv[z] : 0;
    for (int y = 1; y <= n; ++y)
      for (int x = 1; x <= n; ++x, ++id) {
        const uint64_t k = kv[x] | kv[y] << 21 | kz;
        int& g = gid[sv[x] + sv[y] * R + sz];
        if (g < 0) {
          g = (int)P.groups.size();
          P.groups.push_back({k, onv[x] + onv[y] + oz, {}});
        }
        P.groups[g].dofs.push_back(id);
      }
  }
  HIF_REQUIRE(id == N, HIF_ERR_ARG, "internal: level-0 DOF count");
  finish_plan(geo, P);
  return P;
}

LevelPlan plan_next(const Geometry& geo, const LevelPlan& prev,
                    const std::vector<std::vector<int32_t>>& surv) {
  LevelPlan P;
  P.level = prev.level + 1;
  std::vector<int> gid(geo.nslots(P.level), -1);  // slot -> group
  for (int g : prev.seps) {
    const PGroup& pg = prev.groups[g];
    const std::vector<int32_t>& sv = surv[g];
    int target = -1;
    for (size_t s = 0; s < sv.size(); ++s) {
      const int32_t dof = pg.dofs[sv[s]];
      int kind;
      const uint64_t k = geo.key(dof, P.level, &kind);
      int& G = gid[geo.slot(k, P.level)];
      if (G < 0) {
        G = (int)P.groups.size();
        P.groups.push_back({k, kind, {}});
        P.subs.emplace_back();
        P.rows.emplace_back();
      }
      HIF_REQUIRE(target < 0 || target == G, HIF_ERR_ARG,
                  "internal: a group split across two groups of the next level");
      target = G;
      if (P.subs[G].empty() || P.subs[G].back() != g) P.subs[G].push_back(g);
      P.groups[G].dofs.push_back(dof);
      P.rows[G].push_back({(int32_t)P.subs[G].size() - 1, sv[s], (int32_t)s});
    }
  }
  finish_plan(geo, P);
  return P;
}

}  // namespace hifcn
