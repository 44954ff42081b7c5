// Host check of the PHIF level planner (plan.hpp), built with the address and undefined-behaviour
// sanitizers by tests/test_host_asan.py.  For a set of 2D and 3D grids it plans every level and
// checks what the partition of Sec. 2.2 fixes:
//  - every active DOF lies in exactly one group, whose key and kind are the DOF's at that level;
//  - cells (kind 0) are independent: no stencil coupling joins two cells;
//  - at level 0 every coupling of the 5/7-point stencil (Sec. 2) falls in a planned block, and a
//    cell's neighbours outside it lie in its boundary groups;
//  - above level 0 every pair of surviving DOFs that shared a cell closure one level down (the
//    fill of eliminating that cell, eq2_3), and every block between surviving separators, falls
//    in a planned block;
//  - block offsets, row ranges and lookups agree; the provenance of each DOF is exact;
//  - the top level is one group holding every survivor.
// Survivors of a skeletonized group are every other DOF (a stand-in for the ID's choice: the
// planner takes any subset).  Prints one line per grid; exits non-zero on the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "plan.hpp"

using namespace hifcn;

namespace {

int fails = 0;

#define CHECK(cond, ...)                              \
  do {                                                \
    if (!(cond)) {                                    \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);              \
      std::fprintf(stderr, "\n");                     \
      ++fails;                                        \
      return false;                                   \
    }                                                 \
  } while (0)

int level_count(int n, int m) {
  int L = 0;
  while ((int64_t)m << (L + 1) <= n + 1) ++L;
  return L;
}

// Stencil neighbours of DOF i (x fastest, 0-based ids, zero Dirichlet data outside the grid).
void neighbours(const Geometry& geo, int32_t i, std::vector<int32_t>& out) {
  out.clear();
  int c[3];
  geo.coords(i, c);
  const int64_t n = geo.n, stride[3] = {1, n, n * n};
  for (int a = 0; a < geo.dim; ++a) {
    if (c[a] > 1) out.push_back(i - (int32_t)stride[a]);
    if (c[a] < geo.n) out.push_back(i + (int32_t)stride[a]);
  }
}

// The structure shared by every level: groups, keys, cells, separators, blocks.
bool check_level(const Geometry& geo, const LevelPlan& P, const std::vector<int32_t>& active,
                 int64_t N, std::vector<int>& owner, std::vector<int>& pos) {
  owner.assign(N, -1);
  pos.assign(N, -1);
  const int G = (int)P.groups.size();
  int64_t count = 0;
  for (int g = 0; g < G; ++g) {
    const PGroup& pg = P.groups[g];
    CHECK(!pg.dofs.empty(), "level %d group %d is empty", P.level, g);
    if (g > 0) CHECK(P.groups[g - 1].key < pg.key, "level %d groups not sorted at %d", P.level, g);
    for (size_t k = 0; k < pg.dofs.size(); ++k) {
      const int32_t d = pg.dofs[k];
      CHECK(d >= 0 && d < N, "level %d dof %d out of range", P.level, d);
      CHECK(owner[d] < 0, "level %d dof %d in groups %d and %d", P.level, d, owner[d], g);
      owner[d] = g;
      pos[d] = (int)k;
      int kind;
      CHECK(geo.key(d, P.level, &kind) == pg.key && kind == pg.kind,
            "level %d dof %d: key/kind differ from its group %d", P.level, d, g);
      ++count;
    }
  }
  CHECK(count == (int64_t)active.size(), "level %d: %lld DOFs planned, %zu active", P.level,
        (long long)count, active.size());
  for (int32_t d : active) CHECK(owner[d] >= 0, "level %d: active dof %d in no group", P.level, d);
  // cells, separators, skeletonized groups
  std::vector<int> cells, seps, skel;
  for (int g = 0; g < G; ++g) {
    (P.groups[g].kind == 0 ? cells : seps).push_back(g);
    if (geo.skeletonized(P.groups[g].kind)) skel.push_back(g);
  }
  CHECK(cells == P.cells && seps == P.seps && skel == P.skel, "level %d: group classes",
        P.level);
  CHECK(P.cellB.size() == P.cells.size(), "level %d: cellB size", P.level);
  // blocks: offsets, rows, lookups
  CHECK(P.blocks.size() == P.block_keys.size() && P.blocks.size() == P.block_off.size(),
        "level %d: block table sizes", P.level);
  CHECK((int)P.block_row.size() == G + 1 && P.block_row[0] == 0 &&
            P.block_row[G] == (int32_t)P.blocks.size(),
        "level %d: block rows", P.level);
  int64_t off = 0;
  for (size_t b = 0; b < P.blocks.size(); ++b) {
    const int g = P.blocks[b].first, h = P.blocks[b].second;
    CHECK(g >= 0 && g < G && h >= 0 && h < G, "level %d block %zu: groups", P.level, b);
    CHECK(P.block_keys[b] == (((uint64_t)(uint32_t)g << 32) | (uint32_t)h),
          "level %d block %zu: key", P.level, b);
    if (b > 0) CHECK(P.block_keys[b - 1] < P.block_keys[b], "level %d: block order", P.level);
    CHECK((int)b >= P.block_row[g] && (int)b < P.block_row[g + 1], "level %d block %zu: row",
          P.level, b);
    CHECK(P.block_off[b] == off, "level %d block %zu: offset", P.level, b);
    off += (int64_t)P.groups[g].dofs.size() * (int64_t)P.groups[h].dofs.size();
    CHECK(P.find_block(g, h) == (int)b, "level %d: find_block(%d, %d)", P.level, g, h);
    CHECK(P.find_block(h, g) >= 0, "level %d: block (%d, %d) without its transpose", P.level, g,
          h);
  }
  CHECK(P.nvals == off, "level %d: nvals", P.level);
  for (size_t ci = 0; ci < P.cells.size(); ++ci) {
    const int c = P.cells[ci];
    CHECK(P.find_block(c, c) >= 0, "level %d: no diagonal block for cell %d", P.level, c);
    for (int h : P.cellB[ci]) {
      CHECK(h >= 0 && h < G && P.groups[h].kind > 0, "level %d: cell %d boundary %d", P.level,
            c, h);
      CHECK(P.find_block(c, h) >= 0, "level %d: no block (cell %d, boundary %d)", P.level, c, h);
    }
    for (size_t cj = ci + 1; cj < P.cells.size(); ++cj)
      CHECK(P.find_block(c, P.cells[cj]) < 0, "level %d: block between cells %d and %d",
            P.level, c, P.cells[cj]);
  }
  return true;
}

bool check_level0(const Geometry& geo, const LevelPlan& P, int64_t N, std::vector<int>& owner,
                  std::vector<int>& pos) {
  std::vector<int32_t> all(N);
  for (int64_t i = 0; i < N; ++i) all[i] = (int32_t)i;
  if (!check_level(geo, P, all, N, owner, pos)) return false;
  std::vector<int> cell_index(P.groups.size(), -1);
  for (size_t ci = 0; ci < P.cells.size(); ++ci) cell_index[P.cells[ci]] = (int)ci;
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < N; ++i) {
    const int g = owner[i];
    neighbours(geo, (int32_t)i, nb);
    for (int32_t j : nb) {
      const int h = owner[j];
      CHECK(P.find_block(g, h) >= 0, "level 0: coupling %lld-%d outside the blocks", (long long)i,
            j);
      if (g != h && cell_index[g] >= 0) {
        CHECK(P.groups[h].kind > 0, "level 0: cells %d and %d touch", g, h);
        const auto& B = P.cellB[cell_index[g]];
        CHECK(std::find(B.begin(), B.end(), h) != B.end(),
              "level 0: neighbour group %d of cell %d not in its boundary", h, g);
      }
    }
  }
  return true;
}

// Level l+1 from level l with every other DOF of each skeletonized group surviving.
bool check_next(const Geometry& geo, const LevelPlan& prev, const std::vector<int>& prev_owner,
                int64_t N, LevelPlan& next, std::vector<int>& owner, std::vector<int>& pos) {
  std::vector<std::vector<int32_t>> surv(prev.groups.size());
  std::vector<int32_t> active;
  for (int g : prev.seps) {
    const int sz = (int)prev.groups[g].dofs.size();
    const int step = geo.skeletonized(prev.groups[g].kind) && sz > 1 ? 2 : 1;
    for (int k = 0; k < sz; k += step) {
      surv[g].push_back(k);
      active.push_back(prev.groups[g].dofs[k]);
    }
  }
  next = plan_next(geo, prev, surv);
  if (!check_level(geo, next, active, N, owner, pos)) return false;
  // provenance
  CHECK(next.subs.size() == next.groups.size() && next.rows.size() == next.groups.size(),
        "level %d: provenance sizes", next.level);
  for (size_t G = 0; G < next.groups.size(); ++G) {
    const auto& dofs = next.groups[G].dofs;
    CHECK(next.rows[G].size() == dofs.size(), "level %d group %zu: rows", next.level, G);
    for (size_t k = 0; k < dofs.size(); ++k) {
      const RowSrc rs = next.rows[G][k];
      CHECK(rs.sub >= 0 && rs.sub < (int)next.subs[G].size(), "level %d: row sub", next.level);
      const int g = next.subs[G][rs.sub];
      CHECK(prev.groups[g].dofs[rs.pos] == dofs[k] && prev_owner[dofs[k]] == g,
            "level %d group %zu dof %zu: provenance", next.level, G, k);
      CHECK(rs.spos >= 0 && rs.spos < (int)surv[g].size() && surv[g][rs.spos] == rs.pos,
            "level %d group %zu dof %zu: survivor position", next.level, G, k);
    }
  }
  // fill of each eliminated cell: its closure's survivors are coupled one level up
  for (size_t ci = 0; ci < prev.cells.size(); ++ci) {
    std::vector<int32_t> sv;
    for (int h : prev.cellB[ci])
      for (int k : surv[h]) sv.push_back(prev.groups[h].dofs[k]);
    for (int32_t a : sv)
      for (int32_t b : sv)
        CHECK(next.find_block(owner[a], owner[b]) >= 0,
              "level %d: fill of cell %d between dofs %d and %d not in a block", next.level,
              prev.cells[ci], a, b);
  }
  // couplings already present between surviving separators stay in blocks
  for (const auto& bl : prev.blocks) {
    const int g = bl.first, h = bl.second;
    if (prev.groups[g].kind == 0 || prev.groups[h].kind == 0) continue;
    for (int ka : surv[g])
      for (int kb : surv[h]) {
        const int32_t a = prev.groups[g].dofs[ka], b = prev.groups[h].dofs[kb];
        CHECK(next.find_block(owner[a], owner[b]) >= 0,
              "level %d: coupling %d-%d of level %d lost", next.level, a, b, prev.level);
      }
  }
  return true;
}

bool run(int dim, int n, int m, bool edges) {
  Geometry geo{dim, n, m, level_count(n, m)};
  geo.skel_edges = edges;
  int64_t N = 1;
  for (int d = 0; d < dim; ++d) N *= n;
  std::vector<int> owner, pos, owner2, pos2;
  LevelPlan P = plan_level0(geo);
  if (!check_level0(geo, P, N, owner, pos)) return false;
  for (int l = 0; l < geo.L; ++l) {
    LevelPlan Pn;
    if (!check_next(geo, P, owner, N, Pn, owner2, pos2)) return false;
    P = std::move(Pn);
    owner.swap(owner2);
    pos.swap(pos2);
  }
  CHECK(P.level == geo.L && P.groups.size() == 1 && P.groups[0].kind == 0 && P.seps.empty(),
        "top level %d: %zu groups, %zu separators", P.level, P.groups.size(), P.seps.size());
  std::printf("ok dim=%d n=%d m=%d L=%d edges=%d top=%zu\n", dim, n, m, geo.L, edges ? 1 : 0,
              P.groups[0].dofs.size());
  return true;
}

}  // namespace

int main() {
  struct Case { int dim, n, m; bool edges; };
  const Case cases[] = {
      {2, 7, 2, false},   {2, 15, 4, false},  {2, 31, 4, false}, {2, 33, 4, false},
      {2, 63, 8, false},  {2, 64, 8, false},  {2, 100, 8, false}, {2, 127, 8, false},
      {3, 7, 2, false},   {3, 15, 4, false},  {3, 16, 4, false}, {3, 15, 4, true},
      {3, 31, 4, false},  {3, 31, 4, true},
  };
  for (const Case& c : cases)
    if (!run(c.dim, c.n, c.m, c.edges)) break;
  if (fails) return 1;
  std::printf("all plans ok\n");
  return 0;
}
