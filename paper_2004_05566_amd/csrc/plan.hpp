// Host-side structure of one level of the PHIF build (Sec. 2.2): the quad/oct-tree cells and
// separator groups of the active DOFs, the boundary of every cell, and the table of dense
// blocks that can be non-zero in the active matrix.
//
// Partition: L = max{l : m 2^l <= n+1}; separator coordinates S_l = {k m 2^l : 1 <= k <=
// 2^(L-l) - 1} per axis (1-based node indices).  An active DOF with c coordinates in S_l is a
// cell interior (c = 0), an edge/face (c = 1), a corner (2D, c = 2) or a 3D edge (c = 2) or
// corner (c = 3).  For n = 2^L m - 1 this is the paper's layout; otherwise the last cell per
// axis absorbs the extra nodes.
#pragma once

#include <cstdint>
#include <algorithm>
#include <vector>

namespace hifcn {

struct PGroup {
  uint64_t key;                // per axis 21 bits: (on_separator << 20) | value
  int kind;                    // number of axes on a separator (0 = cell interior)
  std::vector<int32_t> dofs;   // global DOF ids, in group order
};

// Where a DOF of a level-(l+1) group came from at level l (for assembling its blocks).
struct RowSrc {
  int32_t sub;   // index of the level-l group among the sub-groups of the new group
  int32_t pos;   // position of the DOF in that level-l group's full order
  int32_t spos;  // position among the level-l group's surviving DOFs
};

struct LevelPlan {
  int level = 0;
  std::vector<PGroup> groups;                 // sorted by key
  std::vector<int> cells;                     // groups of kind 0
  std::vector<int> seps;                      // groups of kind > 0
  std::vector<int> skel;                      // skeletonized groups (Geometry::skeletonized)
  std::vector<std::vector<int>> cellB;        // per cell: boundary groups coupled to it
  // dense blocks (g, h) that may be non-zero: every ordered pair inside a cell closure
  std::vector<std::pair<int, int>> blocks;
  std::vector<uint64_t> block_keys;           // (g << 32 | h) of each block, ascending
  std::vector<int64_t> block_off;             // value offsets (row-major |g| x |h|)
  std::vector<int32_t> block_row;             // blocks of group g: [block_row[g], block_row[g+1])
  int64_t nvals = 0;
  // provenance of each group's DOFs from the previous level (empty at level 0)
  std::vector<std::vector<int>> subs;         // per group: previous-level groups, in order
  std::vector<std::vector<RowSrc>> rows;      // per group: one entry per DOF

  int find_block(int g, int h) const {
    const uint64_t k = ((uint64_t)(uint32_t)g << 32) | (uint32_t)h;
    auto lo = block_keys.begin(), hi = block_keys.end();
    if (g >= 0 && (size_t)g + 1 < block_row.size()) {  // search only the blocks of row g
      lo = block_keys.begin() + block_row[g];
      hi = block_keys.begin() + block_row[g + 1];
    }
    auto it = std::lower_bound(lo, hi, k);
    return (it == hi || *it != k) ? -1 : (int)(it - block_keys.begin());
  }
};

struct Geometry {
  int dim, n, m, L;
  bool skel_edges = false;  // 3D: edges skeletonized too
  // Groups that step (3) skeletonizes: kind 1 (2D edges, 3D faces), and 3D edges (kind 2)
  // with skel_edges.
  bool skeletonized(int kind) const { return kind == 1 || (skel_edges && dim == 3 && kind == 2); }
  int step(int lev) const { return m << lev; }
  int nsep(int lev) const { return lev >= L ? 0 : (1 << (L - lev)) - 1; }
  void coords(int32_t id, int c[3]) const {  // 1-based (x, y, z)
    c[0] = id % n + 1;
    c[1] = (id / n) % n + 1;
    c[2] = dim == 3 ? id / (n * n) + 1 : 0;
  }
  uint64_t key(int32_t id, int lev, int* kind) const;
  // Dense index of a group key at level lev: per axis the rank of the coordinate class (the
  // 2 nsep + 1 classes interval 0..nsep, then separator 1..nsep), slowest axis most
  // significant, so that slots ascend with keys.
  int64_t slot(uint64_t key, int lev) const;
  int64_t nslots(int lev) const;
};

// Level-0 plan: every DOF is active, groups ordered by key, DOFs by id.
LevelPlan plan_level0(const Geometry& geo);

// Plan of level l+1 from the surviving DOFs of level l's separator groups, given in the order of
// those groups; `surv[g]` lists positions (in group g's order) that survive; every group of
// level l+1 is the concatenation of the surviving DOFs of its sub-groups in that order.
LevelPlan plan_next(const Geometry& geo, const LevelPlan& prev,
                    const std::vector<std::vector<int32_t>>& surv);

}  // namespace hifcn
