// Internal interfaces between the translation units of the hifcn library.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace hifcn {

struct LevelPlan;

// One level of the factor as the apply kernels read it.
struct LevelDev {
  int ncell = 0, ngroup = 0;
  int maxI = 0, maxB = 0;            // largest cell interior / boundary
  int maxG = 0, maxK = 0, maxR = 0;  // largest group, skeleton and redundant set
  int maxCV = 0, maxGV = 0;          // largest cell / group value block (elements)
  int cmode = 0;                     // coupling mode of every cell of the level (CellDesc.mode)
  int64_t cell_bytes[2] = {0, 0};    // algorithmic bytes per launch: [forward, backward]
  int64_t group_bytes[2] = {0, 0};
  DevBuf<CellDesc> cells;
  DevBuf<GroupDesc> groups;
  // Cells too large for one workgroup are tiled: row tiles and column tiles of 64 / 16
  // (cell, first row or column, scratch offset of the cell's interior, unused).
  bool tiled = false;
  int tthreads = 1024;               // workgroup size of the tiles (256, 512 or 1024)
  int nrt = 0, nct = 0;
  DevBuf<int4> rtiles, ctiles;
  // Blocks that one workgroup cannot hold are applied in dense form (FactorDev::dvals), spread
  // over many workgroups: link-mode cells of tiled levels (cdense: A_II^-1, row tiles) and the
  // groups of gtiled levels (the whole group step G: row tiles forward, column tiles backward,
  // results written back from the scratch vector by a scatter list).  Tiles: (block, first row
  // or column, first column of the tile's range, scratch offset); ddoff: dvals offset per block.
  bool cdense = false, gtiled = false;
  int ncdt = 0, ngrt = 0, ngct = 0, ngsc = 0;
  DevBuf<int4> cdtiles, grtiles, gctiles, gscat;
  DevBuf<int64_t> cddoff, gddoff;
  // The group stage of this level runs in one launch with the cell stage of the next level:
  // owned = the descriptors of the groups each next-level cell runs, maxown per cell (padded
  // with empty descriptors).
  bool fuse = false;
  int maxown = 0;
  // Block records (descriptor with record-relative offsets, then its index lists), fixed
  // stride in int32 per block: cells, groups, and (fused levels) each next-level cell's record
  // followed by those of the groups it owns.
  DevBuf<int32_t> crec, grec, frec;
  int cstride = 0, gstride = 0, fstride = 0;
  int cfwd = 0;  // int32 of each cell record the forward stage reads (descriptor, I, couplings)
  // symmetric-inverse cells (cmode 2): cells of at most sqn interior DOFs go to an LDS square of
  // leading dimension sqld (odd), larger ones stay packed; sqmat: LDS elements for either
  int sqn = 0, sqld = 0, sqmat = 0;
  int sqoff = 0;  // start of order sqn's entries in f.sqtab (its header entry, kept on the host)
  std::vector<int32_t> sqhead;  // f.sqtab's header on the host (written into the records)
  // group stages as one dense product G (forward) / G^T (backward) per group (setup_dense_groups)
  int gdense = 0;
};

// Stages of one apply, as timed by the profiler.
enum { STAGE_CELL_FWD = 0, STAGE_GROUP_FWD = 1, STAGE_ROOT = 2, STAGE_GROUP_BWD = 3,
       STAGE_CELL_BWD = 4 };

// HIP-event timing of every launch of one (level, stage) of the apply.
struct StageProfiler {
  bool enabled = false;
  int level = 0, stage = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  DevBuf<int32_t> live;   // per pending launch: 1 if the kernel did work (0: early exit)
  int64_t launches = 0;
  double ms = 0;
  const char* kernel = "";  // the kernel of the last timed launch (set by its launch site)
  hipEvent_t next_event() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIF_CHECK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~StageProfiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// The factor in its apply layout: per-level descriptors, one int32 index array and one value
// array in the storage precision.
struct FactorDev {
  hif_store_t store = HIF_STORE_F64;
  std::vector<LevelDev> lv;
  DevBuf<int32_t> idx;
  DevBuf<unsigned char> vals;
  int64_t nvals = 0;       // stored elements actually used (unpadded)
  int nroot = 0;
  int32_t offRootIdx = 0;  // root DOF ids in idx
  int64_t offRootV = 0;    // packed L_r^-1 in vals
  DevBuf<double> cb;       // boundary contributions of the cell stage: two halves of cbstride,
  int64_t cbstride = 0;    //   level l uses half l % 2 (consecutive levels may run together)
  bool root_fused = false; // last level's groups, root and backward groups in one launch
  size_t smem_max = 0;
  int64_t root_bytes = 0;
  std::unique_ptr<StageProfiler> prof;
  DevBuf<double> wsc;   // interiors of tiled cells between the forward and backward sweep,
                        // then the results of dense group and root stages within one stage
  // Dense forms (column-major, leading dimension a multiple of 32, storage precision).
  DevBuf<unsigned char> dvals;
  int64_t ndvals = 0;
  // A root of more than 256 KiB is applied as M = L_r^-T L_r^-1 in dense form: row tiles over
  // column ranges of rspan, partial sums added up by the scatter list.
  bool root_tiled = false;
  int rspan = 0, nrdt = 0, nrsc = 0;
  DevBuf<int64_t> rddoff;
  DevBuf<int4> rdtiles, rscat;
  // Dense top: the stages from the group step of level `top` up to the root and back, applied
  // as one symmetric matrix on that level's group DOFs (tvals, column-major, leading dimension
  // ntop rounded up to 32); -1: none.  Inputs: DOF ids (tgid) less the contributions in the
  // slots tgslot[i * tkslot ..] (-1: none); ntdt workgroups of row tiles over column ranges of
  // tspan, partial sums in twsc added up by the write-back list tscat.
  int64_t top_budget = -1;  // entries allowed (set before the build; < 0: default)
  bool skel_edges = false;  // 3D: edges skeletonized as well as faces (set before the build)
  int top = -1, ntop = 0, tspan = 0, ntdt = 0, ntsc = 0, tkslot = 0;
  int64_t top_bytes = 0;
  DevBuf<unsigned char> tvals;
  DevBuf<int32_t> tgid, tgslot;
  DevBuf<int4> tscat;
  DevBuf<double> twsc;
  // tfold: the backward cell stage of level `top` takes its boundary values from the partial
  // sums (and writes them to y) instead of a write-back launch; tpos: per cell of that level,
  // the top position of each boundary DOF (stride tpstride)
  bool tfold = false;
  int tpstride = 0;
  DevBuf<int32_t> tpos;
  // gate: the level-0 cell stage can run the PCG convergence test (CgGate); gcopy: per cell, a
  // count and the DOFs outside every level-0 interior that it copies from the input (stride
  // gcstride), each such DOF in exactly one list
  bool gate = false;
  int gcstride = 0;
  int64_t gate_n = 0;  // DOFs the copy lists cover (0 .. gate_n-1)
  DevBuf<int32_t> gcopy;
  // factor build on the matrix cores (front path): algorithmic FP64 flops, kernel time
  int64_t mfma_flops = 0;
  double mfma_ms = 0;
  // symmetric-inverse cells (CellDesc.mode 2): for every interior size n up to the level's
  // square order sqn, the two LDS square positions (column-major, leading dimension sqld) of
  // per interior order up to sqn (after a header of kSymTabHead starts), in the blocks' storage
  // order: the two square positions (j sqld + i) | (i sqld + j) << 16 of each element, a spare
  // word (sqmat - 1, twice) for padding slots
  DevBuf<int32_t> sqtab;
};

// ---- batched apply over several solves (continuous batching) ----------------------------------
// One solve's part of a batched stage launch: its blocks are launch blocks first .. first +
// nblk - 1.  Cell and group stages read block records; the root reads its DOF ids (recs) and
// packed L_r^-1 (vals).
struct BatchArg {
  const int32_t* recs;
  const void* vals;
  double* y;
  double* cb;
  const int* done;
  const int32_t* sqtab;
  int32_t stride, len;   // record stride (int32) and the part of it one block reads
  int32_t count;         // cells or groups of the level, or the root's DOFs
  int32_t first;         // first launch block of this solve
  int32_t blk_elems, team, seg, per_group, staged;
  int32_t sqn, sqld, sqmat, sqoff;  // symmetric cells (LevelDev)
  int32_t gdense;            // group stages: one dense product per group (LevelDev)
};
enum BatchKind { BK_CELL_FWD_SYM = 0, BK_CELL_FWD = 1, BK_GROUP_FWD = 2, BK_ROOT = 3,
                 BK_GROUP_BWD = 4, BK_CELL_BWD_SYM = 5, BK_CELL_BWD = 6 };
// One launch of a batched apply: its arguments are args[off .. off + nslot) of the plan's array.
struct BatchLaunch {
  int kind = 0, off = 0, nslot = 0, blocks = 0, threads = 0, recmax = 0;
  size_t smem = 0;
};
struct BatchApplyPlan {
  std::vector<BatchLaunch> launches;
  StagedBuf<BatchArg> args;
  hif_store_t store = HIF_STORE_F32;
};
// Whether a factor can take part in a batched apply (2D or 3D, level 0 symmetric cells or none,
// no dense top, no tiled or dense-form levels, no tiled root).
bool batchable(const FactorDev& f);
// The launches of one apply of every factor in fs (all batchable, one storage precision): the
// stages of level l of all of them together, levels aligned from the leaves, then all roots,
// then the backward stages from the top level down.  y[i], done[i]: solve i's vector and stop
// flag (may be null).
void build_batch_apply(const std::vector<const FactorDev*>& fs, const std::vector<double*>& y,
                       const std::vector<const int*>& done, BatchApplyPlan& plan, hipStream_t s);
void run_batch_apply(const BatchApplyPlan& plan, hipStream_t s);

// ---- symmetric-inverse level-0 cells ---------------------------------------------------------
constexpr int kSymMaxCell = 64;  // largest interior held as A_II^-1 by one wavefront
// The LDS form of a symmetric cell stage: the table of square positions, the square order, its
// leading dimension (odd) and the LDS elements reserved for the block (the last one spare).
struct SymCfg {
  const int32_t* tab;
  int n, ld, mat;
  int sqoff;  // tab[n]: where the entries of the square's own order start
};
// In the records of a level of symmetric cells the descriptor's mode word holds the start of
// the cell's order's entries in the table (from the header; at least kSymTabHead), or -1 for a
// cell above the square's order (packed triangle).
// The table's header: entry n (1 <= n <= SymCfg::n) is where the entries of interior order n
// start (a multiple of 4).
constexpr int kSymTabHead = (kSymMaxCell + 1 + 3) / 4 * 4;
// HIFCN_NO_SYM_CELLS set: level-0 cells keep L^-1 (two triangular products per sweep).
bool sym_cells_off();
// Choose level 0's square order (the median interior size with 2048 cells or more, else the
// largest), leading dimension and LDS size for
// its symmetric cells, and upload f.sqtab for interiors of up to that order.
void build_sym_table(FactorDev& f, const std::vector<CellDesc>& cells, hipStream_t s);

// Host-side, FP64 version of the same layout (used by import; the GPU build writes the device
// arrays directly with the same descriptors).
struct LevelHost {
  std::vector<CellDesc> cells;
  std::vector<GroupDesc> groups;
  int maxI = 0, maxB = 0, maxG = 0, maxK = 0, maxR = 0, maxCV = 0, maxGV = 0;
  std::vector<int64_t> group_slots;  // contributions gathered by each group
};
struct FactorHost {
  std::vector<LevelHost> lv;
  std::vector<int32_t> idx;
  std::vector<double> vals;
  int nroot = 0;
  int32_t offRootIdx = 0;
  int64_t offRootV = 0;
  int64_t cbmax = 0;
  int64_t nvals_used = 0;  // stored values excluding alignment padding
};

// PCG state kept on the device (scalars of Algorithm 1's pcg).
struct CgState {
  double gg;      // ||g||^2
  double tol2;    // rtol^2 ||g||^2
  double rzv[2];  // rho = r.z of direction it, in slot it & 1 (kept by the update)
  double pqv[2];  // p.Ap of direction it, in slot it & 1
  double rr;      // ||r||^2 after the latest update
  int32_t iters, done, status, maxit;
  // hold: set by the right-hand side of a step queued ahead of the previous step's outcome when
  // that step did not end well (it goes on, or failed); the step's test of g then sets done, so
  // the rest of it does nothing; cleared by the next right-hand side or by the resume of the
  // previous step
  int32_t hold;
  int32_t ok_next;  // the closing test's verdict for a step queued behind: it ended well
};

// A convergence test of the PCG run by the first stage of a preconditioner apply instead of its
// own launch: the verdict comes from the partial sums (part, nb of them) of ||g||^2 (init) or
// ||r||^2 after iteration it0; when the iteration goes on, the apply reads its input from src (r)
// and its output vector receives r's values wherever the apply does not overwrite them.
struct CgGate {
  CgState* st = nullptr;
  const double* part = nullptr;
  int nb = 0, init = 0, it0 = 0, maxit = 0;
  double rtol = 0;
  const double* src = nullptr;
};

// The right-hand side of a step made by the first stage of its first apply (hif_apply_rhs):
// the stencil (u, link weights, grid), the reaction, the outputs r, x and the per-cell partial
// sums of ||g||^2, the state, maxit, and whether the step is queued ahead of the previous one.
struct CgRhs {
  const double* u = nullptr;
  const double* links = nullptr;
  int n = 0, dim = 2;
  double dt = 0;
  int kind = 0;
  double k1 = 0, k2 = 1;
  double* r = nullptr;
  double* x = nullptr;
  double* part = nullptr;
  CgState* st = nullptr;
  int maxit = 0, ahead = 0;
};

struct Handle {
  int dim = 2, n = 0, leaf = 8, L = 0;
  int64_t N = 0;
  double dt = 0, h = 0, eps = 0;
  DevBuf<double> links;       // per-axis link weights dt/(2h^2) * a_link, axis-major
  FactorDev f;
  // PCG workspace
  DevBuf<double> x, r, z, p, q, w, partials;  // w = A z
  DevBuf<CgState> st;
  DevBuf<int32_t> step_iters;
  DevBuf<double> step_relres;
  // pinned, device-mapped: [0..2] iters, done, status of the running step (decoded by the host
  // from [8 + 2 (seq & 1)], the 64-bit word that the last convergence test of a queued batch of
  // iterations posts together with its sequence number flag_seq: two steps may be in flight);
  // [4..5] the last batched step's relres
  int32_t* host_flag = nullptr;
  int32_t* flag_dev = nullptr;  // host_flag as seen from the device
  int32_t flag_seq = 0;
  int nblk = 0;
  int last_iters = 2;
  // the right-hand side made by the first apply stage (rhs_fused): ||g||^2 per level-0 cell
  bool rhs_fused = false;
  DevBuf<double> gpart;
  bool built = false;  // factor built here (hif_factor*), not imported: hif_refactor allowed
  // the level-0 structure (it depends on the grid only), kept once the factor has been rebuilt
  // so that later rebuilds skip planning it
  std::shared_ptr<const LevelPlan> plan0;
  bool keep_plan0 = false;
  // changes whenever the factor or the operator is replaced (plans that point into them, such
  // as a batched step's, are made again)
  uint64_t gen = 0;
  ~Handle();
};
uint64_t next_handle_gen();

// ---- factor layout ---------------------------------------------------------------------------
// Every block of values starts at a multiple of kValAlign elements (16-byte aligned in every
// storage precision) so the apply kernels can stage it with vector loads; the value array is
// padded by kValAlign elements at its end.
constexpr int64_t kValAlign = 8;
inline int64_t align_vals(int64_t off) { return (off + kValAlign - 1) / kValAlign * kValAlign; }
void upload_factor(const FactorHost& fh, hif_store_t store, FactorDev& fd, hipStream_t s);
// Algorithmic bytes one launch of each stage of a level moves: factor blocks (storage
// precision), FP64 vector reads/writes, contributions and int32 indices.
void level_stage_bytes(const std::vector<CellDesc>& cells, const std::vector<GroupDesc>& groups,
                       const std::vector<int64_t>& group_slots, size_t eb, LevelDev& ld);
FactorHost import_blob(const void* blob, size_t nbytes, int dim, int n, int leaf);
size_t apply_smem_need(const FactorDev& f, size_t* worst);
// Decide per level whether cells are tiled across workgroups and upload the tile lists;
// `cells` are the host copies of every level's descriptors.
void setup_tiling(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                  const std::vector<std::vector<GroupDesc>>& groups,
                  const std::vector<int32_t>& idx, hipStream_t s);

// Levels whose group stages run as one dense product per group (LevelDev::gdense): each
// group's forward step C^T K^T (block Jacobi, then the skeletonization of eq_T / eq2_9) is
// multiplied out into G (n x n, column-major) in place of its packed blocks, and the backward
// step is G^T.  A level qualifies when it is neither tiled nor under the dense top `top`,
// every group's storage holds n^2 elements (GroupDesc::cap) and G costs at most twice the
// packed blocks' elements (group stages are latency-bound: fewer dependent steps matter more
// than the extra bytes).  HIFCN_NO_DENSE_GROUPS=1: none.  Call after setup_tiling and before
// setup_fusion (the fused plans size LDS for the level's blocks).
void setup_dense_groups(FactorDev& f, const std::vector<std::vector<GroupDesc>>& groups,
                        const std::vector<int32_t>& idx, int top, hipStream_t s);

// The level from which the rest of the apply runs as one dense matrix (-1: none, when no level's
// matrix stays within the element budget f.top_budget, else HIFCN_DENSE_TOP, else 40M entries;
// 0 disables).
int dense_top_level(const FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                    const std::vector<std::vector<GroupDesc>>& groups);
// Choose that level, form its matrix and lay it out.  Call after setup_fusion (it turns the
// fused root off when it takes over the root).
void setup_dense_top(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                     const std::vector<std::vector<GroupDesc>>& groups,
                     const std::vector<int32_t>& idx, int64_t N, hipStream_t s);

// One block put in dense form (column-major n x n, leading dimension ld, at dst in dvals).
struct DenseJob {
  int32_t kind;      // 0: M = L^-T L^-1 from a packed L^-1 at src; 1: the step of a group whose
                     //    value block starts at src
  int32_t n, nr, ld;
  int64_t src, dst;
  int32_t offPerm, pad;  // kind 1: pivot order in idx
};
// Form the dense blocks (FP64 on the matrix cores, stored in the factor's precision); dvals
// must be allocated and vals final.
void build_dense_forms(FactorDev& f, const std::vector<DenseJob>& jobs, hipStream_t s);
// The same products in FP64, written column-major to out + dst (leading dimension ld).
void build_dense_forms_f64(FactorDev& f, const std::vector<DenseJob>& jobs, double* out,
                           hipStream_t s);
// Decide which group stages run together with the next level's cell stage (and the last level
// with the root) and upload the ownership lists; call after setup_tiling.
void setup_fusion(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                  const std::vector<std::vector<GroupDesc>>& groups,
                  const std::vector<int32_t>& idx, int64_t N, hipStream_t s);
void set_apply_smem_limits(size_t bytes);

// ---- kernels --------------------------------------------------------------------------------
void hif_apply_inplace(const FactorDev& f, double* y, const int* done, hipStream_t s);
// The apply with the convergence test in its first stage (requires f.gate): y <- M^-1 src when
// the iteration goes on, nothing when it stops; later stages skip on g.st->done.
void hif_apply_gated(const FactorDev& f, double* y, const CgGate& g, hipStream_t s);
// The apply whose first stage makes the step's right-hand side first (requires f.gate): y <-
// M^-1 g; later stages skip on r.st->done.
void hif_apply_rhs(const FactorDev& f, double* y, const CgRhs& r, hipStream_t s);
// Lay out the copy lists of the gated apply (f.gate stays false when level 0 does not run as
// one workgroup per cell).
void setup_cg_gate(FactorDev& f, const std::vector<std::vector<CellDesc>>& cells,
                   const std::vector<int32_t>& idx, int64_t N, hipStream_t s);
void launch_links(const double* a_cells, int dim, int n, double scale, double* links,
                  hipStream_t s);
void launch_spmv(const Handle& h, const double* x, double* y, hipStream_t s);
// PCG kernels; `it` is the 0-based index of the CG iteration (host-side count).
int cg_partial_slots();
// ahead: the step is queued before the previous one is known to have ended; it does nothing if
// that one holds.
// warm: r = g - A u (the warm-started step's r0) and its partials of ||r0||^2 beside ||g||^2.
void launch_cg_rhs(Handle& h, const double* u, int kind, double k1, double k2, bool ahead,
                   hipStream_t s, bool warm = false);
// Before more iterations of a step whose closing test held: done = hold = 0.
void launch_cg_resume(Handle& h, hipStream_t s);
// warm: the step started from x0 = u^k, so PCG runs on the correction d = x - u^k from 0
// (r0 = g - A u^k); its initial test takes ||g||^2 and ||r0||^2.
void launch_cg_check_copy(Handle& h, int it /* -1: initial */, double rtol, int maxit,
                          hipStream_t s, bool warm = false);
// The test closing a queued batch of iterations: as launch_cg_check_copy, and when the iteration
// stops (here or earlier in the batch) u = x and the records of step `step`; then the outcome is
// posted to the handle's host flag with sequence number seq.
// warm: the step ends with u = u^k + d (u = 0 when g = 0).
void launch_cg_check_finish(Handle& h, int it, double rtol, double* u, int step, int seq,
                            hipStream_t s, bool warm = false);
// The same test as arguments of a gated apply.
CgGate cg_gate_args(Handle& h, int it /* -1: initial */, double rtol, int maxit);
// Iteration `it` after z = M^-1 r: w = A z with the partials of r.z, z.w, z.q, then the update
// of p, q = A p, x and r with the partials of ||r||^2.
void launch_cg_dir_dots(Handle& h, int it, hipStream_t s);
// (rtol: for the first update of a step whose right-hand side the apply made, which also tests
// g: it totals ||g||^2 and starts tol2.)
// fused_g: the step's g was made by the first apply stage (iteration 0 then tests it)
void launch_cg_update(Handle& h, int it, double rtol, hipStream_t s, bool fused_g);
// One solve's part of a batched PCG vector launch: its blocks are launch blocks first ..
// first + nb - 1 (nb: the solve's own block count, so its reductions are those it makes alone).
struct BatchCg {
  int64_t N;
  int32_t n, nb, first, maxit;
  const double* links;
  double *u, *x, *r, *z, *p, *q, *w, *part;
  CgState* st;
  int32_t* hflag;
  int32_t* it_out;
  double* rel_out;
  double dt, k1, k2, rtol;
  int32_t kind, pad;
};
// The PCG kernels of Algorithm 1 over a batch of solves of one dimension (args on the device,
// nslot entries, `blocks` launch blocks in all): the right-hand side (and a new step's
// scalars), the convergence test (init: of g; else after iteration it0) with z = r when the
// iteration goes on (fin: closing a queued batch of iterations, u = x and the outcome posted to
// hflag with sequence number seq when it stops), the direction kernel and the update.
void launch_bcg_rhs(const BatchCg* args, int nslot, int blocks, int dim, hipStream_t s);
void launch_bcg_check(const BatchCg* args, int nslot, int blocks, int init, int it0, int fin,
                      int seq, hipStream_t s);
void launch_bcg_dir_dots(const BatchCg* args, int nslot, int blocks, int dim, int it,
                         hipStream_t s);
void launch_bcg_update(const BatchCg* args, int nslot, int blocks, int it, hipStream_t s);

// ||I - A F^-1||_2 by `iters` power-iteration steps on E^T E from x0 (device, N values), its
// scratch allocated for the call; *est_host receives the estimate (synchronises s).
hif_status_t inverse_error_impl(Handle& h, const double* x0, int iters, double* est_host,
                                hipStream_t s);
// The same on the library's fixed device scratch (N up to its size): no allocation.
hif_status_t inverse_error_noalloc_impl(Handle& h, const double* x0, int iters,
                                        double* est_host, hipStream_t s);

}  // namespace hifcn
