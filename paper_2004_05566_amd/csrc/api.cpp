// C-ABI entry points of libhifcn (declared in include/hifcn.h).
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <map>
#include <string>
#include <thread>
#include <tuple>

#include "kernels.hpp"

namespace hifcn {

void gpu_build(Handle& h, const double* a_cells, hif_store_t store, hipStream_t s);
int vec_blocks(int64_t N);

Handle::~Handle() {
  if (host_flag) (void)hipHostFree(host_flag);
}

uint64_t next_handle_gen() {
  static std::atomic<uint64_t> g{0};
  return ++g;
}

namespace {

thread_local std::string g_last_error;

hif_status_t fail(hif_status_t s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

template <typename F>
hif_status_t guarded(F&& f) {
  try {
    f();
    return HIF_OK;
  } catch (const HifError& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(HIF_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HIF_ERR_HIP, e.what());
  }
}

int levels_for(int n, int m) {
  int L = 0;
  while ((int64_t)m * (2LL << L) <= n + 1) ++L;
  return L;
}

std::unique_ptr<Handle> make_handle(const double* a_cells, double dt, const hif_grid_t* grid,
                                    double eps, hipStream_t s) {
  HIF_REQUIRE(grid != nullptr && a_cells != nullptr, HIF_ERR_ARG, "NULL argument");
  HIF_REQUIRE(grid->dim == 2 || grid->dim == 3, HIF_ERR_ARG, "dim must be 2 or 3");
  const int n = grid->n[0];
  HIF_REQUIRE(n >= 1 && grid->n[1] == n && (grid->dim == 2 || grid->n[2] == n), HIF_ERR_ARG,
              "the grid must have the same number of interior nodes on every axis");
  HIF_REQUIRE(grid->leaf >= 2, HIF_ERR_ARG, "leaf size must be at least 2");
  HIF_REQUIRE(dt > 0 && std::isfinite(dt), HIF_ERR_ARG, "dt must be positive");
  HIF_REQUIRE(eps >= 0 && std::isfinite(eps), HIF_ERR_ARG, "eps must be >= 0");
  auto h = std::make_unique<Handle>();
  h->gen = next_handle_gen();
  h->dim = grid->dim;
  h->n = n;
  h->leaf = grid->leaf;
  h->L = levels_for(n, grid->leaf);
  h->N = 1;
  for (int d = 0; d < h->dim; ++d) h->N *= n;
  HIF_REQUIRE(h->N < (int64_t)INT32_MAX, HIF_ERR_ARG, "grid too large");
  h->dt = dt;
  h->h = 1.0 / (n + 1);
  h->eps = eps;
  const int64_t per = h->N / n * (n + 1);
  h->links.alloc(per * h->dim);
  launch_links(a_cells, h->dim, n, dt / (2.0 * h->h * h->h), h->links.p, s);
  h->nblk = vec_blocks(h->N);
  h->x.alloc(h->N);
  h->r.alloc(h->N);
  h->z.alloc(h->N);
  h->p.alloc(h->N);
  h->q.alloc(h->N);
  h->w.alloc(h->N);
  h->partials.alloc((size_t)h->nblk * cg_partial_slots());
  h->st.alloc(1);
  HIF_CHECK(hipMemsetAsync(h->st.p, 0, sizeof(CgState), s));
  h->step_iters.alloc(1);
  h->step_relres.alloc(1);
  // see Handle::host_flag
  HIF_CHECK(hipHostMalloc(reinterpret_cast<void**>(&h->host_flag), 16 * sizeof(int32_t),
                          hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(h->host_flag, 0, 16 * sizeof(int32_t));
  HIF_CHECK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->flag_dev), h->host_flag, 0));
  return h;
}

// Host threads that share the launches of one batched step (HIFCN_BATCH_THREADS, default 8).
int batch_threads() {
  static const int n = [] {
    const char* e = std::getenv("HIFCN_BATCH_THREADS");
    return e ? std::max(1, std::atoi(e)) : 8;
  }();
  return n;
}

// One Crank-Nicolson step of one solve, as a small state machine so that several solves can be
// advanced in lockstep (continuous batching).  Iterations are queued without waiting, up to
// the predicted count; the predicted last iteration stops after its convergence test, so a
// converged step leaves no dead preconditioner apply behind.
struct StepState {
  Handle* h = nullptr;
  hipStream_t s = nullptr;
  const hif_reaction_t* r = nullptr;
  const hif_cg_opts_t* o = nullptr;
  double* u = nullptr;
  int step = 0;
  int launched = 0;        // iterations whose update has been queued
  bool tail_open = false;  // the last queued iteration still owes its apply + r.z
  int chunk = 1;
  int seq = 0;             // sequence number of the latest posted convergence test
  bool finished = false;
  int status = 0;
};

// Whether the first apply stage of a step makes its right-hand side: as for the test in that stage
// (check_and_apply), and HIFCN_NO_RHS_FUSE unset.
void setup_rhs(Handle& h) {
  h.rhs_fused = h.f.gate && h.f.gate_n == h.N &&
                (int64_t)h.f.lv[0].ncell * h.nblk <= (int64_t(1) << 20) &&
                !std::getenv("HIFCN_NO_RHS_FUSE");
  if (h.rhs_fused) h.gpart.alloc(h.f.lv[0].ncell);
}

// The convergence test after iteration `it` (-1: of the right-hand side) followed by z = M^-1 r:
// run by the apply's first stage when the factor allows it, else as its own launch.  Every
// workgroup of that stage reads all partials of the test, so it stays a launch of its own where
// that would add up to more than ~8 MB (many level-0 cells: the 1024^2 grid has 16K).
// A warm-started step's initial test (two totals) is always a launch of its own.
void check_and_apply(Handle& h, int it, double rtol, int maxit, hipStream_t s,
                     bool warm = false) {
  if (!(warm && it < 0) && h.f.gate && h.f.gate_n == h.N &&
      (int64_t)h.f.lv[0].ncell * h.nblk <= (int64_t(1) << 20)) {
    hif_apply_gated(h.f, h.z.p, cg_gate_args(h, it, rtol, maxit), s);
  } else {
    launch_cg_check_copy(h, it, rtol, maxit, s, warm);
    hif_apply_inplace(h.f, h.z.p, &h.st.p->done, s);
  }
}

// ahead: queued before the previous step of the same solve is known to have ended well (if it
// did not, the whole step does nothing and is queued again).
void step_begin(StepState& st, bool ahead = false) {
  Handle& h = *st.h;
  const int kind = st.r ? st.r->kind : 0;
  const double k1 = st.r ? st.r->k1 : 0, k2 = st.r ? st.r->k2 : 1;
  const bool warm = st.o->warm_start != 0;  // x0 = u^k: the right-hand side launch forms r0
  if (h.rhs_fused && !warm) {  // the first apply stage makes g (the first update then tests it)
    CgRhs c;
    c.u = st.u;
    c.links = h.links.p;
    c.n = h.n;
    c.dim = h.dim;
    c.dt = h.dt;
    c.kind = kind;
    c.k1 = k1;
    c.k2 = k2;
    c.r = h.r.p;
    c.x = h.x.p;
    c.part = h.gpart.p;
    c.st = h.st.p;
    c.maxit = st.o->maxit;
    c.ahead = ahead ? 1 : 0;
    hif_apply_rhs(h.f, h.z.p, c, st.s);
  } else {
    launch_cg_rhs(h, st.u, kind, k1, k2, ahead, st.s, warm);
    check_and_apply(h, -1, st.o->rtol, st.o->maxit, st.s, warm);
  }
  st.chunk = std::max(1, h.last_iters);
}

// Queue the next chunk of iterations and the read-back of [iters, done, status].
void step_queue(StepState& st) {
  Handle& h = *st.h;
  const bool warm = st.o->warm_start != 0;
  if (st.tail_open) {  // the previous chunk's last iteration did not converge
    launch_cg_resume(h, st.s);  // (a step queued ahead may have stopped everything meanwhile)
    hif_apply_inplace(h.f, h.z.p, &h.st.p->done, st.s);
    st.tail_open = false;
  }
  for (int c = 0; c < st.chunk && st.launched < st.o->maxit; ++c) {
    const int it = st.launched++;
    launch_cg_dir_dots(h, it, st.s);
    launch_cg_update(h, it, st.o->rtol, st.s, h.rhs_fused && !warm);
    if (c + 1 == st.chunk || st.launched == st.o->maxit) {
      // the host reads the verdict before it queues another apply
      st.seq = ++h.flag_seq;
      launch_cg_check_finish(h, it, st.o->rtol, st.u, st.step, st.seq, st.s, warm);
      st.tail_open = true;
      break;
    }
    check_and_apply(h, it, st.o->rtol, st.o->maxit, st.s);
  }
  HIF_CHECK(hipGetLastError());
}

// Wait until the batch queued by step_queue has posted its outcome to the host flag: spin on the
// sequence number (no stream round trip), looking at the stream now and then; an idle stream
// without the post is an error.
void step_wait(StepState& st) {
  int32_t* f = st.h->host_flag;
  const volatile uint64_t* w = reinterpret_cast<const volatile uint64_t*>(f + 8 + 2 * (st.seq & 1));
  uint64_t v = 0;
  for (int64_t n = 1;; ++n) {
    v = *w;
    if ((int32_t)(v >> 32) == st.seq) break;
    if ((n & 255) != 0) continue;
    const hipError_t q = hipStreamQuery(st.s);
    if (q == hipErrorNotReady) continue;
    HIF_CHECK(q);
    v = *w;
    HIF_REQUIRE((int32_t)(v >> 32) == st.seq, HIF_ERR_HIP, "convergence flag was not posted");
    break;
  }
  f[0] = (int32_t)(v & 0xffffff);
  f[1] = (int32_t)(v >> 24 & 0xf);
  f[2] = (int32_t)(v >> 28 & 0xf);
}

// Once the outcome of the batch is posted: the step is over if PCG stopped (the closing test has
// then written u and the step's records; PCG always stops by maxit).
void step_after_sync(StepState& st) {
  Handle& h = *st.h;
  if (h.host_flag[1]) {
    h.last_iters = h.host_flag[0];
    st.status = h.host_flag[2];
    st.finished = true;
  } else {
    HIF_REQUIRE(st.launched < st.o->maxit, HIF_ERR_HIP, "PCG ran past maxit without stopping");
    st.chunk = 2;
  }
}

StepState step_state(Handle& h, const hif_reaction_t* r, const hif_cg_opts_t* o, double* u,
                     int step, hipStream_t s) {
  StepState st;
  st.h = &h;
  st.s = s;
  st.r = r;
  st.o = o;
  st.u = u;
  st.step = step;
  return st;
}

// Steps of one solve.  Step k+1 is queued (ahead) before step k's outcome is read, so the GPU
// does not wait for the host between steps; when step k did not end well within its predicted
// iterations, the step queued ahead does nothing (hold) and is queued again once step k is over.
// Returns the first step that did not converge, or -1.
int cn_steps_dev(Handle& h, const hif_reaction_t* r, const hif_cg_opts_t* o, double* u,
                 int nsteps, hipStream_t s) {
  const bool ahead_on = std::getenv("HIFCN_NO_AHEAD") == nullptr;
  if (nsteps <= 0) return -1;
  StepState cur = step_state(h, r, o, u, 0, s);
  step_begin(cur);
  step_queue(cur);
  for (int k = 0; k < nsteps; ++k) {
    const bool ahead = ahead_on && k + 1 < nsteps;
    StepState nxt = step_state(h, r, o, u, k + 1, s);
    if (ahead) {
      step_begin(nxt, true);
      step_queue(nxt);
    }
    step_wait(cur);
    step_after_sync(cur);
    bool held = !cur.finished;
    while (!cur.finished) {
      step_queue(cur);
      step_wait(cur);
      step_after_sync(cur);
    }
    if (cur.status != 0) return k;
    if (k + 1 == nsteps) break;
    if (!ahead || held) {
      nxt = step_state(h, r, o, u, k + 1, s);
      step_begin(nxt);
      step_queue(nxt);
    }
    cur = nxt;
  }
  return -1;
}

void check_opts(const hif_cg_opts_t* o) {
  HIF_REQUIRE(o != nullptr, HIF_ERR_ARG, "NULL cg options");
  HIF_REQUIRE(o->rtol > 0 && o->maxit > 0, HIF_ERR_ARG, "rtol and maxit must be positive");
  HIF_REQUIRE(o->maxit < (1 << 24), HIF_ERR_ARG, "maxit must be below 2^24");
  HIF_REQUIRE(o->warm_start == 0 || o->warm_start == 1, HIF_ERR_ARG,
              "warm_start must be 0 (x0 = 0) or 1 (x0 = u^k)");
}

void check_reaction(const hif_reaction_t* r) {
  if (!r) return;
  HIF_REQUIRE(r->kind == 0 || r->kind == 1, HIF_ERR_ARG, "unknown reaction kind");
  HIF_REQUIRE(r->kind == 0 || r->k2 != 0.0, HIF_ERR_ARG, "k2 must be non-zero");
}

// Every byte of device memory the handle holds (factor, descriptors, PCG workspace).
int64_t handle_device_bytes(const Handle& h) {
  int64_t b = 0;
  auto add = [&](const auto& buf) { b += (int64_t)(buf.n * sizeof(*buf.p)); };
  add(h.links); add(h.x); add(h.r); add(h.z); add(h.p); add(h.q); add(h.w); add(h.partials);
  add(h.st); add(h.step_iters); add(h.step_relres); add(h.gpart);
  const FactorDev& f = h.f;
  add(f.idx); add(f.vals); add(f.cb); add(f.wsc); add(f.dvals);
  add(f.tvals); add(f.tgid); add(f.tgslot); add(f.tscat); add(f.twsc); add(f.tpos);
  add(f.gcopy);
  add(f.rddoff); add(f.rdtiles); add(f.rscat);
  for (const LevelDev& l : f.lv) {
    add(l.cells); add(l.groups); add(l.rtiles); add(l.ctiles); add(l.crec); add(l.grec); add(l.frec);
    add(l.cdtiles); add(l.grtiles); add(l.gctiles); add(l.gscat); add(l.cddoff); add(l.gddoff);
  }
  return b;
}

// ---- batched kernels over all solves of a batch ---------------------------------------------
// One Crank-Nicolson step of every solve with one launch per stage for all of them: the PCG
// vector kernels over a table of the solves (launch_bcg_*) and the apply as the batched stage
// launches of build_batch_apply (levels aligned from the leaves).  Every solve keeps its own
// block counts and stage plans, so its iterates do not depend on its companions.  The plan is
// kept while the batch's composition and options stay the same.
struct FusedBatch {
  std::vector<std::tuple<const Handle*, uint64_t, const double*, int, double, double, double,
                         int>> key;
  BatchApplyPlan plan;
  StagedBuf<BatchCg> cg;
  int blocks = 0, dim = 2, maxit = 1;
};

bool batch_kernels_on() { return std::getenv("HIFCN_NO_BATCH_KERNELS") == nullptr; }

// The batch key of a solve whose factor allows the batched kernels (dimension and storage: one
// batched launch holds one of each), or -1.
int fused_batch_key(const Handle& h) {
  if (!batch_kernels_on() || !batchable(h.f)) return -1;
  return h.dim * 4 + (int)h.f.store;
}

void fused_batch_setup(FusedBatch& fb, std::vector<StepState>& st, hipStream_t s) {
  decltype(fb.key) key;
  for (const StepState& x : st)
    key.emplace_back(x.h, x.h->gen, x.u, x.r ? x.r->kind : 0,
                     x.r ? x.r->k1 : 0.0, x.r ? x.r->k2 : 1.0, x.o->rtol, x.o->maxit);
  if (key == fb.key) return;
  std::vector<const FactorDev*> fs;
  std::vector<double*> ys;
  std::vector<const int*> dn;
  std::vector<BatchCg> cg;
  int blocks = 0, maxit = 1;
  for (const StepState& x : st) {
    Handle& h = *x.h;
    fs.push_back(&h.f);
    ys.push_back(h.z.p);
    dn.push_back(&h.st.p->done);
    BatchCg a{};
    a.N = h.N;
    a.n = h.n;
    a.nb = h.nblk;
    a.first = blocks;
    a.maxit = x.o->maxit;
    a.links = h.links.p;
    a.u = x.u;
    a.x = h.x.p;
    a.r = h.r.p;
    a.z = h.z.p;
    a.p = h.p.p;
    a.q = h.q.p;
    a.w = h.w.p;
    a.part = h.partials.p;
    a.st = h.st.p;
    a.hflag = h.flag_dev;
    a.it_out = h.step_iters.p;
    a.rel_out = h.step_relres.p;
    a.dt = h.dt;
    a.kind = x.r ? x.r->kind : 0;
    a.k1 = x.r ? x.r->k1 : 0.0;
    a.k2 = x.r ? x.r->k2 : 1.0;
    a.rtol = x.o->rtol;
    cg.push_back(a);
    blocks += h.nblk;
    maxit = std::max(maxit, x.o->maxit);
  }
  build_batch_apply(fs, ys, dn, fb.plan, s);
  fb.cg.upload(cg, s);
  fb.blocks = blocks;
  fb.dim = st[0].h->dim;
  fb.maxit = maxit;
  fb.key = std::move(key);
}

// Wait for every solve's post of sequence number seq; fills each StepState's finished/status.
void fused_batch_wait(std::vector<StepState>& st, int seq, hipStream_t s) {
  for (StepState& x : st) {
    int32_t* f = x.h->host_flag;
    const volatile uint64_t* w = reinterpret_cast<const volatile uint64_t*>(f + 8 + 2 * (seq & 1));
    uint64_t v = 0;
    for (int64_t n = 1;; ++n) {
      v = *w;
      if ((int32_t)(v >> 32) == seq) break;
      if ((n & 255) != 0) continue;
      const hipError_t q = hipStreamQuery(s);
      if (q == hipErrorNotReady) continue;
      HIF_CHECK(q);
      v = *w;
      HIF_REQUIRE((int32_t)(v >> 32) == seq, HIF_ERR_HIP, "convergence flag was not posted");
      break;
    }
    x.finished = (v >> 24 & 0xf) != 0;
    x.status = (int)(v >> 28 & 0xf);
    x.launched = (int)(v & 0xffffff);
  }
}

// One CN step of every solve in st, all on stream s.
void fused_batch_step(FusedBatch& fb, std::vector<StepState>& st, hipStream_t s) {
  fused_batch_setup(fb, st, s);
  const int ns = (int)st.size();
  const BatchCg* cg = fb.cg.p;
  launch_bcg_rhs(cg, ns, fb.blocks, fb.dim, s);
  launch_bcg_check(cg, ns, fb.blocks, 1, -1, 0, 0, s);
  run_batch_apply(fb.plan, s);
  int chunk = 1;
  for (const StepState& x : st) chunk = std::max(chunk, x.h->last_iters);
  int it = 0;
  for (;;) {
    int seq = 0;
    for (const StepState& x : st) seq = std::max(seq, x.h->flag_seq);
    ++seq;
    for (StepState& x : st) x.h->flag_seq = seq;
    for (int c = 0; c < chunk; ++c) {
      launch_bcg_dir_dots(cg, ns, fb.blocks, fb.dim, it, s);
      launch_bcg_update(cg, ns, fb.blocks, it, s);
      const bool close = c + 1 == chunk || it + 1 >= fb.maxit;
      launch_bcg_check(cg, ns, fb.blocks, 0, it, close ? 1 : 0, seq, s);
      ++it;
      if (close) break;
      run_batch_apply(fb.plan, s);
    }
    HIF_CHECK(hipGetLastError());
    fused_batch_wait(st, seq, s);
    bool all = true;
    for (const StepState& x : st) all = all && x.finished;
    if (all) break;
    HIF_REQUIRE(it < fb.maxit, HIF_ERR_HIP, "PCG ran past maxit without stopping");
    run_batch_apply(fb.plan, s);  // the solves that go on: z = r was copied by the test
    chunk = 2;
  }
  for (StepState& x : st) x.h->last_iters = std::max(1, x.launched);
}

}  // namespace
}  // namespace hifcn

using namespace hifcn;

extern "C" {

hif_status_t hif_factor_ex(const double* a_cells_dev, double dt, const hif_grid_t* grid,
                           double eps, hif_store_t store, const hif_factor_opts_t* opts,
                           void* hip_stream, hif_handle_t* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    HIF_REQUIRE(out != nullptr, HIF_ERR_ARG, "NULL output handle");
    HIF_REQUIRE(store >= HIF_STORE_F64 && store <= HIF_STORE_BF16, HIF_ERR_ARG, "bad store");
    if (opts) {
      for (int64_t r : opts->reserved)
        HIF_REQUIRE(r == 0, HIF_ERR_ARG, "reserved option fields must be 0");
      HIF_REQUIRE((opts->flags & ~(int64_t)HIF_FACTOR_SKEL_EDGES) == 0, HIF_ERR_ARG,
                  "unknown factor flags");
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto h = make_handle(a_cells_dev, dt, grid, eps, s);
    h->f.top_budget = opts ? opts->dense_top : -1;
    h->f.skel_edges = opts && (opts->flags & HIF_FACTOR_SKEL_EDGES) != 0;
    gpu_build(*h, a_cells_dev, store, s);
    setup_rhs(*h);
    h->built = true;
    *out = reinterpret_cast<hif_handle_t>(h.release());
  });
}

hif_status_t hif_factor(const double* a_cells_dev, double dt, const hif_grid_t* grid, double eps,
                        hif_store_t store, void* hip_stream, hif_handle_t* out) {
  return hif_factor_ex(a_cells_dev, dt, grid, eps, store, nullptr, hip_stream, out);
}

hif_status_t hif_import(const double* a_cells_dev, double dt, const hif_grid_t* grid,
                        const void* blob_host, size_t nbytes, hif_store_t store, void* hip_stream,
                        hif_handle_t* out) {
  if (out) *out = nullptr;
  return guarded([&] {
    HIF_REQUIRE(out != nullptr, HIF_ERR_ARG, "NULL output handle");
    HIF_REQUIRE(store >= HIF_STORE_F64 && store <= HIF_STORE_BF16, HIF_ERR_ARG, "bad store");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto h = make_handle(a_cells_dev, dt, grid, 0.0, s);
    FactorHost fh = import_blob(blob_host, nbytes, h->dim, h->n, h->leaf);
    HIF_REQUIRE((int)fh.lv.size() == h->L, HIF_ERR_ARG, "HIFB level count does not match grid");
    upload_factor(fh, store, h->f, s);
    setup_rhs(*h);
    *out = reinterpret_cast<hif_handle_t>(h.release());
  });
}

hif_status_t hif_set_coefficient(hif_handle_t hh, const double* a_cells_dev, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && a_cells_dev, HIF_ERR_ARG, "NULL argument");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    launch_links(a_cells_dev, h.dim, h.n, h.dt / (2.0 * h.h * h.h), h.links.p,
                 static_cast<hipStream_t>(hip_stream));
    h.gen = next_handle_gen();
  });
}

hif_status_t hif_refactor(hif_handle_t hh, const double* a_cells_dev, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && a_cells_dev, HIF_ERR_ARG, "NULL argument");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    HIF_REQUIRE(h.built, HIF_ERR_ARG, "hif_refactor: the factor was imported (no eps to build with)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const hif_grid_t g{h.dim, {h.n, h.n, h.dim == 3 ? h.n : 0}, h.leaf};
    // a complete new handle, then its factor and operator moved into this one; the old ones
    // leave with it (the PCG workspace, state and host flag stay)
    auto nh = make_handle(a_cells_dev, h.dt, &g, h.eps, s);
    nh->f.top_budget = h.f.top_budget;
    nh->f.skel_edges = h.f.skel_edges;
    nh->plan0 = h.plan0;
    nh->keep_plan0 = true;
    gpu_build(*nh, a_cells_dev, h.f.store, s);
    setup_rhs(*nh);
    HIF_CHECK(hipStreamSynchronize(s));
    std::swap(h.f, nh->f);
    std::swap(h.links, nh->links);
    h.gen = next_handle_gen();
    std::swap(h.gpart, nh->gpart);
    h.rhs_fused = nh->rhs_fused;
    h.plan0 = nh->plan0;
    DeviceIdle idle;  // the old factor leaves with nh: released after one synchronisation
    nh.reset();
  });
}

hif_status_t hif_apply(hif_handle_t hh, const double* x, double* y, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && x && y, HIF_ERR_ARG, "NULL argument");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (x != y)
      HIF_CHECK(hipMemcpyAsync(y, x, h.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    hif_apply_inplace(h.f, y, nullptr, s);
  });
}

hif_status_t hif_spmv(hif_handle_t hh, const double* x, double* y, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && x && y, HIF_ERR_ARG, "NULL argument");
    HIF_REQUIRE(x != y, HIF_ERR_ARG, "hif_spmv: x and y must not alias");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    launch_spmv(h, x, y, static_cast<hipStream_t>(hip_stream));
  });
}

hif_status_t cn_solve(hif_handle_t hh, const hif_reaction_t* r, const hif_cg_opts_t* o, double* u,
                      int32_t nsteps, int32_t* iters, double* relres, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && u, HIF_ERR_ARG, "NULL argument");
    HIF_REQUIRE(nsteps >= 0, HIF_ERR_ARG, "nsteps must be >= 0");
    check_opts(o);
    check_reaction(r);
    Handle& h = *reinterpret_cast<Handle*>(hh);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if ((int64_t)h.step_iters.n < nsteps) {
      h.step_iters.alloc(std::max(1, nsteps));
      h.step_relres.alloc(std::max(1, nsteps));
    }
    const int failed_step = cn_steps_dev(h, r, o, u, nsteps, s);
    const int done_steps = failed_step >= 0 ? failed_step + 1 : nsteps;
    std::vector<int32_t> it(std::max(1, done_steps));
    std::vector<double> rr(std::max(1, done_steps));
    if (done_steps) {
      HIF_CHECK(hipMemcpyAsync(it.data(), h.step_iters.p, done_steps * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
      HIF_CHECK(hipMemcpyAsync(rr.data(), h.step_relres.p, done_steps * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    HIF_CHECK(hipStreamSynchronize(s));
    for (int k = 0; k < done_steps; ++k) {
      if (iters) iters[k] = it[k];
      if (relres) relres[k] = rr[k];
    }
    HIF_REQUIRE(failed_step < 0, HIF_ERR_NO_CONV,
                "PCG did not converge at step " + std::to_string(failed_step));
  });
}

hif_status_t cn_solve_direct(hif_handle_t hh, const hif_reaction_t* r, double* u, int32_t nsteps,
                             void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && u, HIF_ERR_ARG, "NULL argument");
    HIF_REQUIRE(nsteps >= 0, HIF_ERR_ARG, "nsteps must be >= 0");
    check_reaction(r);
    Handle& h = *reinterpret_cast<Handle*>(hh);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int kind = r ? r->kind : 0;
    const double k1 = r ? r->k1 : 0.0, k2 = r ? r->k2 : 1.0;
    if (!h.rhs_fused) {  // g into r, F^-1 in place there, back into u
      for (int k = 0; k < nsteps; ++k) {
        launch_cg_rhs(h, u, kind, k1, k2, false, s);
        hif_apply_inplace(h.f, h.r.p, nullptr, s);
        HIF_CHECK(hipMemcpyAsync(u, h.r.p, h.N * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
      return;
    }
    // the first apply stage forms g from the state it reads; the state alternates between u and
    // the workspace z, with one copy at the end of an odd count
    double* cur = u;
    double* nxt = h.z.p;
    for (int k = 0; k < nsteps; ++k) {
      CgRhs c;
      c.u = cur;
      c.links = h.links.p;
      c.n = h.n;
      c.dim = h.dim;
      c.dt = h.dt;
      c.kind = kind;
      c.k1 = k1;
      c.k2 = k2;
      c.r = h.r.p;
      c.x = h.x.p;
      c.part = h.gpart.p;
      c.st = h.st.p;
      c.maxit = 1;
      c.ahead = 0;
      hif_apply_rhs(h.f, nxt, c, s);
      std::swap(cur, nxt);
    }
    if (cur != u)
      HIF_CHECK(hipMemcpyAsync(u, cur, h.N * sizeof(double), hipMemcpyDeviceToDevice, s));
  });
}

hif_status_t cn_step(hif_handle_t hh, const hif_reaction_t* r, const hif_cg_opts_t* o, double* u,
                     int32_t* iters, double* relres, void* hip_stream) {
  return cn_solve(hh, r, o, u, 1, iters, relres, hip_stream);
}

hif_status_t cn_batch_step(hif_handle_t* hs, const hif_reaction_t* rs, const hif_cg_opts_t* os,
                           double** us, int32_t count, int32_t* iters, double* relres,
                           int32_t* status, void** streams) {
  return guarded([&] {
    HIF_REQUIRE(count >= 0, HIF_ERR_ARG, "count must be >= 0");
    HIF_REQUIRE(count == 0 || (hs && os && us), HIF_ERR_ARG, "NULL argument");
    std::vector<StepState> st(count);
    for (int i = 0; i < count; ++i) {
      HIF_REQUIRE(hs[i] && us[i], HIF_ERR_ARG, "NULL handle or state");
      check_opts(&os[i]);
      HIF_REQUIRE(os[i].warm_start == 0, HIF_ERR_ARG,
                  "cn_batch_step: warm start is available in cn_step and cn_solve only");
      if (rs) check_reaction(&rs[i]);
      for (int j = 0; j < i; ++j)
        HIF_REQUIRE(hs[j] != hs[i], HIF_ERR_ARG, "a handle appears twice in one batch");
      st[i].h = reinterpret_cast<Handle*>(hs[i]);
      st[i].s = streams ? static_cast<hipStream_t>(streams[i]) : nullptr;
      st[i].r = rs ? &rs[i] : nullptr;
      st[i].o = &os[i];
      st[i].u = us[i];
      st[i].step = 0;
    }
    // Solves whose factors allow it run with one launch per stage for every solve of the same
    // dimension and storage (batched kernels), on the first such solve's stream, with the other
    // streams joined before and after; the rest take the per-solve launches below.
    std::map<int, std::vector<StepState>> fused;
    std::vector<int> fused_at(count, -1);
    std::vector<StepState> rest;
    std::vector<int> rest_at;
    for (int i = 0; i < count; ++i) {
      const int k = fused_batch_key(*st[i].h);
      if (k >= 0) {
        fused_at[i] = (int)fused[k].size();
        fused[k].push_back(st[i]);
      } else {
        rest_at.push_back(i);
        rest.push_back(st[i]);
      }
    }
    for (auto& [k, grp] : fused) {
      thread_local std::map<int, FusedBatch> fbs;
      hipStream_t s0 = grp[0].s;
      std::vector<hipEvent_t> evs;
      auto join = [&](hipStream_t from, hipStream_t to) {
        if (from == to) return;
        hipEvent_t e;
        HIF_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIF_CHECK(hipEventRecord(e, from));
        HIF_CHECK(hipStreamWaitEvent(to, e, 0));
        evs.push_back(e);
      };
      for (size_t i = 1; i < grp.size(); ++i) join(grp[i].s, s0);
      fused_batch_step(fbs[k], grp, s0);
      // the closing test posted each solve's iteration count and wrote its relative residual
      // to host_flag[4..5] ahead of the post
      for (StepState& x : grp) x.h->host_flag[0] = x.launched;
      HIF_CHECK(hipStreamSynchronize(s0));  // u = x may still be under way in other blocks
      for (size_t i = 1; i < grp.size(); ++i) join(s0, grp[i].s);
      for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    }
    for (int i = 0; i < count; ++i)
      if (fused_at[i] >= 0) st[i] = fused[fused_batch_key(*st[i].h)][fused_at[i]];
    const int nrest = (int)rest.size();
    // Solves are split over host threads (launching is host-bound when many solves run), each
    // thread advancing its share in lockstep with one read-back per round.
    auto run = [&](int w, int W, int dev) {
      HIF_CHECK(hipSetDevice(dev));
      std::vector<StepState*> mine;
      for (int i = w; i < nrest; i += W) mine.push_back(&rest[i]);
      for (StepState* x : mine) step_begin(*x);
      size_t open = mine.size();
      while (open > 0) {
        for (StepState* x : mine)
          if (!x->finished) step_queue(*x);
        for (StepState* x : mine)
          if (!x->finished) step_wait(*x);
        for (StepState* x : mine)
          if (!x->finished) {
            step_after_sync(*x);
            if (x->finished) --open;
          }
      }
      for (StepState* x : mine) {  // the finish kernel's statistics, into pinned memory
        HIF_CHECK(hipMemcpyAsync(x->h->host_flag, x->h->step_iters.p, sizeof(int32_t),
                                 hipMemcpyDeviceToHost, x->s));
        HIF_CHECK(hipMemcpyAsync(x->h->host_flag + 4, x->h->step_relres.p, sizeof(double),
                                 hipMemcpyDeviceToHost, x->s));
      }
      for (StepState* x : mine) HIF_CHECK(hipStreamSynchronize(x->s));
    };
    int dev = 0;
    if (nrest > 0) HIF_CHECK(hipGetDevice(&dev));
    const int W = std::min(nrest, batch_threads());
    if (W == 1) {
      run(0, 1, dev);
    } else if (W > 1) {
      std::vector<std::thread> pool;
      std::vector<std::exception_ptr> errs(W);
      for (int w = 0; w < W; ++w)
        pool.emplace_back([&, w] {
          try {
            run(w, W, dev);
          } catch (...) {
            errs[w] = std::current_exception();
          }
        });
      for (std::thread& t : pool) t.join();
      for (std::exception_ptr& e : errs)
        if (e) std::rethrow_exception(e);
    }
    for (int q = 0; q < nrest; ++q) st[rest_at[q]] = rest[q];
    int failed = -1;
    for (int i = 0; i < count; ++i) {
      const Handle& h = *st[i].h;
      double rr;
      std::memcpy(&rr, h.host_flag + 4, sizeof(double));
      if (iters) iters[i] = h.host_flag[0];
      if (relres) relres[i] = rr;
      if (status) status[i] = st[i].status ? HIF_ERR_NO_CONV : HIF_OK;
      if (st[i].status != 0 && failed < 0) failed = i;
    }
    HIF_REQUIRE(failed < 0, HIF_ERR_NO_CONV,
                "PCG did not converge for batch entry " + std::to_string(failed));
  });
}

hif_status_t hif_inverse_error(hif_handle_t hh, const double* x0_dev, int32_t iters,
                               double* est_host, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && x0_dev && est_host, HIF_ERR_ARG, "NULL argument");
    HIF_REQUIRE(iters >= 0, HIF_ERR_ARG, "iters must be >= 0");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    (void)inverse_error_impl(h, x0_dev, iters, est_host, static_cast<hipStream_t>(hip_stream));
  });
}

hif_status_t hif_inverse_error_noalloc(hif_handle_t hh, const double* x0_dev, int32_t iters,
                                       double* est_host, void* hip_stream) {
  return guarded([&] {
    HIF_REQUIRE(hh && x0_dev && est_host, HIF_ERR_ARG, "NULL argument");
    HIF_REQUIRE(iters >= 0, HIF_ERR_ARG, "iters must be >= 0");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    (void)inverse_error_noalloc_impl(h, x0_dev, iters, est_host,
                                     static_cast<hipStream_t>(hip_stream));
  });
}

size_t hif_factor_bytes(hif_handle_t hh) {
  if (!hh) return 0;
  const Handle& h = *reinterpret_cast<const Handle*>(hh);
  return (size_t)h.f.nvals * store_elem_bytes(h.f.store);
}

hif_status_t hif_get_info(hif_handle_t hh, hif_info_t* info) {
  return guarded([&] {
    HIF_REQUIRE(hh && info, HIF_ERR_ARG, "NULL argument");
    const Handle& h = *reinterpret_cast<const Handle*>(hh);
    info->levels = (int32_t)h.f.lv.size();
    info->root = h.f.nroot;
    info->entries = h.f.nvals;
    info->N = h.N;
    info->store = (int32_t)h.f.store;
    info->dim = h.dim;
    info->device_bytes = handle_device_bytes(h);
    info->build_mfma_flops = h.f.mfma_flops;
    info->build_mfma_ms = h.f.mfma_ms;
    // with a dense top, the levels above it and its groups run inside the dense matrix
    const FactorDev& f = h.f;
    const int last = f.top >= 0 ? f.top : (int)f.lv.size() - 1;
    int64_t ab = f.top >= 0 ? f.top_bytes : (f.nroot ? f.root_bytes : 0);
    for (int l = 0; l <= last; ++l) {
      const LevelDev& L = f.lv[l];
      ab += L.cell_bytes[0] + L.cell_bytes[1];
      if (l < f.top || f.top < 0) ab += L.group_bytes[0] + L.group_bytes[1];
    }
    info->apply_bytes = ab;
    info->top_level = f.top;
    info->top_fold = f.top >= 0 && f.tfold ? 1 : 0;
  });
}

hif_status_t hif_profile_stage(hif_handle_t hh, int32_t level, int32_t stage, int32_t enable) {
  return guarded([&] {
    HIF_REQUIRE(hh, HIF_ERR_ARG, "NULL handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    HIF_REQUIRE(stage >= 0 && stage <= 4, HIF_ERR_ARG, "stage must be 0..4");
    HIF_REQUIRE(level >= 0 && level <= (int)h.f.lv.size(), HIF_ERR_ARG, "level out of range");
    if (!h.f.prof) h.f.prof = std::make_unique<StageProfiler>();
    StageProfiler& p = *h.f.prof;
    HIF_CHECK(hipDeviceSynchronize());
    p.enabled = enable != 0;
    if (p.enabled) {
      p.level = level;
      p.stage = stage;
      p.launches = 0;
      p.ms = 0;
      p.pending.clear();
      p.used = 0;
      if (p.live.n < 4096) p.live.alloc(4096);
    }
  });
}

hif_status_t hif_profile_read(hif_handle_t hh, hif_stage_prof_t* out) {
  return guarded([&] {
    HIF_REQUIRE(hh && out, HIF_ERR_ARG, "NULL argument");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    HIF_REQUIRE(h.f.prof != nullptr, HIF_ERR_ARG, "no stage is being timed");
    StageProfiler& p = *h.f.prof;
    HIF_CHECK(hipDeviceSynchronize());
    std::vector<int32_t> live(p.pending.size(), 1);
    if (!live.empty())
      HIF_CHECK(hipMemcpy(live.data(), p.live.p, live.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
    for (size_t q = 0; q < p.pending.size(); ++q) {
      if (!live[q]) continue;  // the kernel returned at once: PCG had already converged
      float ms = 0;
      HIF_CHECK(hipEventElapsedTime(&ms, p.pending[q].first, p.pending[q].second));
      p.ms += ms;
      ++p.launches;
    }
    p.pending.clear();
    p.used = 0;
    out->level = p.level;
    out->stage = p.stage;
    out->launches = p.launches;
    out->ms = p.ms;
    // a fused launch carries the bytes of every stage it runs
    int64_t bytes = 0;
    const int nlev = (int)h.f.lv.size();
    if (p.stage == STAGE_ROOT && h.f.top >= 0) {
      bytes = h.f.top_bytes;
    } else if (p.stage == STAGE_ROOT) {
      bytes = h.f.root_bytes;
      if (h.f.root_fused)
        bytes += h.f.lv[nlev - 1].group_bytes[0] + h.f.lv[nlev - 1].group_bytes[1];
    } else if (p.level < nlev) {
      const LevelDev& L = h.f.lv[p.level];
      bytes = p.stage == STAGE_CELL_FWD   ? L.cell_bytes[0]
              : p.stage == STAGE_CELL_BWD ? L.cell_bytes[1]
              : p.stage == STAGE_GROUP_FWD ? L.group_bytes[0]
                                           : L.group_bytes[1];
      if (p.stage == STAGE_GROUP_FWD && L.fuse) bytes += h.f.lv[p.level + 1].cell_bytes[0];
    }
    out->bytes = bytes;
    std::snprintf(out->kernel, sizeof(out->kernel), "%s", p.kernel);
  });
}

void hif_destroy(hif_handle_t hh) {
  if (!hh) return;
  // one device synchronisation, then every buffer back to the pool without another
  hifcn::DeviceIdle idle;
  delete reinterpret_cast<Handle*>(hh);
}

const char* hif_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
