// Internal interfaces between the translation units of the hifcn library.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace hifcn {

// One level of the factor as the apply kernels read it.
struct LevelDev {
  int ncell = 0, ngroup = 0;
  int maxI = 0, maxB = 0;            // largest cell interior / boundary
  int maxG = 0, maxK = 0, maxR = 0;  // largest group, skeleton and redundant set
  DevBuf<CellDesc> cells;
  DevBuf<GroupDesc> groups;
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
  DevBuf<double> cb;       // boundary contributions of the cell stage (max over levels)
  size_t smem_max = 0;
};

// Host-side, FP64 version of the same layout (used by import; the GPU build writes the device
// arrays directly with the same descriptors).
struct LevelHost {
  std::vector<CellDesc> cells;
  std::vector<GroupDesc> groups;
  int maxI = 0, maxB = 0, maxG = 0, maxK = 0, maxR = 0;
};
struct FactorHost {
  std::vector<LevelHost> lv;
  std::vector<int32_t> idx;
  std::vector<double> vals;
  int nroot = 0;
  int32_t offRootIdx = 0;
  int64_t offRootV = 0;
  int64_t cbmax = 0;
};

// PCG state kept on the device (scalars of Algorithm 1's pcg).
struct CgState {
  double gg;      // ||g||^2
  double tol2;    // rtol^2 ||g||^2
  double rz;      // rho = r.z of the current search direction
  double rz_new;  // r.z after the latest preconditioner apply
  double pq;      // p.(A p)
  double rr;      // ||r||^2 after the latest update
  int32_t iters, done, status, maxit;
};

struct Handle {
  int dim = 2, n = 0, leaf = 8, L = 0;
  int64_t N = 0;
  double dt = 0, h = 0, eps = 0;
  DevBuf<double> links;       // per-axis link weights dt/(2h^2) * a_link, axis-major
  FactorDev f;
  // PCG workspace
  DevBuf<double> x, r, z, p0, p1, q, partials;
  DevBuf<CgState> st;
  DevBuf<uint32_t> counter;
  DevBuf<int32_t> step_iters;
  DevBuf<double> step_relres;
  int32_t* host_flag = nullptr;  // pinned: done flag mirror
  int nblk = 0;
  int last_iters = 2;
  ~Handle();
};

// ---- factor layout ---------------------------------------------------------------------------
void upload_factor(const FactorHost& fh, hif_store_t store, FactorDev& fd, hipStream_t s);
FactorHost import_blob(const void* blob, size_t nbytes, int dim, int n, int leaf);
size_t apply_smem_need(const FactorDev& f, size_t* worst);
void set_apply_smem_limits(size_t bytes);

// ---- kernels --------------------------------------------------------------------------------
void hif_apply_inplace(const FactorDev& f, double* y, const int* done, hipStream_t s);
void launch_links(const double* a_cells, int dim, int n, double scale, double* links,
                  hipStream_t s);
void launch_spmv(const Handle& h, const double* x, double* y, hipStream_t s);
void launch_cg_rhs(Handle& h, const double* u, int kind, double k1, double k2, double rtol,
                   int maxit, hipStream_t s);
void launch_cg_dot_rz(Handle& h, hipStream_t s);
void launch_cg_dir_spmv(Handle& h, const double* pin, double* pout, hipStream_t s);
void launch_cg_update(Handle& h, const double* p, hipStream_t s);
void launch_cg_finish(Handle& h, double* u, int step, hipStream_t s);

}  // namespace hifcn
