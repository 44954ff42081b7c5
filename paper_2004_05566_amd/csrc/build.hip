// placeholder, replaced by the GPU factor build
#include "kernels.hpp"
namespace hifcn {
void gpu_build(Handle& h, const double* a_cells, hif_store_t store, hipStream_t s) {
  (void)h; (void)a_cells; (void)store; (void)s;
  throw HifError(HIF_ERR_ARG, "GPU factor build not available yet");
}
}
