// Adjoint of the combined force pass (placeholder until the kernels land).
#include "gc_internal.h"

extern "C" gc_status gc_backward(gc_batch b, const gc_force_params* prm, const float* nodes_dev,
                                 const int32_t* node_range_dev, int32_t n_nodes, const float* cot_dev, float* gpos_dev,
                                 float* gmass_dev, float* gparam_dev, void* stream) {
  (void)b; (void)prm; (void)nodes_dev; (void)node_range_dev; (void)n_nodes; (void)cot_dev; (void)gpos_dev;
  (void)gmass_dev; (void)gparam_dev; (void)stream;
  return GC_E_UNSUPPORTED;
}
