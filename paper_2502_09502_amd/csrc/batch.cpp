// Batched mixed-precision engine (BF16 MFMA correction products around an FP64 base point).
#include <hip/hip_runtime.h>

#include "engine.h"

namespace cgl {

struct MixedWork {};

Problem::~Problem() { delete mixed; }

void solve_mixed(Problem& P, const cgl_node* nodes, int32_t count, double* beta_out,
                 cgl_result* res) {
  (void)P; (void)nodes; (void)count; (void)beta_out; (void)res;
  invalid("mixed precision is not available in this build");
}

}  // namespace cgl
