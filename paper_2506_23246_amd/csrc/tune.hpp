// Autotuner for the fused kernels' launch shape (LDS exchange depth, persistent workgroups
// per CU).  Results are cached in memory and in a JSON-lines file named by QP_TUNE_CACHE.
#pragma once
#include "capi_internal.hpp"

namespace qp {

struct TuneEntry {
  int exs;
  int wg_per_cu;
  double ms;
};

const TuneEntry* tune_lookup(const qp_ctx* ctx, const qp_circuit* c);
void tune_circuit(qp_ctx* ctx, qp_circuit* c, const float* params, const float* points, const float* angles,
                  const float* jac, int64_t P, const qp_maxwell_desc* ld, void* ws);
std::string tune_key(const qp_ctx* ctx, const qp_circuit* c);

}  // namespace qp
