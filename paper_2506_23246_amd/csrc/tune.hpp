// Autotuner of the Maxwell evaluation: the fused kernels' launch shape (LDS exchange depth,
// persistent workgroups per CU) and the fusion width (2x2 gates in registers, or 32x32 dense
// blocks streamed through HBM on the matrix cores).  Results are cached in memory and in a
// JSON-lines file named by QP_TUNE_CACHE.
#pragma once
#include "capi_internal.hpp"

namespace qp {

struct TuneEntry {
  int exs;
  int wg_per_cu;
  double ms;
  int dense = 0;   // 1: the dense-block path was the fastest
};

const TuneEntry* tune_lookup(const qp_ctx* ctx, const qp_circuit* c);
// dense_ok: the call may take the dense-block path (it has one, the workspace covers it and no
// input gradient is asked for); then that path is timed as one more candidate.
void tune_circuit(qp_ctx* ctx, qp_circuit* c, const float* params, const float* points, const float* angles,
                  const float* jac, int64_t P, const qp_maxwell_desc* ld, void* ws, bool dense_ok);
std::string tune_key(const qp_ctx* ctx, const qp_circuit* c);

}  // namespace qp
