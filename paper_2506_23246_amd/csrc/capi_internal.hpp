// Internal definitions behind the opaque C handles.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qpinn.h"
#include "plain.hpp"
#include "plan.hpp"

struct qp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int cu_count = 0;
  size_t max_lds = 0;
  std::string arch;
  std::string err;
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct qp_circuit {
  qp_ctx* ctx = nullptr;
  qp::HostPlan hp;
  void* dplan_raw = nullptr;
  qp::QPlanDev* dplan = nullptr;
  std::vector<qp::PlainGate> pgates;
  qp::PlainGate* dpgates = nullptr;
  int exs = 4;         // exchange planes per LDS phase
  int wg_per_cu = 1;   // persistent workgroups per CU
  int dense_chunk = 0; // points per chunk of the dense-block path (0: about 2 GiB of statevectors)
  bool use_dense = false;   // the tuner's fusion width for Maxwell calls: dense 32x32 blocks
};

namespace qp {

struct WsLayout { size_t gtab, counts, angles, jac, mpart, lpart, m64, total; };

qp_status fail(qp_ctx* c, qp_status s, const char* fmt, ...);
qp_status hipcheck(qp_ctx* c, hipError_t e, const char* what);
void choose_launch(qp_ctx* ctx, qp_circuit* c);
int fused_grid(const qp_ctx* ctx, const qp_circuit* c, int64_t P);
WsLayout fused_layout(const qp_circuit* c, int64_t P, int grid_cap);
int n_moments(const qp_circuit* c);   // phase-stage moments of the fused adjoint (0 without CRZ)
qp_status run_fused(qp_ctx* ctx, const qp_circuit* c, int mode, const float* params, const float* points,
                    const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld, float* out,
                    float* tan, const float* d_out, const float* d_tan, double* loss, float* d_params,
                    float* d_angles, float* d_jac, void* ws, uint32_t flags, int exs_override, int grid_override,
                    const float* f_mir = nullptr, int n_mir = 0, float w_sym = 0.f, float w_energy = 0.f);
qp_status run_dense(qp_ctx* ctx, const qp_circuit* c, int mode, const float* params, const float* points,
                    const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld, float* out,
                    float* tan, const float* d_out, const float* d_tan, double* loss, float* d_params, void* ws,
                    uint32_t flags);
// Workspace a call with `flags` cannot do without (the fused path's, or the dense path's with
// QP_FLAG_DENSE_MFMA); qp_workspace_bytes may ask for more (see there).
size_t ws_required(const qp_circuit* c, int64_t P, uint32_t flags);
// Argument checks and launch sequence of the fused Maxwell evaluation (who names the entry point
// in error messages).
qp_status maxwell_entry(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                        const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld, float* out,
                        float* tan, double* loss, float* d_params, float* d_angles, float* d_jac, void* ws,
                        size_t ws_bytes, uint32_t flags, const char* who);

}  // namespace qp
