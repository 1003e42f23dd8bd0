// qp_maxwell_fused_noalloc: the fused Maxwell evaluation with its per-call scratch in a fixed
// device array of the library instead of a caller workspace, for callers that cannot allocate.
//
// `scratch` below is a device symbol.  In host code its name is only a host-side stand-in, so
// the host never passes it to a kernel or a copy: on the first call on a device (with that
// device current) hipGetSymbolAddress gives that device's address of its own copy of the array,
// which is kept per device and passed to the kernels as the workspace pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qpinn.h"
#include "capi_internal.hpp"
#include "qp_internal.hpp"

namespace {

static_assert(QP_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) unsigned char scratch[QP_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[qp::kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255u)) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" size_t qp_noalloc_scratch_bytes(void) { return QP_NOALLOC_SCRATCH_BYTES; }

extern "C" qp_status qp_maxwell_fused_noalloc(qp_ctx* ctx, const qp_circuit* c, const float* params,
                                              const float* points, const float* angles, const float* jac,
                                              int64_t P, const qp_maxwell_desc* loss_desc, float* out,
                                              float* tan, double* loss, float* d_params, float* d_angles,
                                              float* d_jac, uint32_t flags) {
  const char* who = "qp_maxwell_fused_noalloc";
  if (!ctx || !c) return qp::fail(ctx, QP_EINVAL, "%s: null context or circuit", who);
  if (flags & (QP_FLAG_TUNE | QP_FLAG_DENSE_MFMA))
    return qp::fail(ctx, QP_EUNSUPPORTED, "%s: QP_FLAG_TUNE and QP_FLAG_DENSE_MFMA need a caller workspace", who);
  if (P < 0) return qp::fail(ctx, QP_EINVAL, "%s: P < 0", who);
  if (ctx->device < 0 || ctx->device >= qp::kMaxDevices)
    return qp::fail(ctx, QP_EUNSUPPORTED, "%s: device index %d out of range", who, ctx->device);
  const size_t need = qp::ws_required(c, P, 0);
  if (need > QP_NOALLOC_SCRATCH_BYTES)
    return qp::fail(ctx, QP_EWORKSPACE, "%s: this call needs %zu scratch bytes, above the fixed %zu; use qp_maxwell_fused "
                    "with a workspace or split the points", who, need, (size_t)QP_NOALLOC_SCRATCH_BYTES);
  hipError_t e = hipSetDevice(ctx->device);
  void* ws = nullptr;
  if (e == hipSuccess) e = scratch_address(ctx->device, &ws);
  if (e != hipSuccess) return qp::hipcheck(ctx, e, "qp_maxwell_fused_noalloc: scratch address");
  return qp::maxwell_entry(ctx, c, params, points, angles, jac, P, loss_desc, out, tan, loss, d_params, d_angles,
                           d_jac, ws, QP_NOALLOC_SCRATCH_BYTES, flags, who);
}
