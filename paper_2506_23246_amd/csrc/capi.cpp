// C ABI of the QPINN circuit engine: contexts, circuit compilation, workspace layout and the
// stream-ordered launch sequences of the fused, plain and batch paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qpinn.h"
#include "batch.hpp"
#include "dense.hpp"
#include "diag.hpp"
#include "capi_internal.hpp"
#include "fused.hpp"
#include "plain.hpp"
#include "plan.hpp"
#include "total.hpp"
#include "tune.hpp"

using namespace qp;

qp_status qp::fail(qp_ctx* c, qp_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

qp_status qp::hipcheck(qp_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return QP_OK;
  return fail(c, QP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- context -------------------
extern "C" qp_status qp_ctx_create(int device, void* stream, qp_ctx** out) {
  if (!out) return QP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return QP_EDEVICE;
  if (device < 0 || device >= ndev) return QP_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return QP_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return QP_EDEVICE;
  auto* c = new qp_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->cu_count = prop.multiProcessorCount;
  c->max_lds = prop.sharedMemPerBlock;
  c->arch = prop.gcnArchName;
  *out = c;
  return QP_OK;
}

extern "C" qp_status qp_ctx_set_stream(qp_ctx* c, void* stream) {
  if (!c) return QP_EINVAL;
  c->stream = static_cast<hipStream_t>(stream);
  return QP_OK;
}

extern "C" void qp_ctx_destroy(qp_ctx* c) {
  if (!c) return;
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  delete c;
}

extern "C" qp_status qp_ctx_enable_kernel_timing(qp_ctx* c, int32_t on) {
  if (!c) return QP_EINVAL;
  hipSetDevice(c->device);
  if (on && !c->ev0) {
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
      return fail(c, QP_EDEVICE, "qp_ctx_enable_kernel_timing: hipEventCreate failed");
  }
  c->timing = on != 0;
  return QP_OK;
}

extern "C" qp_status qp_ctx_last_kernel_ms(qp_ctx* c, float* ms) {
  if (!c || !ms) return QP_EINVAL;
  if (!c->ev0) return fail(c, QP_EINVAL, "qp_ctx_last_kernel_ms: timing was never enabled");
  hipSetDevice(c->device);
  hipError_t e = hipEventSynchronize(c->ev1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, c->ev0, c->ev1);
  return hipcheck(c, e, "qp_ctx_last_kernel_ms");
}

extern "C" const char* qp_last_error(const qp_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" qp_status qp_sync(qp_ctx* c) {
  if (!c) return QP_EINVAL;
  hipSetDevice(c->device);
  return hipcheck(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

extern "C" int32_t qp_device_cu_count(const qp_ctx* c) { return c ? c->cu_count : 0; }

// ---------------------------------------------------------------- circuits ------------------
extern "C" qp_status qp_circuit_compile(qp_ctx* ctx, const qp_circuit_desc* d, qp_circuit** out) {
  if (!ctx || !d || !out) return fail(ctx, QP_EINVAL, "qp_circuit_compile: null argument");
  *out = nullptr;
  auto* c = new qp_circuit();
  c->ctx = ctx;
  int status = QP_OK;
  std::string msg = build_plan(d, &c->hp, &status);
  if (!msg.empty() || status != QP_OK) {
    delete c;
    return fail(ctx, (qp_status)status, "qp_circuit_compile: %s", msg.c_str());
  }
  hipSetDevice(ctx->device);
  // plain-path gate list (device copy for the gate-table kernel)
  c->pgates.resize(c->hp.gates.size());
  for (size_t i = 0; i < c->hp.gates.size(); ++i)
    c->pgates[i] = PlainGate{c->hp.gates[i].kind, c->hp.gates[i].q0, c->hp.gates[i].q1, c->hp.gates[i].param};
  size_t bytes = c->hp.blob.size() + sizeof(PlainGate) * std::max<size_t>(1, c->pgates.size()) + 256;
  if (hipMalloc(&c->dplan_raw, bytes) != hipSuccess) {
    delete c;
    return fail(ctx, QP_EDEVICE, "qp_circuit_compile: hipMalloc of %zu plan bytes failed", bytes);
  }
  c->dplan = static_cast<QPlanDev*>(c->dplan_raw);
  c->dpgates = reinterpret_cast<PlainGate*>(static_cast<char*>(c->dplan_raw) + ((c->hp.blob.size() + 255) & ~size_t(255)));
  hipError_t e = hipMemcpy(c->dplan_raw, c->hp.blob.data(), c->hp.blob.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !c->pgates.empty())
    e = hipMemcpy(c->dpgates, c->pgates.data(), sizeof(PlainGate) * c->pgates.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(c->dplan_raw);
    delete c;
    return fail(ctx, QP_EDEVICE, "qp_circuit_compile: upload failed: %s", hipGetErrorString(e));
  }
  if (c->hp.fused_ok) choose_launch(ctx, c);
  *out = c;
  return QP_OK;
}

extern "C" qp_status qp_circuit_set_launch(qp_circuit* c, int32_t exchange_planes, int32_t wg_per_cu) {
  if (!c) return QP_EINVAL;
  if (!c->hp.fused_ok) return fail(c->ctx, QP_EUNSUPPORTED, "qp_circuit_set_launch: %s", c->hp.fused_reason.c_str());
  if (exchange_planes != 2 && exchange_planes != 4)
    return fail(c->ctx, QP_EINVAL, "qp_circuit_set_launch: exchange_planes must be 2 or 4");
  const int max_wg = fused_max_wg_per_cu(c->hp.n);
  if (exchange_planes == 4 && !c->hp.phases.empty())
    return fail(c->ctx, QP_EINVAL, "qp_circuit_set_launch: circuits with CRZ phase stages run with 2 exchange planes");
  const size_t lds = fused_lds_bytes(c->hp.n, exchange_planes, (int)c->hp.fused.size(), n_moments(c));
  if (wg_per_cu < 1 || wg_per_cu > max_wg || lds * (size_t)wg_per_cu > 160 * 1024)
    return fail(c->ctx, QP_EINVAL, "qp_circuit_set_launch: %d workgroups of %zu LDS bytes do not fit a CU", wg_per_cu, lds);
  c->exs = exchange_planes;
  c->wg_per_cu = wg_per_cu;
  c->use_dense = false;   // an explicit launch shape of the fused kernel
  return QP_OK;
}

extern "C" qp_status qp_circuit_set_dense_chunk(qp_circuit* c, int32_t points) {
  if (!c) return QP_EINVAL;
  if (points < 0 || points % 64 != 0)
    return fail(c->ctx, QP_EINVAL, "qp_circuit_set_dense_chunk: points must be 0 or a positive multiple of 64");
  c->dense_chunk = points;
  return QP_OK;
}

extern "C" qp_status qp_plan_image(const qp_circuit_desc* d, void* host_buf, size_t cap, size_t* bytes) {
  if (!d || !bytes) return QP_EINVAL;
  HostPlan hp;
  int status = QP_OK;
  std::string msg = build_plan(d, &hp, &status);
  if (!msg.empty() || status != QP_OK) return status != QP_OK ? (qp_status)status : QP_EINVAL;
  if (!hp.fused_ok) return QP_EUNSUPPORTED;
  *bytes = hp.blob.size();
  if (!host_buf || cap < hp.blob.size()) return QP_EWORKSPACE;
  std::memcpy(host_buf, hp.blob.data(), hp.blob.size());
  return QP_OK;
}

extern "C" void qp_circuit_destroy(qp_circuit* c) {
  if (!c) return;
  if (c->dplan_raw) hipFree(c->dplan_raw);
  delete c;
}

extern "C" int64_t qp_circuit_info(const qp_circuit* c, int32_t what) {
  if (!c) return -1;
  switch (what) {
    case 0: return c->hp.n;
    case 1: return c->hp.K;
    case 2: return c->hp.m;
    case 3: return (int64_t)c->hp.fused.size();
    case 4: return (int64_t)c->hp.rounds.size();
    case 5: return c->hp.n_exchanges;
    case 6: return c->hp.fused_ok ? fused_threads(c->hp.n) : 0;
    case 7: return c->hp.fused_ok ? fused_points_per_tile(c->hp.n) : 0;
    case 8: return c->exs;
    case 9: return c->wg_per_cu;
    case 10: return c->hp.dense_ok ? (int64_t)c->hp.dgroups.size() : 0;
    case 11: return c->hp.fused_ok ? c->hp.n_head : 0;
    case 12: {
      int64_t h = 0;
      if (c->hp.fused_ok)
        for (const auto& f : c->hp.fused) h += f.stat_out ? 1 : 0;
      return h;
    }
    case 13: return c->use_dense ? 1 : 0;
    default: return -1;
  }
}

// Launch shape: points per tile are fixed by n; the LDS exchange depth (EXS statevector
// planes per phase) and the persistent grid (workgroups per CU) come from the LDS budget,
// optionally refined by the autotuner.
void qp::choose_launch(qp_ctx* ctx, qp_circuit* c) {
  const int n = c->hp.n;
  const int F = (int)c->hp.fused.size();
  const size_t lds_cap = 160 * 1024;
  const int T = fused_threads(n);
  const int max_wg_vgpr = (T == 512) ? 1 : 2;   // ~256 VGPRs per lane: 2 waves per SIMD
  const int NM = n_moments(c);
  c->exs = 4;
  size_t lds = fused_lds_bytes(n, 4, F, NM);
  if (lds * max_wg_vgpr > lds_cap || NM > 0) {   // phase stages are applied by the unpipelined kernel
    c->exs = 2;
    lds = fused_lds_bytes(n, 2, F, NM);
  }
  int wg = (int)std::min<size_t>(max_wg_vgpr, lds_cap / std::max<size_t>(lds, 1));
  c->wg_per_cu = std::max(wg, 1);
  const TuneEntry* te = tune_lookup(ctx, c);
  if (te && !(NM > 0 && te->exs == 4)) {
    c->exs = te->exs;
    c->wg_per_cu = te->wg_per_cu;
    c->use_dense = te->dense != 0 && c->hp.dense_ok;
  }
}

int qp::n_moments(const qp_circuit* c) { return (int)c->hp.phases.size() * phase_terms(c->hp.n); }

int qp::fused_grid(const qp_ctx* ctx, const qp_circuit* c, int64_t P) {
  const int ppw = fused_points_per_tile(c->hp.n);
  const int64_t ntiles = (P + ppw - 1) / ppw;
  const int64_t cap = (int64_t)ctx->cu_count * c->wg_per_cu;
  return (int)std::min<int64_t>(ntiles, cap);
}

WsLayout qp::fused_layout(const qp_circuit* c, int64_t P, int grid_cap) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  WsLayout L{};
  const int F = (int)c->hp.fused.size();
  const int NM = n_moments(c);
  size_t off = 0;
  L.gtab = off; off = al(off + sizeof(float) * kGT * (F + 1) + sizeof(uint32_t) * NM);   // + identity, phases
  L.counts = off; off = al(off + 2 * sizeof(int));
  if (c->hp.enc_kind == QP_ENC_RFF) {
    L.angles = off; off = al(off + sizeof(float) * (size_t)P * c->hp.n);
    L.jac = off; off = al(off + sizeof(float) * (size_t)P * c->hp.n * 3);
  }
  L.mpart = off; off = al(off + sizeof(float) * (size_t)grid_cap * (F * kGS + NM));
  L.lpart = off; off = al(off + sizeof(float) * (size_t)std::max(grid_cap, 1));
  L.m64 = off; off = al(off + sizeof(double) * ((size_t)std::max(F, 1) * kGS + NM));
  L.total = off;
  return L;
}

static int dense_nwg(const qp_ctx* ctx, const qp_circuit* c, int Pc) {
  const long long tiles = (1ll << (c->hp.n - 5)) * ((Pc + 63) / 64);
  return (int)std::max<long long>(1, std::min<long long>(tiles, (long long)ctx->cu_count * 4));
}

static DenseLayout dense_ws(const qp_circuit* c, int64_t P, bool grad, int* Pc_out, int* nwg_out) {
  int Pc = dense_chunk(c->hp.n, P, grad);
  if (c->dense_chunk > 0 && c->dense_chunk < Pc) Pc = c->dense_chunk;
  const int nwg = dense_nwg(c->ctx, c, Pc);
  if (Pc_out) *Pc_out = Pc;
  if (nwg_out) *nwg_out = nwg;
  return dense_layout(c->hp.n, c->hp.m, (int)c->hp.dgroups.size(), (int)c->hp.docc.size() / 2, P, Pc, nwg, grad);
}

size_t qp::ws_required(const qp_circuit* c, int64_t P, uint32_t flags) {
  if (flags & QP_FLAG_DENSE_MFMA) return c->hp.dense_ok ? dense_ws(c, P, true, nullptr, nullptr).total : 0;
  const int cap = c->ctx->cu_count * 4;   // covers every launch shape the tuner may pick
  return fused_layout(c, P, cap).total;
}

// With QP_FLAG_TUNE, or once the tuner chose the dense-block path, also large enough for that
// path, so that the tuner can time it and Maxwell calls can take it; a smaller workspace (at
// least the fused path's) is accepted and then keeps Maxwell calls on the fused path.
extern "C" size_t qp_workspace_bytes(const qp_circuit* c, int64_t P, uint32_t flags) {
  if (!c || P < 0) return 0;
  size_t need = ws_required(c, P, flags);
  if (!(flags & QP_FLAG_DENSE_MFMA) && ((flags & QP_FLAG_TUNE) || c->use_dense) && c->hp.dense_ok)
    need = std::max(need, ws_required(c, P, QP_FLAG_DENSE_MFMA));
  return need;
}

static qp_status check_common(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                              const float* angles, const float* jac, int64_t P, void* ws, size_t ws_bytes,
                              const char* who, uint32_t flags) {
  if (!ctx || !c) return fail(ctx, QP_EINVAL, "%s: null context or circuit", who);
  if (P < 0) return fail(ctx, QP_EINVAL, "%s: P < 0", who);
  if (P > (int64_t)INT32_MAX)   // point and tile indices are 32-bit in the kernels
    return fail(ctx, QP_EUNSUPPORTED, "%s: P = %lld exceeds 2^31 - 1 points per call; split the call", who,
                (long long)P);
  if (!c->hp.fused_ok && !(flags & QP_FLAG_DENSE_MFMA))
    return fail(ctx, QP_EUNSUPPORTED, "%s: %s", who, c->hp.fused_reason.c_str());
  if (c->hp.K > 0 && !params) return fail(ctx, QP_EINVAL, "%s: params is null", who);
  if (P > 0) {
    if (c->hp.enc_kind == QP_ENC_ANGLES) {
      if (!angles || !jac) return fail(ctx, QP_EINVAL, "%s: angle-given encoding needs angles and jac", who);
    } else if (!points) {
      return fail(ctx, QP_EINVAL, "%s: points is null", who);
    }
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(ctx, QP_EWORKSPACE, "%s: workspace null or not 256-byte aligned", who);
  if (ws_bytes < ws_required(c, P, flags))
    return fail(ctx, QP_EWORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, ws_required(c, P, flags));
  return QP_OK;
}

// Dense-block MFMA sequence (QP_FLAG_DENSE_MFMA, or the tuner's choice for Maxwell calls) for the
// three evaluation entry points.
qp_status qp::run_dense(qp_ctx* ctx, const qp_circuit* c, int mode, const float* params, const float* points,
                           const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld, float* out,
                           float* tan, const float* d_out, const float* d_tan, double* loss, float* d_params, void* ws,
                           uint32_t flags) {
  if (!c->hp.dense_ok) return fail(ctx, QP_EUNSUPPORTED, "dense-block path needs 5..12 qubits");
  hipSetDevice(ctx->device);
  hipStream_t st = ctx->stream;
  DenseCall d{};
  d.L = dense_ws(c, P, true, &d.Pc, &d.nwg);
  d.plan = c->dplan;
  d.n = c->hp.n;
  d.m = c->hp.m;
  d.G = (int)c->hp.dgroups.size();
  d.K = c->hp.K;
  d.n_docc = (int)c->hp.docc.size() / 2;
  d.params = params;
  d.points = points;
  d.angles = angles;
  d.jac = jac;
  d.P = P;
  d.apply_grid = ctx->cu_count * 8;
  d.grad = mode != kModeFwd;
  d.out = out;
  d.tan = tan;
  d.loss_out = loss;
  d.d_params = d_params;
  d.ws = ws;
  char* w = static_cast<char*>(ws);
  hipError_t e = hipSuccess;
  if (c->hp.enc_kind == QP_ENC_RFF) {
    d.angles = reinterpret_cast<float*>(w + d.L.angles);
    d.jac = reinterpret_cast<float*>(w + d.L.jac);
    if ((e = launch_rff(c->dplan, points, P, const_cast<float*>(d.angles), const_cast<float*>(d.jac), st)) != hipSuccess)
      return hipcheck(ctx, e, "rff angles");
  }
  int* counts = reinterpret_cast<int*>(w + d.L.counts);
  d.loss.maxwell = mode == kModeMaxwell;
  d.loss.kind = ld ? ld->kind : QP_LOSS_VACUUM;
  d.loss.loss_sum = (flags & QP_FLAG_LOSS_SUM) ? 1 : 0;
  d.loss.eps_r = ld ? ld->eps_r : 1.f;
  d.loss.x_if = ld ? ld->x_interface : 0.f;
  d.loss.w_all = d.loss.loss_sum ? 1.f : (P > 0 ? 1.f / (float)P : 0.f);
  d.loss.counts = counts;
  d.loss.points = points;
  d.loss.d_out = d_out;
  d.loss.d_tan = d_tan;
  if (mode == kModeMaxwell && ld->kind == QP_LOSS_DIEL_SPLIT)
    if ((e = launch_count(points, P, ld->x_interface, counts, st)) != hipSuccess) return hipcheck(ctx, e, "count");
  if (ctx->timing) hipEventRecord(ctx->ev0, st);
  e = dense_run(d, st);
  if (ctx->timing) hipEventRecord(ctx->ev1, st);
  return hipcheck(ctx, e, "dense-block path");
}

// Shared launch sequence of the three fused entry points.
qp_status qp::run_fused(qp_ctx* ctx, const qp_circuit* c, int mode, const float* params, const float* points,
                        const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld, float* out,
                        float* tan, const float* d_out, const float* d_tan, double* loss, float* d_params,
                        float* d_angles, float* d_jac, void* ws, uint32_t flags, int exs_override, int grid_override,
                        const float* f_mir, int n_mir, float w_sym, float w_energy) {
  hipSetDevice(ctx->device);
  hipStream_t st = ctx->stream;
  const int n = c->hp.n;
  const int F = (int)c->hp.fused.size();
  const int cap = ctx->cu_count * 4;
  const WsLayout L = fused_layout(c, P, cap);
  char* w = static_cast<char*>(ws);
  float* gtab = reinterpret_cast<float*>(w + L.gtab);
  int* counts = reinterpret_cast<int*>(w + L.counts);
  const int NM = n_moments(c);
  hipError_t e = launch_gate_table(c->dplan, F, NM, params, gtab, (flags & QP_FLAG_GATES_FP32) ? 1 : 0, st);
  if (e != hipSuccess) return hipcheck(ctx, e, "gate table");
  const float* ang = angles;
  const float* jc = jac;
  if (c->hp.enc_kind == QP_ENC_RFF) {
    ang = reinterpret_cast<float*>(w + L.angles);
    jc = reinterpret_cast<float*>(w + L.jac);
    if ((e = launch_rff(c->dplan, points, P, const_cast<float*>(ang), const_cast<float*>(jc), st)) != hipSuccess)
      return hipcheck(ctx, e, "rff angles");
  }
  if ((mode == kModeMaxwell || mode == kModeTotal) && ld->kind == QP_LOSS_DIEL_SPLIT) {
    if ((e = launch_count(points, P, ld->x_interface, counts, st)) != hipSuccess) return hipcheck(ctx, e, "count");
  }
  // packed modes: four points per thread group, so a tile covers four times the points
  const int64_t P_slots = mode_packed(mode) ? (P + 3) / 4 : P;
  int grid = fused_grid(ctx, c, P_slots);
  if (grid_override > 0)
    grid = (int)std::min<int64_t>(grid_override, (P_slots + fused_points_per_tile(n) - 1) / fused_points_per_tile(n));
  grid = std::min(grid, cap);
  const int exs = NM > 0 ? 2 : (exs_override > 0 ? exs_override : c->exs);   // phases: unpipelined kernel
  const size_t lds = fused_lds_bytes(n, exs, F, NM);
  FusedArgs a{};
  a.plan = c->dplan;
  a.gtab = gtab;
  a.points = points;
  a.angles = ang;
  a.jac = jc;
  a.P = P;
  a.ntiles = (int)((P_slots + fused_points_per_tile(n) - 1) / fused_points_per_tile(n));
  a.n_fused = F;
  a.out = out;
  a.tan = tan;
  a.d_out = d_out;
  a.d_tan = d_tan;
  a.loss_kind = ld ? ld->kind : QP_LOSS_VACUUM;
  a.loss_sum = (flags & QP_FLAG_LOSS_SUM) ? 1 : 0;
  a.eps_r = ld ? ld->eps_r : 1.f;
  a.x_if = ld ? ld->x_interface : 0.f;
  a.counts = counts;
  a.mpart = reinterpret_cast<float*>(w + L.mpart);
  a.lpart = reinterpret_cast<float*>(w + L.lpart);
  a.n_mom = NM;
  a.f_mir = f_mir;
  a.n_mir = n_mir;
  a.w_sym = w_sym;
  a.w_energy = w_energy;
  a.d_angles = (mode == kModeMaxwell || mode == kModeVjp) ? d_angles : nullptr;
  a.d_jac = (mode == kModeMaxwell || mode == kModeVjp) ? d_jac : nullptr;
  if (mode_packed(mode)) { a.tan = nullptr; a.d_tan = nullptr; }
  if (grid > 0) {
    if (ctx->timing) hipEventRecord(ctx->ev0, st);
    if ((e = launch_fused(n, mode, a, grid, exs, c->hp.has_signs, lds, st)) != hipSuccess) return hipcheck(ctx, e, "fused kernel");
    if (ctx->timing) hipEventRecord(ctx->ev1, st);
  }
  if (mode_fwd_only(mode) || (!loss && !d_params)) return QP_OK;   // the tuner times the main kernel only
  double* m64 = reinterpret_cast<double*>(w + L.m64);
  if ((e = launch_reduce(a.mpart, grid, F * kGS + NM, mode == kModeMaxwell ? a.lpart : nullptr, m64,
                         mode == kModeMaxwell ? loss : nullptr, st)) != hipSuccess)
    return hipcheck(ctx, e, "reduce");
  if (d_params && (e = launch_param_grads(c->dplan, c->hp.K, params, m64, d_params, st)) != hipSuccess)
    return hipcheck(ctx, e, "param grads");
  return QP_OK;
}

extern "C" qp_status qp_simulate(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                                 const float* angles, const float* jac, int64_t P, float* out, float* tan, void* ws,
                                 size_t ws_bytes, uint32_t flags) {
  qp_status s = check_common(ctx, c, params, points, angles, jac, P, ws, ws_bytes, "qp_simulate", flags);
  if (s != QP_OK) return s;
  if (P > 0 && !out) return fail(ctx, QP_EINVAL, "qp_simulate: out is null");
  if (P > 0 && !tan && !(flags & QP_FLAG_NO_TANGENTS)) return fail(ctx, QP_EINVAL, "qp_simulate: tan is null");
  if (flags & QP_FLAG_DENSE_MFMA)
    return run_dense(ctx, c, kModeFwd, params, points, angles, jac, P, nullptr, out,
                     (flags & QP_FLAG_NO_TANGENTS) ? nullptr : tan, nullptr, nullptr, nullptr, nullptr, ws, flags);
  // outputs alone: the packed kernel (four points per thread group, no tangent statevectors)
  const bool no_tan = (flags & QP_FLAG_NO_TANGENTS) != 0;
  return run_fused(ctx, c, no_tan ? kModeFwdPk : kModeFwd, params, points, angles, jac, P, nullptr, out,
                   no_tan ? nullptr : tan, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, ws, flags, 0, 0);
}

// Input gradients (dL/d angles, dL/d Jacobian) exist for the angle-given encoding on the fused path.
static qp_status check_input_grads(qp_ctx* ctx, const qp_circuit* c, float* d_angles, float* d_jac, int64_t P,
                                   uint32_t flags, const char* who) {
  if (!d_angles && !d_jac) return QP_OK;
  if (c->hp.enc_kind != QP_ENC_ANGLES)
    return fail(ctx, QP_EINVAL, "%s: d_angles/d_jac need the angle-given encoding (QP_ENC_ANGLES)", who);
  if (flags & QP_FLAG_DENSE_MFMA)
    return fail(ctx, QP_EUNSUPPORTED, "%s: d_angles/d_jac are not computed by the dense-block path", who);
  (void)P;
  return QP_OK;
}

extern "C" qp_status qp_vjp(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                            const float* angles, const float* jac, int64_t P, const float* d_out, const float* d_tan,
                            float* d_params, float* d_angles, float* d_jac, void* ws, size_t ws_bytes,
                            uint32_t flags) {
  qp_status s = check_common(ctx, c, params, points, angles, jac, P, ws, ws_bytes, "qp_vjp", flags);
  if (s != QP_OK) return s;
  if (c->hp.K > 0 && !d_params) return fail(ctx, QP_EINVAL, "qp_vjp: d_params is null");
  if ((s = check_input_grads(ctx, c, d_angles, d_jac, P, flags, "qp_vjp")) != QP_OK) return s;
  if (flags & QP_FLAG_DENSE_MFMA)
    return run_dense(ctx, c, kModeVjp, params, points, angles, jac, P, nullptr, nullptr, nullptr, d_out, d_tan, nullptr,
                     d_params, ws, flags);
  return run_fused(ctx, c, kModeVjp, params, points, angles, jac, P, nullptr, nullptr, nullptr, d_out, d_tan, nullptr,
                   d_params, d_angles, d_jac, ws, flags, 0, 0);
}

qp_status qp::maxwell_entry(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                            const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld, float* out,
                            float* tan, double* loss, float* d_params, float* d_angles, float* d_jac, void* ws,
                            size_t ws_bytes, uint32_t flags, const char* who) {
  qp_status s = check_common(ctx, c, params, points, angles, jac, P, ws, ws_bytes, who, flags);
  if (s != QP_OK) return s;
  if (!ld) return fail(ctx, QP_EINVAL, "%s: loss descriptor is null", who);
  if (ld->kind < QP_LOSS_VACUUM || ld->kind > QP_LOSS_DIEL_INTUITIVE) return fail(ctx, QP_EINVAL, "%s: unknown loss kind", who);
  if (c->hp.m < 3) return fail(ctx, QP_ESHAPE, "%s: the Maxwell loss needs 3 outputs (E_z, H_x, H_y)", who);
  if (ld->kind != QP_LOSS_VACUUM && P > 0 && !points) return fail(ctx, QP_EINVAL, "%s: dielectric loss needs points", who);
  if (!loss || (c->hp.K > 0 && !d_params)) return fail(ctx, QP_EINVAL, "%s: loss/d_params null", who);
  if ((s = check_input_grads(ctx, c, d_angles, d_jac, P, flags, who)) != QP_OK) return s;
  if (flags & QP_FLAG_DENSE_MFMA)
    return run_dense(ctx, c, kModeMaxwell, params, points, angles, jac, P, ld, out, tan, nullptr, nullptr, loss, d_params,
                     ws, flags);
  // the dense-block path is open to this call: the circuit has one, the workspace covers it and
  // no input gradient is asked for (that path does not form them)
  const bool dense_open = c->hp.dense_ok && !d_angles && !d_jac && ws_bytes >= ws_required(c, P, QP_FLAG_DENSE_MFMA);
  if ((flags & QP_FLAG_TUNE) && P > 0)
    tune_circuit(ctx, const_cast<qp_circuit*>(c), params, points, angles, jac, P, ld, ws, dense_open);
  if (c->use_dense && dense_open)
    return run_dense(ctx, c, kModeMaxwell, params, points, angles, jac, P, ld, out, tan, nullptr, nullptr, loss, d_params,
                     ws, flags);
  return run_fused(ctx, c, kModeMaxwell, params, points, angles, jac, P, ld, out, tan, nullptr, nullptr, loss, d_params,
                   d_angles, d_jac, ws, flags, 0, 0);
}

extern "C" qp_status qp_maxwell_fused(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                                      const float* angles, const float* jac, int64_t P, const qp_maxwell_desc* ld,
                                      float* out, float* tan, double* loss, float* d_params, float* d_angles,
                                      float* d_jac, void* ws, size_t ws_bytes, uint32_t flags) {
  return maxwell_entry(ctx, c, params, points, angles, jac, P, ld, out, tan, loss, d_params, d_angles, d_jac, ws,
                       ws_bytes, flags, "qp_maxwell_fused");
}

// ---------------------------------------------------------------- diagnostics ---------------
static PlainProblem plain_problem(const qp_circuit* c, int64_t P);

extern "C" qp_status qp_bloch(qp_ctx* ctx, const qp_circuit* c, int32_t precision, const void* params,
                              const void* points, const void* angles, int64_t P, void* bloch, void* mw, void* ws,
                              size_t ws_bytes) {
  const char* who = "qp_bloch";
  if (!ctx || !c) return fail(ctx, QP_EINVAL, "%s: null context or circuit", who);
  if (precision != 32 && precision != 64) return fail(ctx, QP_EINVAL, "%s: precision must be 32 or 64", who);
  if (P < 0) return fail(ctx, QP_EINVAL, "%s: P < 0", who);
  const bool given = c->hp.enc_kind == QP_ENC_ANGLES;
  if ((c->hp.K > 0 && !params) || (P > 0 && (given ? !angles : !points)) || (P > 0 && !bloch))
    return fail(ctx, QP_EINVAL, "%s: null params, %s or bloch", who, given ? "angles" : "points");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(ctx, QP_EWORKSPACE, "%s: workspace null or misaligned", who);
  if (ws_bytes < qp_plain_workspace_bytes(c, P, precision)) return fail(ctx, QP_EWORKSPACE, "%s: workspace too small", who);
  hipSetDevice(ctx->device);
  return hipcheck(ctx, plain_bloch(plain_problem(c, P), precision, params, given ? nullptr : points,
                                   given ? angles : nullptr, bloch, mw, ws, ctx->stream),
                  "bloch");
}

namespace {
struct EnergyLayout { size_t pts, out, fused, total; int64_t P; };
EnergyLayout energy_layout(const qp_circuit* c, int64_t Nt, int64_t Nx, int64_t Ny) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  EnergyLayout L{};
  L.P = Nt * Nx * Ny;
  size_t off = 0;
  L.pts = off; off = al(off + sizeof(float) * 3 * (size_t)L.P);
  L.out = off; off = al(off + sizeof(float) * c->hp.m * (size_t)L.P);
  L.fused = off; off = al(off + fused_layout(c, L.P, c->ctx->cu_count * 4).total);
  L.total = off;
  return L;
}
}  // namespace

extern "C" size_t qp_energy_workspace_bytes(const qp_circuit* c, int64_t Nt, int64_t Nx, int64_t Ny) {
  if (!c || Nt < 0 || Nx < 0 || Ny < 0) return 0;
  return energy_layout(c, Nt, Nx, Ny).total;
}

extern "C" qp_status qp_energy_profile(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* t,
                                       int64_t Nt, const float* xg, int64_t Nx, const float* yg, int64_t Ny,
                                       const qp_maxwell_desc* desc, double* U, void* ws, size_t ws_bytes,
                                       uint32_t flags) {
  const char* who = "qp_energy_profile";
  if (!ctx || !c) return fail(ctx, QP_EINVAL, "%s: null context or circuit", who);
  if (Nt < 0 || Nx < 0 || Ny < 0) return fail(ctx, QP_EINVAL, "%s: negative grid size", who);
  if (c->hp.enc_kind == QP_ENC_ANGLES) return fail(ctx, QP_EINVAL, "%s: the grid needs a point encoding", who);
  if (!c->hp.fused_ok) return fail(ctx, QP_EUNSUPPORTED, "%s: %s", who, c->hp.fused_reason.c_str());
  if (c->hp.m < 3) return fail(ctx, QP_ESHAPE, "%s: the energy needs 3 outputs (E_z, H_x, H_y)", who);
  if (flags & ~QP_FLAG_GATES_FP32) return fail(ctx, QP_EUNSUPPORTED, "%s: only QP_FLAG_GATES_FP32 is supported", who);
  const EnergyLayout L = energy_layout(c, Nt, Nx, Ny);
  if (L.P > (int64_t)INT32_MAX) return fail(ctx, QP_EUNSUPPORTED, "%s: grid too large for one call", who);
  if ((c->hp.K > 0 && !params) || (Nt > 0 && (!t || !U)) || (L.P > 0 && (!xg || !yg)))
    return fail(ctx, QP_EINVAL, "%s: null pointer argument", who);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(ctx, QP_EWORKSPACE, "%s: workspace null or misaligned", who);
  if (ws_bytes < L.total) return fail(ctx, QP_EWORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, L.total);
  hipSetDevice(ctx->device);
  hipStream_t st = ctx->stream;
  char* w = static_cast<char*>(ws);
  float* pts = reinterpret_cast<float*>(w + L.pts);
  float* f = reinterpret_cast<float*>(w + L.out);
  hipError_t e = launch_energy_grid(t, Nt, xg, Nx, yg, Ny, pts, st);
  if (e != hipSuccess) return hipcheck(ctx, e, "energy grid");
  qp_status s = run_fused(ctx, c, kModeFwdPk, params, pts, nullptr, nullptr, L.P, nullptr, f, nullptr, nullptr, nullptr,
                          nullptr, nullptr, nullptr, nullptr, w + L.fused, flags, 0, 0);
  if (s != QP_OK) return s;
  const int diel = desc && desc->kind != QP_LOSS_VACUUM;
  e = launch_energy_reduce(f, c->hp.m, pts, Nt, Nx * Ny, diel, desc ? desc->eps_r : 1.f, desc ? desc->x_interface : 0.f,
                           U, st);
  return hipcheck(ctx, e, "energy reduce");
}

// ---------------------------------------------------------------- total loss ----------------
namespace {
struct TotalLayout { size_t ext, out, tan, dout, dtan, dtmp, part, counts, fused, total; int64_t P_ext, ic_base; int with_mx; };

TotalLayout total_layout(const qp_circuit* c, int64_t P, int64_t P0, int phys_kind) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  TotalLayout L{};
  L.with_mx = phys_kind == QP_LOSS_VACUUM ? 1 : 0;
  L.ic_base = P * (L.with_mx ? 3 : 2);
  L.P_ext = L.ic_base + P0;
  const size_t m = (size_t)c->hp.m, Pe = (size_t)L.P_ext;
  size_t off = 0;
  L.ext = off; off = al(off + sizeof(float) * 3 * Pe);
  L.out = off; off = al(off + sizeof(float) * m * Pe);
  L.tan = off; off = al(off + sizeof(float) * 3 * m * (size_t)P);   // tangents of the collocation points only
  L.dout = off; off = al(off + sizeof(float) * m * Pe);
  L.dtan = off; off = al(off + sizeof(float) * 3 * m * (size_t)P);
  L.dtmp = off; off = al(off + sizeof(float) * (size_t)std::max(1, c->hp.K));
  L.part = off; off = al(off + sizeof(float) * 4 * (size_t)std::max(1, total_seed_blocks(P, P0)));
  L.counts = off; off = al(off + 2 * sizeof(int));
  L.fused = off; off = al(off + fused_layout(c, L.P_ext, c->ctx->cu_count * 4).total);
  L.total = off;
  return L;
}
}  // namespace

extern "C" size_t qp_total_workspace_bytes(const qp_circuit* c, int64_t P, int64_t P0, int32_t phys_kind) {
  if (!c || P < 0 || P0 < 0) return 0;
  return total_layout(c, P, P0, phys_kind).total;
}

extern "C" qp_status qp_total_loss(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                                   int64_t P, const float* ic_xy, int64_t P0, const qp_total_loss_desc* d,
                                   float* out, float* tan, double* loss_terms, float* d_params, void* ws,
                                   size_t ws_bytes, uint32_t flags) {
  const char* who = "qp_total_loss";
  if (!ctx || !c) return fail(ctx, QP_EINVAL, "%s: null context or circuit", who);
  if (!d) return fail(ctx, QP_EINVAL, "%s: loss descriptor is null", who);
  const int kind = d->phys.kind;
  if (kind < QP_LOSS_VACUUM || kind > QP_LOSS_DIEL_INTUITIVE) return fail(ctx, QP_EINVAL, "%s: unknown loss kind", who);
  if (P < 0 || P0 < 0) return fail(ctx, QP_EINVAL, "%s: P < 0 or P0 < 0", who);
  if (c->hp.enc_kind == QP_ENC_ANGLES)
    return fail(ctx, QP_EINVAL, "%s: the mirrored and initial-condition points need a point encoding", who);
  if (!c->hp.fused_ok) return fail(ctx, QP_EUNSUPPORTED, "%s: %s", who, c->hp.fused_reason.c_str());
  if (c->hp.m < 3) return fail(ctx, QP_ESHAPE, "%s: the loss needs 3 outputs (E_z, H_x, H_y)", who);
  if (flags & (QP_FLAG_DENSE_MFMA | QP_FLAG_LOSS_SUM | QP_FLAG_TUNE))
    return fail(ctx, QP_EUNSUPPORTED, "%s: flags other than QP_FLAG_GATES_FP32 are not supported", who);
  const TotalLayout L = total_layout(c, P, P0, kind);
  if (L.P_ext > (int64_t)INT32_MAX) return fail(ctx, QP_EUNSUPPORTED, "%s: too many points for one call", who);
  if ((c->hp.K > 0 && (!params || !d_params)) || (P > 0 && !points) || (P0 > 0 && !ic_xy) || !loss_terms)
    return fail(ctx, QP_EINVAL, "%s: null pointer argument", who);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(ctx, QP_EWORKSPACE, "%s: workspace null or misaligned", who);
  if (ws_bytes < L.total) return fail(ctx, QP_EWORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, L.total);
  hipSetDevice(ctx->device);
  hipStream_t st = ctx->stream;
  char* w = static_cast<char*>(ws);
  float* ext = reinterpret_cast<float*>(w + L.ext);
  float* fo = reinterpret_cast<float*>(w + L.out);
  float* fg = reinterpret_cast<float*>(w + L.tan);
  float* dout = reinterpret_cast<float*>(w + L.dout);
  float* dtan = reinterpret_cast<float*>(w + L.dtan);
  int* counts = reinterpret_cast<int*>(w + L.counts);
  void* fws = w + L.fused;
  const uint32_t gflags = flags & QP_FLAG_GATES_FP32;
  hipError_t e = launch_total_points(points, P, ic_xy, P0, L.with_mx, ext, st);
  if (e != hipSuccess) return hipcheck(ctx, e, "total-loss points");
  if (kind == QP_LOSS_DIEL_SPLIT && (e = launch_count(points, P, d->phys.x_interface, counts, st)) != hipSuccess)
    return hipcheck(ctx, e, "count");
  // 1. The mirrored and initial-condition points (whose terms use the fields alone): outputs by the
  //    packed forward kernel, four points per thread group.
  const int64_t P_rest = L.P_ext - P;
  const int m = c->hp.m;
  qp_status s = QP_OK;
  if (P_rest > 0 && (s = run_fused(ctx, c, kModeFwdPk, params, ext + 3 * P, nullptr, nullptr, P_rest, nullptr,
                                   fo + (size_t)m * P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   fws, gflags, 0, 0)) != QP_OK)
    return s;
  // 2. The collocation points in one pass: forward with input tangents, the seeds of the residual,
  //    energy and symmetry terms formed in the kernel from the point's own fields and its mirror
  //    images' outputs, then the adjoint (their share of the gradient goes to d_params).
  if ((P > 0 || P_rest == 0) &&
      (s = run_fused(ctx, c, kModeTotal, params, ext, nullptr, nullptr, P, &d->phys, fo, fg, nullptr, nullptr, nullptr,
                     c->hp.K > 0 ? d_params : nullptr, nullptr, nullptr, fws, gflags, 0, 0, fo + (size_t)m * P,
                     L.with_mx ? 2 : 1, d->w_sym, d->w_energy)) != QP_OK)
    return s;
  // 3. The four terms, and the seeds of the mirrored and initial-condition points (the kernel also
  //    writes the collocation points' seeds, which step 2 formed itself and nothing reads).
  TotalSeedArgs a{};
  a.out = fo; a.tan = fg; a.points = points; a.ic_xy = ic_xy;
  a.P = P; a.P0 = P0; a.ic_base = L.ic_base; a.m = c->hp.m; a.with_mx = L.with_mx;
  a.phys_kind = kind; a.eps_r = d->phys.eps_r; a.x_if = d->phys.x_interface; a.counts = counts;
  a.w_ic = d->w_ic; a.w_sym = d->w_sym; a.w_energy = d->w_energy; a.ic_a = d->ic_a;
  a.d_out = dout; a.d_tan = dtan;
  a.part = reinterpret_cast<float*>(w + L.part);
  a.terms = loss_terms;
  if ((e = launch_total_seeds(a, st)) != hipSuccess) return hipcheck(ctx, e, "total-loss seeds");
  if (out && P > 0 && (e = hipMemcpyAsync(out, fo, sizeof(float) * c->hp.m * P, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hipcheck(ctx, e, "copy outputs");
  if (tan && P > 0 && (e = hipMemcpyAsync(tan, fg, sizeof(float) * 3 * c->hp.m * P, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hipcheck(ctx, e, "copy tangents");
  if (c->hp.K == 0) return QP_OK;
  // 4. The adjoint of the mirrored and initial-condition points (packed kernel); with collocation
  //    points as well, their gradient goes to a scratch vector and is added (each part reduced over
  //    its workgroups in FP64, rounded once, then summed).
  const bool two = P > 0 && P_rest > 0;
  float* dtmp = reinterpret_cast<float*>(w + L.dtmp);
  if (P_rest > 0 &&
      (s = run_fused(ctx, c, kModeVjpPk, params, ext + 3 * P, nullptr, nullptr, P_rest, nullptr, nullptr, nullptr,
                     dout + (size_t)m * P, nullptr, nullptr, two ? dtmp : d_params, nullptr, nullptr, fws, gflags, 0,
                     0)) != QP_OK)
    return s;
  if (two && (e = launch_add(d_params, dtmp, c->hp.K, st)) != hipSuccess) return hipcheck(ctx, e, "gradient sum");
  return QP_OK;
}

// ---------------------------------------------------------------- plain ---------------------
static PlainProblem plain_problem(const qp_circuit* c, int64_t P) {
  PlainProblem pr{};
  pr.enc.n = c->hp.n;
  pr.enc.kind = c->hp.enc_kind;
  pr.enc.gate = c->hp.enc_gate;
  pr.enc.scale = c->hp.enc_scale;
  pr.enc.nf = c->hp.n_feat;
  for (int q = 0; q < 16; ++q) pr.enc.coord[q] = c->hp.coord[q];
  const char* pb = reinterpret_cast<const char*>(c->dplan_raw);
  const QPlanDev* h = reinterpret_cast<const QPlanDev*>(c->hp.blob.data());
  pr.enc.B = reinterpret_cast<const float*>(pb + h->off_rff_B);
  pr.enc.W = reinterpret_cast<const float*>(pb + h->off_rff_W);
  pr.m = c->hp.m;
  pr.K = c->hp.K;
  pr.n_gates = (int)c->pgates.size();
  for (int i = 0; i < 8; ++i) pr.oq.q[i] = i < c->hp.m ? c->hp.out_qubits[i] : 0;
  pr.gates_dev = c->dpgates;
  pr.gates_host = c->pgates.data();
  pr.P = P;
  return pr;
}

extern "C" size_t qp_plain_workspace_bytes(const qp_circuit* c, int64_t P, int32_t precision) {
  if (!c || P < 0 || (precision != 32 && precision != 64)) return 0;
  return plain_layout(plain_problem(c, P), precision == 64 ? 8 : 4).total;
}

static qp_status plain_checks(qp_ctx* ctx, const qp_circuit* c, int precision, const void* params, const void* points,
                              int64_t P, void* ws, size_t ws_bytes, const char* who) {
  if (!ctx || !c) return fail(ctx, QP_EINVAL, "%s: null context or circuit", who);
  if (precision != 32 && precision != 64) return fail(ctx, QP_EINVAL, "%s: precision must be 32 or 64", who);
  if (P < 0) return fail(ctx, QP_EINVAL, "%s: P < 0", who);
  if (c->hp.enc_kind == QP_ENC_ANGLES) return fail(ctx, QP_EUNSUPPORTED, "%s: the plain path needs a point encoding", who);
  if ((c->hp.K > 0 && !params) || (P > 0 && !points)) return fail(ctx, QP_EINVAL, "%s: null params/points", who);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(ctx, QP_EWORKSPACE, "%s: workspace null or misaligned", who);
  if (ws_bytes < qp_plain_workspace_bytes(c, P, precision)) return fail(ctx, QP_EWORKSPACE, "%s: workspace too small", who);
  return QP_OK;
}

extern "C" qp_status qp_plain_eval(qp_ctx* ctx, const qp_circuit* c, int32_t precision, const void* params,
                                   const void* points, int64_t P, double fd_h, void* out, void* tan, void* ws,
                                   size_t ws_bytes) {
  qp_status s = plain_checks(ctx, c, precision, params, points, P, ws, ws_bytes, "qp_plain_eval");
  if (s != QP_OK) return s;
  if (P > 0 && !out) return fail(ctx, QP_EINVAL, "qp_plain_eval: out is null");
  if (tan && !(fd_h > 0)) return fail(ctx, QP_EINVAL, "qp_plain_eval: fd_h must be > 0");
  hipSetDevice(ctx->device);
  return hipcheck(ctx, plain_eval(plain_problem(c, P), precision, params, points, fd_h, out, tan, ws, ctx->stream),
                  "plain eval");
}

extern "C" qp_status qp_plain_maxwell_fd(qp_ctx* ctx, const qp_circuit* c, int32_t precision, const void* params,
                                         const void* points, int64_t P, const qp_maxwell_desc* ld, double fd_h,
                                         double fd_h_param, int32_t k_begin, int32_t k_end, double* loss,
                                         void* d_params, void* ws, size_t ws_bytes) {
  qp_status s = plain_checks(ctx, c, precision, params, points, P, ws, ws_bytes, "qp_plain_maxwell_fd");
  if (s != QP_OK) return s;
  if (!ld || !loss) return fail(ctx, QP_EINVAL, "qp_plain_maxwell_fd: null loss descriptor or loss");
  if (c->hp.m < 3) return fail(ctx, QP_ESHAPE, "qp_plain_maxwell_fd: needs 3 outputs");
  if (k_begin < 0 || k_end > c->hp.K || k_begin > k_end) return fail(ctx, QP_EINVAL, "qp_plain_maxwell_fd: bad parameter range");
  if (k_end > k_begin && !d_params) return fail(ctx, QP_EINVAL, "qp_plain_maxwell_fd: d_params is null");
  if (!(fd_h > 0) || (k_end > k_begin && !(fd_h_param > 0))) return fail(ctx, QP_EINVAL, "qp_plain_maxwell_fd: steps must be > 0");
  hipSetDevice(ctx->device);
  return hipcheck(ctx, plain_maxwell(plain_problem(c, P), precision, params, points, *ld, 0, fd_h, fd_h_param, k_begin,
                                     k_end, loss, d_params, ws, ctx->stream),
                  "plain maxwell");
}
