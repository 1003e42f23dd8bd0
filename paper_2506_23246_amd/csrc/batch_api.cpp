// C ABI of the uneven batch: compile (plans, LPT work list), run, and hipGraph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>

#include "../../include/qpinn.h"
#include "batch.hpp"
#include "capi_internal.hpp"

using namespace qp;

// Grids of the low qubit-count class and of the high class when they run at once (the 12-qubit
// class runs after the high class on one 512-thread workgroup per CU).  The low class gets its
// share of `grid` by estimated work, times `bias`; the high class gets the rest of `grid` (split)
// or all of it (stacked: the low class's workgroups come on top, and the slots they leave when
// their class is done go to the high class's waves that share the CU).
// Default: stacked, the low class's share by estimated work x 1.25 (the best of the tuner's
// candidates on the 32-circuit, 4..10-qubit batch, 2.4 % faster than the even split).
constexpr double kStackedBias = 1.25;

static void class_grids(const qp_batch* b, int grid, double bias, bool stacked, int* g_lo, int* g_hi) {
  const double share = b->work_lo + b->work_rest > 0.0 ? b->work_lo / (b->work_lo + b->work_rest) : 0.0;
  int lo = (int)(grid * share * bias + 0.5);
  lo = lo < 1 ? 1 : (lo > grid - 1 ? grid - 1 : lo);
  *g_lo = lo;
  *g_hi = stacked ? grid : std::max(1, grid - lo);
}

extern "C" qp_status qp_batch_compile(qp_ctx* ctx, int32_t count, const qp_circuit_desc* descs, const int64_t* P,
                                      qp_batch** out) {
  if (!ctx || !descs || !P || !out || count < 1) return fail(ctx, QP_EINVAL, "qp_batch_compile: bad arguments");
  *out = nullptr;
  auto* b = new qp_batch();
  b->ctx = ctx;
  auto cleanup = [&](qp_status s) {
    for (auto* c : b->circs) qp_circuit_destroy(c);
    delete b;
    return s;
  };
  for (int i = 0; i < count; ++i) {
    if (P[i] < 0) return cleanup(fail(ctx, QP_EINVAL, "qp_batch_compile: P[%d] < 0", i));
    if (P[i] > (int64_t)INT32_MAX)   // point and tile indices are 32-bit in the kernels
      return cleanup(fail(ctx, QP_EUNSUPPORTED, "qp_batch_compile: P[%d] exceeds 2^31 - 1", i));
    qp_circuit* c = nullptr;
    qp_status s = qp_circuit_compile(ctx, &descs[i], &c);
    if (s != QP_OK) return cleanup(s);
    b->circs.push_back(c);
    if (!c->hp.fused_ok) return cleanup(fail(ctx, QP_EUNSUPPORTED, "qp_batch_compile: circuit %d: %s", i, c->hp.fused_reason.c_str()));
    if (c->hp.m < 3) return cleanup(fail(ctx, QP_ESHAPE, "qp_batch_compile: circuit %d needs 3 outputs", i));
    if (c->hp.enc_kind == QP_ENC_ANGLES)   // qp_batch_io carries no per-point angles
      return cleanup(fail(ctx, QP_EUNSUPPORTED, "qp_batch_compile: circuit %d: angle-given encoding not batched", i));
    b->P.push_back(P[i]);
    int& mc = c->hp.n >= kBatchBig ? b->max_cols_big : b->max_cols;
    mc = std::max(mc, (int)c->hp.fused.size() * kGS + n_moments(c));
    if (!c->hp.phases.empty()) b->table_circs.push_back(i);
    if (c->hp.enc_kind == QP_ENC_RFF) b->rff_circs.push_back(i);
  }
  if ((b->max_cols > 0 && batch_lds_bytes(3, b->max_cols) > 160 * 1024) ||
      (b->max_cols_big > 0 && batch_lds_bytes(kBatchBig, b->max_cols_big) > 160 * 1024))
    return cleanup(fail(ctx, QP_EUNSUPPORTED, "qp_batch_compile: the gate statistics of a member exceed the LDS"));
  // work items: whole tiles, item cost ~ total / (grid * 6), longest first
  b->grid = ctx->cu_count * 2;
  std::vector<double> tile_cost(count);
  std::vector<int64_t> tiles(count);
  double total = 0.0;
  for (int i = 0; i < count; ++i) {
    const auto& hp = b->circs[i]->hp;
    const int ppw = batch_points_per_tile(hp.n);
    tiles[i] = (P[i] + ppw - 1) / ppw;
    tile_cost[i] = (double)hp.fused.size() + 2.0 * (double)hp.rounds.size();
    total += tile_cost[i] * (double)tiles[i];
  }
  const double target = std::max(1.0, total / (double)(b->grid * 6));
  std::vector<int> nitems(count, 0);
  for (int i = 0; i < count; ++i) {
    const int64_t tpi = std::max<int64_t>(1, (int64_t)(target / tile_cost[i]));
    int slot = 0;
    for (int64_t t0 = 0; t0 < tiles[i]; t0 += tpi, ++slot)
      b->items.push_back(BatchItem{i, (int)t0, (int)std::min<int64_t>(tpi, tiles[i] - t0), slot});
    nitems[i] = slot;
  }
  // the segments in order, each longest first
  auto seg = [&](const BatchItem& x) {
    const qp_circuit* c = b->circs[x.circ];
    return batch_segment(c->hp.n, !c->hp.phases.empty());
  };
  std::stable_sort(b->items.begin(), b->items.end(), [&](const BatchItem& x, const BatchItem& y) {
    if (seg(x) != seg(y)) return seg(x) < seg(y);
    return tile_cost[x.circ] * x.ntile > tile_cost[y.circ] * y.ntile;
  });
  b->work_lo = b->work_rest = 0.0;
  for (const auto& it : b->items) {
    const int k = seg(it);
    b->nitems_seg[k] += 1;
    (k == kSegLo || k == kSegLoPh ? b->work_lo : b->work_rest) += tile_cost[it.circ] * it.ntile;
  }
  class_grids(b, b->grid, kStackedBias, true, &b->grid_lo, &b->grid_hi);
  b->grid_big = ctx->cu_count;   // one 512-thread workgroup per CU
  for (int i = 0; i < count; ++i) {
    const int F = (int)b->circs[i]->hp.fused.size();
    const int ncol = F * kGS + n_moments(b->circs[i]);
    for (int c = 0; c <= ncol; ++c) b->cols.push_back(BatchCol{i, c});
    if (b->circs[i]->hp.phases.empty())   // CRZ circuits: the fused path's table kernel (run time)
      for (int f = 0; f <= F; ++f) b->gates.push_back(BatchGate{i, f});   // f == F: identity entry
    for (int k = 0; k < b->circs[i]->hp.K; ++k) b->pars.push_back(BatchGate{i, k});
  }
  // workspace layout
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  BatchLayout& L = b->layout;
  size_t off = 0;
  L.counter = off; off = al(off + kNumSegs * sizeof(int));   // one work counter per segment
  long long mp = 0;
  L.gtab_c.resize(count); L.counts_c.resize(count); L.m64_c.resize(count); L.mpart_c.resize(count);
  L.angles_c.assign(count, 0); L.jac_c.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    const qp_circuit* c = b->circs[i];
    const int F = (int)c->hp.fused.size(), NM = n_moments(c);
    // gate entries + identity, then the phase coefficients (as the fused path's table)
    L.gtab_c[i] = off; off = al(off + sizeof(float) * kGT * (F + 1) + sizeof(uint32_t) * NM);
    L.counts_c[i] = off; off = al(off + 2 * sizeof(int));
    L.m64_c[i] = off; off = al(off + sizeof(double) * std::max(F * kGS + NM, 1));
    if (c->hp.enc_kind == QP_ENC_RFF) {
      L.angles_c[i] = off; off = al(off + sizeof(float) * (size_t)P[i] * c->hp.n);
      L.jac_c[i] = off; off = al(off + sizeof(float) * (size_t)P[i] * c->hp.n * 3);
    }
    L.mpart_c[i] = mp;
    mp += (long long)nitems[i] * (F * kGS + NM);
  }
  L.mpart = off; off = al(off + sizeof(float) * (size_t)std::max<long long>(mp, 1));
  L.lpart = off; off = al(off + sizeof(float) * (size_t)std::max<size_t>(b->items.size(), 1));
  L.total = off;
  // circuit table skeleton (io pointers filled at run time)
  hipSetDevice(ctx->device);
  if (hipHostMalloc((void**)&b->hcirc, sizeof(BatchCirc) * count, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(ctx, QP_EDEVICE, "qp_batch_compile: pinned staging allocation failed"));
  int lp0 = 0;
  for (int i = 0; i < count; ++i) {
    BatchCirc& C = b->hcirc[i];
    std::memset(&C, 0, sizeof(C));
    const auto& hp = b->circs[i]->hp;
    C.n = hp.n;
    C.F = (int)hp.fused.size();
    C.K = hp.K;
    C.nitems = nitems[i];
    C.item_lp0 = lp0;
    C.mpart_off = L.mpart_c[i];
    lp0 += nitems[i];
  }
  // lpart is indexed by (circuit item offset + slot)
  // static device data
  const size_t s_items = al(sizeof(BatchItem) * b->items.size());
  const size_t s_cols = al(sizeof(BatchCol) * b->cols.size());
  const size_t s_gates = al(sizeof(BatchGate) * std::max<size_t>(1, b->gates.size()));
  const size_t s_pars = al(sizeof(BatchGate) * std::max<size_t>(1, b->pars.size()));
  const size_t s_circ = al(sizeof(BatchCirc) * count);
  if (hipMalloc(&b->dstatic, s_items + s_cols + s_gates + s_pars + s_circ) != hipSuccess)
    return cleanup(fail(ctx, QP_EDEVICE, "qp_batch_compile: device allocation failed"));
  char* d = static_cast<char*>(b->dstatic);
  b->ditems = reinterpret_cast<BatchItem*>(d);
  b->dcols = reinterpret_cast<BatchCol*>(d + s_items);
  b->dgates = reinterpret_cast<BatchGate*>(d + s_items + s_cols);
  b->dpars = reinterpret_cast<BatchGate*>(d + s_items + s_cols + s_gates);
  b->dcirc = reinterpret_cast<BatchCirc*>(d + s_items + s_cols + s_gates + s_pars);
  hipError_t e = hipMemcpy(b->ditems, b->items.data(), sizeof(BatchItem) * b->items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->dcols, b->cols.data(), sizeof(BatchCol) * b->cols.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->gates.empty()) e = hipMemcpy(b->dgates, b->gates.data(), sizeof(BatchGate) * b->gates.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->pars.empty()) e = hipMemcpy(b->dpars, b->pars.data(), sizeof(BatchGate) * b->pars.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = batch_prepare(b->max_cols, b->max_cols_big);
  // the second stream keeps the default priority (no other priority is used anywhere)
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    hipFree(b->dstatic);
    hipHostFree(b->hcirc);
    if (b->ev_fork) hipEventDestroy(b->ev_fork);
    if (b->ev_join) hipEventDestroy(b->ev_join);
    if (b->aux) hipStreamDestroy(b->aux);
    return cleanup(fail(ctx, QP_EDEVICE, "qp_batch_compile: upload failed: %s", hipGetErrorString(e)));
  }
  *out = b;
  return QP_OK;
}

extern "C" void qp_batch_destroy(qp_batch* b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->ev_fork) hipEventDestroy(b->ev_fork);
  if (b->ev_join) hipEventDestroy(b->ev_join);
  if (b->aux) hipStreamDestroy(b->aux);
  if (b->dstatic) hipFree(b->dstatic);
  if (b->hcirc) hipHostFree(b->hcirc);
  for (auto* c : b->circs) qp_circuit_destroy(c);
  delete b;
}

extern "C" size_t qp_batch_workspace_bytes(const qp_batch* b) { return b ? b->layout.total : 0; }

extern "C" int64_t qp_batch_info(const qp_batch* b, int32_t what) {
  if (!b) return -1;
  switch (what) {
    case 0: return (int64_t)b->circs.size();
    case 1: return (int64_t)b->items.size();
    case 2: return b->grid;
    case 3: return b->gexec ? 1 : 0;
    case 4: return b->nitems_seg[kSegLo] + b->nitems_seg[kSegLoPh];
    case 5: return b->grid_lo;
    case 6: return b->grid_hi;
    case 7: return b->nitems_seg[kSegBig] + b->nitems_seg[kSegBigPh];
    case 8: return b->nitems_seg[kSegLoPh] + b->nitems_seg[kSegHiPh] + b->nitems_seg[kSegBigPh];
    default: return -1;
  }
}

static uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

// Validates io and (re)uploads the circuit table when pointers or the loss changed.
static qp_status batch_bind(qp_ctx* ctx, qp_batch* b, const qp_batch_io* io, const qp_maxwell_desc* ld, void* ws,
                            size_t ws_bytes, uint32_t flags, uint64_t* key_out) {
  if (!ctx || !b || !io || !ld) return fail(ctx, QP_EINVAL, "qp_batch_run: null argument");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return fail(ctx, QP_EWORKSPACE, "qp_batch_run: workspace null or misaligned");
  if (ws_bytes < b->layout.total) return fail(ctx, QP_EWORKSPACE, "qp_batch_run: workspace %zu < %zu", ws_bytes, b->layout.total);
  if (ld->kind < QP_LOSS_VACUUM || ld->kind > QP_LOSS_DIEL_INTUITIVE) return fail(ctx, QP_EINVAL, "qp_batch_run: bad loss kind");
  const int count = (int)b->circs.size();
  uint64_t key = mix(0, reinterpret_cast<uintptr_t>(ws));
  key = mix(key, (uint64_t)ld->kind);
  uint32_t fe, fx;
  std::memcpy(&fe, &ld->eps_r, 4);
  std::memcpy(&fx, &ld->x_interface, 4);
  key = mix(mix(key, fe), fx);
  key = mix(key, flags & QP_FLAG_LOSS_SUM);
  for (int i = 0; i < count; ++i) {
    const qp_batch_io& o = io[i];
    if ((b->circs[i]->hp.K > 0 && (!o.params || !o.d_params)) || (b->P[i] > 0 && !o.points) || !o.loss)
      return fail(ctx, QP_EINVAL, "qp_batch_run: circuit %d has a null pointer", i);
    for (const void* p : {(const void*)o.params, (const void*)o.points, (const void*)o.out, (const void*)o.tan,
                          (const void*)o.loss, (const void*)o.d_params})
      key = mix(key, reinterpret_cast<uintptr_t>(p));
  }
  *key_out = key;
  if (key == b->io_key) return QP_OK;
  char* w = static_cast<char*>(ws);
  const BatchLayout& L = b->layout;
  for (int i = 0; i < count; ++i) {
    BatchCirc& C = b->hcirc[i];
    const qp_circuit* c = b->circs[i];
    const qp_batch_io& o = io[i];
    FusedArgs& a = C.a;
    a.plan = c->dplan;
    a.gtab = reinterpret_cast<float*>(w + L.gtab_c[i]);
    a.points = o.points;
    const bool rff = c->hp.enc_kind == QP_ENC_RFF;
    a.angles = rff ? reinterpret_cast<const float*>(w + L.angles_c[i]) : nullptr;
    a.jac = rff ? reinterpret_cast<const float*>(w + L.jac_c[i]) : nullptr;
    a.P = b->P[i];
    a.ntiles = (int)((b->P[i] + batch_points_per_tile(c->hp.n) - 1) / batch_points_per_tile(c->hp.n));
    a.n_fused = C.F;
    a.out = o.out;
    a.tan = o.tan;
    a.d_out = nullptr;
    a.d_tan = nullptr;
    a.loss_kind = ld->kind;
    a.loss_sum = (flags & QP_FLAG_LOSS_SUM) ? 1 : 0;
    a.eps_r = ld->eps_r;
    a.x_if = ld->x_interface;
    a.counts = reinterpret_cast<int*>(w + L.counts_c[i]);
    a.mpart = nullptr;
    a.lpart = nullptr;
    a.d_angles = nullptr;
    a.d_jac = nullptr;
    a.n_mom = n_moments(c);
    C.params = o.params;
    C.loss = o.loss;
    C.d_params = o.d_params;
    C.m64 = reinterpret_cast<double*>(w + L.m64_c[i]);
  }
  hipSetDevice(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);   // no replay may still read the old table
  if (e == hipSuccess) e = hipMemcpy(b->dcirc, b->hcirc, sizeof(BatchCirc) * count, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hipcheck(ctx, e, "qp_batch_run: circuit table upload");
  b->io_key = key;
  return QP_OK;
}

static hipError_t batch_launch(qp_ctx* ctx, qp_batch* b, const qp_maxwell_desc* ld, void* ws, int grid, int g_lo,
                               int g_hi) {
  char* w = static_cast<char*>(ws);
  const BatchLayout& L = b->layout;
  // Circuits with CRZ phase stages take the fused path's gate and phase table kernels, RFF
  // circuits the fused path's angle kernel; both write into the batch workspace before the
  // batch kernels read it.
  for (int i : b->table_circs) {
    const qp_circuit* c = b->circs[i];
    hipError_t e = launch_gate_table(c->dplan, (int)c->hp.fused.size(), n_moments(c), b->hcirc[i].params,
                                     reinterpret_cast<float*>(w + L.gtab_c[i]), 0, ctx->stream);
    if (e != hipSuccess) return e;
  }
  for (int i : b->rff_circs) {
    const FusedArgs& a = b->hcirc[i].a;
    hipError_t e = launch_rff(b->circs[i]->dplan, a.points, a.P, const_cast<float*>(a.angles),
                              const_cast<float*>(a.jac), ctx->stream);
    if (e != hipSuccess) return e;
  }
  return launch_batch(b->dcirc, (int)b->circs.size(), b->ditems, b->nitems_seg, b->dgates, (int)b->gates.size(), b->dcols, (int)b->cols.size(), b->dpars, (int)b->pars.size(),
                      reinterpret_cast<int*>(w + L.counter), reinterpret_cast<float*>(w + L.mpart),
                      reinterpret_cast<float*>(w + L.lpart), grid, g_lo, g_hi, b->grid_big, b->max_cols, b->max_cols_big,
                      ld->kind == QP_LOSS_DIEL_SPLIT ? 1 : 0, ctx->stream, b->aux, b->ev_fork, b->ev_join,
                      ctx->timing ? ctx->ev0 : nullptr, ctx->timing ? ctx->ev1 : nullptr);
}

extern "C" qp_status qp_batch_run(qp_ctx* ctx, qp_batch* b, const qp_batch_io* io, const qp_maxwell_desc* ld, void* ws,
                                  size_t ws_bytes, uint32_t flags) {
  uint64_t key = 0;
  qp_status s = batch_bind(ctx, b, io, ld, ws, ws_bytes, flags, &key);
  if (s != QP_OK) return s;
  hipSetDevice(ctx->device);
  if (flags & QP_FLAG_TUNE) {   // time persistent grid sizes and class grids once
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    struct Shape { int grid, lo, hi; };
    std::vector<Shape> shapes;
    const int n_low = b->nitems_seg[kSegLo] + b->nitems_seg[kSegLoPh];
    const bool two = n_low > 0 && n_low < (int)b->items.size();
    for (int mult : {1, 2, 3, 4}) {
      const int g = ctx->cu_count * mult;
      if (!two) { shapes.push_back({g, b->grid_lo, b->grid_hi}); continue; }
      if (mult > 3) continue;
      for (bool stacked : {false, true})
        for (double bias : {0.75, 1.0, 1.25, 1.5, 2.0}) {
          if (!stacked && bias > 1.25) continue;
          Shape sh{b->grid, 0, 0};
          class_grids(b, g, bias, stacked, &sh.lo, &sh.hi);
          shapes.push_back(sh);
        }
    }
    double best = 1e30;
    Shape pick{b->grid, b->grid_lo, b->grid_hi};
    for (const Shape& sh : shapes) {
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        hipEventRecord(e0, ctx->stream);
        batch_launch(ctx, b, ld, ws, sh.grid, sh.lo, sh.hi);
        hipEventRecord(e1, ctx->stream);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_min = std::min(ms_min, ms);
      }
      if (ms_min < best) { best = ms_min; pick = sh; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if ((pick.grid != b->grid || pick.lo != b->grid_lo || pick.hi != b->grid_hi) && b->gexec) {
      hipGraphExecDestroy(b->gexec);   // the captured graph used the old shape
      hipGraphDestroy(b->graph);
      b->gexec = nullptr;
      b->graph = nullptr;
    }
    b->grid = pick.grid;
    b->grid_lo = pick.lo;
    b->grid_hi = pick.hi;
  }
  return hipcheck(ctx, batch_launch(ctx, b, ld, ws, b->grid, b->grid_lo, b->grid_hi), "qp_batch_run");
}

extern "C" qp_status qp_batch_graph_launch(qp_ctx* ctx, qp_batch* b, const qp_batch_io* io, const qp_maxwell_desc* ld,
                                           void* ws, size_t ws_bytes, uint32_t flags) {
  uint64_t key = 0;
  qp_status s = batch_bind(ctx, b, io, ld, ws, ws_bytes, flags, &key);
  if (s != QP_OK) return s;
  if (!ctx->stream) return fail(ctx, QP_EINVAL, "qp_batch_graph_launch: graph capture needs a non-null stream");
  hipSetDevice(ctx->device);
  const uint64_t gkey = mix(mix(mix(key, (uint64_t)b->grid), (uint64_t)b->grid_lo), (uint64_t)b->grid_hi);
  if (!b->gexec || b->graph_key != gkey) {
    if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hipcheck(ctx, e, "hipStreamBeginCapture");
    hipError_t le = batch_launch(ctx, b, ld, ws, b->grid, b->grid_lo, b->grid_hi);
    e = hipStreamEndCapture(ctx->stream, &b->graph);
    if (le != hipSuccess) return hipcheck(ctx, le, "batch capture");
    if (e != hipSuccess) return hipcheck(ctx, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hipcheck(ctx, e, "hipGraphInstantiate");
    b->graph_key = gkey;
  }
  return hipcheck(ctx, hipGraphLaunch(b->gexec, ctx->stream), "hipGraphLaunch");
}
