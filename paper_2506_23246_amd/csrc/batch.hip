// Uneven batch: many circuits (different qubit counts, depths and point counts) evaluated by
// persistent kernels, one per qubit-count class.  The host splits every circuit into work items
// of whole point tiles, sized so that items cost about the same, and orders them
// longest-processing-time first.  Workgroups pull items from an atomic counter (reset by the
// preceding gate-table kernel, so the sequence replays inside a hipGraph without memset nodes).
// Each item writes its own M and loss partials, so the final fixed-order FP64 reduction per
// circuit is deterministic no matter which workgroup ran which item.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "batch_kernel.hpp"
#include "fused_kernel.hpp"
#include "grads_dev.hpp"
#include "rot_dev.hpp"

namespace qp {

__global__ void k_batch_gates(const BatchCirc* __restrict__ circs, const BatchGate* __restrict__ gates, int ngates,
                              int* __restrict__ counter) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0)   // one work counter per segment
    for (int i = 0; i < kNumSegs; ++i) counter[i] = 0;
  if (g >= ngates) return;
  const BatchGate G = gates[g];
  const BatchCirc& C = circs[G.circ];
  if (G.idx == C.F) {   // identity entry used for absent gates of a round
    float u[8];
    set_identity(u);
    store_gate_entry(const_cast<float*>(C.a.gtab) + G.idx * kGT, u);
    return;
  }
  const QPlanDev* plan = C.a.plan;
  const QFused* fu = reinterpret_cast<const QFused*>(reinterpret_cast<const char*>(plan) + plan->off_fused) + G.idx;
  double u[8];
  set_identity(u);
  for (int c = 0; c < fu->ncomp; ++c) {
    double s, co;
    sincos(0.5 * (double)C.params[fu->param[c]], &s, &co);
    left_mul_rot<double>(fu->kind[c], co, s, u);
  }
  store_gate_entry(const_cast<float*>(C.a.gtab) + G.idx * kGT, u);
}

// Dielectric point counts per circuit (one workgroup per circuit).
__global__ void k_batch_counts(const BatchCirc* __restrict__ circs) {
  const BatchCirc& C = circs[blockIdx.x];
  if (C.a.loss_kind != QP_LOSS_DIEL_SPLIT) return;
  __shared__ int sh[4];
  int c = 0;
  for (long long p = threadIdx.x; p < C.a.P; p += blockDim.x) c += C.a.points[p * 3 + 1] >= C.a.x_if ? 1 : 0;
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int s = sh[0] + sh[1] + sh[2] + sh[3];
    int* cnt = const_cast<int*>(C.a.counts);
    cnt[0] = (int)(C.a.P - s);
    cnt[1] = s;
  }
}

// One wave per (circuit, column): fixed-order FP64 sum over the circuit's items.
__global__ void k_batch_reduce(const BatchCirc* __restrict__ circs, const BatchCol* __restrict__ cols, int ncols,
                               const float* __restrict__ mpart, const float* __restrict__ lpart) {
  const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= ncols) return;
  const BatchCol col = cols[w];
  const BatchCirc& C = circs[col.circ];
  const int ncol = C.F * kGS + C.a.n_mom;   // statistics and moments; col == ncol: the loss
  double s = 0.0;
  if (col.col < ncol) {
    for (int b = lane; b < C.nitems; b += 64) s += (double)mpart[C.mpart_off + (long long)b * ncol + col.col];
  } else {
    for (int b = lane; b < C.nitems; b += 64) s += (double)lpart[C.item_lp0 + b];
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    if (col.col < ncol) C.m64[col.col] = s;
    else *C.loss = s;
  }
}

__global__ void k_batch_grads(const BatchCirc* __restrict__ circs, const BatchGate* __restrict__ pars, int npars) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npars) return;
  const BatchGate g = pars[i];
  const BatchCirc& C = circs[g.circ];
  C.d_params[g.idx] = (float)param_grad_one(C.a.plan, C.params, C.m64, g.idx);
}

size_t batch_lds_bytes(int n, int max_cols) {   // static exchange planes + dynamic part
  const int T = batch_threads(n);
  return (size_t)kBEXS * T * 8 * sizeof(float2) + batch_dyn_lds_bytes(T, max_cols);
}

hipError_t launch_batch_seg(int seg, int grid, size_t dyn, hipStream_t s, const BatchCirc* circs,
                            const BatchItem* items, int nitems, int* counter, float* mpart, float* lpart) {
  switch (seg) {
    case kSegLo:
      hipLaunchKernelGGL((k_batch<3, kBatchSplit, 256, false>), dim3(grid), dim3(256), dyn, s, circs, items, nitems,
                         counter, mpart, lpart);
      break;
    case kSegHi:
      hipLaunchKernelGGL((k_batch<kBatchSplit + 1, 11, 256, false>), dim3(grid), dim3(256), dyn, s, circs, items,
                         nitems, counter, mpart, lpart);
      break;
    case kSegBig:
      hipLaunchKernelGGL((k_batch<kBatchBig, kBatchBig, 512, false>), dim3(grid), dim3(512), dyn, s, circs, items,
                         nitems, counter, mpart, lpart);
      break;
    default: return launch_batch_seg_ph(seg, grid, dyn, s, circs, items, nitems, counter, mpart, lpart);
  }
  return hipGetLastError();
}

hipError_t batch_prepare(int max_cols, int max_cols_big) {
  const int lds = (int)batch_dyn_lds_bytes(256, max_cols), lds_big = (int)batch_dyn_lds_bytes(512, max_cols_big);
  hipError_t e = hipSuccess;
  if (max_cols > 0) {
    e = hipFuncSetAttribute((const void*)k_batch<3, kBatchSplit, 256, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_batch<kBatchSplit + 1, 11, 256, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  }
  if (e == hipSuccess && max_cols_big > 0)
    e = hipFuncSetAttribute((const void*)k_batch<kBatchBig, kBatchBig, 512, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_big);
  if (e == hipSuccess) e = batch_prepare_ph(max_cols, max_cols_big);
  return e;
}

hipError_t launch_batch(const BatchCirc* circs, int ncirc, const BatchItem* items, const int* nitems_seg,
                        const BatchGate* gates, int ngates, const BatchCol* cols, int ncols, const BatchGate* pars,
                        int npars, int* counter, float* mpart, float* lpart, int grid, int grid_lo, int grid_hi,
                        int grid_big, int max_cols, int max_cols_big, int count_needed, hipStream_t st,
                        hipStream_t aux, hipEvent_t ev_fork, hipEvent_t ev_join, hipEvent_t ev0, hipEvent_t ev1) {
  hipError_t e = hipSuccess;
  auto keep = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  hipLaunchKernelGGL(k_batch_gates, dim3(ngates > 0 ? (ngates + 127) / 128 : 1), dim3(128), 0, st,
                     circs, gates, ngates, counter);
  if (count_needed) hipLaunchKernelGGL(k_batch_counts, dim3(ncirc), dim3(256), 0, st, circs);
  if (ev0) keep(hipEventRecord(ev0, st));
  const BatchItem* seg_items[kNumSegs];
  for (int sg = 0, off = 0; sg < kNumSegs; off += nitems_seg[sg], ++sg) seg_items[sg] = items + off;
  const int n_low = nitems_seg[kSegLo] + nitems_seg[kSegLoPh];
  int n_all = 0;
  for (int sg = 0; sg < kNumSegs; ++sg) n_all += nitems_seg[sg];
  const bool two = n_low > 0 && n_all > n_low && grid_lo > 0 && grid_hi > 0 && aux;
  auto seg = [&](int sg, hipStream_t s, int g) -> hipError_t {
    if (nitems_seg[sg] == 0 || g <= 0) return hipSuccess;
    const size_t dyn = sg % 3 == kSegBig ? batch_dyn_lds_bytes(512, max_cols_big) : batch_dyn_lds_bytes(256, max_cols);
    return launch_batch_seg(sg, g, dyn, s, circs, seg_items[sg], nitems_seg[sg], counter + sg, mpart, lpart);
  };
  if (two) {
    // the low segments on st, the others one after the other on aux, at the same time
    keep(hipEventRecord(ev_fork, st));
    keep(hipStreamWaitEvent(aux, ev_fork, 0));
    keep(seg(kSegLo, st, grid_lo));
    keep(seg(kSegLoPh, st, grid_lo));
    keep(seg(kSegHi, aux, grid_hi));
    keep(seg(kSegHiPh, aux, grid_hi));
    keep(seg(kSegBig, aux, grid_big));
    keep(seg(kSegBigPh, aux, grid_big));
    keep(hipEventRecord(ev_join, aux));
    keep(hipStreamWaitEvent(st, ev_join, 0));
  } else {
    for (int sg = 0; sg < kNumSegs; ++sg) keep(seg(sg, st, sg % 3 == kSegBig ? grid_big : grid));
  }
  if (ev1) keep(hipEventRecord(ev1, st));
  hipLaunchKernelGGL(k_batch_reduce, dim3((ncols + 3) / 4), dim3(256), 0, st, circs, cols, ncols, mpart, lpart);
  if (npars > 0) hipLaunchKernelGGL(k_batch_grads, dim3((npars + 127) / 128), dim3(128), 0, st, circs, pars, npars);
  keep(hipGetLastError());
  return e;
}

}  // namespace qp
