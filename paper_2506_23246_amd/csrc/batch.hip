// Uneven batch: many circuits (different qubit counts, depths and point counts) evaluated by
// ONE persistent kernel.  The host splits every circuit into work items of whole point tiles,
// sized so that items cost about the same, and orders them longest-processing-time first.
// Workgroups pull items from an atomic counter (reset by the preceding gate-table kernel, so
// the sequence replays inside a hipGraph without memset nodes).  Each item writes its own M and
// loss partials, so the final fixed-order FP64 reduction per circuit is deterministic no matter
// which workgroup ran which item.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "fused_kernel.hpp"
#include "grads_dev.hpp"
#include "rot_dev.hpp"

namespace qp {

constexpr int kBT = 256;   // threads per workgroup (all batch circuits have n <= 11)
// Two exchange planes: the function holds every qubit count's tile code under one 256-VGPR cap;
// with four planes it spills 292 bytes per lane, whose scratch (38 MB over 2048 waves) overflows
// the L2 and nearly doubles the kernel's HBM traffic, at the same speed as two planes (128 bytes).
constexpr int kBEXS = 2;

__global__ void k_batch_gates(const BatchCirc* __restrict__ circs, const BatchGate* __restrict__ gates, int ngates,
                              int* __restrict__ counter) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) { counter[0] = 0; counter[1] = 0; }   // one work counter per qubit-count class
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

template <int N>
__device__ __forceinline__ void batch_tiles(const BatchCirc& C, const BatchItem& it, float2* buf, float* slots,
                                            float* red, float& lacc) {
  for (int t = it.tile0; t < it.tile0 + it.ntile; ++t)
    fused_tile<N, kBT, kBEXS, kModeMaxwell, true, false, false>(C.a, t, buf, slots, nullptr, red, lacc);
}

// One kernel per class of qubit counts [NLO, NHI]: each class's tile code gets its own register
// allocation (all counts 3..11 in one function exceeded the 256-VGPR cap and spilled 128 bytes a
// lane, whose scratch traffic doubled the kernel's HBM bytes; 3..8 and 9..11 each fit).
template <int NLO, int NHI>
__global__ __launch_bounds__(kBT, 2) void k_batch(const BatchCirc* __restrict__ circs, const BatchItem* __restrict__ items,
                                               int nitems, int* __restrict__ counter, float* __restrict__ mpart,
                                               float* __restrict__ lpart) {
  constexpr int WAVES = kBT / 64;
  constexpr int PLANE = kBT * 8;
  __shared__ float4 planes[kBEXS * PLANE / 2];   // exchange planes (static: one-XOR addressing)
  extern __shared__ float4 smem4[];
  float2* buf = reinterpret_cast<float2*>(planes);
  float* slots = reinterpret_cast<float*>(smem4);
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int id = s_item;
    __syncthreads();
    if (id >= nitems) break;
    const BatchItem it = items[id];
    const BatchCirc& C = circs[it.circ];
    const int F = C.F;
    float* red = slots + WAVES * F * kGS;
    for (int i = tid; i < WAVES * F * kGS; i += kBT) slots[i] = 0.f;
    __syncthreads();
    float lacc = 0.f;
    switch (C.n) {
      case 3: if (NLO <= 3 && 3 <= NHI) batch_tiles<3>(C, it, buf, slots, red, lacc); break;
      case 4: if (NLO <= 4 && 4 <= NHI) batch_tiles<4>(C, it, buf, slots, red, lacc); break;
      case 5: if (NLO <= 5 && 5 <= NHI) batch_tiles<5>(C, it, buf, slots, red, lacc); break;
      case 6: if (NLO <= 6 && 6 <= NHI) batch_tiles<6>(C, it, buf, slots, red, lacc); break;
      case 7: if (NLO <= 7 && 7 <= NHI) batch_tiles<7>(C, it, buf, slots, red, lacc); break;
      case 8: if (NLO <= 8 && 8 <= NHI) batch_tiles<8>(C, it, buf, slots, red, lacc); break;
      case 9: if (NLO <= 9 && 9 <= NHI) batch_tiles<9>(C, it, buf, slots, red, lacc); break;
      case 10: if (NLO <= 10 && 10 <= NHI) batch_tiles<10>(C, it, buf, slots, red, lacc); break;
      case 11: if (NLO <= 11 && 11 <= NHI) batch_tiles<11>(C, it, buf, slots, red, lacc); break;
      default: break;
    }
    __syncthreads();
    float* mp = mpart + C.mpart_off + (long long)it.slot * F * kGS;
    for (int i = tid; i < F * kGS; i += kBT) {
      float s = 0.f;
      for (int w = 0; w < WAVES; ++w) s += slots[w * F * kGS + i];
      mp[i] = s;
    }
    for (int off = 32; off >= 1; off >>= 1) lacc += __shfl_xor(lacc, off);
    if (lane == 0) red[wave * 40] = lacc;
    __syncthreads();
    if (tid == 0) {
      float s = 0.f;
      for (int w = 0; w < WAVES; ++w) s += red[w * 40];
      lpart[C.item_lp0 + it.slot] = s;
    }
    __syncthreads();
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
  const int ncol = C.F * kGS;
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

// Dynamic LDS of k_batch: per-wave gate statistics and readout scratch.
static size_t batch_dyn_lds_bytes(int max_fused) {
  return (size_t)(kBT / 64) * max_fused * kGS * sizeof(float) + (size_t)(kBT / 64) * 40 * sizeof(float);
}

size_t batch_lds_bytes(int max_fused) {   // static exchange planes + dynamic part
  return (size_t)kBEXS * kBT * 8 * sizeof(float2) + batch_dyn_lds_bytes(max_fused);
}

hipError_t batch_prepare(int max_fused) {
  const size_t lds = batch_dyn_lds_bytes(max_fused);
  if (lds <= 64 * 1024) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_batch<3, kBatchSplit>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_batch<kBatchSplit + 1, 11>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_batch(const BatchCirc* circs, int ncirc, const BatchItem* items, int nitems, int nitems_lo,
                        const BatchGate* gates, int ngates, const BatchCol* cols, int ncols, const BatchGate* pars,
                        int npars, int* counter, float* mpart, float* lpart, int grid, int grid_lo, int grid_hi,
                        int max_fused, int count_needed, hipStream_t st, hipStream_t aux, hipEvent_t ev_fork,
                        hipEvent_t ev_join, hipEvent_t ev0, hipEvent_t ev1) {
  hipLaunchKernelGGL(k_batch_gates, dim3(ngates > 0 ? (ngates + 127) / 128 : 1), dim3(128), 0, st,
                     circs, gates, ngates, counter);
  if (count_needed) hipLaunchKernelGGL(k_batch_counts, dim3(ncirc), dim3(256), 0, st, circs);
  if (ev0) hipEventRecord(ev0, st);
  // The items of each class are contiguous (the low class first), each in longest-first order.
  // When both classes have work the two kernels run at once on two streams with their own
  // persistent grids (grid_lo, grid_hi); otherwise the one class runs on `grid`.
  const int nitems_hi = nitems - nitems_lo;
  const size_t dyn = batch_dyn_lds_bytes(max_fused);
  if (grid_lo > 0 && grid_hi > 0 && nitems_lo > 0 && nitems_hi > 0 && aux) {
    hipEventRecord(ev_fork, st);
    hipStreamWaitEvent(aux, ev_fork, 0);
    hipLaunchKernelGGL((k_batch<3, kBatchSplit>), dim3(grid_lo), dim3(kBT), dyn, st, circs, items, nitems_lo, counter,
                       mpart, lpart);
    hipLaunchKernelGGL((k_batch<kBatchSplit + 1, 11>), dim3(grid_hi), dim3(kBT), dyn, aux, circs, items + nitems_lo,
                       nitems_hi, counter + 1, mpart, lpart);
    hipEventRecord(ev_join, aux);
    hipStreamWaitEvent(st, ev_join, 0);
  } else {
    if (grid > 0 && nitems_lo > 0)
      hipLaunchKernelGGL((k_batch<3, kBatchSplit>), dim3(grid), dim3(kBT), dyn, st, circs, items, nitems_lo, counter,
                         mpart, lpart);
    if (grid > 0 && nitems_hi > 0)
      hipLaunchKernelGGL((k_batch<kBatchSplit + 1, 11>), dim3(grid), dim3(kBT), dyn, st, circs, items + nitems_lo,
                         nitems_hi, counter + 1, mpart, lpart);
  }
  if (ev1) hipEventRecord(ev1, st);
  hipLaunchKernelGGL(k_batch_reduce, dim3((ncols + 3) / 4), dim3(256), 0, st, circs, cols, ncols, mpart, lpart);
  if (npars > 0) hipLaunchKernelGGL(k_batch_grads, dim3((npars + 127) / 128), dim3(128), 0, st, circs, pars, npars);
  return hipGetLastError();
}

}  // namespace qp
