// Persistent tile kernel of the uneven batch: one instantiation per qubit-count class and phase
// flag (batch.hip holds the classes without CRZ phase stages, batch_ph.hip those with them, so
// the two sets compile in parallel and neither's register allocation sees the other's code).
#pragma once
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "fused_kernel.hpp"

namespace qp {

// Two exchange planes: the function holds every qubit count's tile code of its class under one
// 256-VGPR cap; with four planes the all-counts kernel spilled 292 bytes per lane, whose scratch
// (38 MB over 2048 waves) overflowed the L2 and nearly doubled the kernel's HBM traffic.
constexpr int kBEXS = 2;

// Dynamic LDS of a T-thread k_batch: per-wave gate statistics, phase moments, readout scratch.
inline size_t batch_dyn_lds_bytes(int T, int max_cols) {
  return (size_t)(T / 64) * max_cols * sizeof(float) + (size_t)(T / 64) * 40 * sizeof(float);
}

// The tiles of one work item.  PH: the class kernel for circuits with CRZ phase stages (the tile
// code applies them and accumulates their moments in mslots); the other kernels compile it out.
template <int N, int NLO, int NHI, int T, bool PH>
__device__ __forceinline__ void batch_case(const BatchCirc& C, const BatchItem& it, float2* buf, float* slots,
                                           float* mslots, float* red, float& lacc) {
  if constexpr (NLO <= N && N <= NHI) {
    for (int t = it.tile0; t < it.tile0 + it.ntile; ++t)
      fused_tile<N, T, kBEXS, kModeMaxwell, true, false, PH>(C.a, t, buf, slots, mslots, red, lacc);
  }
}

// One kernel per class of qubit counts [NLO, NHI] on T-thread workgroups: each class's tile code
// gets its own register allocation (all counts 3..11 in one function exceeded the 256-VGPR cap
// and spilled 128 bytes a lane, whose scratch traffic doubled the kernel's HBM bytes; 3..8 and
// 9..11 each fit, and 12 qubits need 512 threads: a tile is one point on 512 threads).
template <int NLO, int NHI, int T, bool PH>
__global__ __launch_bounds__(T, 2) void k_batch(const BatchCirc* __restrict__ circs, const BatchItem* __restrict__ items,
                                             int nitems, int* __restrict__ counter, float* __restrict__ mpart,
                                             float* __restrict__ lpart) {
  constexpr int WAVES = T / 64;
  constexpr int PLANE = T * 8;
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
    const int F = C.F, NM = C.a.n_mom;
    float* mslots = slots + WAVES * F * kGS;   // [WAVES][F][kGS] statistics, [WAVES][NM] moments
    float* red = mslots + WAVES * NM;
    for (int i = tid; i < WAVES * (F * kGS + NM); i += T) slots[i] = 0.f;
    __syncthreads();
    float lacc = 0.f;
    switch (C.n) {
      case 3: batch_case<3, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 4: batch_case<4, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 5: batch_case<5, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 6: batch_case<6, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 7: batch_case<7, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 8: batch_case<8, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 9: batch_case<9, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 10: batch_case<10, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 11: batch_case<11, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      case 12: batch_case<12, NLO, NHI, T, PH>(C, it, buf, slots, mslots, red, lacc); break;
      default: break;
    }
    __syncthreads();
    const int ncol = F * kGS + NM;
    float* mp = mpart + C.mpart_off + (long long)it.slot * ncol;
    for (int i = tid; i < F * kGS; i += T) {
      float s = 0.f;
      for (int w = 0; w < WAVES; ++w) s += slots[w * F * kGS + i];
      mp[i] = s;
    }
    for (int i = tid; i < NM; i += T) {
      float s = 0.f;
      for (int w = 0; w < WAVES; ++w) s += mslots[w * NM + i];
      mp[F * kGS + i] = s;
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

// Launches the class kernel of segment `seg` (see BatchSeg) on `grid` workgroups.
hipError_t launch_batch_seg(int seg, int grid, size_t dyn, hipStream_t s, const BatchCirc* circs,
                            const BatchItem* items, int nitems, int* counter, float* mpart, float* lpart);
hipError_t launch_batch_seg_ph(int seg, int grid, size_t dyn, hipStream_t s, const BatchCirc* circs,
                               const BatchItem* items, int nitems, int* counter, float* mpart, float* lpart);
hipError_t batch_prepare_ph(int max_cols, int max_cols_big);

}  // namespace qp
