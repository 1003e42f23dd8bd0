// Templates of the fused register/LDS kernel (included by the per-qubit-count units).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qp_internal.hpp"
#include "fused.hpp"

namespace qp {

// Uniform, read-only kernel data (plan, gate table) is read through the constant address space,
// so the compiler emits scalar loads (SGPRs) instead of per-lane vector loads that stall a wave.
#define QP_CONST __attribute__((address_space(4)))
template <typename T> using CP = const QP_CONST T*;
template <typename T> __device__ __forceinline__ CP<T> to_const(const T* p) { return (CP<T>)(p); }

__device__ __forceinline__ uint32_t parity(uint32_t x) { return __popc(x) & 1u; }

__device__ __forceinline__ uint32_t swz(uint32_t idx) { return lds_swizzle(idx); }

template <int N, typename TP>
__device__ __forceinline__ uint32_t deposit_thread(uint32_t u, TP tpos) {
  uint32_t j = 0;
#pragma unroll
  for (int k = 3; k < N; ++k) j |= ((u >> (k - 3)) & 1u) << tpos[k];
  return j;
}

__device__ __forceinline__ uint32_t reg_off(int r, uint32_t p0, uint32_t p1, uint32_t p2) {
  return ((uint32_t)(r & 1) << p0) | ((uint32_t)((r >> 1) & 1) << p1) |
         ((uint32_t)((r >> 2) & 1) << p2);
}

// ---- single-qubit gate on register bit B for statevectors [S0, S0+NS) ----------------------
// u: u00r,u00i,u01r,u01i,u10r,u10i,u11r,u11i.  Each lane applies the gate to its own amplitude
// pairs on the matrix cores: v_mfma_f32_4x4x1f32 treats the wave as 16 blocks of 4 lanes,
// C[m][n] += A[m] B[n] with A[m] from lane 4b + m, B[n] from lane 4b + n and C[m][n] in register m
// of lane 4b + n.  With lane 4b + m holding row m of the gate's real 4x4 form M (acting on
// (re x, im x, re y, im y)) as A, and every lane its own pair component k as B, four such steps
// (k = 0..3) leave M (x, y) of each lane's pair in its four C registers.  The 2x2 products thus
// leave the vector ALU, which keeps the gate statistics, exchanges and readout.  Called in
// wave-uniform control flow only: a lane's result depends on the A operands of the other three
// lanes of its block, so all 64 lanes must be active.
template <int B, int S0, int NS>
__device__ __forceinline__ void apply_gate(float (&sr)[8][8], float (&si)[8][8], const float* u) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const uint32_t q = threadIdx.x & 3u;   // row m of M held by this lane
  const bool lo = q < 2, odd = q & 1u;
  // M rows: (u00r, -u00i, u01r, -u01i), (u00i, u00r, u01i, u01r), (u10r, -u10i, u11r, -u11i),
  // (u10i, u10r, u11i, u11r); column k of row q.  (u points at pinned coefficients: selects
  // between the elements of a plain local array would become a per-lane indexed scratch load.)
  const float e0 = lo ? u[0] : u[4], e1 = lo ? u[1] : u[5], e2 = lo ? u[2] : u[6], e3 = lo ? u[3] : u[7];
  const float k0 = odd ? e1 : e0;
  const float k1 = odd ? e0 : -e1;
  const float k2 = odd ? e3 : e2;
  const float k3 = odd ? e2 : -e3;
#pragma unroll
  for (int s = S0; s < S0 + NS; ++s) {
    // the four pairs' chains interleaved step by step (independent MFMAs between dependent ones)
    f32x4 c[4];
    int rr[4], r1s[4];
    int np = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r & (1 << B)) continue;
      rr[np] = r; r1s[np] = r | (1 << B); ++np;
    }
    // Raised wave priority while this wave issues its matrix-core chains: the SIMD's other wave
    // (statistics, exchanges) fills the issue slots between them instead of delaying the next
    // link of a chain (12-qubit step 322 -> 298 ms).
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(k0, sr[s][rr[i]], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(k1, si[s][rr[i]], c[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(k2, sr[s][r1s[i]], c[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(k3, si[s][r1s[i]], c[i], 0, 0, 0);
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sr[s][rr[i]] = c[i][0]; si[s][rr[i]] = c[i][1]; sr[s][r1s[i]] = c[i][2]; si[s][r1s[i]] = c[i][3];
    }
  }
}

// Gate statistic of one statevector pair (lambda-family 4 + C, psi-family C), both taken
// before the gate, for the register pairs on bit B:
//   S_x += Im(conj(x0) y1) + Im(conj(x1) y0)
//   S_y += Re(conj(x1) y0) - Re(conj(x0) y1)
//   S_z += Im(conj(x0) y0) - Im(conj(x1) y1)
template <int B, int C>
__device__ __forceinline__ void accum_s1(const float (&sr)[8][8], const float (&si)[8][8], float* m) {
  // two partial sums per component (alternate register pairs): shorter dependent FMA chains
  float a[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  int np = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (r & (1 << B)) continue;
    const int r1 = r | (1 << B);
    float* mm = a[np & 1];
    ++np;
    const float x0r = sr[4 + C][r], x0i = si[4 + C][r], x1r = sr[4 + C][r1], x1i = si[4 + C][r1];
    const float y0r = sr[C][r], y0i = si[C][r], y1r = sr[C][r1], y1i = si[C][r1];
    mm[0] = fmaf(x0r, y1i, mm[0]); mm[0] = fmaf(-x0i, y1r, mm[0]);
    mm[0] = fmaf(x1r, y0i, mm[0]); mm[0] = fmaf(-x1i, y0r, mm[0]);
    mm[1] = fmaf(x1r, y0r, mm[1]); mm[1] = fmaf(x1i, y0i, mm[1]);
    mm[1] = fmaf(-x0r, y1r, mm[1]); mm[1] = fmaf(-x0i, y1i, mm[1]);
    mm[2] = fmaf(x0r, y0i, mm[2]); mm[2] = fmaf(-x0i, y0r, mm[2]);
    mm[2] = fmaf(-x1r, y1i, mm[2]); mm[2] = fmaf(x1i, y1r, mm[2]);
  }
  m[0] += a[0][0] + a[1][0];
  m[1] += a[0][1] + a[1][1];
  m[2] += a[0][2] + a[1][2];
}

template <int B>
__device__ __forceinline__ void accum_s(const float (&sr)[8][8], const float (&si)[8][8], float* q) {
  // Pauli components of the gate's adjoint product for the pairs on register bit B, with
  // x = lambda-family (statevectors 4..7) and y = psi-family (0..3), both before the gate:
  //   S_x += Im(conj(x0) y1) + Im(conj(x1) y0)
  //   S_y += Re(conj(x1) y0) - Re(conj(x0) y1)
  //   S_z += Im(conj(x0) y0) - Im(conj(x1) y1)
  // Two accumulators per component (even/odd statevector pair) shorten the FMA chains.
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    float* m = q + 3 * (s & 1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r & (1 << B)) continue;
      const int r1 = r | (1 << B);
      const float x0r = sr[4 + s][r], x0i = si[4 + s][r], x1r = sr[4 + s][r1], x1i = si[4 + s][r1];
      const float y0r = sr[s][r], y0i = si[s][r], y1r = sr[s][r1], y1i = si[s][r1];
      m[0] = fmaf(x0r, y1i, m[0]); m[0] = fmaf(-x0i, y1r, m[0]);
      m[0] = fmaf(x1r, y0i, m[0]); m[0] = fmaf(-x1i, y0r, m[0]);
      m[1] = fmaf(x1r, y0r, m[1]); m[1] = fmaf(x1i, y0i, m[1]);
      m[1] = fmaf(-x0r, y1r, m[1]); m[1] = fmaf(-x0i, y1i, m[1]);
      m[2] = fmaf(x0r, y0i, m[2]); m[2] = fmaf(-x0i, y0r, m[2]);
      m[2] = fmaf(-x1r, y1i, m[2]); m[2] = fmaf(x1i, y1r, m[2]);
    }
  }
}

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {   // DPP lane permutation (row-local)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Reduce 8 floats over the 64 lanes of a wave; afterwards lane 8*e holds the sum of entry e.
// Reduce-scatter of four per-lane values over the wave: permlane32_swap pairs lanes l and l+32
// (entries split 2/2), permlane16_swap pairs rows 0/1 and 2/3 (1/1), then DPP row_ror:8,
// quad_perm xor 1, xor 2 and row_half_mirror sum the sixteen lanes of each row.  Lanes of row e
// end with entry e.  No LDS traffic.
__device__ __forceinline__ float wave_reduce_scatter4(const float* v) {
  float a[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_int(v[i]), __float_as_int(v[2 + i]), false, false);
    a[i] = __int_as_float(sw[0]) + __int_as_float(sw[1]);
  }
  const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_int(a[0]), __float_as_int(a[1]), false, false);
  float c = __int_as_float(sw[0]) + __int_as_float(sw[1]);
  c += dppf<0x128>(c);   // row_ror:8  (lane l <- l ^ 8 within a row)
  c += dppf<0xB1>(c);    // quad_perm [1,0,3,2]: xor 1
  c += dppf<0x4E>(c);    // quad_perm [2,3,0,1]: xor 2
  c += dppf<0x141>(c);   // row_half_mirror: lane l <- 7 - l within eight lanes
  return c;
}

// ---- register exchange through LDS ----------------------------------------------------------
// An exchange moves the statevectors from the writer round's mapping to the reader round's
// mapping: each thread writes its registers at their logical indices and reads back the
// amplitudes its registers hold in the new mapping, through the descriptor X (index map A and
// sign (-1)^Q).  Logical index j of a point lives at LDS entry swz(pbase ^ M j), M an invertible
// GF(2) map chosen per exchange for conflict-free banks.  Address arithmetic: pbase is a multiple
// of 2^N and every index is below 2^N, so pbase + x equals pbase ^ x; M and the swizzle are linear
// over GF(2), so the entry of j ^ o is the entry of j XOR swz(M o), and the planner stores
// 8 swz(M o) (byte offsets of complex64 entries) for the eight register offsets (woff for the
// writer, roff for the reader).
// Per exchange a lane needs three words: its writer and reader byte bases and the sign bits of
// its eight reads (the planner tabulates them per thread of a point: QLane); each access then
// costs one XOR.
struct XLane {
  uint32_t wb, rb, sgn;
};

// Per-round uniform data, loaded once before the round's first barrier and pinned in SGPRs:
// scalar loads share the lgkm counter with LDS operations, so a scalar load inside a slot would
// make the next use wait for every outstanding LDS write as well.
template <typename V>
__device__ __forceinline__ void pin_sgpr(V& v) { asm volatile("" : "+s"(v)); }

template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

// Marks statevector S as computed at this point of the instruction stream: keeps the compiler
// from sinking a group's gate arithmetic past the following barrier, which would undo the
// overlap of that group's arithmetic with another group's LDS traffic.
template <int S>
__device__ __forceinline__ void pin_sv(float (&sr)[8][8], float (&si)[8][8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) asm volatile("" : "+v"(sr[S][r]), "+v"(si[S][r]));
}

struct RoundCoef {
  float c[40];   // gate b's 2x2 matrix (U, or U^H in the adjoint) at c[8b .. 8b+7]; b = 3, 4: swap slots
  int gid[5];    // fused-gate ids (-1: none): register bits 0..2, then swap slots 0, 1
};

template <bool ADJ, int NS>
__device__ __forceinline__ RoundCoef load_round(CP<QRound> rk, CP<float> gtab, int F) {
  RoundCoef R;
#pragma unroll
  for (int b = 0; b < 3 + NS; ++b) {
    const int g = b < 3 ? rk->gate[b] : rk->sgate[b - 3];
    R.gid[b] = g;
    const int gi = g >= 0 ? g : F;
#pragma unroll
    for (int e = 0; e < 8; ++e) R.c[8 * b + e] = gtab[gi * kGT + (ADJ ? 8 : 0) + e];
  }
#pragma unroll
  for (int i = 0; i < 8 * (3 + NS); ++i) pin_sgpr(R.c[i]);
#pragma unroll
  for (int b = 0; b < 3 + NS; ++b) pin_sgpr(R.gid[b]);
  return R;
}

struct Offs {
  uint32_t o[8];
};

__device__ __forceinline__ Offs load_offs(CP<uint32_t> p) {
  Offs O;
#pragma unroll
  for (int r = 0; r < 8; ++r) { O.o[r] = p[r]; pin_sgpr(O.o[r]); }
  return O;
}

// The lane words of exchange k in direction dir (0 forward, 1 reverse) for thread u of the point
// whose swizzled base is pb8 = 8 swz(pbase): one 16-byte vector load from the plan's lane table
// (vector loads use their own wait counter, so a load issued early does not hold up LDS waits).
__device__ __forceinline__ XLane lane_words(const QLane* __restrict__ lanes, int dir, int R, int k, int TPn,
                                            uint32_t u, uint32_t pb8) {
  const QLane L = lanes[((size_t)dir * R + k) * TPn + u];
  XLane x;
  x.wb = L.wb ^ pb8;
  x.rb = L.rb ^ pb8;
  x.sgn = L.sgn;
  return x;
}

// Writes statevectors SV0 and SV1 to LDS planes PL and PL + 1 in the writer mapping wr.
template <int T, int SV0, int SV1, int PL>
__device__ __forceinline__ void xwrite(const float (&sr)[8][8], const float (&si)[8][8], float2* __restrict__ buf,
                                       const Offs& wo, uint32_t wb) {
  constexpr uint32_t PLANE = T * 8 * 8;   // bytes; a power of two above every in-plane offset
  char* b = reinterpret_cast<char*>(buf);
  const uint32_t base = wb | (PL * PLANE);   // plane PL folded into the base: one XOR per access
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t o = base ^ wo.o[r];
    *reinterpret_cast<float2*>(b + o) = make_float2(sr[SV0][r], si[SV0][r]);
    *reinterpret_cast<float2*>(b + PLANE + o) = make_float2(sr[SV1][r], si[SV1][r]);
  }
}

// Reads statevectors SV0 and SV1 back from planes PL, PL + 1 through the descriptor X.  SG = false:
// the circuit has no CZ stage, so no exchange carries signs and the sign code is left out.
template <int T, int SV0, int SV1, int PL, bool SG = true>
__device__ __forceinline__ void xread(float (&sr)[8][8], float (&si)[8][8], const float2* __restrict__ buf,
                                      const Offs& ro, bool signs, uint32_t rb, uint32_t sgn) {
  // SV0 is read completely before SV1, so the gates on SV0 can start while SV1 is in flight.
  constexpr uint32_t PLANE = T * 8 * 8;   // bytes; a power of two above every in-plane offset
  const char* b = reinterpret_cast<const char*>(buf);
  const uint32_t base = rb | (PL * PLANE);   // plane PL folded into the base: one XOR per access
  // raised wave priority while issuing the reads (as for the matrix-core chains): after a
  // barrier the wave's reads go out ahead of the other wave's arithmetic (12-qubit step 298 ->
  // 284 ms)
  __builtin_amdgcn_s_setprio(1);
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t o = base ^ ro.o[r];
      const float2 v = *reinterpret_cast<const float2*>(b + h * PLANE + o);
      if (h == 0) { sr[SV0][r] = v.x; si[SV0][r] = v.y; } else { sr[SV1][r] = v.x; si[SV1][r] = v.y; }
    }
  __builtin_amdgcn_s_setprio(0);
  if (SG && signs) {   // a CZ stage: negate the amplitudes whose sign bit is set (uniform branch)
    // The empty volatile asm keeps this a branch: merged into the unconditional path, the flips
    // would cost two XORs per amplitude on every exchange and consume the loaded values at once,
    // which forces the LDS reads to complete before any independent work can cover them.
    asm volatile("");
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t flip = ((sgn >> r) & 1u) << 31;   // negate by flipping the sign bits
      sr[SV0][r] = __uint_as_float(__float_as_uint(sr[SV0][r]) ^ flip);
      si[SV0][r] = __uint_as_float(__float_as_uint(si[SV0][r]) ^ flip);
      sr[SV1][r] = __uint_as_float(__float_as_uint(sr[SV1][r]) ^ flip);
      si[SV1][r] = __uint_as_float(__float_as_uint(si[SV1][r]) ^ flip);
    }
  }
}

// Unpipelined exchange of statevectors [0, NSV) in groups of EXS planes (used when the LDS
// holds only two planes per workgroup).
template <int N, int T, int NSV, int EXS>
__device__ __forceinline__ void exchange(float (&sr)[8][8], float (&si)[8][8], float2* __restrict__ buf,
                                         CP<QXchg> X, const XLane& x) {
  static_assert(EXS == 2, "pairs of planes");
  const Offs wo = load_offs(X->woff), ro = load_offs(X->roff);
  const bool sg = X->nterms != 0;
#pragma unroll
  for (int g = 0; g < NSV; g += 2) {
    if (g == 0) xwrite<T, 0, 1, 0>(sr, si, buf, wo, x.wb);
    if (g == 2) xwrite<T, 2, 3, 0>(sr, si, buf, wo, x.wb);
    if (g == 4) xwrite<T, 4, 5, 0>(sr, si, buf, wo, x.wb);
    if (g == 6) xwrite<T, 6, 7, 0>(sr, si, buf, wo, x.wb);
    __syncthreads();
    if (g == 0) xread<T, 0, 1, 0>(sr, si, buf, ro, sg, x.rb, x.sgn);
    if (g == 2) xread<T, 2, 3, 0>(sr, si, buf, ro, sg, x.rb, x.sgn);
    if (g == 4) xread<T, 4, 5, 0>(sr, si, buf, ro, sg, x.rb, x.sgn);
    if (g == 6) xread<T, 6, 7, 0>(sr, si, buf, ro, sg, x.rb, x.sgn);
    __syncthreads();
  }
}

// Swap slot I of statevectors [S0, S0 + NSV): register bit I trades places with lane bit 4 + I
// (thread bit 4 + I).  For each register pair (r, r | 2^I) a cross-lane swap exchanges odd rows of
// the first with even rows of the second (lane bit 4, permlane16_swap) or the upper half of the
// first with the lower half of the second (lane bit 5, permlane32_swap); the value at (register
// bit q', lane bit h') afterwards is the one that was at (q = h', h = q').  An involution.
template <int I, int S0, int NSV>
__device__ __forceinline__ void swap_slot(float (&sr)[8][8], float (&si)[8][8]) {
#pragma unroll
  for (int s = S0; s < S0 + NSV; ++s)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r & (1 << I)) continue;
      const int r1 = r | (1 << I);
      if (I == 0) {
        const auto a = __builtin_amdgcn_permlane16_swap(__float_as_int(sr[s][r]), __float_as_int(sr[s][r1]), false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(__float_as_int(si[s][r]), __float_as_int(si[s][r1]), false, false);
        sr[s][r] = __int_as_float(a[0]); sr[s][r1] = __int_as_float(a[1]);
        si[s][r] = __int_as_float(b[0]); si[s][r1] = __int_as_float(b[1]);
      } else {
        const auto a = __builtin_amdgcn_permlane32_swap(__float_as_int(sr[s][r]), __float_as_int(sr[s][r1]), false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(__float_as_int(si[s][r]), __float_as_int(si[s][r1]), false, false);
        sr[s][r] = __int_as_float(a[0]); sr[s][r1] = __int_as_float(a[1]);
        si[s][r] = __int_as_float(b[0]); si[s][r1] = __int_as_float(b[1]);
      }
    }
}

// Forward gates of a round on statevectors S0, S0 + 1 (an absent gate is the identity entry):
// gates01 applies the gates on register bits 0 and 1, gate2 the gate on bit 2 (gates on
// different qubits commute, so the split point is free).
template <int S0>
__device__ __forceinline__ void gates01(float (&sr)[8][8], float (&si)[8][8], const RoundCoef& R) {
  apply_gate<0, S0, 1>(sr, si, R.c); apply_gate<1, S0, 1>(sr, si, R.c + 8);
  apply_gate<0, S0 + 1, 1>(sr, si, R.c); apply_gate<1, S0 + 1, 1>(sr, si, R.c + 8);
}
template <int S0>
__device__ __forceinline__ void gate2(float (&sr)[8][8], float (&si)[8][8], const RoundCoef& R) {
  apply_gate<2, S0, 1>(sr, si, R.c + 16); apply_gate<2, S0 + 1, 1>(sr, si, R.c + 16);
}
// The rest of a round after the bit-0/1 gates: the bit-2 gate, then the swap slots with their gates
// (the statevectors end in the round's output mapping).
template <int S0, int NS>
__device__ __forceinline__ void finish(float (&sr)[8][8], float (&si)[8][8], const RoundCoef& R) {
  gate2<S0>(sr, si, R);
  if (NS > 0) {
    swap_slot<0, S0, 2>(sr, si);
    apply_gate<0, S0, 1>(sr, si, R.c + 24); apply_gate<0, S0 + 1, 1>(sr, si, R.c + 24);
  }
  if (NS > 1) {
    swap_slot<1, S0, 2>(sr, si);
    apply_gate<1, S0, 1>(sr, si, R.c + 32); apply_gate<1, S0 + 1, 1>(sr, si, R.c + 32);
  }
}
template <int S0, int NS>
__device__ __forceinline__ void round_fwd(float (&sr)[8][8], float (&si)[8][8], const RoundCoef& R) {
  gates01<S0>(sr, si, R);
  finish<S0, NS>(sr, si, R);
}

// Adds v to a per-wave statistic slot in LDS with an LDS float add that returns nothing, so the
// wave does not wait for its outstanding LDS operations as a read-modify-write would.  Each slot
// belongs to one wave and receives one lane's value per flush, in program order, so the sums are
// those of the read-modify-write, bit for bit.
__device__ __forceinline__ void slot_add(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wave-reduces the round's gate statistics (register bits 0..2, then the NS swap slots) and adds
// them to the per-wave LDS slots.
template <int NS>
__device__ __forceinline__ void round_stat_flush(const RoundCoef& R, float* __restrict__ slots, const float* q, int F,
                                                 int wave, int lane) {
#pragma unroll
  for (int bb = 0; bb < 3 + NS; ++bb) {
    const int gsrc = R.gid[bb];
    const float v4[4] = {q[3 * bb], q[3 * bb + 1], q[3 * bb + 2], 0.f};
    const float v = wave_reduce_scatter4(v4);
    if (gsrc >= 0 && (lane & 15) == 0 && lane < 48) slot_add(slots + (wave * F + gsrc) * kGS + (lane >> 4), v);
  }
}

// Adjoint of a round on the pair (C, 4 + C), starting in the round's output mapping: the swap-slot
// gates are pulled back first, each gate's statistic taken right after its pull-back (q[9 + 3i]),
// the swaps undone, then the three register-bit gates pulled back (their statistics follow in
// stat_accum, at the round input).  PULL = false (a round of the leading stage): nothing is pulled
// back; every statistic is taken at the stage output, where the stage's gates all commute.
template <int C, int NS, bool PULL = true>
__device__ __forceinline__ void round_adj(float (&sr)[8][8], float (&si)[8][8], const RoundCoef& R, float* q) {
  if (NS > 1) {
    if (PULL) { apply_gate<1, C, 1>(sr, si, R.c + 32); apply_gate<1, 4 + C, 1>(sr, si, R.c + 32); }
    accum_s1<1, C>(sr, si, q + 12);
    swap_slot<1, C, 1>(sr, si); swap_slot<1, 4 + C, 1>(sr, si);
  }
  if (NS > 0) {
    if (PULL) { apply_gate<0, C, 1>(sr, si, R.c + 24); apply_gate<0, 4 + C, 1>(sr, si, R.c + 24); }
    accum_s1<0, C>(sr, si, q + 9);
    swap_slot<0, C, 1>(sr, si); swap_slot<0, 4 + C, 1>(sr, si);
  }
  if (PULL) {
    apply_gate<2, C, 1>(sr, si, R.c + 16); apply_gate<2, 4 + C, 1>(sr, si, R.c + 16);
    apply_gate<1, C, 1>(sr, si, R.c + 8);  apply_gate<1, 4 + C, 1>(sr, si, R.c + 8);
    apply_gate<0, C, 1>(sr, si, R.c);      apply_gate<0, 4 + C, 1>(sr, si, R.c);
  }
}

// The pair's share of the round's three register-bit gate statistics, q[3 b + k] += S_k(bit b).
// These gates act on different qubits and commute, so every gate's statistic may be taken with
// both statevectors at the round input (all three gates pulled back): then the pull-backs of the
// other two gates cancel inside <lambda|sigma_b|psi>.
template <int C>
__device__ __forceinline__ void stat_accum(const float (&sr)[8][8], const float (&si)[8][8], float* q) {
  accum_s1<0, C>(sr, si, q);
  accum_s1<1, C>(sr, si, q + 3);
  accum_s1<2, C>(sr, si, q + 6);
}

// One gate's eight coefficients, loaded and pinned in SGPRs like a round's (returned by value:
// a local array read through apply_gate's selects would be kept in scratch memory instead).
struct GateCoef {
  float c[8];
};
__device__ __forceinline__ GateCoef load_gate(CP<float> g) {
  GateCoef G;
#pragma unroll
  for (int e = 0; e < 8; ++e) { G.c[e] = g[e]; pin_sgpr(G.c[e]); }
  return G;
}

template <int NQ>
__device__ __forceinline__ void pin_q(float* q) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) asm volatile("" : "+v"(q[i]));
}

// One gate of round_adj_all: all eight statevectors <- U^H on register bit B (unless PULL is
// false: a gate of the leading stage), its statistic flushed at once.
template <int B, bool PULL>
__device__ __forceinline__ void adj_gate_all(float (&sr)[8][8], float (&si)[8][8], int gsrc, CP<float> gtab, int F,
                                             float* __restrict__ slots, int wave, int lane) {
  float q6[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) q6[e] = 0.f;
  if (PULL) {
    const int gid = gsrc >= 0 ? gsrc : F;
    const GateCoef d = load_gate(gtab + gid * kGT + 8);   // U^H
    apply_gate<B, 0, 8>(sr, si, d.c);
  }
  accum_s<B>(sr, si, q6);
  const float v4[4] = {q6[0] + q6[3], q6[1] + q6[4], q6[2] + q6[5], 0.f};
  const float v = wave_reduce_scatter4(v4);
  if (gsrc >= 0 && (lane & 15) == 0 && lane < 48) slot_add(slots + (wave * F + gsrc) * kGS + (lane >> 4), v);
}

// Adjoint of round rk on all four pairs, gate by gate (where no pipelining separates the pairs;
// keeps one gate's values live at a time): swap-slot gates and swaps in reverse, then the
// register-bit gates.
template <int NS, bool PULL>
__device__ __forceinline__ void round_adj_all(float (&sr)[8][8], float (&si)[8][8], CP<QRound> rk, CP<float> gtab,
                                              int F, float* __restrict__ slots, int wave, int lane) {
  if (NS > 1) {
    adj_gate_all<1, PULL>(sr, si, rk->sgate[1], gtab, F, slots, wave, lane);
    swap_slot<1, 0, 8>(sr, si);
  }
  if (NS > 0) {
    adj_gate_all<0, PULL>(sr, si, rk->sgate[0], gtab, F, slots, wave, lane);
    swap_slot<0, 0, 8>(sr, si);
  }
  adj_gate_all<2, PULL>(sr, si, rk->gate[2], gtab, F, slots, wave, lane);
  adj_gate_all<1, PULL>(sr, si, rk->gate[1], gtab, F, slots, wave, lane);
  adj_gate_all<0, PULL>(sr, si, rk->gate[0], gtab, F, slots, wave, lane);
}

// ---- phase stages (CRZ runs) ------------------------------------------------------------------
// In a round's input mapping, slot k (register bit k < 3, thread bit k - 3 otherwise) holds the
// index bit of qubit N - 1 - tpos[k].  phi(j) = sum_q alpha_q b_q + sum_(q<q') beta_qq' b_q b_q' is
// split into the thread's part and per-register terms; all sums are unsigned 32-bit fractions of a
// turn, so they are exact modulo 2 pi, and only the final angle of each amplitude is rounded.
template <int N>
__device__ __forceinline__ uint32_t phase_beta(CP<uint32_t> coef, int a, int b) {
  return a < b ? coef[N + phase_pair_index(N, a, b)] : coef[N + phase_pair_index(N, b, a)];
}

template <int N>
__device__ __forceinline__ void phase_factors(CP<QRound> rk, CP<uint32_t> coef, uint32_t u, float (&pc)[8],
                                              float (&ps)[8]) {
  int qk[N];
#pragma unroll
  for (int k = 0; k < N; ++k) qk[k] = N - 1 - rk->tpos[k];
  uint32_t th = 0, g0 = coef[qk[0]], g1 = coef[qk[1]], g2 = coef[qk[2]];
#pragma unroll
  for (int k = 3; k < N; ++k) {
    const uint32_t bk = (u >> (k - 3)) & 1u;
    uint32_t t = coef[qk[k]];
#pragma unroll
    for (int k2 = k + 1; k2 < N; ++k2) t += ((u >> (k2 - 3)) & 1u) * phase_beta<N>(coef, qk[k], qk[k2]);
    th += bk * t;
    g0 += bk * phase_beta<N>(coef, qk[0], qk[k]);
    g1 += bk * phase_beta<N>(coef, qk[1], qk[k]);
    g2 += bk * phase_beta<N>(coef, qk[2], qk[k]);
  }
  const uint32_t d01 = phase_beta<N>(coef, qk[0], qk[1]);
  const uint32_t d02 = phase_beta<N>(coef, qk[0], qk[2]);
  const uint32_t d12 = phase_beta<N>(coef, qk[1], qk[2]);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    uint32_t ph = th;
    if (r & 1) ph += g0;
    if (r & 2) ph += g1;
    if (r & 4) ph += g2;
    if ((r & 3) == 3) ph += d01;
    if ((r & 5) == 5) ph += d02;
    if ((r & 6) == 6) ph += d12;
    // angle = 2 pi ph / 2^32 = pi x with x = (signed) ph / 2^31 in [-1, 1)
    sincospif((float)(int32_t)ph * 4.656612873077392578125e-10f, &ps[r], &pc[r]);
  }
}

// Multiply statevectors [S0, S0 + NS) by e^{+i phi} (CONJ: e^{-i phi}).
template <int S0, int NS, bool CONJ>
__device__ __forceinline__ void apply_phase(float (&sr)[8][8], float (&si)[8][8], const float (&pc)[8],
                                            const float (&ps)[8]) {
#pragma unroll
  for (int s = S0; s < S0 + NS; ++s)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const float c = pc[r], sn = CONJ ? -ps[r] : ps[r];
      const float a = sr[s][r], b = si[s][r];
      sr[s][r] = a * c - b * sn;
      si[s][r] = a * sn + b * c;
    }
}

// Phase-stage moments of w_j = Im(conj(lambda_j) psi_j) + sum_c Im(conj(mu_c,j) dpsi_c,j): M_q and
// M_qq' (q < q') summed over the wave, added to the wave's slots mslots[mom_off ...].
template <int N>
__device__ __forceinline__ void phase_moments(const float (&sr)[8][8], const float (&si)[8][8], CP<QRound> rk, uint32_t u,
                                              float* __restrict__ mslots, int lane) {
  float w[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    float v = 0.f;
#pragma unroll
    for (int p = 0; p < 4; ++p) v += sr[4 + p][r] * si[p][r] - si[4 + p][r] * sr[p][r];
    w[r] = v;
  }
  float Wi[3] = {0.f, 0.f, 0.f}, Wii[3] = {0.f, 0.f, 0.f}, Wt = 0.f;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    Wt += w[r];
    if (r & 1) Wi[0] += w[r];
    if (r & 2) Wi[1] += w[r];
    if (r & 4) Wi[2] += w[r];
    if ((r & 3) == 3) Wii[0] += w[r];
    if ((r & 5) == 5) Wii[1] += w[r];
    if ((r & 6) == 6) Wii[2] += w[r];
  }
  int qk[N];
#pragma unroll
  for (int k = 0; k < N; ++k) qk[k] = N - 1 - rk->tpos[k];
  auto flush = [&](float v, int idx) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) slot_add(mslots + idx, v);
  };
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const float v = k < 3 ? Wi[k] : (((u >> (k - 3)) & 1u) ? Wt : 0.f);
    flush(v, qk[k]);
  }
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int k2 = k + 1; k2 < N; ++k2) {
      float v;
      if (k2 < 3) v = Wii[k + k2 - 1];                                  // (0,1) (0,2) (1,2)
      else if (k < 3) v = ((u >> (k2 - 3)) & 1u) ? Wi[k] : 0.f;
      else v = (((u >> (k - 3)) & (u >> (k2 - 3))) & 1u) ? Wt : 0.f;
      const int a = qk[k] < qk[k2] ? qk[k] : qk[k2], b = qk[k] < qk[k2] ? qk[k2] : qk[k];
      flush(v, N + phase_pair_index(N, a, b));
    }
}

// ---- angle encoding of one qubit ------------------------------------------------------------
// Embedded single-qubit state e(b) (b = 0, 1) and its angle derivative d(b) for qubit q, with the
// Jacobian d theta_q / d(t, x, y).  RY: e = (cos, sin), RX: e = (cos, -i sin), of theta/2.  When the
// circuit opens with a rotation stage, the qubit's gate U of that stage is applied here (e <- U e,
// d <- U d): the stage acts on the product state, so the state after it is still a product.
struct QEnc {
  float e0r, e0i, e1r, e1i, d0r, d0i, d1r, d1i, j[3];
};

template <int N>
__device__ __forceinline__ QEnc encode_qubit(CP<QPlanDev> plan, CP<float> gtab, const FusedArgs& a, long long pt,
                                             bool valid, const float* p3, int q) {
  float c, s, j0 = 0.f, j1 = 0.f, j2 = 0.f;
  if (plan->enc_kind == QP_ENC_CYCLE) {
    const int cc = plan->coord_of_qubit[q];
    const float x = cc == 0 ? p3[0] : (cc == 1 ? p3[1] : p3[2]);
    float jv;
    const int sc = plan->enc_scale;
    if (sc == QP_SCALE_PI) {           // theta/2 = pi x/2
      sincospif(0.5f * x, &s, &c);
      jv = 3.14159265358979323846f;
    } else if (sc == QP_SCALE_BIAS) {  // theta/2 = pi (x+1)/4
      sincospif(0.25f * (x + 1.f), &s, &c);
      jv = 1.57079632679489661923f;
    } else if (sc == QP_SCALE_NONE) {
      sincosf(0.5f * x, &s, &c);
      jv = 1.f;
    } else {
      const float xx = fminf(fmaxf(x, -1.f), 1.f);
      const float th = (sc == QP_SCALE_ASIN) ? asinf(xx) + 1.57079632679489661923f : acosf(xx);
      sincosf(0.5f * th, &s, &c);
      const float rs = 1.f / sqrtf(fmaxf(1.f - xx * xx, 0.f));
      jv = (sc == QP_SCALE_ASIN) ? rs : -rs;
    }
    j0 = cc == 0 ? jv : 0.f;
    j1 = cc == 1 ? jv : 0.f;
    j2 = cc == 2 ? jv : 0.f;
  } else {   // angles given per point (QP_ENC_ANGLES, or random Fourier features formed beforehand)
    float th = 0.f;
    if (valid) {
      th = a.angles[pt * N + q];
      j0 = a.jac[(pt * N + q) * 3 + 0];
      j1 = a.jac[(pt * N + q) * 3 + 1];
      j2 = a.jac[(pt * N + q) * 3 + 2];
    }
    sincosf(0.5f * th, &s, &c);
  }
  QEnc E;
  E.e0r = c; E.e0i = 0.f;
  E.d0r = -0.5f * s; E.d0i = 0.f;
  if (plan->enc_gate == QP_ENC_RY) {
    E.e1r = s; E.e1i = 0.f; E.d1r = 0.5f * c; E.d1i = 0.f;
  } else {   // RX|0> = (cos, -i sin)
    E.e1r = 0.f; E.e1i = -s; E.d1r = 0.f; E.d1i = -0.5f * c;
  }
  const int hg = plan->head_gate[q];
  if (hg >= 0) {
    CP<float> g = gtab + hg * kGT;   // U: u00r, u00i, u01r, u01i, u10r, u10i, u11r, u11i
    const float xr = E.e0r, xi = E.e0i, yr = E.e1r, yi = E.e1i;
    E.e0r = g[0] * xr - g[1] * xi + g[2] * yr - g[3] * yi;
    E.e0i = g[0] * xi + g[1] * xr + g[2] * yi + g[3] * yr;
    E.e1r = g[4] * xr - g[5] * xi + g[6] * yr - g[7] * yi;
    E.e1i = g[4] * xi + g[5] * xr + g[6] * yi + g[7] * yr;
    const float ar = E.d0r, ai = E.d0i, br = E.d1r, bi = E.d1i;
    E.d0r = g[0] * ar - g[1] * ai + g[2] * br - g[3] * bi;
    E.d0i = g[0] * ai + g[1] * ar + g[2] * bi + g[3] * br;
    E.d1r = g[4] * ar - g[5] * ai + g[6] * br - g[7] * bi;
    E.d1i = g[4] * ai + g[5] * ar + g[6] * bi + g[7] * br;
  }
  E.j[0] = j0; E.j[1] = j1; E.j[2] = j2;
  return E;
}

// ---- gradients with respect to the per-point angles and their Jacobian ------------------------
// The embedding rotation of qubit q has generator G_q (Y for RY, X for RX): d psi_0/d theta_q =
// -(i/2) G_q psi_0, and the tangents are dpsi_c,0 = sum_q J_qc (-(i/2) G_q) psi_0, so (the G's of
// different qubits commute) d dpsi_c,0/d theta_q = -(i/2) G_q dpsi_c,0.  With lambda, mu_c the
// adjoints pulled back to the embedded state,
//   dL/d theta_q = Im <lambda|G_q|psi> + sum_c Im <mu_c|G_q|dpsi_c>,   dL/d J_qc = Im <mu_c|G_q|psi>,
// the same Pauli statistics the adjoint takes for every gate, but per point.  When the circuit's
// opening rotation stage is folded into the encoding, the sweep ends at that stage's output, and
// G_q is replaced by U_q G_q U_q^H (U_q the stage's gate on qubit q), which the statistics
// contract with as an axis (n_x, n_y, n_z).  At the end of the sweep the statevectors sit in round
// 0's input mapping.  The partner amplitude of a pair (index bit of qubit q flipped) lies in the
// same thread (register bit) or in another thread of the point (thread bit); it is read back from
// the LDS planes, where the psi-family is staged two statevectors at a time.
template <int N, int T>
__device__ __forceinline__ float enc_pair(float nx, float ny, float nz, float sb, float xr, float xi, float yor,
                                          float yoi, float2 yp) {
  const float im_p = xr * yp.y - xi * yp.x;    // Im(conj(x) y_partner)
  const float re_p = xr * yp.x + xi * yp.y;    // Re(conj(x) y_partner)
  const float im_o = xr * yoi - xi * yor;      // Im(conj(x) y_own)
  return nx * im_p + sb * (ny * re_p - nz * im_o);
}

// One of two passes (PASS 0: partners of psi and dpsi_t; PASS 1: of dpsi_x and dpsi_y).  The
// qubits are taken one at a time (a loop, so no per-qubit register arrays), each qubit's sums are
// reduced over the point's threads at once, and the point's first thread writes them (PASS 0) or
// adds its share (PASS 1).
template <int N, int T, int PASS>
__device__ __forceinline__ void enc_grad_pass(const float (&sr)[8][8], const float (&si)[8][8],
                                              float2* __restrict__ buf, float* __restrict__ red, CP<QPlanDev> plan,
                                              CP<QRound> r0, CP<float> gtab, uint32_t jl, const FusedArgs& a,
                                              long long pt, bool valid, uint32_t u) {
  constexpr int PLANE = T * 8;
  constexpr int TP = 1 << (N - 3);
  const uint32_t tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const uint32_t l0 = r0->tpos[0], l1 = r0->tpos[1], l2 = r0->tpos[2];
  __syncthreads();   // the planes are free (every wave is past its last read of the sweep)
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t e = tid * 8 + (r ^ (tid & 7));
    buf[e] = make_float2(sr[2 * PASS][r], si[2 * PASS][r]);
    buf[PLANE + e] = make_float2(sr[2 * PASS + 1][r], si[2 * PASS + 1][r]);
  }
  __syncthreads();
  const bool rx = plan->enc_gate == QP_ENC_RX;
#pragma unroll 1
  for (int q = 0; q < N; ++q) {
    const int pos = N - 1 - q;
    uint32_t rmask = 0, tmask = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (r0->tpos[k] == pos) {
        if (k < 3) rmask = 1u << k;
        else tmask = 1u << (k - 3);
      }
    }
    // axis of U G U^H (U: the opening-stage gate on q, identity if none; G = X or Y)
    float u8[8] = {1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f};
    const int hg = plan->head_gate[q];
    if (hg >= 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) u8[i] = gtab[hg * kGT + i];
    }
    // W = U G: X swaps U's columns; Y gives [[i u01, -i u00], [i u11, -i u10]]
    float w00r, w00i, w01r, w01i;
    if (rx) {
      w00r = u8[2]; w00i = u8[3]; w01r = u8[0]; w01i = u8[1];
    } else {
      w00r = -u8[3]; w00i = u8[2]; w01r = u8[1]; w01i = -u8[0];
    }
    // M = W U^H: M00 = W00 conj(u00) + W01 conj(u01), M01 = W00 conj(u10) + W01 conj(u11)
    const float m00r = w00r * u8[0] + w00i * u8[1] + w01r * u8[2] + w01i * u8[3];
    const float m01r = w00r * u8[4] + w00i * u8[5] + w01r * u8[6] + w01i * u8[7];
    const float m01i = w00i * u8[4] - w00r * u8[5] + w01i * u8[6] - w01r * u8[7];
    const float nx = m01r, ny = -m01i, nz = m00r;
    const uint32_t ptid = tid ^ tmask;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t j = jl ^ reg_off(r, l0, l1, l2);
      const float sb = ((j >> pos) & 1u) ? 1.f : -1.f;
      const uint32_t e = ptid * 8 + (((uint32_t)r ^ rmask) ^ (ptid & 7));
      const float2 y0 = buf[e];
      const float2 y1 = buf[PLANE + e];
      if (PASS == 0) {   // partners of psi and dpsi_t
        s0 += enc_pair<N, T>(nx, ny, nz, sb, sr[4][r], si[4][r], sr[0][r], si[0][r], y0);
        s0 += enc_pair<N, T>(nx, ny, nz, sb, sr[5][r], si[5][r], sr[1][r], si[1][r], y1);
        s1 += enc_pair<N, T>(nx, ny, nz, sb, sr[5][r], si[5][r], sr[0][r], si[0][r], y0);
        s2 += enc_pair<N, T>(nx, ny, nz, sb, sr[6][r], si[6][r], sr[0][r], si[0][r], y0);
        s3 += enc_pair<N, T>(nx, ny, nz, sb, sr[7][r], si[7][r], sr[0][r], si[0][r], y0);
      } else {           // partners of dpsi_x and dpsi_y
        s0 += enc_pair<N, T>(nx, ny, nz, sb, sr[6][r], si[6][r], sr[2][r], si[2][r], y0);
        s0 += enc_pair<N, T>(nx, ny, nz, sb, sr[7][r], si[7][r], sr[3][r], si[3][r], y1);
      }
    }
    // sum over the point's threads
#pragma unroll
    for (int off = 1; off < (TP < 64 ? TP : 64); off <<= 1) {
      s0 += __shfl_xor(s0, off);
      if (PASS == 0) {
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
        s3 += __shfl_xor(s3, off);
      }
    }
    if (TP > 64) {   // the point spans TP / 64 waves: combine them through the scratch slots
      constexpr int WPP = TP > 64 ? TP / 64 : 1;
      if (lane == 0) {
        red[wave * 40 + 0] = s0;
        red[wave * 40 + 1] = s1;
        red[wave * 40 + 2] = s2;
        red[wave * 40 + 3] = s3;
      }
      __syncthreads();
      const int w0 = (wave / WPP) * WPP;
      float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f;
      for (int w = 0; w < WPP; ++w) {
        t0 += red[(w0 + w) * 40 + 0];
        t1 += red[(w0 + w) * 40 + 1];
        t2 += red[(w0 + w) * 40 + 2];
        t3 += red[(w0 + w) * 40 + 3];
      }
      s0 = t0; s1 = t1; s2 = t2; s3 = t3;
      __syncthreads();
    }
    if (valid && u == 0) {
      if (PASS == 0) {
        if (a.d_angles) a.d_angles[pt * N + q] = s0;
        if (a.d_jac) {
          a.d_jac[(pt * N + q) * 3 + 0] = s1;
          a.d_jac[(pt * N + q) * 3 + 1] = s2;
          a.d_jac[(pt * N + q) * 3 + 2] = s3;
        }
      } else if (a.d_angles) {
        a.d_angles[pt * N + q] += s0;
      }
    }
  }
}

template <int N, int T>
__device__ __forceinline__ void encoding_grads(const float (&sr)[8][8], const float (&si)[8][8],
                                               float2* __restrict__ buf, float* __restrict__ red, CP<QPlanDev> plan,
                                               CP<QRound> r0, CP<float> gtab, const FusedArgs& a, long long pt,
                                               bool valid, uint32_t u) {
  const uint32_t jl = deposit_thread<N>(u, r0->tpos);
  enc_grad_pass<N, T, 0>(sr, si, buf, red, plan, r0, gtab, jl, a, pt, valid, u);
  enc_grad_pass<N, T, 1>(sr, si, buf, red, plan, r0, gtab, jl, a, pt, valid, u);
  __syncthreads();   // the next tile's first exchange writes the planes
}

// Packed modes: the product state of point pt0 + SL in statevector slot SL, formed in the mapping
// emap (no input tangents; an out-of-range point gives the zero state).
template <int N, int SL>
__device__ __forceinline__ void packed_state(float (&sr)[8][8], float (&si)[8][8], CP<QPlanDev> plan, CP<float> gtab,
                                             const FusedArgs& a, long long pt0, uint32_t u, CP<int32_t> emap) {
  const long long pts = pt0 + SL;
  const bool vs = pts < a.P;
  float q3[3] = {0.f, 0.f, 0.f};
  if (vs && a.points && plan->enc_kind != QP_ENC_ANGLES) {
    q3[0] = a.points[pts * 3 + 0];
    q3[1] = a.points[pts * 3 + 1];
    q3[2] = a.points[pts * 3 + 2];
  }
  float Pr = vs ? 1.f : 0.f, Pi = 0.f;
#pragma unroll 1
  for (int k = 3; k < N; ++k) {
    const QEnc E = encode_qubit<N>(plan, gtab, a, pts, vs, q3, N - 1 - emap[k]);
    const bool bit = (u >> (k - 3)) & 1u;
    const float er = bit ? E.e1r : E.e0r, ei = bit ? E.e1i : E.e0i;
    const float npr = Pr * er - Pi * ei, npi = Pr * ei + Pi * er;
    Pr = npr; Pi = npi;
  }
  QEnc Q[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Q[i] = encode_qubit<N>(plan, gtab, a, pts, vs, q3, N - 1 - emap[i]);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    float pr = Pr, pi = Pi;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const bool b = (r >> i) & 1;
      const float er = b ? Q[i].e1r : Q[i].e0r, ei = b ? Q[i].e1i : Q[i].e0i;
      const float npr = pr * er - pi * ei, npi = pr * ei + pi * er;
      pr = npr; pi = npi;
    }
    sr[SL][r] = pr; si[SL][r] = pi;
  }
}

// ---- one tile of PPW points: forward, readout, seeds, adjoint --------------------------------
// buf: EXS exchange planes; slots: per-wave gate statistics [WAVES][F][kGS]; red: [WAVES][40].
// PH: the plan may carry CRZ phase stages (false where the caller knows it has none, as the
// uneven-batch kernels do for such circuits: the phase code is then compiled out).
template <int N, int T, int EXS, int MODE, bool SG = true, bool EG = false, bool PH = true>
__device__ __forceinline__ void fused_tile(const FusedArgs& a, int tile, float2* __restrict__ buf,
                                           float* __restrict__ slots, float* __restrict__ mslots,
                                           float* __restrict__ red, float& lacc) {
  constexpr int TP = 1 << (N - 3);         // threads per point
  constexpr int PPW = T / TP;              // points per workgroup tile (x4 in the packed modes)
  constexpr int DIM = 1 << N;
  constexpr bool PK = mode_packed(MODE);
  static_assert(PPW >= 1, "tile too small");
  static_assert(!(PK && EG), "the packed modes carry no input gradients");
  CP<QPlanDev> plan = to_const(a.plan);
  CP<char> pb = reinterpret_cast<CP<char>>(plan);
  CP<QRound> rounds = reinterpret_cast<CP<QRound>>(pb + plan->off_rounds);
  CP<QXchg> xf = reinterpret_cast<CP<QXchg>>(pb + plan->off_xf);
  CP<QXchg> xb = reinterpret_cast<CP<QXchg>>(pb + plan->off_xb);
  CP<float> gtab = to_const(a.gtab);
  // phase stages: descriptors in the plan, coefficients after the gate table
  const QPhaseStage* pstages = reinterpret_cast<const QPhaseStage*>(reinterpret_cast<const char*>(a.plan) + plan->off_phase);
  CP<uint32_t> pcoef = reinterpret_cast<CP<uint32_t>>(gtab + (a.n_fused + 1) * kGT);
  const int R = plan->n_rounds;
  const int m = plan->n_out;
  const int F = a.n_fused;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ps = tid / TP;
  const uint32_t u = (uint32_t)(tid % TP);
  const uint32_t pbase = (uint32_t)ps * DIM;
  // loss weights: 1/P for the mean over all points, 1/N_vac and 1/N_diel for the split loss
  float w_all = 1.f, w_vac = 1.f, w_diel = 1.f;
  if ((MODE == kModeMaxwell || MODE == kModeTotal) && !a.loss_sum) {
    w_all = a.P > 0 ? 1.f / (float)a.P : 0.f;
    if (a.loss_kind == QP_LOSS_DIEL_SPLIT) {
      const int nv = a.counts[0], nd = a.counts[1];
      w_vac = nv > 0 ? 1.f / (float)nv : 0.f;
      w_diel = nd > 0 ? 1.f / (float)nd : 0.f;
    }
  }
  float sr[8][8], si[8][8];
  {
    // packed modes: slot s of the thread group holds point pt0 + s
    const long long pt = PK ? ((long long)tile * PPW + ps) * 4 : (long long)tile * PPW + ps;
    const long long pt0 = pt;
    const bool valid = pt < a.P;

    // ---------------- encoding and product state -------------------------------------------
    // The leading rotation stage (rounds 0 .. H-1) is folded into the product state, which is
    // then formed in round H-1's output mapping (round 0's input mapping if H = 0).  Each qubit's
    // embedded amplitudes are formed where they are used (qubit index uniform across the
    // workgroup), so no per-qubit arrays are indexed at run time.
    const int H = plan->n_head;
    float p3[3] = {0.f, 0.f, 0.f};
    if (valid && a.points && plan->enc_kind != QP_ENC_ANGLES) {
      p3[0] = a.points[pt * 3 + 0];
      p3[1] = a.points[pt * 3 + 1];
      p3[2] = a.points[pt * 3 + 2];
    }
    if constexpr (PK) {
      // four product states, one per slot (no tangents); one call per slot keeps the slot index
      // a compile-time constant (the statevector arrays stay in registers)
      CP<int32_t> emap = H > 0 ? rounds[H - 1].tpost : rounds[0].tpos;
      packed_state<N, 0>(sr, si, plan, gtab, a, pt0, u, emap);
      packed_state<N, 1>(sr, si, plan, gtab, a, pt0, u, emap);
      packed_state<N, 2>(sr, si, plan, gtab, a, pt0, u, emap);
      packed_state<N, 3>(sr, si, plan, gtab, a, pt0, u, emap);
    } else {
      CP<int32_t> emap = H > 0 ? rounds[H - 1].tpost : rounds[0].tpos;
      // thread part: (P, D_c) by the product rule over the thread qubits
      float Pr = valid ? 1.f : 0.f, Pi = 0.f;
      float Dr[3] = {0.f, 0.f, 0.f}, Di[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 3; k < N; ++k) {
        const QEnc E = encode_qubit<N>(plan, gtab, a, pt, valid, p3, N - 1 - emap[k]);
        const bool bit = (u >> (k - 3)) & 1u;
        const float er = bit ? E.e1r : E.e0r, ei = bit ? E.e1i : E.e0i;
        const float dr = bit ? E.d1r : E.d0r, di = bit ? E.d1i : E.d0i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float nr = Dr[c] * er - Di[c] * ei + E.j[c] * (Pr * dr - Pi * di);
          const float ni = Dr[c] * ei + Di[c] * er + E.j[c] * (Pr * di + Pi * dr);
          Dr[c] = nr; Di[c] = ni;
        }
        const float npr = Pr * er - Pi * ei, npi = Pr * ei + Pi * er;
        Pr = npr; Pi = npi;
      }
      QEnc Q[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) Q[i] = encode_qubit<N>(plan, gtab, a, pt, valid, p3, N - 1 - emap[i]);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float pr = Pr, pi = Pi, dr[3] = {Dr[0], Dr[1], Dr[2]}, di[3] = {Di[0], Di[1], Di[2]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const bool b = (r >> i) & 1;
          const float er = b ? Q[i].e1r : Q[i].e0r, ei = b ? Q[i].e1i : Q[i].e0i;
          const float ddr = b ? Q[i].d1r : Q[i].d0r, ddi = b ? Q[i].d1i : Q[i].d0i;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float nr = dr[c] * er - di[c] * ei + Q[i].j[c] * (pr * ddr - pi * ddi);
            const float ni = dr[c] * ei + di[c] * er + Q[i].j[c] * (pr * ddi + pi * ddr);
            dr[c] = nr; di[c] = ni;
          }
          const float npr = pr * er - pi * ei, npi = pr * ei + pi * er;
          pr = npr; pi = npi;
        }
        sr[0][r] = pr; si[0][r] = pi;
#pragma unroll
        for (int c = 0; c < 3; ++c) { sr[1 + c][r] = dr[c]; si[1 + c][r] = di[c]; }
      }
    }
    // ---------------- forward rounds -------------------------------------------------------
    constexpr int NS = swap_slots(N);
    const QLane* __restrict__ lanes = reinterpret_cast<const QLane*>(reinterpret_cast<const char*>(a.plan) + plan->off_lanes);
    const uint32_t pb8 = swz(pbase) * 8u;
    if constexpr (EXS == 4) {
      // Software-pipelined: group A = statevectors {0, 1} (planes 0, 1), group B = {2, 3}
      // (planes 2, 3).  Each slot reads one group, finishes the other group's round (its bit-2
      // gate and swap slots) and writes it, then runs the bit-0/1 gates of the group just read:
      // the finishing work covers the read latency and the writes drain under the following
      // gates.  Every barrier separates a plane pair's reads from its next writes.
      // All four statevectors complete in round k0 - 1's output mapping: the encoding leaves them
      // there when the opening stage is folded (k0 = H); otherwise round 0 runs here (k0 = 1).
      int k0 = H;
      RoundCoef Rc = load_round<false, NS>(rounds + (H > 0 ? H - 1 : 0), gtab, F);
      if (k0 == 0) {
        round_fwd<0, NS>(sr, si, Rc);
        round_fwd<2, NS>(sr, si, Rc);
        k0 = 1;
      }
      if (k0 < R) {
        Offs wo = load_offs(xf[k0].woff);
        // lane words of the current exchange as scalars (updated inside the lambda below)
        uint32_t xwb, xrb, xsg;
        {
          const XLane x0 = lane_words(lanes, 0, R, k0, TP, u, pb8);
          xwb = x0.wb; xrb = x0.rb; xsg = x0.sgn;
        }
        xwrite<T, 0, 1, 0>(sr, si, buf, wo, xwb);
        // Iteration k: group A is read and runs round k; group B lags by half a round (it finishes
        // round k - 1 while A's read is in flight, except in the first iteration, where it is
        // complete).  The first iteration is peeled so that neither copy has a branch around
        // group B's work.
        auto iter = [&](int k, auto lag) {
          constexpr bool LAG = decltype(lag)::value;
          CP<QRound> rk = rounds + k;
          const RoundCoef Rk = load_round<false, NS>(rk, gtab, F);
          const Offs ro = load_offs(xf[k].roff);
          const bool sg = xf[k].nterms != 0;
          // the next exchange's lane words: a vector load issued a whole round ahead of its use
          XLane xn{xwb, xrb, xsg};
          if (k + 1 < R) xn = lane_words(lanes, 0, R, k + 1, TP, u, pb8);
          __syncthreads();
          xread<T, 0, 1, 0, SG>(sr, si, buf, ro, sg, xrb, xsg);
          if (LAG) finish<2, NS>(sr, si, Rc);          // group B finishes round k - 1
          xwrite<T, 2, 3, 2>(sr, si, buf, wo, xwb);
          gates01<0>(sr, si, Rk);
          pin_sv<0>(sr, si); pin_sv<1>(sr, si);
          // The next exchange's write offsets, loaded before the barrier: scalar loads share the
          // wait counter with LDS operations, and waiting here costs nothing.
          if (k + 1 < R) wo = load_offs(xf[k + 1].woff);
          __syncthreads();
          xread<T, 2, 3, 2, SG>(sr, si, buf, ro, sg, xrb, xsg);
          finish<0, NS>(sr, si, Rk);                   // group A finishes round k
          if (k + 1 < R) xwrite<T, 0, 1, 0>(sr, si, buf, wo, xn.wb);
          gates01<2>(sr, si, Rk);
          pin_sv<2>(sr, si); pin_sv<3>(sr, si);
          xwb = xn.wb; xrb = xn.rb; xsg = xn.sgn;
          Rc = Rk;
        };
        iter(k0, BoolC<false>{});
        for (int k = k0 + 1; k < R; ++k) iter(k, BoolC<true>{});
        __syncthreads();
        finish<2, NS>(sr, si, Rc);                     // group B finishes the last round
      }
    } else {
      for (int k = H; k < R; ++k) {
        CP<QRound> rk = rounds + k;
        if (k > 0) exchange<N, T, 4, 2>(sr, si, buf, xf + k, lane_words(lanes, 0, R, k, TP, u, pb8));
        if (PH && rk->phase >= 0) {   // CRZ phase stage after the exchange (unpipelined kernel only)
          float pc[8], ps[8];
          phase_factors<N>(rk, pcoef + to_const(pstages)[rk->phase].coef_off, u, pc, ps);
          apply_phase<0, 4, false>(sr, si, pc, ps);
        }
        const RoundCoef Rk = load_round<false, NS>(rk, gtab, F);
        round_fwd<0, NS>(sr, si, Rk);
        round_fwd<2, NS>(sr, si, Rk);
      }
    }
    // ---------------- readout ----------------------------------------------------------------
    CP<QRound> rl = rounds + (R - 1);   // the statevectors are in the last round's output mapping
    const uint32_t jl = deposit_thread<N>(u, rl->tpost);
    const uint32_t l0 = rl->tpost[0], l1 = rl->tpost[1], l2 = rl->tpost[2];
    float acc[kMaxOut * 4];
#pragma unroll
    for (int i = 0; i < kMaxOut * 4; ++i) acc[i] = 0.f;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t j = jl ^ reg_off(r, l0, l1, l2);
      // per output: <Z> and its three input tangents, or (packed) <Z> of the four slots' points
      const float p2 = sr[0][r] * sr[0][r] + si[0][r] * si[0][r];
      float gc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        gc[c] = PK ? sr[1 + c][r] * sr[1 + c][r] + si[1 + c][r] * si[1 + c][r]
                   : 2.f * (sr[0][r] * sr[1 + c][r] + si[0][r] * si[1 + c][r]);
#pragma unroll
      for (int i = 0; i < kMaxOut; ++i) {
        if (i < m) {
          const float z = parity(plan->zmask[i] & j) ? -1.f : 1.f;
          acc[i * 4 + 0] += z * p2;
          acc[i * 4 + 1] += z * gc[0];
          acc[i * 4 + 2] += z * gc[1];
          acc[i * 4 + 3] += z * gc[2];
        }
      }
    }
    // all-reduce over the point's thread group
    if (TP <= 64) {
#pragma unroll
      for (int off = 1; off < (TP < 64 ? TP : 64); off <<= 1)
#pragma unroll
        for (int i = 0; i < kMaxOut * 4; ++i)
          if (i < 4 * m) acc[i] += __shfl_xor(acc[i], off);
    } else {
#pragma unroll
      for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int i = 0; i < kMaxOut * 4; ++i)
          if (i < 4 * m) acc[i] += __shfl_xor(acc[i], off);
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kMaxOut * 4; ++i)
          if (i < 4 * m) red[wave * 40 + i] = acc[i];
      }
      __syncthreads();
      constexpr int WPP = TP / 64;   // waves per point
      const int w0 = (wave / WPP) * WPP;
#pragma unroll
      for (int i = 0; i < kMaxOut * 4; ++i) {
        if (i < 4 * m) {
          float s = 0.f;
          for (int w = 0; w < WPP; ++w) s += red[(w0 + w) * 40 + i];
          acc[i] = s;
        }
      }
      __syncthreads();
    }
    if (PK && u == 0 && a.out) {
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (pt0 + sl >= a.P) break;
#pragma unroll
        for (int i = 0; i < kMaxOut; ++i) {
          if (i >= m) break;
          a.out[(pt0 + sl) * m + i] = acc[i * 4 + sl];
        }
      }
    }
    if (!PK && valid && u == 0) {
#pragma unroll
      for (int i = 0; i < kMaxOut; ++i) {
        if (i >= m) break;
        if (a.out) a.out[pt * m + i] = acc[i * 4];
        if (a.tan) {
          a.tan[(pt * m + i) * 3 + 0] = acc[i * 4 + 1];
          a.tan[(pt * m + i) * 3 + 1] = acc[i * 4 + 2];
          a.tan[(pt * m + i) * 3 + 2] = acc[i * 4 + 3];
        }
      }
    }
    if constexpr (mode_fwd_only(MODE)) return;

    // ---------------- seeds -----------------------------------------------------------------
    float Wv[kMaxOut][3], Vv[kMaxOut];
#pragma unroll
    for (int i = 0; i < kMaxOut; ++i) { Vv[i] = 0.f; Wv[i][0] = Wv[i][1] = Wv[i][2] = 0.f; }
    if (MODE == kModeMaxwell || MODE == kModeTotal) {
      if (valid) {
        const float gEt = acc[1], gEx = acc[2], gEy = acc[3];
        const float gXt = acc[5], gXy = acc[7];
        const float gYt = acc[9], gYx = acc[10];
        float eps = 1.f, w1 = w_all;
        if (a.loss_kind != QP_LOSS_VACUUM) {
          const float x = a.points[pt * 3 + 1];
          const bool diel = x >= a.x_if;
          eps = diel ? a.eps_r : 1.f;
          if (a.loss_kind == QP_LOSS_DIEL_SPLIT) w1 = diel ? w_diel : w_vac;
        }
        const float ie = 1.f / eps;
        const float r1 = gEt - (gYx - gXy) * ie;
        const float r2 = gXt + gEy;
        const float r3 = gYt - gEx;
        const float w = w_all;
        lacc += (u == 0) ? (w1 * r1 * r1 + w * (r2 * r2 + r3 * r3)) : 0.f;
        const float A = 2.f * w1 * r1, Bq = 2.f * w * r2, C = 2.f * w * r3;
        Wv[0][0] = A;  Wv[2][1] = -A * ie;  Wv[1][2] = A * ie;
        Wv[1][0] = Bq; Wv[0][2] += Bq;
        Wv[2][0] = C;  Wv[0][1] += -C;
        if constexpr (MODE == kModeTotal) {
          // the energy term, mean square of the local Poynting residual e (eq. energy_loss), and
          // this point's share of the symmetry term (eq. 2D_symLoss) against its mirror images
          const float E = acc[0], Hx = acc[4], Hy = acc[8];
          const float e = eps * E * gEt + Hx * gXt + Hy * gYt - (gEx * Hy + E * gYx) + (gEy * Hx + E * gXy);
          const float k = a.w_energy * 2.f * e * w;
          Vv[0] += k * (eps * gEt - gYx + gXy);
          Vv[1] += k * (gXt + gEy);
          Vv[2] += k * (gYt - gEx);
          Wv[0][0] += k * eps * E; Wv[0][1] += -k * Hy; Wv[0][2] += k * Hx;
          Wv[1][0] += k * Hx;      Wv[1][2] += k * E;
          Wv[2][0] += k * Hy;      Wv[2][1] += -k * E;
          const float ks = a.w_sym * 2.f * w;
          for (int j = 0; j < a.n_mir; ++j) {   // parities: y-mirror (+, -, +), x-mirror (+, +, -)
            const float* fm = a.f_mir + ((long long)j * a.P + pt) * m;
            Vv[0] += ks * (E - fm[0]);
            Vv[1] += ks * (j == 0 ? Hx + fm[1] : Hx - fm[1]);
            Vv[2] += ks * (j == 0 ? Hy - fm[2] : Hy + fm[2]);
          }
        }
      }
    } else if (PK) {   // output seeds of the four slots' points: slot 0 in Vv, slot c + 1 in Wv[.][c]
      if (a.d_out) {
#pragma unroll
        for (int i = 0; i < kMaxOut; ++i) {
          if (i >= m) break;
          if (pt0 < a.P) Vv[i] = a.d_out[pt0 * m + i];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (pt0 + 1 + c < a.P) Wv[i][c] = a.d_out[(pt0 + 1 + c) * m + i];
        }
      }
    } else {   // VJP seeds
      if (valid) {
#pragma unroll
        for (int i = 0; i < kMaxOut; ++i) {
          if (i >= m) break;
          if (a.d_out) Vv[i] = a.d_out[pt * m + i];
          if (a.d_tan) {
            Wv[i][0] = a.d_tan[(pt * m + i) * 3 + 0];
            Wv[i][1] = a.d_tan[(pt * m + i) * 3 + 1];
            Wv[i][2] = a.d_tan[(pt * m + i) * 3 + 2];
          }
        }
      }
    }
    // lambda = Df psi + sum_c D_c dpsi_c, mu_c = D_c psi (D real diagonal in the final basis)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t j = jl ^ reg_off(r, l0, l1, l2);
      float Df = 0.f, D0 = 0.f, D1 = 0.f, D2 = 0.f;
#pragma unroll
      for (int i = 0; i < kMaxOut; ++i) {
        if (i < m) {
          const float z = parity(plan->zmask[i] & j) ? -1.f : 1.f;
          Df += z * Vv[i];
          D0 += z * Wv[i][0];
          D1 += z * Wv[i][1];
          D2 += z * Wv[i][2];
        }
      }
      if (PK) {   // lambda of each slot's point, paired with that slot's psi
        sr[4][r] = Df * sr[0][r]; si[4][r] = Df * si[0][r];
        sr[5][r] = D0 * sr[1][r]; si[5][r] = D0 * si[1][r];
        sr[6][r] = D1 * sr[2][r]; si[6][r] = D1 * si[2][r];
        sr[7][r] = D2 * sr[3][r]; si[7][r] = D2 * si[3][r];
      } else {
        sr[4][r] = Df * sr[0][r] + D0 * sr[1][r] + D1 * sr[2][r] + D2 * sr[3][r];
        si[4][r] = Df * si[0][r] + D0 * si[1][r] + D1 * si[2][r] + D2 * si[3][r];
        sr[5][r] = D0 * sr[0][r]; si[5][r] = D0 * si[0][r];
        sr[6][r] = D1 * sr[0][r]; si[6][r] = D1 * si[0][r];
        sr[7][r] = D2 * sr[0][r]; si[7][r] = D2 * si[0][r];
      }
    }
    // ---------------- adjoint sweep with uncompute -----------------------------------------
    // Per round in reverse: psi-family <- U^H (uncompute), lambda-family <- U^H, gate statistics,
    // then the inverse exchange.  The pair (psi_c, lambda_c) for c = 0..3 is a self-contained
    // group (its gates and its share of the statistics need no other statevector).
    if constexpr (EXS == 4) {
      // Software-pipelined over the four pair groups with plane pairs {0, 1} and {2, 3} in turn.
      // Each slot: read one pair group, add the previous group's gate statistics (covering the
      // read latency), write the next group, then pull the group just read back through the
      // round.  Writing after the statistics lets every wave's reads drain from the LDS queue
      // before the writes of the workgroup's waves compete with them.  A round's statistics are
      // flushed in the next round's first slot.
      // The last round is pulled back first, gate by gate (H < R: it is never a leading-stage round).
      CP<QRound> rl = rounds + (R - 1);
      round_adj_all<NS, true>(sr, si, rl, gtab, F, slots, wave, lane);
      if (R > 1) {
        Offs wo = load_offs(xb[R - 1].woff);
        // the current exchange's lane words as plain scalars (the loop body below is a lambda that
        // updates them; an aggregate captured by reference would not stay in registers)
        uint32_t xwb, xrb, xsg;
        {
          const XLane x0 = lane_words(lanes, 1, R, R - 1, TP, u, pb8);
          xwb = x0.wb; xrb = x0.rb; xsg = x0.sgn;
        }
        xwrite<T, 0, 4, 0>(sr, si, buf, wo, xwb);
        constexpr int NQ = 3 * (3 + NS);
        float q[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) q[i] = 0.f;
        RoundCoef Rq = load_round<true, NS>(rl, gtab, F);   // gate ids of the round whose q is pending
        // Iteration k moves the state from round k's input mapping to round k - 1's output mapping
        // and pulls round k - 1 back (PULL), or, for a round of the leading stage, only takes its
        // statistics.  Two loops instead of a branch inside one keep the register allocation of
        // the pulling loop unchanged.
        auto iter = [&](int k, auto pull) {
          constexpr bool PULL = decltype(pull)::value;
          CP<QRound> rp = rounds + (k - 1);
          const RoundCoef Rp = load_round<true, NS>(rp, gtab, F);
          const Offs ro = load_offs(xb[k].roff);
          const bool sg = xb[k].nterms != 0;
          __syncthreads();
          xread<T, 0, 4, 0, SG>(sr, si, buf, ro, sg, xrb, xsg);
          if (k < R - 1) {                             // finish the previous round's statistics
            stat_accum<3>(sr, si, q);
            round_stat_flush<NS>(Rq, slots, q, F, wave, lane);
#pragma unroll
            for (int i = 0; i < NQ; ++i) q[i] = 0.f;
          }
          xwrite<T, 1, 5, 2>(sr, si, buf, wo, xwb);
          round_adj<0, NS, PULL>(sr, si, Rp, q);
          pin_sv<0>(sr, si); pin_sv<4>(sr, si); pin_q<NQ>(q);
          __syncthreads();
          xread<T, 1, 5, 2, SG>(sr, si, buf, ro, sg, xrb, xsg);
          stat_accum<0>(sr, si, q);
          xwrite<T, 2, 6, 0>(sr, si, buf, wo, xwb);
          round_adj<1, NS, PULL>(sr, si, Rp, q);
          pin_sv<1>(sr, si); pin_sv<5>(sr, si); pin_q<NQ>(q);
          __syncthreads();
          xread<T, 2, 6, 0, SG>(sr, si, buf, ro, sg, xrb, xsg);
          stat_accum<1>(sr, si, q);
          xwrite<T, 3, 7, 2>(sr, si, buf, wo, xwb);
          round_adj<2, NS, PULL>(sr, si, Rp, q);
          pin_sv<2>(sr, si); pin_sv<6>(sr, si); pin_q<NQ>(q);
          // the next exchange's write offsets (scalar, before the barrier as in the forward sweep)
          if (k > 1) wo = load_offs(xb[k - 1].woff);
          __syncthreads();
          xread<T, 3, 7, 2, SG>(sr, si, buf, ro, sg, xrb, xsg);
          // and its lane words: a vector load (its own wait counter), covered by the statistics
          XLane xn{xwb, xrb, xsg};
          if (k > 1) xn = lane_words(lanes, 1, R, k - 1, TP, u, pb8);
          stat_accum<2>(sr, si, q);
          if (k > 1) xwrite<T, 0, 4, 0>(sr, si, buf, wo, xn.wb);
          round_adj<3, NS, PULL>(sr, si, Rp, q);
          pin_sv<3>(sr, si); pin_sv<7>(sr, si); pin_q<NQ>(q);
          xwb = xn.wb; xrb = xn.rb; xsg = xn.sgn;
          Rq = Rp;
        };
        for (int k = R - 1; k > H; --k) iter(k, BoolC<true>{});
        for (int k = H; k >= 1; --k) iter(k, BoolC<false>{});
        stat_accum<3>(sr, si, q);                      // round 0's last group
        round_stat_flush<NS>(Rq, slots, q, F, wave, lane);
        __syncthreads();
      }
    } else {
      for (int k = R - 1; k >= H; --k) {
        CP<QRound> rk = rounds + k;
        round_adj_all<NS, true>(sr, si, rk, gtab, F, slots, wave, lane);
        if (PH && rk->phase >= 0) {   // CRZ phase stage: moments at its output, then uncompute and pull back
          CP<QPhaseStage> pst = to_const(pstages) + rk->phase;
          phase_moments<N>(sr, si, rk, u, mslots + wave * a.n_mom + pst->mom_off, lane);
          float pc[8], ps[8];
          phase_factors<N>(rk, pcoef + pst->coef_off, u, pc, ps);
          apply_phase<0, 8, true>(sr, si, pc, ps);
        }
        if (k > 0) exchange<N, T, 8, 2>(sr, si, buf, xb + k, lane_words(lanes, 1, R, k, TP, u, pb8));
      }
      for (int k = H - 1; k >= 0; --k) {   // the leading stage: statistics only
        CP<QRound> rk = rounds + k;
        round_adj_all<NS, false>(sr, si, rk, gtab, F, slots, wave, lane);
        if (k > 0) exchange<N, T, 8, 2>(sr, si, buf, xb + k, lane_words(lanes, 1, R, k, TP, u, pb8));
      }
    }
    if constexpr (EG) {
      // the point index again, from an opaque copy of the thread index: keeping pt and valid live
      // through the adjoint sweep would cost registers there
      uint32_t t2 = threadIdx.x;
      asm volatile("" : "+v"(t2));
      const long long pt2 = PK ? 0 : (long long)tile * PPW + (long long)(t2 / TP);
      encoding_grads<N, T>(sr, si, buf, red, plan, rounds, gtab, a, pt2, pt2 < a.P, u);
    }
  }
}

// ---- the fused kernel: a persistent grid walks the tiles ------------------------------------
template <int N, int T, int EXS, int MODE, bool SG, bool EG = false>
__global__ __launch_bounds__(T, 2) void k_fused(FusedArgs a) {
  constexpr int WAVES = T / 64;
  constexpr int PLANE = T * 8;
  // Exchange planes in static LDS (their address is a link-time constant, so every access is
  // one XOR of a byte offset); gate statistics and readout scratch in the dynamic part.
  __shared__ float4 planes[EXS * PLANE / 2];
  extern __shared__ float4 smem4[];
  float2* buf = reinterpret_cast<float2*>(planes);
  float* slots = reinterpret_cast<float*>(smem4);                   // [WAVES][F][kGS]
  float* mslots = slots + WAVES * a.n_fused * kGS;                   // [WAVES][n_mom] phase moments
  float* red = mslots + WAVES * a.n_mom;                             // [WAVES][40]
  const int F = a.n_fused;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  if (!mode_fwd_only(MODE)) {
    for (int i = tid; i < WAVES * (F * kGS + a.n_mom); i += T) slots[i] = 0.f;
  }
  __syncthreads();
  float lacc = 0.f;
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs (blockIdx % 8), so each
  // XCD walks one contiguous range of tiles and neighbouring points' output lines are written
  // through one L2 instead of eight.
  constexpr int kXcd = 8;
  int t_begin = blockIdx.x, t_end = a.ntiles, t_step = gridDim.x;
  if (gridDim.x % kXcd == 0) {
    const int chunk = (a.ntiles + kXcd - 1) / kXcd;
    t_begin = (blockIdx.x % kXcd) * chunk + blockIdx.x / kXcd;
    t_end = min(a.ntiles, (int)(blockIdx.x % kXcd) * chunk + chunk);
    t_step = gridDim.x / kXcd;
  }
  for (int tile = t_begin; tile < t_end; tile += t_step)
    fused_tile<N, T, EXS, MODE, SG, EG>(a, tile, buf, slots, mslots, red, lacc);
  if (mode_fwd_only(MODE)) return;
  // ---------------- per-workgroup partials (fixed order) -----------------------------------
  __syncthreads();
  const int ncol = F * kGS + a.n_mom;
  for (int i = tid; i < F * kGS; i += T) {
    float s = 0.f;
    for (int w = 0; w < WAVES; ++w) s += slots[w * F * kGS + i];
    a.mpart[(long long)blockIdx.x * ncol + i] = s;
  }
  for (int i = tid; i < a.n_mom; i += T) {
    float s = 0.f;
    for (int w = 0; w < WAVES; ++w) s += mslots[w * a.n_mom + i];
    a.mpart[(long long)blockIdx.x * ncol + F * kGS + i] = s;
  }
  if (MODE == kModeMaxwell) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) lacc += __shfl_xor(lacc, off);
    __syncthreads();
    if (lane == 0) red[wave * 40] = lacc;
    __syncthreads();
    if (tid == 0) {
      float s = 0.f;
      for (int w = 0; w < WAVES; ++w) s += red[w * 40];
      a.lpart[blockIdx.x] = s;
    }
  }
}


template <int N, int EXS, int MODE, bool SG, bool EG = false>
hipError_t launch_one(const FusedArgs& a, int grid, size_t lds, hipStream_t st) {
  constexpr int T = fused_wg_threads(N);
  auto kern = k_fused<N, T, EXS, MODE, SG, EG>;
  // lds counts the static exchange planes and the dynamic part; only the latter is passed.
  const size_t planes = (size_t)EXS * T * 8 * sizeof(float2);
  const size_t dyn = lds > planes ? lds - planes : 0;
  // the attribute is set once per device (and raised when a larger size comes)
  static size_t attr_bytes[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (dyn > 0 && dyn > attr_bytes[dev]) {
    e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    attr_bytes[dev] = dyn;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(T), dyn, st, a);
  return hipGetLastError();
}

// Entry point of one per-N unit.  signs: some exchange of the circuit carries CZ signs (the
// pipelined kernel has a variant without the sign code for circuits that have none).
template <int N>
hipError_t launch_fused_n(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st) {
  if ((mode == kModeMaxwell || mode == kModeVjp) && (a.d_angles || a.d_jac)) {   // per-point input gradients
    if (mode == kModeMaxwell)
      return exs == 2 ? launch_one<N, 2, kModeMaxwell, true, true>(a, grid, lds, st)
                      : launch_one<N, 4, kModeMaxwell, true, true>(a, grid, lds, st);
    return exs == 2 ? launch_one<N, 2, kModeVjp, true, true>(a, grid, lds, st)
                    : launch_one<N, 4, kModeVjp, true, true>(a, grid, lds, st);
  }
  if (mode == kModeFwd) {
    if (exs == 2) return launch_one<N, 2, kModeFwd, true>(a, grid, lds, st);
    return signs ? launch_one<N, 4, kModeFwd, true>(a, grid, lds, st) : launch_one<N, 4, kModeFwd, false>(a, grid, lds, st);
  }
  if (mode == kModeTotal) {
    if (exs == 2) return launch_one<N, 2, kModeTotal, true>(a, grid, lds, st);
    return signs ? launch_one<N, 4, kModeTotal, true>(a, grid, lds, st)
                 : launch_one<N, 4, kModeTotal, false>(a, grid, lds, st);
  }
  if (mode == kModeMaxwell) {
    if (exs == 2) return launch_one<N, 2, kModeMaxwell, true>(a, grid, lds, st);
    return signs ? launch_one<N, 4, kModeMaxwell, true>(a, grid, lds, st)
                 : launch_one<N, 4, kModeMaxwell, false>(a, grid, lds, st);
  }
  if (mode == kModeFwdPk) {
    if (exs == 2) return launch_one<N, 2, kModeFwdPk, true>(a, grid, lds, st);
    return signs ? launch_one<N, 4, kModeFwdPk, true>(a, grid, lds, st)
                 : launch_one<N, 4, kModeFwdPk, false>(a, grid, lds, st);
  }
  if (mode == kModeVjpPk) {
    if (exs == 2) return launch_one<N, 2, kModeVjpPk, true>(a, grid, lds, st);
    return signs ? launch_one<N, 4, kModeVjpPk, true>(a, grid, lds, st)
                 : launch_one<N, 4, kModeVjpPk, false>(a, grid, lds, st);
  }
  if (exs == 2) return launch_one<N, 2, kModeVjp, true>(a, grid, lds, st);
  return signs ? launch_one<N, 4, kModeVjp, true>(a, grid, lds, st) : launch_one<N, 4, kModeVjp, false>(a, grid, lds, st);
}

}  // namespace qp
