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

// LDS index swizzle: XOR the low nibble with the fold of all higher nibbles (a bijection).
__device__ __forceinline__ uint32_t swz(uint32_t idx) {
  uint32_t h = idx >> 4;
  h ^= h >> 4;
  h ^= h >> 8;
  return idx ^ (h & 15u);
}

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
// u: u00r,u00i,u01r,u01i,u10r,u10i,u11r,u11i
template <int B, int S0, int NS>
__device__ __forceinline__ void apply_gate(float (&sr)[8][8], float (&si)[8][8], const float* u) {
  const float a0r = u[0], a0i = u[1], a1r = u[2], a1i = u[3];
  const float b0r = u[4], b0i = u[5], b1r = u[6], b1i = u[7];
#pragma unroll
  for (int s = S0; s < S0 + NS; ++s) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r & (1 << B)) continue;
      const int r1 = r | (1 << B);
      const float xr = sr[s][r], xi = si[s][r], yr = sr[s][r1], yi = si[s][r1];
      sr[s][r] = a0r * xr - a0i * xi + a1r * yr - a1i * yi;
      si[s][r] = a0r * xi + a0i * xr + a1r * yi + a1i * yr;
      sr[s][r1] = b0r * xr - b0i * xi + b1r * yr - b1i * yi;
      si[s][r1] = b0r * xi + b0i * xr + b1r * yi + b1i * yr;
    }
  }
}

// conj-transpose of a gate table entry
__device__ __forceinline__ void dagger(const float* u, float* d) {
  d[0] = u[0]; d[1] = -u[1];   // (0,0) <- conj u00
  d[2] = u[4]; d[3] = -u[5];   // (0,1) <- conj u10
  d[4] = u[2]; d[5] = -u[3];   // (1,0) <- conj u01
  d[6] = u[6]; d[7] = -u[7];   // (1,1) <- conj u11
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
// Writes statevectors [0, NSV) in the writer mapping `wr`, reads them back in mapping `rd`
// through the exchange descriptor X (index map and sign), in groups of EXS planes.
// jc: on entry the thread part of the state index in mapping `wr` (deposit of u), on exit the
// same in mapping `rd`, so consecutive exchanges deposit the thread bits once each.
// Address arithmetic: pbase is a multiple of 2^N and every index below 2^N, so pbase + x equals
// pbase ^ x; swz is linear over GF(2), so swz(pbase ^ j ^ o) = swz(pbase ^ j) ^ swz(o).  The
// register offsets o are uniform across the workgroup, leaving one per-lane XOR per access.
template <int N, int T, int NSV, int EXS>
__device__ __forceinline__ void exchange(float (&sr)[8][8], float (&si)[8][8], float2* __restrict__ buf,
                                         CP<QRound> wr, CP<QRound> rd, CP<QXchg> X, uint32_t u, uint32_t pbase,
                                         uint32_t& jc) {
  constexpr int PLANE = T * 8;
  const uint32_t jw = jc;
  const uint32_t w0 = wr->tpos[0], w1 = wr->tpos[1], w2 = wr->tpos[2];
  const uint32_t jn = deposit_thread<N>(u, rd->tpos);
  jc = jn;
  uint32_t sb;
  uint32_t sgn = 0;   // bit r set: negate amplitude r
  if (X->identity) {
    sb = jn;
  } else {
    // sb = A jn with jn = sum of the thread bits placed at rd->tpos[k]: column A e_tpos[k] is
    // acol[tpos[k]], so only the N - 3 thread bits are visited.
    sb = 0;
#pragma unroll
    for (int k = 3; k < N; ++k) {
      const uint32_t msk = 0u - ((u >> (k - 3)) & 1u);
      sb ^= msk & X->acol[rd->tpos[k]];
    }
    const int nt = X->nterms;
    if (nt > 0) {
      const uint32_t xb = X->sign_at_src ? sb : jn;
      uint32_t pu = 0, pv = 0;
      for (int t = 0; t < nt; ++t) {
        pu |= parity(X->qu[t] & xb) << t;
        pv |= parity(X->qv[t] & xb) << t;
      }
      const uint32_t q0 = parity(pu & pv);
      const uint32_t b0 = parity((pu & X->ve[0]) ^ (X->ue[0] & pv));
      const uint32_t b1 = parity((pu & X->ve[1]) ^ (X->ue[1] & pv));
      const uint32_t b2 = parity((pu & X->ve[2]) ^ (X->ue[2] & pv));
      const uint32_t qs = X->qsign_r;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        uint32_t s = q0 ^ ((qs >> r) & 1u);
        if (r & 1) s ^= b0;
        if (r & 2) s ^= b1;
        if (r & 4) s ^= b2;
        sgn |= s << r;
      }
    }
  }
  const uint32_t wb = swz(pbase ^ jw), rb = swz(pbase ^ sb);
  uint32_t wo[8], ro[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    wo[r] = swz(reg_off(r, w0, w1, w2));
    ro[r] = swz(X->identity ? reg_off(r, rd->tpos[0], rd->tpos[1], rd->tpos[2]) : X->src_r[r]);
  }
#pragma unroll
  for (int g = 0; g < NSV; g += EXS) {
#pragma unroll
    for (int s = 0; s < EXS; ++s)
#pragma unroll
      for (int r = 0; r < 8; ++r)
        buf[s * PLANE + (wb ^ wo[r])] = make_float2(sr[g + s][r], si[g + s][r]);
    __syncthreads();
    if (sgn == 0u) {   // uniform when the stage has no sign terms (e.g. a CNOT ring)
#pragma unroll
      for (int s = 0; s < EXS; ++s)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const float2 v = buf[s * PLANE + (rb ^ ro[r])];
          sr[g + s][r] = v.x;
          si[g + s][r] = v.y;
        }
    } else {
#pragma unroll
      for (int s = 0; s < EXS; ++s)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const float2 v = buf[s * PLANE + (rb ^ ro[r])];
          const uint32_t flip = ((sgn >> r) & 1u) << 31;   // negate by flipping the sign bits
          sr[g + s][r] = __uint_as_float(__float_as_uint(v.x) ^ flip);
          si[g + s][r] = __uint_as_float(__float_as_uint(v.y) ^ flip);
        }
    }
    __syncthreads();
  }
}

// ---- one tile of PPW points: forward, readout, seeds, adjoint --------------------------------
// buf: EXS exchange planes; slots: per-wave gate statistics [WAVES][F][kGS]; red: [WAVES][40].
template <int N, int T, int EXS, int MODE>
__device__ __forceinline__ void fused_tile(const FusedArgs& a, int tile, float2* __restrict__ buf,
                                           float* __restrict__ slots, float* __restrict__ red, float& lacc) {
  constexpr int TP = 1 << (N - 3);         // threads per point
  constexpr int PPW = T / TP;              // points per workgroup tile
  constexpr int DIM = 1 << N;
  static_assert(PPW >= 1, "tile too small");
  CP<QPlanDev> plan = to_const(a.plan);
  CP<char> pb = reinterpret_cast<CP<char>>(plan);
  CP<QRound> rounds = reinterpret_cast<CP<QRound>>(pb + plan->off_rounds);
  CP<QXchg> xf = reinterpret_cast<CP<QXchg>>(pb + plan->off_xf);
  CP<QXchg> xb = reinterpret_cast<CP<QXchg>>(pb + plan->off_xb);
  CP<float> gtab = to_const(a.gtab);
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
  if (MODE == kModeMaxwell && !a.loss_sum) {
    w_all = a.P > 0 ? 1.f / (float)a.P : 0.f;
    if (a.loss_kind == QP_LOSS_DIEL_SPLIT) {
      const int nv = a.counts[0], nd = a.counts[1];
      w_vac = nv > 0 ? 1.f / (float)nv : 0.f;
      w_diel = nd > 0 ? 1.f / (float)nd : 0.f;
    }
  }
  float sr[8][8], si[8][8];
  {
    const long long pt = (long long)tile * PPW + ps;
    const bool valid = pt < a.P;

    // ---------------- encoding: per-qubit embedded amplitudes and derivatives -------------
    float e0r[N], e1r[N], e1i[N], d0r[N], d1r[N], d1i[N], jq[N][3];
    {
      float p3[3] = {0.f, 0.f, 0.f};
      if (valid && a.points && plan->enc_kind != QP_ENC_ANGLES) {
        p3[0] = a.points[pt * 3 + 0];
        p3[1] = a.points[pt * 3 + 1];
        p3[2] = a.points[pt * 3 + 2];
      }
#pragma unroll
      for (int q = 0; q < N; ++q) {
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
        } else {
          float th = 0.f;
          if (valid) {
            th = a.angles[pt * N + q];
            j0 = a.jac[(pt * N + q) * 3 + 0];
            j1 = a.jac[(pt * N + q) * 3 + 1];
            j2 = a.jac[(pt * N + q) * 3 + 2];
          }
          sincosf(0.5f * th, &s, &c);
        }
        e0r[q] = c;
        d0r[q] = -0.5f * s;
        if (plan->enc_gate == QP_ENC_RY) {
          e1r[q] = s; e1i[q] = 0.f; d1r[q] = 0.5f * c; d1i[q] = 0.f;
        } else {   // RX|0> = (cos, -i sin)
          e1r[q] = 0.f; e1i[q] = -s; d1r[q] = 0.f; d1i[q] = -0.5f * c;
        }
        jq[q][0] = j0; jq[q][1] = j1; jq[q][2] = j2;
      }
    }
    // ---------------- product state and tangent seeds in round 0's mapping ---------------
    {
      CP<QRound> r0 = rounds;
      // thread part: (P, D_c) by the product rule over the thread qubits
      float Pr = valid ? 1.f : 0.f, Pi = 0.f;
      float Dr[3] = {0.f, 0.f, 0.f}, Di[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 3; k < N; ++k) {
        const int q = N - 1 - r0->tpos[k];
        const bool bit = (u >> (k - 3)) & 1u;
        float er = 0.f, ei = 0.f, dr = 0.f, di = 0.f, jj[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int qq = 0; qq < N; ++qq)
          if (qq == q) {
            er = bit ? e1r[qq] : e0r[qq];
            ei = bit ? e1i[qq] : 0.f;
            dr = bit ? d1r[qq] : d0r[qq];
            di = bit ? d1i[qq] : 0.f;
            jj[0] = jq[qq][0]; jj[1] = jq[qq][1]; jj[2] = jq[qq][2];
          }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float nr = Dr[c] * er - Di[c] * ei + jj[c] * (Pr * dr - Pi * di);
          const float ni = Dr[c] * ei + Di[c] * er + jj[c] * (Pr * di + Pi * dr);
          Dr[c] = nr; Di[c] = ni;
        }
        const float npr = Pr * er - Pi * ei, npi = Pr * ei + Pi * er;
        Pr = npr; Pi = npi;
      }
      float qer[3][2], qei[3][2], qdr[3][2], qdi[3][2], qj[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int q = N - 1 - r0->tpos[i];
#pragma unroll
        for (int qq = 0; qq < N; ++qq)
          if (qq == q) {
            qer[i][0] = e0r[qq]; qei[i][0] = 0.f; qer[i][1] = e1r[qq]; qei[i][1] = e1i[qq];
            qdr[i][0] = d0r[qq]; qdi[i][0] = 0.f; qdr[i][1] = d1r[qq]; qdi[i][1] = d1i[qq];
            qj[i][0] = jq[qq][0]; qj[i][1] = jq[qq][1]; qj[i][2] = jq[qq][2];
          }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float pr = Pr, pi = Pi, dr[3] = {Dr[0], Dr[1], Dr[2]}, di[3] = {Di[0], Di[1], Di[2]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int b = (r >> i) & 1;
          const float er = qer[i][b], ei = qei[i][b], ddr = qdr[i][b], ddi = qdi[i][b];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float nr = dr[c] * er - di[c] * ei + qj[i][c] * (pr * ddr - pi * ddi);
            const float ni = dr[c] * ei + di[c] * er + qj[i][c] * (pr * ddi + pi * ddr);
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
    uint32_t jc = deposit_thread<N>(u, rounds[0].tpos);   // thread bits in the current mapping
    for (int k = 0; k < R; ++k) {
      CP<QRound> rk = rounds + k;
      if (k > 0) exchange<N, T, 4, (EXS < 4 ? EXS : 4)>(sr, si, buf, rk - 1, rk, xf + k, u, pbase, jc);
      // branch-free: an absent gate is the identity entry F of the gate table
      float g[8];
      const int g0 = rk->gate[0] >= 0 ? rk->gate[0] : F;
      const int g1 = rk->gate[1] >= 0 ? rk->gate[1] : F;
      const int g2 = rk->gate[2] >= 0 ? rk->gate[2] : F;
#pragma unroll
      for (int e = 0; e < 8; ++e) g[e] = gtab[g0 * 8 + e];
      apply_gate<0, 0, 4>(sr, si, g);
#pragma unroll
      for (int e = 0; e < 8; ++e) g[e] = gtab[g1 * 8 + e];
      apply_gate<1, 0, 4>(sr, si, g);
#pragma unroll
      for (int e = 0; e < 8; ++e) g[e] = gtab[g2 * 8 + e];
      apply_gate<2, 0, 4>(sr, si, g);
    }
    // ---------------- readout ----------------------------------------------------------------
    CP<QRound> rl = rounds + (R - 1);
    const uint32_t jl = jc;
    const uint32_t l0 = rl->tpos[0], l1 = rl->tpos[1], l2 = rl->tpos[2];
    float acc[kMaxOut * 4];
#pragma unroll
    for (int i = 0; i < kMaxOut * 4; ++i) acc[i] = 0.f;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t j = jl ^ reg_off(r, l0, l1, l2);
      const float p2 = sr[0][r] * sr[0][r] + si[0][r] * si[0][r];
      float gc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) gc[c] = 2.f * (sr[0][r] * sr[1 + c][r] + si[0][r] * si[1 + c][r]);
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
    if (valid && u == 0) {
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
    if (MODE == kModeFwd) return;

    // ---------------- seeds -----------------------------------------------------------------
    float Wv[kMaxOut][3], Vv[kMaxOut];
#pragma unroll
    for (int i = 0; i < kMaxOut; ++i) { Vv[i] = 0.f; Wv[i][0] = Wv[i][1] = Wv[i][2] = 0.f; }
    if (MODE == kModeMaxwell) {
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
      sr[4][r] = Df * sr[0][r] + D0 * sr[1][r] + D1 * sr[2][r] + D2 * sr[3][r];
      si[4][r] = Df * si[0][r] + D0 * si[1][r] + D1 * si[2][r] + D2 * si[3][r];
      sr[5][r] = D0 * sr[0][r]; si[5][r] = D0 * si[0][r];
      sr[6][r] = D1 * sr[0][r]; si[6][r] = D1 * si[0][r];
      sr[7][r] = D2 * sr[0][r]; si[7][r] = D2 * si[0][r];
    }
    // ---------------- adjoint sweep with uncompute -----------------------------------------
    for (int k = R - 1; k >= 0; --k) {
      CP<QRound> rk = rounds + k;
#pragma unroll
      for (int bb = 2; bb >= 0; --bb) {
        const int gsrc = rk->gate[bb];
        const int gid = gsrc >= 0 ? gsrc : F;   // identity entry: straight-line code, no branch
        float g[8], d[8], q[6];
#pragma unroll
        for (int e = 0; e < 8; ++e) g[e] = gtab[gid * 8 + e];
#pragma unroll
        for (int e = 0; e < 6; ++e) q[e] = 0.f;
        dagger(g, d);
        if (bb == 0) { apply_gate<0, 0, 8>(sr, si, d); accum_s<0>(sr, si, q); }
        if (bb == 1) { apply_gate<1, 0, 8>(sr, si, d); accum_s<1>(sr, si, q); }
        if (bb == 2) { apply_gate<2, 0, 8>(sr, si, d); accum_s<2>(sr, si, q); }
        const float v4[4] = {q[0] + q[3], q[1] + q[4], q[2] + q[5], 0.f};
        const float v = wave_reduce_scatter4(v4);
        if (gsrc >= 0 && (lane & 15) == 0 && lane < 48)
          slots[(wave * F + gsrc) * kGS + (lane >> 4)] += v;
      }
      if (k > 0) exchange<N, T, 8, EXS>(sr, si, buf, rk, rk - 1, xb + k, u, pbase, jc);
    }
  }
}

// ---- the fused kernel: a persistent grid walks the tiles ------------------------------------
template <int N, int T, int EXS, int MODE>
__global__ __launch_bounds__(T, 2) void k_fused(FusedArgs a) {
  constexpr int WAVES = T / 64;
  constexpr int PLANE = T * 8;
  extern __shared__ float4 smem4[];
  float2* buf = reinterpret_cast<float2*>(smem4);
  float* slots = reinterpret_cast<float*>(buf + EXS * PLANE);      // [WAVES][F][kGS]
  float* red = slots + WAVES * a.n_fused * kGS;                      // [WAVES][40]
  const int F = a.n_fused;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  if (MODE != kModeFwd) {
    for (int i = tid; i < WAVES * F * kGS; i += T) slots[i] = 0.f;
  }
  __syncthreads();
  float lacc = 0.f;
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs (blockIdx % 8), so each
  // XCD walks one contiguous range of tiles and neighbouring points' output lines are written
  // through one L2 instead of eight.
  constexpr int kXcd = 8;
  if (gridDim.x % kXcd == 0) {
    const int per = gridDim.x / kXcd;
    const int chunk = (a.ntiles + kXcd - 1) / kXcd;
    const int t0 = (blockIdx.x % kXcd) * chunk;
    const int t1 = min(a.ntiles, t0 + chunk);
    for (int tile = t0 + blockIdx.x / kXcd; tile < t1; tile += per)
      fused_tile<N, T, EXS, MODE>(a, tile, buf, slots, red, lacc);
  } else {
    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x)
      fused_tile<N, T, EXS, MODE>(a, tile, buf, slots, red, lacc);
  }
  if (MODE == kModeFwd) return;
  // ---------------- per-workgroup partials (fixed order) -----------------------------------
  __syncthreads();
  for (int i = tid; i < F * kGS; i += T) {
    float s = 0.f;
    for (int w = 0; w < WAVES; ++w) s += slots[w * F * kGS + i];
    a.mpart[(long long)blockIdx.x * F * kGS + i] = s;
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


template <int N, int EXS, int MODE>
hipError_t launch_one(const FusedArgs& a, int grid, size_t lds, hipStream_t st) {
  constexpr int T = (N == 12) ? 512 : 256;
  auto kern = k_fused<N, T, EXS, MODE>;
  static size_t attr_bytes = 0;
  if (lds > 64 * 1024 && lds > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_bytes = lds;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(T), lds, st, a);
  return hipGetLastError();
}

// Entry point of one per-N unit.
template <int N>
hipError_t launch_fused_n(int mode, const FusedArgs& a, int grid, int exs, size_t lds, hipStream_t st) {
  if (mode == kModeFwd) return exs == 2 ? launch_one<N, 2, kModeFwd>(a, grid, lds, st) : launch_one<N, 4, kModeFwd>(a, grid, lds, st);
  if (mode == kModeMaxwell) return exs == 2 ? launch_one<N, 2, kModeMaxwell>(a, grid, lds, st) : launch_one<N, 4, kModeMaxwell>(a, grid, lds, st);
  return exs == 2 ? launch_one<N, 2, kModeVjp>(a, grid, lds, st) : launch_one<N, 4, kModeVjp>(a, grid, lds, st);
}

}  // namespace qp
