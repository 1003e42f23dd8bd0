// Dense 2^5-blocks on FP32 MFMA (streamed, amplitude-major).
//
// The planner cuts the gate list (rotations delayed to their next entangler) into contiguous
// runs acting on at most five qubits.  Each run is one 32x32 complex block B_g, built in FP64 and
// rounded once to FP32, and applied to all statevectors of a point chunk as a GEMM
//     [64 x 64 real] x [64 x (2^(n-5) * points)]            (complex as interleaved re/im rows)
// with v_mfma_f32_32x32x2f32: A = the block (held in registers per lane), B = 32 consecutive
// points of one (statevector, other-index) column group, loaded straight from HBM (coalesced:
// the points are the contiguous dimension of the [S][2^n][points] layout).  The adjoint applies
// B_g^H (the transposed real form) to uncompute psi and pull back lambda, and accumulates
// M_g = sum_columns conj(Lambda) Psi^T with another MFMA GEMM staged through LDS; the parameter
// gradient is 2 Re sum_ab (dB_g/dtheta)_ab M_g,ab, formed in FP64.
//
// MFMA operand layout (v_mfma_f32_32x32x2f32, checked on the device): A[m][k] in lane m + 32k,
// B[k][n] in lane n + 32k, C[m][n] in lane n + 32*((m/4)%2), register 4*(m/8) + m%4.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dense.hpp"
#include "rot_dev.hpp"

namespace qp {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ const QDenseGroup* dgroup(const QPlanDev* p, int g) {
  return reinterpret_cast<const QDenseGroup*>(reinterpret_cast<const char*>(p) + p->off_dgroups) + g;
}
__device__ __forceinline__ const QDenseGate* dgate(const QPlanDev* p, int i) {
  return reinterpret_cast<const QDenseGate*>(reinterpret_cast<const char*>(p) + p->off_dgates) + i;
}

// Evolve the 5-qubit column vector v (FP64) through gate G; with deriv, the gate is replaced by
// its parameter derivative.
__device__ void dense_gate_apply(const QDenseGate& G, const float* params, double* vr, double* vi, bool deriv) {
  if (G.kind <= QP_RZ) {
    double s, c;
    sincos(0.5 * (double)params[G.param], &s, &c);
    double u[8];
    set_identity(u);
    left_mul_rot<double>(G.kind, c, s, u);
    if (deriv) left_mul_mhalf_i_pauli<double>(G.kind, u);
    const int b = G.lq0;
    for (int a = 0; a < 32; ++a) {
      if (a & (1 << b)) continue;
      const int a1 = a | (1 << b);
      const double xr = vr[a], xi = vi[a], yr = vr[a1], yi = vi[a1];
      vr[a] = u[0] * xr - u[1] * xi + u[2] * yr - u[3] * yi;
      vi[a] = u[0] * xi + u[1] * xr + u[2] * yi + u[3] * yr;
      vr[a1] = u[4] * xr - u[5] * xi + u[6] * yr - u[7] * yi;
      vi[a1] = u[4] * xi + u[5] * xr + u[6] * yi + u[7] * yr;
    }
  } else if (G.kind == QP_CNOT) {
    const int c = G.lq0, t = G.lq1;
    for (int a = 0; a < 32; ++a) {
      if (!(a & (1 << c)) || (a & (1 << t))) continue;
      const int a1 = a | (1 << t);
      double tr = vr[a], ti = vi[a];
      vr[a] = vr[a1]; vi[a] = vi[a1];
      vr[a1] = tr; vi[a1] = ti;
    }
  } else if (G.kind == QP_CZ) {
    for (int a = 0; a < 32; ++a)
      if ((a & (1 << G.lq0)) && (a & (1 << G.lq1))) { vr[a] = -vr[a]; vi[a] = -vi[a]; }
  } else {   // CRZ: phase exp(-i theta/2) (target 0) or exp(+i theta/2) (target 1) where the control is set
    double s, c;
    sincos(0.5 * (double)params[G.param], &s, &c);
    for (int a = 0; a < 32; ++a) {
      if (!(a & (1 << G.lq0))) {
        if (deriv) { vr[a] = 0.0; vi[a] = 0.0; }
        continue;
      }
      const bool one = a & (1 << G.lq1);
      double pr, pi;
      if (!deriv) { pr = c; pi = one ? s : -s; }
      else { pr = -0.5 * s; pi = one ? 0.5 * c : -0.5 * c; }   // d/dtheta of exp(-+ i theta/2)
      const double xr = vr[a], xi = vi[a];
      vr[a] = pr * xr - pi * xi;
      vi[a] = pr * xi + pi * xr;
    }
  }
}

// One thread per block column r: B_g e_r in FP64, written as MFMA A-operands of the real form
// (forward) and of its transpose (adjoint).  tab layout [g][T=2][i=32][lane=64].
__global__ void k_dense_tables(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                               float* __restrict__ tabF, float* __restrict__ tabA) {
  const int g = blockIdx.x, r = threadIdx.x;
  if (r >= 32) return;
  const QDenseGroup* G = dgroup(plan, g);
  double vr[32], vi[32];
  for (int a = 0; a < 32; ++a) { vr[a] = (a == r) ? 1.0 : 0.0; vi[a] = 0.0; }
  for (int k = 0; k < G->ngates; ++k) dense_gate_apply(*dgate(plan, G->gate0 + k), params, vr, vi, false);
  float* tf = tabF + (size_t)g * 4096;
  float* ta = tabA + (size_t)g * 4096;
  // real form: Bre[2a'+0][2r+0] = Br, Bre[2a'+1][2r+0] = Bi, Bre[2a'+0][2r+1] = -Bi, Bre[2a'+1][2r+1] = Br
  for (int m = 0; m < 64; ++m) {
    const int ap = m >> 1, tp = m & 1;
    for (int t = 0; t < 2; ++t) {
      const double v = tp == 0 ? (t == 0 ? vr[ap] : -vi[ap]) : (t == 0 ? vi[ap] : vr[ap]);
      // forward A[m][k = 2r + t]: row tile m/32, k-step r, lane (m%32) + 32 t
      tf[((m >> 5) * 32 + r) * 64 + (m & 31) + 32 * t] = (float)v;
      // adjoint A'[M = 2r + t][K = m] = Bre[m][2r + t]: row tile M/32, k-step m/2, lane (M%32) + 32 (m%2)
      const int M = 2 * r + t;
      ta[((M >> 5) * 32 + (m >> 1)) * 64 + (M & 31) + 32 * (m & 1)] = (float)v;
    }
  }
}

// Per point: cos, sin of half the embedding angle and d theta / d(t, x, y) for every qubit.
__global__ void k_dense_encode(const QPlanDev* __restrict__ plan, const float* __restrict__ points,
                               const float* __restrict__ angles, const float* __restrict__ jac, long long P0,
                               int Pc, int Pv, float* __restrict__ enc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pc) return;
  const int n = plan->n;
  const long long pt = P0 + p;
  for (int q = 0; q < n; ++q) {
    float c = 1.f, s = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
    if (p < Pv) {
      if (plan->enc_kind == QP_ENC_CYCLE) {
        const int cc = plan->coord_of_qubit[q];
        const float x = points[pt * 3 + cc];
        float jv;
        const int sc = plan->enc_scale;
        if (sc == QP_SCALE_PI) { sincospif(0.5f * x, &s, &c); jv = 3.14159265358979323846f; }
        else if (sc == QP_SCALE_BIAS) { sincospif(0.25f * (x + 1.f), &s, &c); jv = 1.57079632679489661923f; }
        else if (sc == QP_SCALE_NONE) { sincosf(0.5f * x, &s, &c); jv = 1.f; }
        else {
          const float xx = fminf(fmaxf(x, -1.f), 1.f);
          const float th = (sc == QP_SCALE_ASIN) ? asinf(xx) + 1.57079632679489661923f : acosf(xx);
          sincosf(0.5f * th, &s, &c);
          const float rs = 1.f / sqrtf(fmaxf(1.f - xx * xx, 0.f));
          jv = (sc == QP_SCALE_ASIN) ? rs : -rs;
        }
        j0 = cc == 0 ? jv : 0.f; j1 = cc == 1 ? jv : 0.f; j2 = cc == 2 ? jv : 0.f;
      } else {
        sincosf(0.5f * angles[pt * n + q], &s, &c);
        j0 = jac[(pt * n + q) * 3]; j1 = jac[(pt * n + q) * 3 + 1]; j2 = jac[(pt * n + q) * 3 + 2];
      }
    } else {
      c = 0.f;   // padding point: zero state
    }
    float* e = enc + (size_t)q * 5 * Pc + p;   // [q][5][Pc]: consecutive points contiguous
    e[0] = c; e[Pc] = s; e[2 * (size_t)Pc] = j0; e[3 * (size_t)Pc] = j1; e[4 * (size_t)Pc] = j2;
  }
}

// psi, dpsi_c (statevectors 0..3) of every (amplitude, point) of the chunk.  Grid (points / 256,
// amplitudes / kDenseRows): each thread builds kDenseRows amplitudes of one point.
constexpr int kDenseRows = 4;
__global__ void k_dense_init(const QPlanDev* __restrict__ plan, const float* __restrict__ enc, int Pc,
                             float2* __restrict__ X) {
  const int n = plan->n;
  const long long DIM = 1ll << n;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pc) return;
  const bool rx = plan->enc_gate == QP_ENC_RX;
  for (int rr = 0; rr < kDenseRows; ++rr) {
  const uint32_t j = blockIdx.y * kDenseRows + rr;
  if (j >= (uint32_t)DIM) break;
  float Pr = 1.f, Pi = 0.f, Dr[3] = {0.f, 0.f, 0.f}, Di[3] = {0.f, 0.f, 0.f};
  for (int q = 0; q < n; ++q) {
    const float* e = enc + (size_t)q * 5 * Pc + p;
    const bool b = (j >> (n - 1 - q)) & 1u;
    const float c = e[0], s = e[Pc];
    float er, ei, dr, di;
    if (!b) { er = c; ei = 0.f; dr = -0.5f * s; di = 0.f; }
    else if (!rx) { er = s; ei = 0.f; dr = 0.5f * c; di = 0.f; }
    else { er = 0.f; ei = -s; dr = 0.f; di = -0.5f * c; }
    for (int k = 0; k < 3; ++k) {
      const float jj = e[(2 + k) * (size_t)Pc];
      const float nr = Dr[k] * er - Di[k] * ei + jj * (Pr * dr - Pi * di);
      const float ni = Dr[k] * ei + Di[k] * er + jj * (Pr * di + Pi * dr);
      Dr[k] = nr; Di[k] = ni;
    }
    const float npr = Pr * er - Pi * ei, npi = Pr * ei + Pi * er;
    Pr = npr; Pi = npi;
  }
  X[((size_t)0 * DIM + j) * Pc + p] = make_float2(Pr, Pi);
  for (int k = 0; k < 3; ++k) X[((size_t)(1 + k) * DIM + j) * Pc + p] = make_float2(Dr[k], Di[k]);
  }
}

// Apply a block (A-operands tab) to statevectors [s0, s0+ns) of the chunk: one wave per
// (statevector, other-index, 32 points) column group, in place.
// The block's A-operands sit in LDS (read per k-step), which keeps the kernel at 4 waves per SIMD
// so that loads of some waves overlap the MFMA chains of others.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_dense_apply(const QPlanDev* __restrict__ plan, const float* __restrict__ tab, int g, float2* __restrict__ X,
                   int s0, int ns, int Pc) {
  __shared__ float sa[2 * 32 * 64];
  const int n = plan->n;
  const QDenseGroup* G = dgroup(plan, g);
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
  const int JO = 1 << (n - 5);
  const int PT = (Pc + 31) / 32;
  const long long tiles = (long long)ns * JO * PT;
  const long long DIM = 1ll << n;
  int pos[5];
  uint32_t free_mask = (1u << n) - 1;
  for (int b = 0; b < 5; ++b) { pos[b] = G->pos[b]; free_mask &= ~(1u << pos[b]); }
  const float* tg = tab + (size_t)g * 4096;
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) sa[e] = tg[e];
  __syncthreads();
  uint32_t boff[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    uint32_t o = 0;
    for (int b = 0; b < 5; ++b) o |= ((uint32_t)(i >> b) & 1u) << pos[b];
    boff[i] = o;
  }
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long t = wave; t < tiles; t += nwaves) {
    asm volatile("" ::: "memory");   // keep the A-operand LDS reads inside the loop (not hoisted to registers)
    const int pt = (int)(t % PT);
    const long long r2 = t / PT;
    const int jo = (int)(r2 % JO);
    const int s = s0 + (int)(r2 / JO);
    uint32_t jb = 0;   // deposit jo into the free (non-block) index bits, ascending
    {
      uint32_t m = free_mask, x = (uint32_t)jo;
      for (int k = 0; k < n; ++k)
        if ((m >> k) & 1u) { jb |= (x & 1u) << k; x >>= 1; }
    }
    const int p = pt * 32 + c;
    const bool ok = p < Pc;
    float2* base = X + (size_t)s * DIM * Pc;
    float bv[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const float2 v = ok ? base[(size_t)(jb | boff[i]) * Pc + p] : make_float2(0.f, 0.f);
      bv[i] = h ? v.y : v.x;
    }
    // two interleaved accumulation chains per row tile (even / odd k-steps), summed at the end:
    // halves the length of each FP32 accumulation chain
    f32x16 acc0, acc1, acc2, acc3;
#pragma unroll
    for (int v = 0; v < 16; ++v) { acc0[v] = 0.f; acc1[v] = 0.f; acc2[v] = 0.f; acc3[v] = 0.f; }
    __builtin_amdgcn_s_setprio(1);   // raised priority while issuing the matrix-core chain
#pragma unroll
    for (int i = 0; i < 32; i += 2) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[(0 * 32 + i) * 64 + lane], bv[i], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[(1 * 32 + i) * 64 + lane], bv[i], acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[(0 * 32 + i + 1) * 64 + lane], bv[i + 1], acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[(1 * 32 + i + 1) * 64 + lane], bv[i + 1], acc3, 0, 0, 0);
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int v = 0; v < 16; ++v) { acc0[v] += acc2[v]; acc1[v] += acc3[v]; }
    if (ok) {
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int m = 8 * (v >> 2) + 4 * h + (v & 3);   // even real row = 2 * amplitude
        base[(size_t)(jb | boff[m >> 1]) * Pc + p] = make_float2(acc0[v], acc0[v + 1]);
        base[(size_t)(jb | boff[16 + (m >> 1)]) * Pc + p] = make_float2(acc1[v], acc1[v + 1]);
      }
    }
  }
}

// Readout, first stage: Z-weighted sums of |psi|^2 and 2 Re(conj(psi) dpsi_c) over a slice of
// the amplitudes.  Grid (Pc / 64, ceil(nsl / 4)), 4 waves of 64 points; wave w of group y takes
// slice 4y + w of nsl equal slices (each a multiple of 32 amplitudes, summed in blocks of 32);
// the four waves are combined in LDS in a fixed order and group y writes
// zpart[(y * 4m + k) * Pc + p].
__global__ __launch_bounds__(256) void k_dense_zsum(const QPlanDev* __restrict__ plan, const float2* __restrict__ X,
                                                    int Pc, int nsl, float* __restrict__ zpart) {
  __shared__ float red[4][kMaxOut * 4][64];
  const int n = plan->n, m = plan->n_out;
  const long long DIM = 1ll << n;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  const int sl = blockIdx.y * 4 + w;
  const long long len = DIM / nsl;
  uint32_t zp[kMaxOut];
  float acc[kMaxOut * 4];
#pragma unroll
  for (int i = 0; i < kMaxOut; ++i) zp[i] = i < m ? plan->zplain[i] : 0u;
#pragma unroll
  for (int i = 0; i < kMaxOut * 4; ++i) acc[i] = 0.f;
  if (p < Pc && sl < nsl) {
    for (long long j0 = sl * len; j0 < (sl + 1) * len; j0 += 32) {
      float blk[kMaxOut * 4];
#pragma unroll
      for (int i = 0; i < kMaxOut * 4; ++i) blk[i] = 0.f;
      const long long j1 = j0 + 32 < DIM ? j0 + 32 : DIM;
      for (long long j = j0; j < j1; ++j) {
        const float2 a = X[j * Pc + p];
        const float2 t0 = X[(DIM + j) * Pc + p], t1 = X[(2 * DIM + j) * Pc + p], t2 = X[(3 * DIM + j) * Pc + p];
        const float p2 = a.x * a.x + a.y * a.y;
        const float g0 = 2.f * (a.x * t0.x + a.y * t0.y), g1 = 2.f * (a.x * t1.x + a.y * t1.y),
                    g2 = 2.f * (a.x * t2.x + a.y * t2.y);
#pragma unroll
        for (int i = 0; i < kMaxOut; ++i) {
          if (i >= m) break;
          const float z = (__popc(zp[i] & (uint32_t)j) & 1) ? -1.f : 1.f;
          blk[i * 4] += z * p2; blk[i * 4 + 1] += z * g0; blk[i * 4 + 2] += z * g1; blk[i * 4 + 3] += z * g2;
        }
      }
#pragma unroll
      for (int i = 0; i < kMaxOut * 4; ++i) acc[i] += blk[i];
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxOut * 4; ++i)
    if (i < 4 * m) red[w][i][lane] = acc[i];
  __syncthreads();
  for (int i = w; i < 4 * m; i += 4) {
    const float v = ((red[0][i][lane] + red[1][i][lane]) + red[2][i][lane]) + red[3][i][lane];
    if (p < Pc) zpart[((size_t)blockIdx.y * 4 * m + i) * Pc + p] = v;
  }
}

// Readout, second stage, one thread per point: the slice groups' sums in order give (f, g); for
// gradient modes also the per-point seeds and loss term.
__global__ void k_dense_readout(const QPlanDev* __restrict__ plan, const float* __restrict__ zpart, int ngy,
                                long long P0, int Pc, int Pv, DenseLoss L, float* __restrict__ out,
                                float* __restrict__ tan, float* __restrict__ seeds, float* __restrict__ lterm) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pc) return;
  const int m = plan->n_out;
  float acc[kMaxOut * 4];
#pragma unroll
  for (int i = 0; i < kMaxOut * 4; ++i) acc[i] = 0.f;
  for (int y = 0; y < ngy; ++y) {
#pragma unroll
    for (int i = 0; i < kMaxOut * 4; ++i)
      if (i < 4 * m) acc[i] += zpart[((size_t)y * 4 * m + i) * Pc + p];
  }
  const bool valid = p < Pv;
  const long long pt = P0 + p;
  if (valid) {
#pragma unroll
    for (int i = 0; i < kMaxOut; ++i) {
      if (i >= m) break;
      if (out) out[pt * m + i] = acc[i * 4];
      if (tan) { tan[(pt * m + i) * 3] = acc[i * 4 + 1]; tan[(pt * m + i) * 3 + 1] = acc[i * 4 + 2]; tan[(pt * m + i) * 3 + 2] = acc[i * 4 + 3]; }
    }
  }
  if (!seeds) return;
  float V[kMaxOut], Wt[kMaxOut][3];
#pragma unroll
  for (int i = 0; i < kMaxOut; ++i) { V[i] = 0.f; Wt[i][0] = Wt[i][1] = Wt[i][2] = 0.f; }
  float lt = 0.f;
  if (valid && L.maxwell) {
    float eps = 1.f, w1 = L.w_all;
    if (L.kind != QP_LOSS_VACUUM) {
      const bool diel = L.points[pt * 3 + 1] >= L.x_if;
      eps = diel ? L.eps_r : 1.f;
      if (L.kind == QP_LOSS_DIEL_SPLIT) {
        const int nv = L.counts[0], nd = L.counts[1];
        if (!L.loss_sum) w1 = diel ? (nd > 0 ? 1.f / nd : 0.f) : (nv > 0 ? 1.f / nv : 0.f);
      }
    }
    const float ie = 1.f / eps, w = L.w_all;
    const float r1 = acc[1] - (acc[10] - acc[7]) * ie, r2 = acc[5] + acc[3], r3 = acc[9] - acc[2];
    lt = w1 * r1 * r1 + w * (r2 * r2 + r3 * r3);
    const float A = 2.f * w1 * r1, Bq = 2.f * w * r2, C = 2.f * w * r3;
    Wt[0][0] = A; Wt[2][1] = -A * ie; Wt[1][2] = A * ie;
    Wt[1][0] = Bq; Wt[0][2] += Bq; Wt[2][0] = C; Wt[0][1] += -C;
  } else if (valid) {
#pragma unroll
    for (int i = 0; i < kMaxOut; ++i) {
      if (i >= m) break;
      if (L.d_out) V[i] = L.d_out[pt * m + i];
      if (L.d_tan) for (int k = 0; k < 3; ++k) Wt[i][k] = L.d_tan[(pt * m + i) * 3 + k];
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxOut; ++i) {
    if (i >= m) break;
    float* sd = seeds + (size_t)i * 4 * Pc + p;   // [i][4][Pc]
    sd[0] = V[i]; sd[Pc] = Wt[i][0]; sd[2 * (size_t)Pc] = Wt[i][1]; sd[3 * (size_t)Pc] = Wt[i][2];
  }
  if (lterm && valid) lterm[pt] = lt;
}

// lambda = Df psi + sum_c D_c dpsi_c and mu_c = D_c psi (statevectors 4..7).
// Grid (points / 256, amplitudes).
__global__ void k_dense_lambda(const QPlanDev* __restrict__ plan, const float* __restrict__ seeds, int Pc,
                               float2* __restrict__ X) {
  const int n = plan->n, m = plan->n_out;
  const long long DIM = 1ll << n;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pc) return;
  const uint32_t j = blockIdx.y;
  float Df = 0.f, D[3] = {0.f, 0.f, 0.f};
  for (int i = 0; i < m; ++i) {
    const float z = (__popc(plan->zplain[i] & j) & 1) ? -1.f : 1.f;
    const float* sd = seeds + (size_t)i * 4 * Pc + p;
    Df += z * sd[0]; D[0] += z * sd[Pc]; D[1] += z * sd[2 * (size_t)Pc]; D[2] += z * sd[3 * (size_t)Pc];
  }
  const float2 a = X[(size_t)j * Pc + p];
  const float2 t0 = X[((size_t)DIM + j) * Pc + p], t1 = X[((size_t)2 * DIM + j) * Pc + p], t2 = X[((size_t)3 * DIM + j) * Pc + p];
  X[((size_t)4 * DIM + j) * Pc + p] = make_float2(Df * a.x + D[0] * t0.x + D[1] * t1.x + D[2] * t2.x,
                                                  Df * a.y + D[0] * t0.y + D[1] * t1.y + D[2] * t2.y);
  for (int k = 0; k < 3; ++k) X[((size_t)(5 + k) * DIM + j) * Pc + p] = make_float2(D[k] * a.x, D[k] * a.y);
}

// Adjoint of block g in one pass over the eight statevectors of the chunk (replaces an
// uncompute pass over psi, the product pass and a pull-back pass over lambda: 16 statevector
// transfers per block instead of 24).  Per (other-index, 64-point) tile and pair s = 0..3 the
// tiles of psi_s and lambda_s, both at the block output, are staged in LDS; waves 0 and 1
// uncompute psi_s <- B^H psi_s for 32 points each, writing the result to HBM and over the psi
// tile; waves 2 and 3 pull lambda_s <- B^H lambda_s back from the staged tile and write it to HBM;
// then every wave adds conj(lambda_out) psi_in^T over 16 of the tile's columns to its M
// accumulators (M taken with psi at the block input and lambda at its output).  At the end the
// four waves are combined in a fixed order into the workgroup's slot of mpart.
__global__ __launch_bounds__(256) void k_dense_adj(const QPlanDev* __restrict__ plan, const float* __restrict__ tab,
                                                   int g, float2* __restrict__ X, int Pc, float* __restrict__ mpart,
                                                   int nwg) {
  constexpr int LD = 65;   // padded row stride (float2)
  __shared__ float2 sm[2 * 32 * LD];   // lambda tile, psi tile; reused for the wave combine
  __shared__ float sa[2 * 32 * 64];    // the block's A-operands (read per k-step: frees 64 VGPRs a lane)
  float2* tl = sm;
  float2* tp = sm + 32 * LD;
  float* red = reinterpret_cast<float*>(sm);
  const int n = plan->n;
  const QDenseGroup* G = dgroup(plan, g);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, c = lane & 31;
  const int JO = 1 << (n - 5);
  const int PT = (Pc + 63) / 64;
  const long long DIM = 1ll << n;
  int pos[5];
  uint32_t free_mask = (1u << n) - 1;
  for (int b = 0; b < 5; ++b) { pos[b] = G->pos[b]; free_mask &= ~(1u << pos[b]); }
  const float* tg = tab + (size_t)g * 4096;
  for (int e = tid; e < 4096; e += 256) sa[e] = tg[e];
  f32x16 mr, mi;
  for (int v = 0; v < 16; ++v) { mr[v] = 0.f; mi[v] = 0.f; }
  // Tile loader: per instruction a wave reads two whole 64-point rows as float4 (2 points a lane);
  // thread tid loads rows 8k + tid/32 (k = 0..3), points 2 (tid % 32) and 2 (tid % 32) + 1.  The
  // next unit's rows are loaded into registers while the current unit is computed.
  const int lc4 = tid & 31, lr0 = tid >> 5;
  uint32_t lboff[4];
  for (int k = 0; k < 4; ++k) {
    uint32_t o = 0;
    for (int b = 0; b < 5; ++b) o |= ((uint32_t)((8 * k + lr0) >> b) & 1u) << pos[b];
    lboff[k] = o;
  }
  const bool is_psi = wave < 2;
  const int c0 = (wave & 1) * 32;     // the 32 tile columns this wave applies the block to
  float2* T = is_psi ? tp : tl;
  const long long ntile = (long long)JO * PT;
  auto tile_jb = [&](long long t) {
    const int jo = (int)(t / PT);
    uint32_t jb = 0;   // deposit jo into the free (non-block) index bits, ascending
    uint32_t m = free_mask, x = (uint32_t)jo;
    for (int k = 0; k < n; ++k)
      if ((m >> k) & 1u) { jb |= (x & 1u) << k; x >>= 1; }
    return jb;
  };
  float4 rl[4], rp[4];
  auto load_unit = [&](long long t, int s) {
    const uint32_t jb = tile_jb(t);
    const int q = (int)(t % PT) * 64 + 2 * lc4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const size_t rowL = ((size_t)(4 + s) * DIM + (jb | lboff[k])) * Pc, rowP = ((size_t)s * DIM + (jb | lboff[k])) * Pc;
      rl[k] = q < Pc ? *reinterpret_cast<const float4*>(X + rowL + q) : make_float4(0.f, 0.f, 0.f, 0.f);
      rp[k] = q < Pc ? *reinterpret_cast<const float4*>(X + rowP + q) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  if ((long long)blockIdx.x < ntile) load_unit(blockIdx.x, 0);
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const int pt = (int)(t % PT);
    const uint32_t jb = tile_jb(t);
    const int p = pt * 64 + c0 + c;
    const bool ok = p < Pc;
    for (int s = 0; s < 4; ++s) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = 8 * k + lr0;
        tl[r * LD + 2 * lc4] = make_float2(rl[k].x, rl[k].y);
        tl[r * LD + 2 * lc4 + 1] = make_float2(rl[k].z, rl[k].w);
        tp[r * LD + 2 * lc4] = make_float2(rp[k].x, rp[k].y);
        tp[r * LD + 2 * lc4 + 1] = make_float2(rp[k].z, rp[k].w);
      }
      __syncthreads();
      if (s < 3) load_unit(t, s + 1);
      else if (t + gridDim.x < ntile) load_unit(t + gridDim.x, 0);
      {   // B^H on 32 columns of the psi tile (waves 0, 1) or of the lambda tile (waves 2, 3)
        const float* Tf = reinterpret_cast<const float*>(T) + 2 * (c0 + c) + h;   // B[k][n]: re (h = 0) or im
        f32x16 acc0, acc1;
#pragma unroll
        for (int v = 0; v < 16; ++v) { acc0[v] = 0.f; acc1[v] = 0.f; }
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int i = 0; i < 32; ++i) {
          const float bv = Tf[2 * i * LD];
          acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[(0 * 32 + i) * 64 + lane], bv, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[(1 * 32 + i) * 64 + lane], bv, acc1, 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        float2* dst = X + (size_t)(is_psi ? s : 4 + s) * DIM * Pc;
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          const int m = 8 * (v >> 2) + 4 * h + (v & 3);   // even real row = 2 * amplitude
          const int a0 = m >> 1, a1 = 16 + (m >> 1);
          uint32_t o0 = 0, o1 = 0;
          for (int b = 0; b < 5; ++b) {
            o0 |= ((uint32_t)(a0 >> b) & 1u) << pos[b];
            o1 |= ((uint32_t)(a1 >> b) & 1u) << pos[b];
          }
          const float2 r0 = make_float2(acc0[v], acc0[v + 1]), r1 = make_float2(acc1[v], acc1[v + 1]);
          if (ok) {
            dst[(size_t)(jb | o0) * Pc + p] = r0;
            dst[(size_t)(jb | o1) * Pc + p] = r1;
          }
          if (is_psi) {   // psi_in replaces psi_out in the tile for the product below
            tp[a0 * LD + c0 + c] = r0;
            tp[a1 * LD + c0 + c] = r1;
          }
        }
      }
      __syncthreads();
      const int a = lane & 31;
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int col = wave * 16 + 2 * kk + h;
        const float2 lv = tl[a * LD + col], pv = tp[a * LD + col];
        // Mr += Lr Pr + Li Pi ; Mi += Lr Pi - Li Pr   (A[m=a][k=col], B[k=col][n=b])
        mr = __builtin_amdgcn_mfma_f32_32x32x2f32(lv.x, pv.x, mr, 0, 0, 0);
        mr = __builtin_amdgcn_mfma_f32_32x32x2f32(lv.y, pv.y, mr, 0, 0, 0);
        mi = __builtin_amdgcn_mfma_f32_32x32x2f32(lv.x, pv.y, mi, 0, 0, 0);
        mi = __builtin_amdgcn_mfma_f32_32x32x2f32(-lv.y, pv.x, mi, 0, 0, 0);
      }
      __builtin_amdgcn_s_setprio(0);
    }
  }
  // combine the four waves (fixed order) and add to this workgroup's slot
  __syncthreads();
  for (int v = 0; v < 16; ++v) {
    red[((wave * 2 + 0) * 16 + v) * 64 + lane] = mr[v];
    red[((wave * 2 + 1) * 16 + v) * 64 + lane] = mi[v];
  }
  __syncthreads();
  float* slot = mpart + ((size_t)g * nwg + blockIdx.x) * 2048;
  for (int e = tid; e < 2 * 16 * 64; e += 256) {
    const int part = e / 1024, v = (e / 64) % 16, l = e % 64;
    float sum = 0.f;
    for (int wv = 0; wv < 4; ++wv) sum += red[((wv * 2 + part) * 16 + v) * 64 + l];
    const int row = 8 * (v >> 2) + 4 * (l >> 5) + (v & 3), col = l & 31;   // M[a = row][b = col]
    slot[part * 1024 + row * 32 + col] += sum;
  }
}

__global__ void k_dense_zero(float* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// FP64 sums: M_g over workgroups (one wave per entry), loss over points (one wave).
__global__ void k_dense_reduce(const float* __restrict__ mpart, int G, int nwg, double* __restrict__ m64,
                               const float* __restrict__ lterm, long long P, double* __restrict__ loss) {
  const long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const long long nm = (long long)G * 2048;
  if (w > nm) return;
  double s = 0.0;
  if (w < nm) {
    const int g = (int)(w / 2048), e = (int)(w % 2048);
    for (int b = lane; b < nwg; b += 64) s += (double)mpart[((size_t)g * nwg + b) * 2048 + e];
  } else if (lterm) {
    for (long long p = lane; p < P; p += 64) s += (double)lterm[p];
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    if (w < nm) m64[w] = s;
    else if (loss) *loss = s;
  }
}

// One workgroup (32 threads used) per parametrised gate occurrence: column b of dB_g/dtheta,
// contracted with M_g: contrib = 2 sum_ab Re(dB_ab M_ab).
__global__ void k_dense_occ(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                            const double* __restrict__ m64, double* __restrict__ contrib) {
  __shared__ double part[64];
  const int o = blockIdx.x, b = threadIdx.x;
  const int* occ = reinterpret_cast<const int*>(reinterpret_cast<const char*>(plan) + plan->off_docc);
  const int g = occ[2 * o], gi = occ[2 * o + 1];
  double s = 0.0;
  if (b < 32) {
    const QDenseGroup* G = dgroup(plan, g);
    double vr[32], vi[32];
    for (int a = 0; a < 32; ++a) { vr[a] = (a == b) ? 1.0 : 0.0; vi[a] = 0.0; }
    for (int k = 0; k < G->ngates; ++k) dense_gate_apply(*dgate(plan, G->gate0 + k), params, vr, vi, k == gi);
    const double* Mr = m64 + (size_t)g * 2048;
    const double* Mi = Mr + 1024;
    for (int a = 0; a < 32; ++a) s += vr[a] * Mr[a * 32 + b] - vi[a] * Mi[a * 32 + b];
  }
  part[b] = s;
  __syncthreads();
  if (b == 0) {
    double t = 0.0;
    for (int k = 0; k < 32; ++k) t += part[k];
    contrib[o] = 2.0 * t;
  }
}

__global__ void k_dense_params(const QPlanDev* __restrict__ plan, const double* __restrict__ contrib,
                               float* __restrict__ grads) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= plan->n_params) return;
  const char* pb = reinterpret_cast<const char*>(plan);
  const int* ptr = reinterpret_cast<const int*>(pb + plan->off_dcsr_ptr);
  const int* idx = reinterpret_cast<const int*>(pb + plan->off_dcsr_idx);
  double s = 0.0;
  for (int e = ptr[k]; e < ptr[k + 1]; ++e) s += contrib[idx[e]];
  grads[k] = (float)s;
}

// ---------------------------------------------------------------------------------------------
static inline unsigned nb(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Amplitude slices of the readout's first stage (a multiple of 32 amplitudes each, at most 64)
// and the number of 4-slice groups.
static inline int dense_readout_slices(int n) {
  const long long dim = 1ll << n;
  long long ns = dim / 32;
  if (ns < 1) ns = 1;
  if (ns > 64) ns = 64;
  return (int)ns;
}
static inline int dense_readout_groups(int n) { return (dense_readout_slices(n) + 3) / 4; }

DenseLayout dense_layout(int n, int m, int G, int n_docc, long long P, int Pc, int nwg, bool grad) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  DenseLayout L{};
  size_t off = 0;
  const int S = grad ? 8 : 4;
  L.tabF = off; off = al(off + sizeof(float) * 4096 * (size_t)(G > 0 ? G : 1));
  L.tabA = off; off = al(off + sizeof(float) * 4096 * (size_t)(G > 0 ? G : 1));
  L.X = off; off = al(off + sizeof(float2) * (size_t)S * ((size_t)1 << n) * Pc);
  L.enc = off; off = al(off + sizeof(float) * 5 * (size_t)n * Pc);
  L.seeds = off; off = al(off + sizeof(float) * 4 * kMaxOut * (size_t)Pc);
  L.zpart = off; off = al(off + sizeof(float) * 4 * kMaxOut * (size_t)dense_readout_groups(n) * Pc);
  L.lterm = off; off = al(off + sizeof(float) * (size_t)(P > 0 ? P : 1));
  L.mpart = off; off = al(off + sizeof(float) * 2048 * (size_t)(G > 0 ? G : 1) * nwg);
  L.m64 = off; off = al(off + sizeof(double) * 2048 * (size_t)(G > 0 ? G : 1));
  L.contrib = off; off = al(off + sizeof(double) * (size_t)(n_docc > 0 ? n_docc : 1));
  L.angles = off; off = al(off + sizeof(float) * (size_t)(P > 0 ? P : 1) * n);
  L.jac = off; off = al(off + sizeof(float) * (size_t)(P > 0 ? P : 1) * n * 3);
  L.counts = off; off = al(off + 2 * sizeof(int));
  L.total = off;
  (void)m;
  return L;
}

int dense_chunk(int n, long long P, bool grad) {
  const size_t per = (size_t)(grad ? 8 : 4) * ((size_t)1 << n) * sizeof(float2);
  long long pc = (long long)((size_t)2 << 30) / (long long)per;   // about 2 GiB of statevectors
  pc = pc / 64 * 64;
  if (pc < 64) pc = 64;
  if (P < pc) pc = (P + 63) / 64 * 64;
  return (int)(pc > 0 ? pc : 64);
}

hipError_t dense_run(const DenseCall& c, hipStream_t st) {
  const QPlanDev* plan = c.plan;
  const int n = c.n, G = c.G;
  char* w = static_cast<char*>(c.ws);
  const DenseLayout& L = c.L;
  float* tabF = reinterpret_cast<float*>(w + L.tabF);
  float* tabA = reinterpret_cast<float*>(w + L.tabA);
  float2* X = reinterpret_cast<float2*>(w + L.X);
  float* enc = reinterpret_cast<float*>(w + L.enc);
  float* seeds = reinterpret_cast<float*>(w + L.seeds);
  float* zpart = reinterpret_cast<float*>(w + L.zpart);
  const int nsl = dense_readout_slices(n), ngy = dense_readout_groups(n);
  float* lterm = reinterpret_cast<float*>(w + L.lterm);
  float* mpart = reinterpret_cast<float*>(w + L.mpart);
  double* m64 = reinterpret_cast<double*>(w + L.m64);
  double* contrib = reinterpret_cast<double*>(w + L.contrib);
  const long long DIM = 1ll << n;
  if (G > 0) hipLaunchKernelGGL(k_dense_tables, dim3(G), dim3(64), 0, st, plan, c.params, tabF, tabA);
  if (c.grad) {
    const long long nm = (long long)G * c.nwg * 2048;
    if (nm > 0) hipLaunchKernelGGL(k_dense_zero, dim3(nb(nm, 256)), dim3(256), 0, st, mpart, nm);
  }
  const int apply_grid = c.apply_grid;
  for (long long P0 = 0; P0 < c.P; P0 += c.Pc) {
    const int Pv = (int)((c.P - P0) < c.Pc ? (c.P - P0) : c.Pc);
    const int Pc = c.Pc;
    hipLaunchKernelGGL(k_dense_encode, dim3(nb(Pc, 128)), dim3(128), 0, st, plan, c.points, c.angles, c.jac, P0, Pc, Pv, enc);
    hipLaunchKernelGGL(k_dense_init, dim3(nb(Pc, 256), nb(DIM, kDenseRows)), dim3(256), 0, st, plan, enc, Pc, X);
    for (int g = 0; g < G; ++g)
      hipLaunchKernelGGL(k_dense_apply, dim3(apply_grid), dim3(256), 0, st, plan, tabF, g, X, 0, 4, Pc);
    hipLaunchKernelGGL(k_dense_zsum, dim3(nb(Pc, 64), ngy), dim3(256), 0, st, plan, X, Pc, nsl, zpart);
    hipLaunchKernelGGL(k_dense_readout, dim3(nb(Pc, 64)), dim3(64), 0, st, plan, zpart, ngy, P0, Pc, Pv, c.loss,
                       c.out, c.tan, c.grad ? seeds : nullptr, c.grad ? lterm : nullptr);
    if (!c.grad) continue;
    hipLaunchKernelGGL(k_dense_lambda, dim3(nb(Pc, 256), (unsigned)DIM), dim3(256), 0, st, plan, seeds, Pc, X);
    for (int g = G - 1; g >= 0; --g)
      hipLaunchKernelGGL(k_dense_adj, dim3(c.nwg), dim3(256), 0, st, plan, tabA, g, X, Pc, mpart, c.nwg);
  }
  if (!c.grad) return hipGetLastError();
  const long long cols = (long long)G * 2048 + 1;
  hipLaunchKernelGGL(k_dense_reduce, dim3(nb(cols * 64, 256)), dim3(256), 0, st, mpart, G, c.nwg, m64,
                     c.loss.maxwell ? lterm : nullptr, c.P, c.loss_out);
  if (c.n_docc > 0) hipLaunchKernelGGL(k_dense_occ, dim3(c.n_docc), dim3(64), 0, st, plan, c.params, m64, contrib);
  if (c.K > 0 && c.d_params)
    hipLaunchKernelGGL(k_dense_params, dim3(nb(c.K, 128)), dim3(128), 0, st, plan, contrib, c.d_params);
  return hipGetLastError();
}

}  // namespace qp
