// Fused per-point circuit kernels for gfx950 (MI355X): helper kernels and dispatch.
// The fused kernel template itself is in fused_kernel.hpp (see the description below).
//
// One workgroup evaluates a tile of collocation points.  Every point's statevector psi and its
// three input tangents dpsi_t, dpsi_x, dpsi_y (and, in the adjoint, lambda and mu_t, mu_x, mu_y)
// live in registers: a thread owns 8 amplitudes of each statevector, addressed by three
// "register" index bits; the other n-3 index bits select the thread inside the point's thread
// group.  A round applies up to three fused single-qubit gates whose qubits sit on the register
// bits (no data movement); between rounds the state is re-distributed through LDS so that the
// next round's qubits land on the register bits.  Entangler stages (CNOT/CZ runs) are folded
// into that exchange as an index map plus a sign, so they cost no extra pass.
//
// Forward-mode tangents: a gate U acts on psi and on each dpsi_c identically because the
// variational gates do not depend on the input point; only the encoding does, and its derivative
// seeds dpsi at the start.  Readout: f_i = sum_j z_i(j)|psi_j|^2,
// g_ic = 2 sum_j z_i(j) Re(conj(psi_j) dpsi_c,j) (section "QPINN architecture": Pauli-Z per qubit).
//
// Adjoint with uncompute: with lambda = dL/dpsi*, mu_c = dL/d(dpsi_c)* at the circuit end,
// each gate (in reverse order) first uncomputes psi <- U^H psi, dpsi_c <- U^H dpsi_c, then adds
//   M_ab += conj(lambda_a) psi_b + sum_c conj(mu_c,a) dpsi_c,b   (a: output row, b: input column)
// over the gate's amplitude pairs, then pulls lambda, mu_c back through U^H.  The parameter
// gradient is dL/dtheta = 2 Re sum_ab (dU/dtheta)_ab M_ab, evaluated after the FP64 reduction.
//
// Arithmetic is complex64 with FP32 accumulation; per-workgroup partials are reduced across
// workgroups in a fixed order in FP64 (separate kernels), so results are deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qp_internal.hpp"
#include "fused.hpp"
#include "grads_dev.hpp"
#include "rot_dev.hpp"

namespace qp {


hipError_t launch_fused_3(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_4(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_5(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_6(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_7(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_8(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_9(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_10(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_11(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
hipError_t launch_fused_12(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);

// ---------------------------------------------------------------------------------------------
// Gate table: U = R_{c-1} ... R_0 for every fused gate, R_P(theta) = exp(-i theta P/2).  The table
// is formed once per call from the K parameters (work independent of the point count) in FP64
// and rounded once to complex64; every per-point operation then runs in FP32.  The FP32-built
// variant (k_gate_table) is kept for comparison (QP_FLAG_GATES_FP32).
__global__ void k_gate_table64(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                               float* __restrict__ gtab) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > plan->n_fused) return;
  if (f == plan->n_fused) {   // identity entry used for absent gates of a round
    float u[8];
    set_identity(u);
    store_gate_entry(gtab + f * kGT, u);
    return;
  }
  const QFused* fu = reinterpret_cast<const QFused*>(reinterpret_cast<const char*>(plan) + plan->off_fused) + f;
  double u[8];
  set_identity(u);
  for (int c = 0; c < fu->ncomp; ++c) {
    double s, co;
    sincos(0.5 * (double)params[fu->param[c]], &s, &co);
    left_mul_rot<double>(fu->kind[c], co, s, u);
  }
  store_gate_entry(gtab + f * kGT, u);
}

__global__ void k_gate_table(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                             float* __restrict__ gtab) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > plan->n_fused) return;
  if (f == plan->n_fused) {   // identity entry used for absent gates of a round
    float u[8];
    set_identity(u);
    store_gate_entry(gtab + f * kGT, u);
    return;
  }
  const QFused* fu = reinterpret_cast<const QFused*>(reinterpret_cast<const char*>(plan) + plan->off_fused) + f;
  float u[8];
  set_identity(u);
  for (int c = 0; c < fu->ncomp; ++c) {
    float s, co;
    sincosf(0.5f * params[fu->param[c]], &s, &co);
    left_mul_rot<float>(fu->kind[c], co, s, u);
  }
  store_gate_entry(gtab + f * kGT, u);
}

// Phase-stage coefficients in 32-bit fractions of a turn (one thread per coefficient):
// alpha_q = -(1/2) sum_t theta_qt, beta_qq' = theta_qq' + theta_q'q (see QPhaseStage).  Like the
// gate table this is O(K) work per call and runs in FP64; the result is reduced modulo one turn.
__global__ void k_phase_table(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                              uint32_t* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = plan->n, nt = phase_terms(n);
  if (i >= plan->n_phase * nt) return;
  const char* pb = reinterpret_cast<const char*>(plan);
  const QPhaseStage& st = reinterpret_cast<const QPhaseStage*>(pb + plan->off_phase)[i / nt];
  const QPhaseGate* gates = reinterpret_cast<const QPhaseGate*>(pb + plan->off_phase_gates) + st.gate0;
  const int e = i % nt;
  int qa = e, qb = -1;   // alpha_qa, or beta of the pair (qa, qb)
  if (e >= n) {
    int r = e - n;
    qa = 0;
    while (r >= n - 1 - qa) { r -= n - 1 - qa; ++qa; }
    qb = qa + 1 + r;
  }
  double turns = 0.0;
  const double inv2pi = 0.15915494309189533577;
  for (int g = 0; g < st.ngates; ++g) {
    const double th = (double)params[gates[g].param];
    if (qb < 0) {
      if (gates[g].c == qa) turns -= 0.5 * th * inv2pi;
    } else if ((gates[g].c == qa && gates[g].t == qb) || (gates[g].c == qb && gates[g].t == qa)) {
      turns += th * inv2pi;
    }
  }
  const double frac = turns - floor(turns);                 // [0, 1)
  coef[st.coef_off + e] = (uint32_t)(unsigned long long)(frac * 4294967296.0);
}

// Random-Fourier-feature angles: phi = [cos(Bp); sin(Bp)], theta = W phi, J = W dphi/dp.
__global__ void k_rff_angles(const QPlanDev* __restrict__ plan, const float* __restrict__ points,
                             long long P, float* __restrict__ angles, float* __restrict__ jac) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const char* pb = reinterpret_cast<const char*>(plan);
  const float* B = reinterpret_cast<const float*>(pb + plan->off_rff_B);
  const float* W = reinterpret_cast<const float*>(pb + plan->off_rff_W);
  const int n = plan->n, F = plan->n_feat;
  const float t = points[p * 3], x = points[p * 3 + 1], y = points[p * 3 + 2];
  float th[kMaxQubits], j0[kMaxQubits], j1[kMaxQubits], j2[kMaxQubits];
  for (int q = 0; q < n; ++q) th[q] = j0[q] = j1[q] = j2[q] = 0.f;
  for (int f = 0; f < F; ++f) {
    const float b0 = B[f * 3], b1 = B[f * 3 + 1], b2 = B[f * 3 + 2];
    const float pr = b0 * t + b1 * x + b2 * y;
    float s, c;
    sincosf(pr, &s, &c);
    for (int q = 0; q < n; ++q) {
      const float wc = W[q * 2 * F + f], ws = W[q * 2 * F + F + f];
      th[q] += wc * c + ws * s;
      const float dd = ws * c - wc * s;   // d/dproj of (wc cos + ws sin)
      j0[q] += dd * b0; j1[q] += dd * b1; j2[q] += dd * b2;
    }
  }
  for (int q = 0; q < n; ++q) {
    angles[p * n + q] = th[q];
    jac[(p * n + q) * 3 + 0] = j0[q];
    jac[(p * n + q) * 3 + 1] = j1[q];
    jac[(p * n + q) * 3 + 2] = j2[q];
  }
}

// Number of points in the dielectric half (x >= x_if); one workgroup, deterministic.
__global__ void k_count_diel(const float* __restrict__ points, long long P, float x_if, int* __restrict__ counts) {
  __shared__ int sh[16];
  int c = 0;
  for (long long p = threadIdx.x; p < P; p += blockDim.x) c += points[p * 3 + 1] >= x_if ? 1 : 0;
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    counts[0] = (int)(P - s);
    counts[1] = s;
  }
}

// FP64 cross-workgroup reduction of the M partials (one wave per entry) and of the loss.
__global__ void k_reduce_m(const float* __restrict__ mpart, int nblk, int ncol,
                           const float* __restrict__ lpart, double* __restrict__ m64,
                           double* __restrict__ loss) {
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col > ncol) return;
  double s = 0.0;
  if (col < ncol) {
    for (int b = lane; b < nblk; b += 64) s += (double)mpart[(long long)b * ncol + col];
  } else if (lpart) {
    for (int b = lane; b < nblk; b += 64) s += (double)lpart[b];
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    if (col < ncol) m64[col] = s;
    else if (loss) *loss = s;
  }
}

// d L / d theta_k for every parameter (FP64; see grads_dev.hpp).
__global__ void k_param_grads(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                              const double* __restrict__ m64, float* __restrict__ grads) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= plan->n_params) return;
  grads[k] = (float)param_grad_one(plan, params, m64, k);
}

int fused_threads(int n) { return fused_wg_threads(n); }
int fused_max_wg_per_cu(int n) { return fused_threads(n) == 512 ? 1 : 4; }
int fused_points_per_tile(int n) { return fused_threads(n) / (1 << (n - 3)); }
size_t fused_lds_bytes(int n, int exs, int n_fused, int n_mom) {
  const int T = fused_threads(n);
  return (size_t)exs * T * 8 * sizeof(float2) + (size_t)(T / 64) * (n_fused * kGS + n_mom) * sizeof(float) +
         (size_t)(T / 64) * 40 * sizeof(float);
}

hipError_t launch_fused(int n, int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st) {
  switch (n) {
    case 3: return launch_fused_3(mode, a, grid, exs, signs, lds, st);
    case 4: return launch_fused_4(mode, a, grid, exs, signs, lds, st);
    case 5: return launch_fused_5(mode, a, grid, exs, signs, lds, st);
    case 6: return launch_fused_6(mode, a, grid, exs, signs, lds, st);
    case 7: return launch_fused_7(mode, a, grid, exs, signs, lds, st);
    case 8: return launch_fused_8(mode, a, grid, exs, signs, lds, st);
    case 9: return launch_fused_9(mode, a, grid, exs, signs, lds, st);
    case 10: return launch_fused_10(mode, a, grid, exs, signs, lds, st);
    case 11: return launch_fused_11(mode, a, grid, exs, signs, lds, st);
    case 12: return launch_fused_12(mode, a, grid, exs, signs, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gate_table(const QPlanDev* plan, int n_fused, int n_phase_coef, const float* params, float* gtab,
                             int fp32, hipStream_t st) {
  const int entries = n_fused + 1;   // + identity
  if (fp32) hipLaunchKernelGGL(k_gate_table, dim3((entries + 127) / 128), dim3(128), 0, st, plan, params, gtab);
  else hipLaunchKernelGGL(k_gate_table64, dim3((entries + 127) / 128), dim3(128), 0, st, plan, params, gtab);
  if (n_phase_coef > 0)
    hipLaunchKernelGGL(k_phase_table, dim3((n_phase_coef + 127) / 128), dim3(128), 0, st, plan, params,
                       reinterpret_cast<uint32_t*>(gtab + (size_t)entries * kGT));
  return hipGetLastError();
}

hipError_t launch_rff(const QPlanDev* plan, const float* points, long long P, float* angles, float* jac, hipStream_t st) {
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rff_angles, dim3((unsigned)((P + 127) / 128)), dim3(128), 0, st, plan, points, P, angles, jac);
  return hipGetLastError();
}

hipError_t launch_count(const float* points, long long P, float x_if, int* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_count_diel, dim3(1), dim3(1024), 0, st, points, P, x_if, counts);
  return hipGetLastError();
}

hipError_t launch_reduce(const float* mpart, int nblk, int ncol, const float* lpart, double* m64, double* loss, hipStream_t st) {
  const int cols = ncol + 1;   // + loss
  const int waves_per_block = 4;
  hipLaunchKernelGGL(k_reduce_m, dim3((cols + waves_per_block - 1) / waves_per_block), dim3(64 * waves_per_block), 0, st,
                     mpart, nblk, ncol, lpart, m64, loss);
  return hipGetLastError();
}

hipError_t launch_param_grads(const QPlanDev* plan, int K, const float* params, const double* m64, float* grads, hipStream_t st) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_param_grads, dim3((K + 127) / 128), dim3(128), 0, st, plan, params, m64, grads);
  return hipGetLastError();
}

}  // namespace qp
