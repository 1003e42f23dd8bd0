// Parameter gradient from the reduced gate statistics (FP64, the final reduction stage).
// A fused gate is U = R_{c-1} ... R_0 with R = exp(-i theta P / 2), so dU/dtheta_c = U (-i/2) G_c
// with the rotated generator G_c = W^H P_c W, W = R_{c-1} ... R_0 (the components before c).
// With lambda and psi both taken before the gate,
//   d L / d theta_c = 2 Re <lambda_after| dU |psi> = Im <lambda|G_c|psi> = sum_k n_k S_k,
// where G_c = n_x X + n_y Y + n_z Z and S_k = Im <lambda|sigma_k|psi> is what the adjoint sweep
// accumulates per gate.  A gate of the leading stage has its statistic taken after the gate
// (lambda_after, psi_after = U psi); the same derivative is then Im <lambda_after|G'_c|psi_after>
// with G'_c = U G_c U^H = V P_c V^H, V = R_{n-1} ... R_{c+1} the components after c (R_c
// commutes with P_c).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"
#include "rot_dev.hpp"

namespace qp {

// Axis (n_x, n_y, n_z) of G_c for component ci of fused gate fu.
__host__ __device__ inline void generator_axis(const QFused& fu, const float* __restrict__ params, int ci, double* nvec) {
  if (fu.stat_out) {
    double v[8];
    set_identity(v);
    for (int c = ci + 1; c < fu.ncomp; ++c) {
      double s, co;
      sincos(0.5 * (double)params[fu.param[c]], &s, &co);
      left_mul_rot<double>(fu.kind[c], co, s, v);
    }
    // a = (-i/2) P V^H, so P V^H = 2i a
    double a[8] = {v[0], -v[1], v[4], -v[5], v[2], -v[3], v[6], -v[7]};
    left_mul_mhalf_i_pauli<double>(fu.kind[ci], a);
    double b[8];
    for (int e = 0; e < 4; ++e) { b[2 * e] = -2.0 * a[2 * e + 1]; b[2 * e + 1] = 2.0 * a[2 * e]; }
    // G' = V b: G'00 = V00 b00 + V01 b10, G'10 = V10 b00 + V11 b10
    const double g00r = v[0] * b[0] - v[1] * b[1] + v[2] * b[4] - v[3] * b[5];
    const double g10r = v[4] * b[0] - v[5] * b[1] + v[6] * b[4] - v[7] * b[5];
    const double g10i = v[4] * b[1] + v[5] * b[0] + v[6] * b[5] + v[7] * b[4];
    nvec[0] = g10r;
    nvec[1] = g10i;
    nvec[2] = g00r;
    return;
  }
  double w[8];
  set_identity(w);
  for (int c = 0; c < ci; ++c) {
    double s, co;
    sincos(0.5 * (double)params[fu.param[c]], &s, &co);
    left_mul_rot<double>(fu.kind[c], co, s, w);
  }
  double v[8];
  for (int e = 0; e < 8; ++e) v[e] = w[e];
  left_mul_mhalf_i_pauli<double>(fu.kind[ci], v);   // v = (-i/2) P W, so P W = 2i v
  double pw[8];
  for (int e = 0; e < 4; ++e) { pw[2 * e] = -2.0 * v[2 * e + 1]; pw[2 * e + 1] = 2.0 * v[2 * e]; }
  // G00 = conj(W00) PW00 + conj(W10) PW10;  G10 = conj(W01) PW00 + conj(W11) PW10
  const double g00r = w[0] * pw[0] + w[1] * pw[1] + w[4] * pw[4] + w[5] * pw[5];
  const double g10r = w[2] * pw[0] + w[3] * pw[1] + w[6] * pw[4] + w[7] * pw[5];
  const double g10i = w[2] * pw[1] - w[3] * pw[0] + w[6] * pw[5] - w[7] * pw[4];
  nvec[0] = g10r;
  nvec[1] = g10i;
  nvec[2] = g00r;
}

__device__ inline double param_grad_one(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                                        const double* __restrict__ s64, int k) {
  const char* pb = reinterpret_cast<const char*>(plan);
  const QFused* fused = reinterpret_cast<const QFused*>(pb + plan->off_fused);
  const int* ptr = reinterpret_cast<const int*>(pb + plan->off_csr_ptr);
  const int* idx = reinterpret_cast<const int*>(pb + plan->off_csr_idx);
  double gsum = 0.0;
  for (int e = ptr[k]; e < ptr[k + 1]; ++e) {
    const int fi = idx[e] >> 2, ci = idx[e] & 3;
    double nv[3];
    generator_axis(fused[fi], params, ci, nv);
    const double* S = s64 + fi * kGS;
    gsum += nv[0] * S[0] + nv[1] * S[1] + nv[2] * S[2];
  }
  // CRZ(c, t) occurrences: dL/dtheta = M_c - 2 M_ct from the phase-stage moments, which follow the
  // fused-gate statistics (see QPhaseStage)
  if (plan->n_phase > 0) {
    const int* pptr = reinterpret_cast<const int*>(pb + plan->off_pcsr_ptr);
    const int* pidx = reinterpret_cast<const int*>(pb + plan->off_pcsr_idx);
    const QPhaseStage* stages = reinterpret_cast<const QPhaseStage*>(pb + plan->off_phase);
    const QPhaseGate* pg = reinterpret_cast<const QPhaseGate*>(pb + plan->off_phase_gates);
    const int n = plan->n;
    for (int e = pptr[k]; e < pptr[k + 1]; ++e) {
      const int gi = pidx[e];
      int s = 0;
      while (s + 1 < plan->n_phase && stages[s + 1].gate0 <= gi) ++s;
      const double* M = s64 + plan->n_fused * kGS + stages[s].mom_off;
      const int c = pg[gi].c, t = pg[gi].t;
      const int a = c < t ? c : t, b = c < t ? t : c;
      gsum += M[c] - 2.0 * M[n + phase_pair_index(n, a, b)];
    }
  }
  return gsum;
}

}  // namespace qp
