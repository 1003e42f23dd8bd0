// Parameter gradient from the reduced gate adjoint products (FP64, the final reduction stage):
//   d L / d theta_k = sum over gate components driven by theta_k of 2 Re sum_ab (dU/dtheta)_ab M_ab,
// with U = R_{c-1} ... R_0 the fused gate and dR/dtheta = -(i/2) P R for R = exp(-i theta P/2).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"
#include "rot_dev.hpp"

namespace qp {

__device__ inline double param_grad_one(const QPlanDev* __restrict__ plan, const float* __restrict__ params,
                                        const double* __restrict__ m64, int k) {
  const char* pb = reinterpret_cast<const char*>(plan);
  const QFused* fused = reinterpret_cast<const QFused*>(pb + plan->off_fused);
  const int* ptr = reinterpret_cast<const int*>(pb + plan->off_csr_ptr);
  const int* idx = reinterpret_cast<const int*>(pb + plan->off_csr_idx);
  double gsum = 0.0;
  for (int e = ptr[k]; e < ptr[k + 1]; ++e) {
    const int fi = idx[e] >> 2, ci = idx[e] & 3;
    const QFused& fu = fused[fi];
    double u[8];
    set_identity(u);
    for (int c = 0; c < fu.ncomp; ++c) {
      double s, co;
      sincos(0.5 * (double)params[fu.param[c]], &s, &co);
      left_mul_rot<double>(fu.kind[c], co, s, u);
      if (c == ci) left_mul_mhalf_i_pauli<double>(fu.kind[c], u);
    }
    const double* M = m64 + fi * 8;
    double re = 0.0;
    for (int ab = 0; ab < 4; ++ab) re += u[2 * ab] * M[2 * ab] - u[2 * ab + 1] * M[2 * ab + 1];
    gsum += 2.0 * re;
  }
  return gsum;
}

}  // namespace qp
