// Parameter gradient from the reduced gate adjoint products (FP64, the final reduction stage):
//   d L / d theta_k = sum over gate components driven by theta_k of 2 Re sum_ab (dU/dtheta)_ab M_ab,
// with U = R_{c-1} ... R_0 the fused gate and dR/dtheta = -(i/2) P R for R = exp(-i theta P/2).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"

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
    double ur[2][2] = {{1, 0}, {0, 1}}, ui[2][2] = {{0, 0}, {0, 0}};
    for (int c = 0; c < fu.ncomp; ++c) {
      double s, co;
      sincos(0.5 * (double)params[fu.param[c]], &s, &co);
      double rr[2][2], ri[2][2];
      const int kd = fu.kind[c];
      if (kd == QP_RX) { rr[0][0] = co; ri[0][0] = 0; rr[0][1] = 0; ri[0][1] = -s; rr[1][0] = 0; ri[1][0] = -s; rr[1][1] = co; ri[1][1] = 0; }
      else if (kd == QP_RY) { rr[0][0] = co; ri[0][0] = 0; rr[0][1] = -s; ri[0][1] = 0; rr[1][0] = s; ri[1][0] = 0; rr[1][1] = co; ri[1][1] = 0; }
      else { rr[0][0] = co; ri[0][0] = -s; rr[0][1] = 0; ri[0][1] = 0; rr[1][0] = 0; ri[1][0] = 0; rr[1][1] = co; ri[1][1] = s; }
      if (c == ci) {   // R -> -(i/2) P R
        double pr[2][2], pi[2][2];
        if (kd == QP_RX) { for (int j = 0; j < 2; ++j) { pr[0][j] = rr[1][j]; pi[0][j] = ri[1][j]; pr[1][j] = rr[0][j]; pi[1][j] = ri[0][j]; } }
        else if (kd == QP_RY) { for (int j = 0; j < 2; ++j) { pr[0][j] = ri[1][j]; pi[0][j] = -rr[1][j]; pr[1][j] = -ri[0][j]; pi[1][j] = rr[0][j]; } }
        else { for (int j = 0; j < 2; ++j) { pr[0][j] = rr[0][j]; pi[0][j] = ri[0][j]; pr[1][j] = -rr[1][j]; pi[1][j] = -ri[1][j]; } }
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) { rr[i][j] = 0.5 * pi[i][j]; ri[i][j] = -0.5 * pr[i][j]; }
      }
      double nr[2][2], ni[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          nr[i][j] = rr[i][0] * ur[0][j] - ri[i][0] * ui[0][j] + rr[i][1] * ur[1][j] - ri[i][1] * ui[1][j];
          ni[i][j] = rr[i][0] * ui[0][j] + ri[i][0] * ur[0][j] + rr[i][1] * ui[1][j] + ri[i][1] * ur[1][j];
        }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) { ur[i][j] = nr[i][j]; ui[i][j] = ni[i][j]; }
    }
    const double* M = m64 + fi * 8;
    double re = 0.0;
    for (int ab = 0; ab < 4; ++ab) re += ur[ab >> 1][ab & 1] * M[2 * ab] - ui[ab >> 1][ab & 1] * M[2 * ab + 1];
    gsum += 2.0 * re;
  }
  return gsum;
}

}  // namespace qp
