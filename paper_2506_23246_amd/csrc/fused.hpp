// Launch interface of the fused register/LDS kernels (fused.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"

namespace qp {

struct FusedArgs {
  const QPlanDev* plan;
  const float* gtab;      // [F + 1][kGT] fused gate matrices U, U^H (entry F: identity)
  const float* points;    // [P][3]
  const float* angles;    // [P][n]   (angle-given or RFF encodings)
  const float* jac;       // [P][n][3]
  long long P;
  int ntiles;
  int n_fused;
  float* out;             // [P][m] or null
  float* tan;             // [P][m][3] or null
  const float* d_out;     // VJP seeds [P][m] or null
  const float* d_tan;     // VJP seeds [P][m][3] or null
  int loss_kind;
  int loss_sum;           // 1: plain sums (weights 1) instead of means
  float eps_r, x_if;
  const int* counts;      // [2]: points with x < x_if, points with x >= x_if
  float* mpart;           // [grid][F][8]
  float* lpart;           // [grid]
  float* d_angles;        // [P][n] dL/d angles (angle-given encoding) or null
  float* d_jac;           // [P][n][3] dL/d Jacobian or null
  int n_mom;              // phase-stage moments per workgroup partial (after the F * kGS statistics)
  const float* f_mir;     // kModeTotal: outputs of the mirror images [n_mir][P][m] (y-mirror first)
  int n_mir;              // kModeTotal: 1 (y-mirror) or 2 (and x-mirror)
  float w_sym, w_energy;  // kModeTotal: weights of the symmetry and energy terms
};

int fused_threads(int n);
// Largest persistent grid, in workgroups per CU, that a launch may ask for: one 512-thread
// workgroup (12 qubits) or four 256-thread ones.  About 256 VGPRs per lane keep two waves per
// SIMD resident, so a grid above two 256-thread workgroups per CU runs in generations.
int fused_max_wg_per_cu(int n);
int fused_points_per_tile(int n);
size_t fused_lds_bytes(int n, int exs, int n_fused, int n_mom);
hipError_t launch_fused(int n, int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st);
// Gate table [F + 1][kGT] and, after it, the phase-stage coefficients (n_phase_coef words).
hipError_t launch_gate_table(const QPlanDev* plan, int n_fused, int n_phase_coef, const float* params, float* gtab,
                             int fp32, hipStream_t st);
hipError_t launch_rff(const QPlanDev* plan, const float* points, long long P, float* angles, float* jac, hipStream_t st);
hipError_t launch_count(const float* points, long long P, float x_if, int* counts, hipStream_t st);
hipError_t launch_reduce(const float* mpart, int nblk, int ncol, const float* lpart, double* m64, double* loss, hipStream_t st);
hipError_t launch_param_grads(const QPlanDev* plan, int K, const float* params, const double* m64, float* grads, hipStream_t st);

}  // namespace qp
