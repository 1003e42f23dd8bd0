// Launch interface of the total-loss kernels (total.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"

namespace qp {

struct TotalSeedArgs {
  const float* out;       // [P_ext][m] outputs of the extended set [X; X_my; X_mx; X_0]
  const float* tan;       // [P][m][3] input tangents of the collocation points
  const float* points;    // [P][3] collocation points X
  const float* ic_xy;     // [P0][2]
  long long P, P0;
  long long ic_base;      // row of the first initial-condition point in the extended set
  int m;
  int with_mx;            // x-mirror terms (vacuum)
  int phys_kind;
  float eps_r, x_if;
  const int* counts;      // [2] vacuum / dielectric point counts (split loss)
  float w_ic, w_sym, w_energy, ic_a;
  float* d_out;           // [P_ext][m] seeds d L_tot / d f
  float* d_tan;           // [P][m][3] seeds d L_tot / d g (collocation points only)
  float* part;            // [blocks][4] FP32 partial sums: phys, ic, sym, energy
  double* terms;          // [5] total, phys, ic, sym, energy
};

int total_seed_blocks(long long P, long long P0);
hipError_t launch_total_points(const float* pts, long long P, const float* ic_xy, long long P0, int with_mx, float* ext,
                               hipStream_t st);
hipError_t launch_total_seeds(const TotalSeedArgs& a, hipStream_t st);
// y[i] += x[i], i < n
hipError_t launch_add(float* y, const float* x, int n, hipStream_t st);

}  // namespace qp
