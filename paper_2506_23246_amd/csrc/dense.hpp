// Dense-block MFMA path (dense.hip): launch description and workspace layout.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"

namespace qp {

struct DenseLoss {
  int maxwell;            // 1: Maxwell seeds; 0: VJP seeds from d_out / d_tan
  int kind, loss_sum;
  float eps_r, x_if, w_all;
  const int* counts;      // [2] dielectric counts (split loss)
  const float* points;
  const float* d_out;
  const float* d_tan;
};

struct DenseLayout { size_t tabF, tabA, X, enc, seeds, zpart, lterm, mpart, m64, contrib, angles, jac, counts, total; };

struct DenseCall {
  const QPlanDev* plan;
  int n, m, G, K, n_docc;
  const float* params;
  const float* points;
  const float* angles;
  const float* jac;
  long long P;
  int Pc, nwg, apply_grid;
  bool grad;
  DenseLoss loss;
  float* out;
  float* tan;
  double* loss_out;
  float* d_params;
  void* ws;
  DenseLayout L;
};

DenseLayout dense_layout(int n, int m, int G, int n_docc, long long P, int Pc, int nwg, bool grad);
int dense_chunk(int n, long long P, bool grad);
hipError_t dense_run(const DenseCall& c, hipStream_t st);

}  // namespace qp
