// Plain per-gate baseline (plain.hip): problem description and entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/qpinn.h"

namespace qp {

struct PlainGate { int32_t kind, q0, q1, param; };

struct PlainEnc {
  int n, kind, gate, scale, nf;
  int coord[16];
  const float* B;    // device [nf][3] (RFF)
  const float* W;    // device [n][2 nf] (RFF)
};

struct PlainOut { int q[8]; };

struct PlainProblem {
  PlainEnc enc;
  int m, K, n_gates;
  PlainOut oq;
  const PlainGate* gates_dev;   // device copy (for the gate-table kernel)
  const PlainGate* gates_host;  // host copy (launch loop)
  long long P;
};

struct PlainLayout {
  size_t off_tab, off_theta, off_state, off_fp, off_fm, off_out, off_tan, off_pbuf, off_loss, total;
};

PlainLayout plain_layout(const PlainProblem& pr, size_t real_bytes);
hipError_t plain_eval(const PlainProblem& pr, int prec, const void* params, const void* points, double h,
                      void* out, void* tan, void* ws, hipStream_t st);
// Per-qubit Bloch vectors [P][n][3] and Meyer-Wallach entanglement [P] (mw may be null) of the
// output states; angles [P][n] replaces the point encoding when given.
hipError_t plain_bloch(const PlainProblem& pr, int prec, const void* params, const void* points, const void* angles,
                       void* bloch, void* mw, void* ws, hipStream_t st);
hipError_t plain_maxwell(const PlainProblem& pr, int prec, const void* params, const void* points,
                         const qp_maxwell_desc& ld, int loss_sum, double h, double hp, int k0, int k1,
                         double* loss, void* dparams, void* ws, hipStream_t st);

}  // namespace qp
