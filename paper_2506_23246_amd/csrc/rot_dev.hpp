// 2x2 complex helpers for gate tables and gradient contraction, as explicit scalars.
// A 2x2 complex matrix is 8 reals, row-major: u00r, u00i, u01r, u01i, u10r, u10i, u11r, u11i.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/qpinn.h"

namespace qp {

// u <- R_P(theta) u with R_P(theta) = c I - i s P, c = cos(theta/2), s = sin(theta/2).
template <typename T>
__host__ __device__ inline void left_mul_rot(int kind, T c, T s, T* u) {
  T n[8];
  if (kind == QP_RX) {         // [[c, -i s], [-i s, c]];  (-i s)(a + i b) = s b - i s a
    n[0] = c * u[0] + s * u[5]; n[1] = c * u[1] - s * u[4];
    n[2] = c * u[2] + s * u[7]; n[3] = c * u[3] - s * u[6];
    n[4] = c * u[4] + s * u[1]; n[5] = c * u[5] - s * u[0];
    n[6] = c * u[6] + s * u[3]; n[7] = c * u[7] - s * u[2];
  } else if (kind == QP_RY) {  // [[c, -s], [s, c]]
    n[0] = c * u[0] - s * u[4]; n[1] = c * u[1] - s * u[5];
    n[2] = c * u[2] - s * u[6]; n[3] = c * u[3] - s * u[7];
    n[4] = s * u[0] + c * u[4]; n[5] = s * u[1] + c * u[5];
    n[6] = s * u[2] + c * u[6]; n[7] = s * u[3] + c * u[7];
  } else {                     // diag(c - i s, c + i s)
    n[0] = c * u[0] + s * u[1]; n[1] = c * u[1] - s * u[0];
    n[2] = c * u[2] + s * u[3]; n[3] = c * u[3] - s * u[2];
    n[4] = c * u[4] - s * u[5]; n[5] = c * u[5] + s * u[4];
    n[6] = c * u[6] - s * u[7]; n[7] = c * u[7] + s * u[6];
  }
  for (int e = 0; e < 8; ++e) u[e] = n[e];
}

// u <- (-i/2) P u, so that applying left_mul_rot then this gives d/dtheta of R_P(theta) u.
template <typename T>
__host__ __device__ inline void left_mul_mhalf_i_pauli(int kind, T* u) {
  T n[8];
  const T h = T(0.5);
  if (kind == QP_RX) {         // rows swap, then (a + i b)(-i/2) = b/2 - i a/2
    n[0] = h * u[5]; n[1] = -h * u[4]; n[2] = h * u[7]; n[3] = -h * u[6];
    n[4] = h * u[1]; n[5] = -h * u[0]; n[6] = h * u[3]; n[7] = -h * u[2];
  } else if (kind == QP_RY) {  // (-i/2)[[0,-i],[i,0]] = [[0,-1/2],[1/2,0]]
    n[0] = -h * u[4]; n[1] = -h * u[5]; n[2] = -h * u[6]; n[3] = -h * u[7];
    n[4] = h * u[0]; n[5] = h * u[1]; n[6] = h * u[2]; n[7] = h * u[3];
  } else {                     // diag(-i/2, i/2)
    n[0] = h * u[1]; n[1] = -h * u[0]; n[2] = h * u[3]; n[3] = -h * u[2];
    n[4] = -h * u[5]; n[5] = h * u[4]; n[6] = -h * u[7]; n[7] = h * u[6];
  }
  for (int e = 0; e < 8; ++e) u[e] = n[e];
}

// Writes U and U^H (rounded to float) to a gate-table entry o[0..15].
template <typename T>
__host__ __device__ inline void store_gate_entry(float* o, const T* u) {
  for (int e = 0; e < 8; ++e) o[e] = (float)u[e];
  o[8] = (float)u[0];  o[9] = -(float)u[1];    // (0,0) <- conj u00
  o[10] = (float)u[4]; o[11] = -(float)u[5];   // (0,1) <- conj u10
  o[12] = (float)u[2]; o[13] = -(float)u[3];   // (1,0) <- conj u01
  o[14] = (float)u[6]; o[15] = -(float)u[7];   // (1,1) <- conj u11
}

template <typename T>
__host__ __device__ inline void set_identity(T* u) {
  u[0] = T(1); u[1] = T(0); u[2] = T(0); u[3] = T(0);
  u[4] = T(0); u[5] = T(0); u[6] = T(1); u[7] = T(0);
}

}  // namespace qp
