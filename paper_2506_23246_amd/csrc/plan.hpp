// Host-side circuit planner: validation, gate fusion, entangler algebra over GF(2), round
// schedule for the register/LDS kernels and the device image of the plan.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qpinn.h"
#include "qp_internal.hpp"

namespace qp {

struct HostPlan {
  int n = 0, K = 0, m = 0;
  std::vector<qp_gate> gates;          // the raw gate list (plain path)
  std::vector<int32_t> out_qubits;
  int enc_kind = 0, enc_gate = 0, enc_scale = 0, n_feat = 0;
  int coord[16] = {0};
  std::vector<float> rffB, rffW;

  // fused-path plan
  bool fused_ok = false;
  std::string fused_reason;
  std::vector<QFused> fused;
  std::vector<QRound> rounds;
  std::vector<QXchg> xf, xb;          // indexed by round (entry 0 unused)
  std::vector<QLane> lanes;            // [2][rounds][2^(n-3)] per-lane exchange words
  uint32_t zmask[kMaxOut] = {0};
  std::vector<int32_t> csr_ptr, csr_idx;
  int n_exchanges = 0;                 // exchanges that move data
  bool has_signs = false;              // some exchange carries CZ signs
  std::vector<QPhaseStage> phases;     // CRZ phase stages, by exchange
  std::vector<QPhaseGate> phase_gates;
  std::vector<int32_t> pcsr_ptr, pcsr_idx;
  int n_head = 0;                      // leading rounds folded into the encoding
  int32_t head_gate[16];               // per qubit: its leading-stage fused gate, or -1
  // dense-block plan (MFMA path)
  bool dense_ok = false;
  std::vector<QDenseGroup> dgroups;
  std::vector<QDenseGate> dgates;
  std::vector<int32_t> docc, dcsr_ptr, dcsr_idx;
  std::vector<unsigned char> blob;     // QPlanDev + arrays (device image)
};

// Returns "" on success, else a message; *status receives the qp_status to return.
std::string build_plan(const qp_circuit_desc* d, HostPlan* hp, int* status);

// GF(2) helpers (exposed for the self-check in the test suite through the C API only).
uint32_t gf2_apply(const uint32_t* cols, int n, uint32_t x);

}  // namespace qp
