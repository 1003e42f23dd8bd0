// Internal types shared by the planner (host C++) and the gfx950 kernels.
//
// All fields are 32-bit so that the kernels read them with scalar loads.
//
// Index conventions: a basis index j of an n-qubit state has qubit q in bit (n-1-q), so
// qubit 0 is the most significant bit.  "Logical" index = the index of the state the circuit
// defines.  In the fused kernels a thread owns 8 amplitudes of each statevector: its three
// "register" bits r0,r1,r2 plus n-3 "thread" bits u.  A round's mapping tpos[k] gives the
// logical index-bit position of physical bit k (k = 0..2 register bits, k >= 3 thread bit k-3).
#pragma once
#include <cstdint>

#if defined(__HIPCC__) || defined(__HIP__)
#define QP_HD __host__ __device__
#else
#define QP_HD
#endif

namespace qp {

// LDS index swizzle of the fused kernels: XOR the low nibble with the fold of all higher
// nibbles.  A bijection, and linear over GF(2): swz(a ^ b) = swz(a) ^ swz(b).
QP_HD inline constexpr uint32_t lds_swizzle(uint32_t idx) {
  return idx ^ (((idx >> 4) ^ (idx >> 8) ^ (idx >> 12) ^ (idx >> 16)) & 15u);
}

constexpr int kMaxQubits = 12;     // fused register/LDS kernels
constexpr int kMaxDevices = 64;    // per-device host-side state (launch attributes, scratch addresses)
constexpr int kMaxQubitsPlain = 14;
constexpr int kMaxOut = 8;
constexpr int kMaxTerms = 32;      // sign terms of one entangler stage
constexpr int kRegBits = 3;        // 8 amplitudes per thread per statevector
// Per fused gate the adjoint sweep accumulates S_k = Im <lambda|sigma_k|psi> (k = x, y, z) over
// all points and statevector pairs, stored as kGS floats/doubles per gate (the last unused).
constexpr int kGS = 4;
// Gate-table entry: U (8 floats, row-major complex) followed by U^H (8 floats), so that the
// adjoint reads its coefficients as they are used.
constexpr int kGT = 16;

// Swap slots of a round: after its three register-bit gates, register bit i (i < swap_slots(n))
// trades places with thread bit 4 + i (lane bit 4 or 5 of the wave, by a cross-lane swap of
// register pairs), and gate sgate[i] acts on the qubit brought in.  They are used where they turn
// a rotation stage into fewer rounds without identity slots (8 qubits: 4 + 4; 10 qubits: 5 + 5
// instead of 3 + 3 + 3 + 1; 12 qubits: 4 + 4 + 4 instead of 3 + 3 + 3 + 3).  At 6 and 9 qubits
// three-gate rounds are already full and at 11 a slot would stay empty; at 12, two swap slots
// (5 + 5 + 2) were slower than none.
QP_HD inline constexpr int swap_slots(int n) { return n == 10 ? 2 : ((n == 8 || n == 12) ? 1 : 0); }

// Threads per workgroup of the fused kernels (a thread holds 8 amplitudes of each statevector).
QP_HD inline constexpr int fused_wg_threads(int n) { return n == 12 ? 512 : 256; }

struct alignas(16) QRound {
  int32_t gate[3];    // fused-gate id applied on register bit b in the round's input mapping (-1: none)
  int32_t phase;      // phase stage applied after the exchange into this round (-1: none)
  int32_t sgate[2];   // fused-gate id applied on register bit i after swap slot i (-1: none)
  int32_t pad1[2];
  int32_t tpos[16];   // input mapping: logical index-bit position of physical bit k
  int32_t tpost[16];  // output mapping (tpos with the swap slots applied)
};
// One direction of the register exchange that precedes a round.  Reader thread (u, r) in the
// read mapping holds logical index jn = base(u) ^ jr(r); it takes the amplitude stored at
// src = A jn (A over GF(2), given by its columns), times (-1)^Q(x), where x = jn (sign in the
// destination coordinates) or x = src (sign in the source coordinates) and
// Q(x) = XOR_t parity(qu[t] & x) * parity(qv[t] & x).
struct alignas(16) QXchg {
  uint32_t acol[16];
  uint32_t src_r[8];  // A jr(r): uniform part of the source index
  uint32_t qu[kMaxTerms];
  uint32_t qv[kMaxTerms];
  uint32_t ue[3];     // bit t: parity(qu[t] & x_e(i)) for register basis i (uniform)
  uint32_t ve[3];
  uint32_t nterms;
  uint32_t sign_at_src;
  uint32_t qsign_r;   // bit r: Q(x_r) for the uniform part x_r
  uint32_t identity;  // A = I and no sign terms
  uint32_t pad1[2];
  // LDS layout of the exchange: logical index j sits at entry swz(pbase ^ M j), M an invertible
  // GF(2) map of the n index bits (columns mcol) that the planner chooses per exchange so that
  // every group of 16 lanes hits 16 distinct banks when writing and when reading.
  uint32_t roff[8];   // 8 swz(M A jr(r)): register r's uniform source offset in bytes, reader side
  uint32_t woff[8];   // 8 swz(M jr(r)): register r's offset in the writer's mapping, in bytes
  uint32_t mcol[16];
};
static_assert(sizeof(QXchg) == 528, "QXchg layout");

// Per-lane words of one exchange for the thread u of a point (u < 2^(n-3)): the writer's and the
// reader's LDS byte bases 8 swz(thread part of the index) in their mappings (the reader's through
// the index map A), and bit r set where register r's amplitude changes sign.  A point's base
// index pbase enters as 8 swz(pbase), XORed into both bases (swz is linear over GF(2)).
struct alignas(16) QLane {
  uint32_t wb, rb, sgn, pad;
};
static_assert(sizeof(QRound) == 160, "QRound layout");

// Fused single-qubit gate: U = R_{c-1} ... R_1 R_0 (component 0 acts first).  stat_out: the
// gate belongs to the leading rotation stage, which acts on the product state and is folded into
// the encoding; its statistic is taken at the gate output instead of the input.
struct alignas(16) QFused {
  int32_t qubit;
  int32_t ncomp;
  int32_t kind[3];
  int32_t param[3];
  int32_t stat_out;
};
static_assert(sizeof(QFused) == 48, "QFused layout");

// Phase stage: a run of CRZ gates (with any CZ of the same stage), all diagonal, applied as one
// phase e^{i phi(j)} per basis index after the exchange that precedes a round.  With
// CRZ(c, t)(theta) = |0><0|_c (x) I + |1><1|_c (x) RZ_t(theta),
//   phi(j) = sum_(c,t) theta_ct (-1/2) b_c(j) (1 - 2 b_t(j)) = sum_q alpha_q b_q + sum_(q<q') beta_qq' b_q b_q',
//   alpha_q = -(1/2) sum_t theta_qt,  beta_qq' = theta_qq' + theta_q'q.
// The coefficients are kept as unsigned 32-bit fractions of a turn (2 pi = 2^32), so phases add
// exactly modulo 2 pi.  Per stage: n alpha's then the n(n-1)/2 beta's (pairs q < q' in row order),
// at coef_off (in 32-bit words) of the phase table that follows the gate table.  The adjoint
// accumulates the moments M_q = sum_j w_j b_q and M_qq' = sum_j w_j b_q b_q' of
// w_j = Im(conj(lambda_j) psi_j) + sum_c Im(conj(mu_c,j) dpsi_c,j) at the stage output (same
// order, at mom_off among the phase moments), and dL/dtheta_ct = M_c - 2 M_ct.
struct alignas(16) QPhaseStage {
  int32_t gate0, ngates;  // range in the QPhaseGate array
  int32_t coef_off;       // first coefficient (32-bit words) in the phase table
  int32_t mom_off;        // first moment among the phase moments
};
struct alignas(16) QPhaseGate {
  int32_t c, t, param, pad;   // control and target qubits, parameter index
};
QP_HD inline constexpr int phase_pair_index(int n, int a, int b) {   // a < b
  return a * n - a * (a + 1) / 2 + (b - a - 1);
}
QP_HD inline constexpr int phase_terms(int n) { return n + n * (n - 1) / 2; }

// Fused-kernel modes.  The packed modes carry no input tangents: the four statevector slots of a
// thread group hold four consecutive points (forward: outputs only; VJP: output seeds only, the
// adjoint slots holding each point's lambda), so a point costs a quarter of a tangent-carrying one.
// kModeTotal: the Maxwell step of the paper's total loss over the collocation points (residual,
// energy and symmetry seeds formed in the kernel; the mirror images' outputs come from memory).
enum Mode : int { kModeFwd = 0, kModeMaxwell = 1, kModeVjp = 2, kModeFwdPk = 3, kModeVjpPk = 4, kModeTotal = 5 };
QP_HD inline constexpr bool mode_packed(int mode) { return mode == kModeFwdPk || mode == kModeVjpPk; }
QP_HD inline constexpr bool mode_fwd_only(int mode) { return mode == kModeFwd || mode == kModeFwdPk; }

// Dense 2^5 blocks (MFMA path): a contiguous run of gates acting on at most five qubits.
constexpr int kDenseK = 5;
struct alignas(16) QDenseGate {
  int32_t kind, lq0, lq1, param;   // local qubit bits inside the block (0..4)
};
struct alignas(16) QDenseGroup {
  int32_t pos[kDenseK];   // logical index-bit position of block bit i
  int32_t gate0, ngates;  // range in the QDenseGate array
  int32_t pad;
};

// Plan header uploaded to the device (followed by the arrays at the given byte offsets).
struct alignas(16) QPlanDev {
  int32_t n, n_params, n_out, n_fused, n_rounds;
  int32_t enc_kind, enc_gate, enc_scale, n_feat;
  int32_t coord_of_qubit[16];
  uint32_t zmask[kMaxOut];          // readout parity mask of output i (trailing entangler folded)
  int32_t off_rounds;               // QRound[n_rounds]
  int32_t off_xf;                   // QXchg[n_rounds]  forward exchange before round k (k>=1)
  int32_t off_xb;                   // QXchg[n_rounds]  inverse exchange after round k (k>=1)
  int32_t off_fused;                // QFused[n_fused]
  int32_t off_csr_ptr;              // int32[n_params+1]
  int32_t off_csr_idx;              // int32[nnz]: fused*4 + component
  int32_t off_rff_B;                // float[F][3]
  int32_t off_rff_W;                // float[n][2F]
  int32_t bytes;
  int32_t n_dgroups;                // dense groups (0: no dense plan)
  int32_t off_dgroups;              // QDenseGroup[n_dgroups]
  int32_t off_dgates;               // QDenseGate[...]
  int32_t n_docc;                   // parametrised gates inside dense groups
  int32_t off_docc;                 // int32[n_docc][2]: group, gate index
  int32_t off_dcsr_ptr;             // int32[n_params+1] over the occurrences
  int32_t off_dcsr_idx;             // int32[n_docc]
  uint32_t zplain[kMaxOut];         // readout parity mask of output i without folding
  int32_t n_head;                   // leading rounds folded into the encoding (rounds 0 .. n_head-1; < n_rounds)
  int32_t head_gate[16];            // per qubit: fused gate of the leading stage, -1 if none
  int32_t off_lanes;                // QLane[2][n_rounds][2^(n-3)]: forward (0) and reverse (1) exchanges
  int32_t n_phase;                  // phase stages (CRZ runs)
  int32_t off_phase;                // QPhaseStage[n_phase]
  int32_t off_phase_gates;          // QPhaseGate[...]
  int32_t n_phase_coef;             // 32-bit words of the phase table (n_phase * phase_terms(n))
  int32_t n_moments;                // phase moments accumulated by the adjoint (same count)
  int32_t off_pcsr_ptr;             // int32[n_params+1]: parameter -> CRZ occurrences
  int32_t off_pcsr_idx;             // int32[...]: phase-gate index
  int32_t pad_end;
};

}  // namespace qp
