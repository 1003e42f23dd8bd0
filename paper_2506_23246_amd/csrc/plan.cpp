// Circuit planner for the fused register/LDS kernels.
//
// A circuit is a time-ordered list of rotations (RX/RY/RZ) and entanglers (CNOT/CZ/CRZ).  The
// planner
//   1. fuses consecutive rotations on one qubit into one 2x2 gate (up to three components,
//      e.g. RZ(omega) RY(theta) RZ(phi) of the Rot gate, eq. rot_gate);
//   2. turns every maximal run of CNOT/CZ gates into one affine stage
//         psi_out(j') = (-1)^Q(j') psi_in(A j'),
//      with A an invertible GF(2) matrix on index bits and Q a quadratic form (a CNOT ring is a
//      pure index permutation, a CZ ring a pure sign function); the CRZ gates of a run (after its
//      CNOTs; all diagonal, so they commute) become one phase stage e^{i phi(j)}, phi quadratic in
//      the index bits with parameter-linear coefficients (the Cross-Mesh layers, eq. crz_cross_mesh);
//   3. groups the fused gates of every rotation stage into rounds of three qubits (the three
//      register bits of a thread) and attaches each entangler stage to the register exchange
//      that precedes the next round; a trailing stage is folded into the readout masks.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <map>

namespace qp {

namespace {

inline int popc(uint32_t x) { return __builtin_popcount(x); }
inline uint32_t par(uint32_t x) { return popc(x) & 1u; }

struct Affine {            // psi_out(j') = (-1)^Q(j') psi_in(A j')
  int n = 0;
  uint32_t acol[16];
  std::vector<std::pair<uint32_t, uint32_t>> terms;
  void init(int nn) {
    n = nn;
    for (int k = 0; k < 16; ++k) acol[k] = (k < n) ? (1u << k) : 0u;
    terms.clear();
  }
  // Append CNOT(control bit bc, target bit bt): A <- A X, Q <- Q o X.
  void cnot(int bc, int bt) {
    acol[bc] ^= acol[bt];
    for (auto& t : terms) {
      if ((t.first >> bt) & 1u) t.first ^= (1u << bc);
      if ((t.second >> bt) & 1u) t.second ^= (1u << bc);
    }
  }
  void cz(int ba, int bb) { terms.emplace_back(1u << ba, 1u << bb); }
  bool is_identity() const {
    for (int k = 0; k < n; ++k)
      if (acol[k] != (1u << k)) return false;
    return terms.empty();
  }
};

uint32_t apply_cols(const uint32_t* cols, int n, uint32_t x) {
  uint32_t y = 0;
  for (int k = 0; k < n; ++k)
    if ((x >> k) & 1u) y ^= cols[k];
  return y;
}

// Inverse of an invertible GF(2) matrix given by columns.
bool gf2_inverse(const uint32_t* cols, int n, uint32_t* inv) {
  // rows of [A | I]
  uint32_t rowsA[16], rowsI[16];
  for (int i = 0; i < n; ++i) {
    rowsA[i] = 0;
    for (int k = 0; k < n; ++k)
      if ((cols[k] >> i) & 1u) rowsA[i] |= (1u << k);
    rowsI[i] = 1u << i;
  }
  for (int c = 0; c < n; ++c) {
    int piv = -1;
    for (int r = c; r < n; ++r)
      if ((rowsA[r] >> c) & 1u) { piv = r; break; }
    if (piv < 0) return false;
    std::swap(rowsA[c], rowsA[piv]);
    std::swap(rowsI[c], rowsI[piv]);
    for (int r = 0; r < n; ++r)
      if (r != c && ((rowsA[r] >> c) & 1u)) { rowsA[r] ^= rowsA[c]; rowsI[r] ^= rowsI[c]; }
  }
  for (int k = 0; k < n; ++k) {   // columns of the inverse from its rows
    inv[k] = 0;
    for (int i = 0; i < n; ++i)
      if ((rowsI[i] >> k) & 1u) inv[k] |= (1u << i);
  }
  for (int k = n; k < 16; ++k) inv[k] = 0;
  return true;
}

uint32_t qform(const std::vector<std::pair<uint32_t, uint32_t>>& terms, uint32_t x) {
  uint32_t s = 0;
  for (auto& t : terms) s ^= par(t.first & x) & par(t.second & x);
  return s;
}

// Thread-bit order for a round: register bits first, then any fixed thread-bit placements
// (qubits of the swap slots), then the remaining positions chosen so that each group of four
// consecutive lane bits lands on distinct position residues mod 4 (the LDS swizzle folds higher
// nibbles into the low four bits).  fixed[k] >= 0 pins thread position k (k >= 3).
void make_tpos(int n, const int reg[3], const int* fixed, int32_t* tpos) {
  bool used[16] = {false};
  for (int k = 0; k < 16; ++k) tpos[k] = -1;
  for (int i = 0; i < 3; ++i) { tpos[i] = reg[i]; used[reg[i]] = true; }
  for (int k = 3; k < n; ++k)
    if (fixed && fixed[k] >= 0) { tpos[k] = fixed[k]; used[fixed[k]] = true; }
  int group_mask = 0;
  for (int k = 3; k < n; ++k) {
    if (((k - 3) & 3) == 0) {
      group_mask = 0;
      for (int j = k; j < k + 4 && j < n; ++j)
        if (tpos[j] >= 0) group_mask |= 1 << (tpos[j] & 3);
    }
    if (tpos[k] >= 0) continue;
    int pick = -1;
    for (int p = 0; p < n; ++p)
      if (!used[p] && !((group_mask >> (p & 3)) & 1)) { pick = p; break; }
    if (pick < 0)
      for (int p = 0; p < n; ++p)
        if (!used[p]) { pick = p; break; }
    used[pick] = true;
    group_mask |= 1 << (pick & 3);
    tpos[k] = pick;
  }
  for (int k = n; k < 16; ++k) tpos[k] = 0;
}

uint32_t jr_of(const int32_t* tpos, int r) {
  return ((uint32_t)(r & 1) << tpos[0]) | ((uint32_t)((r >> 1) & 1) << tpos[1]) |
         ((uint32_t)((r >> 2) & 1) << tpos[2]);
}

void fill_xchg(QXchg* X, int n, const uint32_t* Acols, const Affine& aff, bool sign_at_src,
               const int32_t* read_tpos) {
  std::memset(X, 0, sizeof(QXchg));
  for (int k = 0; k < 16; ++k) X->acol[k] = k < n ? Acols[k] : 0u;
  for (int r = 0; r < 8; ++r) X->src_r[r] = apply_cols(Acols, n, jr_of(read_tpos, r));
  X->nterms = (uint32_t)aff.terms.size();
  for (size_t t = 0; t < aff.terms.size(); ++t) {
    X->qu[t] = aff.terms[t].first;
    X->qv[t] = aff.terms[t].second;
  }
  X->sign_at_src = sign_at_src ? 1 : 0;
  for (int i = 0; i < 3; ++i) {
    uint32_t xe = jr_of(read_tpos, 1 << i);
    if (sign_at_src) xe = apply_cols(Acols, n, xe);
    uint32_t ue = 0, ve = 0;
    for (size_t t = 0; t < aff.terms.size(); ++t) {
      ue |= par(aff.terms[t].first & xe) << t;
      ve |= par(aff.terms[t].second & xe) << t;
    }
    X->ue[i] = ue;
    X->ve[i] = ve;
  }
  uint32_t qs = 0;
  for (int r = 0; r < 8; ++r) {
    uint32_t xr = sign_at_src ? X->src_r[r] : jr_of(read_tpos, r);
    qs |= qform(aff.terms, xr) << r;
  }
  X->qsign_r = qs;
  bool ident = aff.terms.empty();
  for (int k = 0; k < n; ++k) ident = ident && (Acols[k] == (1u << k));
  X->identity = ident ? 1u : 0u;
}

// Thread part of the logical index of thread u in mapping map (thread bit k - 3 at position map[k]).
uint32_t deposit_host(uint32_t u, const int32_t* map, int n) {
  uint32_t j = 0;
  for (int k = 3; k < n; ++k) j |= ((u >> (k - 3)) & 1u) << map[k];
  return j;
}

// ---- LDS layout of one exchange --------------------------------------------------------------
// Logical index j is stored at entry swz(pbase ^ M j).  The 64-bit accesses of a group of 16 lanes
// are served without bank conflicts when the low four bits of their entries are distinct (the
// model the measured conflict counters support; a 32-lane, five-bit criterion raised them 4.6x).
// Each access of a register r adds a uniform offset, which does not change distinctness, so what
// matters is the thread part: the writer's deposit of the thread id and the reader's source index
// A jn.  The planner picks M per exchange: the identity if it already gives distinct banks, else
// the best of a deterministic sequence of candidates (bit permutations, some with extra XORs of
// low bits), keeping M invertible.
struct MapSearch {
  uint32_t state = 0x9E3779B9u;
  uint32_t next() {   // xorshift32
    state ^= state << 13; state ^= state >> 17; state ^= state << 5;
    return state;
  }
};

bool gf2_invertible(const uint32_t* cols, int n) {
  uint32_t inv[16];
  return gf2_inverse(cols, n, inv);
}

// Sum and minimum over the 16-lane groups of a workgroup of the number of distinct banks (low four
// bits of the entry), writer side and reader side.
void bank_score(int n, int T, const uint32_t* M, const std::vector<uint32_t>& wj,
                const std::vector<uint32_t>& rj, int* minv, int* sum) {
  const int TP = 1 << (n - 3);
  *minv = 64;
  *sum = 0;
  for (int side = 0; side < 2; ++side) {
    const std::vector<uint32_t>& J = side ? rj : wj;
    for (int h0 = 0; h0 < T; h0 += 16) {
      uint32_t seen = 0;
      for (int t = h0; t < h0 + 16 && t < T; ++t) {
        const uint32_t pbase = (uint32_t)(t / TP) << n;
        seen |= 1u << (lds_swizzle(pbase ^ apply_cols(M, n, J[t % TP])) & 15u);
      }
      const int d = __builtin_popcount(seen);
      *minv = std::min(*minv, d);
      *sum += d;
    }
  }
}

void choose_index_map(int n, int T, const int32_t* wmap, const int32_t* rmap, const uint32_t* Acols, int salt,
                      uint32_t* M) {
  const int TP = 1 << (n - 3);
  std::vector<uint32_t> wj(TP), rj(TP);
  for (int u = 0; u < TP; ++u) {
    wj[u] = deposit_host((uint32_t)u, wmap, n);
    rj[u] = apply_cols(Acols, n, deposit_host((uint32_t)u, rmap, n));
  }
  const int target = std::min(16, T);
  uint32_t best[16];
  for (int k = 0; k < 16; ++k) best[k] = k < n ? (1u << k) : 0u;
  int bmin, bsum;
  bank_score(n, T, best, wj, rj, &bmin, &bsum);
  MapSearch rng;
  rng.state ^= (uint32_t)salt * 0x85EBCA6Bu;
  for (int it = 0; it < 400 && bmin < target; ++it) {
    uint32_t cand[16];
    int perm[16];
    for (int k = 0; k < n; ++k) perm[k] = k;
    for (int k = n - 1; k > 0; --k) std::swap(perm[k], perm[rng.next() % (uint32_t)(k + 1)]);
    for (int k = 0; k < 16; ++k) cand[k] = k < n ? (1u << perm[k]) : 0u;
    if (it & 1) {   // add low-bit XORs to some columns
      for (int k = 0; k < n; ++k)
        if ((rng.next() & 3u) == 0) cand[k] ^= rng.next() & 15u & ((1u << n) - 1u);
      if (!gf2_invertible(cand, n)) continue;
    }
    int cmin, csum;
    bank_score(n, T, cand, wj, rj, &cmin, &csum);
    if (cmin > bmin || (cmin == bmin && csum > bsum)) {
      bmin = cmin;
      bsum = csum;
      for (int k = 0; k < 16; ++k) best[k] = cand[k];
    }
  }
  for (int k = 0; k < 16; ++k) M[k] = best[k];
}

// Register offsets of both sides in the exchange's LDS layout.
void set_lds_layout(QXchg* X, int n, const uint32_t* M, const int32_t* wmap, const int32_t* rmap, const uint32_t* Acols) {
  for (int k = 0; k < 16; ++k) X->mcol[k] = M[k];
  for (int r = 0; r < 8; ++r) {
    X->woff[r] = 8u * lds_swizzle(apply_cols(M, n, jr_of(wmap, r)));
    X->roff[r] = 8u * lds_swizzle(apply_cols(M, n, apply_cols(Acols, n, jr_of(rmap, r))));
  }
}

// Lane words of one exchange for thread u: the writer writes register r at wdep ^ jr_w(r); the
// reader's register r holds the amplitude of logical index j = jn ^ jr_r(r) in its mapping, read
// from A j and negated where Q(x) = 1, x = A j (sign in source coordinates) or x = j.
QLane lane_words(int n, const uint32_t* Acols, const Affine& aff, bool sign_at_src, const int32_t* wmap,
                 const int32_t* rmap, const uint32_t* M, uint32_t u) {
  QLane L{};
  const uint32_t wdep = deposit_host(u, wmap, n), jn = deposit_host(u, rmap, n);
  L.wb = 8u * lds_swizzle(apply_cols(M, n, wdep));
  L.rb = 8u * lds_swizzle(apply_cols(M, n, apply_cols(Acols, n, jn)));
  for (int r = 0; r < 8; ++r) {
    const uint32_t j = jn ^ jr_of(rmap, r);
    L.sgn |= qform(aff.terms, sign_at_src ? apply_cols(Acols, n, j) : j) << r;
  }
  return L;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

}  // namespace

uint32_t gf2_apply(const uint32_t* cols, int n, uint32_t x) { return apply_cols(cols, n, x); }

// Dense grouping for the MFMA path.  (1) Each rotation is delayed to just before the next
// two-qubit gate on its qubit (rotations commute with gates on other qubits), which keeps
// every qubit's own gate order and the order of the two-qubit gates.  (2) The reordered list is
// cut greedily into contiguous runs touching at most five qubits; each run becomes one 32x32
// block (runs on fewer qubits are padded with untouched qubits, i.e. identity factors).
static void build_dense(HostPlan* hp) {
  const int n = hp->n;
  hp->dense_ok = (n >= kDenseK && n <= kMaxQubits);
  hp->dgroups.clear();
  hp->dgates.clear();
  if (!hp->dense_ok) return;
  std::vector<qp_gate> order;
  std::vector<std::vector<qp_gate>> pend(n);
  for (const auto& g : hp->gates) {
    if (g.kind <= QP_RZ) { pend[g.q0].push_back(g); continue; }
    for (int q : {g.q0, g.q1}) {
      for (auto& r : pend[q]) order.push_back(r);
      pend[q].clear();
    }
    order.push_back(g);
  }
  for (int q = 0; q < n; ++q)
    for (auto& r : pend[q]) order.push_back(r);
  size_t i = 0;
  while (i < order.size()) {
    std::vector<int> qs;
    auto has = [&](int q) { return std::find(qs.begin(), qs.end(), q) != qs.end(); };
    QDenseGroup G{};
    G.gate0 = (int)hp->dgates.size();
    std::vector<qp_gate> run;
    while (i < order.size()) {
      const qp_gate& g = order[i];
      std::vector<int> add;
      if (!has(g.q0)) add.push_back(g.q0);
      if (g.kind >= QP_CNOT && !has(g.q1) && g.q1 != g.q0) add.push_back(g.q1);
      if ((int)(qs.size() + add.size()) > kDenseK) break;
      for (int q : add) qs.push_back(q);
      run.push_back(g);
      ++i;
    }
    // pad to five qubits with the lowest unused qubits, then order block bits by index bit
    for (int q = 0; q < n && (int)qs.size() < kDenseK; ++q)
      if (!has(q)) qs.push_back(q);
    std::sort(qs.begin(), qs.end(), [&](int a, int b) { return (n - 1 - a) < (n - 1 - b); });
    for (int b = 0; b < kDenseK; ++b) G.pos[b] = n - 1 - qs[b];
    auto local = [&](int q) {
      for (int b = 0; b < kDenseK; ++b)
        if (qs[b] == q) return b;
      return -1;
    };
    for (const auto& g : run) {
      QDenseGate d{};
      d.kind = g.kind;
      d.lq0 = local(g.q0);
      d.lq1 = g.kind >= QP_CNOT ? local(g.q1) : -1;
      d.param = (g.kind <= QP_RZ || g.kind == QP_CRZ) ? g.param : -1;
      hp->dgates.push_back(d);
    }
    G.ngates = (int)run.size();
    hp->dgroups.push_back(G);
  }
  // parameter -> (group, gate) occurrences
  hp->docc.clear();
  std::vector<std::vector<int>> per(hp->K);
  for (size_t gi = 0; gi < hp->dgroups.size(); ++gi) {
    const QDenseGroup& G = hp->dgroups[gi];
    for (int k = 0; k < G.ngates; ++k) {
      const QDenseGate& d = hp->dgates[G.gate0 + k];
      if (d.param >= 0) {
        per[d.param].push_back((int)hp->docc.size() / 2);
        hp->docc.push_back((int)gi);
        hp->docc.push_back(k);
      }
    }
  }
  hp->dcsr_ptr.assign(hp->K + 1, 0);
  hp->dcsr_idx.clear();
  for (int k = 0; k < hp->K; ++k) {
    for (int o : per[k]) hp->dcsr_idx.push_back(o);
    hp->dcsr_ptr[k + 1] = (int)hp->dcsr_idx.size();
  }
}

std::string build_plan(const qp_circuit_desc* d, HostPlan* hp, int* status) {
  *status = QP_EINVAL;
  if (!d) return "null circuit descriptor";
  const int n = d->n_qubits;
  if (n < 1 || n > kMaxQubitsPlain) { *status = QP_EUNSUPPORTED; return "n_qubits out of range 1..14"; }
  if (d->n_params < 0) return "n_params < 0";
  if (d->n_gates < 0 || (d->n_gates > 0 && !d->gates)) return "bad gate array";
  if (d->n_out < 1 || d->n_out > kMaxOut || !d->out_qubits) { *status = QP_ESHAPE; return "n_out must be 1..8 with out_qubits"; }
  hp->n = n;
  hp->K = d->n_params;
  hp->m = d->n_out;
  hp->out_qubits.assign(d->out_qubits, d->out_qubits + d->n_out);
  for (int q : hp->out_qubits)
    if (q < 0 || q >= n) return "output qubit out of range";
  hp->gates.assign(d->gates, d->gates + d->n_gates);
  for (const auto& g : hp->gates) {
    if (g.kind < QP_RX || g.kind > QP_CRZ) return "unknown gate kind";
    if (g.q0 < 0 || g.q0 >= n) return "gate qubit out of range";
    if (g.kind >= QP_CNOT) {
      if (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0) return "two-qubit gate needs distinct qubits in range";
    }
    if (g.kind <= QP_RZ || g.kind == QP_CRZ) {
      if (g.param < 0 || g.param >= d->n_params) return "parameter index out of range";
    }
  }
  // encoding
  const qp_encoding& e = d->enc;
  hp->enc_kind = e.kind;
  hp->enc_gate = e.gate;
  hp->enc_scale = e.scale;
  if (e.kind < QP_ENC_CYCLE || e.kind > QP_ENC_RFF) return "unknown encoding kind";
  if (e.gate != QP_ENC_RY && e.gate != QP_ENC_RX) return "unknown encoding gate";
  if (e.scale < QP_SCALE_NONE || e.scale > QP_SCALE_ACOS) return "unknown scaling";
  for (int q = 0; q < 16; ++q) hp->coord[q] = q % 3;
  if (e.kind == QP_ENC_CYCLE && e.coord_of_qubit) {
    for (int q = 0; q < n; ++q) {
      if (e.coord_of_qubit[q] < 0 || e.coord_of_qubit[q] > 2) return "coord_of_qubit must be 0..2";
      hp->coord[q] = e.coord_of_qubit[q];
    }
  }
  if (e.kind == QP_ENC_RFF) {
    if (e.n_features < 1 || e.n_features > 4096 || !e.rff_B || !e.rff_W) return "RFF needs 1..4096 features and B, W";
    hp->n_feat = e.n_features;
    hp->rffB.assign(e.rff_B, e.rff_B + 3 * e.n_features);
    hp->rffW.assign(e.rff_W, e.rff_W + (size_t)n * 2 * e.n_features);
  }
  *status = QP_OK;

  // ---------------- fused plan ----------------
  hp->fused_ok = true;
  if (n < 3 || n > kMaxQubits) { hp->fused_ok = false; hp->fused_reason = "fused kernels support 3..12 qubits"; }

  struct Stage {
    bool rot;
    std::map<int, int> fused_of_qubit;   // qubit -> index into hp->fused
    std::vector<int> order;              // fused ids in creation order
    Affine aff;
    std::vector<QPhaseGate> phase;       // CRZ gates of an entangler stage (after its CNOT map)
  };
  std::vector<Stage> stages;
  hp->fused.clear();
  for (const auto& g : hp->gates) {
    if (g.kind <= QP_RZ) {
      bool need_new = stages.empty() || !stages.back().rot;
      if (!need_new) {
        auto it = stages.back().fused_of_qubit.find(g.q0);
        if (it != stages.back().fused_of_qubit.end() && hp->fused[it->second].ncomp >= 3) need_new = true;
      }
      if (need_new) { stages.push_back(Stage{}); stages.back().rot = true; }
      Stage& s = stages.back();
      auto it = s.fused_of_qubit.find(g.q0);
      int fid;
      if (it == s.fused_of_qubit.end()) {
        QFused f{};
        f.qubit = g.q0;
        f.ncomp = 0;
        fid = (int)hp->fused.size();
        hp->fused.push_back(f);
        s.fused_of_qubit[g.q0] = fid;
        s.order.push_back(fid);
      } else {
        fid = it->second;
      }
      QFused& f = hp->fused[fid];
      f.kind[f.ncomp] = g.kind;
      f.param[f.ncomp] = g.param;
      f.ncomp++;
    } else if (g.kind == QP_CNOT || g.kind == QP_CZ || g.kind == QP_CRZ) {
      if (stages.empty() || stages.back().rot) {
        stages.push_back(Stage{});
        stages.back().rot = false;
        stages.back().aff.init(n);
      }
      Stage& st = stages.back();
      Affine& a = st.aff;
      const int b0 = n - 1 - g.q0, b1 = n - 1 - g.q1;
      if (g.kind == QP_CRZ) {
        st.phase.push_back(QPhaseGate{g.q0, g.q1, g.param, 0});
      } else if (g.kind == QP_CNOT) {
        // the stage applies its index map, then its diagonal (CZ signs and CRZ phases commute
        // with each other); a CNOT after a CRZ would need the phase moved through the map
        if (!st.phase.empty()) { hp->fused_ok = false; hp->fused_reason = "a CNOT after a CRZ in one entangler stage"; }
        a.cnot(b0, b1);
      } else {
        a.cz(b0, b1);
      }
      if ((int)a.terms.size() > kMaxTerms) { hp->fused_ok = false; hp->fused_reason = "too many CZ terms in one entangler stage"; }
    }
  }
  // parameter -> (fused, component) lists
  hp->csr_ptr.assign(hp->K + 1, 0);
  for (const auto& f : hp->fused)
    for (int c = 0; c < f.ncomp; ++c) hp->csr_ptr[f.param[c] + 1]++;
  for (int k = 0; k < hp->K; ++k) hp->csr_ptr[k + 1] += hp->csr_ptr[k];
  hp->csr_idx.assign(hp->csr_ptr[hp->K], 0);
  {
    std::vector<int> fill(hp->csr_ptr.begin(), hp->csr_ptr.end() - 1);
    for (size_t fi = 0; fi < hp->fused.size(); ++fi)
      for (int c = 0; c < hp->fused[fi].ncomp; ++c)
        hp->csr_idx[fill[hp->fused[fi].param[c]]++] = (int)fi * 4 + c;
  }
  build_dense(hp);
  if (!hp->fused_ok) {   // no register rounds; the image still carries the dense plan
    hp->rounds.clear();
    hp->lanes.clear();
    for (int i = 0; i < hp->m; ++i) hp->zmask[i] = 1u << (n - 1 - hp->out_qubits[i]);
    goto image;
  }

  {
  // rounds
  hp->rounds.clear();
  std::vector<Affine> round_ent;    // entangler applied in the exchange before round k
  std::vector<bool> round_has_ent;
  std::vector<std::vector<QPhaseGate>> round_phase;   // CRZ phase applied after that exchange
  Affine pending;
  pending.init(n);
  bool have_pending = false;
  std::vector<QPhaseGate> pending_phase;
  const int nsw = swap_slots(n);
  auto push_round = [&](const int* gate_ids, const int* reg, const int* sgate_ids, const int* spos) {
    QRound R{};
    for (int i = 0; i < 3; ++i) R.gate[i] = gate_ids[i];
    int fixed[16];
    for (int k = 0; k < 16; ++k) fixed[k] = -1;
    for (int i = 0; i < 2; ++i) {
      R.sgate[i] = i < nsw ? sgate_ids[i] : -1;
      if (i < nsw) fixed[3 + 4 + i] = spos[i];
    }
    make_tpos(n, reg, fixed, R.tpos);
    for (int k = 0; k < 16; ++k) R.tpost[k] = R.tpos[k];
    for (int i = 0; i < nsw; ++i) std::swap(R.tpost[i], R.tpost[3 + 4 + i]);
    R.phase = -1;
    hp->rounds.push_back(R);
    round_ent.push_back(pending);
    round_has_ent.push_back(have_pending);
    round_phase.push_back(pending_phase);
    pending.init(n);
    have_pending = false;
    pending_phase.clear();
  };
  // any nsw distinct positions other than reg[] (for rounds whose swap slots carry no gate)
  auto free_spos = [&](const int* reg, int* spos) {
    int c = 0;
    for (int p = 0; p < n && c < nsw; ++p)
      if (p != reg[0] && p != reg[1] && p != reg[2]) spos[c++] = p;
  };
  hp->n_head = 0;
  for (int q = 0; q < 16; ++q) hp->head_gate[q] = -1;
  int stage0_rounds = 0;   // rounds of an opening rotation stage (nothing before it)
  for (size_t si = 0; si < stages.size(); ++si) {
    Stage& s = stages[si];
    if (!s.rot) {
      pending_phase = s.phase;   // (two entangler stages are never adjacent: consecutive gates share one)
      // compose: pending then s.aff  ->  psi(j) = sP(j') ... apply s after pending
      if (!have_pending) { pending = s.aff; have_pending = true; continue; }
      // composition of two affine stages: first P (A1, Q1) then S (A2, Q2):
      // psi2(j) = (-1)^Q2(j) psi1(A2 j) = (-1)^{Q2(j)+Q1(A2 j)} psi0(A1 A2 j)
      Affine c;
      c.init(n);
      for (int k = 0; k < n; ++k) c.acol[k] = apply_cols(pending.acol, n, s.aff.acol[k]);
      c.terms = s.aff.terms;
      for (auto& t : pending.terms) {   // Q1(A2 j): mask u -> A2^T u
        uint32_t u2 = 0, v2 = 0;
        for (int k = 0; k < n; ++k) {
          u2 |= par(t.first & s.aff.acol[k]) << k;
          v2 |= par(t.second & s.aff.acol[k]) << k;
        }
        c.terms.emplace_back(u2, v2);
      }
      pending = c;
      if ((int)pending.terms.size() > kMaxTerms) { hp->fused_ok = false; hp->fused_reason = "too many CZ terms"; return ""; }
      continue;
    }
    if (have_pending && hp->rounds.empty()) {   // leading entangler: empty round first
      int none[3] = {-1, -1, -1}, snone[2] = {-1, -1};
      int reg[3] = {0, 1, 2}, spos[2] = {0, 0};
      free_spos(reg, spos);
      Affine keep = pending;
      bool hk = have_pending;
      std::vector<QPhaseGate> kp = pending_phase;
      pending.init(n);
      have_pending = false;
      pending_phase.clear();
      push_round(none, reg, snone, spos);
      pending = keep;
      have_pending = hk;
      pending_phase = kp;
    }
    // fused gates of the stage sorted by qubit, in chunks of 3 + nsw: three on the register bits,
    // the rest on the swap slots
    std::vector<int> ids;
    for (auto& kv : s.fused_of_qubit) ids.push_back(kv.second);
    std::sort(ids.begin(), ids.end(), [&](int a, int b) { return hp->fused[a].qubit < hp->fused[b].qubit; });
    const size_t cap = 3 + (size_t)nsw;
    for (size_t c0 = 0; c0 < ids.size(); c0 += cap) {
      int gid[3] = {-1, -1, -1}, reg[3] = {-1, -1, -1}, sgid[2] = {-1, -1}, spos[2] = {-1, -1};
      bool used[16] = {false};
      int cnt = 0;
      for (size_t i = c0; i < ids.size() && i < c0 + cap; ++i, ++cnt) {
        const int pos = n - 1 - hp->fused[ids[i]].qubit;
        if (cnt < 3) { gid[cnt] = ids[i]; reg[cnt] = pos; } else { sgid[cnt - 3] = ids[i]; spos[cnt - 3] = pos; }
        used[pos] = true;
      }
      for (int i = 0; i < 3; ++i)   // pad with unused positions
        if (reg[i] < 0) {
          int best = -1;
          for (int p = 0; p < n && best < 0; ++p)
            if (!used[p]) best = p;
          reg[i] = best;
          used[best] = true;
        }
      for (int i = 0; i < nsw; ++i)
        if (spos[i] < 0) {
          int best = -1;
          for (int p = 0; p < n && best < 0; ++p)
            if (!used[p]) best = p;
          spos[i] = best;
          used[best] = true;
        }
      push_round(gid, reg, sgid, spos);
    }
    if (si == 0) stage0_rounds = (int)hp->rounds.size();
  }
  if (hp->rounds.empty()) {   // no rotations at all: one empty round
    int none[3] = {-1, -1, -1}, snone[2] = {-1, -1};
    int reg[3] = {0, 1, 2}, spos[2] = {0, 0};
    free_spos(reg, spos);
    Affine keep = pending;
    bool hk = have_pending;
    std::vector<QPhaseGate> kp = pending_phase;
    pending.init(n);
    have_pending = false;
    pending_phase.clear();
    push_round(none, reg, snone, spos);
    pending = keep;
    have_pending = hk;
    pending_phase = kp;
  }
  // A trailing phase stage (pending_phase here) is diagonal right before the Z readout: it changes
  // neither the readouts nor their tangents (a common phase per amplitude), and its parameters get
  // an exactly zero gradient, so it is dropped.
  // Phase stages before rounds 1..R-1, their coefficient and moment slots, parameter map.
  hp->phases.clear();
  hp->phase_gates.clear();
  for (size_t k = 1; k < hp->rounds.size(); ++k) {
    if (round_phase[k].empty()) continue;
    QPhaseStage ps{};
    ps.gate0 = (int)hp->phase_gates.size();
    ps.ngates = (int)round_phase[k].size();
    ps.coef_off = (int)hp->phases.size() * phase_terms(n);
    ps.mom_off = ps.coef_off;
    hp->rounds[k].phase = (int)hp->phases.size();
    hp->phases.push_back(ps);
    for (const auto& pg : round_phase[k]) hp->phase_gates.push_back(pg);
  }
  hp->pcsr_ptr.assign(hp->K + 1, 0);
  for (const auto& pg : hp->phase_gates) hp->pcsr_ptr[pg.param + 1]++;
  for (int k = 0; k < hp->K; ++k) hp->pcsr_ptr[k + 1] += hp->pcsr_ptr[k];
  hp->pcsr_idx.assign(hp->pcsr_ptr[hp->K], 0);
  {
    std::vector<int> fill(hp->pcsr_ptr.begin(), hp->pcsr_ptr.end() - 1);
    for (size_t gi = 0; gi < hp->phase_gates.size(); ++gi) hp->pcsr_idx[fill[hp->phase_gates[gi].param]++] = (int)gi;
  }
  // An opening rotation stage acts on the product state: one fused gate per qubit, all commuting.
  // Its rounds are folded into the encoding and their gates take their statistics at the stage
  // output.  The last round is never folded (the adjoint sweep starts by pulling it back).
  hp->n_head = std::min(stage0_rounds, (int)hp->rounds.size() - 1);
  for (int k = 0; k < hp->n_head; ++k) {
    const QRound& rd = hp->rounds[k];
    for (int b = 0; b < 5; ++b) {
      const int fid = b < 3 ? rd.gate[b] : rd.sgate[b - 3];
      if (fid < 0) continue;
      hp->fused[fid].stat_out = 1;
      hp->head_gate[hp->fused[fid].qubit] = fid;
    }
  }
  // trailing entangler -> readout masks: z_i(pi j), pi = A^{-1}
  {
    uint32_t pcols[16];
    if (have_pending) {
      if (!gf2_inverse(pending.acol, n, pcols)) { *status = QP_EINVAL; return "singular entangler map"; }
    } else {
      for (int k = 0; k < 16; ++k) pcols[k] = k < n ? (1u << k) : 0;
    }
    for (int i = 0; i < hp->m; ++i) {
      const int b = n - 1 - hp->out_qubits[i];
      uint32_t mask = 0;
      for (int k = 0; k < n; ++k)
        if ((pcols[k] >> b) & 1u) mask |= (1u << k);
      hp->zmask[i] = mask;
    }
  }
  // exchanges
  const int R = (int)hp->rounds.size();
  const int TP = 1 << (n - 3);
  hp->xf.assign(R, QXchg{});
  hp->xb.assign(R, QXchg{});
  hp->lanes.assign((size_t)2 * R * TP, QLane{});
  hp->n_exchanges = 0;
  hp->has_signs = false;
  for (int k = 1; k < R; ++k) {
    const Affine& a = round_ent[k];
    fill_xchg(&hp->xf[k], n, a.acol, a, false, hp->rounds[k].tpos);
    uint32_t inv[16];
    if (!gf2_inverse(a.acol, n, inv)) { *status = QP_EINVAL; return "singular entangler map"; }
    fill_xchg(&hp->xb[k], n, inv, a, true, hp->rounds[k - 1].tpost);
    hp->n_exchanges++;
    if (hp->xf[k].nterms != 0 || hp->xb[k].nterms != 0) hp->has_signs = true;
    // forward: round k-1's output mapping -> round k's input mapping; reverse: the other way
    const int T = fused_wg_threads(n);
    uint32_t Mf[16], Mb[16];
    choose_index_map(n, T, hp->rounds[k - 1].tpost, hp->rounds[k].tpos, a.acol, 2 * k, Mf);
    choose_index_map(n, T, hp->rounds[k].tpos, hp->rounds[k - 1].tpost, inv, 2 * k + 1, Mb);
    set_lds_layout(&hp->xf[k], n, Mf, hp->rounds[k - 1].tpost, hp->rounds[k].tpos, a.acol);
    set_lds_layout(&hp->xb[k], n, Mb, hp->rounds[k].tpos, hp->rounds[k - 1].tpost, inv);
    for (int u = 0; u < TP; ++u) {
      hp->lanes[((size_t)0 * R + k) * TP + u] =
          lane_words(n, a.acol, a, false, hp->rounds[k - 1].tpost, hp->rounds[k].tpos, Mf, (uint32_t)u);
      hp->lanes[((size_t)1 * R + k) * TP + u] =
          lane_words(n, inv, a, true, hp->rounds[k].tpos, hp->rounds[k - 1].tpost, Mb, (uint32_t)u);
    }
  }

  }
image:
  // device image
  const int R = (int)hp->rounds.size();
  if (hp->xf.size() < (size_t)R) { hp->xf.assign(R, QXchg{}); hp->xb.assign(R, QXchg{}); }
  QPlanDev h{};
  h.n = n;
  h.n_params = hp->K;
  h.n_out = hp->m;
  h.n_fused = (int)hp->fused.size();
  h.n_rounds = R;
  h.n_head = hp->fused_ok ? hp->n_head : 0;
  for (int q = 0; q < 16; ++q) h.head_gate[q] = hp->fused_ok ? hp->head_gate[q] : -1;
  h.enc_kind = hp->enc_kind;
  h.enc_gate = hp->enc_gate;
  h.enc_scale = hp->enc_scale;
  h.n_feat = hp->n_feat;
  for (int q = 0; q < 16; ++q) h.coord_of_qubit[q] = hp->coord[q];
  for (int i = 0; i < kMaxOut; ++i) h.zmask[i] = hp->zmask[i];
  for (int i = 0; i < kMaxOut; ++i) h.zplain[i] = i < hp->m ? 1u << (n - 1 - hp->out_qubits[i]) : 0u;
  size_t off = align16(sizeof(QPlanDev));
  h.off_rounds = (int)off; off = align16(off + sizeof(QRound) * R);
  h.off_xf = (int)off; off = align16(off + sizeof(QXchg) * R);
  h.off_xb = (int)off; off = align16(off + sizeof(QXchg) * R);
  h.off_fused = (int)off; off = align16(off + sizeof(QFused) * hp->fused.size());
  h.off_csr_ptr = (int)off; off = align16(off + sizeof(int32_t) * hp->csr_ptr.size());
  h.off_csr_idx = (int)off; off = align16(off + sizeof(int32_t) * std::max<size_t>(1, hp->csr_idx.size()));
  h.off_rff_B = (int)off; off = align16(off + sizeof(float) * hp->rffB.size());
  h.off_rff_W = (int)off; off = align16(off + sizeof(float) * hp->rffW.size());
  h.n_dgroups = hp->dense_ok ? (int)hp->dgroups.size() : 0;
  h.off_dgroups = (int)off; off = align16(off + sizeof(QDenseGroup) * hp->dgroups.size());
  h.off_dgates = (int)off; off = align16(off + sizeof(QDenseGate) * hp->dgates.size());
  h.n_docc = (int)hp->docc.size() / 2;
  h.off_docc = (int)off; off = align16(off + sizeof(int32_t) * hp->docc.size());
  h.off_dcsr_ptr = (int)off; off = align16(off + sizeof(int32_t) * hp->dcsr_ptr.size());
  h.off_dcsr_idx = (int)off; off = align16(off + sizeof(int32_t) * std::max<size_t>(1, hp->dcsr_idx.size()));
  h.off_lanes = (int)off; off = align16(off + sizeof(QLane) * hp->lanes.size());
  h.n_phase = hp->fused_ok ? (int)hp->phases.size() : 0;
  h.n_phase_coef = h.n_phase * phase_terms(n);
  h.n_moments = h.n_phase_coef;
  h.off_phase = (int)off; off = align16(off + sizeof(QPhaseStage) * hp->phases.size());
  h.off_phase_gates = (int)off; off = align16(off + sizeof(QPhaseGate) * hp->phase_gates.size());
  h.off_pcsr_ptr = (int)off; off = align16(off + sizeof(int32_t) * std::max<size_t>(1, hp->pcsr_ptr.size()));
  h.off_pcsr_idx = (int)off; off = align16(off + sizeof(int32_t) * std::max<size_t>(1, hp->pcsr_idx.size()));
  h.bytes = (int)off;
  hp->blob.assign(off, 0);
  std::memcpy(hp->blob.data(), &h, sizeof(h));
  std::memcpy(hp->blob.data() + h.off_rounds, hp->rounds.data(), sizeof(QRound) * R);
  std::memcpy(hp->blob.data() + h.off_xf, hp->xf.data(), sizeof(QXchg) * R);
  std::memcpy(hp->blob.data() + h.off_xb, hp->xb.data(), sizeof(QXchg) * R);
  if (!hp->fused.empty())
    std::memcpy(hp->blob.data() + h.off_fused, hp->fused.data(), sizeof(QFused) * hp->fused.size());
  std::memcpy(hp->blob.data() + h.off_csr_ptr, hp->csr_ptr.data(), sizeof(int32_t) * hp->csr_ptr.size());
  if (!hp->csr_idx.empty())
    std::memcpy(hp->blob.data() + h.off_csr_idx, hp->csr_idx.data(), sizeof(int32_t) * hp->csr_idx.size());
  if (!hp->rffB.empty()) std::memcpy(hp->blob.data() + h.off_rff_B, hp->rffB.data(), sizeof(float) * hp->rffB.size());
  if (!hp->rffW.empty()) std::memcpy(hp->blob.data() + h.off_rff_W, hp->rffW.data(), sizeof(float) * hp->rffW.size());
  if (!hp->dgroups.empty()) std::memcpy(hp->blob.data() + h.off_dgroups, hp->dgroups.data(), sizeof(QDenseGroup) * hp->dgroups.size());
  if (!hp->dgates.empty()) std::memcpy(hp->blob.data() + h.off_dgates, hp->dgates.data(), sizeof(QDenseGate) * hp->dgates.size());
  if (!hp->docc.empty()) std::memcpy(hp->blob.data() + h.off_docc, hp->docc.data(), sizeof(int32_t) * hp->docc.size());
  std::memcpy(hp->blob.data() + h.off_dcsr_ptr, hp->dcsr_ptr.data(), sizeof(int32_t) * hp->dcsr_ptr.size());
  if (!hp->dcsr_idx.empty()) std::memcpy(hp->blob.data() + h.off_dcsr_idx, hp->dcsr_idx.data(), sizeof(int32_t) * hp->dcsr_idx.size());
  if (!hp->lanes.empty()) std::memcpy(hp->blob.data() + h.off_lanes, hp->lanes.data(), sizeof(QLane) * hp->lanes.size());
  if (!hp->phases.empty()) std::memcpy(hp->blob.data() + h.off_phase, hp->phases.data(), sizeof(QPhaseStage) * hp->phases.size());
  if (!hp->phase_gates.empty())
    std::memcpy(hp->blob.data() + h.off_phase_gates, hp->phase_gates.data(), sizeof(QPhaseGate) * hp->phase_gates.size());
  if (!hp->pcsr_ptr.empty()) std::memcpy(hp->blob.data() + h.off_pcsr_ptr, hp->pcsr_ptr.data(), sizeof(int32_t) * hp->pcsr_ptr.size());
  if (!hp->pcsr_idx.empty()) std::memcpy(hp->blob.data() + h.off_pcsr_idx, hp->pcsr_idx.data(), sizeof(int32_t) * hp->pcsr_idx.size());
  return "";
}

}  // namespace qp
