// Uneven batch of circuits evaluated by one persistent kernel (batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "capi_internal.hpp"
#include "fused.hpp"

namespace qp {

struct BatchCirc {          // per circuit, device side
  FusedArgs a;              // plan, gate table, points, RFF angles, outputs, loss description
  const float* params;
  double* loss;
  float* d_params;
  double* m64;              // [F][8] gate statistics, then the phase-stage moments [a.n_mom]
  long long mpart_off;      // float offset of this circuit's item partials
  int n, F, K, nitems, item_lp0;   // item_lp0: offset into the loss partials
};

struct BatchItem { int circ, tile0, ntile, slot; };
struct BatchCol { int circ, col; };      // col == F*8 + n_mom means the loss column
struct BatchGate { int circ, idx; };     // fused gate (gate table) or parameter (gradients)

struct BatchLayout {
  size_t counter, gtab, counts, m64, mpart, lpart, total;
  std::vector<size_t> gtab_c, counts_c, m64_c;
  std::vector<size_t> angles_c, jac_c;   // RFF circuits: per-point angles and Jacobian (else 0)
  std::vector<long long> mpart_c;
};

// Qubit-count classes of the persistent kernels: [3, kBatchSplit] and [kBatchSplit + 1, 11] on
// 256-thread workgroups, and 12 qubits on 512-thread workgroups (one per CU, as the fused kernel).
constexpr int kBatchSplit = 8;
constexpr int kBatchBig = 12;
inline int batch_threads(int n) { return n >= kBatchBig ? 512 : 256; }
inline int batch_points_per_tile(int n) { return batch_threads(n) >> (n - 3); }

// Work-item segments, in list order: the three classes for circuits without CRZ phase stages,
// then the same three classes for circuits with them (their own kernels, so that the phase code
// never enters the register allocation of the others).  Each segment has its own work counter.
enum BatchSegment { kSegLo = 0, kSegHi = 1, kSegBig = 2, kSegLoPh = 3, kSegHiPh = 4, kSegBigPh = 5, kNumSegs = 6 };
inline int batch_segment(int n, bool phases) {
  return (n >= kBatchBig ? kSegBig : (n > kBatchSplit ? kSegHi : kSegLo)) + (phases ? 3 : 0);
}

// items: the segments' items back to back, nitems_seg[kNumSegs] (host) items each; counter:
// kNumSegs work counters.  With work in a low segment (kSegLo, kSegLoPh) and in another and a
// second stream (aux, with the events that fork it from st and join it back), the low segments
// run on st on grid_lo workgroups while the others run on aux (high segments on grid_hi, 12-qubit
// segments on grid_big) at the same time; otherwise every segment runs on st, on `grid`
// workgroups (grid_big for 12 qubits).  max_cols, max_cols_big: the largest F * 8 + n_mom of
// the circuits below 12 qubits and of those with 12 (the dynamic LDS of the two block sizes).
hipError_t launch_batch(const BatchCirc* circs, int ncirc, const BatchItem* items, const int* nitems_seg,
                        const BatchGate* gates, int ngates, const BatchCol* cols, int ncols, const BatchGate* pars,
                        int npars, int* counter, float* mpart, float* lpart, int grid, int grid_lo, int grid_hi,
                        int grid_big, int max_cols, int max_cols_big, int count_needed, hipStream_t st, hipStream_t aux,
                        hipEvent_t ev_fork, hipEvent_t ev_join, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t batch_prepare(int max_cols, int max_cols_big);   // 0: no circuit of that block size
size_t batch_lds_bytes(int n, int max_cols);

}  // namespace qp

struct qp_batch {
  qp_ctx* ctx = nullptr;
  std::vector<qp_circuit*> circs;
  std::vector<int64_t> P;
  std::vector<qp::BatchItem> items;
  std::vector<qp::BatchCol> cols;
  std::vector<qp::BatchGate> gates, pars;
  void* dstatic = nullptr;          // items, cols, gates, pars, circ table
  qp::BatchItem* ditems = nullptr;
  qp::BatchCol* dcols = nullptr;
  qp::BatchGate* dgates = nullptr;
  qp::BatchGate* dpars = nullptr;
  qp::BatchCirc* dcirc = nullptr;
  qp::BatchCirc* hcirc = nullptr;   // pinned staging of the circuit table
  qp::BatchLayout layout;
  int grid = 0;                     // persistent grid of a batch with one class
  int grid_lo = 0, grid_hi = 0;     // grids of the low and high classes when they run at once
  int grid_big = 0;                 // grid of the 12-qubit class
  int max_cols = 0, max_cols_big = 0;   // largest F * 8 + n_mom below 12 qubits and at 12
  int nitems_seg[qp::kNumSegs] = {};   // work items per segment (listed in segment order)
  double work_lo = 0.0, work_rest = 0.0;   // estimated work of the low segments and of the others
  std::vector<int> table_circs;     // circuits whose gate table comes from the fused path's kernel
                                    // (CRZ phase stages: the table carries phase coefficients)
  std::vector<int> rff_circs;       // circuits whose RFF angles are formed before the batch kernels
  hipStream_t aux = nullptr;        // second stream: the low and the other segments run at once
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  uint64_t io_key = 0;              // pointers the uploaded circuit table refers to
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t graph_key = 0;
};
