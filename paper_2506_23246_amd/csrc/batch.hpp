// Uneven batch of circuits evaluated by one persistent kernel (batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "capi_internal.hpp"
#include "fused.hpp"

namespace qp {

struct BatchCirc {          // per circuit, device side
  FusedArgs a;              // plan, gate table, points, outputs, loss description
  const float* params;
  double* loss;
  float* d_params;
  double* m64;              // [F][8]
  long long mpart_off;      // float offset of this circuit's item partials
  int n, F, K, nitems, item_lp0;   // item_lp0: offset into the loss partials
};

struct BatchItem { int circ, tile0, ntile, slot; };
struct BatchCol { int circ, col; };      // col == F*8 means the loss column
struct BatchGate { int circ, idx; };     // fused gate (gate table) or parameter (gradients)

struct BatchLayout {
  size_t counter, gtab, counts, m64, mpart, lpart, total;
  std::vector<size_t> gtab_c, counts_c, m64_c;
  std::vector<long long> mpart_c;
};

// Qubit-count classes of the persistent kernel: [3, kBatchSplit] and [kBatchSplit + 1, 11].
constexpr int kBatchSplit = 8;

// items [nitems]: the first nitems_lo belong to the low class; counter: two work counters.  With
// work in both classes and a second stream (aux, with the events that fork it from st and join it
// back) the classes run at once on grids grid_lo and grid_hi; otherwise one after the other on
// `grid` each.
hipError_t launch_batch(const BatchCirc* circs, int ncirc, const BatchItem* items, int nitems, int nitems_lo,
                        const BatchGate* gates, int ngates, const BatchCol* cols, int ncols, const BatchGate* pars,
                        int npars, int* counter, float* mpart, float* lpart, int grid, int grid_lo, int grid_hi,
                        int max_fused, int count_needed, hipStream_t st, hipStream_t aux, hipEvent_t ev_fork,
                        hipEvent_t ev_join, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t batch_prepare(int max_fused);
size_t batch_lds_bytes(int max_fused);

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
  int grid_lo = 0, grid_hi = 0;     // grids of the two classes when both have work
  int max_fused = 0;
  int nitems_lo = 0;                // work items of the low qubit-count class (listed first)
  double work_lo = 0.0, work_hi = 0.0;   // estimated work of the two classes
  hipStream_t aux = nullptr;        // second stream: the two classes run at once
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  uint64_t io_key = 0;              // pointers the uploaded circuit table refers to
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t graph_key = 0;
};
