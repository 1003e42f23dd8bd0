// Class kernels of the uneven batch for circuits with CRZ phase stages (compiled apart from the
// others: see batch_kernel.hpp).
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "batch_kernel.hpp"

namespace qp {

hipError_t launch_batch_seg_ph(int seg, int grid, size_t dyn, hipStream_t s, const BatchCirc* circs,
                               const BatchItem* items, int nitems, int* counter, float* mpart, float* lpart) {
  switch (seg) {
    case kSegLoPh:
      hipLaunchKernelGGL((k_batch<3, kBatchSplit, 256, true>), dim3(grid), dim3(256), dyn, s, circs, items, nitems,
                         counter, mpart, lpart);
      break;
    case kSegHiPh:
      hipLaunchKernelGGL((k_batch<kBatchSplit + 1, 11, 256, true>), dim3(grid), dim3(256), dyn, s, circs, items,
                         nitems, counter, mpart, lpart);
      break;
    case kSegBigPh:
      hipLaunchKernelGGL((k_batch<kBatchBig, kBatchBig, 512, true>), dim3(grid), dim3(512), dyn, s, circs, items,
                         nitems, counter, mpart, lpart);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t batch_prepare_ph(int max_cols, int max_cols_big) {
  const int lds = (int)batch_dyn_lds_bytes(256, max_cols), lds_big = (int)batch_dyn_lds_bytes(512, max_cols_big);
  hipError_t e = hipSuccess;
  if (max_cols > 0) {
    e = hipFuncSetAttribute((const void*)k_batch<3, kBatchSplit, 256, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_batch<kBatchSplit + 1, 11, 256, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  }
  if (e == hipSuccess && max_cols_big > 0)
    e = hipFuncSetAttribute((const void*)k_batch<kBatchBig, kBatchBig, 512, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_big);
  return e;
}

}  // namespace qp
