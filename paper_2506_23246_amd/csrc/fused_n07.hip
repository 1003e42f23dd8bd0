// Instantiation of the fused kernel for 7 qubits.
#include "fused_kernel.hpp"

namespace qp {
hipError_t launch_fused_7(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st) {
  return launch_fused_n<7>(mode, a, grid, exs, signs, lds, st);
}
}  // namespace qp
