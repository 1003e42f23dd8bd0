// Instantiation of the fused kernel for 5 qubits.
#include "fused_kernel.hpp"

namespace qp {
hipError_t launch_fused_5(int mode, const FusedArgs& a, int grid, int exs, bool signs, size_t lds, hipStream_t st) {
  return launch_fused_n<5>(mode, a, grid, exs, signs, lds, st);
}
}  // namespace qp
