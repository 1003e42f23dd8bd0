// Launch interface of the energy-profile kernels (diag.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace qp {

hipError_t launch_energy_grid(const float* t, long long Nt, const float* xg, long long Nx, const float* yg, long long Ny,
                              float* pts, hipStream_t st);
hipError_t launch_energy_reduce(const float* f, int m, const float* pts, long long Nt, long long per_slice, int dielectric,
                                float eps_r, float x_if, double* U, hipStream_t st);

}  // namespace qp
