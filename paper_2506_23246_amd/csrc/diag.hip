// Diagnostics of the "black hole" study (section "'Black hole' loss landscape"): the total field
// energy U(t) = sum over a spatial grid of (eps E_z^2 + H_x^2 + H_y^2) / 2 per time slice, from the
// fused forward kernel's outputs on the grid (t-major), summed in FP64 per slice.
#include <hip/hip_runtime.h>

#include "diag.hpp"

namespace qp {

namespace {

__global__ void k_energy_grid(const float* __restrict__ t, long long Nt, const float* __restrict__ xg, long long Nx,
                              const float* __restrict__ yg, long long Ny, float* __restrict__ pts) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nt * Nx * Ny) return;
  const long long it = i / (Nx * Ny), ix = (i / Ny) % Nx, iy = i % Ny;
  pts[i * 3] = t[it];
  pts[i * 3 + 1] = xg[ix];
  pts[i * 3 + 2] = yg[iy];
}

// One workgroup per time slice; fixed-order FP64 sums.
__global__ void k_energy_reduce(const float* __restrict__ f, int m, const float* __restrict__ pts, long long per_slice,
                                int dielectric, float eps_r, float x_if, double* __restrict__ U) {
  __shared__ double sh[4];
  const long long base = (long long)blockIdx.x * per_slice;
  double s = 0.0;
  for (long long i = threadIdx.x; i < per_slice; i += blockDim.x) {
    const long long p = base + i;
    const float eps = (dielectric && pts[p * 3 + 1] >= x_if) ? eps_r : 1.f;
    const double E = f[p * m], Hx = f[p * m + 1], Hy = f[p * m + 2];
    s += 0.5 * ((double)eps * E * E + Hx * Hx + Hy * Hy);
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) U[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

}  // namespace

hipError_t launch_energy_grid(const float* t, long long Nt, const float* xg, long long Nx, const float* yg, long long Ny,
                              float* pts, hipStream_t st) {
  const long long total = Nt * Nx * Ny;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_energy_grid, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, t, Nt, xg, Nx, yg, Ny, pts);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const float* f, int m, const float* pts, long long Nt, long long per_slice, int dielectric,
                                float eps_r, float x_if, double* U, hipStream_t st) {
  if (Nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_energy_reduce, dim3((unsigned)Nt), dim3(256), 0, st, f, m, pts, per_slice, dielectric, eps_r, x_if, U);
  return hipGetLastError();
}

}  // namespace qp
