// The paper's total loss on the GPU (eq. 2D_lossTot): L_phys + w_ic L_IC + w_sym L_sym + w_energy L_energy.
//
// The symmetry term couples a collocation point with its mirror images, so the step runs in
// stream-ordered phases over an extended point set [X; X_my; X_mx (vacuum only); X_0]:
//   1. the packed forward kernel: outputs of the mirrored and initial-condition points,
//   2. one fused pass over the collocation points X (kModeTotal): forward with input tangents,
//      the seeds d L_tot / d(f, g) of the residual, energy and symmetry terms formed in the kernel
//      from the point's own fields and its images' outputs, adjoint with uncompute,
//   3. k_total_seeds: the four terms (per collocation point the residual, energy and symmetry
//      terms, per initial-condition point the IC term; FP32 per-block partial sums) and the seeds
//      d L_tot / d f of the mirrored and initial-condition points (it also writes the collocation
//      points' seeds, which phase 2 formed itself),
//   4. the packed VJP kernel over the mirrored and initial-condition points, then the FP64
//      reductions.
// The loss terms are summed across blocks in FP64 in a fixed order (k_total_reduce).
#include <hip/hip_runtime.h>

#include "total.hpp"

namespace qp {

namespace {

constexpr int kSeedThreads = 256;

// Build [X; X_my; X_mx; X_0]: mirror rows negate x (column 1) or y (column 2); IC rows are (0, x, y).
__global__ void k_total_points(const float* __restrict__ pts, long long P, const float* __restrict__ ic_xy,
                               long long P0, int with_mx, float* __restrict__ ext) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nmir = with_mx ? 2 : 1;
  const long long total = P * (1 + nmir) + P0;
  if (i >= total) return;
  float t, x, y;
  if (i < P * (1 + nmir)) {
    const long long p = i % P, set = i / P;   // 0: X, 1: X_my, 2: X_mx
    t = pts[p * 3];
    x = pts[p * 3 + 1];
    y = pts[p * 3 + 2];
    if (set == 1) y = -y;
    if (set == 2) x = -x;
  } else {
    const long long k = i - P * (1 + nmir);
    t = 0.f;
    x = ic_xy[k * 2];
    y = ic_xy[k * 2 + 1];
  }
  ext[i * 3] = t;
  ext[i * 3 + 1] = x;
  ext[i * 3 + 2] = y;
}

__device__ __forceinline__ float block_sum(float v, float* sh) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  float s = 0.f;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  return s;
}

// One thread per collocation point p (< P) and per initial-condition point k (< P0).
__global__ void k_total_seeds(TotalSeedArgs a) {
  __shared__ float sh[kSeedThreads / 64];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = a.m;
  float l_phys = 0.f, l_ic = 0.f, l_sym = 0.f, l_energy = 0.f;
  if (i < a.P) {
    const long long p = i;
    const long long pmy = a.P + p, pmx = 2 * a.P + p;
    const float* f = a.out + p * m;
    const float* g = a.tan + p * m * 3;
    float* vf = a.d_out + p * m;
    float* wg = a.d_tan + p * m * 3;
    for (int j = 0; j < m; ++j) vf[j] = 0.f;
    for (int j = 0; j < 3 * m; ++j) wg[j] = 0.f;
    const float invP = 1.f / (float)a.P;
    // residuals (eqs. residual_1_vac / residual_1_diel, residuals_2_and_3), loss weights
    float eps = 1.f, w1 = invP;
    const float x = a.points[p * 3 + 1];
    if (a.phys_kind != QP_LOSS_VACUUM) {
      const bool diel = x >= a.x_if;
      eps = diel ? a.eps_r : 1.f;
      if (a.phys_kind == QP_LOSS_DIEL_SPLIT) {
        const int nv = a.counts[0], nd = a.counts[1];
        w1 = diel ? (nd > 0 ? 1.f / (float)nd : 0.f) : (nv > 0 ? 1.f / (float)nv : 0.f);
      }
    }
    const float E = f[0], Hx = f[1], Hy = f[2];
    const float Et = g[0], Ex = g[1], Ey = g[2];
    const float Hxt = g[3], Hxy = g[5];
    const float Hyt = g[6], Hyx = g[7];
    const float ie = 1.f / eps;
    const float r1 = Et - (Hyx - Hxy) * ie;
    const float r2 = Hxt + Ey;
    const float r3 = Hyt - Ex;
    l_phys = w1 * r1 * r1 + invP * (r2 * r2 + r3 * r3);
    const float A = 2.f * w1 * r1, B = 2.f * invP * r2, C = 2.f * invP * r3;
    wg[0] += A; wg[7] += -A * ie; wg[5] += A * ie;
    wg[3] += B; wg[2] += B;
    wg[6] += C; wg[1] += -C;
    // energy: e = eps E Et + Hx Hxt + Hy Hyt - (Ex Hy + E Hyx) + (Ey Hx + E Hxy)
    const float e = eps * E * Et + Hx * Hxt + Hy * Hyt - (Ex * Hy + E * Hyx) + (Ey * Hx + E * Hxy);
    l_energy = e * e * invP;
    const float k = a.w_energy * 2.f * e * invP;
    vf[0] += k * (eps * Et - Hyx + Hxy);
    vf[1] += k * (Hxt + Ey);
    vf[2] += k * (Hyt - Ex);
    wg[0] += k * eps * E; wg[1] += -k * Hy; wg[2] += k * Hx;
    wg[3] += k * Hx; wg[5] += k * E;
    wg[6] += k * Hy; wg[7] += -k * E;
    // symmetry (eq. 2D_symLoss): y-mirror parities (+, -, +), x-mirror parities (+, +, -)
    const float ks = a.w_sym * 2.f * invP;
    {
      const float* fm = a.out + pmy * m;
      float* vm = a.d_out + pmy * m;
      for (int j = 0; j < m; ++j) vm[j] = 0.f;
      const float s[3] = {1.f, -1.f, 1.f};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float d = f[c] - s[c] * fm[c];
        l_sym += d * d * invP;
        vf[c] += ks * d;
        vm[c] = -ks * s[c] * d;
      }
    }
    if (a.with_mx) {
      const float* fm = a.out + pmx * m;
      float* vm = a.d_out + pmx * m;
      for (int j = 0; j < m; ++j) vm[j] = 0.f;
      const float s[3] = {1.f, 1.f, -1.f};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float d = f[c] - s[c] * fm[c];
        l_sym += d * d * invP;
        vf[c] += ks * d;
        vm[c] = -ks * s[c] * d;
      }
    }
  }
  if (i < a.P0) {   // initial condition (eqs. pulse_IC_Ez/Hx/Hy, IC_loss)
    const long long q = a.ic_base + i;
    const float* f = a.out + q * m;
    float* vf = a.d_out + q * m;
    for (int j = 0; j < m; ++j) vf[j] = 0.f;
    const float x = a.ic_xy[i * 2], y = a.ic_xy[i * 2 + 1];
    const float E0 = expf(-a.ic_a * (x * x + y * y));
    const float invP0 = 1.f / (float)a.P0;
    const float dE = f[0] - E0;
    l_ic = (dE * dE + f[1] * f[1] + f[2] * f[2]) * invP0;
    const float ki = a.w_ic * 2.f * invP0;
    vf[0] = ki * dE;
    vf[1] = ki * f[1];
    vf[2] = ki * f[2];
  }
  const float s0 = block_sum(l_phys, sh);
  const float s1 = block_sum(l_ic, sh);
  const float s2 = block_sum(l_sym, sh);
  const float s3 = block_sum(l_energy, sh);
  if (threadIdx.x == 0) {
    a.part[blockIdx.x * 4 + 0] = s0;
    a.part[blockIdx.x * 4 + 1] = s1;
    a.part[blockIdx.x * 4 + 2] = s2;
    a.part[blockIdx.x * 4 + 3] = s3;
  }
}

// FP64 sums of the four terms over the blocks (one wave per term, fixed order), then the total.
__global__ void k_total_reduce(const float* __restrict__ part, int nblk, float w_ic, float w_sym, float w_energy,
                               double* __restrict__ terms) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;   // 4 waves
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += (double)part[b * 4 + wave];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    terms[1] = sh[0];
    terms[2] = sh[1];
    terms[3] = sh[2];
    terms[4] = sh[3];
    terms[0] = sh[0] + (double)w_ic * sh[1] + (double)w_sym * sh[2] + (double)w_energy * sh[3];
  }
}

__global__ void k_add(float* __restrict__ y, const float* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

}  // namespace

hipError_t launch_add(float* y, const float* x, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3((n + 255) / 256), dim3(256), 0, st, y, x, n);
  return hipGetLastError();
}

int total_seed_blocks(long long P, long long P0) {
  const long long n = P > P0 ? P : P0;
  return (int)((n + kSeedThreads - 1) / kSeedThreads);
}

hipError_t launch_total_points(const float* pts, long long P, const float* ic_xy, long long P0, int with_mx, float* ext,
                               hipStream_t st) {
  const long long total = P * (with_mx ? 3 : 2) + P0;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_total_points, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, pts, P, ic_xy, P0, with_mx,
                     ext);
  return hipGetLastError();
}

hipError_t launch_total_seeds(const TotalSeedArgs& a, hipStream_t st) {
  const int nblk = total_seed_blocks(a.P, a.P0);
  if (nblk > 0) hipLaunchKernelGGL(k_total_seeds, dim3(nblk), dim3(kSeedThreads), 0, st, a);
  hipLaunchKernelGGL(k_total_reduce, dim3(1), dim3(256), 0, st, a.part, nblk, a.w_ic, a.w_sym, a.w_energy, a.terms);
  return hipGetLastError();
}

}  // namespace qp
