// Plain baseline: one kernel launch per gate on a statevector batch held in HBM, a readout
// kernel, input tangents by central finite differences and parameter gradients by central
// finite differences of the loss - the evaluation-count model of the paper's hardware
// derivatives (cost per point ~ 1 + sum over derivatives of 2^order x occurrences; section
// "Maxwell's equations in two dimensions and problem setup").  This path is the speedup
// denominator; it is deliberately unfused.  Real type TR is float (complex64 state) or double
// (complex128 state).  State layout: [P][2^n] interleaved complex.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plain.hpp"

namespace qp {

template <typename TR> struct C2 { TR r, i; };

template <typename TR>
__device__ __forceinline__ void sc(TR x, TR* s, TR* c);
template <> __device__ __forceinline__ void sc<float>(float x, float* s, float* c) { sincosf(x, s, c); }
template <> __device__ __forceinline__ void sc<double>(double x, double* s, double* c) { sincos(x, s, c); }

// Gate matrices for every gate of the raw list (rotations, CRZ), in the working precision.
template <typename TR>
__global__ void k_plain_gates(const PlainGate* __restrict__ gates, int ng, const TR* __restrict__ params,
                              TR* __restrict__ tab) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const PlainGate G = gates[g];
  TR* o = tab + g * 8;
  for (int e = 0; e < 8; ++e) o[e] = 0;
  if (G.param < 0) return;
  TR s, c;
  sc<TR>(params[G.param] * (TR)0.5, &s, &c);
  if (G.kind == QP_RX) { o[0] = c; o[3] = -s; o[5] = -s; o[6] = c; }
  else if (G.kind == QP_RY) { o[0] = c; o[2] = -s; o[4] = s; o[6] = c; }
  else { o[0] = c; o[1] = -s; o[6] = c; o[7] = s; }   // RZ, and the RZ block of CRZ
}

// Embedding angles per point with one coordinate shifted by delta: theta [P][n].
template <typename TR>
__global__ void k_plain_angles(const PlainEnc enc, const TR* __restrict__ points, long long P,
                               int coord, TR delta, TR* __restrict__ theta) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  TR x[3] = {points[p * 3], points[p * 3 + 1], points[p * 3 + 2]};
  if (coord >= 0) x[coord] += delta;
  if (enc.kind == QP_ENC_CYCLE) {
    for (int q = 0; q < enc.n; ++q) {
      const TR a = x[enc.coord[q]];
      TR th;
      switch (enc.scale) {
        case QP_SCALE_NONE: th = a; break;
        case QP_SCALE_PI: th = (TR)3.14159265358979323846 * a; break;
        case QP_SCALE_BIAS: th = (a + 1) * (TR)1.57079632679489661923; break;
        case QP_SCALE_ASIN: th = asin(a) + (TR)1.57079632679489661923; break;
        default: th = acos(a); break;
      }
      theta[p * enc.n + q] = th;
    }
  } else {   // RFF
    for (int q = 0; q < enc.n; ++q) theta[p * enc.n + q] = 0;
    for (int f = 0; f < enc.nf; ++f) {
      const TR pr = (TR)enc.B[f * 3] * x[0] + (TR)enc.B[f * 3 + 1] * x[1] + (TR)enc.B[f * 3 + 2] * x[2];
      TR s, c;
      sc<TR>(pr, &s, &c);
      for (int q = 0; q < enc.n; ++q)
        theta[p * enc.n + q] += (TR)enc.W[q * 2 * enc.nf + f] * c + (TR)enc.W[q * 2 * enc.nf + enc.nf + f] * s;
    }
  }
}

// Product state psi[p][j] = prod_q G(theta_q)|0>_{b_q(j)}.
template <typename TR>
__global__ void k_plain_init(int n, int gate, const TR* __restrict__ theta, long long P, C2<TR>* __restrict__ st) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long dim = 1ll << n;
  if (idx >= P * dim) return;
  const long long p = idx >> n;
  const uint32_t j = (uint32_t)(idx & (dim - 1));
  TR ar = 1, ai = 0;
  for (int q = 0; q < n; ++q) {
    TR s, c;
    sc<TR>(theta[p * n + q] * (TR)0.5, &s, &c);
    const int b = (j >> (n - 1 - q)) & 1;
    TR er, ei;
    if (!b) { er = c; ei = 0; }
    else if (gate == QP_ENC_RY) { er = s; ei = 0; }
    else { er = 0; ei = -s; }
    const TR nr = ar * er - ai * ei, ni = ar * ei + ai * er;
    ar = nr; ai = ni;
  }
  st[idx] = C2<TR>{ar, ai};
}

template <typename TR>
__global__ void k_plain_rot(int n, int q, const TR* __restrict__ U, long long P, C2<TR>* __restrict__ st) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long half = 1ll << (n - 1);
  if (idx >= P * half) return;
  const long long p = idx >> (n - 1);
  const uint32_t i = (uint32_t)(idx & (half - 1));
  const int b = n - 1 - q;
  const uint32_t j0 = ((i >> b) << (b + 1)) | (i & ((1u << b) - 1));
  const uint32_t j1 = j0 | (1u << b);
  C2<TR>* s = st + (p << n);
  const C2<TR> x = s[j0], y = s[j1];
  s[j0] = C2<TR>{U[0] * x.r - U[1] * x.i + U[2] * y.r - U[3] * y.i, U[0] * x.i + U[1] * x.r + U[2] * y.i + U[3] * y.r};
  s[j1] = C2<TR>{U[4] * x.r - U[5] * x.i + U[6] * y.r - U[7] * y.i, U[4] * x.i + U[5] * x.r + U[6] * y.i + U[7] * y.r};
}

// CNOT(c,t): swap amplitude pairs with control bit set; CZ: negate where both bits set;
// CRZ(c,t): phase e^{-+i theta/2} on the target where the control bit is set.
template <typename TR>
__global__ void k_plain_two(int n, int kind, int c, int t, const TR* __restrict__ U, long long P, C2<TR>* __restrict__ st) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long dim = 1ll << n;
  if (idx >= P * dim) return;
  const long long p = idx >> n;
  const uint32_t j = (uint32_t)(idx & (dim - 1));
  const uint32_t mc = 1u << (n - 1 - c), mt = 1u << (n - 1 - t);
  if (!(j & mc)) return;
  C2<TR>* s = st + (p << n);
  if (kind == QP_CNOT) {
    if (j & mt) return;   // the thread with target bit 0 swaps the pair
    const C2<TR> a = s[j], b = s[j | mt];
    s[j] = b;
    s[j | mt] = a;
  } else if (kind == QP_CZ) {
    if (j & mt) { s[j].r = -s[j].r; s[j].i = -s[j].i; }
  } else {
    const TR pr = (j & mt) ? U[6] : U[0], pi = (j & mt) ? U[7] : U[1];
    const C2<TR> a = s[j];
    s[j] = C2<TR>{pr * a.r - pi * a.i, pr * a.i + pi * a.r};
  }
}

// f[p][i] = sum_j z_i(j)|psi_j|^2; one wave per point.
template <typename TR>
__global__ void k_plain_readout(int n, int m, PlainOut oq, long long P, const C2<TR>* __restrict__ st, TR* __restrict__ f) {
  const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= P) return;
  const C2<TR>* s = st + (p << n);
  TR acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (uint32_t j = lane; j < (1u << n); j += 64) {
    const TR pr = s[j].r * s[j].r + s[j].i * s[j].i;
    for (int i = 0; i < m; ++i) acc[i] += ((j >> (n - 1 - oq.q[i])) & 1) ? -pr : pr;
  }
  for (int i = 0; i < m; ++i) {
    TR v = acc[i];
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) f[p * m + i] = v;
  }
}

template <typename TR>
__global__ void k_plain_fd(long long n_el, const TR* __restrict__ fp, const TR* __restrict__ fm, TR inv2h, int c,
                           TR* __restrict__ tan) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_el) return;
  tan[e * 3 + c] = (fp[e] - fm[e]) * inv2h;
}

// Maxwell loss from FD tangents; per-point terms reduced in FP64 by one workgroup.
template <typename TR>
__global__ void k_plain_loss(const TR* __restrict__ tan, const TR* __restrict__ points, long long P, int m,
                             int kind, int loss_sum, double eps_r, double x_if, double* __restrict__ loss) {
  __shared__ double sh[16];
  __shared__ int shc[16];
  int nd = 0;
  for (long long p = threadIdx.x; p < P; p += blockDim.x) nd += (double)points[p * 3 + 1] >= x_if ? 1 : 0;
  for (int off = 32; off >= 1; off >>= 1) nd += __shfl_xor(nd, off);
  if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = nd;
  __syncthreads();
  int ndt = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) ndt += shc[w];
  const long long nvt = P - ndt;
  double s = 0.0;
  for (long long p = threadIdx.x; p < P; p += blockDim.x) {
    const TR* g = tan + p * m * 3;
    const double gEt = g[0], gEx = g[1], gEy = g[2], gXt = g[3], gXy = g[5], gYt = g[6], gYx = g[7];
    double eps = 1.0, w1 = loss_sum ? 1.0 : 1.0 / (double)P;
    if (kind != QP_LOSS_VACUUM) {
      const bool diel = (double)points[p * 3 + 1] >= x_if;
      eps = diel ? eps_r : 1.0;
      if (kind == QP_LOSS_DIEL_SPLIT && !loss_sum) w1 = diel ? 1.0 / (double)(ndt > 0 ? ndt : 1) : 1.0 / (double)(nvt > 0 ? nvt : 1);
    }
    const double w = loss_sum ? 1.0 : 1.0 / (double)P;
    const double r1 = gEt - (gYx - gXy) / eps, r2 = gXt + gEy, r3 = gYt - gEx;
    s += w1 * r1 * r1 + w * (r2 * r2 + r3 * r3);
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    *loss = t;
  }
}

template <typename TR>
__global__ void k_plain_copy_shift(const TR* __restrict__ src, TR* __restrict__ dst, int K, int k, TR delta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) dst[i] = src[i] + (i == k ? delta : (TR)0);
}

__global__ void k_plain_fd_param(const double* __restrict__ lp, const double* __restrict__ lm, double inv2h, int is_double,
                                 void* __restrict__ dst, int k) {
  const double v = (*lp - *lm) * inv2h;
  if (is_double) static_cast<double*>(dst)[k] = v;
  else static_cast<float*>(dst)[k] = (float)v;
}

// ---------------------------------------------------------------------------------------------
static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Bloch vectors r_k = (<X_k>, <Y_k>, <Z_k>) of every qubit of every point's state, and the global
// Meyer-Wallach entanglement Q = 2 (1 - (1/n) sum_k Tr rho_k^2) = 1 - (1/n) sum_k |r_k|^2 (a qubit's
// reduced state is rho_k = (I + r_k . sigma) / 2); one wave per point.
template <typename TR>
__global__ void k_plain_bloch(int n, long long P, const C2<TR>* __restrict__ st, TR* __restrict__ bloch,
                              TR* __restrict__ mw) {
  const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= P) return;
  const C2<TR>* s = st + (p << n);
  TR q = 0;
  for (int k = 0; k < n; ++k) {
    const uint32_t mk = 1u << (n - 1 - k);
    TR x = 0, y = 0, z = 0;
    for (uint32_t i = lane; i < (1u << (n - 1)); i += 64) {
      const uint32_t lo = i & (mk - 1);
      const uint32_t j0 = ((i ^ lo) << 1) | lo, j1 = j0 | mk;
      const C2<TR> a = s[j0], b = s[j1];
      x += 2 * (a.r * b.r + a.i * b.i);      // 2 Re(conj(a) b)
      y += 2 * (a.r * b.i - a.i * b.r);      // 2 Im(conj(a) b)
      z += (a.r * a.r + a.i * a.i) - (b.r * b.r + b.i * b.i);
    }
    for (int off = 32; off >= 1; off >>= 1) {
      x += __shfl_xor(x, off);
      y += __shfl_xor(y, off);
      z += __shfl_xor(z, off);
    }
    if (lane == 0) {
      bloch[(p * n + k) * 3 + 0] = x;
      bloch[(p * n + k) * 3 + 1] = y;
      bloch[(p * n + k) * 3 + 2] = z;
    }
    q += x * x + y * y + z * z;
  }
  if (lane == 0 && mw) mw[p] = 1 - q / (TR)n;
}

template <typename TR>
hipError_t plain_forward_t(const PlainProblem& pr, const TR* params, const TR* points, int coord, double delta,
                           TR* f, void* ws, hipStream_t st, const TR* angles = nullptr) {
  const PlainLayout L = plain_layout(pr, sizeof(TR));
  char* w = static_cast<char*>(ws);
  TR* tab = reinterpret_cast<TR*>(w + L.off_tab);
  TR* theta = reinterpret_cast<TR*>(w + L.off_theta);
  C2<TR>* s = reinterpret_cast<C2<TR>*>(w + L.off_state);
  const int ng = pr.n_gates;
  const long long P = pr.P;
  const int n = pr.enc.n;
  if (P == 0) return hipSuccess;
  if (ng > 0) hipLaunchKernelGGL(k_plain_gates<TR>, dim3(nblk(ng, 128)), dim3(128), 0, st, pr.gates_dev, ng, params, tab);
  if (angles) theta = const_cast<TR*>(angles);   // angle-given encoding: the angles are the input
  else hipLaunchKernelGGL(k_plain_angles<TR>, dim3(nblk(P, 128)), dim3(128), 0, st, pr.enc, points, P, coord, (TR)delta, theta);
  hipLaunchKernelGGL(k_plain_init<TR>, dim3(nblk(P << n, 256)), dim3(256), 0, st, n, pr.enc.gate, theta, P, s);
  for (int g = 0; g < ng; ++g) {
    const PlainGate G = pr.gates_host[g];
    if (G.kind <= QP_RZ)
      hipLaunchKernelGGL(k_plain_rot<TR>, dim3(nblk(P << (n - 1), 256)), dim3(256), 0, st, n, G.q0, tab + g * 8, P, s);
    else
      hipLaunchKernelGGL(k_plain_two<TR>, dim3(nblk(P << n, 256)), dim3(256), 0, st, n, G.kind, G.q0, G.q1, tab + g * 8, P, s);
  }
  if (f) hipLaunchKernelGGL(k_plain_readout<TR>, dim3(nblk(P, 4)), dim3(256), 0, st, n, pr.m, pr.oq, P, s, f);
  return hipGetLastError();
}

template <typename TR>
hipError_t plain_bloch_t(const PlainProblem& pr, const TR* params, const TR* points, const TR* angles, TR* bloch, TR* mw,
                         void* ws, hipStream_t st) {
  hipError_t e = plain_forward_t<TR>(pr, params, points, -1, 0.0, nullptr, ws, st, angles);
  if (e != hipSuccess || pr.P == 0) return e;
  const PlainLayout L = plain_layout(pr, sizeof(TR));
  const C2<TR>* s = reinterpret_cast<const C2<TR>*>(static_cast<char*>(ws) + L.off_state);
  hipLaunchKernelGGL(k_plain_bloch<TR>, dim3(nblk(pr.P, 4)), dim3(256), 0, st, pr.enc.n, pr.P, s, bloch, mw);
  return hipGetLastError();
}

template <typename TR>
hipError_t plain_eval_t(const PlainProblem& pr, const TR* params, const TR* points, double h, TR* out, TR* tan,
                        void* ws, hipStream_t st) {
  const PlainLayout L = plain_layout(pr, sizeof(TR));
  char* w = static_cast<char*>(ws);
  TR* fp = reinterpret_cast<TR*>(w + L.off_fp);
  TR* fm = reinterpret_cast<TR*>(w + L.off_fm);
  hipError_t e = plain_forward_t<TR>(pr, params, points, -1, 0.0, out, ws, st);
  if (e != hipSuccess || !tan) return e;
  const long long nel = pr.P * pr.m;
  for (int c = 0; c < 3; ++c) {
    if ((e = plain_forward_t<TR>(pr, params, points, c, h, fp, ws, st)) != hipSuccess) return e;
    if ((e = plain_forward_t<TR>(pr, params, points, c, -h, fm, ws, st)) != hipSuccess) return e;
    if (nel > 0) hipLaunchKernelGGL(k_plain_fd<TR>, dim3(nblk(nel, 256)), dim3(256), 0, st, nel, fp, fm, (TR)(0.5 / h), c, tan);
  }
  return hipGetLastError();
}

template <typename TR>
hipError_t plain_maxwell_t(const PlainProblem& pr, const TR* params, const TR* points, const qp_maxwell_desc& ld, int loss_sum,
                           double h, double hp, int k0, int k1, double* loss, TR* dparams, void* ws, hipStream_t st) {
  const PlainLayout L = plain_layout(pr, sizeof(TR));
  char* w = static_cast<char*>(ws);
  TR* out = reinterpret_cast<TR*>(w + L.off_out);
  TR* tan = reinterpret_cast<TR*>(w + L.off_tan);
  TR* pbuf = reinterpret_cast<TR*>(w + L.off_pbuf);
  double* lp = reinterpret_cast<double*>(w + L.off_loss);
  hipError_t e = plain_eval_t<TR>(pr, params, points, h, out, tan, ws, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plain_loss<TR>, dim3(1), dim3(1024), 0, st, tan, points, pr.P, pr.m, ld.kind, loss_sum,
                     (double)ld.eps_r, (double)ld.x_interface, loss);
  for (int k = k0; k < k1; ++k) {
    for (int sgn = 0; sgn < 2; ++sgn) {
      hipLaunchKernelGGL(k_plain_copy_shift<TR>, dim3(nblk(pr.K, 256)), dim3(256), 0, st, params, pbuf, pr.K, k,
                         (TR)(sgn ? -hp : hp));
      if ((e = plain_eval_t<TR>(pr, pbuf, points, h, out, tan, ws, st)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_plain_loss<TR>, dim3(1), dim3(1024), 0, st, tan, points, pr.P, pr.m, ld.kind, loss_sum,
                         (double)ld.eps_r, (double)ld.x_interface, lp + sgn);
    }
    hipLaunchKernelGGL(k_plain_fd_param, dim3(1), dim3(1), 0, st, lp, lp + 1, 0.5 / hp, (int)(sizeof(TR) == 8),
                       (void*)dparams, k);
  }
  return hipGetLastError();
}

PlainLayout plain_layout(const PlainProblem& pr, size_t tr) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  PlainLayout L{};
  size_t off = 0;
  L.off_tab = off; off = al(off + tr * 8 * (size_t)(pr.n_gates > 0 ? pr.n_gates : 1));
  L.off_theta = off; off = al(off + tr * (size_t)pr.P * pr.enc.n);
  L.off_state = off; off = al(off + 2 * tr * ((size_t)pr.P << pr.enc.n));
  L.off_fp = off; off = al(off + tr * (size_t)pr.P * pr.m);
  L.off_fm = off; off = al(off + tr * (size_t)pr.P * pr.m);
  L.off_out = off; off = al(off + tr * (size_t)pr.P * pr.m);
  L.off_tan = off; off = al(off + tr * (size_t)pr.P * pr.m * 3);
  L.off_pbuf = off; off = al(off + tr * (size_t)(pr.K > 0 ? pr.K : 1));
  L.off_loss = off; off = al(off + 2 * sizeof(double));
  L.total = off;
  return L;
}

hipError_t plain_eval(const PlainProblem& pr, int prec, const void* params, const void* points, double h, void* out,
                      void* tan, void* ws, hipStream_t st) {
  if (prec == 64)
    return plain_eval_t<double>(pr, (const double*)params, (const double*)points, h, (double*)out, (double*)tan, ws, st);
  return plain_eval_t<float>(pr, (const float*)params, (const float*)points, h, (float*)out, (float*)tan, ws, st);
}

hipError_t plain_bloch(const PlainProblem& pr, int prec, const void* params, const void* points, const void* angles,
                       void* bloch, void* mw, void* ws, hipStream_t st) {
  if (prec == 64)
    return plain_bloch_t<double>(pr, (const double*)params, (const double*)points, (const double*)angles, (double*)bloch,
                                 (double*)mw, ws, st);
  return plain_bloch_t<float>(pr, (const float*)params, (const float*)points, (const float*)angles, (float*)bloch,
                              (float*)mw, ws, st);
}

hipError_t plain_maxwell(const PlainProblem& pr, int prec, const void* params, const void* points, const qp_maxwell_desc& ld,
                         int loss_sum, double h, double hp, int k0, int k1, double* loss, void* dparams, void* ws,
                         hipStream_t st) {
  if (prec == 64)
    return plain_maxwell_t<double>(pr, (const double*)params, (const double*)points, ld, loss_sum, h, hp, k0, k1, loss,
                                   (double*)dparams, ws, st);
  return plain_maxwell_t<float>(pr, (const float*)params, (const float*)points, ld, loss_sum, h, hp, k0, k1, loss,
                                (float*)dparams, ws, st);
}

}  // namespace qp
