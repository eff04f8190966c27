// Krylov kernels of GMRES (Sec. 3, [S03]): deterministic two-stage dot
// products and norms, the Gram-Schmidt projections V^T w and w -= V h over up
// to VK_MAX_RESTART + 1 basis vectors in one pass, scaling by a device scalar,
// the Givens update of the Hessenberg column and the small triangular solve.
// Partial sums are reduced in a fixed order, so results are reproducible.
#include "vk_internal.h"

namespace {

constexpr int RB = 256;  // reduction block size

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

__global__ __launch_bounds__(RB) void dot_partial_kernel(int64_t n, const double* __restrict__ x,
                                                         const double* __restrict__ y, double* partial) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(RB) void reduce_kernel(int32_t np, const double* __restrict__ partial, double* out,
                                                    int sqrt_out) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += RB) s += partial[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = sqrt_out ? sqrt(s) : s;
}

// partial[b * m + i] = sum over block b's rows of V_i . w
template <int MB>
__global__ __launch_bounds__(RB) void mdot_partial_kernel(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                          int32_t m, const double* __restrict__ w,
                                                          double* partial) {
  __shared__ double sh[RB / 64];
  double acc[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) acc[i] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < n; r += (int64_t)gridDim.x * RB) {
    const double wr = w[r];
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (i < m) acc[i] += V[(int64_t)i * ldv + r] * wr;
  }
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (i < m) {  // m is uniform: the barriers inside block_sum are reached by all threads
      const double t = block_sum(acc[i], sh);
      if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * m + i] = t;
    }
  }
}

// out[i] = sum_b partial[b * m + i]; one workgroup per coefficient i
__global__ __launch_bounds__(RB) void mreduce_kernel(int32_t nb, int32_t m, const double* __restrict__ partial,
                                                     double* out) {
  __shared__ double sh[RB / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) s += partial[(int64_t)b * m + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[i] = s;
}

// w += sign * sum_i h_i V_i
template <int MB>
__global__ __launch_bounds__(RB) void maxpy_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, int32_t m,
                                                   const double* __restrict__ h, double sign, double* w) {
  __shared__ double sh[MB];
  if (threadIdx.x < MB) sh[threadIdx.x] = threadIdx.x < m ? h[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * RB + threadIdx.x; r < n; r += (int64_t)gridDim.x * RB) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (i < m) s += sh[i] * V[(int64_t)i * ldv + r];
    w[r] += sign * s;
  }
}

__global__ void scale_by_inv_kernel(int64_t n, const double* __restrict__ x, const double* __restrict__ den,
                                    double* y) {
  const double d = den[0];
  const double s = d != 0.0 ? 1.0 / d : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * s;
}

// Column j of H holds the first CGS pass h (rows 0..j) and ||w|| in row j+1;
// h2 the second pass.  Applies the previous rotations, forms rotation j,
// updates g and writes |g_{j+1}| and ||w|| to out[0], out[1].
__global__ void givens_kernel(int32_t j, int32_t ldh, double* H, const double* __restrict__ h2, double* cs,
                              double* sn, double* g, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* col = H + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) col[i] += h2[i];
  const double hn = col[j + 1];
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], b = col[j + 1];
  const double den = hypot(a, b);
  const double c = den != 0.0 ? a / den : 1.0;
  const double s = den != 0.0 ? b / den : 0.0;
  cs[j] = c;
  sn[j] = s;
  col[j] = den;
  col[j + 1] = 0.0;
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  out[0] = fabs(g[j + 1]);
  out[1] = hn;
}

__global__ void gmres_init_kernel(int32_t m, double* H, double* g, const double* __restrict__ beta) {
  const int64_t total = (int64_t)(m + 1) * m;
  for (int64_t i = threadIdx.x; i < total; i += blockDim.x) H[i] = 0.0;
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = (i == 0) ? beta[0] : 0.0;
}

// back substitution R y = g on the leading jn x jn block of the rotated H
__global__ void trisolve_kernel(int32_t jn, int32_t ldh, const double* __restrict__ H, const double* __restrict__ g,
                                double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = jn - 1; i >= 0; --i) {
    double s = g[i];
    for (int k = i + 1; k < jn; ++k) s -= H[(int64_t)k * ldh + i] * y[k];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

inline unsigned grid_n(int64_t n, int cap) {
  int64_t g = (n + RB - 1) / RB;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial,
                      int32_t n_partial, double* out, bool sqrt_out) {
  unsigned g = (unsigned)((n + RB * 4 - 1) / (RB * 4));
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  if (g > (unsigned)n_partial) g = (unsigned)n_partial;
  dot_partial_kernel<<<g, RB, 0, s>>>(n, x, y, partial);
  reduce_kernel<<<1, RB, 0, s>>>((int32_t)g, partial, out, sqrt_out ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mdot(hipStream_t s, int64_t n, const double* V, int64_t ldv, int32_t m, const double* w,
                       double* partial, int32_t n_partial, double* out) {
  int cap = n_partial / (m > 0 ? m : 1);
  if (cap < 1) cap = 1;
  if (cap > 256) cap = 256;
  unsigned g = (unsigned)((n + RB * 4 - 1) / (RB * 4));
  if (g < 1) g = 1;
  if (g > (unsigned)cap) g = (unsigned)cap;
  if (m <= 8) mdot_partial_kernel<8><<<g, RB, 0, s>>>(n, V, ldv, m, w, partial);
  else if (m <= 16) mdot_partial_kernel<16><<<g, RB, 0, s>>>(n, V, ldv, m, w, partial);
  else if (m <= 32) mdot_partial_kernel<32><<<g, RB, 0, s>>>(n, V, ldv, m, w, partial);
  else mdot_partial_kernel<VK_MAX_RESTART + 1><<<g, RB, 0, s>>>(n, V, ldv, m, w, partial);
  mreduce_kernel<<<(unsigned)m, RB, 0, s>>>((int32_t)g, m, partial, out);
  return hipGetLastError();
}

hipError_t launch_maxpy(hipStream_t s, int64_t n, const double* V, int64_t ldv, int32_t m, const double* h,
                        double sign, double* w) {
  const unsigned g = grid_n(n, 2048);
  if (m <= 8) maxpy_kernel<8><<<g, RB, 0, s>>>(n, V, ldv, m, h, sign, w);
  else if (m <= 16) maxpy_kernel<16><<<g, RB, 0, s>>>(n, V, ldv, m, h, sign, w);
  else if (m <= 32) maxpy_kernel<32><<<g, RB, 0, s>>>(n, V, ldv, m, h, sign, w);
  else maxpy_kernel<VK_MAX_RESTART + 1><<<g, RB, 0, s>>>(n, V, ldv, m, h, sign, w);
  return hipGetLastError();
}

hipError_t launch_scale_by_inv(hipStream_t s, int64_t n, const double* x, const double* den, double* y) {
  scale_by_inv_kernel<<<grid_n(n, 2048), RB, 0, s>>>(n, x, den, y);
  return hipGetLastError();
}

hipError_t launch_givens(hipStream_t s, int32_t j, int32_t ldh, double* H, const double* h2, double* cs, double* sn,
                         double* g, double* out) {
  givens_kernel<<<1, 64, 0, s>>>(j, ldh, H, h2, cs, sn, g, out);
  return hipGetLastError();
}

hipError_t launch_gmres_init(hipStream_t s, int32_t m, double* H, double* g, const double* beta) {
  gmres_init_kernel<<<1, 256, 0, s>>>(m, H, g, beta);
  return hipGetLastError();
}

hipError_t launch_trisolve(hipStream_t s, int32_t jn, int32_t ldh, const double* H, const double* g, double* y) {
  trisolve_kernel<<<1, 64, 0, s>>>(jn, ldh, H, g, y);
  return hipGetLastError();
}
