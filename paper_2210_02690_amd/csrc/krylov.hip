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

// acc[i] += V_i[r] w[r] over the rows r = r0, r0 + stride, ... below e.  U rows at a time: their loads
// are all issued before the first product, then the rows are added in order (the same sums, in the
// same order, as one row at a time)
template <int MB, int U>
__device__ inline void rows_mdot(int64_t r, int64_t e, int64_t stride, const double* __restrict__ V, int64_t ldv,
                                 int32_t m, const double* __restrict__ w, double (&acc)[MB]) {
  for (; r + (U - 1) * stride < e; r += U * stride) {
    double wr[U], v[U][MB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      wr[u] = w[r + u * stride];
#pragma unroll
      for (int i = 0; i < MB; ++i) v[u][i] = i < m ? V[(int64_t)i * ldv + r + u * stride] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < MB; ++i)
        if (i < m) acc[i] += v[u][i] * wr[u];
  }
  for (; r < e; r += stride) {
    const double wr = w[r];
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (i < m) acc[i] += V[(int64_t)i * ldv + r] * wr;
  }
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
  // one workgroup per CU at most: the rows of a thread are many, so several are loaded at once
  rows_mdot<MB, MB <= 8 ? 4 : (MB <= 16 ? 2 : 1)>((int64_t)blockIdx.x * RB + threadIdx.x, n, (int64_t)gridDim.x * RB, V,
                                                  ldv, m, w, acc);
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
  if (threadIdx.x < MB) sh[threadIdx.x] = (int)threadIdx.x < m ? h[threadIdx.x] : 0.0;
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

// ---- segmented kernels: one independent system per segment [seg[s], seg[s+1]) ----

// partial[s * nc + c] = sum over chunk c of segment s of x * y
__global__ __launch_bounds__(RB) void seg_dot_partial_kernel(const int64_t* __restrict__ seg, int32_t nc,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ y, double* partial) {
  __shared__ double sh[RB / 64];
  const int sg = blockIdx.y, c = blockIdx.x;
  const int64_t e = seg[sg + 1];
  double acc = 0.0;
  for (int64_t i = seg[sg] + (int64_t)c * RB + threadIdx.x; i < e; i += (int64_t)nc * RB) acc += x[i] * y[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)sg * nc + c] = acc;
}

__global__ __launch_bounds__(RB) void seg_reduce_kernel(int32_t nc, const double* __restrict__ partial, double* out,
                                                        int sqrt_out) {
  __shared__ double sh[RB / 64];
  const int sg = blockIdx.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < nc; c += RB) acc += partial[(int64_t)sg * nc + c];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[sg] = sqrt_out ? sqrt(acc) : acc;
}

// partial[((s * nc + c) * m) + i] = chunk c of segment s of V_i . w
template <int MB>
__global__ __launch_bounds__(RB) void seg_mdot_partial_kernel(const int64_t* __restrict__ seg, int32_t nc,
                                                              const double* __restrict__ V, int64_t ldv, int32_t m,
                                                              const double* __restrict__ w, double* partial) {
  __shared__ double sh[RB / 64];
  const int sg = blockIdx.y, c = blockIdx.x;
  const int64_t e = seg[sg + 1];
  double acc[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) acc[i] = 0.0;
  // many workgroups: two rows at a time keeps the registers (and the occupancy) low
  rows_mdot<MB, MB <= 8 ? 2 : 1>(seg[sg] + (int64_t)c * RB + threadIdx.x, e, (int64_t)nc * RB, V, ldv, m, w, acc);
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (i < m) {  // uniform
      const double t = block_sum(acc[i], sh);
      if (threadIdx.x == 0) partial[((int64_t)sg * nc + c) * m + i] = t;
    }
  }
}

// out[s * ldo + i] = sum_c partial[(s * nc + c) * m + i]
__global__ __launch_bounds__(RB) void seg_mreduce_kernel(int32_t nc, int32_t m, const double* __restrict__ partial,
                                                         double* out, int32_t ldo) {
  __shared__ double sh[RB / 64];
  const int i = blockIdx.x, sg = blockIdx.y;
  double acc = 0.0;
  for (int c = threadIdx.x; c < nc; c += RB) acc += partial[((int64_t)sg * nc + c) * m + i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(int64_t)sg * ldo + i] = acc;
}

// w[r] += sign * sum_i h[s * ldh + i] V_i[r] for r in segment s
template <int MB>
__global__ __launch_bounds__(RB) void seg_maxpy_kernel(const int64_t* __restrict__ seg, int32_t nc,
                                                       const double* __restrict__ V, int64_t ldv, int32_t m,
                                                       const double* __restrict__ h, int32_t ldh, double sign,
                                                       double* w) {
  __shared__ double sh[MB];
  const int sg = blockIdx.y, c = blockIdx.x;
  if (threadIdx.x < MB) sh[threadIdx.x] = (int)threadIdx.x < m ? h[(int64_t)sg * ldh + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t e = seg[sg + 1];
  for (int64_t r = seg[sg] + (int64_t)c * RB + threadIdx.x; r < e; r += (int64_t)nc * RB) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (i < m) acc += sh[i] * V[(int64_t)i * ldv + r];
    w[r] += sign * acc;
  }
}

// y = x / den[s] on active segments, 0 on inactive ones
__global__ __launch_bounds__(RB) void seg_scale_kernel(const int64_t* __restrict__ seg, int32_t nc,
                                                       const double* __restrict__ x, const double* __restrict__ den,
                                                       const int32_t* __restrict__ active, double* y) {
  const int sg = blockIdx.y, c = blockIdx.x;
  const double d = den[sg];
  const double sc = (active[sg] && d != 0.0) ? 1.0 / d : 0.0;
  const int64_t e = seg[sg + 1];
  for (int64_t r = seg[sg] + (int64_t)c * RB + threadIdx.x; r < e; r += (int64_t)nc * RB) y[r] = x[r] * sc;
}

// per segment: clear H, g = beta e_1, activity from the true residual
__global__ void seg_init_kernel(int32_t m, double* H, double* g, const double* __restrict__ beta,
                                const double* __restrict__ tol, const int32_t* __restrict__ its, int32_t max_iter,
                                int32_t* active, int32_t* jn) {
  const int sg = blockIdx.x;
  const int64_t hs = (int64_t)(m + 1) * m;
  for (int64_t i = threadIdx.x; i < hs; i += blockDim.x) H[sg * hs + i] = 0.0;
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[(int64_t)sg * (m + 1) + i] = (i == 0) ? beta[sg] : 0.0;
  if (threadIdx.x == 0) {
    active[sg] = (beta[sg] > tol[sg] && its[sg] < max_iter) ? 1 : 0;
    jn[sg] = 0;
  }
}

// one thread per segment: complete column j of H, rotate, update g, counters
__global__ void seg_givens_kernel(int32_t n_seg, int32_t j, int32_t m, double* H, const double* __restrict__ h2,
                                  const double* __restrict__ nrm, double* cs, double* sn, double* g,
                                  const double* __restrict__ tol, int32_t* its, int32_t max_iter, int32_t* active,
                                  int32_t* jn, double* resid) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= n_seg || !active[sg]) return;
  const int ldh = m + 1;
  double* col = H + (int64_t)sg * ldh * m + (int64_t)j * ldh;
  const double* hh = h2 + (int64_t)sg * ldh;
  double* c_ = cs + (int64_t)sg * m;
  double* s_ = sn + (int64_t)sg * m;
  double* gg = g + (int64_t)sg * ldh;
  for (int i = 0; i <= j; ++i) col[i] += hh[i];
  const double hn = nrm[sg];
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = c_[i] * col[i] + s_[i] * col[i + 1];
    col[i + 1] = -s_[i] * col[i] + c_[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], b = col[j + 1];
  const double den = hypot(a, b);
  const double c = den != 0.0 ? a / den : 1.0;
  const double s = den != 0.0 ? b / den : 0.0;
  c_[j] = c;
  s_[j] = s;
  col[j] = den;
  col[j + 1] = 0.0;
  gg[j + 1] = -s * gg[j];
  gg[j] = c * gg[j];
  const double res = fabs(gg[j + 1]);
  resid[sg] = res;
  its[sg] += 1;
  jn[sg] = j + 1;
  if (!(res > tol[sg]) || hn == 0.0 || its[sg] >= max_iter || !isfinite(res)) active[sg] = 0;
}

// y_s = R_s^{-1} g_s on the first jn[s] entries, zero beyond
__global__ void seg_trisolve_kernel(int32_t n_seg, int32_t m, const double* __restrict__ H,
                                    const double* __restrict__ g, const int32_t* __restrict__ jn, double* y) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= n_seg) return;
  const int ldh = m + 1;
  const double* Hs = H + (int64_t)sg * ldh * m;
  const double* gs = g + (int64_t)sg * ldh;
  double* ys = y + (int64_t)sg * m;
  const int n = jn[sg];
  for (int i = m - 1; i >= n; --i) ys[i] = 0.0;
  for (int i = n - 1; i >= 0; --i) {
    double acc = gs[i];
    for (int k = i + 1; k < n; ++k) acc -= Hs[(int64_t)k * ldh + i] * ys[k];
    ys[i] = acc / Hs[(int64_t)i * ldh + i];
  }
}

inline int32_t seg_chunks(int64_t max_len, int32_t n_seg, int32_t n_partial, int32_t m) {
  int64_t nc = (max_len + RB * 4 - 1) / (RB * 4);
  if (nc < 1) nc = 1;
  if (nc > 64) nc = 64;
  const int64_t cap = n_partial / ((int64_t)n_seg * (m > 0 ? m : 1));
  if (nc > cap) nc = cap;
  return (int32_t)(nc < 1 ? 1 : nc);
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

hipError_t launch_seg_dot(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* x,
                          const double* y, double* partial, int32_t n_partial, double* out, bool sqrt_out) {
  const int32_t nc = seg_chunks(max_len, n_seg, n_partial, 1);
  seg_dot_partial_kernel<<<dim3(nc, n_seg), RB, 0, s>>>(seg, nc, x, y, partial);
  seg_reduce_kernel<<<n_seg, RB, 0, s>>>(nc, partial, out, sqrt_out ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_seg_mdot(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* V,
                           int64_t ldv, int32_t m, const double* w, double* partial, int32_t n_partial, double* out,
                           int32_t ldo) {
  const int32_t nc = seg_chunks(max_len, n_seg, n_partial, m);
  const dim3 g(nc, n_seg);
  if (m <= 8) seg_mdot_partial_kernel<8><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, w, partial);
  else if (m <= 16) seg_mdot_partial_kernel<16><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, w, partial);
  else if (m <= 32) seg_mdot_partial_kernel<32><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, w, partial);
  else seg_mdot_partial_kernel<VK_MAX_RESTART + 1><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, w, partial);
  seg_mreduce_kernel<<<dim3(m, n_seg), RB, 0, s>>>(nc, m, partial, out, ldo);
  return hipGetLastError();
}

hipError_t launch_seg_maxpy(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* V,
                            int64_t ldv, int32_t m, const double* h, int32_t ldh, const int32_t* mcount,
                            double sign, double* w) {
  (void)mcount;
  if (m <= 0) return hipSuccess;
  const int32_t nc = seg_chunks(max_len, n_seg, 1 << 30, 1);
  const dim3 g(nc, n_seg);
  if (m <= 8) seg_maxpy_kernel<8><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, h, ldh, sign, w);
  else if (m <= 16) seg_maxpy_kernel<16><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, h, ldh, sign, w);
  else if (m <= 32) seg_maxpy_kernel<32><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, h, ldh, sign, w);
  else seg_maxpy_kernel<VK_MAX_RESTART + 1><<<g, RB, 0, s>>>(seg, nc, V, ldv, m, h, ldh, sign, w);
  return hipGetLastError();
}

hipError_t launch_seg_scale(hipStream_t s, int32_t n_seg, const int64_t* seg, int64_t max_len, const double* x,
                            const double* den, const int32_t* active, double* y) {
  const int32_t nc = seg_chunks(max_len, n_seg, 1 << 30, 1);
  seg_scale_kernel<<<dim3(nc, n_seg), RB, 0, s>>>(seg, nc, x, den, active, y);
  return hipGetLastError();
}

hipError_t launch_seg_init(hipStream_t s, int32_t n_seg, int32_t m, double* H, double* g, const double* beta,
                           const double* tol, const int32_t* its, int32_t max_iter, int32_t* active, int32_t* jn) {
  seg_init_kernel<<<n_seg, 256, 0, s>>>(m, H, g, beta, tol, its, max_iter, active, jn);
  return hipGetLastError();
}

hipError_t launch_seg_givens(hipStream_t s, int32_t n_seg, int32_t j, int32_t m, double* H, const double* h2,
                             double* cs, double* sn, double* g, const double* tol, int32_t* its, int32_t max_iter,
                             int32_t* active, int32_t* jn, double* resid) {
  // h2 holds the second Gram-Schmidt pass; resid[n_seg..2 n_seg) holds the norms of the new vectors
  seg_givens_kernel<<<(n_seg + 63) / 64, 64, 0, s>>>(n_seg, j, m, H, h2, resid + n_seg, cs, sn, g, tol, its,
                                                      max_iter, active, jn, resid);
  return hipGetLastError();
}

hipError_t launch_seg_trisolve(hipStream_t s, int32_t n_seg, int32_t m, const double* H, const double* g,
                               const int32_t* jn, double* y) {
  seg_trisolve_kernel<<<(n_seg + 63) / 64, 64, 0, s>>>(n_seg, m, H, g, jn, y);
  return hipGetLastError();
}
