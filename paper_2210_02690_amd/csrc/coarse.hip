// Coarsest-level direct solve (Sec. 3: a direct solver for J_0 d_0 = b_0 on T_0).
//
// Setup inverts the dense FP64 J_0 by blocked Gauss-Jordan elimination with
// partial pivoting (first row of maximal |value| among the rows not yet used).
// For each panel of NB columns:
//   panel kernel  (one workgroup, rows of the panel in registers): the NB
//                 elimination steps restricted to the panel columns; it
//                 records the row interchanges;
//   update kernel (whole GPU): the same transformation applied to every other
//                 column, as the rank-NB update
//                   out[i, c] = (i in panel rows ? 0 : in[src(i), c])
//                               + sum_j X[i, j] in[src(k0 + j), c],
//                 X the eliminated panel, src the panel's row interchanges.
// Two buffers alternate so no workgroup reads what another writes.  The row
// interchanges are not undone on the columns: with rowmap the composition of
// all interchanges, J_0^{-1} b = W b[rowmap], which the V-cycle applies.
#include <climits>

#include "vk_internal.h"

namespace {

constexpr int PT = 1024;  // panel kernel threads

__global__ void csr_to_dense_kernel(int64_t n, const int64_t* __restrict__ row_ptr,
                                    const int32_t* __restrict__ col, const double* __restrict__ val, double* M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) M[i * n + col[e]] = val[e];
}

__global__ void iota_kernel(int64_t n, int32_t* x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (int32_t)i;
}

template <int R, int NB>
__global__ __launch_bounds__(PT) void coarse_panel_kernel(int64_t n, int64_t k0, int nb,
                                                          const double* __restrict__ Min, double* __restrict__ Mout,
                                                          int32_t* __restrict__ src_g, int32_t* rowmap,
                                                          int32_t* status) {
  extern __shared__ int src_l[];  // n entries
  __shared__ double red_abs[PT / 64], red_val[PT / 64];
  __shared__ int red_idx[PT / 64];
  __shared__ double prow[NB], xk[NB], xp[NB];
  __shared__ int s_p, s_piv[NB];
  __shared__ double s_pv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double P[R][NB];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = tid + (int64_t)r * PT;
#pragma unroll
    for (int c = 0; c < NB; ++c) P[r][c] = (i < n && c < nb) ? Min[i * n + k0 + c] : 0.0;
  }
  for (int64_t i = tid; i < n; i += PT) src_l[i] = (int)i;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {  // uniform: every thread sees the same nb
    const int64_t k = k0 + j;
    double babs = -1.0, bval = 0.0;
    int bidx = INT_MAX;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = tid + (int64_t)r * PT;
      if (i >= k && i < n) {
        const double a = fabs(P[r][j]);
        if (a > babs) { babs = a; bval = P[r][j]; bidx = (int)i; }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(babs, o, 64), ov = __shfl_xor(bval, o, 64);
      const int oi = __shfl_xor(bidx, o, 64);
      if (ob > babs || (ob == babs && oi < bidx)) { babs = ob; bval = ov; bidx = oi; }
    }
    if (lane == 0) { red_abs[wave] = babs; red_val[wave] = bval; red_idx[wave] = bidx; }
    __syncthreads();
    if (wave == 0) {
      babs = lane < PT / 64 ? red_abs[lane] : -1.0;
      bval = lane < PT / 64 ? red_val[lane] : 0.0;
      bidx = lane < PT / 64 ? red_idx[lane] : INT_MAX;
      for (int o = 8; o > 0; o >>= 1) {
        const double ob = __shfl_xor(babs, o, 64), ov = __shfl_xor(bval, o, 64);
        const int oi = __shfl_xor(bidx, o, 64);
        if (ob > babs || (ob == babs && oi < bidx)) { babs = ob; bval = ov; bidx = oi; }
      }
      if (lane == 0) {
        const bool bad = bidx >= n || !(babs > 0.0) || !isfinite(babs);
        if (bad) atomicMin(&status[0], -1);
        s_p = bad ? (int)k : bidx;
        s_pv = bad ? 1.0 : bval;
      }
    }
    __syncthreads();
    const int64_t p = s_p;
    const double pv = s_pv;
    const int tk = (int)(k % PT), rk = (int)(k / PT);
    const int tp = (int)(p % PT), rp = (int)(p / PT);
    if (p != k) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (tid == tk && r == rk)
#pragma unroll
          for (int c = 0; c < NB; ++c) xk[c] = P[r][c];
        if (tid == tp && r == rp)
#pragma unroll
          for (int c = 0; c < NB; ++c) xp[c] = P[r][c];
      }
      if (tid == 0) {
        const int t = src_l[k];
        src_l[k] = src_l[p];
        src_l[p] = t;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (tid == tk && r == rk)
#pragma unroll
          for (int c = 0; c < NB; ++c) P[r][c] = xp[c];
        if (tid == tp && r == rp)
#pragma unroll
          for (int c = 0; c < NB; ++c) P[r][c] = xk[c];
      }
    }
    if (tid == 0) s_piv[j] = (int)p;
    const double inv = 1.0 / pv;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (tid == tk && r == rk)
#pragma unroll
        for (int c = 0; c < NB; ++c) prow[c] = (c == j ? 1.0 : P[r][c]) * inv;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = tid + (int64_t)r * PT;
      if (i < n) {
        if (i == k) {
#pragma unroll
          for (int c = 0; c < NB; ++c) P[r][c] = prow[c];
        } else {
          const double f = P[r][j];
#pragma unroll
          for (int c = 0; c < NB; ++c) P[r][c] = (c == j ? 0.0 : P[r][c]) - f * prow[c];
        }
      }
    }
    __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = tid + (int64_t)r * PT;
    if (i < n)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) Mout[i * n + k0 + c] = P[r][c];
  }
  for (int64_t i = tid; i < n; i += PT) src_g[i] = src_l[i];
  if (tid == 0) {
    for (int j = 0; j < nb; ++j) {
      const int64_t k = k0 + j, p = s_piv[j];
      const int32_t t = rowmap[k];
      rowmap[k] = rowmap[p];
      rowmap[p] = t;
    }
  }
}

// Rank-NB update of the columns outside the panel; tiles of 32 rows x 64 columns.
template <int NB>
__global__ __launch_bounds__(256) void coarse_update_kernel(int64_t n, int64_t k0, int nb,
                                                            const double* __restrict__ Min, double* Mout,
                                                            const int32_t* __restrict__ src) {
  __shared__ double Rt[NB][64];
  __shared__ double Xt[32][NB + 1];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * 64; e += 256) {
    const int j = e >> 6, cc = e & 63;
    const int64_t c = c0 + cc;
    Rt[j][cc] = (j < nb && c < n) ? Min[(int64_t)src[k0 + j] * n + c] : 0.0;
  }
  for (int e = tid; e < 32 * NB; e += 256) {
    const int rr = e / NB, j = e - rr * NB;
    const int64_t i = r0 + rr;
    Xt[rr][j] = (i < n && j < nb) ? Mout[i * n + k0 + j] : 0.0;
  }
  __syncthreads();
  const int tx = tid & 63, ty = tid >> 6;
  const int64_t c = c0 + tx;
  if (c >= n || (c >= k0 && c < k0 + nb)) return;
  for (int s = 0; s < 8; ++s) {
    const int rr = ty + 4 * s;
    const int64_t i = r0 + rr;
    if (i >= n) break;
    double acc = (i >= k0 && i < k0 + nb) ? 0.0 : Min[(int64_t)src[i] * n + c];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc = fma(Xt[rr][j], Rt[j][tx], acc);
    Mout[i * n + c] = acc;
  }
}

// y = W x[rowmap], W dense row-major n x n, one wavefront per row.
__global__ __launch_bounds__(256) void coarse_apply_kernel(int64_t n, const double* __restrict__ W,
                                                           const int32_t* __restrict__ rowmap,
                                                           const double* __restrict__ x, double* __restrict__ y) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* w = W + row * n;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s = fma(w[j], x[rowmap[j]], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[row] = s;
}

// out[r, rowmap[i]] = W[r, i]: the inverse with the interchanges undone
__global__ void coarse_export_kernel(int64_t n, const double* __restrict__ W, const int32_t* __restrict__ rowmap,
                                     double* out) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, i = e - r * n;
    out[r * n + rowmap[i]] = W[e];
  }
}

template <int R, int NB>
hipError_t run_blocked(hipStream_t s, int64_t n, double** a, double** b, int32_t* src, int32_t* rowmap,
                       int32_t* status) {
  const size_t lds = (size_t)n * sizeof(int);
  const dim3 ugrid((unsigned)((n + 63) / 64), (unsigned)((n + 31) / 32));
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int nb = (int)((n - k0) < NB ? (n - k0) : NB);
    coarse_panel_kernel<R, NB><<<1, PT, lds, s>>>(n, k0, nb, *a, *b, src, rowmap, status);
    coarse_update_kernel<NB><<<ugrid, 256, 0, s>>>(n, k0, nb, *a, *b, src);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* t = *a;
    *a = *b;
    *b = t;
  }
  return hipSuccess;
}

}  // namespace

int64_t vk_coarse_max_n() { return 15360; }

hipError_t launch_coarse_invert(hipStream_t s, const vk_csr& J0, double* buf0, double* buf1, int32_t* perm,
                                int32_t* status, double** result) {
  const int64_t n = J0.n_rows;
  hipError_t e = launch_fill(s, n * n, 0.0, buf0);
  if (e != hipSuccess) return e;
  csr_to_dense_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, J0.row_ptr, J0.col, J0.val, buf0);
  int32_t* rowmap = perm;
  int32_t* src = perm + n;
  iota_kernel<<<(unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096), 256, 0, s>>>(n, rowmap);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double* a = buf0;
  double* b = buf1;
  const int64_t R = (n + PT - 1) / PT;
  // R rows x NB panel columns per thread, R * NB <= 32 doubles (the register
  // budget of a 1024-thread workgroup)
  if (R <= 1) e = run_blocked<1, 32>(s, n, &a, &b, src, rowmap, status);
  else if (R <= 2) e = run_blocked<2, 16>(s, n, &a, &b, src, rowmap, status);
  else if (R <= 4) e = run_blocked<4, 8>(s, n, &a, &b, src, rowmap, status);
  else if (R <= 8) e = run_blocked<8, 4>(s, n, &a, &b, src, rowmap, status);
  else e = run_blocked<16, 2>(s, n, &a, &b, src, rowmap, status);
  *result = a;
  return e;
}

hipError_t launch_coarse_apply(hipStream_t s, int64_t n, const double* W, const int32_t* rowmap, const double* x,
                               double* y) {
  coarse_apply_kernel<<<(unsigned)((n * 64 + 255) / 256), 256, 0, s>>>(n, W, rowmap, x, y);
  return hipGetLastError();
}

hipError_t launch_coarse_export(hipStream_t s, int64_t n, const double* W, const int32_t* rowmap, double* out) {
  int64_t g = (n * n + 255) / 256;
  if (g > 8192) g = 8192;
  coarse_export_kernel<<<(unsigned)g, 256, 0, s>>>(n, W, rowmap, out);
  return hipGetLastError();
}
