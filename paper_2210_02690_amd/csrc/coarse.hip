// Coarsest-level direct solve (Sec. 3: a direct solver for J_0 d_0 = b_0 on T_0).
// Setup forms the FP64 inverse of J_0 by Gauss-Jordan elimination with partial
// pivoting spread over the whole GPU: per column k one small kernel picks the
// pivot (first row of maximal |value|) and one grid-wide kernel writes the
// eliminated matrix into the other of two buffers, so no workgroup reads what
// another one writes in the same step.  Each V-cycle then applies the inverse
// with a dense matrix-vector product.
#include "vk_internal.h"

namespace {

__global__ void csr_to_dense_kernel(int64_t n, const int64_t* __restrict__ row_ptr,
                                    const int32_t* __restrict__ col, const double* __restrict__ val, double* M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) M[i * n + col[e]] = val[e];
}

// pivot search in column k over rows k..n-1 of M (one workgroup)
__global__ __launch_bounds__(1024) void coarse_pivot_kernel(int64_t n, int64_t k, const double* __restrict__ M,
                                                            int32_t* perm, int32_t* status) {
  __shared__ double sb[16];
  __shared__ int si[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double best = -1.0;
  int bi = (int)n;
  for (int64_t i = k + tid; i < n; i += blockDim.x) {
    const double a = fabs(M[i * n + k]);
    if (a > best) { best = a; bi = (int)i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if (lane == 0) { sb[wave] = best; si[wave] = bi; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (sb[w] > best || (sb[w] == best && si[w] < bi)) { best = sb[w]; bi = si[w]; }
    const bool bad = bi >= n || !(best > 0.0) || !isfinite(best);
    if (bad) {
      atomicMin(&status[0], -1);
      bi = (int)k;
    }
    perm[k] = bi;
  }
}

// One elimination step: Mout = elimination of column k of Min after swapping
// rows k and p = perm[k].
__global__ __launch_bounds__(256) void coarse_eliminate_kernel(int64_t n, int64_t k, const double* __restrict__ Min,
                                                               double* __restrict__ Mout,
                                                               const int32_t* __restrict__ perm) {
  const int64_t p = perm[k];
  const double pv = Min[p * n + k];
  const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    const double prow = (j == k ? 1.0 : Min[p * n + j]) * inv;
    if (i == k) {
      Mout[e] = prow;
    } else {
      const int64_t src = (i == p) ? k : i;
      const double f = Min[src * n + k];
      Mout[e] = (j == k ? 0.0 : Min[src * n + j]) - f * prow;
    }
  }
}

// Undo the column interchanges: apply the row swaps' inverse to the columns.
__global__ void coarse_colmap_kernel(int64_t n, const int32_t* __restrict__ perm, int32_t* colmap) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int64_t j = 0; j < n; ++j) colmap[j] = (int32_t)j;
  for (int64_t k = n - 1; k >= 0; --k) {
    const int64_t p = perm[k];
    const int32_t t = colmap[k];
    colmap[k] = colmap[p];
    colmap[p] = t;
  }
}

__global__ void coarse_permute_kernel(int64_t n, const double* __restrict__ Min, const int32_t* __restrict__ colmap,
                                      double* __restrict__ Mout) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    Mout[e] = Min[i * n + colmap[j]];
  }
}

// y = A x, A dense row-major n x n, one wavefront per row.
__global__ __launch_bounds__(256) void dense_gemv_kernel(int64_t n, const double* __restrict__ A,
                                                         const double* __restrict__ x, double* __restrict__ y) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = A + row * n;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s += a[j] * x[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[row] = s;
}

}  // namespace

hipError_t launch_coarse_invert(hipStream_t s, const vk_csr& J0, double* inv, double* tmp, int32_t* perm,
                                int32_t* status) {
  const int64_t n = J0.n_rows;
  hipError_t e = launch_fill(s, n * n, 0.0, inv);
  if (e != hipSuccess) return e;
  csr_to_dense_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, J0.row_ptr, J0.col, J0.val, inv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t g = (n * n + 1023) / 1024;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  double* a = inv;
  double* b = tmp;
  for (int64_t k = 0; k < n; ++k) {
    coarse_pivot_kernel<<<1, 1024, 0, s>>>(n, k, a, perm, status);
    coarse_eliminate_kernel<<<(unsigned)g, 256, 0, s>>>(n, k, a, b, perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* t = a;
    a = b;
    b = t;
  }
  // a holds the row-eliminated matrix; the permuted result goes to inv
  int32_t* colmap = perm + n;
  coarse_colmap_kernel<<<1, 1, 0, s>>>(n, perm, colmap);
  if (a == inv) {
    // move to tmp first so the permutation does not read what it writes
    coarse_permute_kernel<<<(unsigned)g, 256, 0, s>>>(n, inv, colmap, tmp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipMemcpyAsync(inv, tmp, (size_t)(n * n) * sizeof(double), hipMemcpyDeviceToDevice, s);
  }
  coarse_permute_kernel<<<(unsigned)g, 256, 0, s>>>(n, a, colmap, inv);
  return hipGetLastError();
}

hipError_t launch_dense_gemv(hipStream_t s, int64_t n, const double* A, const double* x, double* y) {
  dense_gemv_kernel<<<(unsigned)((n * 64 + 255) / 256), 256, 0, s>>>(n, A, x, y);
  return hipGetLastError();
}
