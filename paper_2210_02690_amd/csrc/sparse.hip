// CSR kernels: y = alpha A x + beta z (defects r = b - J d, restriction R r,
// prolongation d += P e), structural validation and fills.
#include "vk_internal.h"

namespace {

// LPR lanes cooperate on one row; LPR divides the 64-wide wavefront.  A lane takes two
// consecutive entries at a time (one 16-byte load of the values, one 8-byte load of the columns),
// the row's lanes together 2 LPR consecutive entries, so a row's stream is read in whole 16-byte
// pieces: an odd first entry (whose pair would straddle the 16-byte boundary) goes to the row's
// last lane on its own, and an odd last entry is the lone half of the last pair.  Two pairs are in
// flight per lane and iteration.  (The value array is 16-byte aligned, as device allocations are.)
template <int LPR>
__global__ __launch_bounds__(256) void spmv_kernel(int64_t n_rows, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x, double alpha, double beta,
                                                   const double* z, double* y) {
  const int64_t gid = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t row = gid / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (row < n_rows) {
    int64_t e0 = row_ptr[row];
    const int64_t e1 = row_ptr[row + 1];
    if ((e0 & 1) && e0 < e1) {  // the odd head entry
      if (lane == LPR - 1) s3 = val[e0] * x[col[e0]];
      ++e0;
    }
    int64_t e = e0 + 2 * lane;
    for (; e + 2 * LPR + 1 < e1; e += 4 * LPR) {
      const int2 c01 = *reinterpret_cast<const int2*>(col + e);
      const int2 c23 = *reinterpret_cast<const int2*>(col + e + 2 * LPR);
      const double2 v01 = *reinterpret_cast<const double2*>(val + e);
      const double2 v23 = *reinterpret_cast<const double2*>(val + e + 2 * LPR);
      s0 = fma(v01.x, x[c01.x], s0);
      s1 = fma(v01.y, x[c01.y], s1);
      s2 = fma(v23.x, x[c23.x], s2);
      s3 = fma(v23.y, x[c23.y], s3);
    }
    for (; e + 1 < e1; e += 2 * LPR) {
      const int2 c01 = *reinterpret_cast<const int2*>(col + e);
      const double2 v01 = *reinterpret_cast<const double2*>(val + e);
      s0 = fma(v01.x, x[c01.x], s0);
      s1 = fma(v01.y, x[c01.y], s1);
    }
    if (e < e1) s2 = fma(val[e], x[col[e]], s2);  // the odd tail entry
  }
  double sum = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, LPR);
  if (row < n_rows && lane == 0) {
    double v = alpha * sum;
    if (beta != 0.0) v += beta * z[row];
    y[row] = v;
  }
}

// Grouped CSR (gcsr): g_row[g] .. g_row[g + 1] - 1 are G <= 4 consecutive rows of equal length m
// whose columns agree entry by entry up to a shift, col[r + c][j] = col[r][j] + c d_j with d_j in
// {0, 1} (in a dG slab matrix: the velocity components of one node, or the pressure modes of one
// cell).  The group's column list is stored once, gcol[g_coff[g] + j] = col[r][j] | d_j << 31; the
// values are the CSR values as they are (the rows are consecutive, so row r + c's entries start at
// row_ptr[r] + c m; g_v0[g] = row_ptr[r] is stored with the group).  LPR lanes per group, each
// takes entry j of all G rows: one 4-byte column word serves G values.
// sum over the 64 lanes, complete in lane 63: DPP shifts within rows of 16, then row broadcasts
__device__ inline double wave_sum_to63(double v) {
  v += dpp_move<0x111, 0xF>(v, 0.0);
  v += dpp_move<0x112, 0xF>(v, 0.0);
  v += dpp_move<0x114, 0xF>(v, 0.0);
  v += dpp_move<0x118, 0xF>(v, 0.0);
  v += dpp_move<0x142, 0xA>(v, 0.0);
  v += dpp_move<0x143, 0xC>(v, 0.0);
  return v;
}

__device__ inline double readlane_d(double v, int l) {
  const int2 a = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(a.x, l);
  r.y = __builtin_amdgcn_readlane(a.y, l);
  return __builtin_bit_cast(double, r);
}

template <int LPR>
__global__ __launch_bounds__(256) void spmv_g_kernel(int64_t n_groups, const int32_t* __restrict__ g_row,
                                                     const int64_t* __restrict__ g_coff,
                                                     const int64_t* __restrict__ g_v0,
                                                     const uint32_t* __restrict__ gcol,
                                                     const double* __restrict__ val, const double* __restrict__ x,
                                                     double alpha, double beta, const double* z, double* y) {
  const int64_t gid = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t g = gid / LPR;
  const int lane = threadIdx.x & (LPR - 1);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t r = 0;
  int G = 0;
  if (g < n_groups) {
    r = g_row[g];
    G = g_row[g + 1] - (int)r;
    // independent loads: the group's rows, column list and first value (no chain through row_ptr)
    const int64_t c0 = g_coff[g], m = g_coff[g + 1] - c0, v0 = g_v0[g];
    const double* v = val + v0;
    int64_t j = lane;
    // x at the group's column of entry jj, for rows 0..3 of the group: unshifted columns (d = 0,
    // most entries of a velocity node's rows) read x once; shifted ones read the next entries too
    auto xg = [&](uint32_t cw, double (&xv)[4]) {
      const int64_t b = (int64_t)(cw & 0x7fffffffu);
      xv[0] = x[b];
      xv[1] = xv[2] = xv[3] = xv[0];
      if (cw >> 31) {
        if (G > 1) xv[1] = x[b + 1];
        if (G > 2) xv[2] = x[b + 2];
        if (G > 3) xv[3] = x[b + 3];
      }
    };
    // two entries per lane and iteration: their value loads and gathers in flight together.  All
    // loads go through the caches: non-temporal value and column loads made the batch's 1.8 GB J
    // slower here (the autotuner then kept CSR for it), unlike in the one-group-per-wavefront kernel
    auto ldv = [&](int64_t i) { return v[i]; };
    auto ldc = [&](int64_t i) { return gcol[i]; };
    for (; j + LPR < m; j += 2 * LPR) {
      const uint32_t ca = ldc(c0 + j), cb = ldc(c0 + j + LPR);
      double xa[4], xb[4];
      xg(ca, xa);
      xg(cb, xb);
      s0 = fma(ldv(j), xa[0], s0);
      s0 = fma(ldv(j + LPR), xb[0], s0);
      if (G > 1) {
        s1 = fma(ldv(m + j), xa[1], s1);
        s1 = fma(ldv(m + j + LPR), xb[1], s1);
      }
      if (G > 2) {
        s2 = fma(ldv(2 * m + j), xa[2], s2);
        s2 = fma(ldv(2 * m + j + LPR), xb[2], s2);
      }
      if (G > 3) {
        s3 = fma(ldv(3 * m + j), xa[3], s3);
        s3 = fma(ldv(3 * m + j + LPR), xb[3], s3);
      }
    }
    if (j < m) {
      double xa[4];
      xg(ldc(c0 + j), xa);
      s0 = fma(ldv(j), xa[0], s0);
      if (G > 1) s1 = fma(ldv(m + j), xa[1], s1);
      if (G > 2) s2 = fma(ldv(2 * m + j), xa[2], s2);
      if (G > 3) s3 = fma(ldv(3 * m + j), xa[3], s3);
    }
  }
  if constexpr (LPR == 64) {
    // one group per wavefront: DPP sums (rows of 16, then across rows), read from lane 63
    s0 = wave_sum_to63(s0);
    s1 = wave_sum_to63(s1);
    s2 = wave_sum_to63(s2);
    s3 = wave_sum_to63(s3);
    s0 = readlane_d(s0, 63);
    s1 = readlane_d(s1, 63);
    s2 = readlane_d(s2, 63);
    s3 = readlane_d(s3, 63);
  } else {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o, LPR);
      s1 += __shfl_xor(s1, o, LPR);
      s2 += __shfl_xor(s2, o, LPR);
      s3 += __shfl_xor(s3, o, LPR);
    }
  }
  if (g < n_groups && lane < G) {
    const double sum = lane == 0 ? s0 : (lane == 1 ? s1 : (lane == 2 ? s2 : s3));
    double out = alpha * sum;
    if (beta != 0.0) out += beta * z[r + lane];
    y[r + lane] = out;
  }
}

// One group per wavefront (64 lanes per group, the J of 3D patches with rows of a few hundred
// entries).  The group is the same for the whole wavefront, so its description is read with scalar
// loads and its size G selects straight-line code: per iteration a lane takes the adjacent entries
// j and j + 1 of all G rows, issues its two column words and one 16-byte value load per row first and
// then the gathers of x, so the values stream while the gathers wait on their column words (16-byte
// value loads instead of two 8-byte ones: 0.667 -> 0.635 ms for the 3D finest J).  A lane past the
// row's end keeps its sums.  x of a shifted entry's rows 1..G-1 is loaded only on the lanes that need
// it, into registers that start at zero, so no loaded value is copied before the wait for it.  Two
// entries per lane keep 8 wavefronts per SIMD (four entries needed 94 registers and were slower).
// With NTL the values, read once, load non-temporally; the column words stay cacheable (a line of
// them is shared by neighbouring groups).
template <int G, int E, bool NTL>
__device__ inline void group_dot64(int lane, int64_t m, const uint32_t* __restrict__ gc,
                                   const double* __restrict__ v, const double* __restrict__ x, double (&s)[4]) {
  static_assert(E == 2, "a lane takes two adjacent entries");
  if (m < 2) {  // a row of one entry (or none) has no pair: lane 0 alone
    if (m == 1 && lane == 0) {
      const uint32_t cw = gc[0];
      const int64_t b0 = (int64_t)(cw & 0x7fffffffu);
#pragma unroll
      for (int c = 0; c < G; ++c) s[c] = fma(v[c], x[b0 + ((cw >> 31) ? c : 0)], s[c]);
    }
    return;
  }
  // the group's values through a buffer resource: 16-byte loads that need only 4-byte alignment
  // (a row's pair starts on any 8-byte boundary), the non-temporal hint as an immediate
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(v), (short)0, (int)(G * m * (int64_t)sizeof(double)), 0x00020000);
  for (int64_t jb = 0; jb < m; jb += 128) {
    // entries j0 and j0 + 1 of every row; the 16-byte pair is read at p0, inside the row (near its
    // end p0 = m - 2, and an odd last entry is the pair's second half)
    const int64_t j0 = jb + 2 * lane;
    bool ok[E];
    uint32_t cw[E];
    ok[0] = j0 < m;
    ok[1] = j0 + 1 < m;
    cw[0] = gc[ok[0] ? j0 : m - 1];
    cw[1] = gc[ok[1] ? j0 + 1 : m - 1];
    const int64_t p0 = j0 < m - 1 ? j0 : m - 2;
    const bool second = j0 != p0;
    double vv[E][G];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int off = (int)((c * m + p0) * (int64_t)sizeof(double));
      const double2 d = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, NTL ? 2 : 0));
      vv[0][c] = second ? d.y : d.x;
      vv[1][c] = d.y;
    }
    // the shifted entries' loads go first: the gathers at the columns come after the branches, so
    // the choice between the two cannot be folded into a branch's default value (which would copy
    // a gather, and wait for it, before the other entries' loads issue)
    int64_t b[E];
    double xs[E][G];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      b[e] = (int64_t)(cw[e] & 0x7fffffffu);
#pragma unroll
      for (int c = 0; c < G; ++c) xs[e][c] = 0.0;
      if (G > 1 && (cw[e] >> 31)) {
#pragma unroll
        for (int c = 1; c < G; ++c) xs[e][c] = x[b[e] + c];
      }
    }
    double x0[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x0[e] = x[b[e]];
#pragma unroll
    for (int c = 0; c < G; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double p = fma(vv[e][c], c == 0 || !(cw[e] >> 31) ? x0[e] : xs[e][c], s[c]);
        s[c] = ok[e] ? p : s[c];
      }
  }
}

__device__ inline int64_t uniform64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <bool NTL>
__global__ __launch_bounds__(256) void spmv_g64_kernel(int64_t n_groups, const int32_t* __restrict__ g_row,
                                                       const int64_t* __restrict__ g_coff,
                                                       const int64_t* __restrict__ g_v0,
                                                       const uint32_t* __restrict__ gcol,
                                                       const double* __restrict__ val,
                                                       const double* __restrict__ x, double alpha, double beta,
                                                       const double* z, double* y) {
  const int64_t g = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (g >= n_groups) return;
  const int lane = threadIdx.x & 63;
  const int64_t r = g_row[g];
  const int G = (int)(g_row[g + 1] - r);
  const int64_t c0 = uniform64(g_coff[g]), m = uniform64(g_coff[g + 1]) - c0, v0 = uniform64(g_v0[g]);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  switch (__builtin_amdgcn_readfirstlane(G)) {
    case 4: group_dot64<4, 2, NTL>(lane, m, gcol + c0, val + v0, x, s); break;
    case 3: group_dot64<3, 2, NTL>(lane, m, gcol + c0, val + v0, x, s); break;
    case 2: group_dot64<2, 2, NTL>(lane, m, gcol + c0, val + v0, x, s); break;
    default: group_dot64<1, 2, NTL>(lane, m, gcol + c0, val + v0, x, s); break;
  }
  double t[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) t[c] = c < G ? readlane_d(wave_sum_to63(s[c]), 63) : 0.0;
  if (lane < G) {
    const double sum = lane == 0 ? t[0] : (lane == 1 ? t[1] : (lane == 2 ? t[2] : t[3]));
    double out = alpha * sum;
    if (beta != 0.0) out += beta * z[r + lane];
    y[r + lane] = out;
  }
}

__global__ void validate_csr_kernel(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                    int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && (row_ptr[0] != 0 || row_ptr[n_rows] != nnz)) atomicOr(flag, 1);
  if (i >= n_rows) return;
  const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
  if (e0 < 0 || e1 > nnz || e0 > e1) {
    atomicOr(flag, 2);
    return;
  }
  int64_t prev = -1;
  for (int64_t e = e0; e < e1; ++e) {
    const int64_t c = col[e];
    if (c < 0 || c >= n_cols) {
      atomicOr(flag, 4);
      return;
    }
    if (c <= prev) {
      atomicOr(flag, 8);
      return;
    }
    prev = c;
  }
}

__global__ void validate_cells_kernel(int32_t n_cells, int32_t n_K, const int32_t* __restrict__ cell_dofs,
                                      int64_t n, const int32_t* __restrict__ colour_cells, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)n_cells * n_K) {
    const int32_t v = cell_dofs[i];
    if (v < 0 || v >= n) atomicOr(flag, 16);
  }
  if (i < n_cells) {
    const int32_t c = colour_cells[i];
    if (c < 0 || c >= n_cells) atomicOr(flag, 32);
  }
}

// Colour c of a cell group: every cell of the colour sets bit c of its DoFs' masks; a bit that was
// already set means two cells of the colour share that DoF.
__global__ void colour_conflict_kernel(int32_t c, int32_t n0, int32_t cnt, int32_t n_K,
                                       const int32_t* __restrict__ cell_dofs,
                                       const int32_t* __restrict__ colour_cells, unsigned long long* mask,
                                       int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)cnt * n_K) return;
  const int32_t K = colour_cells[n0 + i / n_K];
  const int32_t mu = cell_dofs[(int64_t)K * n_K + i % n_K];
  const unsigned long long bit = 1ull << c;
  if (atomicOr(mask + mu, bit) & bit) atomicOr(flag, 1);
}

__global__ void fill_kernel(int64_t n, double v, double* x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void fill_i32_kernel(int64_t n, int32_t v, int32_t* x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

inline unsigned grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int vk_pick_lpr(int64_t n_rows, int64_t nnz) {
  const double avg = n_rows > 0 ? (double)nnz / (double)n_rows : 0.0;
  if (avg >= 96) return 64;
  if (avg >= 40) return 32;
  if (avg >= 20) return 16;
  if (avg >= 10) return 8;
  return 4;
}

hipError_t launch_spmv(hipStream_t s, const vk_csr& A, int lpr, double alpha, const double* x, double beta,
                       const double* z, double* y) {
  if (A.n_rows == 0) return hipSuccess;
  const unsigned grid = grid_for(A.n_rows * lpr, 256);
  switch (lpr) {
    case 1: spmv_kernel<1><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
    case 2: spmv_kernel<2><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
    case 4: spmv_kernel<4><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
    case 8: spmv_kernel<8><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
    case 16: spmv_kernel<16><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
    case 32: spmv_kernel<32><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
    default: spmv_kernel<64><<<grid, 256, 0, s>>>(A.n_rows, A.row_ptr, A.col, A.val, x, alpha, beta, z, y); break;
  }
  return hipGetLastError();
}

hipError_t launch_spmv_g(hipStream_t s, const vk_csr& A, const vk_gcsr& g, int lpr, double alpha, const double* x,
                         double beta, const double* z, double* y) {
  if (g.n_groups == 0) return hipSuccess;
  const unsigned grid = grid_for(g.n_groups * lpr, 256);
  const bool ntl = A.nnz * 12 > (1ll << 30);  // well beyond the 256 MB last-level cache
#define VK_SPMV_G(LL)                                                                                          \
  spmv_g_kernel<LL><<<grid, 256, 0, s>>>(g.n_groups, g.g_row, g.g_coff, g.g_v0, g.gcol, A.val, x, alpha, beta, z, y)
  switch (lpr) {
    case 4: VK_SPMV_G(4); break;
    case 8: VK_SPMV_G(8); break;
    case 16: VK_SPMV_G(16); break;
    case 32: VK_SPMV_G(32); break;
    default:
      if (ntl)
        spmv_g64_kernel<true><<<grid, 256, 0, s>>>(g.n_groups, g.g_row, g.g_coff, g.g_v0, g.gcol, A.val, x, alpha,
                                                   beta, z, y);
      else
        spmv_g64_kernel<false><<<grid, 256, 0, s>>>(g.n_groups, g.g_row, g.g_coff, g.g_v0, g.gcol, A.val, x, alpha,
                                                    beta, z, y);
      break;
  }
#undef VK_SPMV_G
  return hipGetLastError();
}

hipError_t launch_validate_csr(hipStream_t s, const vk_csr& A, int32_t* flag) {
  validate_csr_kernel<<<grid_for(A.n_rows + 1, 256), 256, 0, s>>>(A.n_rows, A.n_cols, A.nnz, A.row_ptr, A.col,
                                                                    flag);
  return hipGetLastError();
}

hipError_t launch_validate_cells(hipStream_t s, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs, int64_t n,
                                 const int32_t* colour_cells, int32_t* flag) {
  validate_cells_kernel<<<grid_for((int64_t)n_cells * n_K, 256), 256, 0, s>>>(n_cells, n_K, cell_dofs, n,
                                                                              colour_cells, flag);
  return hipGetLastError();
}

hipError_t launch_colour_check(hipStream_t s, int32_t n_K, const int32_t* cell_dofs, const int32_t* colour_cells,
                               const int32_t* colour_ptr, int32_t n_colours, unsigned long long* mask,
                               int32_t* flag) {
  for (int32_t c = 0; c < n_colours && c < 64; ++c) {
    const int32_t n0 = colour_ptr[c], cnt = colour_ptr[c + 1] - colour_ptr[c];
    if (cnt <= 0) continue;
    colour_conflict_kernel<<<grid_for((int64_t)cnt * n_K, 256), 256, 0, s>>>(c, n0, cnt, n_K, cell_dofs,
                                                                             colour_cells, mask, flag);
  }
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, int64_t n, double v, double* x) {
  if (n == 0) return hipSuccess;
  unsigned g = grid_for(n, 256);
  if (g > 4096) g = 4096;
  fill_kernel<<<g, 256, 0, s>>>(n, v, x);
  return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t s, int64_t n, int32_t v, int32_t* x) {
  if (n == 0) return hipSuccess;
  unsigned g = grid_for(n, 256);
  if (g > 4096) g = 4096;
  fill_i32_kernel<<<g, 256, 0, s>>>(n, v, x);
  return hipGetLastError();
}
