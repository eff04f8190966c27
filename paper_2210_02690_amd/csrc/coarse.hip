// Directly solved diagonal blocks: the coarsest level (Sec. 3: a direct solver
// for J_0 d_0 = b_0 on T_0), and in a batch of independent systems every
// system's coarsest level.  All blocks of a level are processed together.
//
// Setup inverts each dense FP64 block in place by blocked Gauss-Jordan
// elimination with implicit partial pivoting: the pivot of column k is the
// not-yet-used row q_k with the largest |value| (the first such row on ties);
// rows never move.  The stored matrix W then satisfies
// J^{-1}[k][q_j] = W[q_k][j], so the solve is y[k] = sum_j W[q_k][j] b[q_j].
//
// During the elimination each block is stored column-major, so a panel's
// columns are contiguous; a final in-place transpose leaves W row-major for the
// solve.
//
// Two levels of blocking.  The columns are taken in outer blocks of NBO = 128
// (levels with one or a few blocks) or 64 columns; within an outer block, inner
// panels of NB columns:
//   panel kernel  (one workgroup per block, the panel rows in registers): the
//                 NB elimination steps restricted to the panel's columns; it
//                 records each new pivot row's column and copies the pivot
//                 rows' old values in the rest of the outer block;
//   inner update: the same steps on the rest of the outer block (rank NB).
// After the outer block's columns are eliminated, one rank-NBO update brings
// every other column along; eliminating a set of pivots P at once gives, for
// the eliminated columns C and any other column c,
//   W'[i, c] = (i in P ? 0 : W[i, c]) + sum_{t in C} W'[i, t] W[q_t, c],
// a GEMM on the FP64 matrix cores (the pivot rows' old values are copied out
// first, so the update runs in place).
#include <climits>

#include "vk_internal.h"

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));


__device__ inline int block_of(const int64_t* __restrict__ rows, int nb, int64_t r) {
  int lo = 0, hi = nb;  // last block with rows[b] <= r
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rows[mid] <= r) lo = mid; else hi = mid;
  }
  return lo;
}

// dense block b from the CSR rows of its rows; a coupling outside the block
// flags status[1] (the blocks must be diagonal blocks of J)
__global__ void block_to_dense_kernel(int n_blocks, const int64_t* __restrict__ rows,
                                      const int64_t* __restrict__ woff, const int64_t* __restrict__ row_ptr,
                                      const int32_t* __restrict__ col, const double* __restrict__ val, double* M,
                                      int32_t* status) {
  const int64_t total = rows[n_blocks];
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= total - rows[0]) return;
  const int64_t r = rows[0] + t;
  const int b = block_of(rows, n_blocks, r);
  const int64_t r0 = rows[b], nbk = rows[b + 1] - r0;
  double* W = M + woff[b];
  for (int64_t e = row_ptr[r] + lane; e < row_ptr[r + 1]; e += 64) {
    const int64_t c = col[e];
    if (c < r0 || c >= r0 + nbk) {
      atomicOr(&status[1], 1);
      continue;
    }
    W[(c - r0) * nbk + (r - r0)] = val[e];  // column-major during the elimination
  }
}

// maximum over the 16 lanes of each DPP row, read from lane 15 (row 0's result)
__device__ inline double row16_max(double v) {
  const double id = -__builtin_inf();
  v = fmax(v, dpp_move<0x111, 0xF>(v, id));
  v = fmax(v, dpp_move<0x112, 0xF>(v, id));
  v = fmax(v, dpp_move<0x114, 0xF>(v, id));
  v = fmax(v, dpp_move<0x118, 0xF>(v, id));
  const int2 a = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(a.x, 15);
  r.y = __builtin_amdgcn_readlane(a.y, 15);
  return __builtin_bit_cast(double, r);
}

// Pivot keys.  A candidate row i with |a| finite maps to the non-negative double whose bits are
// those of |a| with the low 14 bits replaced by KEY_MASK - i, so one floating-point maximum picks
// the largest |a| and, among values equal in all but those bits (relative 2^-38), the lowest
// row: partial pivoting up to that tolerance, deterministic.  An infinite |a| takes the
// largest finite magnitude (it wins, and the pivot test then rejects it); NaN and rows already
// used take -1.
constexpr int64_t KEY_MASK = (1 << 14) - 1;  // rows per block < 2^14
__device__ inline double pivot_key(double a, int64_t i) {
  const double av = fabs(a);
  if (!(av == av)) return -1.0;
  const int64_t bits = __builtin_bit_cast(int64_t, av < __builtin_inf() ? av : 1.7976931348623157e308);
  return __builtin_bit_cast(double, (bits & ~KEY_MASK) | (KEY_MASK - i));
}
__device__ inline int key_row(double key) { return (int)(KEY_MASK - (__builtin_bit_cast(int64_t, key) & KEY_MASK)); }

// Panel of columns [k0, k0 + NB) of every block (blockIdx.x), in place.  pcol[i] is
// 0 for a row not yet used as a pivot, else 1 + the column it was pivot of.  gi: the
// new pivot rows' old values in the outer block's other columns, laid out [t][c - c0o].
// Each column step has one barrier: every wave's best candidate row goes to LDS with its key
// before it, and after it every thread reads the winner's row and scales it itself.
template <int CTT, int R, int NB>
__global__ __launch_bounds__(CTT) void block_panel_kernel(const int64_t* __restrict__ rows,
                                                          const int64_t* __restrict__ woff, int64_t k0, int64_t c0o,
                                                          double* W_all, int32_t* __restrict__ q_all,
                                                          int32_t* __restrict__ pcol_all, double* __restrict__ gi_all,
                                                          int32_t nbo, int32_t bad_base, int32_t* status) {
  constexpr int NW = CTT / 64;
  static_assert(NW <= 16, "the cross-wave step reduces over one 16-lane row");
  static_assert(R <= 32, "the used-row mask has 32 bits");
  // double-buffered by column parity: a thread that runs ahead into column j + 1 writes the
  // other buffer, and it cannot reach column j + 2 before every thread has left column j
  __shared__ double w_key[2][NW];
  __shared__ double w_row[2][NW][NB];
  __shared__ int s_q[NB];
  const int bk = blockIdx.x;
  const int64_t r0 = rows[bk], n = rows[bk + 1] - r0;
  const int64_t left = n - k0;
  const int nb = left <= 0 ? 0 : (left < NB ? (int)left : NB);
  if (nb == 0) return;  // uniform for the workgroup
  double* W = W_all + woff[bk];
  int32_t* q_g = q_all + r0;
  int32_t* pcol_g = pcol_all + r0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // P[r][.]: panel row tid + r * CTT
  double P[R][NB];
  uint32_t used = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = tid + (int64_t)r * CTT;
    const bool ok = i < n;
#pragma unroll
    for (int c = 0; c < NB; ++c) P[r][c] = (ok && c < nb) ? W[(k0 + c) * n + i] : 0.0;
    if (!ok || pcol_g[i] != 0) used |= 1u << r;
  }
  // The column loop stays a loop over groups of U columns: the kernel runs as one workgroup per
  // block, so a fully unrolled body would be fetched from memory once per column.  Inside a
  // group the columns have compile-time indices; after it the register columns rotate by U, so
  // group g always finds its columns at P[.][0 .. U); after NB / U groups they are back in order.
  constexpr int U = NB < 4 ? NB : 4;
  static_assert(NB % U == 0, "panel width must be a multiple of the group size");
#pragma unroll 1
  for (int g = 0; g < NB; g += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = g + u;
      if (j < nb) {  // uniform
        const int buf = j & 1;
        double kr[R], key = -1.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          kr[r] = ((used >> r) & 1u) ? -1.0 : pivot_key(P[r][u], tid + r * CTT);
          key = fmax(key, kr[r]);
        }
        const double wk = wave_max(key);
        // this wave's best candidate row (one row of one lane: keys are distinct)
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (kr[r] == wk && wk >= 0.0) {
            w_key[buf][wave] = wk;
#pragma unroll
            for (int c = 0; c < NB; ++c) w_row[buf][wave][c] = P[r][c];
          }
        if (wk < 0.0 && lane == 0) w_key[buf][wave] = -1.0;
        __syncthreads();
        const int wl = lane & 15;
        const double pk = row16_max(wl < NW ? w_key[buf][wl] : -1.0);
        const int p = key_row(pk);
        const int otid = p % CTT, oslot = p / CTT, ow = otid >> 6;
        double pr[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) pr[c] = w_row[buf][ow][c];
        const double piv = pr[u];
        const bool bad = pk < 0.0 || !(piv != 0.0) || !isfinite(piv);
        // failure path only: -1, or the first failing block's number from bad_base on
        if (bad && tid == 0) atomicMin(&status[0], bad_base < 0 ? -1 : bad_base + bk);
        if (tid == 0) s_q[j] = bad ? 0 : p;
        // The update runs whether or not the pivot is usable (a branch around it would keep two
        // copies of the panel live): after a failure the status word reports the block and its
        // values are void.
        const double inv = bad ? 0.0 : 1.0 / piv;
#pragma unroll
        for (int c = 0; c < NB; ++c) pr[c] = (c == u ? 1.0 : pr[c]) * inv;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double f = P[r][u];
#pragma unroll
          for (int c = 0; c < NB; ++c) P[r][c] = (c == u) ? -f * pr[c] : fma(-f, pr[c], P[r][c]);
        }
        // the pivot row becomes the scaled row
        if (!bad && tid == otid) {
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (r == oslot) {  // uniform
#pragma unroll
              for (int c = 0; c < NB; ++c) P[r][c] = pr[c];
            }
          used |= 1u << oslot;
        }
      }
    }
    if (U < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = P[r][u];
#pragma unroll
        for (int c = 0; c + U < NB; ++c) P[r][c] = P[r][c + U];
#pragma unroll
        for (int u = 0; u < U; ++u) P[r][NB - U + u] = t[u];
      }
    }
  }
  __syncthreads();  // s_q complete
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = tid + (int64_t)r * CTT;
    if (i < n) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) W[(k0 + c) * n + i] = P[r][c];
    }
  }
  if (tid < nb) {
    q_g[k0 + tid] = s_q[tid];
    pcol_g[s_q[tid]] = (int32_t)(k0 + tid + 1);
  }
  // old values of the new pivot rows in the other columns of the outer block (this kernel
  // writes only the panel's columns); nb * gw <= NB * nbo fits an int
  const int64_t ge = (c0o + nbo < n ? c0o + nbo : n);
  const int gw = (int)(ge - c0o);
  double* gi = gi_all + (int64_t)bk * NB * nbo;
  for (int e = tid; e < nb * gw; e += CTT) {
    const int t = e / gw;
    const int64_t c = c0o + (e - t * gw);
    if (c < k0 || c >= k0 + nb) gi[t * nbo + (c - c0o)] = W[c * n + s_q[t]];
  }
}

// ---- Tournament pivoting for the panels of wide blocks ----
// Partial pivoting over all n rows makes every column step a reduction over the whole block, one
// workgroup wide, n steps in a row.  For wide blocks the pivots of a TP-column panel are chosen by
// a tournament instead: every leaf (512 rows, one workgroup) runs the panel's TP elimination
// steps on its own rows with partial pivoting and proposes the TP rows it chose; one workgroup
// then plays off the proposals the same way and chooses the panel's TP pivots.  Each proposal
// set spans its rows' panel (the rows a leaf leaves behind are reduced to zero in the panel's
// columns), so the final round finds a nonzero pivot at every step exactly when partial
// pivoting over all rows would.  The pivots differ from those of partial pivoting over all
// rows, the inverse does not (up to rounding).  The final round also records the scaled pivot
// row of every step; a separate launch then applies the TP steps to every row, with the same
// arithmetic as the single-workgroup panel.  Per 16 columns this is four launches (leaves, final
// round, apply, the rank-16 update of the outer block) instead of four single-workgroup panels
// and four rank-4 updates.
constexpr int TP = 16;          // panel width
constexpr int TLW = 8;          // wavefronts per leaf: 512 rows
constexpr int TL = TLW * 64;
constexpr int TRW = 5;          // wavefronts of the final round: up to 320 proposals

// The panel's TP elimination steps over one workgroup's rows (NW wavefronts, one row per thread:
// panel values P, block-local id, -1 for none).  Step t takes the unused row of largest |value|
// in the panel's column t (lowest id on ties; a zero value is taken like any other, then
// eliminates nothing), scales it by its pivot and eliminates column t from every other row.
// sel[t] receives the chosen id (-1: no row left).  The rounds before the final one only propose
// rows: they update just the columns still to come, and a chosen row is not replaced by its
// scaled copy (its values are not read again).  The final round (FINAL) carries the full steps
// and writes prs[t][.], the scaled pivot row of step t (in the rotated order below), and bad[t],
// whether step t failed (no row, or a zero or non-finite pivot).
// The step loop is not unrolled beyond groups of TU steps (a workgroup runs it once; an unrolled
// body would be fetched from memory instruction by instruction): the columns rotate by TU after
// each group, so in group g (steps g .. g + TU - 1) P[c] holds the panel's column (g + c) mod TP
// and step t's column sits at P[t - g].  One barrier per step; the LDS exchange is
// double-buffered by step parity, as in the single-workgroup panel.
constexpr int TU = 4;
template <int NW, bool FINAL>
__device__ __attribute__((always_inline)) inline void wg_panel_steps(double (&P)[TP], int id, int nb,
                                                                   double (*xkey)[16], int (*xid)[16],
                                                                   double (*xrow)[16][TP], int* sel, double* prs,
                                                                   int* bad) {
  static_assert(NW <= 16, "the cross-wave step reduces over one 16-lane row");
  static_assert(TP % TU == 0, "the rotation groups tile the panel");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0)
    for (int t = nb; t < TP; ++t) sel[t] = -1;
  bool used = id < 0;
#pragma unroll 1
  for (int g = 0; g < nb; g += TU) {
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int t = g + u;
      if (t >= nb) break;  // uniform
      const int buf = t & 1;
      const double key = used ? -1.0 : pivot_key(P[u], id);
      const double wk = wave_max(key);
      if (wk >= 0.0 && key == wk) {  // one lane per wavefront (keys are distinct)
        xkey[buf][wave] = wk;
        xid[buf][wave] = id;
#pragma unroll
        for (int c = 0; c < TP; ++c) xrow[buf][wave][c] = P[c];
      }
      if (!(wk >= 0.0) && lane == 0) xkey[buf][wave] = -1.0;
      __syncthreads();
      const int wl = lane & 15;
      const double kw = wl < NW ? xkey[buf][wl] : -1.0;
      const double pk = row16_max(kw);
      if (!(pk >= 0.0)) {  // uniform: no unused row left
        if (tid == 0) {
          sel[t] = -1;
          if (FINAL) {
            bad[t] = 1;
            for (int c = 0; c < TP; ++c) prs[t * TP + c] = 0.0;
          }
        }
        continue;
      }
      const uint64_t hit = __ballot(wl < NW && kw == pk) & 0xFFFFull;
      const int ow = __ffsll((unsigned long long)hit) - 1;
      double pr[TP];
#pragma unroll
      for (int c = 0; c < TP; ++c) pr[c] = xrow[buf][ow][c];
      const int p = xid[buf][ow];
      const double piv = pr[u];
      const bool zero = !(piv != 0.0) || !isfinite(piv);
      const double inv = zero ? 0.0 : 1.0 / piv;
      if (FINAL) {
#pragma unroll
        for (int c = 0; c < TP; ++c) pr[c] = (c == u ? 1.0 : pr[c]) * inv;
        const double f = P[u];
#pragma unroll
        for (int c = 0; c < TP; ++c) P[c] = (c == u) ? -f * pr[c] : fma(-f, pr[c], P[c]);
      } else {
        const double q = P[u] * inv;
#pragma unroll
        for (int c = u + 1; c < TP; ++c) P[c] = fma(-q, pr[c], P[c]);
      }
      if (id == p) used = true;
      if (tid == 0) {
        sel[t] = p;
        if (FINAL) {
          bad[t] = zero ? 1 : 0;
#pragma unroll
          for (int c = 0; c < TP; ++c) prs[t * TP + c] = pr[c];
        }
      }
    }
    // rotate by TU: the next group's columns to P[0 .. TU)
    double keep[TU];
#pragma unroll
    for (int c = 0; c < TU; ++c) keep[c] = P[c];
#pragma unroll
    for (int c = 0; c + TU < TP; ++c) P[c] = P[c + TU];
#pragma unroll
    for (int c = 0; c < TU; ++c) P[TP - TU + c] = keep[c];
  }
  __syncthreads();
}

// Pivots of the panel [k0, k0 + nb) of every block (blockIdx.y) by tournament, first round; W is
// only read.  Workgroup x of a block is the leaf of rows [TL x, TL x + TL); its TP winners go to
// cand[TP x ..].
__global__ __launch_bounds__(TL) void tourney_leaf_kernel(const int64_t* __restrict__ rows,
                                                          const int64_t* __restrict__ woff, int64_t k0,
                                                          const double* __restrict__ W_all,
                                                          const int32_t* __restrict__ pcol_all,
                                                          int32_t* __restrict__ cand_all, int32_t cand_stride) {
  __shared__ double xkey[2][16];
  __shared__ int xid[2][16];
  __shared__ double xrow[2][16][TP];
  __shared__ int s_win[TP];
  const int bk = blockIdx.y;
  const int64_t r0 = rows[bk], n = rows[bk + 1] - r0;
  const int64_t left = n - k0;
  const int nb = left <= 0 ? 0 : (left < TP ? (int)left : TP);
  if (nb == 0 || (int64_t)blockIdx.x * TL >= n) return;  // uniform for the workgroup
  const double* W = W_all + woff[bk];
  const int64_t i = (int64_t)blockIdx.x * TL + threadIdx.x;
  const int id = (i < n && pcol_all[r0 + (i < n ? i : 0)] == 0) ? (int)i : -1;
  double P[TP];
#pragma unroll
  for (int c = 0; c < TP; ++c) P[c] = (i < n && c < nb) ? W[(k0 + c) * n + (i < n ? i : 0)] : 0.0;
  wg_panel_steps<TLW, false>(P, id, nb, xkey, xid, xrow, s_win, nullptr, nullptr);
  if (threadIdx.x < TP) cand_all[(int64_t)bk * cand_stride + blockIdx.x * TP + threadIdx.x] = s_win[threadIdx.x];
}

// Final round (one workgroup per block, blockIdx.x): the panel's TP pivots from the leaves'
// proposals (at most 64 TRW).  It records q, pcol, the scaled pivot rows prs, the pivot rows pq
// (-1 for a failed step) and gi (the new pivot rows' old values in the outer block's other
// columns, laid out [t][c - c0o]).
__global__ __launch_bounds__(64 * TRW) void tourney_root_kernel(
    const int64_t* __restrict__ rows, const int64_t* __restrict__ woff, int64_t k0, int64_t c0o,
    const double* __restrict__ W_all, int32_t* __restrict__ q_all, int32_t* __restrict__ pcol_all,
    double* __restrict__ gi_all, int32_t nbo, const int32_t* __restrict__ cand_all, int32_t cand_stride,
    double* __restrict__ prs_all, int32_t* __restrict__ pq_all, int32_t bad_base, int32_t* status) {
  __shared__ double xkey[2][16];
  __shared__ int xid[2][16];
  __shared__ double xrow[2][16][TP];
  __shared__ int s_fin[TP];
  __shared__ int s_bad[TP];
  __shared__ double s_prs[TP * TP];
  const int bk = blockIdx.x;
  const int64_t r0 = rows[bk], n = rows[bk + 1] - r0;
  const int64_t left = n - k0;
  const int nb = left <= 0 ? 0 : (left < TP ? (int)left : TP);
  if (nb == 0) return;  // uniform
  const double* W = W_all + woff[bk];
  const int tid = threadIdx.x;
  const int C = (int)((n + TL - 1) / TL) * TP;
  const int id = tid < C ? cand_all[(int64_t)bk * cand_stride + tid] : -1;
  double P[TP];
#pragma unroll
  for (int c = 0; c < TP; ++c) P[c] = (id >= 0 && c < nb) ? W[(k0 + c) * n + (id >= 0 ? id : 0)] : 0.0;
  wg_panel_steps<TRW, true>(P, id, nb, xkey, xid, xrow, s_fin, s_prs, s_bad);
  int32_t* q_g = q_all + r0;
  int32_t* pcol_g = pcol_all + r0;
  if (tid < nb) {
    const bool bad = s_bad[tid] != 0 || s_fin[tid] < 0;
    // failure path only: -1, or the first failing block's number from bad_base on
    if (bad) atomicMin(&status[0], bad_base < 0 ? -1 : bad_base + bk);
    const int p = bad ? 0 : s_fin[tid];
    s_fin[tid] = p;
    q_g[k0 + tid] = p;
    pcol_g[p] = (int32_t)(k0 + tid + 1);
    pq_all[bk * TP + tid] = bad ? -1 : p;
  }
  for (int e = tid; e < TP * TP; e += 64 * TRW) prs_all[(int64_t)bk * TP * TP + e] = s_prs[e];
  __syncthreads();
  const int64_t ge = (c0o + nbo < n ? c0o + nbo : n);
  const int gw = (int)(ge - c0o);
  double* gi = gi_all + (int64_t)bk * TP * nbo;
  for (int e = tid; e < nb * gw; e += 64 * TRW) {
    const int t = e / gw;
    const int64_t c = c0o + (e - t * gw);
    if (c < k0 || c >= k0 + nb) gi[t * nbo + (c - c0o)] = W[c * n + s_fin[t]];
  }
}

// The panel's steps applied to every row of every block (blockIdx.y), one row per thread, with
// the (rotated) scaled pivot rows of the tournament: the pivot row of step t becomes prs[t];
// every other row loses f = its column-t value times prs[t] (and column t becomes -f times the
// scaled pivot).  The same
// operations in the same order as in the single-workgroup panel.
__global__ __launch_bounds__(256) void panel_apply_kernel(const int64_t* __restrict__ rows,
                                                          const int64_t* __restrict__ woff, int64_t k0,
                                                          double* W_all, const double* __restrict__ prs_all,
                                                          const int32_t* __restrict__ pq_all) {
  __shared__ double s_pr[TP][TP];
  __shared__ int s_pq[TP];
  const int bk = blockIdx.y;
  const int64_t r0 = rows[bk], n = rows[bk + 1] - r0;
  const int64_t left = n - k0;
  const int nb = left <= 0 ? 0 : (left < TP ? (int)left : TP);
  if (nb == 0 || (int64_t)blockIdx.x * 256 >= n) return;  // uniform
  const int tid = threadIdx.x;
  s_pr[tid >> 4][tid & 15] = prs_all[(int64_t)bk * TP * TP + tid];
  if (tid < TP) s_pq[tid] = pq_all[bk * TP + tid];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  if (i >= n) return;
  double* W = W_all + woff[bk];
  double P[TP];
#pragma unroll
  for (int c = 0; c < TP; ++c) P[c] = c < nb ? W[(k0 + c) * n + i] : 0.0;
  // rolled over groups of TU steps, as in the tournament: in group g, P[c] holds the panel's
  // column (g + c) mod TP, as do the scaled pivot rows
#pragma unroll 1
  for (int g = 0; g < nb; g += TU) {
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int t = g + u;
      if (t >= nb) break;  // uniform
      if (i == s_pq[t]) {
#pragma unroll
        for (int c = 0; c < TP; ++c) P[c] = s_pr[t][c];
      } else {
        const double f = P[u];
#pragma unroll
        for (int c = 0; c < TP; ++c) P[c] = (c == u) ? -f * s_pr[t][c] : fma(-f, s_pr[t][c], P[c]);
      }
    }
    double keep[TU];
#pragma unroll
    for (int c = 0; c < TU; ++c) keep[c] = P[c];
#pragma unroll
    for (int c = 0; c + TU < TP; ++c) P[c] = P[c + TU];
#pragma unroll
    for (int c = 0; c < TU; ++c) P[TP - TU + c] = keep[c];
  }
  const int rot = (nb + TU - 1) / TU * TU;  // the rotation after the last group
#pragma unroll
  for (int c = 0; c < TP; ++c) {
    const int a = (rot + c) & (TP - 1);  // the panel column at P[c]
    if (a < nb) W[(k0 + a) * n + i] = P[c];
  }
}

// old values of the outer block's pivot rows in every column: go[t][c] = W[q[c0o + t]][c]
__global__ void gather_pivot_rows_kernel(const int64_t* __restrict__ rows, const int64_t* __restrict__ woff,
                                         int64_t c0o, int32_t nbo, const double* __restrict__ W_all,
                                         const int32_t* __restrict__ q_all, double* __restrict__ go_all) {
  const int bk = blockIdx.z;
  const int64_t r0 = rows[bk], n = rows[bk + 1] - r0;
  const int64_t kk = n - c0o < nbo ? n - c0o : nbo;
  const int t = blockIdx.y;
  if (t >= kk) return;
  const double* W = W_all + woff[bk];
  const int64_t q = q_all[r0 + c0o + t];
  double* go = go_all + (int64_t)nbo * (r0 - rows[0]) + (int64_t)t * n;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    go[c] = W[c * n + q];
}

// In-place update of columns [cb, ce) \ [sk0, sk1) of every block (blockIdx.z), W column-major:
//   W[i, c] = (pcol[i] - 1 in [p0, p1) ? 0 : W[i, c]) + sum_{t < K} W[i, kc + t] G[t][c - gc0]
// with K clipped to the block.  G: inner mode (g_stride > 0) block b at b * g_stride with
// leading dimension ldg; outer mode (g_stride == 0) block b at K * (rows[b] - rows[0]) with
// leading dimension n_b.  Workgroup tile 64 rows x 64 columns, wavefront w the columns
// [16 w, 16 w + 16).  The FP64 matrix cores (16 x 16 x 4) compute the transposed tile
// D(c, i) = sum_t G(t, c) W(i, t): lane l holds A = G(l / 16, c_0 + l % 16) and
// B = W(i_0 + l % 16, l / 16), and accumulator element v holds D(4 v + l / 16, l % 16), so
// lanes 0..15 own 16 consecutive rows of one column (contiguous in memory).
// At least three workgroups per CU (three waves per SIMD) caps the registers at 168: the
// 128-step update then spills a few bytes per lane and still runs faster than with two.
template <int KMAX>
__global__ __launch_bounds__(256, 3) void gj_update_kernel(const int64_t* __restrict__ rows,
                                                        const int64_t* __restrict__ woff, double* W_all,
                                                        const int32_t* __restrict__ pcol_all, int64_t kc, int32_t K,
                                                        const double* __restrict__ G_all, int64_t g_stride,
                                                        int64_t ldg, int64_t gc0, int64_t cb, int64_t ce,
                                                        int64_t sk0, int64_t sk1, int64_t p0, int64_t p1,
                                                        int64_t tile_c0) {
  const int bk = blockIdx.z;
  const int64_t rb0 = rows[bk], n = rows[bk + 1] - rb0;
  const int64_t kk = (n - kc < K) ? n - kc : K;
  const int64_t ceb = ce < n ? ce : n;
  // consecutive workgroups take consecutive row tiles of one column tile (adjacent 512-byte
  // pieces of the same columns)
  const int64_t rt = (int64_t)blockIdx.x * 64;
  const int64_t ct = tile_c0 + (int64_t)blockIdx.y * 64;
  if (kk <= 0 || ct >= ceb || rt >= n) return;  // uniform for the workgroup
  if (ct >= sk0 && ct + 64 <= sk1) return;       // every column of the tile is skipped
  double* W = W_all + woff[bk];
  const int32_t* pcol = pcol_all + rb0;
  const double* G = g_stride > 0 ? G_all + (int64_t)bk * g_stride : G_all + (int64_t)K * (rb0 - rows[0]);
  const int64_t lg = g_stride > 0 ? ldg : n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  // Both operands of the tile are staged in LDS once per workgroup (each wave needs all 64 rows of
  // the W panel; loaded per wave from global memory they were read four times): sG[k][c] =
  // G(k, tile column c), sW[k][r] = W(tile row r, kc + k), zero outside the block and beyond kk.
  // The first chunk's operand loads and the tile's old values are all issued before the first
  // wait: out-of-range elements load a valid address and are replaced by zero.
  constexpr int LP = 64 + 1;  // padded row length (doubles)
  // The operands go through LDS in chunks of KC steps (more workgroups per CU than the whole
  // depth would allow).  Up to 64 steps all operand loads are issued up front (QL = Q); deeper
  // updates load each chunk while the previous one is multiplied (QL = QC registers per operand).
  constexpr int KC = KMAX < 32 ? KMAX : 32, QC = KC / 4;  // QC: elements per thread per operand
  constexpr bool PIPE = KMAX > 64;
  constexpr int QL = PIPE ? QC : KMAX / 4;
  __shared__ double sG[KC][LP];
  __shared__ double sW[KC][LP];
  double gv[QL], wv[QL];
  auto load = [&](int k0, int nq) {  // elements k0 * 64 + threadIdx.x + 256 q, q < nq
#pragma unroll
    for (int q = 0; q < nq; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int k = k0 + (e >> 6), c = e & 63;
      const bool okg = k < kk && ct + c < ceb;
      const bool okw = k < kk && rt + c < n;
      const double g = G[okg ? k * lg + (ct + c - gc0) : 0];
      const double w = W[okw ? (kc + k) * n + rt + c : 0];
      gv[q] = okg ? g : 0.0;
      wv[q] = okw ? w : 0.0;
    }
  };
  load(0, QL);
  // old values of this lane's 16 outputs (column c_v, row r_j), and the rows' pivot records
  double old[4][4];
  int32_t prow[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t r = rt + 16 * j + i16;
    prow[j] = pcol[r < n ? r : 0];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t c = ct + 16 * wave + 4 * v + kq;
      old[v][j] = W[(c < ceb && r < n) ? c * n + r : 0];
    }
  }
  f64x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < KMAX; k0 += KC) {
    if (k0 > 0) __syncthreads();  // the previous chunk's products have read the LDS
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int e = threadIdx.x + 256 * q;  // element (k0 + e / 64, e % 64)
      sG[e >> 6][e & 63] = gv[PIPE ? q : k0 / 4 + q];
      sW[e >> 6][e & 63] = wv[PIPE ? q : k0 / 4 + q];
    }
    __syncthreads();
    if (PIPE && k0 + KC < KMAX) load(k0 + KC, QC);
#pragma unroll
    for (int s4 = 0; s4 < KC / 4; ++s4) {
      const int k = 4 * s4 + kq;
      const double a = sG[k][16 * wave + i16];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sW[k][16 * j + i16], acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t c = ct + 16 * wave + 4 * v + kq;
    if (c < cb || c >= ceb || (c >= sk0 && c < sk1)) continue;
    double* wc = W + c * n;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = rt + 16 * j + i16;
      if (r >= n) continue;
      const int32_t u = prow[j] - 1;
      const bool zero = u >= p0 && u < p1;
      wc[r] = (zero ? 0.0 : old[v][j]) + acc[j][v];
    }
  }
}

// In-place transpose of every block (column-major -> row-major), 32 x 32 tiles through LDS:
// workgroup (I, J) with I <= J swaps tiles (I, J) and (J, I).
__global__ __launch_bounds__(256) void block_transpose_kernel(const int64_t* __restrict__ rows,
                                                              const int64_t* __restrict__ woff, double* W_all) {
  __shared__ double ta[32][33];
  __shared__ double tb[32][33];
  const int bk = blockIdx.z;
  const int64_t n = rows[bk + 1] - rows[bk];
  const int64_t I = blockIdx.y, J = blockIdx.x;
  if (I > J || I * 32 >= n || J * 32 >= n) return;  // uniform
  double* W = W_all + woff[bk];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = I * 32 + y, c = J * 32 + tx;
    ta[y][tx] = (r < n && c < n) ? W[r * n + c] : 0.0;
    const int64_t r2 = J * 32 + y, c2 = I * 32 + tx;
    tb[y][tx] = (r2 < n && c2 < n) ? W[r2 * n + c2] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = I * 32 + y, c = J * 32 + tx;
    if (r < n && c < n) W[r * n + c] = tb[tx][y];
    const int64_t r2 = J * 32 + y, c2 = I * 32 + tx;
    if (r2 < n && c2 < n) W[r2 * n + c2] = ta[tx][y];
  }
}

// y[r0 + k] = sum_j W_b[q_k][j] x[r0 + q_j] for every row of every block,
// one wavefront per row
__global__ __launch_bounds__(256) void block_apply_kernel(int n_blocks, const int64_t* __restrict__ rows,
                                                          const int64_t* __restrict__ woff,
                                                          const double* __restrict__ W_,
                                                          const int32_t* __restrict__ q_all,
                                                          const double* __restrict__ x, double* __restrict__ y) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= rows[n_blocks] - rows[0]) return;
  const int64_t r = rows[0] + t;
  const int b = block_of(rows, n_blocks, r);
  const int64_t r0 = rows[b], n = rows[b + 1] - r0, k = r - r0;
  const int32_t* q = q_all + r0;
  const double* w = W_ + woff[b] + (int64_t)q[k] * n;
  // four independent (q, x[q], w) load chains in flight per lane
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t j = lane;
  for (; j + 192 < n; j += 256) {
    const int32_t q0 = q[j], q1 = q[j + 64], q2 = q[j + 128], q3 = q[j + 192];
    const double w0 = w[j], w1 = w[j + 64], w2 = w[j + 128], w3 = w[j + 192];
    s0 = fma(w0, x[r0 + q0], s0);
    s1 = fma(w1, x[r0 + q1], s1);
    s2 = fma(w2, x[r0 + q2], s2);
    s3 = fma(w3, x[r0 + q3], s3);
  }
  for (; j < n; j += 64) s0 = fma(w[j], x[r0 + q[j]], s0);
  double s = (s0 + s1) + (s2 + s3);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[r] = s;
}

// out[k][q_j] = W_b[q_k][j]: block b's inverse in natural order
__global__ void block_export_kernel(int64_t n, const double* __restrict__ W, const int32_t* __restrict__ q,
                                    double* out) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / n, j = e - k * n;
    out[k * n + q[j]] = W[(int64_t)q[k] * n + j];
  }
}

// TN: panels of TP columns with tournament pivoting (CTT and R unused)
template <int CTT, int R, int NB, int NBO, bool TN = false>
hipError_t run_blocked(hipStream_t s, const vk_level& L, int32_t* status, int32_t bad_base = -1,
                       const vk_lookahead* la = nullptr) {
  static_assert(NBO % NB == 0 && NB <= VK_GJ_NBI_MAX && NBO % 64 == 0 && NBO <= VK_GJ_NBO,
                "inner panels must tile the outer block, whose columns come in whole 64-column tiles");
  static_assert(!TN || NB == TP, "tournament panels are TP columns wide");
  const int nbk = (int)L.cb_rows.size() - 1;
  const int64_t n = L.cb_max;
  const unsigned row_tiles = (unsigned)((n + 63) / 64);
  hipError_t e = hipSuccess;
  bool bulk_pending = false;  // a rank-NBO update of the other columns is running on la->aux
  for (int64_t c0o = 0; c0o < n; c0o += NBO) {
    for (int64_t k0 = c0o; k0 < c0o + NBO && k0 < n; k0 += NB) {
      if constexpr (TN) {
        tourney_leaf_kernel<<<dim3((unsigned)((n + TL - 1) / TL), nbk), TL, 0, s>>>(
            L.d_cb_rows, L.d_cb_woff, k0, L.cb_a, L.cb_used, L.cb_cand, (int32_t)L.cb_cand_stride);
        tourney_root_kernel<<<nbk, 64 * TRW, 0, s>>>(L.d_cb_rows, L.d_cb_woff, k0, c0o, L.cb_a, L.cb_q, L.cb_used,
                                               L.cb_gi, NBO, L.cb_cand, (int32_t)L.cb_cand_stride, L.cb_prs,
                                               L.cb_pq, bad_base, status);
        panel_apply_kernel<<<dim3((unsigned)((n + 255) / 256), nbk), 256, 0, s>>>(L.d_cb_rows, L.d_cb_woff, k0,
                                                                                 L.cb_a, L.cb_prs, L.cb_pq);
      } else {
        block_panel_kernel<CTT, R, NB><<<nbk, CTT, 0, s>>>(L.d_cb_rows, L.d_cb_woff, k0, c0o, L.cb_a, L.cb_q,
                                                           L.cb_used, L.cb_gi, NBO, bad_base, status);
      }
      // the same steps on the outer block's other columns, before and after the panel
      if (n > NB)
        gj_update_kernel<NB><<<dim3(row_tiles, NBO / 64, nbk), 256, 0, s>>>(
            L.d_cb_rows, L.d_cb_woff, L.cb_a, L.cb_used, k0, NB, L.cb_gi, (int64_t)NB * NBO, NBO, c0o, c0o,
            c0o + NBO, k0, k0 + NB, k0, k0 + NB, c0o);
    }
    // the previous outer block's update of the other columns must be complete before its pivot
    // rows' values are gathered here (and before the gather buffer is overwritten)
    if (bulk_pending && (e = hipStreamWaitEvent(s, la->bulk_done, 0)) != hipSuccess) return e;
    bulk_pending = false;
    gather_pivot_rows_kernel<<<dim3((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), NBO, nbk), 256, 0, s>>>(
        L.d_cb_rows, L.d_cb_woff, c0o, NBO, L.cb_a, L.cb_q, L.cb_go);
    const int64_t c1 = c0o + NBO, c2 = c1 + NBO < n ? c1 + NBO : n;
    if (la && c1 < n) {
      // Look-ahead: the next outer block's columns first, on the chain's stream (its panels need
      // only them); the rest on the second stream, overlapping those panels.  The two column sets
      // are disjoint from each other and from the next panels' columns.
      gj_update_kernel<NBO><<<dim3(row_tiles, (unsigned)((c2 - c1 + 63) / 64), nbk), 256, 0, s>>>(
          L.d_cb_rows, L.d_cb_woff, L.cb_a, L.cb_used, c0o, NBO, L.cb_go, 0, 0, 0, c1, c2, c0o, c0o + NBO, c0o,
          c0o + NBO, c1);
      if ((e = hipEventRecord(la->gathered, s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(la->aux, la->gathered, 0)) != hipSuccess) return e;
      gj_update_kernel<NBO><<<dim3(row_tiles, row_tiles, nbk), 256, 0, la->aux>>>(
          L.d_cb_rows, L.d_cb_woff, L.cb_a, L.cb_used, c0o, NBO, L.cb_go, 0, 0, 0, 0, n, c0o, c2, c0o, c0o + NBO,
          0);
      if ((e = hipEventRecord(la->bulk_done, la->aux)) != hipSuccess) return e;
      bulk_pending = true;
    } else {
      gj_update_kernel<NBO><<<dim3(row_tiles, row_tiles, nbk), 256, 0, s>>>(L.d_cb_rows, L.d_cb_woff, L.cb_a,
                                                                       L.cb_used, c0o, NBO, L.cb_go, 0, 0, 0, 0, n,
                                                                       c0o, c0o + NBO, c0o, c0o + NBO, 0);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (bulk_pending && (e = hipStreamWaitEvent(s, la->bulk_done, 0)) != hipSuccess) return e;
  const unsigned tiles = (unsigned)((n + 31) / 32);
  block_transpose_kernel<<<dim3(tiles, tiles, nbk), 256, 0, s>>>(L.d_cb_rows, L.d_cb_woff, L.cb_a);
  return hipGetLastError();
}

}  // namespace

int64_t vk_coarse_max_n() { return 9216; }

hipError_t launch_block_invert(hipStream_t s, const vk_level& L, int32_t* status, double** result,
                               const vk_lookahead* la, int64_t min_tourney) {
  const int nbk = (int)L.cb_rows.size() - 1;
  *result = L.cb_a;
  if (nbk <= 0) return hipSuccess;
  const int64_t rows_total = L.cb_rows[nbk] - L.cb_rows[0];
  hipError_t e = launch_fill(s, L.cb_sq, 0.0, L.cb_a);
  if (e != hipSuccess) return e;
  block_to_dense_kernel<<<(unsigned)((rows_total * 64 + 255) / 256), 256, 0, s>>>(
      nbk, L.d_cb_rows, L.d_cb_woff, L.J.row_ptr, L.J.col, L.J.val, L.cb_a, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_i32(s, L.J.n_rows, 0, L.cb_used)) != hipSuccess) return e;
  // panel rows per thread R, panel width NB: R * NB <= 64 doubles in registers (<= 36 at
  // 1024 threads, whose waves may hold 128 registers each)
  // outer blocks of 128 columns halve the passes of the rank-NBO updates over the blocks (HBM
  // traffic) at twice the inner updates' width: worth it for one or a few blocks, whose updates
  // are few workgroups wide; many blocks per level keep 64
  const int64_t m = L.cb_max;
  const bool wide = nbk <= 8;
  if (m > min_tourney) {
    // proposals: TP per TL rows, at most one per thread of the final round
    if ((m + TL - 1) / TL * TP > 64 * TRW || L.cb_cand_stride < (m + TL - 1) / TL * TP) return hipErrorInvalidValue;
    return wide ? run_blocked<256, 1, TP, VK_TOURNEY_NBO, true>(s, L, status, -1, la)
                : run_blocked<256, 1, TP, 64, true>(s, L, status, -1, la);
  }
  if (m <= 1024)
    e = wide ? run_blocked<512, 2, 16, 128>(s, L, status, -1, la) : run_blocked<512, 2, 16, 64>(s, L, status, -1, la);
  else if (m <= 2048)
    e = wide ? run_blocked<256, 8, 8, 128>(s, L, status, -1, la) : run_blocked<256, 8, 8, 64>(s, L, status, -1, la);
  else if (m <= 4096)
    e = wide ? run_blocked<512, 8, 8, 128>(s, L, status, -1, la) : run_blocked<512, 8, 8, 64>(s, L, status, -1, la);
  else if (m <= 8192)
    e = wide ? run_blocked<1024, 8, 4, 128>(s, L, status, -1, la) : run_blocked<1024, 8, 4, 64>(s, L, status, -1, la);
  else
    e = wide ? run_blocked<1024, 9, 4, 128>(s, L, status, -1, la) : run_blocked<1024, 9, 4, 64>(s, L, status, -1, la);
  return e;
}

hipError_t launch_block_invert_dense_any(hipStream_t s, const vk_level& L, int32_t* status) {
  const int nbk = (int)L.cb_rows.size() - 1;
  if (nbk <= 0) return hipSuccess;
  const hipError_t e = launch_fill_i32(s, L.cb_rows[nbk] - L.cb_rows[0], 0, L.cb_used);
  if (e != hipSuccess) return e;
  const int64_t m = L.cb_max;
  if (m <= 1024) return run_blocked<512, 2, 16, 128>(s, L, status);
  if (m <= 2048) return run_blocked<256, 8, 8, 128>(s, L, status);
  if (m <= 4096) return run_blocked<512, 8, 8, 128>(s, L, status);
  if (m <= 8192) return run_blocked<1024, 8, 4, 128>(s, L, status);
  return run_blocked<1024, 9, 4, 128>(s, L, status);
}

hipError_t launch_blocks_invert_dense(hipStream_t s, const vk_level& L, int32_t* status, int32_t bad_base) {
  const int nbk = (int)L.cb_rows.size() - 1;
  if (nbk <= 0) return hipSuccess;
  if (L.cb_max > 512) return hipErrorInvalidValue;
  const hipError_t e = launch_fill_i32(s, L.cb_rows[nbk] - L.cb_rows[0], 0, L.cb_used);
  if (e != hipSuccess) return e;
  // blocks of at most 512 rows: 256 threads x 2 rows hold a 16-column panel; 64-column outer
  // blocks (the buffers of the blocked patch inversion are sized for them)
  return run_blocked<256, 2, 16, 64>(s, L, status, bad_base);
}

hipError_t launch_block_apply(hipStream_t s, const vk_level& L, const double* x, double* y) {
  const int nbk = (int)L.cb_rows.size() - 1;
  if (nbk <= 0) return hipSuccess;
  const int64_t rows_total = L.cb_rows[nbk] - L.cb_rows[0];
  block_apply_kernel<<<(unsigned)((rows_total * 64 + 255) / 256), 256, 0, s>>>(nbk, L.d_cb_rows, L.d_cb_woff,
                                                                              L.cb_W, L.cb_q, x, y);
  return hipGetLastError();
}

hipError_t launch_block_export(hipStream_t s, const vk_level& L, int32_t block, double* out) {
  const int64_t n = L.cb_rows[block + 1] - L.cb_rows[block];
  int64_t woff = 0;
  for (int b = 0; b < block; ++b) {
    const int64_t nb = L.cb_rows[b + 1] - L.cb_rows[b];
    woff += nb * nb;
  }
  int64_t g = (n * n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  block_export_kernel<<<(unsigned)g, 256, 0, s>>>(n, L.cb_W + woff, L.cb_q + L.cb_rows[block], out);
  return hipGetLastError();
}
