// Learned Newton initial guess: BF16 multilayer perceptron (forward, mean-squared-error
// gradient, Adam) on the matrix cores, and the patch gather / average kernels around it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "vk_mlp.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;  // NaN stays NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

enum { EPI_TANH = 0, EPI_LINEAR = 1, EPI_DTANH = 2, EPI_STORE = 3 };

// C(m, n) = sum_k A(m, k) B(k, n) over one 16 x 16 tile per wavefront, BF16 operands and
// FP32 accumulation on v_mfma_f32_16x16x16_bf16.  Operand element addresses:
//   A(m, k) = A[ra(m) * a_rs + k * a_ks],  ra(m) = arow ? arow[m] : m
//   B(k, n) = B[rb(k) * b_ks + n * b_ns],  rb(k) = brow ? brow[k] : k
// Lane l holds A rows l % 16 and B columns l % 16, k = 4 (l / 16) + i of every 16-deep step;
// the accumulator's element i of lane l is C(4 (l / 16) + i, l % 16).
template <int EPI>
__global__ __launch_bounds__(64) void gemm_kernel(int32_t M, int32_t N, int32_t K, const uint16_t* __restrict__ A,
                                                  const int32_t* __restrict__ arow, int64_t a_rs, int64_t a_ks,
                                                  const uint16_t* __restrict__ B, const int32_t* __restrict__ brow,
                                                  int64_t b_ks, int64_t b_ns, const float* __restrict__ bias,
                                                  const uint16_t* __restrict__ act, float* __restrict__ outf,
                                                  uint16_t* __restrict__ outb, int64_t ldo) {
  const int lane = threadIdx.x;
  const int r = lane & 15, q = lane >> 4;
  const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 16;
  const int am = m0 + r, bn = n0 + r;
  const bool am_ok = am < M, bn_ok = bn < N;
  const int64_t a_base = am_ok ? (int64_t)(arow ? arow[am] : am) * a_rs : 0;
  const int64_t b_col = bn_ok ? (int64_t)bn * b_ns : 0;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + 4 * q + i;
      const bool k_ok = k < K;
      a[i] = (am_ok && k_ok) ? (short)A[a_base + (int64_t)k * a_ks] : (short)0;
      const int64_t rk = k_ok ? (int64_t)(brow ? brow[k] : k) : 0;
      b[i] = (bn_ok && k_ok) ? (short)B[rk * b_ks + b_col] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * q + i, n = n0 + r;
    if (m >= M || n >= N) continue;
    const int64_t o = (int64_t)m * ldo + n;
    const float v = acc[i];
    if (EPI == EPI_TANH) {
      outb[o] = f2bf(tanhf(v + bias[n]));
    } else if (EPI == EPI_LINEAR) {
      outf[o] = v + bias[n];
    } else if (EPI == EPI_DTANH) {
      const float a_v = bf2f(act[o]);
      outb[o] = f2bf(v * (1.0f - a_v * a_v));
    } else {
      outf[o] = v;
    }
  }
}

// dY = 2 (y - t) / (batch n_out) as BF16 and per-block partial sums of (y - t)^2
__global__ __launch_bounds__(256) void mse_kernel(int32_t batch, int32_t n_out, const float* __restrict__ y,
                                                  const float* __restrict__ t, const int32_t* __restrict__ rows,
                                                  float scale, uint16_t* __restrict__ dz, float* __restrict__ part) {
  __shared__ float red[256];
  const int64_t total = (int64_t)batch * n_out;
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / n_out, j = i - m * n_out;
    const int64_t tr = rows ? (int64_t)rows[m] : m;
    const float d = y[i] - t[tr * n_out + j];
    s += d * d;
    dz[i] = f2bf(scale * d);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(int32_t n_part, const float* __restrict__ part, float inv_count,
                                  float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n_part; ++i) s += part[i];
    loss[0] = s * inv_count;
  }
}

// db[n] = sum_m dz[m, n] (one workgroup per column, fixed reduction order)
__global__ __launch_bounds__(256) void colsum_kernel(int32_t batch, int32_t N, const uint16_t* __restrict__ dz,
                                                     float* __restrict__ out) {
  __shared__ float red[256];
  const int n = blockIdx.x;
  float s = 0.0f;
  for (int m = threadIdx.x; m < batch; m += blockDim.x) s += bf2f(dz[(int64_t)m * N + n]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

__global__ void adam_kernel(int64_t P, float* __restrict__ theta, float* __restrict__ m1, float* __restrict__ m2,
                            const float* __restrict__ g, uint16_t* __restrict__ wb, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float m = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = m;
    m2[i] = v;
    const float th = theta[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    theta[i] = th;
    wb[i] = f2bf(th);
  }
}

__global__ void set_params_kernel(int64_t P, const float* __restrict__ src, float* __restrict__ theta,
                                  float* __restrict__ m1, float* __restrict__ m2, uint16_t* __restrict__ wb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = src[i];
    theta[i] = v;
    m1[i] = 0.0f;
    m2[i] = 0.0f;
    wb[i] = f2bf(v);
  }
}

__global__ void copy_f32_kernel(int64_t n, const float* __restrict__ src, float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void features_kernel(int32_t n_cells, int32_t n_K, const int32_t* __restrict__ dofs,
                                const double* __restrict__ X1, const double* __restrict__ X2,
                                const double* __restrict__ B, const float* __restrict__ mean,
                                const float* __restrict__ inv_std, uint16_t* __restrict__ out) {
  const int64_t w = 2 * (int64_t)n_K;
  const int64_t total = (int64_t)n_cells * w;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / w;
    const int j = (int)(i - c * w);
    const int jl = j < n_K ? j : j - n_K;
    const int32_t d = dofs[c * n_K + jl];
    const double x = X2[d] - (j < n_K ? X1 : B)[d];
    out[i] = f2bf((float)(x - (double)mean[j]) * inv_std[j]);
  }
}

__global__ void targets_kernel(int32_t n_cells, int32_t n_K, const int32_t* __restrict__ dofs,
                               const double* __restrict__ X, const double* __restrict__ base,
                               const float* __restrict__ mean, const float* __restrict__ inv_std,
                               float* __restrict__ out) {
  const int64_t total = (int64_t)n_cells * n_K;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % n_K);
    const int32_t d = dofs[i];
    out[i] = (float)((X[d] - base[d] - (double)mean[j]) * (double)inv_std[j]);
  }
}

__global__ void average_kernel(int64_t n, const int64_t* __restrict__ ptr, const int64_t* __restrict__ list,
                               int32_t n_K, const float* __restrict__ pred, const float* __restrict__ mean,
                               const float* __restrict__ sd, const double* __restrict__ base,
                               double* __restrict__ out) {
  for (int64_t mu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; mu < n; mu += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e0 = ptr[mu], e1 = ptr[mu + 1];
    double s = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
      const int64_t idx = list[e];
      const int j = (int)(idx % n_K);
      s += (double)pred[idx] * (double)sd[j] + (double)mean[j];
    }
    out[mu] = base[mu] + (e1 > e0 ? s / (double)(e1 - e0) : 0.0);
  }
}

struct ext_coef {
  double e[64];
};

__global__ void extrapolate_kernel(int64_t ns, int32_t nt, ext_coef E, const double* __restrict__ X,
                                   double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    double x[8];
    for (int b = 0; b < nt; ++b) x[b] = X[b * ns + i];
    for (int a = 0; a < nt; ++a) {
      double s = 0.0;
      for (int b = 0; b < nt; ++b) s += E.e[a * 8 + b] * x[b];
      out[a * ns + i] = s;
    }
  }
}

inline unsigned grid_for(int64_t work, int per, unsigned cap = 4096) {
  int64_t g = (work + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

char g_mlp_create_err[256] = "";
constexpr int kLossParts = 64;

}  // namespace

struct vk_mlp {
  hipStream_t stream = nullptr;
  std::string err;
  int32_t n_in = 0, width = 0, n_hidden = 0, n_out = 0, max_batch = 0;
  std::vector<int32_t> lin, lout;     // per layer fan-in / fan-out
  std::vector<int64_t> woff, boff;    // offsets of W_l and b_l in the packed vector
  int64_t P = 0;
  // workspace
  bool ready = false;
  float* theta = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* grad = nullptr;
  uint16_t* wb = nullptr;
  std::vector<uint16_t*> act;  // hidden activations, max_batch x width each
  float* y = nullptr;          // max_batch x n_out
  uint16_t* dz_a = nullptr;    // back-propagated pre-activation gradients (ping-pong)
  uint16_t* dz_b = nullptr;
  float* part = nullptr;
  float* loss = nullptr;
  int64_t step = 0;
  bool have_grad = false;
};

namespace {

vk_status mfail(vk_mlp* c, vk_status st, const std::string& msg) {
  c->err = msg;
  return st;
}

vk_status mfail_hip(vk_mlp* c, hipError_t e, const char* what) {
  (void)hipGetLastError();
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return VK_ERR_HIP;
}

#define MLP_TRY(expr)                                     \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return mfail_hip(c, _e, #expr); \
  } while (0)

#define MLP_LAUNCHED(what)                               \
  do {                                                   \
    hipError_t _e = hipGetLastError();                   \
    if (_e != hipSuccess) return mfail_hip(c, _e, what); \
  } while (0)

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t plan(vk_mlp* c, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t P = (size_t)c->P, mb = (size_t)c->max_batch;
  c->theta = reinterpret_cast<float*>(take(P * 4));
  c->m1 = reinterpret_cast<float*>(take(P * 4));
  c->m2 = reinterpret_cast<float*>(take(P * 4));
  c->grad = reinterpret_cast<float*>(take(P * 4));
  c->wb = reinterpret_cast<uint16_t*>(take(P * 2));
  c->act.assign(c->n_hidden, nullptr);
  for (int l = 0; l < c->n_hidden; ++l) c->act[l] = reinterpret_cast<uint16_t*>(take(mb * c->width * 2));
  c->y = reinterpret_cast<float*>(take(mb * c->n_out * 4));
  const size_t wmax = (size_t)(c->width > c->n_out ? c->width : c->n_out);
  c->dz_a = reinterpret_cast<uint16_t*>(take(mb * wmax * 2));
  c->dz_b = reinterpret_cast<uint16_t*>(take(mb * wmax * 2));
  c->part = reinterpret_cast<float*>(take(kLossParts * 4));
  c->loss = reinterpret_cast<float*>(take(4));
  return off;
}

vk_status check_ready(vk_mlp* c) {
  if (!c) return VK_ERR_ARG;
  if (!c->ready) return mfail(c, VK_ERR_WORKSPACE, "workspace not set");
  return VK_OK;
}

template <int EPI>
hipError_t gemm(hipStream_t s, int32_t M, int32_t N, int32_t K, const uint16_t* A, const int32_t* arow, int64_t a_rs,
                int64_t a_ks, const uint16_t* B, const int32_t* brow, int64_t b_ks, int64_t b_ns, const float* bias,
                const uint16_t* act, float* outf, uint16_t* outb, int64_t ldo) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16));
  gemm_kernel<EPI><<<grid, 64, 0, s>>>(M, N, K, A, arow, a_rs, a_ks, B, brow, b_ks, b_ns, bias, act, outf, outb,
                                       ldo);
  return hipGetLastError();
}

// forward over `batch` samples; hidden activations stay in the workspace for the gradient
vk_status run_forward(vk_mlp* c, int32_t batch, const uint16_t* x, const int32_t* rows) {
  hipStream_t s = c->stream;
  const int L = c->n_hidden + 1;
  const uint16_t* a_in = x;
  const int32_t* a_rows = rows;
  int64_t a_ld = c->n_in;
  for (int l = 0; l < L; ++l) {
    const uint16_t* W = c->wb + c->woff[l];
    const float* bias = c->theta + c->boff[l];
    // Z = A W^T: B(k, n) = W[n * in + k]
    if (l + 1 < L) {
      MLP_TRY(gemm<EPI_TANH>(s, batch, c->lout[l], c->lin[l], a_in, a_rows, a_ld, 1, W, nullptr, 1, c->lin[l], bias,
                             nullptr, nullptr, c->act[l], c->width));
      a_in = c->act[l];
      a_rows = nullptr;
      a_ld = c->width;
    } else {
      MLP_TRY(gemm<EPI_LINEAR>(s, batch, c->lout[l], c->lin[l], a_in, a_rows, a_ld, 1, W, nullptr, 1, c->lin[l],
                               bias, nullptr, c->y, nullptr, c->n_out));
    }
  }
  return VK_OK;
}

}  // namespace

extern "C" {

vk_status vk_mlp_create(vk_mlp** out, int32_t n_in, int32_t width, int32_t n_hidden, int32_t n_out,
                        int32_t max_batch, void* hip_stream) {
  if (!out) {
    snprintf(g_mlp_create_err, sizeof(g_mlp_create_err), "null output pointer");
    return VK_ERR_ARG;
  }
  *out = nullptr;
  if (n_hidden < 1 || n_hidden > 8 || n_in < 1 || n_in > 1024 || width < 1 || width > 1024 || n_out < 1 ||
      n_out > 1024 || max_batch < 1 || max_batch > (1 << 20)) {
    snprintf(g_mlp_create_err, sizeof(g_mlp_create_err), "layer sizes or max_batch out of range");
    return VK_ERR_ARG;
  }
  vk_mlp* c = new (std::nothrow) vk_mlp;
  if (!c) {
    snprintf(g_mlp_create_err, sizeof(g_mlp_create_err), "host allocation failed");
    return VK_ERR_ARG;
  }
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->n_in = n_in;
  c->width = width;
  c->n_hidden = n_hidden;
  c->n_out = n_out;
  c->max_batch = max_batch;
  int64_t off = 0;
  for (int l = 0; l <= n_hidden; ++l) {
    const int32_t fi = l == 0 ? n_in : width, fo = l == n_hidden ? n_out : width;
    c->lin.push_back(fi);
    c->lout.push_back(fo);
    c->woff.push_back(off);
    off += (int64_t)fi * fo;
    c->boff.push_back(off);
    off += fo;
  }
  c->P = off;
  *out = c;
  return VK_OK;
}

void vk_mlp_destroy(vk_mlp* mlp) {
  if (!mlp) return;
  if (mlp->stream) (void)hipStreamSynchronize(mlp->stream);
  else (void)hipDeviceSynchronize();
  delete mlp;
}

const char* vk_mlp_last_error(const vk_mlp* mlp) { return mlp ? mlp->err.c_str() : g_mlp_create_err; }

int64_t vk_mlp_param_count(const vk_mlp* mlp) { return mlp ? mlp->P : 0; }

size_t vk_mlp_workspace_bytes(const vk_mlp* mlp) {
  if (!mlp) return 0;
  vk_mlp tmp = *mlp;
  return plan(&tmp, nullptr);
}

vk_status vk_mlp_set_workspace(vk_mlp* c, void* dev, size_t bytes) {
  if (!c) return VK_ERR_ARG;
  c->ready = false;
  if (!dev) return mfail(c, VK_ERR_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev) % 256 != 0) return mfail(c, VK_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < vk_mlp_workspace_bytes(c)) return mfail(c, VK_ERR_WORKSPACE, "workspace smaller than required");
  plan(c, static_cast<char*>(dev));
  c->ready = true;
  c->step = 0;
  c->have_grad = false;
  return VK_OK;
}

vk_status vk_mlp_set_params(vk_mlp* c, const float* params) {
  vk_status st = check_ready(c);
  if (st != VK_OK) return st;
  if (!params) return mfail(c, VK_ERR_ARG, "null parameter vector");
  set_params_kernel<<<grid_for(c->P, 256), 256, 0, c->stream>>>(c->P, params, c->theta, c->m1, c->m2, c->wb);
  MLP_LAUNCHED("set_params_kernel");
  c->step = 0;
  c->have_grad = false;
  return VK_OK;
}

vk_status vk_mlp_get_params(vk_mlp* c, float* params) {
  vk_status st = check_ready(c);
  if (st != VK_OK) return st;
  if (!params) return mfail(c, VK_ERR_ARG, "null output");
  copy_f32_kernel<<<grid_for(c->P, 256), 256, 0, c->stream>>>(c->P, c->theta, params);
  MLP_LAUNCHED("copy_f32_kernel");
  return VK_OK;
}

vk_status vk_mlp_forward(vk_mlp* c, int32_t batch, const uint16_t* x, const int32_t* rows, float* y) {
  vk_status st = check_ready(c);
  if (st != VK_OK) return st;
  if (batch < 0 || batch > c->max_batch) return mfail(c, VK_ERR_ARG, "batch exceeds max_batch");
  if (batch == 0) return VK_OK;
  if (!x || !y) return mfail(c, VK_ERR_ARG, "null input or output");
  st = run_forward(c, batch, x, rows);
  if (st != VK_OK) return st;
  const int64_t n = (int64_t)batch * c->n_out;
  copy_f32_kernel<<<grid_for(n, 256), 256, 0, c->stream>>>(n, c->y, y);
  MLP_LAUNCHED("copy_f32_kernel");
  return VK_OK;
}

vk_status vk_mlp_gradient(vk_mlp* c, int32_t batch, const uint16_t* x, const int32_t* rows, const float* target,
                          float* loss, float* grad) {
  vk_status st = check_ready(c);
  if (st != VK_OK) return st;
  if (batch < 1 || batch > c->max_batch) return mfail(c, VK_ERR_ARG, "batch must be in [1, max_batch]");
  if (!x || !target) return mfail(c, VK_ERR_ARG, "null input or target");
  hipStream_t s = c->stream;
  st = run_forward(c, batch, x, rows);
  if (st != VK_OK) return st;
  const int L = c->n_hidden + 1;
  const float count = (float)batch * (float)c->n_out;
  mse_kernel<<<kLossParts, 256, 0, s>>>(batch, c->n_out, c->y, target, rows, 2.0f / count, c->dz_a, c->part);
  MLP_LAUNCHED("mse_kernel");
  loss_final_kernel<<<1, 64, 0, s>>>(kLossParts, c->part, 1.0f / count, c->loss);
  MLP_LAUNCHED("loss_final_kernel");
  uint16_t* dz = c->dz_a;
  uint16_t* dz_next = c->dz_b;
  for (int l = L - 1; l >= 0; --l) {
    const int32_t fi = c->lin[l], fo = c->lout[l];
    // input of layer l: the features (rows indexed) or the previous activation
    const uint16_t* a_prev = l == 0 ? x : c->act[l - 1];
    const int32_t* a_rows = l == 0 ? rows : nullptr;
    // dW(j, i) = sum_m dz[m, j] a_prev[m, i]
    MLP_TRY(gemm<EPI_STORE>(s, fo, fi, batch, dz, nullptr, 1, fo, a_prev, a_rows, fi, 1, nullptr, nullptr,
                            c->grad + c->woff[l], nullptr, fi));
    colsum_kernel<<<fo, 256, 0, s>>>(batch, fo, dz, c->grad + c->boff[l]);
    MLP_LAUNCHED("colsum_kernel");
    if (l > 0) {
      // dz_prev(m, i) = (sum_j dz[m, j] W[j, i]) (1 - a_prev(m, i)^2)
      MLP_TRY(gemm<EPI_DTANH>(s, batch, fi, fo, dz, nullptr, fo, 1, c->wb + c->woff[l], nullptr, fi, 1, nullptr,
                              a_prev, nullptr, dz_next, fi));
      uint16_t* t = dz;
      dz = dz_next;
      dz_next = t;
    }
  }
  if (loss) {
    copy_f32_kernel<<<1, 64, 0, s>>>(1, c->loss, loss);
    MLP_LAUNCHED("copy_f32_kernel");
  }
  if (grad) {
    copy_f32_kernel<<<grid_for(c->P, 256), 256, 0, s>>>(c->P, c->grad, grad);
    MLP_LAUNCHED("copy_f32_kernel");
  }
  c->have_grad = true;
  return VK_OK;
}

vk_status vk_mlp_adam(vk_mlp* c, float lr, float beta1, float beta2, float eps) {
  vk_status st = check_ready(c);
  if (st != VK_OK) return st;
  if (!c->have_grad) return mfail(c, VK_ERR_STATE, "no gradient since the parameters were set");
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return mfail(c, VK_ERR_ARG, "Adam hyper-parameters out of range");
  ++c->step;
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)c->step));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)c->step));
  adam_kernel<<<grid_for(c->P, 256), 256, 0, c->stream>>>(c->P, c->theta, c->m1, c->m2, c->grad, c->wb, lr, beta1,
                                                           beta2, eps, (float)c1, (float)c2);
  MLP_LAUNCHED("adam_kernel");
  return VK_OK;
}

vk_status vk_mlp_patch_features(vk_mlp* c, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs, const double* X1,
                                const double* X2, const double* B, const float* mean, const float* inv_std,
                                uint16_t* out) {
  if (!c) return VK_ERR_ARG;
  if (n_cells < 0 || n_K < 1) return mfail(c, VK_ERR_ARG, "bad patch sizes");
  if (n_cells == 0) return VK_OK;
  if (!cell_dofs || !X1 || !X2 || !B || !mean || !inv_std || !out) return mfail(c, VK_ERR_ARG, "null array");
  const int64_t total = (int64_t)n_cells * 2 * n_K;
  features_kernel<<<grid_for(total, 256), 256, 0, c->stream>>>(n_cells, n_K, cell_dofs, X1, X2, B, mean, inv_std,
                                                               out);
  MLP_LAUNCHED("features_kernel");
  return VK_OK;
}

vk_status vk_mlp_patch_targets(vk_mlp* c, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs, const double* X,
                               const double* base, const float* mean, const float* inv_std, float* out) {
  if (!c) return VK_ERR_ARG;
  if (n_cells < 0 || n_K < 1) return mfail(c, VK_ERR_ARG, "bad patch sizes");
  if (n_cells == 0) return VK_OK;
  if (!cell_dofs || !X || !base || !mean || !inv_std || !out) return mfail(c, VK_ERR_ARG, "null array");
  const int64_t total = (int64_t)n_cells * n_K;
  targets_kernel<<<grid_for(total, 256), 256, 0, c->stream>>>(n_cells, n_K, cell_dofs, X, base, mean, inv_std, out);
  MLP_LAUNCHED("targets_kernel");
  return VK_OK;
}

vk_status vk_mlp_patch_average(vk_mlp* c, int64_t n, const int64_t* dof_ptr, const int64_t* dof_list, int32_t n_K,
                               const float* pred, const float* mean, const float* std, const double* base,
                               double* out) {
  if (!c) return VK_ERR_ARG;
  if (n < 0 || n_K < 1) return mfail(c, VK_ERR_ARG, "bad sizes");
  if (n == 0) return VK_OK;
  if (!dof_ptr || !dof_list || !pred || !mean || !std || !base || !out) return mfail(c, VK_ERR_ARG, "null array");
  average_kernel<<<grid_for(n, 256), 256, 0, c->stream>>>(n, dof_ptr, dof_list, n_K, pred, mean, std, base, out);
  MLP_LAUNCHED("average_kernel");
  return VK_OK;
}

vk_status vk_mlp_slab_extrapolate(vk_mlp* c, int64_t n_space, int32_t n_time, const double* E, const double* X,
                                  double* out) {
  if (!c) return VK_ERR_ARG;
  if (n_space < 0 || n_time < 1 || n_time > 8) return mfail(c, VK_ERR_ARG, "n_time must be in [1, 8]");
  if (!E || !X || !out) return mfail(c, VK_ERR_ARG, "null array");
  if (X == out) return mfail(c, VK_ERR_ARG, "out must not alias X");
  if (n_space == 0) return VK_OK;
  ext_coef co{};
  for (int a = 0; a < n_time; ++a)
    for (int b = 0; b < n_time; ++b) co.e[a * 8 + b] = E[a * n_time + b];
  extrapolate_kernel<<<grid_for(n_space, 256), 256, 0, c->stream>>>(n_space, n_time, co, X, out);
  MLP_LAUNCHED("extrapolate_kernel");
  return VK_OK;
}

}  // extern "C"
