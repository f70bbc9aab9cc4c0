// Kernels of the learned first-stage filter (see surrogate.hpp).
//
// Training runs in FP32 on hand-written kernels: a 64x64-tiled GEMM with
// optional transposes, fused bias/SiLU, the mean-squared-error gradient, the
// SiLU backward, column sums and Adam.  Inference packs features, weights and
// activations as BF16 and multiplies them on the matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation); the 1-wide output layer is a
// per-row dot product in FP32.
#include <hip/hip_runtime.h>

#include "rng.hpp"
#include "surrogate.hpp"

namespace tca {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 with round-to-nearest-even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

SurrogateDims surrogate_dims(int Lc, int H) {
  SurrogateDims d;
  d.n_in = 3 * Lc * Lc + 4;
  d.hidden = H;
  d.kpad = (d.n_in + 15) / 16 * 16;
  d.oW1 = 0;
  d.ob1 = (size_t)H * d.n_in;
  d.oW2 = d.ob1 + H;
  d.ob2 = d.oW2 + (size_t)H * H;
  d.oW3 = d.ob2 + H;
  d.ob3 = d.oW3 + H;
  d.nparam = d.ob3 + 1;
  return d;
}

// ------------------------------------------------------------------ init
// Uniform(-a, a), a = sqrt(6/(fan_in + fan_out)) from Philox stream 4; biases 0.
__global__ void sg_init_kernel(float* W, SurrogateDims dm, uint64_t seed) {
  const size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (q >= dm.nparam) return;
  double a;
  if (q < dm.ob1)
    a = sqrt(6.0 / (dm.n_in + dm.hidden));
  else if (q >= dm.oW2 && q < dm.ob2)
    a = sqrt(6.0 / (2.0 * dm.hidden));
  else if (q >= dm.oW3 && q < dm.ob3)
    a = sqrt(6.0 / (dm.hidden + 1.0));
  else {
    W[q] = 0.0f;
    return;
  }
  const U64x4 r = philox4x64_10(seed, 0, kInitSweep, q, 4, 0);
  W[q] = (float)(a * (2.0 * u53(r.w0) - 1.0));
}

hipError_t sg_init_weights(float* W, const SurrogateDims& dm, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(sg_init_kernel, dim3((unsigned)((dm.nparam + 255) / 256)), dim3(256), 0, st,
                     W, dm, seed);
  return hipGetLastError();
}

__global__ void sg_to_bf16_kernel(const float* W, SurrogateDims dm, uint16_t* W1b,
                                  uint16_t* W2b) {
  const int H = dm.hidden;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = H * dm.kpad;
  if (q < n1) {
    const int j = q / dm.kpad, k = q % dm.kpad;
    W1b[q] = k < dm.n_in ? f2bf(W[dm.oW1 + (size_t)j * dm.n_in + k]) : (uint16_t)0;
  } else if (q < n1 + H * H) {
    const int r = q - n1;
    W2b[r] = f2bf(W[dm.oW2 + r]);
  }
}

hipError_t sg_to_bf16(const float* W, const SurrogateDims& dm, uint16_t* W1b, uint16_t* W2b,
                      hipStream_t st) {
  const int n = dm.hidden * dm.kpad + dm.hidden * dm.hidden;
  hipLaunchKernelGGL(sg_to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, st, W, dm, W1b, W2b);
  return hipGetLastError();
}

// ------------------------------------------------------------------ FP32 GEMM
// C[M x N] = alpha * op(A) op(B) + beta * C, op(A)(i,k) = tA ? A[k lda + i] : A[i lda + k],
// op(B)(k,j) = tB ? B[j ldb + k] : B[k ldb + j].  64 x 64 tile per workgroup, K step 16.
__global__ __launch_bounds__(256) void sgemm_kernel(int M, int N, int K, float alpha,
                                                    const float* __restrict__ A, int lda, int tA,
                                                    const float* __restrict__ B, int ldb, int tB,
                                                    float beta, float* __restrict__ C, int ldc) {
  __shared__ float As[16][65], Bs[16][65];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int kk = e / 64, ii = e % 64;
      const int i = i0 + ii, j = j0 + ii, k = k0 + kk;
      As[kk][ii] = (i < M && k < K) ? (tA ? A[(size_t)k * lda + i] : A[(size_t)i * lda + k]) : 0.0f;
      Bs[kk][ii] = (j < N && k < K) ? (tB ? B[(size_t)j * ldb + k] : B[(size_t)k * ldb + j]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ty + 16 * r, j = j0 + tx + 16 * c;
      if (i < M && j < N) {
        float v = alpha * acc[r][c];
        if (beta != 0.0f) v += beta * C[(size_t)i * ldc + j];
        C[(size_t)i * ldc + j] = v;
      }
    }
}

static hipError_t sgemm(int M, int N, int K, float alpha, const float* A, int lda, int tA,
                        const float* B, int ldb, int tB, float beta, float* C, int ldc,
                        hipStream_t st) {
  const dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(sgemm_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, tA, B, ldb, tB,
                     beta, C, ldc);
  return hipGetLastError();
}

// Z += bias (per column), H = silu(Z)
__global__ void bias_silu_kernel(float* Z, float* Hh, const float* bias, int M, int N) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M * N) return;
  const float z = Z[q] + bias[q % N];
  Z[q] = z;
  Hh[q] = silu_f(z);
}

// out[i] = h[i] . w + b  (fixed order)
__global__ void rowdot_kernel(const float* Hh, const float* w, const float* b, int M, int N,
                              float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  float s = 0.0f;
  for (int j = 0; j < N; ++j) s = fmaf(Hh[(size_t)i * N + j], w[j], s);
  out[i] = s + b[0];
}

// r = out - y, dout = 2 r / M, loss = mean(r^2) (one workgroup, fixed order)
__global__ __launch_bounds__(256) void mse_kernel(const float* out, const float* y, int M,
                                                  float* dout, double* loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) {
    const float r = out[i] - y[i];
    dout[i] = 2.0f * r / (float)M;
    s += (double)r * (double)r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss != nullptr) *loss = red[0] / M;
}

// gw[j] = sum_i dout[i] h[i][j],  gb = sum_i dout[i]
__global__ void out_layer_grad_kernel(const float* dout, const float* Hh, int M, int N, float* gw,
                                      float* gb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) {
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s = fmaf(dout[i], Hh[(size_t)i * N + j], s);
    gw[j] = s;
  }
  if (j == N) {
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += dout[i];
    gb[0] = s;
  }
}

// dz[i][j] = dout[i] w[j] silu'(z[i][j])
__global__ void out_back_kernel(const float* dout, const float* w, const float* Z, int M, int N,
                                float* dz) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M * N) return;
  dz[q] = dout[q / N] * w[q % N] * silu_grad_f(Z[q]);
}

// dz = dh * silu'(z)
__global__ void silu_back_kernel(const float* dh, const float* Z, int n, float* dz) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dz[q] = dh[q] * silu_grad_f(Z[q]);
}

// g[j] = sum_i D[i][j]
__global__ void colsum_kernel(const float* D, int M, int N, float* g) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int i = 0; i < M; ++i) s += D[(size_t)i * N + j];
  g[j] = s;
}

static inline dim3 grid1(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t sg_forward(const float* W, const SurrogateDims& dm, int rows, SgTrainBufs b,
                      hipStream_t st) {
  const int H = dm.hidden, nin = dm.n_in;
  hipError_t e;
  if ((e = sgemm(rows, H, nin, 1.0f, b.Xb, nin, 0, W + dm.oW1, nin, 1, 0.0f, b.z1, H, st))) return e;
  hipLaunchKernelGGL(bias_silu_kernel, grid1((long)rows * H), dim3(256), 0, st, b.z1, b.h1,
                     W + dm.ob1, rows, H);
  if ((e = sgemm(rows, H, H, 1.0f, b.h1, H, 0, W + dm.oW2, H, 1, 0.0f, b.z2, H, st))) return e;
  hipLaunchKernelGGL(bias_silu_kernel, grid1((long)rows * H), dim3(256), 0, st, b.z2, b.h2,
                     W + dm.ob2, rows, H);
  hipLaunchKernelGGL(rowdot_kernel, grid1(rows), dim3(256), 0, st, b.h2, W + dm.oW3, W + dm.ob3,
                     rows, H, b.out);
  return hipGetLastError();
}

hipError_t sg_forward_backward(const float* W, const SurrogateDims& dm, int rows, SgTrainBufs b,
                               float* G, hipStream_t st) {
  const int H = dm.hidden, nin = dm.n_in;
  hipError_t e;
  if ((e = sg_forward(W, dm, rows, b, st))) return e;
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, st, b.out, b.yb, rows, b.dout, b.loss);
  hipLaunchKernelGGL(out_layer_grad_kernel, grid1(H + 1), dim3(256), 0, st, b.dout, b.h2, rows, H,
                     G + dm.oW3, G + dm.ob3);
  hipLaunchKernelGGL(out_back_kernel, grid1((long)rows * H), dim3(256), 0, st, b.dout, W + dm.oW3,
                     b.z2, rows, H, b.dz2);
  // gW2 = dz2^T h1, gb2 = colsum(dz2)
  if ((e = sgemm(H, H, rows, 1.0f, b.dz2, H, 1, b.h1, H, 0, 0.0f, G + dm.oW2, H, st))) return e;
  hipLaunchKernelGGL(colsum_kernel, grid1(H), dim3(256), 0, st, b.dz2, rows, H, G + dm.ob2);
  // dh1 = dz2 W2, dz1 = dh1 * silu'(z1)
  if ((e = sgemm(rows, H, H, 1.0f, b.dz2, H, 0, W + dm.oW2, H, 0, 0.0f, b.dh, H, st))) return e;
  hipLaunchKernelGGL(silu_back_kernel, grid1((long)rows * H), dim3(256), 0, st, b.dh, b.z1,
                     rows * H, b.dz1);
  // gW1 = dz1^T X, gb1 = colsum(dz1)
  if ((e = sgemm(H, nin, rows, 1.0f, b.dz1, H, 1, b.Xb, nin, 0, 0.0f, G + dm.oW1, nin, st)))
    return e;
  hipLaunchKernelGGL(colsum_kernel, grid1(H), dim3(256), 0, st, b.dz1, rows, H, G + dm.ob1);
  return hipGetLastError();
}

// Adam (Kingma & Ba): beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected.
__global__ void adam_kernel(float* W, const float* G, float* m, float* v, size_t n, float lr,
                            float c1, float c2) {
  const size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float g = G[q];
  const float mq = 0.9f * m[q] + 0.1f * g;
  const float vq = 0.999f * v[q] + 0.001f * g * g;
  m[q] = mq;
  v[q] = vq;
  W[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + 1e-8f);
}

hipError_t sg_adam(float* W, const float* G, float* m, float* v, size_t n, float lr, int64_t t,
                   hipStream_t st) {
  const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
  hipLaunchKernelGGL(adam_kernel, grid1((long)n), dim3(256), 0, st, W, G, m, v, n, lr, c1, c2);
  return hipGetLastError();
}

__global__ void fill_f32_kernel(float* p, size_t n, float value) {
  const size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (q < n) p[q] = value;
}

hipError_t sg_fill_f32(float* p, size_t n, float value, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, grid1((long)n), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void sse_kernel(const float* out, const float* y, int M,
                                                  double* sse) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) {
    const double r = (double)out[i] - (double)y[i];
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *sse = red[0];
}

hipError_t sg_sse(const float* out, const float* y, int rows, double* sse, hipStream_t st) {
  hipLaunchKernelGGL(sse_kernel, dim3(1), dim3(256), 0, st, out, y, rows, sse);
  return hipGetLastError();
}

// batch row i of training step `step`: dataset row row_begin + (philox % span)
__global__ void gather_kernel(const float* X, const float* y, int nin, int64_t row_begin,
                              int64_t span, int batch, uint64_t seed, uint64_t step, float* Xb,
                              float* yb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= batch * nin) return;
  const int i = q / nin, k = q % nin;
  const U64x4 r = philox4x64_10(seed, 0, step, (uint64_t)i, 5, 0);
  const int64_t row = row_begin + (int64_t)(r.w0 % (uint64_t)span);
  Xb[q] = X[row * nin + k];
  if (k == 0) yb[i] = y[row];
}

hipError_t sg_gather_batch(const float* X, const float* y, int n_in, int64_t row_begin,
                           int64_t row_end, int batch, uint64_t seed, uint64_t step, float* Xb,
                           float* yb, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, grid1((long)batch * n_in), dim3(256), 0, st, X, y, n_in,
                     row_begin, row_end - row_begin, batch, seed, step, Xb, yb);
  return hipGetLastError();
}

// ------------------------------------------------------------------ BF16 MFMA inference
// Y[rows x N] = act(X[rows x K] W^T + bias) with X, W, Y in BF16 (K multiple of 16),
// FP32 accumulation.  64 x 64 output tile per workgroup of four wavefronts; wavefront
// w owns tile rows 16w..16w+15 and the four 16 x 16 column blocks.  Operand layout of
// v_mfma_f32_16x16x16_bf16: lane l supplies A[l%16][4(l/16)..+3] and
// B[4(l/16)..+3][l%16] and receives D[4(l/16)..+3][l%16].
constexpr int kMfmaKChunk = 64;

template <bool SILU>
__global__ __launch_bounds__(256) void mlp_layer_bf16_kernel(const uint16_t* __restrict__ X,
                                                             int rows, int K,
                                                             const uint16_t* __restrict__ Wb,
                                                             const float* __restrict__ bias,
                                                             int N, uint16_t* __restrict__ Y) {
  constexpr int KP = kMfmaKChunk + 4;  // padded LDS row (keeps 8-byte alignment)
  __shared__ uint16_t Xs[64 * KP], Ws[64 * KP];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int am = 16 * wave + (lane % 16);
  const int kl = 4 * (lane / 16);
  for (int kc = 0; kc < K; kc += kMfmaKChunk) {
    const int kw = (K - kc) < kMfmaKChunk ? (K - kc) : kMfmaKChunk;  // multiple of 16
    for (int e = threadIdx.x; e < 64 * (kw / 4); e += 256) {
      const int rr = e / (kw / 4), kq = (e % (kw / 4)) * 4;
      uint2 vx = make_uint2(0u, 0u), vw = make_uint2(0u, 0u);
      if (r0 + rr < rows) vx = *(const uint2*)(X + (size_t)(r0 + rr) * K + kc + kq);
      if (c0 + rr < N) vw = *(const uint2*)(Wb + (size_t)(c0 + rr) * K + kc + kq);
      *(uint2*)(Xs + rr * KP + kq) = vx;
      *(uint2*)(Ws + rr * KP + kq) = vw;
    }
    __syncthreads();
    for (int k0 = 0; k0 < kw; k0 += 16) {
      const bf16x4 a = *(const bf16x4*)(Xs + am * KP + k0 + kl);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bf16x4 b = *(const bf16x4*)(Ws + (16 * t + (lane % 16)) * KP + k0 + kl);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = r0 + 16 * wave + kl + j, col = c0 + 16 * t + (lane % 16);
      if (row < rows && col < N) {
        float z = acc[t][j] + bias[col];
        if (SILU) z = silu_f(z);
        Y[(size_t)row * N + col] = f2bf(z);
      }
    }
  }
}

__global__ void rowdot_bf16_kernel(const uint16_t* Hh, const float* w, const float* b, int M,
                                   int N, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  float s = 0.0f;
  for (int j = 0; j < N; ++j) s = fmaf(bf2f(Hh[(size_t)i * N + j]), w[j], s);
  out[i] = s + b[0];
}

hipError_t sg_infer_bf16(const uint16_t* Fin, int rows, const float* W, const uint16_t* W1b,
                         const uint16_t* W2b, const SurrogateDims& dm, SgInferBufs b, float* out,
                         hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int H = dm.hidden;
  const dim3 grid((rows + 63) / 64, (H + 63) / 64);
  hipLaunchKernelGGL(mlp_layer_bf16_kernel<true>, grid, dim3(256), 0, st, Fin, rows, dm.kpad, W1b,
                     W + dm.ob1, H, b.H1);
  hipLaunchKernelGGL(mlp_layer_bf16_kernel<true>, grid, dim3(256), 0, st, b.H1, rows, H, W2b,
                     W + dm.ob2, H, b.H2);
  hipLaunchKernelGGL(rowdot_bf16_kernel, grid1(rows), dim3(256), 0, st, b.H2, W + dm.oW3,
                     W + dm.ob3, rows, H, out);
  return hipGetLastError();
}

__global__ void f32_to_bf16_rows_kernel(const float* X, int rows, int nin, int kpad,
                                        uint16_t* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * kpad) return;
  const int i = q / kpad, k = q % kpad;
  out[q] = k < nin ? f2bf(X[(size_t)i * nin + k]) : (uint16_t)0;
}

hipError_t sg_f32_to_bf16_rows(const float* X, int rows, int n_in, int kpad, uint16_t* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(f32_to_bf16_rows_kernel, grid1((long)rows * kpad), dim3(256), 0, st, X, rows,
                     n_in, kpad, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sweep-side kernels
// One workgroup per cluster: feature values of the forward move (cluster spins,
// proposal, T) and of the reverse move (corner = proposal, proposing the old spin).
template <bool COLLECT>
__global__ __launch_bounds__(64) void sg_features_kernel(const double* __restrict__ S,
                                                         BlockGeom g, int K, int Lc, ModelParams m,
                                                         SweepRef sr, SurrogateDims dm,
                                                         uint16_t* Fin, const double* F, float* X,
                                                         float* y, int64_t row0) {
  __shared__ double prop[3];
  const int c = blockIdx.x;
  const int px = g.x0 + c % g.h, py = g.y0 + c / g.h;
  const double T = sr.T();
  if (threadIdx.x == 0)
    sphere_point(m.seed, sr.sweep(), (uint64_t)(px + g.L * py), kStreamProposal, prop);
  __syncthreads();
  const int Nc = Lc * Lc;
  const int width = COLLECT ? dm.n_in : dm.kpad;
  const int64_t row = row0 + ((int64_t)sr.s() * 4 + K) * (int64_t)(g.h * g.h) + c;
  for (int k = threadIdx.x; k < width; k += 64) {
    double vf = 0.0, vr = 0.0;
    if (k < 3 * Nc) {
      const int l = k / 3, comp = k % 3;
      const int sx = (px + l % Lc) % g.L, sy = (py + l / Lc) % g.L;
      vf = S[3 * (sx + g.L * sy) + comp];
      vr = (l == 0) ? prop[comp] : vf;
    } else if (k < 3 * Nc + 3) {
      const int comp = k - 3 * Nc;
      vf = prop[comp];
      vr = S[3 * (px + g.L * py) + comp];
    } else if (k == 3 * Nc + 3) {
      vf = vr = T / kSurrogateTRef;
    }
    if (COLLECT) {
      X[row * dm.n_in + k] = (float)vf;
    } else {
      Fin[(size_t)(2 * c) * dm.kpad + k] = f2bf((float)vf);
      Fin[(size_t)(2 * c + 1) * dm.kpad + k] = f2bf((float)vr);
    }
  }
  if (COLLECT && threadIdx.x == 0) y[row] = (float)(F[2 * c + 1] - F[2 * c]);
}

hipError_t sg_block_features(const double* S, BlockGeom g, int Lc, ModelParams m, SweepRef sr,
                             const SurrogateDims& dm, uint16_t* Fin, hipStream_t st) {
  hipLaunchKernelGGL(sg_features_kernel<false>, dim3(g.h * g.h), dim3(64), 0, st, S, g, 0, Lc, m,
                     sr, dm, Fin, (const double*)nullptr, (float*)nullptr, (float*)nullptr,
                     (int64_t)0);
  return hipGetLastError();
}

hipError_t sg_block_collect(const double* S, BlockGeom g, int K, int Lc, ModelParams m,
                            SweepRef sr, const SurrogateDims& dm, const double* F, float* X,
                            float* y, int64_t row0, hipStream_t st) {
  hipLaunchKernelGGL(sg_features_kernel<true>, dim3(g.h * g.h), dim3(64), 0, st, S, g, K, Lc, m,
                     sr, dm, (uint16_t*)nullptr, F, X, y, row0);
  return hipGetLastError();
}

// Stage 1: pass iff u1 == 0 or ln u1 < min(0, -dS_f/T) (u1 = word 1 of the Metropolis block).
__global__ void sg_stage1_kernel(const float* dS, BlockGeom g, ModelParams m, SweepRef sr,
                                 uint8_t* pass, int32_t* count, int32_t* list) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.h * g.h) return;
  const double T = sr.T();
  const int site = (g.x0 + c % g.h) + g.L * (g.y0 + c / g.h);
  const U64x4 r = philox4x64_10(m.seed, 0, sr.sweep(), (uint64_t)site, kStreamMetropolis, 0);
  const double u1 = u53(r.w1);
  const double rhs = fmin(0.0, -(double)dS[2 * c] / T);
  const bool p = (u1 <= 0.0) || (log(u1) < rhs);
  pass[c] = p ? 1 : 0;
  if (p) list[atomicAdd(count, 1)] = c;
}

__global__ void zero_i32_one(int32_t* p) { *p = 0; }

hipError_t sg_stage1(const float* dS, BlockGeom g, ModelParams m, SweepRef sr, uint8_t* pass,
                     int32_t* count, int32_t* list, hipStream_t st) {
  hipLaunchKernelGGL(zero_i32_one, dim3(1), dim3(1), 0, st, count);
  const int hh = g.h * g.h;
  hipLaunchKernelGGL(sg_stage1_kernel, grid1(hh), dim3(256), 0, st, dS, g, m, sr, pass, count,
                     list);
  return hipGetLastError();
}

}  // namespace tca
