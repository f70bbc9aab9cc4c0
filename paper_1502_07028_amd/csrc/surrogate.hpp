// Learned first-stage filter of delayed-acceptance Metropolis: a 3-layer MLP
// (n_in -> H -> H -> 1, SiLU) predicting the fermionic dF of a cluster move from
// the cluster spins, the proposed spin and T / kSurrogateTRef.  FP32 master weights, trained by
// hand-written FP32 forward/backward/Adam kernels; inference in BF16 on MFMA.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace tca {

constexpr double kSurrogateTRef = 0.1;  // temperature input is T / kSurrogateTRef

struct SurrogateDims {
  int n_in;    // 3 Lc^2 + 4
  int hidden;  // H
  int kpad;    // n_in rounded up to a multiple of 16 (MFMA K step)
  // offsets of the parameter blocks in the flat FP32 array
  size_t oW1, ob1, oW2, ob2, oW3, ob3, nparam;
};

SurrogateDims surrogate_dims(int Lc, int hidden);

// ---- training-side launches (FP32)
hipError_t sg_init_weights(float* W, const SurrogateDims& dm, uint64_t seed, hipStream_t st);
hipError_t sg_to_bf16(const float* W, const SurrogateDims& dm, uint16_t* W1b, uint16_t* W2b,
                      hipStream_t st);

struct SgTrainBufs {
  float *Xb, *yb, *z1, *h1, *z2, *h2, *out, *dz1, *dz2, *dh, *dout;
  double* loss;  // [1]
};
// gather `batch` rows of the dataset [row_begin, row_end) chosen by Philox(seed, step)
hipError_t sg_gather_batch(const float* X, const float* y, int n_in, int64_t row_begin,
                           int64_t row_end, int batch, uint64_t seed, uint64_t step, float* Xb,
                           float* yb, hipStream_t st);
// forward + backward of the mean squared error; grads G laid out like W
hipError_t sg_forward_backward(const float* W, const SurrogateDims& dm, int rows, SgTrainBufs b,
                               float* G, hipStream_t st);
// FP32 forward only (predictions into b.out)
hipError_t sg_forward(const float* W, const SurrogateDims& dm, int rows, SgTrainBufs b,
                      hipStream_t st);
hipError_t sg_adam(float* W, const float* G, float* m, float* v, size_t n, float lr, int64_t t,
                   hipStream_t st);
// p[0..n) = value
hipError_t sg_fill_f32(float* p, size_t n, float value, hipStream_t st);
// *sse = sum_i (out[i] - y[i])^2 in FP64, fixed order (one workgroup)
hipError_t sg_sse(const float* out, const float* y, int rows, double* sse, hipStream_t st);

// ---- inference (BF16 MFMA): rows x kpad BF16 features -> out[rows] FP32
struct SgInferBufs {
  uint16_t *H1, *H2;  // rows x H BF16 activations
};
hipError_t sg_infer_bf16(const uint16_t* Fin, int rows, const float* W, const uint16_t* W1b,
                         const uint16_t* W2b, const SurrogateDims& dm, SgInferBufs b, float* out,
                         hipStream_t st);
hipError_t sg_f32_to_bf16_rows(const float* X, int rows, int n_in, int kpad, uint16_t* out,
                               hipStream_t st);

// ---- sweep-side launches
// BF16 feature rows 2c (forward move) and 2c+1 (reverse move) of every cluster
// of a block, from the block-start spins
hipError_t sg_block_features(const double* S, BlockGeom g, int Lc, ModelParams m, SweepRef sr,
                             const SurrogateDims& dm, uint16_t* Fin, hipStream_t st);
// dataset rows (FP32 forward-move features, target dF = F[2c+1] - F[2c]) of block K:
// row row0 + (s*4 + K)*h*h + c, s the sweep index inside the call
hipError_t sg_block_collect(const double* S, BlockGeom g, int K, int Lc, ModelParams m,
                            SweepRef sr, const SurrogateDims& dm, const double* F, float* X,
                            float* y, int64_t row0, hipStream_t st);
// stage 1 of delayed acceptance: pass flags and the compacted list of passing clusters
hipError_t sg_stage1(const float* dS, BlockGeom g, ModelParams m, SweepRef sr, uint8_t* pass,
                     int32_t* count, int32_t* list, hipStream_t st);

}  // namespace tca
