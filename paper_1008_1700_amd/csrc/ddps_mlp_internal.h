// Internal declarations of the learned-guess network kernels (k_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

struct ddps_mlp_ctx;

namespace ddps {

// Shape and stream of a network (for the handle's learned guess).
int mlp_shape(const ddps_mlp_ctx* M, int* d_in, int* d_out, int* max_batch, hipStream_t* stream);

enum MlpEpilogue : int {
  MLP_BIAS = 1,        // add bias[n]
  MLP_F32 = 2,         // store the FP32 result
  MLP_RELU_BF16 = 4,   // store bf16(max(z, 0))
  MLP_BF16 = 8,        // store bf16(z)
};

void mlp_gemm(bool ta, bool tb, int M, int N, int K, const __bf16* A, int lda, const __bf16* B, int ldb,
              const float* bias, int epi, float* Cf, __bf16* Cb, int ldc, hipStream_t s);
void mlp_to_bf16(int64_t n, const float* x, __bf16* y, hipStream_t s);
int mlp_mse(int64_t n, float scale, const float* Y, const float* T, __bf16* dY, double* part, hipStream_t s);
void mlp_relu_bwd(int64_t n, const float* dA, const float* Z, __bf16* dZ, hipStream_t s);
void mlp_bias_grad(int rows, int cols, const __bf16* dZ, float* db, hipStream_t s);
void mlp_adam(int64_t n, float lr, float b1, float b2, float eps, int t, float* p, const float* g, float* m,
              float* v, __bf16* pb, hipStream_t s);
// reduced vectors: k right-hand sides of mc = nif * t2 entries each; mask has mc entries
void guess_features(int nif, int k, int t2, int d_in, const double* rr, const double* zp, const double* mask,
                    double c, double sn, float* X, float* scale, hipStream_t s);
void guess_compose(int64_t m, int64_t mc, int t2, const double* zp, const float* Y, const float* scale,
                   const double* mask, double* z0, hipStream_t s);
void guess_target(int64_t m, int64_t mc, int t2, const double* zh, const double* zp, const float* scale,
                  const double* mask, float* T, hipStream_t s);

}  // namespace ddps
