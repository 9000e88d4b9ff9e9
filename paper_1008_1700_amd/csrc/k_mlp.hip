// Kernels of the learned initial guess: a multilayer perceptron with bf16
// weights and activations and FP32 accumulation, trained with MSE and Adam
// (FP32 master weights), and the device plumbing that turns reduced vectors
// of a DDPS handle into network inputs and back.
//
// All matrices are row-major.  k_mlp_gemm computes C = op(A) op(B) on bf16
// MFMA 32x32x16 with arbitrary (ragged) M, N, K: out-of-range elements load
// as zero and are not stored.
#include "ddps_internal.h"
#include "ddps_mlp_internal.h"

namespace ddps {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Tile 64 x 64, 256 threads = 4 waves (2 x 2), each one 32 x 32 MFMA block.
// MFMA operand X = A block (32 m x 16 k): lane l holds A[l%32][8(l/32)..+8);
// operand Y = B block (16 k x 32 n): lane l holds B[8(l/32)..+8)[l%32];
// register v of lane l is C[8(v/4) + 4(l/32) + v%4][l%32].
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_mlp_gemm(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                                  const __bf16* __restrict__ B, int ldb,
                                                  const float* __restrict__ bias, int epi,
                                                  float* __restrict__ Cf, __bf16* __restrict__ Cb, int ldc) {
  constexpr int BK = 32, LDK = BK + 8;
  __shared__ __attribute__((aligned(16))) __bf16 As[64][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[64][LDK];
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  // staging: thread -> (row = tid / 4, k = 8 (tid % 4) .. +8)
  const int sr = tid >> 2, sk = 8 * (tid & 3);
  const __bf16 zero = (__bf16)0.f;
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int m = m0 + sr, k = k0 + sk + e;
      __bf16 av = zero;
      if (m < M && k < K) av = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
      As[sr][sk + e] = av;
      const int n = n0 + sr;
      __bf16 bv = zero;
      if (n < N && k < K) bv = TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
      Bs[sr][sk + e] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int kk = ks * 16 + 8 * (lane >> 5);
      const bf16x8 x = *(const bf16x8*)&As[wm * 32 + (lane & 31)][kk];
      const bf16x8 y = *(const bf16x8*)&Bs[wn * 32 + (lane & 31)][kk];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int n = n0 + wn * 32 + (lane & 31);
    if (m < M && n < N) {
      float z = acc[v];
      if (epi & MLP_BIAS) z += bias[n];
      if (epi & MLP_F32) Cf[(int64_t)m * ldc + n] = z;
      if (epi & MLP_RELU_BF16) Cb[(int64_t)m * ldc + n] = (__bf16)fmaxf(z, 0.f);
      else if (epi & MLP_BF16) Cb[(int64_t)m * ldc + n] = (__bf16)z;
    }
  }
}

__global__ void k_f32_to_bf16(int64_t n, const float* __restrict__ x, __bf16* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (__bf16)x[i];
}

// dY = 2 (Y - T) / (rows * cols) in bf16, with per-block partial sums of (Y-T)^2
__global__ __launch_bounds__(256) void k_mse(int64_t n, float scale, const float* __restrict__ Y,
                                             const float* __restrict__ T, __bf16* __restrict__ dY,
                                             double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = (__bf16)(2.f * d * scale);
    acc += (double)d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dZ = bf16(dA * (Z > 0))
__global__ void k_relu_bwd(int64_t n, const float* __restrict__ dA, const float* __restrict__ Z,
                           __bf16* __restrict__ dZ) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dZ[i] = (__bf16)(Z[i] > 0.f ? dA[i] : 0.f);
}

// db[c] = sum over rows of dZ[r][c] (bf16 input, FP32 sum in row order)
__global__ void k_bias_grad(int rows, int cols, const __bf16* __restrict__ dZ, float* __restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += (float)dZ[(int64_t)r * cols + c];
  db[c] = s;
}

// Adam (Kingma & Ba 2015, Algorithm 1) on FP32 master parameters; the bf16
// copy used by the products is refreshed in the same pass.
__global__ void k_adam(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, __bf16* __restrict__ pb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = (__bf16)pi;
  }
}

// ------------------------------------------------------------ guess plumbing
// Interface j of the reduced vector holds its 2t entries at [2 j t, 2 (j+1) t).
// Features of interface j: [r_j / s_j, z^prev_j / q_j, cos, sin, 0 ...] with
// s_j = max |r_j| and q_j = max |z^prev_j| on c (each 1 where the vector is
// zero); one row of d_in floats per interface.
__device__ double block_absmax(const double* v, const double* mk, int t2, double* red) {
  double mx = 0.0;
  for (int i = threadIdx.x; i < t2; i += blockDim.x) mx = fmax(mx, fabs(v[i] * (mk ? mk[i] : 1.0)));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + q]);
    __syncthreads();
  }
  const double r = red[0] > 1e-300 ? red[0] : 1.0;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_features(int nif, int t2, int d_in, const double* __restrict__ rr,
                                                  const double* __restrict__ zp, const double* __restrict__ mask,
                                                  double c, double s, float* __restrict__ X,
                                                  float* __restrict__ scale) {
  __shared__ double red[256];
  const int j = blockIdx.x;   // interface (j % nif) of right-hand side j / nif
  const double* r = rr + (int64_t)j * t2;
  const double* z = zp + (int64_t)j * t2;
  const double* mk = mask + (int64_t)(j % nif) * t2;
  const double sc = block_absmax(r, nullptr, t2, red);
  const double qc = block_absmax(z, mk, t2, red);
  float* x = X + (int64_t)j * d_in;
  for (int i = threadIdx.x; i < d_in; i += blockDim.x) {
    double v = 0.0;
    if (i < t2) v = r[i] / sc;
    else if (i < 2 * t2) v = z[i - t2] * mk[i - t2] / qc;
    else if (i == 2 * t2) v = c;
    else if (i == 2 * t2 + 1) v = s;
    x[i] = (float)v;
  }
  if (threadIdx.x == 0) scale[j] = (float)sc;
}

// z0 = (z^prev + s_j * Y_j) * mask; vectors of mc entries per right-hand side
__global__ void k_compose(int64_t m, int64_t mc, int t2, const double* __restrict__ zp, const float* __restrict__ Y,
                          const float* __restrict__ scale, const double* __restrict__ mask, double* __restrict__ z0) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = q / t2;
    z0[q] = (zp[q] + (double)scale[j] * (double)Y[q]) * mask[q % mc];
  }
}

// target of interface j: (z^_j - z^prev_j) / s_j
__global__ void k_target(int64_t m, int64_t mc, int t2, const double* __restrict__ zh, const double* __restrict__ zp,
                         const float* __restrict__ scale, const double* __restrict__ mask, float* __restrict__ T) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = q / t2;
    T[q] = (float)((zh[q] - zp[q] * mask[q % mc]) / (double)scale[j]);
  }
}

// ------------------------------------------------------------ launchers
static unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

void mlp_gemm(bool ta, bool tb, int M, int N, int K, const __bf16* A, int lda, const __bf16* B, int ldb,
              const float* bias, int epi, float* Cf, __bf16* Cb, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const dim3 g((M + 63) / 64, (N + 63) / 64), b(256);
  if (!ta && !tb) hipLaunchKernelGGL((k_mlp_gemm<false, false>), g, b, 0, s, M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc);
  else if (ta && !tb) hipLaunchKernelGGL((k_mlp_gemm<true, false>), g, b, 0, s, M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc);
  else if (!ta && tb) hipLaunchKernelGGL((k_mlp_gemm<false, true>), g, b, 0, s, M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc);
  else hipLaunchKernelGGL((k_mlp_gemm<true, true>), g, b, 0, s, M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc);
}
void mlp_to_bf16(int64_t n, const float* x, __bf16* y, hipStream_t s) {
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid1(n)), dim3(256), 0, s, n, x, y);
}
int mlp_mse(int64_t n, float scale, const float* Y, const float* T, __bf16* dY, double* part, hipStream_t s) {
  const int W = (int)std::min<int64_t>((n + 255) / 256, 256);
  hipLaunchKernelGGL(k_mse, dim3(W), dim3(256), 0, s, n, scale, Y, T, dY, part);
  return W;
}
void mlp_relu_bwd(int64_t n, const float* dA, const float* Z, __bf16* dZ, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(n)), dim3(256), 0, s, n, dA, Z, dZ);
}
void mlp_bias_grad(int rows, int cols, const __bf16* dZ, float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_bias_grad, dim3((cols + 255) / 256), dim3(256), 0, s, rows, cols, dZ, db);
}
void mlp_adam(int64_t n, float lr, float b1, float b2, float eps, int t, float* p, const float* g, float* m,
              float* v, __bf16* pb, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, s, n, lr, b1, b2, eps, c1, c2, p, g, m, v, pb);
}
void guess_features(int nif, int k, int t2, int d_in, const double* rr, const double* zp, const double* mask,
                    double c, double sn, float* X, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(nif * k), dim3(256), 0, s, nif, t2, d_in, rr, zp, mask, c, sn, X, scale);
}
void guess_compose(int64_t m, int64_t mc, int t2, const double* zp, const float* Y, const float* scale,
                   const double* mask, double* z0, hipStream_t s) {
  hipLaunchKernelGGL(k_compose, dim3(grid1(m)), dim3(256), 0, s, m, mc, t2, zp, Y, scale, mask, z0);
}
void guess_target(int64_t m, int64_t mc, int t2, const double* zh, const double* zp, const float* scale,
                  const double* mask, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_target, dim3(grid1(m)), dim3(256), 0, s, m, mc, t2, zh, zp, scale, mask, T);
}

}  // namespace ddps
