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

// Tile T x T (T = 64 or 128), 256 threads = 4 waves (2 x 2), each a
// (T/2) x (T/2) sub-tile of 32 x 32 MFMA blocks; K advances in chunks of 32
// through LDS in layout [row][k] (k contiguous, padded by 8), and the next
// chunk's global loads are held in registers while the current one is
// multiplied.  Every operand is read in segments of 8 elements along its
// contiguous dimension: one 16-byte load when the leading dimension and the
// base allow it and the segment is inside the matrix, four 4-byte loads when
// only 4-byte alignment holds, else one element at a time with zero fill.
// Per output element the products are summed in the same K order whatever
// T is (chunks of 32, two 16-deep MFMAs each).
// MFMA operand X = A block (32 m x 16 k): lane l holds A[l%32][8(l/32)..+8);
// operand Y = B block (16 k x 32 n): lane l holds B[8(l/32)..+8)[l%32];
// register v of lane l is C[8(v/4) + 4(l/32) + v%4][l%32].
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// 8 elements p[0..8) (contiguous), the first `valid` of them in range;
// vw: 8 = 16-byte loads allowed, 2 = 4-byte loads allowed, 1 = elements.
__device__ __forceinline__ u16x8 load_seg(const unsigned short* __restrict__ p, int valid, int vw) {
  u16x8 r;
  if (valid >= 8 && vw == 8) return *(const u16x8*)p;
  if (valid >= 8 && vw == 2) {
    const unsigned int* q = (const unsigned int*)p;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned int w = q[e];
      r[2 * e] = (unsigned short)(w & 0xffffu);
      r[2 * e + 1] = (unsigned short)(w >> 16);
    }
    return r;
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = e < valid ? p[e] : (unsigned short)0;
  return r;
}

template <bool TA, bool TB, int T>
__global__ __launch_bounds__(256) void k_mlp_gemm(int M, int N, int K, const __bf16* __restrict__ A_, int lda,
                                                  const __bf16* __restrict__ B_, int ldb,
                                                  const float* __restrict__ bias, int epi,
                                                  float* __restrict__ Cf, __bf16* __restrict__ Cb, int ldc,
                                                  int va, int vb) {
  constexpr int BK = 32, LDK = BK + 8;
  constexpr int SEG = T * BK / 8 / 256;   // segments per thread and operand
  constexpr int WB = T / 64;              // 32 x 32 blocks per wave and dimension
  __shared__ __attribute__((aligned(16))) unsigned short As[T][LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[T][LDK];
  const unsigned short* A = (const unsigned short*)A_;
  const unsigned short* B = (const unsigned short*)B_;
  const int m0 = blockIdx.x * T, n0 = blockIdx.y * T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f32x16 acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // Segment q of a chunk: with the operand's k contiguous (A, or B stored
  // transposed) it is (row q / 4, k 8 (q % 4)); with rows contiguous (A
  // stored transposed, or B) it is (k q / (T/8), row 8 (q % (T/8))).
  u16x8 ra[SEG], rb[SEG];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const int q = tid + 256 * j;
      if (!TA) {
        const int r = q >> 2, k = k0 + 8 * (q & 3), m = m0 + r;
        ra[j] = load_seg(A + (int64_t)m * lda + k, m < M ? K - k : 0, va);
      } else {
        const int k = k0 + q / (T / 8), r = 8 * (q % (T / 8)), m = m0 + r;
        ra[j] = load_seg(A + (int64_t)k * lda + m, k < K ? M - m : 0, va);
      }
      if (TB) {
        const int r = q >> 2, k = k0 + 8 * (q & 3), n = n0 + r;
        rb[j] = load_seg(B + (int64_t)n * ldb + k, n < N ? K - k : 0, vb);
      } else {
        const int k = k0 + q / (T / 8), r = 8 * (q % (T / 8)), n = n0 + r;
        rb[j] = load_seg(B + (int64_t)k * ldb + n, k < K ? N - n : 0, vb);
      }
    }
  };
  auto stage = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const int q = tid + 256 * j;
      if (!TA) {
        *(u16x8*)&As[q >> 2][8 * (q & 3)] = ra[j];
      } else {
        const int k = q / (T / 8), r = 8 * (q % (T / 8));
#pragma unroll
        for (int e = 0; e < 8; ++e) As[r + e][k] = ra[j][e];
      }
      if (TB) {
        *(u16x8*)&Bs[q >> 2][8 * (q & 3)] = rb[j];
      } else {
        const int k = q / (T / 8), r = 8 * (q % (T / 8));
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[r + e][k] = rb[j][e];
      }
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();   // every wave is done with the previous chunk
    stage();
    __syncthreads();
    if (k0 + BK < K) fetch(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int kk = ks * 16 + 8 * (lane >> 5);
      bf16x8 x[WB], y[WB];
#pragma unroll
      for (int i = 0; i < WB; ++i) x[i] = *(const bf16x8*)&As[wm * (T / 2) + 32 * i + (lane & 31)][kk];
#pragma unroll
      for (int j = 0; j < WB; ++j) y[j] = *(const bf16x8*)&Bs[wn * (T / 2) + 32 * j + (lane & 31)][kk];
#pragma unroll
      for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[i], y[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = m0 + wm * (T / 2) + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int n = n0 + wn * (T / 2) + 32 * j + (lane & 31);
        if (m < M && n < N) {
          float z = acc[i][j][v];
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
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
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

// db[c] = sum over rows of dZ[r][c] (bf16 input, FP32 sums).  A workgroup
// takes 64 columns (one wave reads 64 consecutive entries of a row); its 16
// row groups g sum rows g, g + 16, ... in order, and the 16 partial sums are
// added pairwise in a fixed tree, so the result does not depend on timing.
constexpr int kBiasGroups = 16;
__global__ __launch_bounds__(64 * kBiasGroups) void k_bias_grad(int rows, int cols, const __bf16* __restrict__ dZ,
                                                                float* __restrict__ db) {
  __shared__ float part[kBiasGroups][64];
  const int lc = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lc;
  float s = 0.f;
  if (c < cols)
    for (int r = g; r < rows; r += kBiasGroups) s += (float)dZ[(int64_t)r * cols + c];
  part[g][lc] = s;
  __syncthreads();
  for (int h = kBiasGroups / 2; h > 0; h >>= 1) {
    if (g < h) part[g][lc] += part[g + h][lc];
    __syncthreads();
  }
  if (g == 0 && c < cols) db[c] = part[0][lc];
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
    if ((int)threadIdx.x < q) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + q]);
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

// widest load along an operand's contiguous dimension that every segment
// start allows: 16 bytes (leading dimension a multiple of 8 elements, base
// 16-byte aligned), 4 bytes, or single elements
static int seg_width(const void* p, int ld) {
  const uintptr_t a = (uintptr_t)p;
  if (ld % 8 == 0 && a % 16 == 0) return 8;
  if (ld % 2 == 0 && a % 4 == 0) return 2;
  return 1;
}

template <bool TA, bool TB>
static void mlp_gemm_t(int M, int N, int K, const __bf16* A, int lda, const __bf16* B, int ldb, const float* bias,
                       int epi, float* Cf, __bf16* Cb, int ldc, hipStream_t s) {
  const int va = seg_width(A, lda), vb = seg_width(B, ldb);
  // 128 x 128 tiles where they still give every CU at least two
  // workgroups, else 64 x 64
  const int64_t big = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
  if (big >= 512) {
    const dim3 g((M + 127) / 128, (N + 127) / 128);
    hipLaunchKernelGGL((k_mlp_gemm<TA, TB, 128>), g, dim3(256), 0, s, M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc,
                       va, vb);
  } else {
    const dim3 g((M + 63) / 64, (N + 63) / 64);
    hipLaunchKernelGGL((k_mlp_gemm<TA, TB, 64>), g, dim3(256), 0, s, M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc,
                       va, vb);
  }
}

void mlp_gemm(bool ta, bool tb, int M, int N, int K, const __bf16* A, int lda, const __bf16* B, int ldb,
              const float* bias, int epi, float* Cf, __bf16* Cb, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  if (!ta && !tb) mlp_gemm_t<false, false>(M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc, s);
  else if (ta && !tb) mlp_gemm_t<true, false>(M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc, s);
  else if (!ta && tb) mlp_gemm_t<false, true>(M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc, s);
  else mlp_gemm_t<true, true>(M, N, K, A, lda, B, ldb, bias, epi, Cf, Cb, ldc, s);
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
  hipLaunchKernelGGL(k_bias_grad, dim3((cols + 63) / 64), dim3(64 * kBiasGroups), 0, s, rows, cols, dZ, db);
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
