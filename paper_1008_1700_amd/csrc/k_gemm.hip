// Grouped GEMM on CDNA4 matrix cores: D = C0 +/- op(A) op(B) over a list of
// independent problems (one launch covers every block of the partition).
//
// Workgroup tile 64 x 64, 256 threads = 4 waves, each wave a 32 x 32 sub-tile
// made of 2 x 2 MFMA 16x16 blocks.  K advances in chunks of 16 (f64/f32) or 32
// (bf16) staged through LDS with one register prefetch stage.  Operands are
// column-major (LAPACK layout).  Triangular operands are exploited twice:
// the K range of each output tile is clipped to where both operands can be
// nonzero, and masked loads read the unit-lower / upper halves of the packed
// inverse tiles.
//
// The MFMA is fed with B^T as its first and A^T as its second operand, so it
// accumulates D^T: the 16 lanes of a lane group hold 16 consecutive rows of
// one column of D, and the stores to the column-major D are 128-byte (f64)
// segments.
#include "ddps_internal.h"

namespace ddps {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Logical workgroup index such that each XCD (hardware dispatches workgroups
// round-robin over the 8 XCDs) receives one contiguous range of tiles: tiles
// of the same block then share that XCD's L2.
__device__ __forceinline__ int xcd_swizzle(int bid, int n) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + min(xcd, rem) + idx;
}

__device__ __forceinline__ int find_prob(const GemmProb* __restrict__ probs, int nprob, int wg) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile0 <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ T masked(T v, int r, int c, int flags_lu, int flags_up) {
  if (flags_lu) return r > c ? v : (r == c ? T(1) : T(0));
  if (flags_up) return r <= c ? v : T(0);
  return v;
}

template <typename T> struct Mma;
// Accumulator layouts (lane l, register v) -> row of the 16 x 16 result:
// f32 16x16x4: 4 (l >> 4) + v;   f64 16x16x4: (l >> 4) + 4 v  (measured).
template <> struct Mma<double> {
  using acc = f64x4;
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<float> {
  using acc = f32x4;
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// ------------------------------------------------------------------------
// f64 / f32: K chunk 16, one MFMA 16x16x4 per (k4, mi, ni).
// ------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_std(const GemmProb* __restrict__ probs, int nprob) {
  constexpr int BK = 16, LDP = 64 + 4;
  __shared__ T As[2][BK][LDP];
  __shared__ T Bs[2][BK][LDP];
  using acc_t = typename Mma<T>::acc;

  const int wg = xcd_swizzle(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprob, wg)];
  const int tiles_m = P.M >> 6;
  const int local = wg - P.tile0;
  const int I0 = (local % tiles_m) << 6;
  const int J0 = (local / tiles_m) << 6;
  const int fl = P.flags;

  int kb = 0, ke = P.K;
  if (fl & G_A_UP) kb = max(kb, I0);
  if (fl & G_B_LO) kb = max(kb, J0);
  if (fl & G_A_LO) ke = min(ke, I0 + 64);
  if (fl & G_B_UP) ke = min(ke, J0 + 64);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const T* __restrict__ A = (const T*)P.A;
  const T* __restrict__ B = (const T*)P.B;
  const int a_lu = fl & G_A_MLU, a_up = fl & G_A_MUP, b_lu = fl & G_B_MLU, b_up = fl & G_B_MUP;

  acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // A chunk: 64 rows x 16 k; thread -> (m = tid&63, kk = tid>>6 + 4i)
  // B chunk: 16 k x 64 cols; thread -> (kk = tid&15, n = tid>>4 + 16i)
  const int am = tid & 63, ak = tid >> 6;
  const int bk = tid & 15, bn = tid >> 4;
  T ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = I0 + am, c = k0 + ak + 4 * i;
      T v = T(0);
      const bool need = a_lu ? (r > c) : (a_up ? (r <= c) : true);
      if (need) v = A[(int64_t)c * P.lda + r];
      ra[i] = masked(v, r, c, a_lu, a_up);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = k0 + bk, c = J0 + bn + 16 * i;
      T v = T(0);
      const bool need = b_lu ? (r > c) : (b_up ? (r <= c) : true);
      if (need) v = B[(int64_t)c * P.ldb + r];
      rb[i] = masked(v, r, c, b_lu, b_up);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) As[buf][ak + 4 * i][am] = ra[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) Bs[buf][bk][bn + 16 * i] = rb[i];
  };

  if (kb < ke) {
    load(kb);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = (k0 + BK) < ke;
      if (more) load(k0 + BK);
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kk = k4 * 4 + (lane >> 4);
        T xa[2], xb[2];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) xa[ni] = Bs[cur][kk][wn * 32 + ni * 16 + (lane & 15)];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) xb[mi] = As[cur][kk][wm * 32 + mi * 16 + (lane & 15)];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = Mma<T>::run(xa[ni], xb[mi], acc[mi][ni]);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }

  // Epilogue: lane holds D[row = .. + (lane&15)][col = .. + Mma::row(lane, v)]
  // (the MFMA computed D^T, so its rows are D's columns)
  const T* __restrict__ C0 = (const T*)P.C0;
  T* __restrict__ D = (T*)P.D;
  const bool has_c0 = fl & G_C0, neg = fl & G_NEG;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = I0 + wm * 32 + mi * 16 + (lane & 15);
        const int c = J0 + wn * 32 + ni * 16 + Mma<T>::row(lane, v);
        T val = acc[mi][ni][v];
        if (neg) val = -val;
        if (has_c0) val += C0[(int64_t)c * P.ldc0 + r];
        D[(int64_t)c * P.ldd + r] = val;
      }
}

// ------------------------------------------------------------------------
// bf16 MFMA (16x16x32, FP32 accumulation) on FP32-stored operands.  With
// SPLIT each FP32 operand x is written as hi + lo, hi = bf16(x),
// lo = bf16(x - hi), and the product is hi*hi + hi*lo + lo*hi (the lo*lo
// term is below FP32 rounding of the result's leading part).
// ------------------------------------------------------------------------
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_gemm_bf16(const GemmProb* __restrict__ probs, int nprob) {
  constexpr int BK = 32;
  constexpr int LDK = BK + 8;  // k-contiguous rows of 32 bf16, padded
  __shared__ __bf16 Ah[64][LDK];
  __shared__ __bf16 Bh[64][LDK];
  __shared__ __bf16 Al[SPLIT ? 64 : 1][LDK];
  __shared__ __bf16 Bl[SPLIT ? 64 : 1][LDK];

  const int wg = xcd_swizzle(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprob, wg)];
  const int tiles_m = P.M >> 6;
  const int local = wg - P.tile0;
  const int I0 = (local % tiles_m) << 6;
  const int J0 = (local / tiles_m) << 6;
  const int fl = P.flags;
  int kb = 0, ke = P.K;
  if (fl & G_A_UP) kb = max(kb, I0);
  if (fl & G_B_LO) kb = max(kb, J0);
  if (fl & G_A_LO) ke = min(ke, I0 + 64);
  if (fl & G_B_UP) ke = min(ke, J0 + 64);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const float* __restrict__ A = (const float*)P.A;
  const float* __restrict__ B = (const float*)P.B;
  const int a_lu = fl & G_A_MLU, a_up = fl & G_A_MUP, b_lu = fl & G_B_MLU, b_up = fl & G_B_MUP;

  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  // A chunk 64 x 32: thread -> (m = tid&63, k = tid>>6 + 4i), i < 8
  // B chunk 32 x 64: thread -> (k = tid&31, n = tid>>5 + 8i), i < 8
  const int am = tid & 63, ak = tid >> 6;
  const int bk = tid & 31, bn = tid >> 5;
  for (int k0 = kb; k0 < ke; k0 += BK) {
    float ra[8], rb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = I0 + am, c = k0 + ak + 4 * i;
      float v = 0.f;
      const bool need = a_lu ? (r > c) : (a_up ? (r <= c) : true);
      if (need) v = A[(int64_t)c * P.lda + r];
      ra[i] = masked(v, r, c, a_lu, a_up);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = k0 + bk, c = J0 + bn + 8 * i;
      float v = 0.f;
      const bool need = b_lu ? (r > c) : (b_up ? (r <= c) : true);
      if (need) v = B[(int64_t)c * P.ldb + r];
      rb[i] = masked(v, r, c, b_lu, b_up);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const __bf16 h = to_bf16(ra[i]);
      Ah[am][ak + 4 * i] = h;
      if (SPLIT) Al[am][ak + 4 * i] = to_bf16(ra[i] - (float)h);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const __bf16 h = to_bf16(rb[i]);
      Bh[bn + 8 * i][bk] = h;
      if (SPLIT) Bl[bn + 8 * i][bk] = to_bf16(rb[i] - (float)h);
    }
    __syncthreads();
    // MFMA 16x16x32 bf16: operand X (16 x 32): lane holds row lane&15,
    // k = 8*(lane>>4) .. +8; operand Y (32 x 16): lane holds col lane&15,
    // the same k range.  X = B^T block, Y = A^T block.
    const int kk = 8 * (lane >> 4);
    bf16x8 xh[2], yh[2], xl[2], yl[2];
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int n = wn * 32 + ni * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        xh[ni][e] = Bh[n][kk + e];
        if (SPLIT) xl[ni][e] = Bl[n][kk + e];
      }
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int m = wm * 32 + mi * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        yh[mi][e] = Ah[m][kk + e];
        if (SPLIT) yl[mi][e] = Al[m][kk + e];
      }
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        if (SPLIT) {
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[ni], yh[mi], acc[mi][ni], 0, 0, 0);
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[ni], yl[mi], acc[mi][ni], 0, 0, 0);
        }
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[ni], yh[mi], acc[mi][ni], 0, 0, 0);
      }
  }

  const float* __restrict__ C0 = (const float*)P.C0;
  float* __restrict__ D = (float*)P.D;
  const bool has_c0 = fl & G_C0, neg = fl & G_NEG;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = I0 + wm * 32 + mi * 16 + (lane & 15);
        const int c = J0 + wn * 32 + ni * 16 + 4 * (lane >> 4) + v;
        float val = acc[mi][ni][v];
        if (neg) val = -val;
        if (has_c0) val += C0[(int64_t)c * P.ldc0 + r];
        D[(int64_t)c * P.ldd + r] = val;
      }
}

void launch_gemm(int dtype, int mode, const GemmProb* probs, int nprob, int nwg, hipStream_t s) {
  (void)mode;
  if (nwg <= 0 || nprob <= 0) return;
  switch (dtype) {
    case 0: hipLaunchKernelGGL(k_gemm_std<double>, dim3(nwg), dim3(256), 0, s, probs, nprob); break;
    case 1: hipLaunchKernelGGL(k_gemm_std<float>, dim3(nwg), dim3(256), 0, s, probs, nprob); break;
    case 2: hipLaunchKernelGGL(k_gemm_bf16<true>, dim3(nwg), dim3(256), 0, s, probs, nprob); break;
    default: hipLaunchKernelGGL(k_gemm_bf16<false>, dim3(nwg), dim3(256), 0, s, probs, nprob); break;
  }
}

}  // namespace ddps
