// Grouped GEMM on CDNA4 matrix cores: D = C0 +/- op(A) op(B) over a list of
// independent problems (one launch covers every block of the partition).
//
// Three kernels: k_gemm_std (f64 / f32 MFMA 16x16x4), k_gemm_bf16 (bf16 MFMA
// on FP32 operands staged through registers) and k_gemm_dl (the same bf16
// products with the operands copied straight into LDS).  For k_gemm_std the
// workgroup tile is BM x BN (64 x 64 or 128 x 128), 256 threads = 4 waves in
// a 2 x 2 arrangement, each wave a (BM/2) x (BN/2) sub-tile of 16 x 16 MFMA
// blocks; K advances in chunks of 16 staged through LDS, with the next
// chunk's global loads in flight while the current chunk is multiplied.  Operands are column-major (LAPACK layout); M and N need
// only be multiples of 64 (a 128-tile on the edge is masked).  Triangular
// operands are exploited twice: the K range of each output tile is clipped
// to where both operands can be nonzero, and masked loads read the
// unit-lower / upper halves of the packed inverse tiles.
//
// The MFMA is fed with B^T as its first and A^T as its second operand, so it
// accumulates D^T: the 16 lanes of a lane group hold 16 consecutive rows of
// one column of D, and the stores to the column-major D are 64-128-byte
// segments.
#include "ddps_internal.h"

namespace ddps {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// The problem records hold generic pointers; loads through them compile to
// flat loads, which also count against the LDS wait counter, so every wait
// for LDS would wait for them too.  Casting to the global address space gives
// global loads and stores with their own counter.
template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> using gmut = __attribute__((address_space(1))) T*;
__device__ __forceinline__ float4 gload4(const float* p) {
  const f32x4 v = *(gptr<f32x4>)p;
  return make_float4(v[0], v[1], v[2], v[3]);
}

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

// Value of op(X)(r, c) given the stored value v: masks of the packed
// triangles (unit lower, upper, lower with its diagonal) and zero outside the
// problem (rows >= rmax or columns >= cmax).  A select, so whatever the other
// triangle of a packed tile holds never reaches a product.
template <typename T>
__device__ __forceinline__ T select_op(T v, int r, int c, bool lu, bool up, bool lo, int rmax, int cmax) {
  if (lu) v = r > c ? v : (r == c ? T(1) : T(0));
  if (up) v = r <= c ? v : T(0);
  if (lo) v = r >= c ? v : T(0);
  return (r < rmax && c < cmax) ? v : T(0);
}

// Output mask of the epilogue: G_D_UP stores only entries on or above the
// diagonal, G_D_LO only entries on or below it (the two halves of a packed
// pair of triangles); the other half of the destination is left untouched.
__device__ __forceinline__ bool store_ok(int fl, int r, int c) {
  if ((fl & G_D_UP) && r > c) return false;
  if ((fl & G_D_LO) && r < c) return false;
  return true;
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

struct TileCoord {
  int I0, J0, kb, ke;
};

template <int BM, int BN>
__device__ __forceinline__ TileCoord tile_of(const GemmProb& P, int wg) {
  const int tiles_m = (P.M + BM - 1) / BM;
  const int local = wg - P.tile0;
  TileCoord t;
  t.I0 = (local % tiles_m) * BM;
  t.J0 = (local / tiles_m) * BN;
  const int fl = P.flags;
  t.kb = 0;
  t.ke = P.K;
  if (fl & G_A_UP) t.kb = max(t.kb, t.I0);
  if (fl & G_B_LO) t.kb = max(t.kb, t.J0);
  if (fl & G_A_LO) t.ke = min(t.ke, t.I0 + BM);
  if (fl & G_B_UP) t.ke = min(t.ke, t.J0 + BN);
  return t;
}

// ------------------------------------------------------------------------
// f64 / f32: K chunk 16, one MFMA 16x16x4 per (k4, mi, ni).
// ------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK = 16, int OCC = 1>
__global__ __launch_bounds__(256, OCC) void k_gemm_std(const GemmProb* __restrict__ probs, int nprob,
                                                 const int32_t* __restrict__ order) {
  constexpr int PADL = 4;
  constexpr int MB = BM / 32, NB = BN / 32;          // 16x16 blocks per wave
  constexpr int AE = BM * BK / 256, BE = BN * BK / 256;  // elements per thread
  __shared__ T As[2][BK][BM + PADL];
  __shared__ T Bs[2][BK][BN + PADL];
  using acc_t = typename Mma<T>::acc;

  const int wg = order ? order[xcd_swizzle(blockIdx.x, gridDim.x)] : xcd_swizzle(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprob, wg)];
  const TileCoord tc = tile_of<BM, BN>(P, wg);
  const int I0 = tc.I0, J0 = tc.J0, kb = tc.kb, ke = tc.ke;
  const int fl = P.flags;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  gptr<T> A = (gptr<T>)P.A;
  gptr<T> B = (gptr<T>)P.B;
  const bool a_lu = fl & G_A_MLU, a_up = fl & G_A_MUP, b_lu = fl & G_B_MLU, b_up = fl & G_B_MUP;
  const bool a_lo = fl & G_A_MLO, b_lo = fl & G_B_MLO;

  acc_t acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // A chunk BM x 16: thread -> row m = tid % BM, k = tid / BM + (256/BM) i
  // B chunk 16 x BN: thread -> col n = tid % BN, k = (tid / BN) * BE + i  (BE consecutive k)
  constexpr int ASTEP = 256 / BM;
  static_assert(AE * ASTEP == BK, "A chunk mapping");
  const int am = tid % BM, ak = tid / BM;
  const int bn = tid % BN, bk0 = (tid / BN) * BE;
  const int arow = min(I0 + am, P.M - 1);
  const int bcol = min(J0 + bn, P.N - 1);
  T ra[AE], rb[BE];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int c = k0 + ak + ASTEP * i;
      ra[i] = select_op(A[(int64_t)c * P.lda + arow], I0 + am, c, a_lu, a_up, a_lo, P.M, 1 << 30);
    }
    gptr<T> bp = B + (int64_t)bcol * P.ldb + k0 + bk0;
#pragma unroll
    for (int i = 0; i < BE; ++i) rb[i] = select_op(bp[i], k0 + bk0 + i, J0 + bn, b_lu, b_up, b_lo, 1 << 30, P.N);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AE; ++i) As[buf][ak + ASTEP * i][am] = ra[i];
#pragma unroll
    for (int i = 0; i < BE; ++i) Bs[buf][bk0 + i][bn] = rb[i];
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
        T xa[NB], xb[MB];
#pragma unroll
        for (int ni = 0; ni < NB; ++ni) xa[ni] = Bs[cur][kk][wn * (BN / 2) + ni * 16 + (lane & 15)];
#pragma unroll
        for (int mi = 0; mi < MB; ++mi) xb[mi] = As[cur][kk][wm * (BM / 2) + mi * 16 + (lane & 15)];
#pragma unroll
        for (int mi = 0; mi < MB; ++mi)
#pragma unroll
          for (int ni = 0; ni < NB; ++ni) acc[mi][ni] = Mma<T>::run(xa[ni], xb[mi], acc[mi][ni]);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }

  // Epilogue: lane holds D[row = .. + (lane&15)][col = .. + Mma::row(lane, v)].
  // Whole tiles load their C0 values in one batch per 16 x 16 block.
  gptr<T> C0 = (gptr<T>)P.C0;
  gmut<T> D = (gmut<T>)P.D;
  const bool has_c0 = fl & G_C0;
  const T sg = (fl & G_NEG) ? T(-1) : T(1);
  if (I0 + BM <= P.M && J0 + BN <= P.N && !(fl & (G_D_UP | G_D_LO))) {
#pragma unroll
    for (int mi = 0; mi < MB; ++mi)
#pragma unroll
      for (int ni = 0; ni < NB; ++ni) {
        const int r = I0 + wm * (BM / 2) + mi * 16 + (lane & 15);
        const int c = J0 + wn * (BN / 2) + ni * 16;
        if (has_c0) {
          T cv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) cv[v] = C0[(int64_t)(c + Mma<T>::row(lane, v)) * P.ldc0 + r];
#pragma unroll
          for (int v = 0; v < 4; ++v) D[(int64_t)(c + Mma<T>::row(lane, v)) * P.ldd + r] = sg * acc[mi][ni][v] + cv[v];
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) D[(int64_t)(c + Mma<T>::row(lane, v)) * P.ldd + r] = sg * acc[mi][ni][v];
        }
      }
    return;
  }
#pragma unroll
  for (int mi = 0; mi < MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < NB; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = I0 + wm * (BM / 2) + mi * 16 + (lane & 15);
        const int c = J0 + wn * (BN / 2) + ni * 16 + Mma<T>::row(lane, v);
        if (r < P.M && c < P.N && store_ok(fl, r, c)) {
          T val = sg * acc[mi][ni][v];
          if (has_c0) val += C0[(int64_t)c * P.ldc0 + r];
          D[(int64_t)c * P.ldd + r] = val;
        }
      }
}

// ------------------------------------------------------------------------
// bf16 MFMA (32x32x16, FP32 accumulation) on FP32-stored operands.  With
// SPLIT each FP32 operand x is written as hi + lo, hi = bf16(x),
// lo = bf16(x - hi), and the product is hi*hi + hi*lo + lo*hi (the lo*lo
// term lies below the FP32 rounding of the result).  The split is done once
// per element while the chunk is staged into LDS, in layout [row][k] with k
// contiguous, so each MFMA operand is one 16-byte LDS read.
//
// MFMA 32x32x16 bf16 lane layout (measured): operand X (32 x 16) lane l
// holds X[l%32][8(l/32) .. +8), operand Y (16 x 32) lane l holds
// Y[8(l/32) .. +8)[l%32]; accumulator register v of lane l is element
// (8(v/4) + 4(l/32) + v%4, l%32).
// ------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Epilogue of MB x NB accumulator blocks of 32 x 32: register v of lane l in
// block (mi, ni) is D(r0 + 32 mi + l % 32, c0 + 32 ni + 8 (v / 4) + 4 (l / 32) + v % 4),
// and D = C0 -/+ acc.  Whole tiles (full) load C0 in batches of 16.
template <int MB, int NB>
__device__ __forceinline__ void store_tile32(const GemmProb& P, const f32x16 (&acc)[MB][NB], int r0, int c0,
                                             int lane, bool full) {
  gptr<float> C0 = (gptr<float>)P.C0;
  gmut<float> D = (gmut<float>)P.D;
  const bool has_c0 = P.flags & G_C0;
  const float sg = (P.flags & G_NEG) ? -1.f : 1.f;
  if (full && !(P.flags & (G_D_UP | G_D_LO))) {
#pragma unroll
    for (int mi = 0; mi < MB; ++mi)
#pragma unroll
      for (int ni = 0; ni < NB; ++ni) {
        const int r = r0 + mi * 32 + (lane & 31);
        const int c = c0 + ni * 32 + 4 * (lane >> 5);
        if (has_c0) {
          float cv[16];
#pragma unroll
          for (int v = 0; v < 16; ++v) cv[v] = C0[(int64_t)(c + 8 * (v >> 2) + (v & 3)) * P.ldc0 + r];
#pragma unroll
          for (int v = 0; v < 16; ++v) D[(int64_t)(c + 8 * (v >> 2) + (v & 3)) * P.ldd + r] = sg * acc[mi][ni][v] + cv[v];
        } else {
#pragma unroll
          for (int v = 0; v < 16; ++v) D[(int64_t)(c + 8 * (v >> 2) + (v & 3)) * P.ldd + r] = sg * acc[mi][ni][v];
        }
      }
    return;
  }
#pragma unroll
  for (int mi = 0; mi < MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < NB; ++ni)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = r0 + mi * 32 + (lane & 31);
        const int c = c0 + ni * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (r < P.M && c < P.N && store_ok(P.flags, r, c)) {
          float val = sg * acc[mi][ni][v];
          if (has_c0) val += C0[(int64_t)c * P.ldc0 + r];
          D[(int64_t)c * P.ldd + r] = val;
        }
      }
}

template <bool SPLIT, int BM, int BN, int OCC = 1, int ST = 1, int BK = 32, int NW = 4>
__global__ __launch_bounds__(64 * NW, OCC) void k_gemm_bf16(const GemmProb* __restrict__ probs, int nprob,
                                                 const int32_t* __restrict__ order) {
  // NW waves in a 2 x NW/2 arrangement, wave tile BM/2 x 2BN/NW of 32 x 32 blocks
  constexpr int NT = 64 * NW;
  constexpr int LDK = BK + 8;
  constexpr int MB = BM / 64, NB = BN / (16 * NW);
  constexpr int NS = SPLIT ? 2 : 1;
  __shared__ __attribute__((aligned(16))) __bf16 As[ST][NS][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[ST][NS][BN][LDK];

  const int wg = order ? order[xcd_swizzle(blockIdx.x, gridDim.x)] : xcd_swizzle(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprob, wg)];
  const TileCoord tc = tile_of<BM, BN>(P, wg);
  const int I0 = tc.I0, J0 = tc.J0, kb = tc.kb, ke = tc.ke;
  const int fl = P.flags;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const float* __restrict__ A = (const float*)P.A;
  const float* __restrict__ B = (const float*)P.B;
  const bool a_lu = fl & G_A_MLU, a_up = fl & G_A_MUP, b_lu = fl & G_B_MLU, b_up = fl & G_B_MUP;
  const bool a_lo = fl & G_A_MLO, b_lo = fl & G_B_MLO;
  const bool a_edge = I0 + BM > P.M, b_edge = J0 + BN > P.N;

  f32x16 acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // A chunk BM x BK: thread -> 4 consecutive rows (a float4 per k) x AK k
  // (float4 loads along the contiguous row index).
  // B chunk BK x BN: thread -> one column, BKT consecutive k (float4 loads,
  // 16-byte LDS stores).
  constexpr int AROWG = BM / 4;
  constexpr int AK = BK * AROWG / NT;
  constexpr int BKT = BK * BN / NT;
  static_assert(AK >= 1 && BKT % 8 == 0, "chunk split");
  const int arg = tid % AROWG, akg = tid / AROWG;
  const int ar = I0 + 4 * arg;
  const int bn = tid % BN, bkg = tid / BN;
  const int bc = J0 + bn;
  const int arow_ld = min(ar, P.M - 4);
  const int bcol_ld = min(bc, P.N - 1);
  float4 ra[AK];
  float4 rb[BKT / 4];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < AK; ++i)
      ra[i] = gload4(A + (int64_t)(k0 + akg * AK + i) * P.lda + arow_ld);
    const float* bp = B + (int64_t)bcol_ld * P.ldb + k0 + bkg * BKT;
#pragma unroll
    for (int i = 0; i < BKT / 4; ++i) rb[i] = gload4(bp + 4 * i);
  };
  typedef __bf16 bfa __attribute__((ext_vector_type(AK)));
  // Stage one chunk into LDS as bf16 (hi, and lo = x - hi when split).  The
  // masked form applies the packed-triangle and edge masks; it is taken only
  // for chunks that cross a packed triangle's diagonal or the problem edge.
  auto store_chunk = [&](int st, int k0, bool am, bool bm) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ar + q;
      bfa h, l;
#pragma unroll
      for (int i = 0; i < AK; ++i) {
        float x = ra[i][q];
        if (am) x = select_op(x, r, k0 + akg * AK + i, a_lu, a_up, a_lo, P.M, 1 << 30);
        h[i] = (__bf16)x;
        if (SPLIT) l[i] = (__bf16)(x - (float)h[i]);
      }
      *(bfa*)&As[st][0][4 * arg + q][akg * AK] = h;
      if (SPLIT) *(bfa*)&As[st][NS - 1][4 * arg + q][akg * AK] = l;
    }
#pragma unroll
    for (int j = 0; j < BKT / 8; ++j) {
      bf16x8 h, l;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float x = rb[2 * j + e / 4][e % 4];
        if (bm) x = select_op(x, k0 + bkg * BKT + 8 * j + e, bc, b_lu, b_up, b_lo, 1 << 30, P.N);
        h[e] = (__bf16)x;
        if (SPLIT) l[e] = (__bf16)(x - (float)h[e]);
      }
      *(bf16x8*)&Bs[st][0][bn][bkg * BKT + 8 * j] = h;
      if (SPLIT) *(bf16x8*)&Bs[st][NS - 1][bn][bkg * BKT + 8 * j] = l;
    }
  };
  auto stage = [&](int st, int k0) __attribute__((always_inline)) {
    const bool am = a_edge || ((a_lu || a_up || a_lo) && k0 + BK > I0 && k0 < I0 + BM);
    const bool bm = b_edge || ((b_lu || b_up || b_lo) && k0 + BK > J0 && k0 < J0 + BN);
    if (am || bm) store_chunk(st, k0, am, bm);
    else store_chunk(st, k0, false, false);
  };
  auto compute = [&](int st) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int kk = ks * 16 + 8 * (lane >> 5);
      bf16x8 xh[NB], xl[NB], yh[MB], yl[MB];
#pragma unroll
      for (int ni = 0; ni < NB; ++ni) {
        const int n = wn * (2 * BN / NW) + ni * 32 + (lane & 31);
        xh[ni] = *(const bf16x8*)&Bs[st][0][n][kk];
        if (SPLIT) xl[ni] = *(const bf16x8*)&Bs[st][NS - 1][n][kk];
      }
#pragma unroll
      for (int mi = 0; mi < MB; ++mi) {
        const int m = wm * (BM / 2) + mi * 32 + (lane & 31);
        yh[mi] = *(const bf16x8*)&As[st][0][m][kk];
        if (SPLIT) yl[mi] = *(const bf16x8*)&As[st][NS - 1][m][kk];
      }
      // one term over every block before the next, so consecutive MFMAs
      // write different accumulators (small terms first)
      if (SPLIT) {
#pragma unroll
        for (int mi = 0; mi < MB; ++mi)
#pragma unroll
          for (int ni = 0; ni < NB; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[ni], yh[mi], acc[mi][ni], 0, 0, 0);
#pragma unroll
        for (int mi = 0; mi < MB; ++mi)
#pragma unroll
          for (int ni = 0; ni < NB; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ni], yl[mi], acc[mi][ni], 0, 0, 0);
      }
#pragma unroll
      for (int mi = 0; mi < MB; ++mi)
#pragma unroll
        for (int ni = 0; ni < NB; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ni], yh[mi], acc[mi][ni], 0, 0, 0);
    }
  };

  if (kb < ke) {
    if (ST == 2) {
      // two LDS stages: the next chunk is loaded before and staged after the
      // current chunk's products, one barrier per chunk
      load(kb);
      stage(0, kb);
      __syncthreads();
      int st = 0;
      for (int kcur = kb; kcur < ke; kcur += BK) {
        const bool more = kcur + BK < ke;
        if (more) load(kcur + BK);
        compute(st);
        if (more) stage(st ^ 1, kcur + BK);
        __syncthreads();
        st ^= 1;
      }
    } else {
      load(kb);
      for (int kcur = kb; kcur < ke; kcur += BK) {
        __syncthreads();             // previous chunk's LDS reads are done
        stage(0, kcur);
        __syncthreads();
        if (kcur + BK < ke) load(kcur + BK);
        compute(0);
      }
    }
  }

  store_tile32<MB, NB>(P, acc, I0 + wm * (BM / 2), J0 + wn * (2 * BN / NW), lane, !a_edge && !b_edge);
}


// ------------------------------------------------------------------------
// bf16 MFMA with the operands copied from global memory straight into LDS
// (global_load_lds_dwordx4: each lane's 16 bytes land at lane * 16 of the
// wave's 1 KiB destination), FP32 in LDS, split into hi/lo in registers as
// the fragments are read.  No VGPRs hold operands in flight and no staging
// pass stands between the loads and the products.
//
// LDS, two stages of a 32-deep K chunk:
//   A as [k][m] (m contiguous, as in global memory): one wave instruction
//     fills 256 / BM rows of k; a fragment (8 consecutive k of one row) is
//     eight 4-byte reads.
//   B as [n][k] (k contiguous): one wave instruction fills 8 columns; the
//     eight 16-byte slots of column n hold k pieces slot ^ (n & 7), so that
//     the 16-byte fragment reads of 8 consecutive columns hit distinct banks.
// Per chunk: one barrier (the chunk has landed, the other stage is free), the
// first 16-deep step's LDS reads, the DMA of the next chunk into the other
// stage, then the products.  Chunks crossing a packed triangle's diagonal get
// their masks applied in LDS first (one more barrier).  Rows beyond M and
// column groups beyond N load clamped in-range data: they only feed outputs
// that are not stored.  Same split and the same MFMA order per 16-deep step
// as k_gemm_bf16, so the results are bitwise the same.
// ------------------------------------------------------------------------
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) void* dma_src_t;
typedef __attribute__((address_space(3))) void* dma_dst_t;

// hi = bf16(x), lo = bf16(x - hi) for 8 values, converted two at a time
template <bool SPLIT>
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& h, bf16x8& l) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const f32x2 v = {x[e], x[e + 1]};
    const bf16x2 hv = __builtin_convertvector(v, bf16x2);
    h[e] = hv[0];
    h[e + 1] = hv[1];
    if (SPLIT) {
      const f32x2 r = {x[e] - (float)hv[0], x[e + 1] - (float)hv[1]};
      const bf16x2 lv = __builtin_convertvector(r, bf16x2);
      l[e] = lv[0];
      l[e + 1] = lv[1];
    }
  }
}

// One K chunk of k_gemm_dl.  The LDS pointers are restrict: the compiler then
// sees that the reads of the current stage (ca, cb) do not alias the DMA into
// the next stage (na, nb), and does not make them wait for it.
template <bool SPLIT, int BM, int BN, int NW>
__device__ __forceinline__ void dl_chunk(const float* __restrict__ ca, const float* __restrict__ cb,
                                         float* __restrict__ na, float* __restrict__ nb,
                                         const char* __restrict__ ga, const char* __restrict__ gb,
                                         const int64_t (&goff)[16], bool issue_next, int lane, int wm, int wn,
                                         f32x16 (&acc)[BM / 64][BN / (16 * NW)]) {
  constexpr int BK = 32;
  constexpr int MB = BM / 64, NB = BN / (16 * NW);
  constexpr int NA = BK * BM / 256 / NW, NBI = BN / 8 / NW;
  auto read = [&](int ks, float (&xb)[NB][8], float (&xa)[MB][8]) __attribute__((always_inline)) {
    const int kk = ks * 16 + 8 * (lane >> 5);
#pragma unroll
    for (int ni = 0; ni < NB; ++ni) {
      const int n = wn * (2 * BN / NW) + ni * 32 + (lane & 31);
      const int s0 = (kk >> 2) ^ (n & 7), s1 = ((kk >> 2) + 1) ^ (n & 7);
      const f32x4 v0 = *(const f32x4*)&cb[n * BK + 4 * s0];
      const f32x4 v1 = *(const f32x4*)&cb[n * BK + 4 * s1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xb[ni][e] = v0[e];
        xb[ni][e + 4] = v1[e];
      }
    }
#pragma unroll
    for (int mi = 0; mi < MB; ++mi) {
      const int m = wm * (BM / 2) + mi * 32 + (lane & 31);
#pragma unroll
      for (int e = 0; e < 8; ++e) xa[mi][e] = ca[(kk + e) * BM + m];
    }
  };
  auto mult = [&](const float (&xb)[NB][8], const float (&xa)[MB][8]) __attribute__((always_inline)) {
    bf16x8 xh[NB], xl[NB];
#pragma unroll
    for (int ni = 0; ni < NB; ++ni) split8<SPLIT>(xb[ni], xh[ni], xl[ni]);
#pragma unroll
    for (int mi = 0; mi < MB; ++mi) {
      bf16x8 yh, yl;
      split8<SPLIT>(xa[mi], yh, yl);
      if (SPLIT) {
#pragma unroll
        for (int ni = 0; ni < NB; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[ni], yh, acc[mi][ni], 0, 0, 0);
#pragma unroll
        for (int ni = 0; ni < NB; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ni], yl, acc[mi][ni], 0, 0, 0);
      }
#pragma unroll
      for (int ni = 0; ni < NB; ++ni)
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[ni], yh, acc[mi][ni], 0, 0, 0);
    }
  };
  float xb[NB][8], xa[MB][8];
  read(0, xb, xa);
  __builtin_amdgcn_sched_barrier(0);
  if (issue_next) {
#pragma unroll
    for (int q = 0; q < NA; ++q)
      __builtin_amdgcn_global_load_lds((dma_src_t)(ga + goff[q]), (dma_dst_t)(na + q * 256), 16, 0, 0);
#pragma unroll
    for (int q = 0; q < NBI; ++q)
      __builtin_amdgcn_global_load_lds((dma_src_t)(gb + goff[NA + q]), (dma_dst_t)(nb + q * 256), 16, 0, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
  mult(xb, xa);
#pragma unroll
  for (int ks = 1; ks < BK / 16; ++ks) {
    __builtin_amdgcn_sched_barrier(0);
    read(ks, xb, xa);
    mult(xb, xa);
  }
}

template <bool SPLIT, int BM, int BN, int NW, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void k_gemm_dl(const GemmProb* __restrict__ probs, int nprob,
                                                 const int32_t* __restrict__ order) {
  constexpr int BK = 32;
  constexpr int MB = BM / 64, NB = BN / (16 * NW);
  constexpr int NA = BK * BM / 256 / NW;   // A instructions per wave and chunk
  constexpr int NBI = BN / 8 / NW;         // B instructions per wave and chunk
  constexpr int KPI = BM >= 256 ? 1 : 256 / BM;   // k rows per A instruction
  static_assert(BM <= 256 && NA >= 1 && NBI >= 1 && NA + NBI <= 16 && (BK * BM) % (256 * NW) == 0 &&
                    BN % (8 * NW) == 0 && NB >= 1,
                "chunk split");
  __shared__ __attribute__((aligned(16))) float As[2][BK * BM];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN * BK];

  const int wg = order ? order[xcd_swizzle(blockIdx.x, gridDim.x)] : xcd_swizzle(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprob, wg)];
  const TileCoord tc = tile_of<BM, BN>(P, wg);
  const int I0 = tc.I0, J0 = tc.J0, kb = tc.kb, ke = tc.ke;
  const int fl = P.flags;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const char* A = (const char*)P.A;
  const char* B = (const char*)P.B;
  const bool a_lu = fl & G_A_MLU, a_up = fl & G_A_MUP, b_lu = fl & G_B_MLU, b_up = fl & G_B_MUP;
  const bool a_lo = fl & G_A_MLO, b_lo = fl & G_B_MLO;

  f32x16 acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // byte offsets of this lane's 16-byte pieces: a wave-uniform part per
  // instruction and one per-lane part for A and one for B
  const int64_t a_lane =
      ((int64_t)((lane * 4) / BM) * P.lda + min(I0 + (lane * 4) % BM, P.M - 4)) * 4;
  const int64_t b_lane = ((int64_t)(lane >> 3) * P.ldb + 4 * ((lane & 7) ^ ((lane >> 3) & 7))) * 4;
  auto a_off = [&](int k, int q) __attribute__((always_inline)) {
    return (int64_t)(k + (wave * NA + q) * KPI) * P.lda * 4 + a_lane;
  };
  auto b_off = [&](int k, int q) __attribute__((always_inline)) {
    return ((int64_t)min(J0 + 8 * (wave * NBI + q), P.N - 8) * P.ldb + k) * 4 + b_lane;
  };

  if (kb < ke) {
#pragma unroll
    for (int q = 0; q < NA; ++q)
      __builtin_amdgcn_global_load_lds((dma_src_t)(A + a_off(kb, q)), (dma_dst_t)&As[0][(wave * NA + q) * 256], 16,
                                       0, 0);
#pragma unroll
    for (int q = 0; q < NBI; ++q)
      __builtin_amdgcn_global_load_lds((dma_src_t)(B + b_off(kb, q)), (dma_dst_t)&Bs[0][(wave * NBI + q) * 256], 16,
                                       0, 0);
    int st = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      __syncthreads();   // chunk k0 has landed; every wave is done with the other stage
      const bool am = (a_lu || a_up || a_lo) && k0 + BK > I0 && k0 < I0 + BM;
      const bool bm = (b_lu || b_up || b_lo) && k0 + BK > J0 && k0 < J0 + BN;
      if (am || bm) {
        if (am)
          for (int i = tid; i < BK * BM; i += 64 * NW) {
            const int k = i / BM, m = i % BM;
            As[st][i] = select_op(As[st][i], I0 + m, k0 + k, a_lu, a_up, a_lo, 1 << 30, 1 << 30);
          }
        if (bm)
          for (int i = tid; i < BN * BK; i += 64 * NW) {
            const int n = i / BK, k = 4 * (((i % BK) >> 2) ^ (n & 7)) + (i & 3);
            Bs[st][i] = select_op(Bs[st][i], k0 + k, J0 + n, b_lu, b_up, b_lo, 1 << 30, 1 << 30);
          }
        __syncthreads();
      }
      const int k1 = k0 + BK;
      int64_t goff[16];
#pragma unroll
      for (int q = 0; q < NA; ++q) goff[q] = a_off(k1, q);
#pragma unroll
      for (int q = 0; q < NBI; ++q) goff[NA + q] = b_off(k1, q);
      dl_chunk<SPLIT, BM, BN, NW>(As[st], Bs[st], &As[st ^ 1][wave * NA * 256], &Bs[st ^ 1][wave * NBI * 256], A, B,
                                  goff, k1 < ke, lane, wm, wn, acc);
      st ^= 1;
    }
  }
  store_tile32<MB, NB>(P, acc, I0 + wm * (BM / 2), J0 + wn * (2 * BN / NW), lane,
                       I0 + BM <= P.M && J0 + BN <= P.N);
}

// mode: 0 = 64 x 64 tiles, 1 = 128 x 128 tiles, 2 = 256 x 128 tiles (bf16 only),
// 3 = 128 x 128 tiles with direct LDS loads (bf16 only; otherwise as 1),
// 4 = 256 x 256 tiles on 8 waves with direct LDS loads (bf16 only; otherwise as 1)
void launch_gemm(int dtype, int mode, const GemmProb* probs, int nprob, int nwg, hipStream_t s,
                 const int32_t* order) {
  if (nwg <= 0 || nprob <= 0) return;
  const dim3 g(nwg), b(256);
  // two workgroups per CU (two waves per SIMD) measured best for f64/f32
  if (dtype <= 1) {
    if (mode >= 1) {
      if (dtype == 0) hipLaunchKernelGGL((k_gemm_std<double, 128, 128, 16, 2>), g, b, 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_std<float, 128, 128, 16, 2>), g, b, 0, s, probs, nprob, order);
    } else {
      if (dtype == 0) hipLaunchKernelGGL((k_gemm_std<double, 64, 64, 16, 2>), g, b, 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_std<float, 64, 64, 16, 2>), g, b, 0, s, probs, nprob, order);
    }
    return;
  }
  const bool split = dtype == 2;
  switch (mode) {
    case 4:
      if (split) hipLaunchKernelGGL((k_gemm_dl<true, 256, 256, 8, 1>), g, dim3(512), 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_dl<false, 256, 256, 8, 1>), g, dim3(512), 0, s, probs, nprob, order);
      break;
    case 3:
      if (split) hipLaunchKernelGGL((k_gemm_dl<true, 128, 128, 4, 2>), g, b, 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_dl<false, 128, 128, 4, 2>), g, b, 0, s, probs, nprob, order);
      break;
    case 2:
      if (split) hipLaunchKernelGGL((k_gemm_bf16<true, 256, 128, 1, 2>), g, b, 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_bf16<false, 256, 128, 1, 2>), g, b, 0, s, probs, nprob, order);
      break;
    case 1:
      if (split) hipLaunchKernelGGL((k_gemm_bf16<true, 128, 128, 2>), g, b, 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_bf16<false, 128, 128, 2>), g, b, 0, s, probs, nprob, order);
      break;
    default:
      if (split) hipLaunchKernelGGL((k_gemm_bf16<true, 64, 64, 2>), g, b, 0, s, probs, nprob, order);
      else hipLaunchKernelGGL((k_gemm_bf16<false, 64, 64, 2>), g, b, 0, s, probs, nprob, order);
      break;
  }
}

// tile edge (rows, columns) of a launch mode
void gemm_tile_shape(int dtype, int mode, int* bm, int* bn) {
  if (mode == 4 && dtype >= 2) { *bm = 256; *bn = 256; }
  else if (mode == 2 && dtype >= 2) { *bm = 256; *bn = 128; }
  else if (mode >= 1) { *bm = 128; *bn = 128; }
  else { *bm = 64; *bn = 64; }
}

}  // namespace ddps
