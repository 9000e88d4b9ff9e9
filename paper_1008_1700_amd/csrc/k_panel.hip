// Diagonal sub-tile kernel of the tile LU: for each problem, one wave (64
// threads) factors a 64 x 64 sub-tile without pivoting (A = L U, L unit
// lower), then inverts both triangles and writes back L^{-1} strictly below
// the diagonal and U^{-1} on and above it.
//
// The kernel runs once per wave and is latency bound, so its code is kept
// small: a fully unrolled 64 x 64 elimination and inversion is tens of
// thousands of instructions, and a single wave then waits on instruction
// fetch more than on arithmetic.  Every phase here is a short loop over
// 16-column blocks whose body is unrolled.
//
// Elimination.  Lane r owns row r in registers, a[c] = A(r, j0 + c) for the
// current block start j0.  Step k reads row k of U from lane k's registers
// (v_readlane, lane index k uniform), lane r > k forms its multiplier
// l = a(r,k) / u(k,k) and updates the rest of its row.  After 16 steps the
// block's 16 finished columns go to LDS (row-major, L below the diagonal, U
// on and above it) and the row is shifted left by 16 registers.  The first
// two blocks run a 64-wide body, the last two a 32-wide one.
//
// Inversion, one 16-column block at a time, with the lane's own row of the
// inverse in registers and the earlier blocks' rows in LDS:
//   Y = U^{-1}, blocks left to right:
//       Y(r,r) = 1/u(r,r),  Y(r,j) = -( sum_{r<=l<j} Y(r,l) U(l,j) ) / u(j,j),  j > r
//   X = L^{-1}, blocks right to left (unit diagonal implied, not stored):
//       X(r,j) = -( L(r,j) + sum_{j<l<r} X(r,l) L(l,j) ),  j < r
// Entries outside each triangle are held at zero so that every sum runs over
// its whole range without conditions.
//
// Pivot check, after the elimination: lane r tests its own pivot u_rr
// against thresh[row] (the row's threshold in the padded layout); a pivot at
// or below it, or not finite, records (block, global row) in *bad through an
// atomic minimum, so the first bad pivot in (block, row) order is reported.
#include "ddps_internal.h"

namespace ddps {

namespace {

constexpr int kN = kTile;      // 64
constexpr int kB = 16;         // column block
constexpr int kLdLU = kN + 4;  // row-major LU: 16-byte aligned 16-column pieces
constexpr int kLdR = kN + 1;   // per-lane rows: conflict-free column access

// value of x in lane `lane` (wave-uniform), broadcast to the wave
__device__ __forceinline__ float lane_value(float x, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}
__device__ __forceinline__ double lane_value(double x, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// 16 elimination steps k = j0 .. j0+15 on the live registers a[0, W);
// a[c] holds column j0 + c.  Stores the 16 finished columns of the lane's row
// to LU and 1/u(k,k) to Rv, then shifts the row left by 16.
template <typename T, int W>
__device__ __forceinline__ void elim_block(T (&a)[kN], int r, int j0, T (*LU)[kLdLU], T* Rv) {
#pragma unroll
  for (int kk = 0; kk < kB; ++kk) {
    const int k = j0 + kk;
    const T rp = T(1) / lane_value(a[kk], k);
    if (r == 0) Rv[k] = rp;
    // rows at or above the pivot take multiplier 0 (their entries are final)
    const T l = r > k ? a[kk] * rp : T(0);
    a[kk] = r > k ? l : a[kk];
#pragma unroll
    for (int c = kk + 1; c < W; ++c) a[c] -= l * lane_value(a[c], k);
  }
#pragma unroll
  for (int c = 0; c < kB; ++c) LU[r][j0 + c] = a[c];
#pragma unroll
  for (int c = 0; c + kB < W; ++c) a[c] = a[c + kB];
#pragma unroll
  for (int c = W - kB; c < W; ++c) a[c] = T(0);
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(64) void k_panel(const PanelProb* __restrict__ probs,
                                              const double* __restrict__ thresh,
                                              unsigned long long* __restrict__ bad) {
  __shared__ __attribute__((aligned(16))) T LU[kN][kLdLU];  // L (c < r) and U (c >= r), row-major
  __shared__ T Wr[kN][kLdR];                               // rows of U^{-1}, then of L^{-1}
  __shared__ T Rv[kN];                                     // 1 / u(k, k)
  const PanelProb P = probs[blockIdx.x];
  T* __restrict__ D = (T*)P.D;
  const int r = threadIdx.x;
  const int64_t ld = P.ld;

  T a[kN];
#pragma unroll
  for (int c = 0; c < kN; ++c) a[c] = D[c * ld + r];
  const double th = thresh[P.vrow0 + r];   // pivot threshold of this lane's row

#pragma unroll 1
  for (int j0 = 0; j0 < 2 * kB; j0 += kB) elim_block<T, kN>(a, r, j0, LU, Rv);
#pragma unroll 1
  for (int j0 = 2 * kB; j0 < kN; j0 += kB) elim_block<T, kN / 2>(a, r, j0, LU, Rv);
  __syncthreads();

  {
    const double av = fabs((double)LU[r][r]);
    if (!(av > th) || !(av <= 1.7e308))
      atomicMin(bad, ((unsigned long long)P.block << 40) | (unsigned long long)(P.row0 + r));
  }

  // Y = U^{-1}, 16-column blocks left to right
#pragma unroll 1
  for (int j0 = 0; j0 < kN; j0 += kB) {
    T acc[kB];
#pragma unroll
    for (int jj = 0; jj < kB; ++jj) acc[jj] = T(0);
    // earlier columns: Y(r, l) for l < j0 from LDS (zero for l < r)
#pragma unroll 4
    for (int l = 0; l < j0; ++l) {
      const T yl = Wr[r][l];
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) acc[jj] += yl * LU[l][j0 + jj];
    }
    T y[kB];
#pragma unroll
    for (int jj = 0; jj < kB; ++jj) {
      const int j = j0 + jj;
      T s = acc[jj];
#pragma unroll
      for (int ll = 0; ll < jj; ++ll) s += y[ll] * LU[j0 + ll][j];
      const T rv = Rv[j];
      y[jj] = j < r ? T(0) : (j == r ? rv : -s * rv);
    }
#pragma unroll
    for (int jj = 0; jj < kB; ++jj) Wr[r][j0 + jj] = y[jj];
  }
  // U^{-1} goes out now (on and above the diagonal); Wr then holds L^{-1}
#pragma unroll 4
  for (int c = 0; c < kN; ++c)
    if (c >= r) D[c * ld + r] = Wr[r][c];

  // X = L^{-1}, 16-column blocks right to left
#pragma unroll 1
  for (int j0 = kN - kB; j0 >= 0; j0 -= kB) {
    T acc[kB];
#pragma unroll
    for (int jj = 0; jj < kB; ++jj) acc[jj] = j0 + jj < r ? LU[r][j0 + jj] : T(0);
    // later columns: X(r, l) for l >= j0 + 16 from LDS (zero for l >= r)
#pragma unroll 4
    for (int l = j0 + kB; l < kN; ++l) {
      const T xl = Wr[r][l];
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) acc[jj] += xl * LU[l][j0 + jj];
    }
    T x[kB];
#pragma unroll
    for (int jj = kB - 1; jj >= 0; --jj) {
      const int j = j0 + jj;
      T s = acc[jj];
#pragma unroll
      for (int ll = jj + 1; ll < kB; ++ll) s += x[ll] * LU[j0 + ll][j];
      x[jj] = j < r ? -s : T(0);
    }
#pragma unroll
    for (int jj = 0; jj < kB; ++jj) Wr[r][j0 + jj] = x[jj];
  }
#pragma unroll 4
  for (int c = 0; c < kN; ++c)
    if (c < r) D[c * ld + r] = Wr[r][c];
}

void launch_panel(int dtype, const PanelProb* probs, int nprob, const double* thresh,
                  unsigned long long* bad, hipStream_t s) {
  if (nprob <= 0) return;
  if (dtype == 0)
    hipLaunchKernelGGL(k_panel<double>, dim3(nprob), dim3(64), 0, s, probs, thresh, bad);
  else
    hipLaunchKernelGGL(k_panel<float>, dim3(nprob), dim3(64), 0, s, probs, thresh, bad);
}

}  // namespace ddps
