// Diagonal sub-tile kernel of the tile LU: for each problem, one wave (64
// threads) factors a 64 x 64 sub-tile without pivoting (A = L U, L unit
// lower), then inverts both triangles in place and writes back L^{-1}
// strictly below the diagonal and U^{-1} on and above it.
//
// Lane r owns row r of the sub-tile in registers.  Elimination step k:
// every lane reads row k of U from lane k (a register broadcast), lane r > k
// forms its multiplier l = a(r,k) * (1/u(k,k)) (kept in place, and saved in
// LDS as column k of L), and updates its row.  A single wave needs no cross-wave barrier between
// steps (the LDS operations of one wave complete in order); with four waves
// the two barriers per step dominated this latency-bound kernel.
//
// Inversion, all in the lane's own row, with the factors read from LDS
// (Ur: rows of U, Lc: columns of L) and no per-element conditions: lane r
// zeroes the entries of its row outside the triangle being inverted, so
// every sum can run over the whole row.
//   Y = U^{-1}, columns j left to right (entries l < r held at zero):
//       Y(r,r) = 1/u(r,r);  Y(r,j) = -( sum_{l<j} Y(r,l) U(l,j) ) / u(j,j)
//   the Y row is parked in Ur[r][.] (after every lane has read U), then
//   X = L^{-1}, columns j right to left (entries l >= r held at zero):
//       X(r,j) = -( L(r,j) + sum_{l>j} X(r,l) L(l,j) )
// and the row written back is X left of the diagonal, Y from it on.
//
// Pivot check, after the elimination: lane r tests its own pivot u_rr
// against thresh[row] (the row's threshold in the padded layout); a pivot at
// or below it, or not finite, records (block, global row) in *bad through an
// atomic minimum, so the first bad pivot in (block, row) order is reported.
#include "ddps_internal.h"

namespace ddps {

// value of x in lane `lane` (a compile-time constant), broadcast to the wave
__device__ __forceinline__ float lane_value(float x, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}
__device__ __forceinline__ double lane_value(double x, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T>
__global__ __launch_bounds__(64) void k_panel(const PanelProb* __restrict__ probs,
                                              const double* __restrict__ thresh,
                                              unsigned long long* __restrict__ bad) {
  constexpr int N = kTile, LD = kTile + 4;
  __shared__ __attribute__((aligned(16))) T Ur[N][LD];   // Ur[k][c] = U(k, c), c >= k
  __shared__ __attribute__((aligned(16))) T Lc[N][LD];   // Lc[k][r] = L(r, k), r > k
  __shared__ T Rv[N];                                     // Rv[k] = 1 / u(k, k)
  const PanelProb P = probs[blockIdx.x];
  T* __restrict__ D = (T*)P.D;
  const int r = threadIdx.x;
  T a[N];
#pragma unroll
  for (int c = 0; c < N; ++c) a[c] = D[(int64_t)c * P.ld + r];
  const double th = thresh[P.vrow0 + r];   // pivot threshold of this lane's row

  // Every loop is fully unrolled: register indices are compile-time
  // constants and the triangular loop bounds prune at compile time.  Step
  // k reads row k of U straight from lane k's registers (v_readlane into
  // scalars), so the elimination chain has no LDS round trip.
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const T rp = T(1) / lane_value(a[k], k);
    if (r == 0) Rv[k] = rp;
    // branch-free update: rows at or above the pivot take multiplier 0
    // (their entries are final; only a singular tile can turn them NaN,
    // after its first bad pivot, which is what gets reported)
    const T l = r > k ? a[k] * rp : T(0);
    Lc[k][r] = l;
    a[k] = r > k ? l : a[k];
#pragma unroll
    for (int c = k + 1; c < N; ++c) a[c] -= l * lane_value(a[c], k);
  }
  // rows of U for the inversion (entries left of the diagonal are not read)
#pragma unroll
  for (int c = 0; c < N; ++c) Ur[r][c] = a[c];
  __syncthreads();
  {
    T piv = a[0];
#pragma unroll
    for (int c = 1; c < N; ++c)
      if (c == r) piv = a[c];
    const double av = fabs((double)piv);
    if (!(av > th) || !(av <= 1.7e308))
      atomicMin(bad, ((unsigned long long)P.block << 40) | (unsigned long long)(P.row0 + r));
  }

  // Y = U^{-1}: zero the L part, then columns left to right
#pragma unroll
  for (int l = 0; l < N; ++l) a[l] = l < r ? T(0) : a[l];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T acc0 = T(0), acc1 = T(0), acc2 = T(0), acc3 = T(0);
#pragma unroll
    for (int l = 0; l + 3 < j; l += 4) {
      acc0 += a[l] * Ur[l][j];
      acc1 += a[l + 1] * Ur[l + 1][j];
      acc2 += a[l + 2] * Ur[l + 2][j];
      acc3 += a[l + 3] * Ur[l + 3][j];
    }
#pragma unroll
    for (int l = j & ~3; l < j; ++l) acc0 += a[l] * Ur[l][j];
    const T acc = (acc0 + acc1) + (acc2 + acc3);
    const T yj = j == r ? Rv[j] : -acc * Rv[j];
    a[j] = j < r ? T(0) : yj;
  }
  __syncthreads();   // every lane is done reading U
#pragma unroll
  for (int c = 0; c < N; ++c) Ur[r][c] = a[c];
  // X = L^{-1}: the lane's L row (unit diagonal implied), zero from the diagonal on
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const T v = Lc[l][r];   // every entry of Lc was written (0 on and above the diagonal)
    a[l] = l < r ? v : T(0);
  }
#pragma unroll
  for (int j = N - 2; j >= 0; --j) {
    T acc0 = a[j], acc1 = T(0), acc2 = T(0), acc3 = T(0);
#pragma unroll
    for (int l = j + 1; l + 3 < N; l += 4) {
      acc0 += a[l] * Lc[j][l];
      acc1 += a[l + 1] * Lc[j][l + 1];
      acc2 += a[l + 2] * Lc[j][l + 2];
      acc3 += a[l + 3] * Lc[j][l + 3];
    }
#pragma unroll
    for (int l = j + 1 + ((N - j - 1) & ~3); l < N; ++l) acc0 += a[l] * Lc[j][l];
    const T acc = (acc0 + acc1) + (acc2 + acc3);
    a[j] = j < r ? -acc : T(0);
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const T u = Ur[r][c];
    a[c] = c < r ? a[c] : u;
  }
#pragma unroll
  for (int c = 0; c < N; ++c) D[(int64_t)c * P.ld + r] = a[c];
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
