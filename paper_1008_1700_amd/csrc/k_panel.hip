// Diagonal sub-tile kernel of the tile LU: for each problem, one wave (64
// threads) factors a 64 x 64 sub-tile without pivoting (A = L U, L unit
// lower), then inverts both triangles in place and writes back L^{-1}
// strictly below the diagonal and U^{-1} on and above it.
//
// Lane r owns row r of the sub-tile in registers.  Elimination step k: lane
// k publishes row k of U in LDS, every lane r > k forms its multiplier
// l = a(r,k) / u(k,k) (kept in place, and saved in LDS as column k of L),
// and updates its row.  A single wave needs no cross-wave barrier between
// steps (the LDS operations of one wave complete in order); with four waves
// the two barriers per step dominated this latency-bound kernel.
//
// Inversion, all in the lane's own row (no communication), using the saved
// L columns and U rows:
//   X = L^{-1}, columns j from right to left:
//       X(r,j) = -( L(r,j) + sum_{j<l<r} X(r,l) L(l,j) )
//   Y = U^{-1}, columns j from left to right:
//       Y(j,j) = 1/u(j,j);  Y(r,j) = -( sum_{r<=l<j} Y(r,l) U(l,j) ) / u(j,j)
// (the Y sums read Y(r,l) for l < j, already final since columns go left to
// right; the X sums read X(r,l) for l > j, final since columns go right to
// left; both read the factors from LDS, never from other lanes).
//
// Pivot check: a pivot u_kk with |u_kk| <= thresh[row] (the row's own
// threshold in the padded layout) or not finite records (block, global row)
// in *bad through an atomic minimum, so the first bad pivot in (block, row)
// order is reported.
#include "ddps_internal.h"

namespace ddps {

template <typename T>
__global__ __launch_bounds__(64) void k_panel(const PanelProb* __restrict__ probs,
                                              const double* __restrict__ thresh,
                                              unsigned long long* __restrict__ bad) {
  constexpr int N = kTile, LD = kTile + 4;
  __shared__ __attribute__((aligned(16))) T Ur[N][LD];   // Ur[k][c] = U(k, c), c >= k
  __shared__ __attribute__((aligned(16))) T Lc[N][LD];   // Lc[k][r] = L(r, k), r > k
  const PanelProb P = probs[blockIdx.x];
  T* __restrict__ D = (T*)P.D;
  const int r = threadIdx.x;
  T a[N];
#pragma unroll
  for (int c = 0; c < N; ++c) a[c] = D[(int64_t)c * P.ld + r];
  const double th = thresh[P.vrow0 + r];   // pivot threshold of this lane's row

  // Every loop is fully unrolled: register indices are compile-time
  // constants and the triangular loop bounds prune at compile time.
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (r == k) {
#pragma unroll
      for (int c = k; c < N; ++c) Ur[k][c] = a[c];
      const double av = fabs((double)a[k]);
      if (!(av > th) || !(av <= 1.7e308)) {
        const unsigned long long key =
            ((unsigned long long)P.block << 40) | (unsigned long long)(P.row0 + k);
        atomicMin(bad, key);
      }
    }
    __syncthreads();   // a single wave: orders the LDS accesses only
    const T piv = Ur[k][k];
    if (r > k) {
      const T l = a[k] / piv;
      Lc[k][r] = l;
      a[k] = l;
#pragma unroll
      for (int c = k + 1; c < N; ++c) a[c] -= l * Ur[k][c];
    }
  }
  __syncthreads();

  // X = L^{-1} in the strictly lower part, columns right to left
#pragma unroll
  for (int j = N - 2; j >= 0; --j) {
    if (r > j) {
      T acc = a[j];
#pragma unroll
      for (int l = j + 1; l < N - 1; ++l)
        if (l < r) acc += a[l] * Lc[j][l];
      a[j] = -acc;
    }
  }
  // Y = U^{-1} in the upper part, columns left to right
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const T d = T(1) / Ur[j][j];
    if (r < j) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < j; ++l)
        if (l >= r) acc += a[l] * Ur[l][j];
      a[j] = -acc * d;
    } else if (r == j) {
      a[j] = d;
    }
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
