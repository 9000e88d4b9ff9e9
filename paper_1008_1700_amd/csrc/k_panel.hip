// Diagonal sub-tile kernel of the blocked block-LU: for each problem, one
// workgroup loads a 64 x 64 sub-tile into LDS, factors it without pivoting
// (A = L U, L unit lower), then inverts both triangles and writes back
// L^{-1} strictly below the diagonal and U^{-1} on and above it.
//
// Pivot check: a pivot u_kk with |u_kk| <= thresh[block] (or not finite)
// records (block, global row) in *bad through an atomic minimum, so the
// first bad pivot in (block, row) order is reported.
#include "ddps_internal.h"

namespace ddps {

template <typename T>
__global__ __launch_bounds__(256) void k_panel(const PanelProb* __restrict__ probs,
                                               const double* __restrict__ thresh,
                                               unsigned long long* __restrict__ bad) {
  constexpr int N = kTile, LD = kTile + 1;
  __shared__ T S[N][LD];   // S[row][col]
  __shared__ T X[N][LD];   // inverses: X[r][c], r > c from L^{-1}, r <= c from U^{-1}
  const PanelProb P = probs[blockIdx.x];
  T* __restrict__ D = (T*)P.D;
  const int tid = threadIdx.x;
  for (int e = tid; e < N * N; e += 256) {
    const int r = e & (N - 1), c = e >> 6;
    S[r][c] = D[(int64_t)c * P.ld + r];
  }
  __syncthreads();
  const double th = thresh[P.block];
  for (int k = 0; k < N; ++k) {
    const T piv = S[k][k];
    if (tid == 0) {
      const double a = fabs((double)piv);
      if (!(a > th) || !(a <= 1.7e308)) {
        const unsigned long long key =
            ((unsigned long long)P.block << 40) | (unsigned long long)(P.row0 + k);
        atomicMin(bad, key);
      }
    }
    if (tid > k && tid < N) S[tid][k] = S[tid][k] / piv;
    __syncthreads();
    const int m = N - 1 - k;
    for (int e = tid; e < m * m; e += 256) {
      const int r = k + 1 + e % m, c = k + 1 + e / m;
      S[r][c] -= S[r][k] * S[k][c];
    }
    __syncthreads();
  }
  // Wave 0: column c of L^{-1} (forward substitution, unit diagonal implied).
  // Wave 1: column c of U^{-1} (back substitution).
  if (tid < N) {
    const int c = tid;
    for (int r = c + 1; r < N; ++r) {
      T s = S[r][c];
      for (int l = c + 1; l < r; ++l) s += S[r][l] * X[l][c];
      X[r][c] = -s;
    }
  } else if (tid < 2 * N) {
    const int c = tid - N;
    X[c][c] = T(1) / S[c][c];
    for (int r = c - 1; r >= 0; --r) {
      T s = T(0);
      for (int l = r + 1; l <= c; ++l) s += S[r][l] * X[l][c];
      X[r][c] = -s / S[r][r];
    }
  }
  __syncthreads();
  for (int e = tid; e < N * N; e += 256) {
    const int r = e & (N - 1), c = e >> 6;
    D[(int64_t)c * P.ld + r] = X[r][c];
  }
}

void launch_panel(int dtype, const PanelProb* probs, int nprob, const double* thresh,
                  unsigned long long* bad, hipStream_t s) {
  if (nprob <= 0) return;
  if (dtype == 0)
    hipLaunchKernelGGL(k_panel<double>, dim3(nprob), dim3(256), 0, s, probs, thresh, bad);
  else
    hipLaunchKernelGGL(k_panel<float>, dim3(nprob), dim3(256), 0, s, probs, thresh, bad);
}

}  // namespace ddps
