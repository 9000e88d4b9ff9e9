// Diagonal sub-tile kernel of the tile LU: for each problem, one workgroup of
// four waves factors a 64 x 64 sub-tile without pivoting (A = L U, L unit
// lower), then inverts both triangles and writes back L^{-1} strictly below
// the diagonal and U^{-1} on and above it.
//
// The kernel is latency bound (a few of them run at a time, one per block of
// the partition), so the work of one sub-tile is spread over four waves.
//
// Elimination.  Wave w owns columns 16w .. 16w+15: lane r holds
// a[c] = A(r, 16w + c) in registers.  In round b the wave owning columns
// 16b .. 16b+15 runs their 16 elimination steps k: it reads the pivot u(k,k)
// from lane k (v_readlane), forms the multipliers l(r) = a(r,k) / u(k,k) for
// r > k, keeps them as column k of L, updates its own columns right of k and
// puts the multipliers in LDS.  After one barrier every wave right of it
// applies the same 16 steps to its columns, a(r,c) -= l(r) a(k,c), with the
// pivot row read from lane k of its own registers.  The multipliers of
// consecutive rounds alternate between two LDS buffers.  The operations and
// their order per entry are those of a one-wave elimination, so the factors
// do not depend on the split.
//
// Inversion, with the factors in LDS (row-major, L below the diagonal, U on
// and above it); wave 0 forms Y = U^{-1} and wave 1 X = L^{-1} at the same
// time, each with lane r computing row r one 16-column block at a time and
// the earlier blocks' rows in LDS:
//   Y = U^{-1}, blocks left to right:
//       Y(r,r) = 1/u(r,r),  Y(r,j) = -( sum_{r<=l<j} Y(r,l) U(l,j) ) / u(j,j),  j > r
//   X = L^{-1}, blocks right to left (unit diagonal implied, not stored):
//       X(r,j) = -( L(r,j) + sum_{j<l<r} X(r,l) L(l,j) ),  j < r
// Entries outside each triangle are held at zero so that every sum runs over
// its whole range without conditions.
//
// Pivot check, after the elimination: lane r of wave 2 tests u_rr against
// thresh[row] (the row's threshold in the padded layout); a pivot at or below
// it, or not finite, records (block, global row) in *bad through an atomic
// minimum, so the first bad pivot in (block, row) order is reported.
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

}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_panel(const PanelProb* __restrict__ probs,
                                               const double* __restrict__ thresh,
                                               unsigned long long* __restrict__ bad) {
  __shared__ __attribute__((aligned(16))) T LU[kN][kLdLU];  // L (c < r) and U (c >= r), row-major
  __shared__ T Wy[kN][kLdR];                               // rows of U^{-1}
  __shared__ T Wx[kN][kLdR];                               // rows of L^{-1}
  __shared__ T Rv[kN];                                     // 1 / u(k, k)
  __shared__ T Lm[2][kB][kN];                              // multipliers of the current 16 steps
  const PanelProb P = probs[blockIdx.x];
  T* __restrict__ D = (T*)P.D;
  const int r = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ld = P.ld;

  T a[kB];   // a[c] = A(r, 16 w + c)
#pragma unroll
  for (int c = 0; c < kB; ++c) a[c] = D[(int64_t)(kB * w + c) * ld + r];

#pragma unroll 1
  for (int kb = 0; kb < kN / kB; ++kb) {
    // the owner eliminates its 16 columns and publishes their multipliers
    if (w == kb) {
#pragma unroll
      for (int kc = 0; kc < kB; ++kc) {
        const int k = kB * kb + kc;
        const T rp = T(1) / lane_value(a[kc], k);
        if (r == 0) Rv[k] = rp;
        const T l = r > k ? a[kc] * rp : T(0);
        a[kc] = r > k ? l : a[kc];
        Lm[kb & 1][kc][r] = l;
#pragma unroll
        for (int c = kc + 1; c < kB; ++c) a[c] -= l * lane_value(a[c], k);
      }
    }
    __syncthreads();
    // the waves right of it apply the 16 steps to their columns
    if (w > kb) {
#pragma unroll
      for (int kc = 0; kc < kB; ++kc) {
        const int k = kB * kb + kc;
        const T l = Lm[kb & 1][kc][r];
#pragma unroll
        for (int c = 0; c < kB; ++c) a[c] -= l * lane_value(a[c], k);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kB; ++c) LU[r][kB * w + c] = a[c];
  __syncthreads();

  if (w == 2) {
    const double th = thresh[P.vrow0 + r];   // pivot threshold of this lane's row
    const double av = fabs((double)LU[r][r]);
    if (!(av > th) || !(av <= 1.7e308))
      atomicMin(bad, ((unsigned long long)P.block << 40) | (unsigned long long)(P.row0 + r));
  } else if (w == 0) {
    // Y = U^{-1}, 16-column blocks left to right
#pragma unroll 1
    for (int j0 = 0; j0 < kN; j0 += kB) {
      T acc[kB];
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) acc[jj] = T(0);
      // earlier columns: Y(r, l) for l < j0 from LDS (zero for l < r)
#pragma unroll 4
      for (int l = 0; l < j0; ++l) {
        const T yl = Wy[r][l];
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
      for (int jj = 0; jj < kB; ++jj) Wy[r][j0 + jj] = y[jj];
    }
    // U^{-1} on and above the diagonal
#pragma unroll 4
    for (int c = 0; c < kN; ++c)
      if (c >= r) D[c * ld + r] = Wy[r][c];
  } else if (w == 1) {
    // X = L^{-1}, 16-column blocks right to left
#pragma unroll 1
    for (int j0 = kN - kB; j0 >= 0; j0 -= kB) {
      T acc[kB];
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) acc[jj] = j0 + jj < r ? LU[r][j0 + jj] : T(0);
      // later columns: X(r, l) for l >= j0 + 16 from LDS (zero for l >= r)
#pragma unroll 4
      for (int l = j0 + kB; l < kN; ++l) {
        const T xl = Wx[r][l];
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
      for (int jj = 0; jj < kB; ++jj) Wx[r][j0 + jj] = x[jj];
    }
    // L^{-1} strictly below the diagonal
#pragma unroll 4
    for (int c = 0; c < kN; ++c)
      if (c < r) D[c * ld + r] = Wx[r][c];
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
