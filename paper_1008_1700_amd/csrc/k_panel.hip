// Diagonal sub-tile kernel of the tile LU: for each problem, one workgroup of
// eight waves factors a 64 x 64 sub-tile without pivoting (A = L U, L unit
// lower), then inverts both triangles and writes back L^{-1} strictly below
// the diagonal and U^{-1} on and above it.
//
// The kernel is latency bound (a few of them run at a time, one per block of
// the partition), so the work of one sub-tile is spread over eight waves.
//
// Elimination.  Wave w owns columns 8w .. 8w+7: lane r holds
// a[c] = A(r, 8w + c) in registers.  In round b the wave owning columns
// 8b .. 8b+7 runs their 8 elimination steps k: it reads the pivot u(k,k)
// from lane k (v_readlane), forms the multipliers l(r) = a(r,k) / u(k,k) for
// r > k, keeps them as column k of L, updates its own columns right of k and
// puts the multipliers in LDS.  After one barrier every wave right of it
// applies the same 8 steps to its columns, a(r,c) -= l(r) a(k,c), with the
// pivot row read from lane k of its own registers.  The multipliers of
// consecutive rounds alternate between two LDS buffers.  The operations and
// their order per entry are those of a one-wave elimination, so the factors
// do not depend on the split.
//
// Inversion, with the factors in LDS (row-major, L below the diagonal, U on
// and above it); waves 0 and 2 form Y = U^{-1} and waves 1 and 3 X = L^{-1}
// at the same time (waves 4-7 only meet the barriers), lane r computing row
// r one 16-column block at a time (each wave 8 of its columns) with the
// earlier blocks' rows in LDS:
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
constexpr int kB = 16;         // column block of the inversions
constexpr int kW = 8;          // waves of the workgroup
constexpr int kE = kN / kW;    // columns per wave in the elimination
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
__global__ __launch_bounds__(64 * kW) void k_panel(const PanelProb* __restrict__ probs,
                                               const double* __restrict__ thresh,
                                               unsigned long long* __restrict__ bad) {
  __shared__ __attribute__((aligned(16))) T LU[kN][kLdLU];  // L (c < r) and U (c >= r), row-major
  __shared__ T Wy[kN][kLdR];                               // rows of U^{-1}
  __shared__ T Wx[kN][kLdR];                               // rows of L^{-1}
  __shared__ T Rv[kN];                                     // 1 / u(k, k)
  __shared__ T Lm[2][kE][kN];                              // multipliers of the current round
  const PanelProb P = probs[blockIdx.x];
  T* __restrict__ D = (T*)P.D;
  const int r = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ld = P.ld;

  T a[kE];   // a[c] = A(r, kE w + c)
#pragma unroll
  for (int c = 0; c < kE; ++c) a[c] = D[(int64_t)(kE * w + c) * ld + r];

#pragma unroll 1
  for (int kb = 0; kb < kW; ++kb) {
    // the owner eliminates its kE columns and publishes their multipliers
    if (w == kb) {
#pragma unroll
      for (int kc = 0; kc < kE; ++kc) {
        const int k = kE * kb + kc;
        const T rp = T(1) / lane_value(a[kc], k);
        if (r == 0) Rv[k] = rp;
        const T l = r > k ? a[kc] * rp : T(0);
        a[kc] = r > k ? l : a[kc];
        Lm[kb & 1][kc][r] = l;
#pragma unroll
        for (int c = kc + 1; c < kE; ++c) a[c] -= l * lane_value(a[c], k);
      }
    }
    __syncthreads();
    // the waves right of it apply the same steps to their columns
    if (w > kb) {
#pragma unroll
      for (int kc = 0; kc < kE; ++kc) {
        const int k = kE * kb + kc;
        const T l = Lm[kb & 1][kc][r];
#pragma unroll
        for (int c = 0; c < kE; ++c) a[c] -= l * lane_value(a[c], k);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kE; ++c) LU[r][kE * w + c] = a[c];
  __syncthreads();

  if (w == 2) {
    const double th = thresh[P.vrow0 + r];   // pivot threshold of this lane's row
    const double av = fabs((double)LU[r][r]);
    if (!(av > th) || !(av <= 1.7e308))
      atomicMin(bad, ((unsigned long long)P.block << 40) | (unsigned long long)(P.row0 + r));
  }

  // Inversions, four rounds on all four waves: round b takes block 16b of
  // Y = U^{-1} (waves 0 and 2) and block 48 - 16b of X = L^{-1} (waves 1
  // and 3).  Each wave sums the earlier (Y) or later (X) blocks' terms for 8
  // of the 16 columns.  Within a block, Y's columns depend on those to their
  // left and X's on those to their right: wave 0 finishes Y's left half and
  // wave 3 X's right half first; after a barrier wave 2 and wave 1 finish
  // the other halves with those from LDS.  Every entry takes the terms in
  // the same order as a one-wave inversion.
  constexpr int kH = kB / 2;
  const bool isY = (w & 1) == 0;
  const int h0 = (w == 0 || w == 1) ? 0 : kH;   // first column of this wave's half
#pragma unroll 1
  for (int b = 0; b < kN / kB; ++b) {
    const int j0 = isY ? kB * b : kN - kB - kB * b;
    T acc[kH];
    if (w >= 4) {
    } else if (isY) {
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) acc[jj] = T(0);
#pragma unroll 4
      for (int l = 0; l < j0; ++l) {
        const T yl = Wy[r][l];
#pragma unroll
        for (int jj = 0; jj < kH; ++jj) acc[jj] += yl * LU[l][j0 + h0 + jj];
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) acc[jj] = j0 + h0 + jj < r ? LU[r][j0 + h0 + jj] : T(0);
#pragma unroll 4
      for (int l = j0 + kB; l < kN; ++l) {
        const T xl = Wx[r][l];
#pragma unroll
        for (int jj = 0; jj < kH; ++jj) acc[jj] += xl * LU[l][j0 + h0 + jj];
      }
    }
    // first halves: Y's left (wave 0), X's right (wave 3)
    if (w == 0) {
      T y[kH];
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) {
        const int j = j0 + jj;
        T s = acc[jj];
#pragma unroll
        for (int ll = 0; ll < jj; ++ll) s += y[ll] * LU[j0 + ll][j];
        const T rv = Rv[j];
        y[jj] = j < r ? T(0) : (j == r ? rv : -s * rv);
      }
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) Wy[r][j0 + jj] = y[jj];
    } else if (w == 3) {
      T x[kH];
#pragma unroll
      for (int jj = kH - 1; jj >= 0; --jj) {
        const int j = j0 + kH + jj;
        T s = acc[jj];
#pragma unroll
        for (int ll = jj + 1; ll < kH; ++ll) s += x[ll] * LU[j0 + kH + ll][j];
        x[jj] = j < r ? -s : T(0);
      }
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) Wx[r][j0 + kH + jj] = x[jj];
    }
    __syncthreads();
    // second halves, with the first halves from LDS
    if (w == 2) {
      T y[kH];
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) {
        const int j = j0 + kH + jj;
        T s = acc[jj];
#pragma unroll
        for (int ll = 0; ll < kH; ++ll) s += Wy[r][j0 + ll] * LU[j0 + ll][j];
#pragma unroll
        for (int ll = 0; ll < jj; ++ll) s += y[ll] * LU[j0 + kH + ll][j];
        const T rv = Rv[j];
        y[jj] = j < r ? T(0) : (j == r ? rv : -s * rv);
      }
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) Wy[r][j0 + kH + jj] = y[jj];
    } else if (w == 1) {
      T x[kH];
#pragma unroll
      for (int jj = kH - 1; jj >= 0; --jj) {
        const int j = j0 + jj;
        T s = acc[jj];
#pragma unroll
        for (int ll = jj + 1; ll < kH; ++ll) s += x[ll] * LU[j0 + ll][j];
#pragma unroll
        for (int ll = kH; ll < kB; ++ll) s += Wx[r][j0 + ll] * LU[j0 + ll][j];
        x[jj] = j < r ? -s : T(0);
      }
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) Wx[r][j0 + jj] = x[jj];
    }
    __syncthreads();
  }
  // U^{-1} on and above the diagonal, L^{-1} strictly below it: each wave
  // writes kE of the 64 columns
#pragma unroll
  for (int cc = 0; cc < kE; ++cc) {
    const int c = kE * w + cc;
    D[c * ld + r] = c >= r ? Wy[r][c] : Wx[r][c];
  }
}

void launch_panel(int dtype, const PanelProb* probs, int nprob, const double* thresh,
                  unsigned long long* bad, hipStream_t s) {
  if (nprob <= 0) return;
  if (dtype == 0)
    hipLaunchKernelGGL(k_panel<double>, dim3(nprob), dim3(64 * kW), 0, s, probs, thresh, bad);
  else
    hipLaunchKernelGGL(k_panel<float>, dim3(nprob), dim3(64 * kW), 0, s, probs, thresh, bad);
}

}  // namespace ddps
