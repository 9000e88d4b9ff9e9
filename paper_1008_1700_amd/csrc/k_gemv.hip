// Grouped tile GEMV for 1..8 right-hand sides: y_out = y_in +/- A x.
//
// Used by every HBM-bound stream of the solve phase: the block sweeps of
// step 6.1 (triangular inverse tiles and coupling tiles), the reduced-matrix
// product of 6.3 (spike-tip rows, masked to the index set c) and the
// retrieval z = g - G z^ of 6.5.  Each workgroup owns 64 consecutive output
// rows of one problem; its 4 waves take interleaved columns, so one wave
// load reads 64 consecutive rows of one column (512 B for f64 matrices), and
// the vector entries are wave-uniform (scalar loads).  Triangular problems
// clip the column range per 64-row slab and mask the diagonal slab.
#include "ddps_internal.h"

namespace ddps {

__device__ __forceinline__ int find_gemv(const GemvProb* __restrict__ probs, int nprob, int wg) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].wg0 <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, int R>
__global__ __launch_bounds__(256) void k_gemv(const GemvProb* __restrict__ probs, int nprob,
                                              int64_t ldx, int64_t ldy,
                                              const double* __restrict__ dotv,
                                              double* __restrict__ partial,
                                              const int32_t* __restrict__ stop) {
  __shared__ double red[4][64][R];
  if (stop) {
    bool all = true;
#pragma unroll
    for (int j = 0; j < R; ++j) all &= stop[j] != KS_RUNNING;
    if (all) return;
  }
  const int wg = blockIdx.x;
  const GemvProb& Pg = probs[find_gemv(probs, nprob, wg)];
  const GemvProb P = Pg;
  const int r0 = (wg - P.wg0) * 64;
  int cb = P.cb, ce = P.ce;
  if (P.tri == 1) ce = min(ce, r0 + 64);
  if (P.tri == 2) cb = max(cb, r0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = r0 + lane;
  const int fl = P.flags;
  const bool mlu = fl & V_A_MLU, mup = fl & V_A_MUP;
  const T* __restrict__ A = (const T*)P.A + r;
  const int64_t lda = P.lda;
  const int split = P.split;

  double acc[R];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j] = 0.0;

  auto xval = [&](int c, int j) -> double {
    return c < split ? P.x1[c + j * ldx] : P.x2[(c - split) + j * ldx];
  };
  int c = cb + g;
  // four independent columns per step for memory-level parallelism
  for (; c + 12 < ce; c += 16) {
    T a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = A[(int64_t)(c + 4 * u) * lda];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = c + 4 * u;
      double av = (double)a[u];
      if (mlu) av = r > cc ? av : (r == cc ? 1.0 : 0.0);
      if (mup) av = r <= cc ? av : 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) acc[j] += av * xval(cc, j);
    }
  }
  for (; c < ce; c += 4) {
    double av = (double)A[(int64_t)c * lda];
    if (mlu) av = r > c ? av : (r == c ? 1.0 : 0.0);
    if (mup) av = r <= c ? av : 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] += av * xval(c, j);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) red[g][lane][j] = acc[j];
  __syncthreads();
  if (tid < 64) {
    double dot[R], dd[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double s = red[0][lane][j] + red[1][lane][j] + red[2][lane][j] + red[3][lane][j];
      if (fl & V_MASK) s *= P.mask[r];
      if (fl & V_NEG) s = -s;
      if (fl & V_YIN) s += P.yin[r + j * ldy];
      if (r >= P.row_skip) P.yout[r + j * ldy] = s;
      dot[j] = (fl & V_DOT) ? dotv[P.dot_off + r + j * ldy] * s : 0.0;
      dd[j] = (fl & V_DOT2) ? s * s : 0.0;
    }
    if (fl & V_DOT) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        double v = dot[j], w = dd[j];
        for (int off = 32; off > 0; off >>= 1) {
          v += __shfl_xor(v, off, 64);
          w += __shfl_xor(w, off, 64);
        }
        if (lane == 0) {
          partial[((int64_t)wg * R + j) * 2 + 0] = v;
          partial[((int64_t)wg * R + j) * 2 + 1] = w;
        }
      }
    }
  }
}

template <typename T>
static void gemv_dispatch(int nrhs, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                          int64_t ldy, const double* dotv, double* partial, const int32_t* stop,
                          hipStream_t s) {
  switch (nrhs) {
    case 1: hipLaunchKernelGGL((k_gemv<T, 1>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break;
    case 2: hipLaunchKernelGGL((k_gemv<T, 2>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break;
    case 4: hipLaunchKernelGGL((k_gemv<T, 4>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break;
    default: hipLaunchKernelGGL((k_gemv<T, 8>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break;
  }
}

void launch_gemv(int dtype, int nrhs, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                 int64_t ldy, const double* dotv, double* partial, const int32_t* stop, hipStream_t s) {
  if (nwg <= 0 || nprob <= 0) return;
  if (dtype == 0) gemv_dispatch<double>(nrhs, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s);
  else gemv_dispatch<float>(nrhs, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s);
}

}  // namespace ddps
