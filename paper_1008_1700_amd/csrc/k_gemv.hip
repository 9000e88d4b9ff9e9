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
  const bool mlu = fl & V_A_MLU, mup = fl & V_A_MUP, mlo = fl & V_A_MLO;
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
      if (mlo) av = r >= cc ? av : 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) acc[j] += av * xval(cc, j);
    }
  }
  for (; c < ce; c += 4) {
    double av = (double)A[(int64_t)c * lda];
    if (mlu) av = r > c ? av : (r == c ? 1.0 : 0.0);
    if (mup) av = r <= c ? av : 0.0;
    if (mlo) av = r >= c ? av : 0.0;
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

// ------------------------------------------------------------------------
// Wide-load form of k_gemv for 16-byte aligned problems: a lane reads VEC
// consecutive rows of one column in one 16-byte load, so one wave load
// covers 64 rows of VEC columns (1 KB) instead of 64 rows of one column.
// The VEC column slots of a wave are summed by lane shuffles, the 4 waves
// through LDS; epilogue, flags and partial sums as in k_gemv.
// ------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(256) void k_gemv_w(const GemvProb* __restrict__ probs, int nprob,
                                                int64_t ldx, int64_t ldy,
                                                const double* __restrict__ dotv,
                                                double* __restrict__ partial,
                                                const int32_t* __restrict__ stop) {
  constexpr int VEC = 16 / sizeof(T);   // rows per lane
  constexpr int LPC = 64 / VEC;         // lanes per column
  constexpr int STEP = 4 * VEC;         // columns per round of the workgroup
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
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
  const int q = lane / LPC;             // column slot of this lane
  const int rl = (lane % LPC) * VEC;    // first local row of this lane
  const int fl = P.flags;
  const bool mlu = fl & V_A_MLU, mup = fl & V_A_MUP, mlo = fl & V_A_MLO;
  const T* __restrict__ A = (const T*)P.A + r0 + rl;
  const int64_t lda = P.lda;
  const int split = P.split;

  double acc[VEC][R];
#pragma unroll
  for (int e = 0; e < VEC; ++e)
#pragma unroll
    for (int j = 0; j < R; ++j) acc[e][j] = 0.0;

  auto add = [&](const vec_t& a, int cc) __attribute__((always_inline)) {
    double xv[R];
#pragma unroll
    for (int j = 0; j < R; ++j) xv[j] = cc < split ? P.x1[cc + j * ldx] : P.x2[(cc - split) + j * ldx];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int rr = r0 + rl + e;
      double av = (double)a[e];
      if (mlu) av = rr > cc ? av : (rr == cc ? 1.0 : 0.0);
      if (mup) av = rr <= cc ? av : 0.0;
      if (mlo) av = rr >= cc ? av : 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) acc[e][j] += av * xv[j];
    }
  };
  if constexpr (R >= 4) {
    // many right-hand sides: the vector entries of each round of 4 STEP
    // columns are staged once per workgroup in LDS (double-buffered), so a
    // lane reads its columns' R entries as 16-byte LDS reads instead of R
    // separate global loads
    constexpr int RC = 4 * STEP;   // columns per round
    __shared__ __attribute__((aligned(16))) double xs[2][RC][R];
    int buf = 0;
    for (int c0 = cb; c0 < ce; c0 += RC) {
      for (int i = tid; i < RC * R; i += 256) {
        const int cc = c0 + i / R, j = i % R;
        xs[buf][i / R][j] = cc < ce ? (cc < split ? P.x1[cc + j * ldx] : P.x2[(cc - split) + j * ldx]) : 0.0;
      }
      __syncthreads();
      vec_t a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cc = c0 + g * VEC + q + u * STEP;
        a[u] = cc < ce ? *(const vec_t*)(A + (int64_t)cc * lda) : vec_t{};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cl = g * VEC + q + u * STEP, cc = c0 + cl;
        double xv[R];
#pragma unroll
        for (int j = 0; j < R; ++j) xv[j] = xs[buf][cl][j];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int rr = r0 + rl + e;
          double av = (double)a[u][e];
          if (mlu) av = rr > cc ? av : (rr == cc ? 1.0 : 0.0);
          if (mup) av = rr <= cc ? av : 0.0;
          if (mlo) av = rr >= cc ? av : 0.0;
#pragma unroll
          for (int j = 0; j < R; ++j) acc[e][j] += av * xv[j];
        }
      }
      buf ^= 1;
    }
  } else {
    int c = cb + g * VEC + q;
    // four independent columns per lane per step for memory-level parallelism
    for (; c + 3 * STEP < ce; c += 4 * STEP) {
      vec_t a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = *(const vec_t*)(A + (int64_t)(c + u * STEP) * lda);
#pragma unroll
      for (int u = 0; u < 4; ++u) add(a[u], c + u * STEP);
    }
    for (; c < ce; c += STEP) add(*(const vec_t*)(A + (int64_t)c * lda), c);
  }
  // sum the column slots of the wave (lanes with equal lane % LPC)
#pragma unroll
  for (int e = 0; e < VEC; ++e)
#pragma unroll
    for (int j = 0; j < R; ++j)
      for (int off = LPC; off < 64; off <<= 1) acc[e][j] += __shfl_xor(acc[e][j], off, 64);
  if (lane < LPC) {
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
      for (int j = 0; j < R; ++j) red[g][rl + e][j] = acc[e][j];
  }
  __syncthreads();
  if (tid < 64) {
    const int r = r0 + lane;
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

// ------------------------------------------------------------------------
// Reduced-matrix product on packed spike tips.  The rows of G^ are the
// first and last t rows of each spike G_i (2t columns each), which inside
// the column-major spikes are 4t-byte column pieces N_i apart.  After every
// factorisation they are packed row-major (k_pack_tips), and the product
// streams each row as one contiguous run: a wave owns a row at a time, its
// lanes read consecutive 16-byte pieces of it, the right-hand-side entries
// come from L1/L2 (2t values shared by every row of the part), and the row
// sum is a wave reduction.  Lane rr keeps the sum of the wave's row rr,
// and one epilogue per wave then serves its 16 rows at once.  Same problem
// records, flags and partial-sum layout as k_gemv (A = first packed row,
// lda = row length 2t).
// ------------------------------------------------------------------------
template <typename T, int R, int NSEG>
__global__ __launch_bounds__(256) void k_tipmv(const GemvProb* __restrict__ probs, int nprob,
                                               int64_t ldx, int64_t ldy,
                                               const double* __restrict__ dotv,
                                               double* __restrict__ partial,
                                               const int32_t* __restrict__ stop) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int RPW = 16;                       // rows per wave (64 per workgroup)
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  __shared__ double red[4][R][2];
  if (stop) {
    bool all = true;
#pragma unroll
    for (int j = 0; j < R; ++j) all &= stop[j] != KS_RUNNING;
    if (all) return;
  }
  const int wg = blockIdx.x;
  const GemvProb& P = probs[find_gemv(probs, nprob, wg)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fl = P.flags;
  const int cb = P.cb, ce = P.ce, split = P.split;
  const int rbase = (wg - P.wg0) * 64 + wave * RPW;
  // the right-hand-side entries of this lane's columns, once for all rows
  double xr[NSEG][VEC][R];
#pragma unroll
  for (int sg = 0; sg < NSEG; ++sg)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int c = cb + (sg * 64 + lane) * VEC + e;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        double v = 0.0;
        if (c < ce) v = c < split ? P.x1[c + j * ldx] : P.x2[(c - split) + j * ldx];
        xr[sg][e][j] = v;
      }
    }
  // row rr's sum is kept by lane rr; one epilogue per wave for its 16 rows
  double mine[R];
#pragma unroll
  for (int j = 0; j < R; ++j) mine[j] = 0.0;
#pragma unroll 2
  for (int rr = 0; rr < RPW; ++rr) {
    const int r = rbase + rr;
    const T* __restrict__ Arow = (const T*)P.A + (int64_t)r * P.lda + cb;
    vec_t a[NSEG];
#pragma unroll
    for (int sg = 0; sg < NSEG; ++sg) {
      const int c0 = (sg * 64 + lane) * VEC;
      if (cb + c0 < ce) a[sg] = *(const vec_t*)(Arow + c0);
      else a[sg] = vec_t{};
    }
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
#pragma unroll
    for (int sg = 0; sg < NSEG; ++sg)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[j] += (double)a[sg][e] * xr[sg][e][j];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
      mine[j] = lane == rr ? acc[j] : mine[j];
    }
  }
  double dot[R], dd[R];
#pragma unroll
  for (int j = 0; j < R; ++j) dot[j] = dd[j] = 0.0;
  if (lane < RPW) {
    const int r = rbase + lane;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double v = mine[j];
      if (fl & V_MASK) v *= P.mask[r];
      if (fl & V_NEG) v = -v;
      if (fl & V_YIN) v += P.yin[r + j * ldy];
      P.yout[r + j * ldy] = v;
      if (fl & V_DOT) dot[j] = dotv[P.dot_off + r + j * ldy] * v;
      if (fl & V_DOT2) dd[j] = v * v;
    }
  }
  if (fl & (V_DOT | V_DOT2)) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      for (int off = RPW / 2; off > 0; off >>= 1) {
        dot[j] += __shfl_xor(dot[j], off, 64);
        dd[j] += __shfl_xor(dd[j], off, 64);
      }
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        red[wave][j][0] = dot[j];
        red[wave][j][1] = dd[j];
      }
    __syncthreads();
    if (tid < R) {
      const int j = tid;
      partial[((int64_t)wg * R + j) * 2 + 0] = (red[0][j][0] + red[1][j][0]) + (red[2][j][0] + red[3][j][0]);
      partial[((int64_t)wg * R + j) * 2 + 1] = (red[0][j][1] + red[1][j][1]) + (red[2][j][1] + red[3][j][1]);
    }
  }
}

// Packs the spike tips row-major: part q (q = 0 .. 2(p-1)-1; block
// i = (q+1)/2, its first t rows for q odd, its last t rows for q even) to
// tips[q][r][c], r < t, c < 2t, through a 64 x 64 LDS tile so both the
// column-major reads and the row-major writes are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_tips(const BlockInfo* __restrict__ blocks, int t,
                                                   const T* __restrict__ spikes, T* __restrict__ tips) {
  __shared__ T tile[64][65];
  const int q = blockIdx.z;
  const int i = (q + 1) / 2;
  const BlockInfo B = blocks[i];
  const int64_t row0 = (q & 1) ? B.pad : B.N - t;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const T* __restrict__ G = spikes + B.goff;
  T* __restrict__ out = tips + (int64_t)q * t * 2 * t;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int c = ty + 4 * k;
    tile[c][tx] = G[(int64_t)(c0 + c) * B.N + row0 + r0 + tx];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = ty + 4 * k;
    out[(int64_t)(r0 + r) * 2 * t + c0 + tx] = tile[tx][r];
  }
}

// segments of 64 x (16-byte piece) per row: 2t elements need ceil(2t / (64 VEC))
int tipmv_segments(int dtype, int t) {
  const int vec = dtype == 0 ? 2 : 4;
  const int need = (2 * t + 64 * vec - 1) / (64 * vec);
  for (int n : {4, 8, 16})
    if (need <= n) return n;
  return 0;   // longer rows: the product on the spikes themselves
}

template <typename T, int NSEG>
static void tipmv_dispatch(int nrhs, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                           int64_t ldy, const double* dotv, double* partial, const int32_t* stop,
                           hipStream_t s) {
  if (nrhs == 1)
    hipLaunchKernelGGL((k_tipmv<T, 1, NSEG>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop);
  else
    hipLaunchKernelGGL((k_tipmv<T, 2, NSEG>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop);
}

void launch_tipmv(int dtype, int nrhs, int nseg, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                  int64_t ldy, const double* dotv, double* partial, const int32_t* stop, hipStream_t s) {
  if (nwg <= 0 || nprob <= 0) return;
#define DDPS_TIPMV(T)                                                                                   \
  switch (nseg) {                                                                                       \
    case 4: tipmv_dispatch<T, 4>(nrhs, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s); break;     \
    case 8: tipmv_dispatch<T, 8>(nrhs, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s); break;     \
    default: tipmv_dispatch<T, 16>(nrhs, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s); break;   \
  }
  if (dtype == 0) { DDPS_TIPMV(double) }
  else { DDPS_TIPMV(float) }
#undef DDPS_TIPMV
}

void pack_tips(int dtype, int p, int t, const BlockInfo* blocks, const void* spikes, void* tips, hipStream_t s) {
  if (p < 2) return;
  const dim3 g(2 * t / 64, t / 64, 2 * (p - 1)), b(256);
  if (dtype == 0) hipLaunchKernelGGL(k_pack_tips<double>, g, b, 0, s, blocks, t, (const double*)spikes, (double*)tips);
  else hipLaunchKernelGGL(k_pack_tips<float>, g, b, 0, s, blocks, t, (const float*)spikes, (float*)tips);
}

// ------------------------------------------------------------------------
// Many right-hand sides (R >= 4) on FP32 operands, as products on the FP32
// matrix cores (16x16x4).  One
// workgroup per 64-row slab; its 4 waves take interleaved groups of 4
// columns.  Lane l loads rows 4(l & 15) .. +3 of column c + (l >> 4) (one
// float4; a wave load covers 64 rows x 4 columns), and the four products q
// take its component q, so product q accumulates the slab rows 4i + q.  The
// second operand of lane l is x(c + (l >> 4), rhs l & 15) rounded to FP32
// (0 for rhs >= R).  The sums are FP32, each over a quarter of the columns;
// the four quarters are added in FP64 in a fixed order.  Register v of
// accumulator q in lane l holds slab row 16 (l >> 4) + 4 v + q, rhs l & 15.
// Triangular problems clip the column range as the other kernels do; the
// masks of packed triangles change only the columns [r0, r0 + 64) of a
// slab, so only loads of those columns go through the selects.
// ------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_gemv_mf32(const GemvProb* __restrict__ probs, int nprob,
                                                   int64_t ldx, int64_t ldy,
                                                   const double* __restrict__ dotv,
                                                   double* __restrict__ partial,
                                                   const int32_t* __restrict__ stop) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  static_assert(R >= 1 && R <= 16, "right-hand sides per product");
  constexpr int U = 4;   // column groups in flight per wave
  __shared__ float red[4][64][R];
  if (stop) {
    bool all = true;
#pragma unroll
    for (int j = 0; j < R; ++j) all &= stop[j] != KS_RUNNING;
    if (all) return;
  }
  const int wg = blockIdx.x;
  const GemvProb P = probs[find_gemv(probs, nprob, wg)];
  const int r0 = (wg - P.wg0) * 64;
  int cb = P.cb, ce = P.ce;
  if (P.tri == 1) ce = min(ce, r0 + 64);
  if (P.tri == 2) cb = max(cb, r0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int fl = P.flags;
  const bool mlu = fl & V_A_MLU, mup = fl & V_A_MUP, mlo = fl & V_A_MLO;
  const bool masked = mlu || mup || mlo;
  const float* __restrict__ A = (const float*)P.A + r0 + 4 * li;
  const int64_t lda = P.lda;
  const int split = P.split;
  const bool live = li < R;
  const int jx = live ? li : 0;
  f32x4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto xval = [&](int cc) __attribute__((always_inline)) -> float {
    const double v = cc < split ? P.x1[cc + jx * ldx] : P.x2[(cc - split) + jx * ldx];
    return live ? (float)v : 0.f;
  };
  // the packed-triangle masks on the 4 rows of a lane's load of column cc
  auto fix = [&](float4& a, int cc) __attribute__((always_inline)) {
    if (masked && cc >= r0 && cc < r0 + 64) {
      float e[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = r0 + 4 * li + q;
        if (mlu) e[q] = rr > cc ? e[q] : (rr == cc ? 1.f : 0.f);
        if (mup) e[q] = rr <= cc ? e[q] : 0.f;
        if (mlo) e[q] = rr >= cc ? e[q] : 0.f;
      }
      a = float4{e[0], e[1], e[2], e[3]};
    }
  };
  auto mma = [&](const float4& a, float x) __attribute__((always_inline)) {
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, x, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, x, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, x, acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, x, acc[3], 0, 0, 0);
  };
  // wave g takes the column groups cb + 4 (g + 4 s), s = 0, 1, ...
  int c = cb + 4 * g;
  for (; c + 16 * (U - 1) + 3 < ce; c += 16 * U) {
    float4 a[U];
    float x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int cc = c + 16 * u + lk;
      a[u] = *(const float4*)(A + (int64_t)cc * lda);
      x[u] = xval(cc);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      fix(a[u], c + 16 * u + lk);
      mma(a[u], x[u]);
    }
  }
  for (; c < ce; c += 16) {
    const int cc = c + lk;
    const bool in = cc < ce;
    float4 a = in ? *(const float4*)(A + (int64_t)cc * lda) : float4{0.f, 0.f, 0.f, 0.f};
    fix(a, cc);
    mma(a, in ? xval(cc) : 0.f);
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[g][16 * lk + 4 * v + q][li] = acc[q][v];
  }
  __syncthreads();
  if (tid < 64) {
    const int r = r0 + lane;
    double dot[R], dd[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double s = (double)red[0][lane][j] + (double)red[1][lane][j] + (double)red[2][lane][j] + (double)red[3][lane][j];
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
static void gemv_dispatch(int nrhs, bool wide, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                          int64_t ldy, const double* dotv, double* partial, const int32_t* stop,
                          hipStream_t s) {
#define DDPS_GEMV(K)                                                                                           \
  switch (nrhs) {                                                                                              \
    case 1: hipLaunchKernelGGL((K<T, 1>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break; \
    case 2: hipLaunchKernelGGL((K<T, 2>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break; \
    case 4: hipLaunchKernelGGL((K<T, 4>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break; \
    default: hipLaunchKernelGGL((K<T, 8>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop); break; \
  }
  if (wide) { DDPS_GEMV(k_gemv_w) }
  else { DDPS_GEMV(k_gemv) }
#undef DDPS_GEMV
}

void launch_gemv(int dtype, int nrhs, int form, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                 int64_t ldy, const double* dotv, double* partial, const int32_t* stop, hipStream_t s) {
  if (nwg <= 0 || nprob <= 0) return;
  if (dtype == 1 && form == 2 && nrhs >= 4) {
    if (nrhs == 4)
      hipLaunchKernelGGL((k_gemv_mf32<4>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop);
    else
      hipLaunchKernelGGL((k_gemv_mf32<8>), dim3(nwg), dim3(256), 0, s, probs, nprob, ldx, ldy, dotv, partial, stop);
    return;
  }
  if (dtype == 0) gemv_dispatch<double>(nrhs, form >= 1, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s);
  else gemv_dispatch<float>(nrhs, form >= 1, probs, nprob, nwg, ldx, ldy, dotv, partial, stop, s);
}

}  // namespace ddps
