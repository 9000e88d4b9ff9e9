// Incomplete block factors (Section 3: D~ built from L~_i U~_i), read as
// ILU(0): L~_i unit lower and U~_i upper with the sparsity pattern of A_ii,
// so that (L~_i U~_i)(r, j) = a_rj wherever A_ii stores an entry.
//
// Storage.  The factor values sit at A's own CSR positions (fv, double):
// for global row r of block i, positions [lo[r], dg[r]) hold the strictly
// lower entries of L~ (unit diagonal implied), dg[r] the pivot and
// (dg[r], hi[r]) the rest of U~'s row (columns sorted; the positions outside
// [lo, hi) are coupling entries and are not touched).
//
// Order.  Both the factorisation and the forward solve need, for row r, the
// finished rows of its lower pattern; the backward solve the finished rows
// of its upper pattern.  The host groups each block's rows into levels
// (level of r = 1 + the largest level of the rows it refers to), so the rows
// of a level are independent; one workgroup runs one block level by level.
//
// Spikes.  G_i = D~_i^{-1} R~_i has 2t dense columns per block; one thread
// owns one column and runs both triangular solves down and up the block in
// row order (no barriers: the columns are independent), in a row-major
// workspace so that a wave's 64 columns of one row are one coalesced access.
// Only the spike tips (first and last t rows) are kept, transposed into the
// column-major tip store by an LDS-tiled copy.
#include "ddps_internal.h"

namespace ddps {
namespace {

constexpr int kIluThreads = 256;

// ILU(0) of every diagonal block, one workgroup per block.  IKJ form per
// row: for each k < r of its pattern, in increasing order, l_rk = a_rk / u_kk,
// then a_rj -= l_rk u_kj for every j > k stored in both row r and row k (the
// two sorted column lists are merged).  A pivot at or below the row's
// threshold is reported through `bad` (block << 40 | row, smallest wins).
__global__ __launch_bounds__(kIluThreads) void k_ilu0(const IluBlock* __restrict__ blocks,
                                                        const int32_t* __restrict__ lrows,
                                                        const int64_t* __restrict__ lptr,
                                                        const int64_t* __restrict__ lo, const int64_t* __restrict__ dg,
                                                        const int64_t* __restrict__ hi,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, double* fv,
                                                        const double* __restrict__ thresh,
                                                        unsigned long long* __restrict__ bad) {
  const int bi = blockIdx.x;
  const IluBlock B = blocks[bi];
  for (int64_t r = B.s + threadIdx.x; r < B.s + B.n; r += blockDim.x)
    for (int64_t q = lo[r]; q < hi[r]; ++q) fv[q] = val[q];
  __syncthreads();
  for (int64_t lv = 0; lv < B.lnum; ++lv) {
    const int64_t a = lptr[B.lbeg + lv], e = lptr[B.lbeg + lv + 1];
    for (int64_t idx = a + threadIdx.x; idx < e; idx += blockDim.x) {
      const int64_t r = lrows[idx];
      const int64_t rdg = dg[r], rhi = hi[r];
      for (int64_t q = lo[r]; q < rdg; ++q) {
        const int64_t k = col[q];
        const int64_t kdg = dg[k], khi = hi[k];
        const double l = fv[q] / fv[kdg];
        fv[q] = l;
        int64_t w = q + 1;
        for (int64_t u = kdg + 1; u < khi && w < rhi; ++u) {
          const int32_t j = col[u];
          while (w < rhi && col[w] < j) ++w;
          if (w < rhi && col[w] == j) fv[w] -= l * fv[u];
        }
      }
      const double piv = fv[rdg];
      if (!(fabs(piv) > thresh[B.vbase + (r - B.s)]))
        atomicMin(bad, ((unsigned long long)bi << 40) | (unsigned long long)r);
    }
    __syncthreads();
  }
}

// Spike columns of a batch of blocks: workgroup (x = position in the batch,
// y = chunk of kIluThreads columns).  Column c < t is the left coupling
// column c (right-hand side C_i(:, c) on the block's first t rows, upper
// triangular: rows <= c), column c >= t the right coupling column c - t
// (B_i(:, c - t) on the last t rows, lower triangular: rows >= c - t).  The
// right-hand sides come from the compact coupling store, one t x (t+1) pair
// per block (C_i at offset t, B_i at offset 0, leading dimension t).
template <typename T>
__global__ __launch_bounds__(kIluThreads) void k_ilu_spikes(const IluBlock* __restrict__ blocks,
                                                              const int32_t* __restrict__ batch, int t,
                                                              const T* __restrict__ rhs, const int64_t* __restrict__ lo,
                                                              const int64_t* __restrict__ dg,
                                                              const int64_t* __restrict__ hi,
                                                              const int32_t* __restrict__ col,
                                                              const double* __restrict__ fv, T* ws,
                                                              int64_t slot_elems) {
  const int c = blockIdx.y * kIluThreads + threadIdx.x;
  const int t2 = 2 * t;
  if (c >= t2) return;
  const int bi = batch[blockIdx.x];
  const IluBlock B = blocks[bi];
  const bool left = c < t;
  if (left ? !B.left : !B.right) return;
  T* __restrict__ W = ws + (int64_t)blockIdx.x * slot_elems;
  const int64_t pt = (int64_t)t * t + t;
  const T* __restrict__ P = rhs + (int64_t)bi * pt;
  const int64_t n = B.n;
  const int64_t r0 = left ? 0 : n - t;   // rows above r0 stay zero in the forward solve
  const int j = left ? c : c - t;
  // the row just finished (r - 1 down the block, r + 1 up it) is taken from
  // a register, as stored (rounded to T), instead of being loaded back right
  // after its store; the row index is the same in every lane, so the choice
  // does not diverge
  double prev = 0.0;
  for (int64_t r = r0; r < n; ++r) {
    const int64_t R = B.s + r;
    double acc;
    if (left) acc = (r < t && r <= j) ? (double)P[t + (int64_t)j * t + r] : 0.0;
    else {
      const int64_t rr = r - r0;
      acc = rr >= j ? (double)P[(int64_t)j * t + rr] : 0.0;
    }
    const int64_t qe = dg[R];
    for (int64_t q = lo[R]; q < qe; ++q) {
      const int64_t k = col[q] - B.s;
      if (k >= r0) acc -= fv[q] * (k == r - 1 ? prev : (double)W[k * t2 + c]);
    }
    const T y = (T)acc;
    W[r * t2 + c] = y;
    prev = (double)y;
  }
  double next = 0.0;
  for (int64_t r = n - 1; r >= 0; --r) {
    const int64_t R = B.s + r;
    const int64_t d = dg[R];
    double acc = r >= r0 ? (double)W[r * t2 + c] : 0.0;
    for (int64_t q = d + 1; q < hi[R]; ++q) {
      const int64_t k = col[q] - B.s;
      acc -= fv[q] * (k == r + 1 ? next : (double)W[k * t2 + c]);
    }
    const T x = (T)(acc / fv[d]);
    W[r * t2 + c] = x;
    next = (double)x;
  }
}

// Tips of a batch: rows [0, t) of block i's spikes into tip part 2i - 1 and
// rows [n - t, n) into part 2i, each part t x 2t column-major (leading
// dimension t).  64 x 64 tiles through LDS: read along the workspace rows,
// written along the part's columns.  Columns of a coupling the block does
// not have (left of block 0, right of block p-1) are written as zeros.
template <typename T>
__global__ __launch_bounds__(kIluThreads) void k_ilu_tips(const IluBlock* __restrict__ blocks,
                                                            const int32_t* __restrict__ batch, int p, int t,
                                                            const T* __restrict__ ws, int64_t slot_elems,
                                                            T* __restrict__ tips) {
  __shared__ T tile[64][65];
  const int bi = batch[blockIdx.x];
  const IluBlock B = blocks[bi];
  const int part = blockIdx.y;   // 0: top rows, 1: bottom rows
  if (part == 0 ? bi == 0 : bi == p - 1) return;
  const int t2 = 2 * t;
  const int ct = t2 / 64;
  const int tr = blockIdx.z / ct, tc = blockIdx.z % ct;   // tile row (of t / 64), tile column
  const T* __restrict__ W = ws + (int64_t)blockIdx.x * slot_elems;
  const int64_t rbase = part == 0 ? 0 : B.n - t;
  const int64_t q = part == 0 ? 2 * (int64_t)bi - 1 : 2 * (int64_t)bi;
  T* __restrict__ D = tips + q * (int64_t)t2 * t;
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;   // 64 x 4 threads
  for (int rr = ly; rr < 64; rr += 4) {
    const int64_t r = rbase + (int64_t)tr * 64 + rr;
    const int c = tc * 64 + lx;
    const bool have = c < t ? B.left : B.right;
    tile[rr][lx] = have ? W[r * t2 + c] : T(0);
  }
  __syncthreads();
  for (int cc = ly; cc < 64; cc += 4) {
    const int c = tc * 64 + cc;
    const int64_t r = (int64_t)tr * 64 + lx;
    D[(int64_t)c * t + r] = tile[lx][cc];
  }
}

// D~^{-1} y for every block, in place on the padded vector (R columns,
// column stride ldy), one workgroup of kSolveThreads per block: forward
// solve with L~ level by level, then backward with U~.  The solve is bound
// by the latency of its dependent loads (level list -> row -> entries ->
// vector), so each level-ordered slot carries its row's entry range (lq:
// [lo, dg) of the forward order, uq: [dg + 1, hi) of the backward one,
// pivot at uq.x - 1), read together with the row number, and a workgroup
// runs 16 waves; the R lanes of one row are adjacent.  Entries are taken
// four at a time with their loads issued together (columns and values,
// then the vector entries), so a row costs three dependent loads, not two
// per entry.
constexpr int kSolveThreads = 1024;

// acc - sum over q in [q0, q1) of fv[q] * Yc[(col[q] - s) * R]
__device__ __forceinline__ double row_dot(double acc, int64_t q0, int64_t q1, const int32_t* __restrict__ col,
                                          const double* __restrict__ fv, const double* Yc, int64_t s, int R) {
  for (int64_t q = q0; q < q1; q += 4) {
    int64_t c[4];
    double v[4], x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = q + u < q1;
      c[u] = ok ? ((int64_t)col[q + u] - s) * R : 0;
      v[u] = ok ? fv[q + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = q + u < q1 ? Yc[c[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc -= v[u] * x[u];
  }
  return acc;
}
__global__ __launch_bounds__(kSolveThreads) void k_ilu_solve(const IluBlock* __restrict__ blocks,
                                                               const int32_t* __restrict__ lrows,
                                                               const int64_t* __restrict__ lptr,
                                                               const longlong2* __restrict__ lq,
                                                               const int32_t* __restrict__ urows,
                                                               const int64_t* __restrict__ uptr,
                                                               const longlong2* __restrict__ uq,
                                                               const int32_t* __restrict__ col,
                                                               const double* __restrict__ fv, double* y,
                                                               int64_t ldy, int R, double* __restrict__ yt) {
  const IluBlock B = blocks[blockIdx.x];
  // y: entry of global row r in column j at y[j * ldy + vbase + (r - s)].
  // The solves run on a row-major copy (yt + vbase * R, R entries per row),
  // so that the R lanes of a row read one stretch of R doubles.
  double* __restrict__ Yt = yt + B.vbase * R;
  const int64_t nR = B.n * R;
  for (int64_t w = threadIdx.x; w < nR; w += blockDim.x) {
    const int64_t r = w % B.n, j = w / B.n;
    Yt[r * R + j] = y[j * ldy + B.vbase + r];
  }
  __syncthreads();
  for (int64_t lv = 0; lv < B.lnum; ++lv) {
    const int64_t a = lptr[B.lbeg + lv], e = lptr[B.lbeg + lv + 1];
    for (int64_t w = threadIdx.x; w < (e - a) * R; w += blockDim.x) {
      const int64_t j = a + w / R;
      const int64_t r = lrows[j];
      const longlong2 qr = lq[j];
      double* __restrict__ Yc = Yt + (w % R);
      Yc[(r - B.s) * R] = row_dot(Yc[(r - B.s) * R], qr.x, qr.y, col, fv, Yc, B.s, R);
    }
    __syncthreads();
  }
  for (int64_t lv = 0; lv < B.unum; ++lv) {
    const int64_t a = uptr[B.ubeg + lv], e = uptr[B.ubeg + lv + 1];
    for (int64_t w = threadIdx.x; w < (e - a) * R; w += blockDim.x) {
      const int64_t j = a + w / R;
      const int64_t r = urows[j];
      const longlong2 qr = uq[j];
      double* __restrict__ Yc = Yt + (w % R);
      const double piv = fv[qr.x - 1];
      Yc[(r - B.s) * R] = row_dot(Yc[(r - B.s) * R], qr.x, qr.y, col, fv, Yc, B.s, R) / piv;
    }
    __syncthreads();
  }
  for (int64_t w = threadIdx.x; w < nR; w += blockDim.x) {
    const int64_t r = w % B.n, j = w / B.n;
    y[j * ldy + B.vbase + r] = Yt[r * R + j];
  }
}

}  // namespace

void ilu_factor(int p, const IluBlock* blocks, const int32_t* lrows, const int64_t* lptr, const int64_t* lo,
                const int64_t* dg, const int64_t* hi, const int32_t* col, const double* val, double* fv,
                const double* thresh, unsigned long long* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_ilu0, dim3(p), dim3(kIluThreads), 0, s, blocks, lrows, lptr, lo, dg, hi, col, val, fv, thresh,
                     bad);
}

void ilu_spikes(int dtype, int nb, const IluBlock* blocks, const int32_t* batch, int p, int t, const void* rhs,
                const int64_t* lo, const int64_t* dg, const int64_t* hi, const int32_t* col, const double* fv,
                void* ws, int64_t slot_elems, void* tips, hipStream_t s) {
  if (nb <= 0) return;
  const dim3 g1((unsigned)nb, (unsigned)((2 * t + kIluThreads - 1) / kIluThreads));
  const dim3 g2((unsigned)nb, 2u, (unsigned)((t / 64) * (2 * t / 64)));
  if (dtype == 0) {
    hipLaunchKernelGGL(k_ilu_spikes<double>, g1, dim3(kIluThreads), 0, s, blocks, batch, t, (const double*)rhs, lo, dg,
                       hi, col, fv, (double*)ws, slot_elems);
    hipLaunchKernelGGL(k_ilu_tips<double>, g2, dim3(kIluThreads), 0, s, blocks, batch, p, t, (const double*)ws,
                       slot_elems, (double*)tips);
  } else {
    hipLaunchKernelGGL(k_ilu_spikes<float>, g1, dim3(kIluThreads), 0, s, blocks, batch, t, (const float*)rhs, lo, dg,
                       hi, col, fv, (float*)ws, slot_elems);
    hipLaunchKernelGGL(k_ilu_tips<float>, g2, dim3(kIluThreads), 0, s, blocks, batch, p, t, (const float*)ws,
                       slot_elems, (float*)tips);
  }
}

void ilu_solve(int p, const IluBlock* blocks, const int32_t* lrows, const int64_t* lptr, const void* lq,
               const int32_t* urows, const int64_t* uptr, const void* uq, const int32_t* col, const double* fv,
               double* y, int64_t ldy, int R, double* yt, hipStream_t s) {
  hipLaunchKernelGGL(k_ilu_solve, dim3(p), dim3(kSolveThreads), 0, s, blocks, lrows, lptr, (const longlong2*)lq, urows,
                     uptr, (const longlong2*)uq, col, fv, y, ldy, R, yt);
}

}  // namespace ddps
