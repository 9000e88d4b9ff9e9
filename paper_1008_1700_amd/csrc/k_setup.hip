// Stages 1, 3 and 5 of the method on the device: validation and bandwidth of
// the CSR input, the split A = D + R into the tile layout of each block
// (block-tridiagonal t x t tiles, identity padding on top of short blocks),
// the coupling entries of R_i placed as the right-hand sides of the spike
// solves, the column inf-norms of R_i, and the dropping rule that yields the
// index set c (as a 0/1 mask over the candidate coupling columns).
#include "ddps_internal.h"
#include <algorithm>

namespace ddps {

__device__ __forceinline__ int find_block(const int64_t* __restrict__ part, int p, int64_t r) {
  int lo = 0, hi = p - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (part[mid] <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One thread per row; band and flags are reduced inside the workgroup first,
// so only one atomic per workgroup reaches memory.
__global__ __launch_bounds__(256) void k_scan_rows(int64_t n, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, int64_t nnz,
                                                   unsigned long long* __restrict__ band,
                                                   unsigned int* __restrict__ flags) {
  __shared__ unsigned long long sb[256];
  __shared__ unsigned int sf[256];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long bw = 0;
  unsigned int f = 0;
  if (r == 0 && (row_ptr[0] != 0 || row_ptr[n] != nnz)) f |= 1u;
  if (r < n) {
    const int64_t a = row_ptr[r], b = row_ptr[r + 1];
    if (b < a || a < 0 || b > nnz) {
      f |= 1u;
    } else {
      for (int64_t q = a; q < b; ++q) {
        const int64_t c = col[q];
        const double v = val[q];
        if (c < 0 || c >= n) { f |= 2u; continue; }
        if (!isfinite(v)) f |= 4u;
        const unsigned long long d = (unsigned long long)(c > r ? c - r : r - c);
        bw = d > bw ? d : bw;
      }
    }
  }
  const int t = threadIdx.x;
  sb[t] = bw; sf[t] = f;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) {
      sb[t] = sb[t] > sb[t + s2] ? sb[t] : sb[t + s2];
      sf[t] |= sf[t + s2];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (sf[0]) atomicOr(flags, sf[0]);
    atomicMax(band, sb[0]);
  }
}

// Pivot threshold of every row: 1e3 eps max_j |a_rj| over the row's entries
// inside its own block, written at the row's place in the padded layout.  A
// pivot at or below it is numerically zero on the scale of its own row, so
// badly scaled but nonsingular blocks (coefficients over many decades) pass.
__global__ void k_row_thresh(int64_t n, int p, const int64_t* __restrict__ part,
                             const BlockInfo* __restrict__ blocks, const int64_t* __restrict__ row_ptr,
                             const int32_t* __restrict__ col, const double* __restrict__ val, double scale,
                             double* __restrict__ thresh) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const BlockInfo B = blocks[find_block(part, p, r)];
  double mx = 0.0;
  for (int64_t q = row_ptr[r]; q < row_ptr[r + 1]; ++q) {
    const int64_t c = col[q];
    if (c >= B.s && c < B.s + B.n) mx = fmax(mx, fabs(val[q]));
  }
  thresh[B.voff + B.pad + (r - B.s)] = scale * mx;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Zero the parts of the spike array that the scatter fills with coupling
// entries: in block i > 0 the rows [0, min(2t, N)) of the t left-coupling
// columns, in block i < p-1 the last t rows of the t right-coupling columns.
// Every other spike entry the factorisation reads is written by it first.
template <typename T>
__global__ void k_zero_spike_rhs(int p, int t, const BlockInfo* __restrict__ blocks, T* __restrict__ spikes) {
  const int i = blockIdx.x;
  const BlockInfo B = blocks[i];
  T* G = spikes + B.goff;
  const int64_t top_rows = min((int64_t)2 * t, B.N);
  for (int j = blockIdx.y; j < 2 * t; j += gridDim.y) {
    const bool top = j < t;
    if (top ? i == 0 : i == p - 1) continue;
    const int64_t r0 = top ? 0 : B.N - t, r1 = top ? top_rows : B.N;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) G[(int64_t)j * B.N + r] = T(0);
  }
}

// Entries of A into the tile layout of their block: A_kk into diagonal tile
// k, A_{k,k+1} (lower triangular, diagonal included) into the lower half of
// pair k and A_{k+1,k} (upper triangular) into its upper half (a pair is a
// t x (t+1) column-major array holding both triangles: lower(i, j) at
// i + j t, upper(i, j) at i + (j + 1) t).  Coupling entries (columns of the
// neighbouring blocks) become the right-hand sides of the spike solves:
// into the spike array (rhs == null), or into the compact store rhs, one
// pair per block with the left coupling C_i (rows of block i against the
// last t columns of block i-1, upper triangular) in the upper half and the
// right coupling B_i (the last t rows against the first t columns of block
// i+1, lower triangular) in the lower half.
template <typename T>
__global__ void k_scatter(int64_t n, int p, int t, const int64_t* __restrict__ part,
                          const BlockInfo* __restrict__ blocks, const int64_t* __restrict__ row_ptr,
                          const int32_t* __restrict__ col, const double* __restrict__ val,
                          T* __restrict__ tiles, T* __restrict__ spikes, T* __restrict__ rhs,
                          unsigned long long* __restrict__ colnorm, unsigned int* __restrict__ flags) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int blk = find_block(part, p, r);
  const BlockInfo B = blocks[blk];
  const int64_t tt = (int64_t)t * t, pt = tt + t;
  const int64_t lr = B.pad + (r - B.s);
  const int64_t kr = lr / t, rr = lr % t;
  T* __restrict__ G = spikes + B.goff;
  T* __restrict__ W = tiles ? tiles + B.tiles : nullptr;   // null: no tiles (incomplete factors)
  for (int64_t q = row_ptr[r]; q < row_ptr[r + 1]; ++q) {
    const int64_t c = col[q];
    const double v = val[q];
    if (c >= B.s && c < B.s + B.n) {
      const int64_t lc = B.pad + (c - B.s);
      const int64_t kc = lc / t, cc = lc % t;
      int64_t idx;
      if (kc == kr) idx = kr * tt + cc * t + rr;                                    // A_kk
      else if (kc == kr + 1 && rr >= cc) idx = B.T * tt + kr * pt + cc * t + rr;      // A_{k,k+1}
      else if (kc == kr - 1 && rr <= cc) idx = B.T * tt + kc * pt + t + cc * t + rr;  // A_{k+1,k}
      else { atomicOr(flags, 8u); continue; }
      if (W) W[idx] += (T)v;
    } else if (c < B.s) {
      const int64_t jj = c - (B.s - t);
      const int64_t ir = r - B.s;
      if (jj < 0 || ir >= t || ir > jj) { atomicOr(flags, 8u); continue; }
      if (rhs) rhs[(int64_t)blk * pt + t + jj * t + ir] += (T)v;
      else G[jj * B.N + lr] += (T)v;
      atomicMax(&colnorm[(int64_t)blk * 2 * t + jj], (unsigned long long)__double_as_longlong(fabs(v)));
    } else {
      const int64_t jj = c - (B.s + B.n);
      const int64_t ir = r - (B.s + B.n - t);
      if (jj >= t || ir < jj) { atomicOr(flags, 8u); continue; }
      if (rhs) rhs[(int64_t)blk * pt + jj * t + ir] += (T)v;
      else G[(t + jj) * B.N + lr] += (T)v;
      atomicMax(&colnorm[(int64_t)blk * 2 * t + t + jj],
                (unsigned long long)__double_as_longlong(fabs(v)));
    }
  }
}

// Identity rows on top of short blocks (padding): diagonal of tile 0.
template <typename T>
__global__ void k_pad_identity(int /*p*/, int t, const BlockInfo* __restrict__ blocks, T* __restrict__ tiles) {
  const BlockInfo B = blocks[blockIdx.x];
  for (int64_t i = threadIdx.x; i < B.pad; i += blockDim.x)
    tiles[B.tiles + i * t + i] = T(1);
}

// Dropping rule (one workgroup per block): column k of R_i is kept iff
// ||R_i(:,k)||_inf > delta * max_j ||R_i(:,j)||_inf.  Writes the reduced
// mask and clears the right-hand sides of dropped columns.
template <typename T>
__global__ void k_mask(int p, int t, double delta, const BlockInfo* __restrict__ blocks,
                       const unsigned long long* __restrict__ colnorm, double* __restrict__ mask,
                       T* __restrict__ spikes, T* __restrict__ rhs) {
  __shared__ double red[256];
  const int blk = blockIdx.x;
  const BlockInfo B = blocks[blk];
  const unsigned long long* cn = colnorm + (int64_t)blk * 2 * t;
  double mu = 0.0;
  for (int j = threadIdx.x; j < 2 * t; j += blockDim.x) mu = fmax(mu, __longlong_as_double((long long)cn[j]));
  red[threadIdx.x] = mu;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mu = red[0];
  T* G = spikes + B.goff;
  for (int j = threadIdx.x; j < 2 * t; j += blockDim.x) {
    const double nrm = __longlong_as_double((long long)cn[j]);
    const bool keep = nrm > delta * mu;
    const bool top = j < t;
    if (top && blk == 0) continue;
    if (!top && blk == p - 1) continue;
    const int64_t q = top ? (int64_t)2 * (blk - 1) * t + j : (int64_t)(2 * blk + 1) * t + (j - t);
    mask[q] = keep ? 1.0 : 0.0;
    if (!keep && rhs) {
      // column j of C_i (upper half, rows 0..j) or column j - t of B_i
      // (lower half, rows j - t .. t-1) in the compact store
      const int64_t pt = (int64_t)t * t + t;
      T* P = rhs + (int64_t)blk * pt;
      if (top) for (int64_t r = 0; r <= j; ++r) P[t + (int64_t)j * t + r] = T(0);
      else for (int64_t r = j - t; r < t; ++r) P[(int64_t)(j - t) * t + r] = T(0);
    } else if (!keep) {
      const int64_t r0 = top ? 0 : B.N - t;
      const int64_t r1 = top ? min((int64_t)2 * t, B.N) : B.N;
      for (int64_t r = r0; r < r1; ++r) G[(int64_t)j * B.N + r] = T(0);
    }
  }
}

// ------------------------------------------------------------------ launchers
void setup_scan(int64_t n, int p, const int64_t* part, const int64_t* row_ptr, const int32_t* col,
                const double* val, int64_t nnz, unsigned long long* band, unsigned int* flags, hipStream_t s) {
  (void)p;
  (void)part;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)nb), dim3(256), 0, s, n, row_ptr, col, val, nnz, band, flags);
}

void zero_spike_rhs(int dtype, int p, int t, const BlockInfo* blocks, void* spikes, hipStream_t s) {
  if (p <= 1) return;
  const dim3 g((unsigned)p, (unsigned)std::min(2 * t, 512));
  if (dtype == 0) hipLaunchKernelGGL(k_zero_spike_rhs<double>, g, dim3(256), 0, s, p, t, blocks, (double*)spikes);
  else hipLaunchKernelGGL(k_zero_spike_rhs<float>, g, dim3(256), 0, s, p, t, blocks, (float*)spikes);
}

void fill_f64(double* ptr, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return;
  const int64_t nb = std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)nb), dim3(256), 0, s, ptr, count, v);
}
void fill_f32(float* ptr, int64_t count, float v, hipStream_t s) {
  if (count <= 0) return;
  const int64_t nb = std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<float>, dim3((unsigned)nb), dim3(256), 0, s, ptr, count, v);
}
void fill_u64(unsigned long long* ptr, int64_t count, unsigned long long v, hipStream_t s) {
  if (count <= 0) return;
  const int64_t nb = std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<unsigned long long>, dim3((unsigned)nb), dim3(256), 0, s, ptr, count, v);
}

void setup_scatter(int dtype, int64_t n, int p, int t, const int64_t* part, const BlockInfo* blocks,
                   const int64_t* row_ptr, const int32_t* col, const double* val, void* tiles,
                   void* spikes, void* rhs, unsigned long long* colnorm, unsigned int* flags, hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  if (dtype == 0) {
    hipLaunchKernelGGL(k_scatter<double>, dim3((unsigned)nb), dim3(256), 0, s, n, p, t, part, blocks,
                       row_ptr, col, val, (double*)tiles, (double*)spikes, (double*)rhs, colnorm, flags);
    if (tiles) hipLaunchKernelGGL(k_pad_identity<double>, dim3(p), dim3(256), 0, s, p, t, blocks, (double*)tiles);
  } else {
    hipLaunchKernelGGL(k_scatter<float>, dim3((unsigned)nb), dim3(256), 0, s, n, p, t, part, blocks,
                       row_ptr, col, val, (float*)tiles, (float*)spikes, (float*)rhs, colnorm, flags);
    if (tiles) hipLaunchKernelGGL(k_pad_identity<float>, dim3(p), dim3(256), 0, s, p, t, blocks, (float*)tiles);
  }
}

void setup_mask(int dtype, int p, int t, double delta, const BlockInfo* blocks,
                const unsigned long long* colnorm, double* mask, void* spikes, void* rhs, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_mask<double>, dim3(p), dim3(256), 0, s, p, t, delta, blocks, colnorm, mask,
                       (double*)spikes, (double*)rhs);
  else
    hipLaunchKernelGGL(k_mask<float>, dim3(p), dim3(256), 0, s, p, t, delta, blocks, colnorm, mask,
                       (float*)spikes, (float*)rhs);
}

void setup_row_thresh(int64_t n, int p, int64_t Np, const int64_t* part, const BlockInfo* blocks,
                      const int64_t* row_ptr, const int32_t* col, const double* val, double eps, double* thresh,
                      hipStream_t s) {
  fill_f64(thresh, Np, 0.0, s);
  hipLaunchKernelGGL(k_row_thresh, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, part, blocks, row_ptr,
                     col, val, 1e3 * eps, thresh);
}

}  // namespace ddps
