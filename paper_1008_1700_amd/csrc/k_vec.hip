// FP64 vector kernels of the solve phase.
//
//  * gather/scatter between the global row order and the padded block layout;
//  * the gather g^ = g(c) of step 6.2 (mask applied: entries outside c are 0);
//  * unpreconditioned BiCGStab on G^ z^ = g^ (step 6.3) with every scalar kept
//    on the device: kernels write per-workgroup partial sums, a one-workgroup
//    kernel adds them in a fixed order (deterministic results, no
//    cross-workgroup synchronisation inside a kernel), and every consumer
//    recomputes the scalar decisions it needs from those sums.  Per-RHS
//    status words stop finished columns;
//  * CSR residual r = f - A x with inf- and 2-norm partials (outer layer);
//  * linear combinations and dot products for the outer Krylov method.
#include "ddps_internal.h"

namespace ddps {

template <int R>
__device__ __forceinline__ void block_sum(double (&v)[R][2], double (*sh)[R][2]) {
  // sum v over the 256 threads; result valid in thread 0
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      double x = v[j][q];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      v[j][q] = x;
    }
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) { sh[wave][j][0] = v[j][0]; sh[wave][j][1] = v[j][1]; }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
      for (int q = 0; q < 2; ++q) v[j][q] = sh[0][j][q] + sh[1][j][q] + sh[2][j][q] + sh[3][j][q];
}

// Fixed-order reduction of partials laid out [w][R][2] into out[R][2]: one
// workgroup; thread i adds w = i, i + 256, ... in order, then a fixed tree.
template <int R>
__global__ __launch_bounds__(256) void k_reduce2(int W, const double* __restrict__ part,
                                                 double* __restrict__ out,
                                                 const int32_t* __restrict__ stop) {
  __shared__ double sh[4][R][2];
  if (stop) {
    bool all = true;
    for (int j = 0; j < R; ++j) all &= stop[j] != KS_RUNNING;
    if (all) return;
  }
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int w = threadIdx.x; w < W; w += 256)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      acc[j][0] += part[((int64_t)w * R + j) * 2 + 0];
      acc[j][1] += part[((int64_t)w * R + j) * 2 + 1];
    }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) { out[2 * j] = acc[j][0]; out[2 * j + 1] = acc[j][1]; }
}

// First level of a two-level reduction of [w][R][2] partials: workgroup b
// sums the contiguous range w in [b per, (b + 1) per) in fixed order (as
// k_reduce2 does over all of them) into out1[b][R][2].
template <int R>
__global__ __launch_bounds__(256) void k_reduce2_part(int W, int per, const double* __restrict__ part,
                                                      double* __restrict__ out1, const int32_t* __restrict__ stop) {
  __shared__ double sh[4][R][2];
  if (stop) {
    bool all = true;
    for (int j = 0; j < R; ++j) all &= stop[j] != KS_RUNNING;
    if (all) return;
  }
  const int w0 = blockIdx.x * per, w1 = min(W, w0 + per);
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int w = w0 + (int)threadIdx.x; w < w1; w += 256)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      acc[j][0] += part[((int64_t)w * R + j) * 2 + 0];
      acc[j][1] += part[((int64_t)w * R + j) * 2 + 1];
    }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      out1[((int64_t)blockIdx.x * R + j) * 2 + 0] = acc[j][0];
      out1[((int64_t)blockIdx.x * R + j) * 2 + 1] = acc[j][1];
    }
}

__device__ __forceinline__ double sum_of(const double* __restrict__ sums, int j, int q) {
  return sums[2 * j + q];
}

// ------------------------------------------------------------ layout moves
__device__ __forceinline__ int find_voff(const BlockInfo* __restrict__ b, int p, int64_t q) {
  int lo = 0, hi = p - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b[mid].voff <= q) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// R columns of the padded vector; only the first k exist in y, the rest are zeroed
__global__ void k_to_padded(int64_t Np, int R, int k, int p, const BlockInfo* __restrict__ blocks,
                            const double* __restrict__ y, int64_t ldy, double* __restrict__ yp) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < Np;
       q += (int64_t)gridDim.x * blockDim.x) {
    const BlockInfo B = blocks[find_voff(blocks, p, q)];
    const int64_t lr = q - B.voff;
    for (int j = 0; j < R; ++j)
      yp[q + j * Np] = (lr < B.pad || j >= k) ? 0.0 : y[B.s + (lr - B.pad) + j * ldy];
  }
}

// writes the first k columns of y
__global__ void k_from_padded(int64_t Np, int k, int p, const BlockInfo* __restrict__ blocks,
                              const double* __restrict__ yp, double* __restrict__ y, int64_t ldy) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < Np;
       q += (int64_t)gridDim.x * blockDim.x) {
    const BlockInfo B = blocks[find_voff(blocks, p, q)];
    const int64_t lr = q - B.voff;
    if (lr >= B.pad)
      for (int j = 0; j < k; ++j) y[B.s + (lr - B.pad) + j * ldy] = yp[q + j * Np];
  }
}

__global__ void k_gather_reduced(int64_t m, int R, const int64_t* __restrict__ rrow,
                                 const double* __restrict__ mask, const double* __restrict__ gp,
                                 int64_t Np, double* __restrict__ gh) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = rrow[q];
    const double mk = mask[q];
    for (int j = 0; j < R; ++j) gh[q + j * m] = mk * gp[row + j * Np];
  }
}

// ------------------------------------------------------------ reduced BiCGStab
// init: x = masked guess (or 0), r = r~ = p = g^ - G^ x; partials (r.r, g^.g^)
template <int R>
__global__ __launch_bounds__(256) void k_bicg_init(int64_t m, int use_guess, const double* __restrict__ gh,
                                                   double* __restrict__ x, const double* __restrict__ v,
                                                   double* __restrict__ r, double* __restrict__ rt,
                                                   double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[4][R][2];
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t k = i + j * m;
      const double g = gh[k];
      double rr = g;
      if (use_guess) rr -= v[k]; else x[k] = 0.0;
      r[k] = rr; rt[k] = rr; p[k] = rr;
      acc[j][0] += rr * rr;
      acc[j][1] += g * g;
    }
  }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      part[((int64_t)blockIdx.x * R + j) * 2 + 0] = acc[j][0];
      part[((int64_t)blockIdx.x * R + j) * 2 + 1] = acc[j][1];
    }
}

template <int R>
__global__ void k_bicg_init_state(int k, double tol, const double* __restrict__ sums,
                                  KState* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= R) return;
  const double rr = sum_of(sums, j, 0), gg = sum_of(sums, j, 1);
  const double ref = gg > 0.0 ? sqrt(gg) : 1.0;
  st->ref[j] = ref;
  st->rho[1][j] = rr;
  st->alpha[j] = 0.0;
  st->omega[j] = 0.0;
  const double res = sqrt(rr) / ref;
  st->res[j] = res;
  st->iters2[j] = 0;
  st->status[1][j] = (j >= k) ? KS_UNUSED : (res <= tol ? KS_CONVERGED : KS_RUNNING);
}

// Decisions of iteration `it` for column j, identical in every workgroup:
// they depend only on the status at the start of the iteration
// (status[it & 1], never written during the iteration) and reduced sums.
__device__ __forceinline__ bool s_ok(const KState* st, int it, int j, double rtv, double& alpha) {
  alpha = st->rho[it & 1][j] / rtv;
  return st->status[it & 1][j] == KS_RUNNING && rtv != 0.0 && isfinite(alpha);
}

// s = r - alpha v, alpha = rho / (r~.v); partial s.s
template <int R>
__global__ __launch_bounds__(256) void k_bicg_s(int it, int64_t m, const double* __restrict__ s1,
                                                KState* __restrict__ st, const double* __restrict__ r,
                                                const double* __restrict__ v, double* __restrict__ s,
                                                double* __restrict__ part) {
  __shared__ double sh[4][R][2];
  double al[R];
  bool run[R];
  bool any = false;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    run[j] = s_ok(st, it, j, sum_of(s1, j, 0), al[j]);
    any |= run[j];
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) st->alpha[j] = al[j];
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  if (any)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (run[j]) {
          const int64_t k = i + j * m;
          const double sv = r[k] - al[j] * v[k];
          s[k] = sv;
          acc[j][0] += sv * sv;
        }
    }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      part[((int64_t)blockIdx.x * R + j) * 2 + 0] = acc[j][0];
      part[((int64_t)blockIdx.x * R + j) * 2 + 1] = 0.0;
    }
}

// half-step test on ||s||: x += alpha p; otherwise omega = t.s / t.t,
// x += alpha p + omega s, r = s - omega t; partials (r.r, r~.r)
template <int R>
__global__ __launch_bounds__(256) void k_bicg_xr(int it, int64_t m, double tol, const double* __restrict__ s1,
                                                 const double* __restrict__ s2,
                                                 const double* __restrict__ s3,
                                                 KState* __restrict__ st, double* __restrict__ x,
                                                 const double* __restrict__ /*p: the update uses px*/,
                                                 const double* __restrict__ s,
                                                 const double* __restrict__ t, double* __restrict__ r,
                                                 const double* __restrict__ rt, double* __restrict__ part,
                                                 const double* __restrict__ px, const double* __restrict__ sx) {
  // px, sx: the directions added to x (M^{-1}p, M^{-1}s when preconditioned, else p, s)
  __shared__ double sh[4][R][2];
  double al[R], om[R];
  bool run[R], half[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const bool ok = s_ok(st, it, j, sum_of(s1, j, 0), al[j]);
    const double ts = sum_of(s3, j, 0), tt = sum_of(s3, j, 1);
    half[j] = ok && sqrt(sum_of(s2, j, 0)) / st->ref[j] <= tol;
    run[j] = ok && !half[j];
    om[j] = tt != 0.0 ? ts / tt : 0.0;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) st->omega[j] = om[j];
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t k = i + j * m;
      if (half[j]) {
        x[k] += al[j] * px[k];
      } else if (run[j]) {
        const double sv = s[k];
        x[k] += al[j] * px[k] + om[j] * sx[k];
        const double rv = sv - om[j] * t[k];
        r[k] = rv;
        acc[j][0] += rv * rv;
        acc[j][1] += rt[k] * rv;
      }
    }
  }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      part[((int64_t)blockIdx.x * R + j) * 2 + 0] = acc[j][0];
      part[((int64_t)blockIdx.x * R + j) * 2 + 1] = acc[j][1];
    }
}

// End of iteration `it`: every decision of the iteration is re-derived from
// the reduced sums, the next status is written to status[(it+1) & 1], and
// p = r + beta (p - omega v) for the columns that continue.
template <int R>
__global__ __launch_bounds__(256) void k_bicg_p(int it, int maxit, int64_t m, double tol,
                                                const double* __restrict__ s1,
                                                const double* __restrict__ s2,
                                                const double* __restrict__ s3,
                                                const double* __restrict__ s4,
                                                KState* __restrict__ st, const double* __restrict__ r,
                                                double* __restrict__ p, const double* __restrict__ v) {
  double be[R], om[R], rho_new[R], res[R];
  int32_t nst[R], it2[R];
  bool cont[R];
  bool any = false;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double al;
    const int32_t st0 = st->status[it & 1][j];
    const bool ok = s_ok(st, it, j, sum_of(s1, j, 0), al);
    const double ref = st->ref[j];
    const double ress = sqrt(sum_of(s2, j, 0)) / ref;
    const double ts = sum_of(s3, j, 0), tt = sum_of(s3, j, 1);
    om[j] = tt != 0.0 ? ts / tt : 0.0;
    rho_new[j] = sum_of(s4, j, 1);
    const double rho_old = st->rho[it & 1][j];
    be[j] = (rho_new[j] / rho_old) * (al / om[j]);
    res[j] = st->res[j];
    it2[j] = st->iters2[j];
    if (st0 != KS_RUNNING) {
      nst[j] = st0;
    } else if (!ok) {
      nst[j] = KS_BREAKDOWN;
    } else if (ress <= tol) {
      nst[j] = KS_CONVERGED; it2[j] = 2 * it - 1; res[j] = ress;
    } else {
      res[j] = sqrt(sum_of(s4, j, 0)) / ref;
      it2[j] = 2 * it;
      if (res[j] <= tol) nst[j] = KS_CONVERGED;
      else if (om[j] == 0.0 || rho_new[j] == 0.0 || !isfinite(be[j])) nst[j] = KS_BREAKDOWN;
      else if (it >= maxit) nst[j] = KS_MAXIT;
      else nst[j] = KS_RUNNING;
    }
    cont[j] = nst[j] == KS_RUNNING;
    any |= cont[j];
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      st->status[(it + 1) & 1][j] = nst[j];
      st->rho[(it + 1) & 1][j] = rho_new[j];
      st->iters2[j] = it2[j];
      st->res[j] = res[j];
    }
  if (!any) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (cont[j]) {
        const int64_t k = i + j * m;
        p[k] = r[k] + be[j] * (p[k] - om[j] * v[k]);
      }
  }
}

// restart after a breakdown: r~ = r, p = r for the flagged columns
template <int R>
__global__ __launch_bounds__(256) void k_bicg_restart(int64_t m, const int32_t* __restrict__ flag,
                                                      const double* __restrict__ r, double* __restrict__ rt,
                                                      double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[4][R][2];
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (flag[j]) {
        const int64_t k = i + j * m;
        const double rv = r[k];
        rt[k] = rv; p[k] = rv;
        acc[j][0] += rv * rv;
      }
  }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      part[((int64_t)blockIdx.x * R + j) * 2 + 0] = acc[j][0];
      part[((int64_t)blockIdx.x * R + j) * 2 + 1] = 0.0;
    }
}

// the next iteration is it + 1: its rho and status slots are (it + 1) & 1
template <int R>
__global__ void k_bicg_restart_state(int it, const int32_t* __restrict__ flag,
                                     const double* __restrict__ sums, KState* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= R || !flag[j]) return;
  st->rho[(it + 1) & 1][j] = sum_of(sums, j, 0);
  st->status[(it + 1) & 1][j] = KS_RUNNING;
}

// ------------------------------------------------------------ outer layer
// r = f - A x for R columns; partials (max|r|, sum r^2, max|f|, sum f^2).
// f = null gives r = A x; row_ptr = null gives r = f (norms of f only).
template <int R>
__global__ __launch_bounds__(256) void k_csr_resid(int64_t n, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x, int64_t ldx,
                                                   const double* __restrict__ f, int64_t ldf,
                                                   double* __restrict__ r, int64_t ldr,
                                                   double* __restrict__ part) {
  __shared__ double sh[4][R][4];
  double mx[R], ss[R], mf[R], sf[R];
#pragma unroll
  for (int j = 0; j < R; ++j) mx[j] = ss[j] = mf[j] = sf[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    if (row_ptr) {
      const int64_t a = row_ptr[i], b = row_ptr[i + 1];
      for (int64_t q = a; q < b; ++q) {
        const double v = val[q];
        const int64_t c = col[q];
#pragma unroll
        for (int j = 0; j < R; ++j) acc[j] += v * x[c + j * ldx];
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const double fv = f ? f[i + j * ldf] : 0.0;
      const double rv = f ? fv - acc[j] : acc[j];
      if (r) r[i + j * ldr] = rv;
      mx[j] = fmax(mx[j], fabs(rv));
      ss[j] += rv * rv;
      mf[j] = fmax(mf[j], fabs(fv));
      sf[j] += fv * fv;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    for (int off = 32; off > 0; off >>= 1) {
      mx[j] = fmax(mx[j], __shfl_xor(mx[j], off, 64));
      ss[j] += __shfl_xor(ss[j], off, 64);
      mf[j] = fmax(mf[j], __shfl_xor(mf[j], off, 64));
      sf[j] += __shfl_xor(sf[j], off, 64);
    }
    if (lane == 0) { sh[wave][j][0] = mx[j]; sh[wave][j][1] = ss[j]; sh[wave][j][2] = mf[j]; sh[wave][j][3] = sf[j]; }
  }
  __syncthreads();
  if (threadIdx.x < R) {
    const int j = threadIdx.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int w = 0; w < 4; ++w) {
      a0 = fmax(a0, sh[w][j][0]); a1 += sh[w][j][1]; a2 = fmax(a2, sh[w][j][2]); a3 += sh[w][j][3];
    }
    double* o = part + ((int64_t)blockIdx.x * R + j) * 4;
    o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3;
  }
}

// Right-hand side of the re-solved retrieval (step 6.5 written as
// z = D~^{-1}(y - R~ z)): yp = y - R~ z in the padded block layout, for k of
// R columns (columns k..R-1 and the padding rows are zero).  R~ z takes the
// off-block entries of each row of A against the reduced solution z^ (the
// candidate layout: interface j owns the 2t columns [s_{j+1} - t,
// s_{j+1} + t), t after the end of block j), masked to the index set c, so
// that dropped columns of R do not contribute.
template <int R>
__global__ __launch_bounds__(256) void k_coupling_rhs(int64_t Np, int p, int t, int k,
                                                      const BlockInfo* __restrict__ blocks,
                                                      const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ y, int64_t ldy,
                                                      const double* __restrict__ zh, int64_t m,
                                                      const double* __restrict__ mask, double* __restrict__ yp) {
  for (int64_t pr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pr < Np;
       pr += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = p - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (blocks[mid].voff <= pr) lo = mid; else hi = mid - 1;
    }
    const BlockInfo B = blocks[lo];
    const int64_t lr = pr - B.voff;
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    if (lr >= B.pad) {
      const int64_t r = B.s + (lr - B.pad);
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (j < k) acc[j] = y[r + j * ldy];
      for (int64_t q = row_ptr[r]; q < row_ptr[r + 1]; ++q) {
        const int64_t c = col[q];
        int64_t idx;
        if (c < B.s) idx = (int64_t)2 * (lo - 1) * t + (c - (B.s - t));
        else if (c >= B.s + B.n) idx = (int64_t)2 * lo * t + t + (c - (B.s + B.n));
        else continue;
        const double w = val[q] * mask[idx];
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (j < k) acc[j] -= w * zh[idx + j * m];
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) yp[pr + j * Np] = acc[j];
  }
}

// yout = yin -/+ (parts[0] + ... + parts[ns-1]) over `rows` entries of R
// columns (column stride ld; part s at parts + s * pstride), summed in that
// fixed order: the split-column products of the direct reduced solve.
__global__ __launch_bounds__(256) void k_sum_parts(int rows, int R, int ns, const double* __restrict__ parts,
                                                   int64_t pstride, int64_t ld, const double* yin, double* yout,
                                                   int neg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  for (int j = 0; j < R; ++j) {
    double acc = 0.0;
    for (int q = 0; q < ns; ++q) acc += parts[q * pstride + i + j * ld];
    const double base = yin ? yin[i + j * ld] : 0.0;
    yout[i + j * ld] = neg ? base - acc : base + acc;
  }
}

// Reduce [W][R][4] residual partials to out[R][4] (max, sum, max, sum).
template <int R>
__global__ void k_resid_reduce(int W, const double* __restrict__ part, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= R) return;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int w = 0; w < W; ++w) {
    const double* o = part + ((int64_t)w * R + j) * 4;
    a0 = fmax(a0, o[0]); a1 += o[1]; a2 = fmax(a2, o[2]); a3 += o[3];
  }
  out[j * 4 + 0] = a0; out[j * 4 + 1] = a1; out[j * 4 + 2] = a2; out[j * 4 + 3] = a3;
}

// out = a X + b Y + c Z (per column coefficients); Z may be null
template <int R>
__global__ void k_lincomb(int64_t n, Coef3 cf, const double* X, const double* Y, const double* Z,
                          double* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t k = i + j * n;
      double v = cf.a[j] * X[k];
      if (Y) v += cf.b[j] * Y[k];
      if (Z) v += cf.c[j] * Z[k];
      out[k] = v;
    }
  }
}

// partial dot products of up to two vector pairs; [W][R][2]
template <int R>
__global__ __launch_bounds__(256) void k_dot2(int64_t n, const double* __restrict__ a0,
                                              const double* __restrict__ b0, const double* __restrict__ a1,
                                              const double* __restrict__ b1, double* __restrict__ part) {
  __shared__ double sh[4][R][2];
  double acc[R][2];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t k = i + j * n;
      acc[j][0] += a0[k] * b0[k];
      if (a1) acc[j][1] += a1[k] * b1[k];
    }
  }
  block_sum<R>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      part[((int64_t)blockIdx.x * R + j) * 2 + 0] = acc[j][0];
      part[((int64_t)blockIdx.x * R + j) * 2 + 1] = acc[j][1];
    }
}


// x *= mask (entries outside the index set c are not unknowns)
__global__ void k_apply_mask(int64_t m, int R, const double* __restrict__ mask, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int j = 0; j < R; ++j) x[i + j * m] *= mask[i];
}

// ------------------------------------------------------------ launchers
#define DDPS_R_DISPATCH(R_, CALL) \
  switch (R_) {                   \
    case 1: { constexpr int RR = 1; CALL; } break; \
    case 2: { constexpr int RR = 2; CALL; } break; \
    case 4: { constexpr int RR = 4; CALL; } break; \
    default: { constexpr int RR = 8; CALL; } break; \
  }

static inline unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kVecGrid));
}

void vec_to_padded(int64_t Np, int R, int k, int p, const BlockInfo* blocks, const double* y, int64_t ldy,
                   double* yp, hipStream_t s) {
  hipLaunchKernelGGL(k_to_padded, dim3(grid_for(Np)), dim3(256), 0, s, Np, R, k, p, blocks, y, ldy, yp);
}
void vec_from_padded(int64_t Np, int k, int p, const BlockInfo* blocks, const double* yp, double* y,
                     int64_t ldy, hipStream_t s) {
  hipLaunchKernelGGL(k_from_padded, dim3(grid_for(Np)), dim3(256), 0, s, Np, k, p, blocks, yp, y, ldy);
}
void vec_gather_reduced(int64_t m, int R, const int64_t* rrow, const double* mask, const double* gp,
                        int64_t Np, double* gh, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_reduced, dim3(grid_for(m)), dim3(256), 0, s, m, R, rrow, mask, gp, Np, gh);
}

int vec_grid(int64_t n) { return (int)grid_for(n); }

void vec_apply_mask(int64_t m, int R, const double* mask, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_mask, dim3(grid_for(m)), dim3(256), 0, s, m, R, mask, x);
}

void reduce2(int R, int W, const double* part, double* out, const int32_t* stop, hipStream_t s, double* scratch) {
  if (scratch && W > kReduceSplit) {
    // one workgroup cannot stream many thousand partials quickly: first
    // kReduceGroups workgroups over contiguous ranges, then one over theirs
    const int per = (W + kReduceGroups - 1) / kReduceGroups;
    const int G = (W + per - 1) / per;
    DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_reduce2_part<RR>, dim3(G), dim3(256), 0, s, W, per, part, scratch, stop));
    DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_reduce2<RR>, dim3(1), dim3(256), 0, s, G, scratch, out, stop));
    return;
  }
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_reduce2<RR>, dim3(1), dim3(256), 0, s, W, part, out, stop));
}
void bicg_init(int R, int64_t m, int use_guess, const double* gh, double* x, const double* v, double* r,
               double* rt, double* p, double* part, int W, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_init<RR>, dim3(W), dim3(256), 0, s, m, use_guess, gh, x, v, r, rt, p, part));
}
void bicg_init_state(int R, int k, double tol, const double* sums, KState* st, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_init_state<RR>, dim3(1), dim3(64), 0, s, k, tol, sums, st));
}
void bicg_s(int R, int it, int64_t m, const double* s1, KState* st, const double* r, const double* v,
            double* sv, double* part, int W, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_s<RR>, dim3(W), dim3(256), 0, s, it, m, s1, st, r, v, sv, part));
}
void bicg_xr(int R, int it, int64_t m, double tol, const double* s1, const double* s2, const double* s3,
             KState* st, double* x, const double* p, const double* sv, const double* t, double* r,
             const double* rt, double* part, int W, hipStream_t s, const double* px, const double* sx) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_xr<RR>, dim3(W), dim3(256), 0, s, it, m, tol, s1, s2, s3, st, x, p, sv, t, r, rt, part,
                                        px ? px : p, sx ? sx : sv));
}
void bicg_p(int R, int it, int maxit, int64_t m, double tol, const double* s1, const double* s2,
            const double* s3, const double* s4, KState* st, const double* r, double* p, const double* v,
            int W, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_p<RR>, dim3(W), dim3(256), 0, s, it, maxit, m, tol, s1, s2, s3, s4, st, r, p, v));
}
void bicg_restart(int R, int it, int64_t m, const int32_t* flag, const double* r, double* rt, double* p,
                  double* part, int W, double* sums, KState* st, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_restart<RR>, dim3(W), dim3(256), 0, s, m, flag, r, rt, p, part));
  reduce2(R, W, part, sums, nullptr, s);
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_bicg_restart_state<RR>, dim3(1), dim3(64), 0, s, it, flag, sums, st));
}
void csr_resid(int R, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
               const double* x, int64_t ldx, const double* f, int64_t ldf, double* r, int64_t ldr,
               double* part, int W, double* out, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_csr_resid<RR>, dim3(W), dim3(256), 0, s, n, row_ptr, col, val, x, ldx, f, ldf, r, ldr, part));
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_resid_reduce<RR>, dim3(1), dim3(64), 0, s, W, part, out));
}
// Residual norms of k <= 8 columns in column groups of 8, 4, 2 and 1 (the
// kernels' widths), each group through the same two kernels as the outer
// layer; part holds [W][8][4] partials, out [k][4] (device).
void residual_norms_cols(int64_t n, int k, const int64_t* row_ptr, const int32_t* col, const double* val,
                         const double* X, int64_t ldx, const double* F, int64_t ldf, double* R, int64_t ldr,
                         double* part, double* out, hipStream_t s) {
  const int W = (int)grid_for(n);
  int j0 = 0;
  while (j0 < k) {
    const int rest = k - j0;
    const int g = rest >= 8 ? 8 : rest >= 4 ? 4 : rest >= 2 ? 2 : 1;
    csr_resid(g, n, row_ptr, col, val, X + (int64_t)j0 * ldx, ldx, F + (int64_t)j0 * ldf, ldf,
              R ? R + (int64_t)j0 * ldr : nullptr, ldr, part, W, out + 4 * j0, s);
    j0 += g;
  }
}
void coupling_rhs(int64_t Np, int R, int k, int p, int t, const BlockInfo* blocks, const int64_t* row_ptr,
                  const int32_t* col, const double* val, const double* y, int64_t ldy, const double* zh, int64_t m,
                  const double* mask, double* yp, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_coupling_rhs<RR>, dim3(grid_for(Np)), dim3(256), 0, s, Np, p, t, k, blocks,
                                        row_ptr, col, val, y, ldy, zh, m, mask, yp));
}
void sum_parts(int rows, int R, int ns, const double* parts, int64_t pstride, int64_t ld, const double* yin,
               double* yout, int neg, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3((rows + 255) / 256), dim3(256), 0, s, rows, R, ns, parts, pstride, ld, yin,
                     yout, neg);
}
void lincomb(int R, int64_t n, const Coef3& cf, const double* X, const double* Y, const double* Z,
             double* out, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_lincomb<RR>, dim3(grid_for(n)), dim3(256), 0, s, n, cf, X, Y, Z, out));
}
void dot2(int R, int64_t n, const double* a0, const double* b0, const double* a1, const double* b1,
          double* part, int W, double* out, hipStream_t s) {
  DDPS_R_DISPATCH(R, hipLaunchKernelGGL(k_dot2<RR>, dim3(W), dim3(256), 0, s, n, a0, b0, a1, b1, part));
  reduce2(R, W, part, out, nullptr, s);
}

}  // namespace ddps
