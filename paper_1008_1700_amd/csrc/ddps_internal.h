// Internal declarations shared by the host runtime (ddps.cpp) and the HIP
// kernels.  Every bulk operation is launched as a "grouped" kernel: the host
// builds, once per handle, a list of problem descriptors in device memory
// (one descriptor per block and operand set), and a launch processes a
// contiguous range of that list.  The factorisation and the solve phase are
// fixed sequences of such launches (schedules), so they can be replayed and
// captured in a HIP graph unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddps {

// Tile edge of the grouped GEMM and of the diagonal-tile LU panel.  The
// coupling tile size t is always a multiple of this.
constexpr int kTile = 64;

// ---------------------------------------------------------------- GEMM
// D = C0 (+|-) op(A) op(B), column-major, M, N multiples of 64, K multiple of
// 64 (K = 0 makes the problem a copy D = C0).
enum GemmFlag : int32_t {
  G_NEG = 1,      // D = C0 - A B   (else C0 + A B; without G_C0: D = -AB / AB)
  G_C0 = 2,       // C0 is read
  G_A_UP = 4,     // A upper triangular: only k >= row contributes
  G_A_LO = 8,     // A lower triangular: only k <= row contributes
  G_B_UP = 16,    // B upper triangular: only k <= col contributes
  G_B_LO = 32,    // B lower triangular: only k >= col contributes
  G_A_MLU = 64,   // A read as unit lower: strictly-lower entries, 1 on the diagonal, 0 above
  G_A_MUP = 128,  // A read as upper: entries on/above the diagonal, 0 below
  G_B_MLU = 256,
  G_B_MUP = 512,
  G_A_MLO = 1024, // A read as lower: entries on/below the diagonal, 0 above
  G_B_MLO = 2048,
  G_D_UP = 4096,  // store only the entries of D on/above the diagonal
  G_D_LO = 8192,  // store only the entries of D on/below the diagonal
};

struct GemmProb {
  const void* A;
  const void* B;
  const void* C0;
  void* D;
  int32_t M, N, K;
  int32_t lda, ldb, ldc0, ldd;
  int32_t flags;
  int32_t tile0;  // first workgroup of this problem within its launch
  int32_t pad_;
};

// ---------------------------------------------------------------- panel LU
// In-place unpivoted LU of a 64 x 64 diagonal sub-tile followed by the
// inversion of both triangles: on exit the strictly-lower part holds
// L^{-1} (unit diagonal implied) and the upper part U^{-1}.
struct PanelProb {
  void* D;        // first element of the 64 x 64 sub-tile
  int32_t ld;
  int32_t block;  // block index (error report)
  int64_t row0;   // global row of the sub-tile's first row (may be < block start: padding)
  int64_t vrow0;  // the same row in the padded layout (indexes the per-row pivot thresholds)
};

// ---------------------------------------------------------------- GEMV
// y_out(rows) = y_in (+|-) A(rows, cb:ce) x  for R right-hand sides.
// Columns [0, split) multiply x1[c], columns [split, ...) multiply x2[c-split].
enum GemvFlag : int32_t {
  V_NEG = 1,
  V_YIN = 2,      // y_in is read (else treated as 0)
  V_A_MLU = 4,    // A read as unit lower (masked)
  V_A_MUP = 8,    // A read as upper (masked)
  V_MASK = 16,    // the product is multiplied row-wise by mask[] before accumulation
  V_DOT = 32,     // emit per-workgroup partials [wg][R][2] of dot(dotv, y_out) (reduced space)
  V_DOT2 = 64,    // ... and of dot(y_out, y_out) in the second slot
  V_A_MLO = 128,  // A read as lower (masked), diagonal included
};

struct GemvProb {
  const void* A;
  int64_t lda;
  const double* x1;
  const double* x2;
  const double* yin;
  double* yout;
  const double* mask;   // indexed like yout rows
  int64_t dot_off;      // offset of these output rows inside the reduced vector (V_DOT)
  int32_t rows;         // multiple of 64
  int32_t split;
  int32_t cb, ce;       // column range [cb, ce) (further narrowed per slab by the masks)
  int32_t row_skip;     // output rows < row_skip are computed but not written (padding)
  int32_t flags;
  int32_t wg0;          // first workgroup of this problem within its launch
  int32_t tri;          // 0 dense, 1 lower (cols <= row), 2 upper (cols >= row): skip ranges
};

// ---------------------------------------------------------------- layout
// Block i owns global rows [s, s+n).  It is padded on top with `pad` identity
// rows to N = T t rows; padded row pad + j is global row s + j.  Its tiles
// start at element `tiles` of the tile array: the T diagonal tiles A_kk
// (later the inverse factors), t x t each, then T-1 pairs of t x (t+1)
// elements, pair k holding A_{k,k+1} (lower triangular) at offset 0 and
// A_{k+1,k} (upper triangular) at offset t, both with leading dimension t.
// Its spike matrix (N x 2t, leading dimension N) starts at element `goff` of
// the spike array (of its workspace slot when only the tips are kept);
// padded vectors of block i start at `voff`.
struct BlockInfo {
  int64_t s, n, pad, N, T;
  int64_t tiles;
  int64_t goff;
  int64_t voff;
};

// ---------------------------------------------------------------- ILU(0) blocks
// Block of the incomplete-factor form: global rows [s, s + n), the padded
// vector index of row s (vbase), its forward levels (rows lrows[lptr[lbeg +
// l] .. lptr[lbeg + l + 1]) for l < lnum) and backward levels (urows, uptr,
// ubeg, unum), and whether it has a left / right coupling.
struct IluBlock {
  int64_t s, n, vbase;
  int64_t lbeg, lnum, ubeg, unum;
  int32_t left, right;
};
// ILU(0) of every block (values from val into fv at the CSR positions),
// pivots checked against thresh (padded layout) into bad.
void ilu_factor(int p, const IluBlock* blocks, const int32_t* lrows, const int64_t* lptr, const int64_t* lo,
                const int64_t* dg, const int64_t* hi, const int32_t* col, const double* val, double* fv,
                const double* thresh, unsigned long long* bad, hipStream_t s);
// Spike columns of the nb blocks listed in batch (block b in workspace slot
// b: n x 2t row-major, slot_elems apart) from the compact coupling store
// rhs, then their tips into the column-major tip store; dtype 0 double,
// 1 float (rhs, ws and tips alike).
void ilu_spikes(int dtype, int nb, const IluBlock* blocks, const int32_t* batch, int p, int t, const void* rhs,
                const int64_t* lo, const int64_t* dg, const int64_t* hi, const int32_t* col, const double* fv,
                void* ws, int64_t slot_elems, void* tips, hipStream_t s);
// y = D~^{-1} y in place on the padded vector (R columns, stride ldy).
// lq / uq: int64 pairs per level-ordered slot of lrows / urows, the entry
// range of that row's L~ part [lo, dg) / of its U~ part [dg + 1, hi).
// yt: work vector of the same size as y (ldy * R doubles, ldy >= padded rows).
void ilu_solve(int p, const IluBlock* blocks, const int32_t* lrows, const int64_t* lptr, const void* lq,
               const int32_t* urows, const int64_t* uptr, const void* uq, const int32_t* col, const double* fv,
               double* y, int64_t ldy, int R, double* yt, hipStream_t s);

// ---------------------------------------------------------------- Krylov state
constexpr int kMaxRhs = 8;
constexpr int kVecGrid = 1024;  // workgroups of the grid-stride vector kernels
enum KStatus : int32_t {
  KS_RUNNING = 0,
  KS_CONVERGED = 1,
  KS_BREAKDOWN = 2,
  KS_MAXIT = 3,
  KS_UNUSED = 4,   // padding column of a multi-RHS batch
};
// Device-resident scalars of the reduced BiCGStab, one column per RHS.  A
// field written by workgroup 0 of a kernel is read only by later kernels.
// rho and status of iteration `it` live in slot it & 1: slot it & 1 is
// read-only during iteration it and the iteration's last kernel writes the
// other slot.
struct KState {
  double ref[kMaxRhs];       // ||g^||_2 (1 if zero)
  double rho[2][kMaxRhs];    // rho of iteration it in slot it & 1
  double alpha[kMaxRhs];
  double omega[kMaxRhs];
  double res[kMaxRhs];       // last relative residual
  int32_t status[2][kMaxRhs];
  int32_t iters2[kMaxRhs];   // iterations counted in half steps
};

struct Coef3 {
  double a[kMaxRhs], b[kMaxRhs], c[kMaxRhs];
};

// Launch wrappers (kernels are in the .hip files).  `stream` is the handle's
// stream; the problem arrays live in device memory.
// order (device, may be null): logical tile of each workgroup slot, a
// permutation of [0, nwg) (longest K range first within each XCD's range)
void launch_gemm(int dtype, int mode, const GemmProb* probs, int nprob, int nwg, hipStream_t s,
                 const int32_t* order = nullptr);
void gemm_tile_shape(int dtype, int mode, int* bm, int* bn);
void launch_panel(int dtype, const PanelProb* probs, int nprob, const double* thresh,
                  unsigned long long* bad, hipStream_t s);
// form 0: plain (k_gemv); 1: every problem's A and column stride are 16-byte
// aligned (k_gemv_w); 2: aligned, and for FP32 operands with 4 or more
// right-hand sides run on the FP32 matrix cores with FP32 sums (k_gemv_mf32),
// otherwise as form 1
void launch_gemv(int dtype, int nrhs, int form, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                 int64_t ldy, const double* dotv, double* partial, const int32_t* stop, hipStream_t s);
// reduced-matrix product on the packed tips (same records as launch_gemv,
// A = first packed row, lda = 2t; nrhs 1 or 2; nseg from tipmv_segments, 0 if
// 2t is too long for the register-held right-hand side) and the packing of
// the tips after a factorisation
int tipmv_segments(int dtype, int t);
void launch_tipmv(int dtype, int nrhs, int nseg, const GemvProb* probs, int nprob, int nwg, int64_t ldx,
                  int64_t ldy, const double* dotv, double* partial, const int32_t* stop, hipStream_t s);
void pack_tips(int dtype, int p, int t, const BlockInfo* blocks, const void* spikes, void* tips, hipStream_t s);

void setup_scan(int64_t n, int p, const int64_t* part, const int64_t* row_ptr, const int32_t* col,
                const double* val, int64_t nnz, unsigned long long* band, unsigned int* flags, hipStream_t s);
// rhs: null (coupling entries into the spike array) or the compact store of
// one t x (t+1) pair per block (left coupling in the upper half, right
// coupling in the lower half)
void setup_scatter(int dtype, int64_t n, int p, int t, const int64_t* part, const BlockInfo* blocks,
                   const int64_t* row_ptr, const int32_t* col, const double* val, void* tiles,
                   void* spikes, void* rhs, unsigned long long* colnorm, unsigned int* flags, hipStream_t s);
void setup_mask(int dtype, int p, int t, double delta, const BlockInfo* blocks,
                const unsigned long long* colnorm, double* mask, void* spikes, void* rhs, hipStream_t s);
// Pivot thresholds per row of the padded layout (Np entries): 1e3 eps times the
// row's largest in-block magnitude; 0 on padding rows.
void setup_row_thresh(int64_t n, int p, int64_t Np, const int64_t* part, const BlockInfo* blocks,
                      const int64_t* row_ptr, const int32_t* col, const double* val, double eps, double* thresh,
                      hipStream_t s);
// zero the coupling (right-hand side) parts of every block's spikes, which
// the scatter fills; the rest of the spike array is written by the
// factorisation before it is read, once the whole array has been zeroed once
void zero_spike_rhs(int dtype, int p, int t, const BlockInfo* blocks, void* spikes, hipStream_t s);
void fill_f64(double* ptr, int64_t count, double v, hipStream_t s);
void fill_f32(float* ptr, int64_t count, float v, hipStream_t s);
void fill_u64(unsigned long long* ptr, int64_t count, unsigned long long v, hipStream_t s);

// y holds k <= R columns (leading dimension ldy); the padded vector has R,
// and its columns k..R-1 are zeroed.  from_padded writes k columns of y.
void vec_to_padded(int64_t Np, int R, int k, int p, const BlockInfo* blocks, const double* y, int64_t ldy,
                   double* yp, hipStream_t s);
void vec_from_padded(int64_t Np, int k, int p, const BlockInfo* blocks, const double* yp, double* y,
                     int64_t ldy, hipStream_t s);
void vec_gather_reduced(int64_t m, int R, const int64_t* rrow, const double* mask, const double* gp,
                        int64_t Np, double* gh, hipStream_t s);
int vec_grid(int64_t n);
void vec_apply_mask(int64_t m, int R, const double* mask, double* x, hipStream_t s);
// sums of [W][R][2] partials into out[R][2] in a fixed order; with scratch
// (kReduceGroups x R x 2 doubles) and W > kReduceSplit in two levels
constexpr int kReduceSplit = 4096;
constexpr int kReduceGroups = 64;
void reduce2(int R, int W, const double* part, double* out, const int32_t* stop, hipStream_t s,
             double* scratch = nullptr);
void bicg_init(int R, int64_t m, int use_guess, const double* gh, double* x, const double* v, double* r,
               double* rt, double* p, double* part, int W, hipStream_t s);
void bicg_init_state(int R, int k, double tol, const double* sums, KState* st, hipStream_t s);
void bicg_s(int R, int it, int64_t m, const double* s1, KState* st, const double* r, const double* v,
            double* sv, double* part, int W, hipStream_t s);
// px, sx (may be null = p, sv): directions added to x, M^{-1}p and M^{-1}s when preconditioned
void bicg_xr(int R, int it, int64_t m, double tol, const double* s1, const double* s2, const double* s3,
             KState* st, double* x, const double* p, const double* sv, const double* t, double* r,
             const double* rt, double* part, int W, hipStream_t s, const double* px = nullptr,
             const double* sx = nullptr);
void bicg_p(int R, int it, int maxit, int64_t m, double tol, const double* s1, const double* s2,
            const double* s3, const double* s4, KState* st, const double* r, double* p, const double* v,
            int W, hipStream_t s);
void bicg_restart(int R, int it, int64_t m, const int32_t* flag, const double* r, double* rt, double* p,
                  double* part, int W, double* sums, KState* st, hipStream_t s);
void csr_resid(int R, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
               const double* x, int64_t ldx, const double* f, int64_t ldf, double* r, int64_t ldr,
               double* part, int W, double* out, hipStream_t s);
// r = f - A x and per-column norms (max|r|, sum r^2, max|f|, sum f^2) for
// k <= kMaxRhs columns; part: device, kVecGrid * kMaxRhs * 4 doubles of
// partial sums; out: device, 4k doubles.
void residual_norms_cols(int64_t n, int k, const int64_t* row_ptr, const int32_t* col, const double* val,
                         const double* X, int64_t ldx, const double* F, int64_t ldf, double* R, int64_t ldr,
                         double* part, double* out, hipStream_t s);
// yp = y - R~ z^ (padded layout, R columns, k from y, the rest zero): the
// right-hand side of the re-solved retrieval; zh in the candidate layout
// (m entries per column), masked to c
void coupling_rhs(int64_t Np, int R, int k, int p, int t, const BlockInfo* blocks, const int64_t* row_ptr,
                  const int32_t* col, const double* val, const double* y, int64_t ldy, const double* zh, int64_t m,
                  const double* mask, double* yp, hipStream_t s);
// yout = yin -/+ sum of ns partial vectors (fixed order), rows x R, column
// stride ld, part q at parts + q * pstride; yin may be null, may alias yout
void sum_parts(int rows, int R, int ns, const double* parts, int64_t pstride, int64_t ld, const double* yin,
               double* yout, int neg, hipStream_t s);
void lincomb(int R, int64_t n, const Coef3& cf, const double* X, const double* Y, const double* Z,
             double* out, hipStream_t s);
void dot2(int R, int64_t n, const double* a0, const double* b0, const double* a1, const double* b1,
          double* part, int W, double* out, hipStream_t s);

}  // namespace ddps
