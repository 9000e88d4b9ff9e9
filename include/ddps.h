/*
 * ddps.h -- C ABI of the MI355X (gfx950) DDPS solver.
 *
 * DDPS (Manguoglu, "A domain-decomposing parallel sparse linear system
 * solver", arXiv 1008.1700) solves Ax = f for a row-partitioned sparse A:
 * Section 3, Figure 1, stages 1-5 form the preconditioner P = D~ + R~ without
 * a right-hand side (ddps_setup + ddps_factor), and stage 6 runs a Krylov
 * method with P applied as in Figure 2 (ddps_solve).
 *
 * Conventions for every entry point:
 *   - Return value: a ddps_status (0 = DDPS_OK, negative = error).  No C++
 *     exception ever crosses the ABI.
 *   - "device" pointers are HIP device memory of the current device (for
 *     example a torch tensor's data_ptr()); "host" pointers are ordinary CPU
 *     memory.  Every pointer argument below says which it is.
 *   - All GPU work is ordered on the stream given in ddps_options.stream
 *     (0 = the null stream).  Calls that return ddps_info synchronise that
 *     stream before returning.
 *   - A handle is not thread-safe; calls on one handle must not overlap.
 *
 * Matrix requirements of the GPU path (checked by ddps_setup, DDPS_E_ARG if
 * violated): A is square, CSR with int64 row pointers and int32 column
 * indices (sorted or not), finite values; the half-bandwidth
 * b = max |i - j| over stored entries satisfies b >= 1, and, with
 * t = b rounded up to a multiple of 64, every block has at least 2t rows
 * when p > 1.  Then each block A_ii is block tridiagonal in t x t tiles and
 * R_i couples block i only with the last t rows of block i-1 and the first
 * t rows of block i+1.
 */
#ifndef DDPS_H
#define DDPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddps_ctx* ddps_handle;

typedef enum {
  DDPS_OK = 0,
  DDPS_E_ARG = -1,        /* invalid argument or unsupported matrix structure */
  DDPS_E_NOMEM = -2,      /* the plan does not fit the memory budget (the paper's failure F1) */
  DDPS_E_NOCONV = -3,     /* tolerance not met after outer_maxit (the paper's failure F2) */
  DDPS_E_SINGULAR = -4,   /* a pivot of a diagonal-block LU is (numerically) zero */
  DDPS_E_BREAKDOWN = -5,  /* BiCGStab broke down twice (after one restart) */
  DDPS_E_STATE = -6,      /* call out of order (e.g. solve before factor) */
  DDPS_E_HIP = -7         /* a HIP runtime call failed */
} ddps_status;

/* Arithmetic of the block factors and spikes (stages 2 and 4). */
typedef enum {
  DDPS_F64 = 0,     /* FP64 storage, FP64 MFMA */
  DDPS_F32 = 1,     /* FP32 storage, FP32 MFMA */
  DDPS_BF16X3 = 2,  /* FP32 storage; products on bf16 MFMA with each FP32 operand split
                       into two bf16 terms (hi*hi + hi*lo + lo*hi), FP32 accumulation */
  DDPS_BF16 = 3     /* FP32 storage; products on bf16 MFMA with one bf16 term per operand */
} ddps_dtype;

typedef struct {
  int32_t struct_size;     /* sizeof(ddps_options), for forward compatibility */
  double drop_delta;       /* delta of the column-dropping rule (Section 3), in [0,1]; 0 keeps
                              every nonzero coupling column */
  int32_t factor_dtype;    /* ddps_dtype */
  double inner_tol;        /* BiCGStab on the reduced system: stop at ||g^ - G^ z^||_2 / ||g^||_2
                              <= inner_tol (Figure 2, step 6.3) */
  int32_t inner_maxit;     /* maximum inner iterations */
  int32_t outer_maxit;     /* maximum outer iterations (Section 4 uses 1000) */
  int32_t outer_method;    /* 0 = preconditioned BiCGStab (Section 4), 1 = iterative refinement
                              x += P^{-1}(f - Ax).  Under refinement a step's inner tolerance is
                              inner_tol, raised to 0.1 tol ||f|| / ||r|| when that is larger (at
                              most 1e-2).  rho_f is the residual ratio of the last step taken at
                              that tolerance; once rho_f <= 1e-2 (the factors, not the inner
                              solve, then limit the steps), later steps are loosened to
                              0.1 rho_f.  A loosened step whose ratio exceeds loosen_ratio *
                              rho_f is undone (x and its residual restored) and redone at the
                              unloosened tolerance, and loosening stops for the solve; so every
                              kept loosened step cuts the residual by at most loosen_ratio *
                              rho_f */
  int32_t guess;           /* 0: reduced solve starts at z^ = 0; 1: from the vector given to
                              ddps_set_guess (kept until replaced) */
  int32_t use_x0;          /* 1: x is read as the initial outer iterate */
  int32_t max_rhs;         /* largest k passed to ddps_solve_many (>= 1) */
  size_t mem_budget;       /* bytes the handle may allocate; 0 = free device memory */
  void* stream;            /* hipStream_t on which all work is ordered */
  int32_t factor_streams;  /* stream groups of the factorisation (blocks assigned longest
                              first); 0 = automatic */
  int32_t factor_graph;    /* 1: ddps_factor is captured once as a HIP graph and replayed */
  int32_t inner_prec;      /* preconditioner of the inner BiCGStab: 0 = none (the paper's
                              method, Section 4); 1 = z -> z - N z, N the interface-local part
                              of G(c,c) (entries whose row and column lie at the same block
                              boundary), right-preconditioned; it changes the iterates, not
                              the solved system */
  int32_t retrieval;       /* step 6.5 of Figure 2: 0 = z = g - G z (z(c) = z^), with the
                              spikes G kept in full; 1 = the same vector written without the
                              spikes, z = D~^{-1}(y - R~ z) (G = D~^{-1} R~): one more block
                              solve per application, and only the spike rows at c (the tips
                              that form G^) are kept.  The spikes are then computed batch by
                              batch in a workspace of work_slots blocks, which is what lets
                              large systems fit */
  int32_t norm;            /* norm of the outer stopping test ||f - Ax|| / ||f|| <= tol:
                              0 = inf-norm (Section 4), 2 = 2-norm */
  int32_t work_slots;      /* retrieval 1: blocks whose spikes are computed at once (0 = as
                              many as the memory budget allows, at most p) */
  int32_t reduced_solve;   /* step 6.3 of Figure 2: 0 = BiCGStab to inner_tol (Section 4);
                              1 = solved directly (Section 3 allows either): block LU of G^
                              over the interfaces, computed by ddps_factor (one t x t
                              Schur complement factored per interface, a sequential chain),
                              then a forward and a backward substitution per application.
                              A zero pivot there is reported as DDPS_E_SINGULAR with
                              bad_block = p and bad_row = the reduced row */
  double loosen_ratio;     /* refinement: the factor by which a loosened step may fall short
                              of rho_f before it is undone (see outer_method); 0 = 10,
                              negative = never loosen */
  int32_t gemv_sums;       /* FP32 factor storage, 4 or more right-hand sides: the tile and
                              spike products of the solve phase (block sweeps of step 6.1, the
                              reduced-matrix products, the retrieval) run as 0 = FP32 products
                              with FP32 sums on the matrix cores (default), 1 = FP64 sums on
                              the vector units.  Either way the sums of four column ranges are
                              added in FP64, and vectors, dots and residuals stay FP64 */
  int32_t block_factor;    /* stage 2 of Figure 1: 0 = exact LU of every A_ii (unpivoted, in
                              t x t band tiles); 1 = incomplete factors A~_ii = L~_i U~_i
                              (Section 3), read as ILU(0): L~_i unit lower and U~_i upper
                              with the sparsity pattern of A_ii and (L~_i U~_i)(r, j) = a_rj
                              wherever A_ii stores an entry.  Factors in FP64 at A's CSR
                              positions; the spikes D~^{-1} R~ come from sparse triangular
                              solves in the storage type of factor_dtype (FP64 for DDPS_F64,
                              else FP32) and only their tips are kept, so p > 1 requires
                              retrieval = 1 (DDPS_E_ARG otherwise).  Every row must store its
                              diagonal entry and its columns sorted without repeats
                              (DDPS_E_ARG otherwise).  ddps_get_tile, ddps_set_execution
                              and ddps_autotune then return DDPS_E_STATE */
} ddps_options;

typedef struct {
  double outer_iters;       /* outer iterations in half steps, as counted in the paper's
                               iteration tables (0.5 = converged after the first half step) */
  double inner_iters_avg;   /* average BiCGStab iterations per reduced solve */
  int64_t inner_iters_total;
  int32_t applications;     /* preconditioner applications (Figure 2 solves) */
  double relres_inf;        /* ||f - Ax||_inf / ||f||_inf of the returned x (worst column) */
  double relres_2;          /* ||f - Ax||_2 / ||f||_2 of the returned x (worst column) */
  double t_setup_ms, t_factor_ms, t_solve_ms;   /* device time of the last call of each */
  int32_t bad_block;        /* DDPS_E_SINGULAR: block of the first bad pivot, else -1 */
  int64_t bad_row;          /* DDPS_E_SINGULAR: global row of that pivot, else -1 */
  int32_t loosened_steps;   /* refinement steps taken at a loosened inner tolerance */
  int32_t undone_steps;     /* of these, steps undone and redone (see outer_method) */
} ddps_info;

/* Fills *opt with the defaults: delta 0, FP64 factors, inner_tol 1e-12,
 * inner_maxit 1000, outer_maxit 1000, iterative refinement, zero guess,
 * max_rhs 1, no memory budget, null stream, automatic stream groups, no
 * graph, no inner preconditioner, spikes kept in full (retrieval 0),
 * inf-norm stopping test, automatic workspace slots, BiCGStab reduced
 * solve, FP32 sums on the matrix cores, exact block factors. */
void ddps_default_options(ddps_options* opt);

/* Stages 1, 3 and 5 (Section 3, Figure 1): split A = D + R for the row
 * partition part_ptr, apply the dropping rule to the columns of each R_i and
 * build the index set c of kept coupling columns.
 *   n, p:        matrix order and number of blocks (p >= 1).
 *   part_ptr:    host, int64[p+1]; block i owns rows [part_ptr[i], part_ptr[i+1]);
 *                part_ptr[0] = 0, strictly increasing, part_ptr[p] = n.  A host
 *                array because the block layout and the memory plan (and so
 *                the F1 check) are made on the host before any large
 *                allocation; the library keeps its own copies.
 *   row_ptr:     device, int64[n+1]; col: device, int32[nnz]; val: device, double[nnz].
 *   opt:         host, may be NULL for the defaults.
 * The library copies what it needs: the caller may free the CSR arrays when
 * the call returns.  On success *h owns all device memory of the solver.
 * Errors: DDPS_E_ARG (bad partition, indices out of range, non-finite values,
 * unsupported structure), DDPS_E_NOMEM (plan larger than the budget: nothing
 * is left allocated), DDPS_E_HIP. */
int ddps_setup(ddps_handle* h, int64_t n, int32_t p, const int64_t* part_ptr,
               const int64_t* row_ptr, const int32_t* col, const double* val, int64_t nnz,
               const ddps_options* opt);

/* Stages 2 and 4 (Figure 1): LU of every diagonal block A_ii, without
 * pivoting, and the spikes G_i = A_ii^{-1} R~_i(:, c_i) for all blocks, in
 * the factor dtype.  The reduced matrix G^ = I(c,c) + G(c,c) of Figure 2,
 * step 6.2, is the set of spike rows at c; it is used in place.
 * Errors: DDPS_E_SINGULAR when a pivot |u_kk| <= 1e3 eps max_j |a_kj| (the
 * largest in-block entry of that row, eps of the factor dtype) or is not
 * finite (info of the next ddps_solve reports the block and row; also
 * readable with ddps_last_singular), DDPS_E_HIP. */
int ddps_factor(ddps_handle h);

/* Replaces the values of A (same sparsity pattern as at setup; device,
 * double[nnz]) and redoes stages 1, 3 and 5; call ddps_factor next. */
int ddps_refactor_values(ddps_handle h, const double* val);

/* Stage 6 (Figure 1) with P z = y solved as in Figure 2: solves Ax = f to
 * ||f - Ax||_inf / ||f||_inf <= tol.
 *   f: device, double[n], read only.  x: device, double[n], written (read
 *   first if use_x0).  info: host, may be NULL.
 * Errors: DDPS_E_STATE (not factored), DDPS_E_NOCONV (the paper's F2; x
 * holds the last iterate), DDPS_E_BREAKDOWN, DDPS_E_HIP. */
int ddps_solve(ddps_handle h, const double* f, double* x, double tol, ddps_info* info);

/* As ddps_solve for k right-hand sides at once (columns of F, X, column-major
 * with leading dimensions ldf, ldx >= n; device).  Each column runs its own
 * Krylov scalars; the block sweeps, reduced-matrix products and retrievals
 * are shared passes over the factors and spikes.  1 <= k <= max_rhs. */
int ddps_solve_many(ddps_handle h, int32_t k, const double* F, int64_t ldf, double* X, int64_t ldx,
                    double tol, ddps_info* info);

/* Sets the initial guess of the reduced solve (used when opt.guess = 1):
 * device, double[m * k] laid out like ddps_reduced_layout's c, one column of
 * m entries per right-hand side.  The vector is copied. */
int ddps_set_guess(ddps_handle h, const double* zhat0, int32_t k);

/* Reduced-system layout.  *m receives the number of candidate coupling
 * columns m = 2 t (p - 1) (host).  If c is not NULL it receives (device,
 * int64[m]) the global column index of each candidate, ascending; if mask is
 * not NULL it receives (device, double[m]) 1 for candidates in the index set
 * c of stage 5 and 0 for dropped or structurally zero columns; the dropping
 * rule is applied by ddps_factor, so asking for the mask before a successful
 * factorisation (or after ddps_refactor_values, before the next one) returns
 * DDPS_E_STATE.  t and b (host, may be NULL) receive the tile size and
 * half-bandwidth. */
int ddps_reduced_layout(ddps_handle h, int64_t* m, int64_t* c, double* mask, int32_t* t, int32_t* b);

/* Reduced vectors of the last preconditioner application of the last solve
 * (for recording training pairs of the learned guess): g^ (Figure 2, 6.2)
 * and z^ (6.3), device double[m * k] each; either may be NULL. */
int ddps_last_reduced(ddps_handle h, double* ghat, double* zhat);

/* One application of P^{-1} (Figure 2, steps 6.1-6.5): z = P^{-1} y for k
 * columns (device, column-major, leading dimension n).  If ghat/zhat are not
 * NULL they receive g^ and z^ (device, double[m*k]).  The inner solve uses
 * opt.inner_tol and the current guess setting.  inner_iters (host, may be
 * NULL) receives the iterations of each column's reduced solve. */
int ddps_apply_preconditioner(ddps_handle h, int32_t k, const double* y, double* z, double* ghat,
                              double* zhat, double* inner_iters);

/* Step 6.1 only: g = D~^{-1} y (device, double[n*k]). */
int ddps_block_solve(ddps_handle h, int32_t k, const double* y, double* g);

/* The reduced operator of step 6.2: v = G^ x restricted to the index set c
 * (entries outside c act as the identity); device double[m*k]. */
int ddps_reduced_matvec(ddps_handle h, int32_t k, const double* x, double* v);

/* Copies of the factored blocks, as double, for checking.  Block `blk`
 * (0-based) has T = ceil(n_i / t) tile rows and is padded at the top with
 * pad = T t - n_i identity rows.
 *   which = 0: the diagonal tile k holding inverse factors: strictly below
 *              the diagonal L_kk^{-1} (unit diagonal implied), on and above
 *              it U_kk^{-1};
 *   which = 1: L_{k+1,k}, the sub-diagonal tile of L (k < T-1), upper
 *              triangular (zero below the diagonal);
 *   which = 2: U_{k,k+1}, the super-diagonal tile of U (k < T-1), lower
 *              triangular (zero above the diagonal).
 * The two off-diagonal factors of a tile row share one t x (t+1) array (a
 * pair of triangles).  dst: device, double[t*t], column-major. */
int ddps_get_tile(ddps_handle h, int32_t blk, int32_t k, int32_t which, double* dst);

/* Spikes of block blk as double: dst (device, double[n_i * 2t], column-major,
 * leading dimension n_i, padding rows removed); columns [0,t) multiply the
 * last t columns of block blk-1, columns [t,2t) the first t columns of block
 * blk+1 (all zero where that neighbour does not exist).  DDPS_E_STATE with
 * retrieval 1 (only the tips are kept). */
int ddps_get_spikes(ddps_handle h, int32_t blk, double* dst);

/* Tile size t and per-block padded sizes: tiles (host, int32[p]) receives
 * T_i and pads (host, int32[p]) the padding of each block; either may be NULL. */
int ddps_block_shape(ddps_handle h, int32_t* t, int32_t* tiles, int32_t* pads);

/* Block and global row of the first bad pivot found by the last ddps_factor
 * (host pointers; -1 if none). */
int ddps_last_singular(ddps_handle h, int32_t* block, int64_t* row);

/* Execution form of ddps_factor (the method's result does not depend on it):
 * streams = stream groups over which the blocks are distributed (blocks of
 * different groups factor concurrently; 0 = automatic), graph = 1 to capture
 * the factorisation once as a HIP graph and replay it, and tile_policy the
 * GEMM tile of each launch:
 *   0  128 x 128 where every problem of the launch allows it,
 *   1  64 x 64 only,
 *   2  256 x 128 where every problem allows it (bf16 arithmetic, else as 0),
 *   3  a tile chosen per launch by ddps_autotune (as 0 until it has run),
 *   4  128 x 128 with operands loaded straight into LDS (bf16 arithmetic,
 *      else as 0),
 *   5  256 x 256 on 8 waves, operands loaded straight into LDS (bf16
 *      arithmetic, else as 0; launches with a side below 256 take 4's tile).
 * Rebuilds the launch schedules; call before ddps_factor.  Errors:
 * DDPS_E_ARG, DDPS_E_NOMEM, DDPS_E_HIP. */
int ddps_set_execution(ddps_handle h, int32_t streams, int32_t graph, int32_t tile_policy);

/* Autotuner of the execution form.  It times ddps_factor on the device for
 * stream groups {1, 2, 3, 4, 6, 8} (at most p, and at most the workspace
 * slots with retrieval 1) and the fixed tile policies (0, 1, 2, 4, 5 for the
 * bf16 dtypes; 0, 1 otherwise), and takes the fewest groups within 3% of the
 * fastest form.  For every group count within 10% of the fastest it then
 * times each GEMM launch of the factorisation under each fixed policy and
 * builds policy 3 from the fastest tile of each launch; the fewest groups
 * within 3% of the fastest such form are kept if they beat the fixed form.
 * budget_s > 0 bounds the search: once that many seconds have passed no
 * further form is timed and the best form so far is taken (the first form
 * is always timed).  One progress line per timed form goes to stderr.  The
 * choice, with policy 3's per-launch tiles, is recorded in the JSON file
 * cache_path (may be NULL) under a key made of the GPU architecture, factor
 * dtype, tile size t, p, the largest tile-row count and (retrieval 1) the
 * workspace slots; a later call with the same key takes the cached choice
 * without timing.  Host outputs (may be NULL): chosen streams, tile policy
 * and its factor time in milliseconds.  The handle is left factored with the
 * chosen form. */
int ddps_autotune(ddps_handle h, const char* cache_path, double budget_s, int32_t* streams, int32_t* tile_policy,
                  double* factor_ms);

/* Per-kernel timing for roofline reporting.  ddps_timing_enable(h, kind, 1)
 * records HIP events around every launch of that kernel kind on the stream it
 * is launched on (while kind 0 or 1 is timed, the stream groups of
 * ddps_factor run one after another, so that the intervals do not overlap);
 * ddps_timing_read reports launches, summed device milliseconds and
 * the algorithmic flops and bytes of those launches (host pointers), then
 * clears the counters.  kind: 0 = grouped GEMM (factor and spikes),
 * 1 = diagonal-tile LU, 2 = block-sweep GEMV, 3 = reduced-matrix product
 * (and the direct reduced solve's substitutions), 4 = retrieval, 5 = CSR
 * SpMV, 6 = the direct reduced solve's factorisation. */
int ddps_timing_enable(ddps_handle h, int32_t kind, int32_t on);
int ddps_timing_read(ddps_handle h, int32_t kind, int64_t* launches, double* ms, double* flops,
                     double* bytes);

/* ------------------------------------------------------------------------
 * Learned initial guess of the reduced solve.
 *
 * The method leaves the starting vector of the inner Krylov solve of step
 * 6.3 free (Figure 2).  Over a sequence of related systems (time steps of
 * the loop of Section 1) a small network predicts it per interface from the
 * previous step's reduced solution z^prev and its reduced residual
 * r = g^ - G^ z^prev.  The reduced vector is p-1 interfaces of 2t entries
 * (interface j: the last t rows of block j, then the first t rows of block
 * j+1); one network row maps [r_j / s_j, z^prev_j / q_j, cos, sin]
 * (s_j = max |r_j|, q_j = max |z^prev_j|; d_in >= 4t+2 floats, zero padded)
 * to the correction (z^_j - z^prev_j) / s_j (2t floats).  The caller judges
 * candidates with ddps_reduced_residual and passes the winner to
 * ddps_set_guess.  Reduced vectors are device double[m*k], one column of m
 * entries per right-hand side (k <= max_rhs).
 * ------------------------------------------------------------------------ */

/* Steps 6.1-6.2 for k columns y (device, double[n*k]): ghat = (D~^{-1} y)
 * on the index set c, zero elsewhere.  Requires a factored handle
 * (DDPS_E_STATE otherwise). */
int ddps_reduced_rhs(ddps_handle h, int32_t k, const double* y, double* ghat);

/* Restriction to the reduced layout: z = x on the index set c, zero
 * elsewhere, for k columns x (device, double[n*k]); z is device double[m*k].
 * With exact coupling (drop_delta 0) the reduced solution of a right-hand
 * side f is the restriction of the solution of Ax = f. */
int ddps_reduced_restrict(ddps_handle h, int32_t k, const double* x, double* z);

/* Selection residual of a candidate guess: res (host, double[k]) receives
 * ||ghat - G^ z||_2 over the index set c for each column (z is masked to c
 * first); if rvec (device, double[m*k]) is not NULL it receives the residual
 * vector itself, zero off c.  Uses the handle's reduced work vectors, so the
 * vectors of ddps_last_reduced are overwritten. */
int ddps_reduced_residual(ddps_handle h, int32_t k, const double* ghat, const double* z, double* res,
                          double* rvec);

/* Network inputs of the k (p-1) interfaces from the reduced residual r of
 * zprev (ddps_reduced_residual's rvec): X (device, float[k (p-1) * d_in],
 * row-major, row j = interface j % (p-1) of column j / (p-1)) and the scales
 * s_j (device, float[k (p-1)]).  zprev is masked to c.  cos_t, sin_t are the
 * two scalar features (for example the phase of a rotating velocity).
 * DDPS_E_ARG if d_in < 4t + 2. */
int ddps_guess_features(ddps_handle h, int32_t k, const double* r, const double* zprev, double cos_t,
                        double sin_t, int32_t d_in, float* X, float* scale);

/* zhat0 = (zprev + s_j Y_j) on c, 0 elsewhere, from network outputs Y
 * (device, float[k (p-1) * 2t], row-major) and the scales of
 * ddps_guess_features; zhat0 is device double[m*k]. */
int ddps_guess_compose(ddps_handle h, int32_t k, const double* zprev, const float* Y, const float* scale,
                       double* zhat0);

/* Training target of the network: T = (zhat - zprev on c) / s_j (device,
 * float[k (p-1) * 2t], row-major) for a reduced solution zhat. */
int ddps_guess_target(ddps_handle h, int32_t k, const double* zhat, const double* zprev, const float* scale,
                      float* T);

/* The network itself: 4 layers d_in -> H -> H -> H -> d_out, ReLU between
 * layers, bf16 weights and activations on MFMA with FP32 accumulation, FP32
 * master parameters, mean-squared-error loss, Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8).  Parameters are one packed float vector
 * [W1, b1, W2, b2, W3, b3, W4, b4], W_l row-major (fan-in x fan-out).
 * Every call is ordered on `stream`; X, Y, T are device float, row-major,
 * batch x d_in / d_out, 1 <= batch <= max_batch. */
typedef struct ddps_mlp_ctx* ddps_mlp;

/* Creates a network with He-uniform weights drawn from `seed` (splitmix64)
 * and zero biases.  DDPS_E_ARG on non-positive sizes, DDPS_E_NOMEM if the
 * device allocation fails. */
int ddps_mlp_create(ddps_mlp* m, int32_t d_in, int32_t hidden, int32_t d_out, int32_t max_batch, uint64_t seed,
                    void* stream);
/* Number of floats of the packed parameter vector (-1 for NULL). */
int64_t ddps_mlp_param_count(ddps_mlp m);
/* Host float[param_count] in and out; set_params also resets Adam's state. */
int ddps_mlp_set_params(ddps_mlp m, const float* host_params);
int ddps_mlp_get_params(ddps_mlp m, float* host_params);
/* Y = net(X).  Asynchronous on the stream. */
int ddps_mlp_forward(ddps_mlp m, int32_t batch, const float* X, float* Y);
/* One Adam step on mean((net(X) - T)^2) with learning rate lr > 0; loss
 * (host, may be NULL) receives the loss before the step (synchronises). */
int ddps_mlp_train_step(ddps_mlp m, int32_t batch, const float* X, const float* T, float lr, double* loss);
/* Gradients of mean((net(X) - T)^2) without a step: host_grads (host,
 * float[param_count], may be NULL) and loss (host, may be NULL). */
int ddps_mlp_gradients(ddps_mlp m, int32_t batch, const float* X, const float* T, float* host_grads,
                       double* loss);
/* Releases the network; NULL is ignored. */
void ddps_mlp_destroy(ddps_mlp m);

/* Residual of the outer stopping test (Section 4: ||f - Ax||_inf / ||f||_inf,
 * Section 3: the relative residual of the outer iteration) for k columns,
 * without a handle: r = f - A x for the CSR matrix A (device: int64 row_ptr
 * [n+1], int32 col and double val [nnz]) and X, F (device, column-major n x k
 * with leading dimensions ldx, ldf >= n).  R (device, may be NULL) receives r
 * (leading dimension ldr >= n).  norms (host, double[4k]) receives per column
 * j: ||r||_inf, ||r||_2, ||f||_inf, ||f||_2.  1 <= k <= 8.  Ordered on
 * `stream` (a hipStream_t, NULL = null stream) and synchronises it.  The
 * partial sums of the reduction (256 KiB of device memory) are allocated
 * and freed by the call.  Errors: DDPS_E_ARG, DDPS_E_NOMEM, DDPS_E_HIP. */
int ddps_residual_norms(int64_t n, int32_t k, const int64_t* row_ptr, const int32_t* col, const double* val,
                        const double* X, int64_t ldx, const double* F, int64_t ldf, double* R, int64_t ldr,
                        double* norms, void* stream);

/* As ddps_residual_norms, for callers that cannot allocate device memory
 * (for example code that must not call hipMalloc in a serving loop): the call
 * allocates nothing.  Its partial sums live in a fixed device array of the
 * library (262,400 bytes per GPU, held until the process ends); k > 8 is
 * refused with DDPS_E_ARG since the array holds 8 columns.  Every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (other host
 * threads, or other streams before this call's synchronisation) race; calls
 * in sequence are safe, since every entry a call reads it first writes.
 * Same arguments, results and errors as ddps_residual_norms (DDPS_E_HIP also
 * if the array's device address cannot be found). */
int ddps_residual_norms_noalloc(int64_t n, int32_t k, const int64_t* row_ptr, const int32_t* col,
                                const double* val, const double* X, int64_t ldx, const double* F, int64_t ldf,
                                double* R, int64_t ldr, double* norms, void* stream);

/* Learned guess in every preconditioner application.  Attaches a network
 * (d_in >= 4t + 2, d_out = 2t, max_batch >= R (p-1) for R = max_rhs rounded
 * up to 1, 2, 4 or 8; created on the handle's stream) to the handle; NULL
 * detaches it.  While attached, each application of Figure 2 starts the
 * reduced solve of step 6.3 from the best of three vectors per right-hand
 * side, judged by ||g^ - G^ z0||_2 on c: z0 = 0, z0 = g^ (since
 * G^ = I + G(c,c)), and z0 = g^ + s_j Y_j per interface j, Y the network's
 * output for the input row [r_j / s_j, g^_j / q_j, 0, 0] (r = g^ - G^ g^,
 * s_j = max |r_j|, q_j = max |g^_j|; the layout of ddps_guess_features with
 * z^prev = g^).  A vector set with ddps_set_guess is not used meanwhile.
 * After 8 reduced solves in a row in which the network's candidate was not
 * the smallest, the network is retired: the reduced solves start from zero
 * (the method's start) without trying candidates, until a network is
 * attached again.  A smaller starting residual does not always mean fewer
 * iterations, so the first reduced solves after attaching also run a trial:
 * every other one leaves the network out of the choice.  Once each arm has
 * 8 solves, the network is retired unless its solves took at least half an
 * inner iteration fewer on average (ddps_guess_trial reports the arms).
 * The network is used, not owned: keep it alive while attached.  Buffers for
 * the network's inputs and outputs are allocated here (not during solves).
 * Errors: DDPS_E_ARG (shape or stream mismatch), DDPS_E_NOMEM. */
int ddps_set_guess_model(ddps_handle h, ddps_mlp net);

/* Host int64[4]: reduced solves started so far from z0 = 0, from g^ and
 * from the network after trying the candidates, and those started without
 * trying them (network retired), over the handle's lifetime. */
int ddps_guess_counts(ddps_handle h, int64_t* counts);

/* The trial of the attached network against its absence (see
 * ddps_set_guess_model): host int64[2] solves and double[2] mean inner
 * iterations per solve, index 0 without the network, 1 with it; *state:
 * 0 = running, 1 = done and the network kept, 2 = the network retired (by
 * the trial or by 8 lost reduced solves in a row).  Errors: DDPS_E_ARG. */
int ddps_guess_trial(ddps_handle h, int64_t* solves, double* mean_iters, int32_t* state);

/* ---------------------------------------------------------------- general
 * sparse matrices.  The paper partitions general sparse matrices after a
 * fill-reducing / bandwidth-reducing reordering (Section 3; it uses METIS);
 * this path needs banded blocks, so a general matrix is first reordered by
 * reverse Cuthill-McKee (Cuthill & McKee 1969, reversed, started from a
 * pseudo-peripheral node after George & Liu 1979), which
 * makes the profile of A + A^T narrow, and then cut into equal row slabs.
 * All arrays here are host arrays; nothing touches the GPU. */

/* Reverse Cuthill-McKee ordering of the symmetric pattern of A + A^T (CSR,
 * n rows, int64 row_ptr[n+1], int32 col[nnz]; the diagonal is ignored).
 * Each connected component starts from a pseudo-peripheral node (George-Liu
 * search from a node of minimum degree); neighbours are visited in
 * increasing degree, ties by index; the whole order is reversed.  perm[i] =
 * the original index of new row i (int64[n], written).  Errors: DDPS_E_ARG
 * (n < 0, null pointers for n > 0, a column outside [0, n)). */
int ddps_rcm(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* perm);

/* Half-bandwidth b = max |i - j| over the stored entries (int64, written).
 * Errors: DDPS_E_ARG (n < 0, null pointers, a column outside [0, n)). */
int ddps_bandwidth(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* b);

/* B = P A P^T for perm from ddps_rcm (new row i = old row perm[i]):
 * out_row_ptr[n+1], out_col[nnz], out_val[nnz] written, columns sorted
 * ascending within each row.  val / out_val may be null (pattern only).
 * Errors: DDPS_E_ARG (perm not a permutation of [0, n), a column outside
 * [0, n), null pointers). */
int ddps_permute_csr(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                     const int64_t* perm, int64_t* out_row_ptr, int32_t* out_col, double* out_val);

/* Row partition of a matrix with half-bandwidth b into at most p_max equal
 * slabs (sizes differing by at most one row) such that every slab has at
 * least 2t rows, t = b rounded up to a multiple of 64 and at least 64
 * (what ddps_setup requires); one slab when n < 4t.  part_ptr (int64[p_max + 1]) and *p (the slabs used, >= 1) are
 * written.  Errors: DDPS_E_ARG (p_max < 1, n < 1, b < 0). */
int ddps_partition_rows(int64_t n, int64_t b, int32_t p_max, int64_t* part_ptr, int32_t* p);

/* Device bytes held by the handle (host pointer). */
int ddps_memory(ddps_handle h, size_t* bytes);

/* Releases every resource of the handle; NULL is ignored. */
void ddps_destroy(ddps_handle h);

/* Static string for a status code. */
const char* ddps_status_string(int s);

/* After DDPS_E_HIP: the HIP runtime's description of the error that caused
 * it (the one recorded by the failing call, else the runtime's last error of
 * this thread), then cleared.  A static string. */
const char* ddps_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDPS_H */
