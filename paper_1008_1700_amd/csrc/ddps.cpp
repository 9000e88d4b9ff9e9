// Host runtime and C ABI of the DDPS solver (see include/ddps.h).
//
// Layout.  With b the half-bandwidth of A and t = b rounded up to 64, every
// block A_ii is block tridiagonal in t x t tiles (block rows shorter than a
// multiple of t are padded on top with identity rows).  ddps_factor performs
// an unpivoted LU of each block in this tile form:
//     for k = 0..T-1:  S_k = A_kk - L_{k,k-1} U_{k-1,k}        (Schur update)
//                      S_k = L_kk U_kk, stored as L_kk^{-1}, U_kk^{-1}
//                      L_{k+1,k} = A_{k+1,k} U_kk^{-1},  U_{k,k+1} = L_kk^{-1} A_{k,k+1}
// and the spikes G_i = A_ii^{-1} R_i(:, c_i) by a forward sweep (only the
// columns coupling to block i-1 need one: the others are supported on the
// last tile) and a backward sweep over all 2t columns.  Keeping the inverse
// triangles of the diagonal tiles turns every step of both sweeps into a
// GEMM (factor phase, MFMA) or a GEMV (solve phase, HBM stream).
//
// Execution.  Every phase is a static schedule of grouped launches built once
// per handle: a launch carries one problem descriptor per block, so all
// blocks advance together and one launch fills the GPU.
#include "../../include/ddps.h"
#include "ddps_internal.h"
#include "ddps_mlp_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

using namespace ddps;

namespace {

enum LaunchKind { LK_GEMM = 0, LK_PANEL = 1, LK_GEMV = 2, LK_TIPMV = 3, LK_SUM = 4 };

// A fixed-order sum of split-column partial products (LK_SUM launches).
struct SumRec {
  const double* parts;
  int64_t pstride;
  const double* yin;
  double* yout;
  int rows, ns, neg;
};
enum TimingKind { TK_GEMM = 0, TK_PANEL = 1, TK_SWEEP = 2, TK_RSPMV = 3, TK_RETR = 4, TK_CSR = 5, TK_RFAC = 6,
                  TK_N = 7 };

struct Launch {
  int kind;
  int64_t off;
  int nprob;
  int nwg;
  double flops;
  double bytes;
  int mode;  // GEMM: tile mode; GEMV: 1 = every problem 16-byte aligned (wide loads)
  int64_t ord = -1;  // GEMM: offset of its tile order in d_order, -1 for the plain order
};

struct TimingRec {
  hipEvent_t a, b;
  double flops, bytes;
};

struct Status {
  int code;
};

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) {                        \
      last_hip_error() = e_;                       \
      return DDPS_E_HIP;                           \
    }                                              \
  } while (0)

hipError_t& last_hip_error() {
  static thread_local hipError_t e = hipSuccess;
  return e;
}

}  // namespace

struct ddps_ctx {
  ddps_options opt{};
  hipStream_t stream = nullptr;
  int64_t n = 0, nnz = 0;
  int p = 0;
  std::vector<int64_t> part;
  int32_t b = 0, t = 0;
  int sdt = 0;   // storage dtype of factors/spikes: 0 f64, 1 f32
  int gdt = 0;   // GEMM arithmetic: 0 f64, 1 f32, 2 bf16x3, 3 bf16
  size_t elt = 8;
  std::vector<BlockInfo> blk;
  int Tmax = 0;
  int64_t Np = 0, m = 0, tile_elems = 0, nspike = 0, scr_per_block = 0;
  // Tips only (retrieval = 1): the spikes are computed in a workspace of
  // `nslots` block slots (scratch and an Nmax x 2t spike matrix each), batch
  // after batch, and only their tips are kept (d_tipcm); the coupling entries
  // wait in the compact store d_rhs.  wslot[i] is block i's slot in the
  // current schedules (i itself when every block has its own).
  bool tips_only = false;
  int64_t nslots = 0, Nmax = 0;
  std::vector<int64_t> wslot;
  void* d_rhs = nullptr;     // p pairs of t x (t+1): left coupling (upper), right coupling (lower)
  // Direct reduced solve (reduced_solve = 1): block LU of G^ over the p-1
  // interfaces.  d_rP: P_j, d_rS: Sigma_j factored (inverse triangles), t x t
  // each per interface; d_rW: work tiles T1, T2, Y0, Y1, an identity, and the
  // two inversion work areas of the tile LU.
  void *d_rP = nullptr, *d_rS = nullptr, *d_rW = nullptr;
  std::vector<Launch> sch_rfac, sch_rsol;
  std::vector<SumRec> sums;   // records of the LK_SUM launches
  void* d_tipcm = nullptr;   // 2(p-1) tip parts, t x 2t column-major (ld t), part 2i-1 / 2i as in d_tips
  // Incomplete block factors (block_factor = 1): ILU(0) values at A's CSR
  // positions (d_fv), per row the positions of its lower part, pivot and
  // end (d_ilo, d_idg, d_ihi), the forward and backward level lists, and
  // the spike workspace of nslots blocks (ilu_nmax x 2t, row-major each);
  // ilu_batches lists the blocks batch after batch (d_ibatch, same order)
  bool ilu = false;
  double* d_fv = nullptr;
  int64_t *d_ilo = nullptr, *d_idg = nullptr, *d_ihi = nullptr, *d_lptr = nullptr, *d_uptr = nullptr;
  int32_t *d_lrows = nullptr, *d_urows = nullptr, *d_ibatch = nullptr;
  int64_t *d_lq = nullptr, *d_uq = nullptr;   // entry ranges per level-ordered row (pairs)
  IluBlock* d_iblk = nullptr;
  void* d_iws = nullptr;
  int64_t ilu_nmax = 0, ilu_nnz = 0, ilu_levels = 0;
  std::vector<std::pair<int, int>> ilu_batches;   // (first entry in d_ibatch, blocks)
  int R = 1;
  // device data
  int64_t *d_part = nullptr, *d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  double* d_val = nullptr;
  BlockInfo* d_blk = nullptr;
  void *d_tiles = nullptr, *d_spikes = nullptr, *d_scratch = nullptr;
  // Off-diagonal factors L_{k+1,k}, U_{k,k+1} in storage of their own (when
  // memory allows): the coupling tiles then keep A's entries, so the factor
  // products read them in place instead of from copies.  lu_off[i] is block
  // i's first tile in d_lu (its L tiles, then its U tiles).
  void* d_lu = nullptr;
  std::vector<int64_t> lu_off;
  bool spikes_zeroed = false;   // the whole spike array has been zeroed once (by an executed fill)
  void* d_tips = nullptr;   // spike tips packed row-major (rows of G^), 2(p-1) parts of t x 2t
  int tip_nseg = 0;         // > 0: reduced products on the packed tips (R <= 2 and 2t short enough)
  unsigned long long *d_colnorm = nullptr, *d_bad = nullptr, *d_band = nullptr;
  unsigned int* d_flags = nullptr;
  double* d_thresh = nullptr;   // per padded row: pivot threshold
  double* d_mask = nullptr;
  int64_t *d_c = nullptr, *d_rrow = nullptr;
  GemmProb* d_gemm = nullptr;
  int32_t* d_order = nullptr;   // tile orders of the GEMM launches with uneven tiles
  PanelProb* d_panel = nullptr;
  GemvProb* d_gemv = nullptr;
  double *d_ypad = nullptr, *d_vpad = nullptr;
  double *d_gh = nullptr, *d_zh = nullptr, *d_r = nullptr, *d_rt = nullptr, *d_p = nullptr,
         *d_v = nullptr, *d_s = nullptr, *d_tv = nullptr, *d_guess = nullptr;
  double *d_mp = nullptr, *d_ms = nullptr;  // M^{-1}p, M^{-1}s of the locally preconditioned inner solve
  double *d_part_buf = nullptr, *d_sums = nullptr, *d_out = nullptr;
  double* d_red1 = nullptr;   // first-level sums of two-level reductions (kReduceGroups x kMaxRhs x 2)
  KState* d_state = nullptr;
  int32_t* d_flag = nullptr;
  double *d_fo = nullptr, *d_xo = nullptr, *d_ro = nullptr, *d_z = nullptr, *d_rto = nullptr,
         *d_po = nullptr, *d_vo = nullptr, *d_ph = nullptr, *d_sh = nullptr, *d_to = nullptr;
  int64_t part_cap = 0;
  // host staging (pinned)
  KState* h_state = nullptr;
  double* h_out = nullptr;
  // schedules: the factorisation is split over stream groups of blocks
  std::vector<std::vector<Launch>> sch_group;
  std::vector<int> group_of;
  std::vector<Launch> sch_fwd, sch_bwd, sch_retr;
  int groups = 1;          // stream groups of the factor schedule
  int tile_policy = 0;     // 0: 128 x 128 GEMM tiles where every problem allows, 1: 64 x 64 only,
                           // 2: 256 x 128 (bf16 arithmetic) where every problem allows,
                           // 3: per launch, from mode_choice
  std::vector<int8_t> mode_choice;  // policy 3: requested tile mode of each factor GEMM launch, in order
  int mode_cursor = 0;              // next factor GEMM launch while the schedules are built
  bool use_graph = false;  // capture ddps_factor once as a HIP graph, then replay it
  hipStream_t fstream = nullptr;          // internal stream of the factorisation
  std::vector<hipStream_t> gstream;       // one per group beyond the first
  std::vector<hipEvent_t> gevent;
  // fork/join events of a factorisation being captured: created for each
  // capture and used by nothing else, so that no event object recorded inside
  // a capture is ever recorded or waited on outside it (and the reverse)
  hipEvent_t cap_fork = nullptr;
  std::vector<hipEvent_t> cap_gevent;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool capturing = false;
  Launch l_pv{}, l_st{}, l_zv{};  // reduced products: p->v (dot r~), s->t (dots), z->v
  Launch l_lp{}, l_ls{};          // local preconditioner: p -> p - N p, s -> s - N s
  Launch l_pvh{}, l_sth{};        // reduced products of the preconditioned directions
  int W1 = 0;
  bool factored = false;
  int guess_k = 0;
  // learned guess in every preconditioner application (ddps_set_guess_model)
  ddps_mlp gnet = nullptr;
  int gnet_din = 0;
  float *d_gX = nullptr, *d_gS = nullptr, *d_gY = nullptr;
  int64_t guess_counts[3] = {0, 0, 0};   // reduced solves started from 0, from g^, from the network
  int gnet_losses = 0;                    // reduced solves in a row in which the network's candidate lost
  // trial of the network against its absence: reduced solves alternate
  // between starting from the best of {0, g^, network} (arm 1) and of
  // {0, g^} (arm 0); arm of each column of the current application, the
  // solves and inner iterations per arm, and the alternation counter
  std::vector<int> garm;
  int64_t gtrial_n[2] = {0, 0}, gtrial_its[2] = {0, 0};
  int64_t gtrial_seq = 0;
  bool gtrial_done = false;
  int64_t gnet_skipped = 0;               // reduced solves started without trying (the network was retired)
  // last solve
  int last_k = 0;
  // timing
  bool tim_on[TK_N] = {};
  std::vector<TimingRec> tim[TK_N];
  std::vector<hipEvent_t> ev_pool;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double t_setup_ms = 0, t_factor_ms = 0, t_solve_ms = 0;
  int32_t bad_block = -1;
  int64_t bad_row = -1;
  std::vector<void*> allocs;
  size_t bytes = 0;

  template <typename T>
  int alloc(T*& ptr, int64_t count) {
    ptr = nullptr;
    if (count <= 0) return DDPS_OK;
    void* q = nullptr;
    const size_t sz = (size_t)count * sizeof(T);
    if (hipMalloc(&q, sz) != hipSuccess) return DDPS_E_NOMEM;
    allocs.push_back(q);
    bytes += sz;
    ptr = (T*)q;
    return DDPS_OK;
  }
  int alloc_raw(void*& ptr, size_t sz) {
    ptr = nullptr;
    if (sz == 0) return DDPS_OK;
    if (hipMalloc(&ptr, sz) != hipSuccess) return DDPS_E_NOMEM;
    allocs.push_back(ptr);
    bytes += sz;
    return DDPS_OK;
  }

  // ---- addressing -------------------------------------------------------
  // Elements of a pair of triangles: a t x (t+1) column-major array holding
  // a lower triangle (diagonal included) at offset 0 and an upper one at
  // offset t, both read with leading dimension t.
  int64_t pair_elems() const { return (int64_t)t * t + t; }
  // which 0: diagonal tile k; 1: A_{k+1,k} (upper half of pair k); 2:
  // A_{k,k+1} (lower half of pair k).  Halves are read through masks.
  char* tile(int i, int which, int k) const {
    const BlockInfo& B = blk[i];
    const int64_t tt = (int64_t)t * t;
    const int64_t idx = which == 0 ? B.tiles + k * tt
                                   : B.tiles + B.T * tt + k * pair_elems() + (which == 1 ? t : 0);
    return (char*)d_tiles + (size_t)idx * elt;
  }
  // L_{k+1,k} (which 1, upper triangular) or U_{k,k+1} (which 2, lower
  // triangular) of block i: halves of one pair
  char* lu(int i, int which, int k) const {
    if (!d_lu) return tile(i, which, k);
    const int64_t idx = lu_off[i] + k * pair_elems() + (which == 1 ? t : 0);
    return (char*)d_lu + (size_t)idx * elt;
  }
  // compact coupling store of block i: which 1 = left coupling C_i (upper),
  // 2 = right coupling B_i (lower)
  char* rhs(int i, int which) const {
    return (char*)d_rhs + (size_t)(i * pair_elems() + (which == 1 ? t : 0)) * elt;
  }
  // column-major tip part q (t x 2t, leading dimension t)
  char* tipcm(int64_t q) const { return (char*)d_tipcm + (size_t)(q * 2 * t * (int64_t)t) * elt; }
  // t x t spike tip of block i: its first t real rows (top) or last t rows,
  // against the left (half 0) or right (half 1) coupling columns, with its
  // leading dimension
  std::pair<char*, int> tipv(int i, bool top, int half) const {
    const BlockInfo& B = blk[i];
    if (tips_only) return {tipcm(top ? 2 * i - 1 : 2 * i) + (size_t)half * t * t * elt, t};
    return {spike(i, top ? B.pad : B.N - t, half ? t : 0), (int)B.N};
  }
  char* sub(char* tile_base, int r, int c) const {  // element (r, c) of a t x t tile
    return tile_base + ((size_t)c * t + r) * elt;
  }
  char* spike(int i, int64_t row, int64_t col) const {
    const BlockInfo& B = blk[i];
    return (char*)d_spikes + (size_t)(B.goff + col * B.N + row) * elt;
  }
  // scratch of block i: [WY | WA1 | WA2 | WB | WL | WU]: four t x t tiles,
  // then two t x (t/2 + 64) areas (leading dimension t) for the products of
  // the recursive triangle inversion
  static int64_t scratch_elems(int t) { return 4 * (int64_t)t * t + 2 * (int64_t)t * (t / 2 + 64); }
  char* scr(int i, int which) const {
    const int64_t tt = (int64_t)t * t, half = (int64_t)t * (t / 2 + 64);
    int64_t off = 0;
    switch (which) {
      case 0: off = 0; break;
      case 1: off = tt; break;
      case 2: off = 2 * tt; break;
      case 3: off = 3 * tt; break;
      case 4: off = 4 * tt; break;
      default: off = 4 * tt + half; break;
    }
    return (char*)d_scratch + (size_t)(wslot[i] * scr_per_block + off) * elt;
  }

  void tim_begin(int kind, hipEvent_t& a, hipStream_t s) {
    a = nullptr;
    if (!tim_on[kind] || capturing) return;
    a = get_event();
    (void)hipEventRecord(a, s);
  }
  void tim_begin(int kind, hipEvent_t& a) { tim_begin(kind, a, stream); }
  void tim_end(int kind, hipEvent_t a, double flops, double bytes_, hipStream_t s) {
    if (!a) return;
    hipEvent_t b2 = get_event();
    (void)hipEventRecord(b2, s);
    tim[kind].push_back({a, b2, flops, bytes_});
  }
  void tim_end(int kind, hipEvent_t a, double flops, double bytes_) { tim_end(kind, a, flops, bytes_, stream); }
  void free_ptr(void* q) {
    if (!q) return;
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == q) {
        allocs.erase(allocs.begin() + i);
        break;
      }
    (void)hipFree(q);
  }
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    drop_capture_events();
  }
  void drop_capture_events() {
    if (cap_fork) (void)hipEventDestroy(cap_fork);
    for (auto e : cap_gevent) (void)hipEventDestroy(e);
    cap_fork = nullptr;
    cap_gevent.clear();
  }
  hipEvent_t get_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
};

namespace {

// Flops of a problem as executed with BT x BT tiles (the K range of each
// tile clipped by the triangular structure, edge tiles counted at their size).
double gemm_prob_flops(const GemmProb& P, int BM, int BN) {
  double f = 0.0;
  for (int I0 = 0; I0 < P.M; I0 += BM)
    for (int J0 = 0; J0 < P.N; J0 += BN) {
      int kb = 0, ke = P.K;
      if (P.flags & G_A_UP) kb = std::max(kb, I0);
      if (P.flags & G_B_LO) kb = std::max(kb, J0);
      if (P.flags & G_A_LO) ke = std::min(ke, I0 + BM);
      if (P.flags & G_B_UP) ke = std::min(ke, J0 + BN);
      const int mm = std::min(BM, P.M - I0), nn = std::min(BN, P.N - J0);
      if (ke > kb) f += 2.0 * mm * nn * (ke - kb);
    }
  return f;
}

struct ScheduleBuilder {
  ddps_ctx* h;
  std::vector<GemmProb> gemm;
  std::vector<int32_t> order;   // tile orders (see tile_order)
  int64_t cur_ord = -1;
  std::vector<PanelProb> panel;
  std::vector<GemvProb> gemv;
  // current launch
  int kind = -1;
  int64_t off = 0;
  int nwg = 0;
  double flops = 0, bytes = 0;
  bool gemv_aligned = true;

  void begin(int k) {
    kind = k;
    nwg = 0;
    flops = bytes = 0;
    gemv_aligned = true;
    off = k == LK_GEMM ? (int64_t)gemm.size() : k == LK_PANEL ? (int64_t)panel.size() : (int64_t)gemv.size();
  }
  // Tile mode the policy asks for (0: 64 x 64, 1: 128 x 128, 2: 256 x 128).
  int requested_mode() const {
    if (h->tile_policy == 3)
      return h->mode_cursor < (int)h->mode_choice.size() ? h->mode_choice[h->mode_cursor] : 1;
    if (h->tile_policy == 4) return 3;
    if (h->tile_policy == 5) return 4;
    return h->tile_policy == 1 ? 0 : (h->tile_policy == 2 && h->gdt >= 2) ? 2 : 1;
  }
  // GEMM launches: the requested tile, narrowed to the largest one every
  // problem of the launch fills (256 x 128 only for bf16 arithmetic, 128 x 128,
  // else 64 x 64); assigns each problem its first workgroup.
  int finish_gemm() {
    int mode = requested_mode();
    if (mode >= 2 && h->gdt < 2) mode = 1;
    for (size_t q = (size_t)off; q < gemm.size(); ++q) {
      if (gemm[q].M < 128 || gemm[q].N < 128) mode = 0;
      else if (mode == 2 && gemm[q].M < 256) mode = 1;
      else if (mode == 4 && (gemm[q].M < 256 || gemm[q].N < 256)) mode = 3;
    }
    int BM, BN;
    gemm_tile_shape(h->gdt, mode, &BM, &BN);
    nwg = 0;
    flops = 0;
    for (size_t q = (size_t)off; q < gemm.size(); ++q) {
      GemmProb& P = gemm[q];
      P.tile0 = nwg;
      nwg += ((P.M + BM - 1) / BM) * ((P.N + BN - 1) / BN);
      flops += gemm_prob_flops(P, BM, BN);
    }
    tile_order(BM, BN);
    return mode;
  }
  // Dispatch order of the launch's tiles.  The kernels map workgroup b to
  // logical tile (b % 8) * (n / 8) + ... (a contiguous range per XCD, which
  // the XCD's CUs take in order).  Where triangular operands make the tiles'
  // K ranges unequal, each XCD's range is sorted longest first (stable), so
  // the short tiles fill in at the end instead of a long one starting last;
  // the XCD still gets the same tiles.  The kernel reads order[logical] for
  // the tile to compute.  Plain launches keep the identity (cur_ord = -1).
  void tile_order(int BM, int BN) {
    cur_ord = -1;
    bool tri = false;
    for (size_t q = (size_t)off; q < gemm.size(); ++q)
      tri = tri || (gemm[q].flags & (G_A_UP | G_A_LO | G_B_UP | G_B_LO));
    if (!tri || nwg < 2) return;
    std::vector<int32_t> klen(nwg);
    for (size_t q = (size_t)off; q < gemm.size(); ++q) {
      const GemmProb& P = gemm[q];
      const int tm = (P.M + BM - 1) / BM, tn = (P.N + BN - 1) / BN;
      for (int l = 0; l < tm * tn; ++l) {
        const int I0 = (l % tm) * BM, J0 = (l / tm) * BN;
        int kb = 0, ke = P.K;
        if (P.flags & G_A_UP) kb = std::max(kb, I0);
        if (P.flags & G_B_LO) kb = std::max(kb, J0);
        if (P.flags & G_A_LO) ke = std::min(ke, I0 + BM);
        if (P.flags & G_B_UP) ke = std::min(ke, J0 + BN);
        klen[P.tile0 + l] = std::max(0, ke - kb);
      }
    }
    cur_ord = (int64_t)order.size();
    order.resize(order.size() + nwg);
    int32_t* o = order.data() + cur_ord;
    const int per = nwg >> 3, rem = nwg & 7;
    for (int x = 0; x < 8; ++x) {
      const int lo = x * per + std::min(x, rem), cnt = per + (x < rem ? 1 : 0);
      for (int r = 0; r < cnt; ++r) o[lo + r] = lo + r;
      std::stable_sort(o + lo, o + lo + cnt, [&](int32_t a, int32_t b) { return klen[a] > klen[b]; });
    }
  }
  // GEMV kernel form of the current launch (see launch_gemv); the matrix
  // cores take FP32 operands only when the handle's factors are not FP64
  int gemv_form() const {
    if (!gemv_aligned) return 0;
    return (h->opt.factor_dtype != DDPS_F64 && h->opt.gemv_sums == 0) ? 2 : 1;
  }
  void end(std::vector<Launch>& out) {
    const int64_t cnt = (kind == LK_GEMM ? (int64_t)gemm.size() : kind == LK_PANEL ? (int64_t)panel.size()
                                                                              : (int64_t)gemv.size()) - off;
    const int mode = kind == LK_GEMM ? finish_gemm() : gemv_form();
    if (cnt > 0 && nwg > 0) {
      out.push_back({kind, off, (int)cnt, nwg, flops, bytes, mode, kind == LK_GEMM ? cur_ord : -1});
      if (kind == LK_GEMM) ++h->mode_cursor;
    }
  }
  Launch end_one() {
    const int64_t cnt = (kind == LK_GEMM ? (int64_t)gemm.size() : (int64_t)gemv.size()) - off;
    const int mode = kind == LK_GEMM ? finish_gemm() : gemv_form();
    return Launch{kind, off, (int)cnt, nwg, flops, bytes, mode, kind == LK_GEMM ? cur_ord : -1};
  }
  void add_gemm(const void* A, int lda, const void* B, int ldb, const void* C0, int ldc0, void* D, int ldd,
                int M, int N, int K, int flags) {
    if (M <= 0 || N <= 0) return;
    GemmProb P{};
    P.A = A; P.B = B; P.C0 = C0; P.D = D;
    P.M = M; P.N = N; P.K = K;
    P.lda = lda; P.ldb = ldb; P.ldc0 = ldc0; P.ldd = ldd;
    P.flags = flags | (C0 ? G_C0 : 0);
    gemm.push_back(P);
    nwg += 1;   // provisional: finish_gemm() assigns the tiles
  }
  void add_copy(const void* src, int lds, void* dst, int ldd, int M, int N) {
    add_gemm(nullptr, 0, nullptr, 0, src, lds, dst, ldd, M, N, 0, 0);
  }
  void add_panel(void* D, int ld, int block, int64_t row0, int64_t vrow0) {
    PanelProb P{};
    P.D = D; P.ld = ld; P.block = block; P.row0 = row0; P.vrow0 = vrow0;
    panel.push_back(P);
    nwg += 1;
    flops += 2.0 / 3.0 * 64 * 64 * 64 * 2.0;
  }
  void add_gemv(const GemvProb& G0, double elt_bytes) {
    GemvProb G = G0;
    if (G.rows <= 0) return;
    gemv_aligned = gemv_aligned && reinterpret_cast<uintptr_t>(G.A) % 16 == 0 &&
                   (G.lda * (int64_t)elt_bytes) % 16 == 0;
    G.wg0 = nwg;
    nwg += G.rows / 64;
    double cols = std::max(0, G.ce - G.cb);
    double frac = G.tri ? 0.5 : 1.0;
    flops += 2.0 * G.rows * cols * frac;
    bytes += (double)G.rows * cols * frac * elt_bytes + 8.0 * G.rows * 2;
    gemv.push_back(G);
  }
};

int fac_dtype_code(int d) {
  switch (d) {
    case DDPS_F64: return 0;
    case DDPS_F32: return 1;
    case DDPS_BF16X3: return 2;
    case DDPS_BF16: return 3;
    default: return -1;
  }
}

// One t x t tile of a schedule's tile LU: its storage (leading dimension t),
// two work areas of t x (t/2 + 64) for the inversion products, and the
// block, global row and padded-layout row (pivot threshold index) of its
// first row for the singular-pivot report.
struct TileLu {
  char* D;
  char* w4;
  char* w5;
  int block;
  int64_t row0, vrow0;
};

// Unpivoted LU of every tile of `items` in place, batched over the tiles,
// then the inverses of both triangles: on exit a tile holds L^{-1} strictly
// below the diagonal (unit diagonal implied) and U^{-1} on and above it.
void build_tile_lu(ddps_ctx* h, ScheduleBuilder& sb, const std::vector<TileLu>& items, std::vector<Launch>& S) {
  const int t = h->t, Q = t / 64;
  // LU in 64-column panels (panel LU with the inverses of its 64 x 64
  // triangles, then column and row panels), blocked in two levels: inside
  // an outer panel of kOuter columns [J0, J1) each 64-column step updates
  // only the rows of the outer panel (all columns to its right) and the
  // columns of the outer panel (all rows below); the rest of the trailing
  // matrix, rows and columns >= J1, takes the sum of those steps' products
  // as one rank-(J1 - J0) update after the outer panel.  Same products as a
  // rank-64 update per step, grouped so that the trailing matrix is read
  // and written once per outer panel instead of once per step.
  constexpr int kOuter = 256;
  for (int J0 = 0; J0 < t; J0 += kOuter) {
    const int J1 = std::min(t, J0 + kOuter);
    for (int j64 = J0; j64 < J1; j64 += 64) {
      const int rest = t - j64 - 64, w = J1 - j64 - 64;
      sb.begin(LK_PANEL);
      for (const TileLu& it : items) sb.add_panel(h->sub(it.D, j64, j64), t, it.block, it.row0 + j64, it.vrow0 + j64);
      sb.end(S);
      if (rest <= 0) continue;
      sb.begin(LK_GEMM);
      for (const TileLu& it : items) {
        char* D = it.D;
        sb.add_gemm(h->sub(D, j64 + 64, j64), t, h->sub(D, j64, j64), t, nullptr, 0, h->sub(D, j64 + 64, j64), t,
                    rest, 64, 64, G_B_MUP | G_B_UP);
        sb.add_gemm(h->sub(D, j64, j64), t, h->sub(D, j64, j64 + 64), t, nullptr, 0, h->sub(D, j64, j64 + 64), t,
                    64, rest, 64, G_A_MLU | G_A_LO);
      }
      sb.end(S);
      if (w <= 0) continue;
      sb.begin(LK_GEMM);
      for (const TileLu& it : items) {
        char* D = it.D;
        // rows of the outer panel below this step, every column to the right
        sb.add_gemm(h->sub(D, j64 + 64, j64), t, h->sub(D, j64, j64 + 64), t, h->sub(D, j64 + 64, j64 + 64), t,
                    h->sub(D, j64 + 64, j64 + 64), t, w, rest, 64, G_NEG);
        // rows below the outer panel, columns of the outer panel
        if (t > J1)
          sb.add_gemm(h->sub(D, J1, j64), t, h->sub(D, j64, j64 + 64), t, h->sub(D, J1, j64 + 64), t,
                      h->sub(D, J1, j64 + 64), t, t - J1, w, 64, G_NEG);
      }
      sb.end(S);
    }
    if (t > J1) {
      sb.begin(LK_GEMM);
      for (const TileLu& it : items) {
        char* D = it.D;
        sb.add_gemm(h->sub(D, J1, J0), t, h->sub(D, J0, J1), t, h->sub(D, J1, J1), t, h->sub(D, J1, J1), t, t - J1,
                    t - J1, J1 - J0, G_NEG);
      }
      sb.end(S);
    }
  }
  // inverse triangles of the whole tile by recursive halving of the panel
  // range: for a split [lo, mid) | [mid, hi) whose halves are inverted,
  //   X10 = -X11 (L10 X00),   Y01 = -(Y00 U01) Y11
  // (X = L^{-1}, Y = U^{-1}); all splits of one depth, over all blocks,
  // share a launch pair.
  {
    std::vector<std::vector<std::array<int, 3>>> levels;
    std::function<void(int, int, int)> rec = [&](int lo, int hi, int d) {
      if (hi - lo <= 1) return;
      const int mid = (lo + hi) / 2;
      if ((int)levels.size() <= d) levels.resize(d + 1);
      levels[d].push_back({lo, mid, hi});
      rec(lo, mid, d + 1);
      rec(mid, hi, d + 1);
    };
    rec(0, Q, 0);
    for (int d = (int)levels.size() - 1; d >= 0; --d) {
      sb.begin(LK_GEMM);
      for (const TileLu& it : items) {
        char* D = it.D;
        for (auto& c : levels[d]) {
          const int lo = c[0] * 64, mid = c[1] * 64, hi = c[2] * 64;
          const int m0 = mid - lo, m1 = hi - mid;
          sb.add_gemm(h->sub(D, mid, lo), t, h->sub(D, lo, lo), t, nullptr, 0, it.w4 + (size_t)mid * h->elt, t,
                      m1, m0, m0, G_B_MLU | G_B_LO);
          sb.add_gemm(h->sub(D, lo, lo), t, h->sub(D, lo, mid), t, nullptr, 0, it.w5 + (size_t)lo * h->elt, t,
                      m0, m1, m0, G_A_MUP | G_A_UP);
        }
      }
      sb.end(S);
      sb.begin(LK_GEMM);
      for (const TileLu& it : items) {
        char* D = it.D;
        for (auto& c : levels[d]) {
          const int lo = c[0] * 64, mid = c[1] * 64, hi = c[2] * 64;
          const int m0 = mid - lo, m1 = hi - mid;
          sb.add_gemm(h->sub(D, mid, mid), t, it.w4 + (size_t)mid * h->elt, t, nullptr, 0, h->sub(D, mid, lo), t,
                      m1, m0, m1, G_NEG | G_A_MLU | G_A_LO);
          sb.add_gemm(it.w5 + (size_t)lo * h->elt, t, h->sub(D, mid, mid), t, nullptr, 0, h->sub(D, lo, mid), t,
                      m0, m1, m1, G_NEG | G_B_MUP | G_B_UP);
        }
      }
      sb.end(S);
    }
  }
}

// Factor schedule of the blocks in `members` (ascending), appended to S.
void build_factor_schedule(ddps_ctx* h, ScheduleBuilder& sb, const std::vector<int>& members,
                           std::vector<Launch>& S) {
  const int t = h->t, p = h->p;
  int Tmax = 0;
  for (int i : members) Tmax = std::max<int>(Tmax, (int)h->blk[i].T);
  for (int k = 0; k < Tmax; ++k) {
    std::vector<int> act;
    for (int i : members)
      if (h->blk[i].T > k) act.push_back(i);
    // pre(k): Schur update, top-spike right-hand side, staging copies
    sb.begin(LK_GEMM);
    for (int i : act) {
      const BlockInfo& B = h->blk[i];
      const int N = (int)B.N;
      if (k >= 1)
        sb.add_gemm(h->lu(i, 1, k - 1), t, h->lu(i, 2, k - 1), t, h->tile(i, 0, k), t, h->tile(i, 0, k), t,
                    t, t, t, G_NEG | G_A_UP | G_A_MUP | G_B_LO | G_B_MLO);
      if (i > 0) {
        // the right-hand side of the left spike is nonzero in rows < 2t only
        if (k >= 1)
          sb.add_gemm(h->lu(i, 1, k - 1), t, h->spike(i, (int64_t)(k - 1) * t, 0), N,
                      (int64_t)k * t < 2 * (int64_t)t ? h->spike(i, (int64_t)k * t, 0) : nullptr, N, h->scr(i, 0), t,
                      t, t, t, G_NEG | G_A_UP | G_A_MUP);
        else
          sb.add_copy(h->spike(i, 0, 0), N, h->scr(i, 0), t, t, t);
      }
      if (k < B.T - 1 && !h->d_lu) {   // the factors overwrite the coupling tiles: copies of A's entries
        sb.add_copy(h->tile(i, 1, k), t, h->scr(i, 1), t, t, t);
        sb.add_copy(h->tile(i, 2, k), t, h->scr(i, 2), t, t, t);
      }
      if (k == B.T - 1 && i < p - 1) sb.add_copy(h->spike(i, (int64_t)k * t, t), N, h->scr(i, 3), t, t, t);
    }
    sb.end(S);
    {
      std::vector<TileLu> items;
      for (int i : act) {
        const BlockInfo& B = h->blk[i];
        items.push_back({h->tile(i, 0, k), h->scr(i, 4), h->scr(i, 5), i, B.s - B.pad + (int64_t)k * t,
                         B.voff + (int64_t)k * t});
      }
      build_tile_lu(h, sb, items, S);
    }
    // post(k): off-diagonal factors and forward spike sweep
    sb.begin(LK_GEMM);
    for (int i : act) {
      const BlockInfo& B = h->blk[i];
      const int N = (int)B.N;
      char* D = h->tile(i, 0, k);
      if (k < B.T - 1) {
        const char* a_lo = h->d_lu ? h->tile(i, 1, k) : h->scr(i, 1);   // A_{k+1,k}
        const char* a_up = h->d_lu ? h->tile(i, 2, k) : h->scr(i, 2);   // A_{k,k+1}
        // each product writes its own half of the pair
        sb.add_gemm(a_lo, t, D, t, nullptr, 0, h->lu(i, 1, k), t, t, t, t,
                    G_A_UP | G_A_MUP | G_B_MUP | G_B_UP | G_D_UP);
        sb.add_gemm(D, t, a_up, t, nullptr, 0, h->lu(i, 2, k), t, t, t, t,
                    G_A_MLU | G_A_LO | G_B_LO | G_B_MLO | G_D_LO);
      }
      if (i > 0) sb.add_gemm(D, t, h->scr(i, 0), t, nullptr, 0, h->spike(i, (int64_t)k * t, 0), N, t, t, t, G_A_MLU | G_A_LO);
      if (k == B.T - 1 && i < p - 1)
        sb.add_gemm(D, t, h->scr(i, 3), t, nullptr, 0, h->spike(i, (int64_t)k * t, t), N, t, t, t,
                    G_A_MLU | G_A_LO | G_B_LO);
    }
    sb.end(S);
  }
  // backward spike sweep over all spike columns
  if (p > 1) {
    for (int s = 0; s < Tmax; ++s) {
      std::vector<int> act;
      for (int i : members)
        if (h->blk[i].T > s) act.push_back(i);
      sb.begin(LK_GEMM);
      for (int i : act) {
        const BlockInfo& B = h->blk[i];
        const int N = (int)B.N, k = (int)B.T - 1 - s;
        const int c0 = i == 0 ? t : 0, c1 = i == p - 1 ? t : 2 * t;
        char* W = h->scr(i, 0) + (size_t)c0 * t * h->elt;
        if (k < B.T - 1) {
          // left columns: W = G_k - U_{k,k+1} G_{k+1}; right columns: the
          // forward sweep left them zero above the last tile row
          const int cm = std::max(c0, t);
          if (cm > c0)
            sb.add_gemm(h->lu(i, 2, k), t, h->spike(i, (int64_t)(k + 1) * t, c0), N,
                        h->spike(i, (int64_t)k * t, c0), N, W, t, t, cm - c0, t, G_NEG | G_A_LO | G_A_MLO);
          if (c1 > cm)
            sb.add_gemm(h->lu(i, 2, k), t, h->spike(i, (int64_t)(k + 1) * t, cm), N, nullptr, 0,
                        h->scr(i, 0) + (size_t)cm * t * h->elt, t, t, c1 - cm, t, G_NEG | G_A_LO | G_A_MLO);
        } else {
          sb.add_copy(h->spike(i, (int64_t)k * t, c0), N, W, t, t, c1 - c0);
        }
      }
      sb.end(S);
      sb.begin(LK_GEMM);
      for (int i : act) {
        const BlockInfo& B = h->blk[i];
        const int N = (int)B.N, k = (int)B.T - 1 - s;
        const int c0 = i == 0 ? t : 0, c1 = i == p - 1 ? t : 2 * t;
        char* W = h->scr(i, 0) + (size_t)c0 * t * h->elt;
        sb.add_gemm(h->tile(i, 0, k), t, W, t, nullptr, 0, h->spike(i, (int64_t)k * t, c0), N, t, c1 - c0, t,
                    G_A_MUP | G_A_UP);
      }
      sb.end(S);
    }
  }
}

// Tips only: the spike right-hand sides of one batch into its workspace
// slots.  The regions the factorisation reads as right-hand sides are
// cleared (rows [0, 2t) of the left-coupling columns, the last t rows of the
// right-coupling columns), then the left coupling C_i (upper triangular)
// lands at rows [pad, pad + t) and the right coupling B_i (lower triangular)
// at the last t rows, each copied through an output mask from its half of
// the compact store.
void build_batch_rhs(ddps_ctx* h, ScheduleBuilder& sb, const std::vector<int>& mem, std::vector<Launch>& S) {
  const int t = h->t, p = h->p;
  sb.begin(LK_GEMM);
  for (int i : mem) {
    const BlockInfo& B = h->blk[i];
    const int N = (int)B.N;
    if (i > 0) sb.add_copy(nullptr, 0, h->spike(i, 0, 0), N, 2 * t, t);
    if (i < p - 1) sb.add_copy(nullptr, 0, h->spike(i, B.N - t, t), N, t, t);
  }
  sb.end(S);
  sb.begin(LK_GEMM);
  for (int i : mem) {
    const BlockInfo& B = h->blk[i];
    const int N = (int)B.N;
    if (i > 0) sb.add_gemm(nullptr, 0, nullptr, 0, h->rhs(i, 1), t, h->spike(i, B.pad, 0), N, t, t, 0, G_D_UP);
    if (i < p - 1) sb.add_gemm(nullptr, 0, nullptr, 0, h->rhs(i, 2), t, h->spike(i, B.N - t, t), N, t, t, 0, G_D_LO);
  }
  sb.end(S);
}

// Tips only: after a batch's backward sweep, its spike tips (the first t
// real rows and the last t rows of every G_i, all 2t columns) are copied to
// the tip store, which is all the reduced system needs.
void build_batch_tips(ddps_ctx* h, ScheduleBuilder& sb, const std::vector<int>& mem, std::vector<Launch>& S) {
  const int t = h->t, p = h->p;
  sb.begin(LK_GEMM);
  for (int i : mem) {
    const BlockInfo& B = h->blk[i];
    if (i > 0) sb.add_copy(h->spike(i, B.pad, 0), (int)B.N, h->tipcm(2 * i - 1), t, t, 2 * t);
    if (i < p - 1) sb.add_copy(h->spike(i, B.N - t, 0), (int)B.N, h->tipcm(2 * i), t, t, 2 * t);
  }
  sb.end(S);
}

// Direct solve of the reduced system (Figure 2, step 6.3 solved "directly").
// In the interface ordering (interface j = the last t rows of block j, a_j,
// then the first t rows of block j+1, b_j) G^ is block tridiagonal with
// 2t x 2t blocks: D_j = [[I, V_j^bot], [W_{j+1}^top, I]], the coupling of
// a_j to a_{j-1} is W_j^bot and that of b_j to b_{j+1} is V_{j+1}^top (W, V:
// the left and right spikes, ^top / ^bot their first / last t rows).  Block
// LU without pivoting then keeps the identity diagonal blocks:
//   S_j = [[I, P_j], [Q_j, I]],  Q_j = W_{j+1}^top,
//   P_0 = V_0^bot,  P_j = V_j^bot - W_j^bot Y_{j-1} V_j^top,
//   Y_j = -Sigma_j^{-1} P_j (the top-right block of S_j^{-1}),
//   Sigma_j = I - P_j Q_j,
// so each interface factors one t x t matrix Sigma_j (unpivoted, inverse
// triangles), a sequential chain over the interfaces.  Its forward and
// backward substitutions apply S_j^{-1}[u; v] = [x1; v - Q_j x1] with
// x1 = Sigma_j^{-1}(u - P_j v).  The tips are used unmasked: columns of G
// outside c are zero, so the solution on c is that of the masked system, and
// the entries outside c are zeroed afterwards.
void build_reduced_direct(ddps_ctx* h, ScheduleBuilder& sb) {
  h->sch_rfac.clear();
  h->sch_rsol.clear();
  h->sums.clear();
  if (!h->d_rP || h->p < 2) return;
  const int t = h->t, M = h->p - 1;
  const size_t tt = (size_t)t * t * h->elt;
  auto rP = [&](int j) { return (char*)h->d_rP + (size_t)j * tt; };
  auto rS = [&](int j) { return (char*)h->d_rS + (size_t)j * tt; };
  char* W = (char*)h->d_rW;
  char *T1 = W, *T2 = W + tt, *Y[2] = {W + 2 * tt, W + 3 * tt}, *I = W + 4 * tt, *w4 = W + 5 * tt;
  char* w5 = w4 + (size_t)t * (t / 2 + 64) * h->elt;
  // these launches hold one t x t problem each: 64 x 64 tiles fill the GPU
  // best; they leave the factor schedule's per-launch tile choices (read by
  // launch index) alone
  const int pol = h->tile_policy, cur = h->mode_cursor;
  h->tile_policy = 1;
  for (int j = 0; j < M; ++j) {
    auto Vb = h->tipv(j, false, 1), Wb = h->tipv(j, false, 0), Q = h->tipv(j + 1, true, 0);
    sb.begin(LK_GEMM);
    if (j == 0) {
      sb.add_copy(Vb.first, Vb.second, rP(0), t, t, t);
    } else {
      auto Vt = h->tipv(j, true, 1);
      sb.add_gemm(Y[(j - 1) & 1], t, Vt.first, Vt.second, nullptr, 0, T1, t, t, t, t, 0);
      sb.end(h->sch_rfac);
      sb.begin(LK_GEMM);
      sb.add_gemm(Wb.first, Wb.second, T1, t, Vb.first, Vb.second, rP(j), t, t, t, t, G_NEG);
    }
    sb.end(h->sch_rfac);
    sb.begin(LK_GEMM);
    sb.add_gemm(rP(j), t, Q.first, Q.second, I, t, rS(j), t, t, t, t, G_NEG);
    sb.end(h->sch_rfac);
    build_tile_lu(h, sb, {TileLu{rS(j), w4, w5, h->p, (int64_t)j * 2 * t, h->Np}}, h->sch_rfac);
    if (j < M - 1) {
      sb.begin(LK_GEMM);
      sb.add_gemm(rS(j), t, rP(j), t, nullptr, 0, T2, t, t, t, t, G_A_MLU | G_A_LO);
      sb.end(h->sch_rfac);
      sb.begin(LK_GEMM);
      sb.add_gemm(rS(j), t, T2, t, nullptr, 0, Y[j & 1], t, t, t, t, G_NEG | G_A_MUP | G_A_UP);
      sb.end(h->sch_rfac);
    }
  }
  h->tile_policy = pol;
  h->mode_cursor = cur;
  // substitutions on d_zh (holding g^ on entry), with temporaries in d_r,
  // d_p.  Each t x t product is one launch of `ns` column ranges (partial
  // products in d_tv, part q at offset q t) and one fixed-order sum: a single
  // t x t product has only t/64 row slabs, too few to keep the GPU's loads
  // in flight.
  const double eb = (double)h->elt;
  double* z = h->d_zh;
  double* tmp = h->d_r;
  double* tmp2 = h->d_p;
  double* parts = h->d_tv;
  const int ns = std::max(1, std::min<int>({8, 2 * M, t / 64}));
  auto vec = [&](int j, int half) { return z + (int64_t)(2 * j + half) * t; };
  auto gemv = [&](const char* A, int lda, const double* x, const double* yin, double* yout, int flags, int tri) {
    sb.begin(LK_GEMV);
    for (int q = 0; q < ns; ++q) {
      GemvProb G{};
      G.A = A;
      G.lda = lda;
      G.x1 = x;
      G.x2 = x;
      G.split = t;
      G.rows = t;
      G.cb = (int)((int64_t)t * q / ns);
      G.ce = (int)((int64_t)t * (q + 1) / ns);
      G.yout = parts + (int64_t)q * t;
      G.flags = flags & (V_A_MLU | V_A_MUP | V_A_MLO);
      G.tri = tri;
      sb.add_gemv(G, eb);
    }
    sb.end(h->sch_rsol);
    h->sums.push_back(SumRec{parts, t, yin, yout, t, ns, (flags & V_NEG) ? 1 : 0});
    h->sch_rsol.push_back(Launch{LK_SUM, (int64_t)h->sums.size() - 1, 1, (t + 255) / 256, 0.0, 0.0, 0, -1});
  };
  for (int j = 1; j < M; ++j) {
    // w_j(a) -= W_j^bot x1, x1 = Sigma_{j-1}^{-1}(u_{j-1} - P_{j-1} v_{j-1})
    gemv(rP(j - 1), t, vec(j - 1, 1), vec(j - 1, 0), tmp, V_NEG, 0);
    gemv(rS(j - 1), t, tmp, nullptr, tmp2, V_A_MLU, 1);
    gemv(rS(j - 1), t, tmp2, nullptr, tmp, V_A_MUP, 2);
    auto Wb = h->tipv(j, false, 0);
    gemv(Wb.first, Wb.second, tmp, vec(j, 0), vec(j, 0), V_NEG, 0);
  }
  for (int j = M - 1; j >= 0; --j) {
    if (j < M - 1) {
      auto Vt = h->tipv(j + 1, true, 1);
      gemv(Vt.first, Vt.second, vec(j + 1, 1), vec(j, 1), vec(j, 1), V_NEG, 0);
    }
    gemv(rP(j), t, vec(j, 1), vec(j, 0), tmp, V_NEG, 0);
    gemv(rS(j), t, tmp, nullptr, tmp2, V_A_MLU, 1);
    gemv(rS(j), t, tmp2, nullptr, vec(j, 0), V_A_MUP, 2);
    auto Q = h->tipv(j + 1, true, 0);
    gemv(Q.first, Q.second, vec(j, 0), vec(j, 1), vec(j, 1), V_NEG, 0);
  }
}

void build_solve_schedules(ddps_ctx* h, ScheduleBuilder& sb) {
  const int t = h->t, p = h->p;
  const double eb = (double)h->elt;
  double* yp = h->d_ypad;
  double* vp = h->d_vpad;
  // (incomplete factors: the block solves are level-scheduled kernels, no tile sweeps)
  for (int k = 0; k < (h->ilu ? 0 : h->Tmax); ++k) {
    sb.begin(LK_GEMV);
    for (int i = 0; i < p; ++i) {
      const BlockInfo& B = h->blk[i];
      if (B.T <= k) continue;
      GemvProb G{};
      G.A = k >= 1 ? h->lu(i, 1, k - 1) : h->tile(i, 0, k);
      G.lda = t;
      G.x1 = yp + B.voff + (int64_t)(k >= 1 ? k - 1 : 0) * t;
      G.x2 = G.x1;
      G.split = t;
      G.rows = t;
      G.cb = 0;
      G.ce = k >= 1 ? t : 0;
      G.yin = yp + B.voff + (int64_t)k * t;
      G.yout = vp + B.voff + (int64_t)k * t;
      G.flags = V_NEG | V_YIN | (k >= 1 ? V_A_MUP : 0);   // L_{k,k-1}: upper half of a pair
      G.tri = 2;
      sb.add_gemv(G, eb);
    }
    sb.end(h->sch_fwd);
    sb.begin(LK_GEMV);
    for (int i = 0; i < p; ++i) {
      const BlockInfo& B = h->blk[i];
      if (B.T <= k) continue;
      GemvProb G{};
      G.A = h->tile(i, 0, k);
      G.lda = t;
      G.x1 = vp + B.voff + (int64_t)k * t;
      G.x2 = G.x1;
      G.split = t;
      G.rows = t;
      G.cb = 0;
      G.ce = t;
      G.yout = yp + B.voff + (int64_t)k * t;
      G.flags = V_A_MLU;
      G.tri = 1;
      sb.add_gemv(G, eb);
    }
    sb.end(h->sch_fwd);
  }
  for (int s = 0; s < (h->ilu ? 0 : h->Tmax); ++s) {
    sb.begin(LK_GEMV);
    for (int i = 0; i < p; ++i) {
      const BlockInfo& B = h->blk[i];
      if (B.T <= s) continue;
      const int k = (int)B.T - 1 - s;
      GemvProb G{};
      G.A = k < B.T - 1 ? h->lu(i, 2, k) : h->tile(i, 0, k);
      G.lda = t;
      G.x1 = yp + B.voff + (int64_t)(k < B.T - 1 ? k + 1 : k) * t;
      G.x2 = G.x1;
      G.split = t;
      G.rows = t;
      G.cb = 0;
      G.ce = k < B.T - 1 ? t : 0;
      G.yin = yp + B.voff + (int64_t)k * t;
      G.yout = vp + B.voff + (int64_t)k * t;
      G.flags = V_NEG | V_YIN | (k < B.T - 1 ? V_A_MLO : 0);   // U_{k,k+1}: lower half of a pair
      G.tri = 1;
      sb.add_gemv(G, eb);
    }
    sb.end(h->sch_bwd);
    sb.begin(LK_GEMV);
    for (int i = 0; i < p; ++i) {
      const BlockInfo& B = h->blk[i];
      if (B.T <= s) continue;
      const int k = (int)B.T - 1 - s;
      GemvProb G{};
      G.A = h->tile(i, 0, k);
      G.lda = t;
      G.x1 = vp + B.voff + (int64_t)k * t;
      G.x2 = G.x1;
      G.split = t;
      G.rows = t;
      G.cb = 0;
      G.ce = t;
      G.yout = yp + B.voff + (int64_t)k * t;
      G.flags = V_A_MUP;
      G.tri = 2;
      sb.add_gemv(G, eb);
    }
    sb.end(h->sch_bwd);
  }
  // retrieval z = g - G z^ into vpad (with the full spikes only)
  sb.begin(LK_GEMV);
  for (int i = 0; i < p && !h->tips_only; ++i) {
    const BlockInfo& B = h->blk[i];
    GemvProb G{};
    G.A = h->spike(i, 0, 0);
    G.lda = B.N;
    G.x1 = h->d_zh + (i > 0 ? (int64_t)2 * (i - 1) * t : 0);
    G.x2 = h->d_zh + (i < p - 1 ? (int64_t)(2 * i + 1) * t : 0);
    G.split = t;
    G.rows = (int)B.N;
    G.cb = (i == 0 || p == 1) ? t : 0;
    G.ce = (i == p - 1) ? t : 2 * t;
    if (p == 1) G.cb = G.ce = 0;
    G.yin = yp + B.voff;
    G.yout = vp + B.voff;
    G.flags = V_NEG | V_YIN;
    G.tri = 0;
    sb.add_gemv(G, eb);
  }
  sb.end(h->sch_retr);
  // reduced products
  // local = true: only the interface-local part N of G(c,c) (top rows of a
  // block against its left-coupling columns, bottom rows against its right
  // ones), Y = X - N X
  auto reduced = [&](const double* X, double* Y, const double* dotv, int dflags, bool local = false) {
    sb.begin(h->tip_nseg > 0 ? LK_TIPMV : LK_GEMV);
    for (int i = 0; i < p && p > 1; ++i) {
      const BlockInfo& B = h->blk[i];
      for (int part = 0; part < 2; ++part) {
        if (part == 0 && i == 0) continue;
        if (part == 1 && i == p - 1) continue;
        const int64_t ro = part == 0 ? (int64_t)(2 * i - 1) * t : (int64_t)2 * i * t;
        GemvProb G{};
        if (h->tip_nseg > 0) {
          // packed part q = 2i - 1 (first t rows of block i) or 2i (last t rows)
          const int64_t q = part == 0 ? 2 * i - 1 : 2 * i;
          G.A = (const char*)h->d_tips + (size_t)q * t * 2 * t * h->elt;
          G.lda = 2 * t;
        } else if (h->tips_only) {
          G.A = h->tipcm(part == 0 ? 2 * i - 1 : 2 * i);
          G.lda = t;
        } else {
          G.A = h->spike(i, part == 0 ? B.pad : B.N - t, 0);
          G.lda = B.N;
        }
        G.x1 = X + (i > 0 ? (int64_t)2 * (i - 1) * t : 0);
        G.x2 = X + (i < p - 1 ? (int64_t)(2 * i + 1) * t : 0);
        G.split = t;
        G.rows = t;
        G.cb = i == 0 ? t : 0;
        G.ce = i == p - 1 ? t : 2 * t;
        if (local) {
          G.cb = part == 0 ? 0 : t;
          G.ce = part == 0 ? t : 2 * t;
        }
        G.yin = X + ro;
        G.yout = Y + ro;
        G.mask = h->d_mask + ro;
        G.dot_off = ro;
        G.flags = V_YIN | V_MASK | dflags | (local ? V_NEG : 0);
        G.tri = 0;
        sb.add_gemv(G, eb);
      }
    }
    (void)dotv;
    return sb.end_one();
  };
  h->l_pv = reduced(h->d_p, h->d_v, h->d_rt, V_DOT);
  h->l_st = reduced(h->d_s, h->d_tv, h->d_s, V_DOT | V_DOT2);
  h->l_zv = reduced(h->d_zh, h->d_v, nullptr, 0);
  if (h->opt.inner_prec == 1) {
    h->l_lp = reduced(h->d_p, h->d_mp, nullptr, 0, true);
    h->l_ls = reduced(h->d_s, h->d_ms, nullptr, 0, true);
    h->l_pvh = reduced(h->d_mp, h->d_v, h->d_rt, V_DOT);
    h->l_sth = reduced(h->d_ms, h->d_tv, h->d_s, V_DOT | V_DOT2);
  }
  h->W1 = h->l_pv.nwg;
}

int run_launch(ddps_ctx* h, const Launch& L, int R, int64_t ldx, int64_t ldy, const double* dotv,
               double* partial, const int32_t* stop, int tkind, hipStream_t s) {
  hipEvent_t a;
  h->tim_begin(tkind, a, s);
  switch (L.kind) {
    case LK_GEMM:
      launch_gemm(h->gdt, L.mode, h->d_gemm + L.off, L.nprob, L.nwg, s, L.ord >= 0 ? h->d_order + L.ord : nullptr);
      break;
    case LK_PANEL: launch_panel(h->sdt, h->d_panel + L.off, L.nprob, h->d_thresh, h->d_bad, s); break;
    case LK_SUM: {
      const SumRec& q = h->sums[L.off];
      sum_parts(q.rows, R, q.ns, q.parts, q.pstride, ldy, q.yin, q.yout, q.neg, s);
      break;
    }
    case LK_TIPMV:
      launch_tipmv(h->sdt, R, h->tip_nseg, h->d_gemv + L.off, L.nprob, L.nwg, ldx, ldy, dotv, partial, stop, s);
      break;
    default:
      launch_gemv(h->sdt, R, L.mode, h->d_gemv + L.off, L.nprob, L.nwg, ldx, ldy, dotv, partial, stop, s);
      break;
  }
  h->tim_end(tkind, a, L.flops * (L.kind == LK_GEMV || L.kind == LK_TIPMV ? R : 1), L.bytes, s);
  return DDPS_OK;
}
int run_launch(ddps_ctx* h, const Launch& L, int R, int64_t ldx, int64_t ldy, const double* dotv,
               double* partial, const int32_t* stop, int tkind) {
  return run_launch(h, L, R, ldx, ldy, dotv, partial, stop, tkind, h->stream);
}

int rhs_alloc(int k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8; }

// Default number of stream groups: enough to overlap one group's
// latency-bound panel launches with the others' GEMMs, while each group
// still has several blocks per launch.
int default_groups(const ddps_ctx* h) { return std::max(1, std::min(4, h->p / 8)); }

// ---------------------------------------------------------------- phases
int do_scatter(ddps_ctx* h, hipStream_t s) {
  const int64_t tcount = h->tile_elems;
  // Spikes: the first factorisation zeroes the whole array (the halves no
  // block uses stay zero for good); later ones only the coupling parts that
  // the scatter fills, since the sweeps write every other entry before it
  // is read.  A fill recorded into a graph under capture has not run yet.
  // With the tips only, the coupling entries go to the compact store (zeroed
  // here, since the scatter adds into it) and each batch of the
  // factorisation places them in its workspace slots.
  const bool whole = !h->spikes_zeroed;
  const int64_t rcount = h->tips_only ? (int64_t)h->p * h->pair_elems() : 0;
  if (h->sdt == 0) {
    fill_f64((double*)h->d_tiles, tcount, 0.0, s);
    if (whole) fill_f64((double*)h->d_spikes, h->nspike, 0.0, s);
    fill_f64((double*)h->d_rhs, rcount, 0.0, s);
  } else {
    fill_f32((float*)h->d_tiles, tcount, 0.f, s);
    if (whole) fill_f32((float*)h->d_spikes, h->nspike, 0.f, s);
    fill_f32((float*)h->d_rhs, rcount, 0.f, s);
  }
  if (!whole && !h->tips_only) zero_spike_rhs(h->sdt, h->p, h->t, h->d_blk, h->d_spikes, s);
  if (!h->capturing) h->spikes_zeroed = true;
  fill_u64(h->d_colnorm, (int64_t)h->p * 2 * h->t, 0ull, s);
  fill_u64(h->d_bad, 1, ~0ull, s);
  fill_f64(h->d_mask, h->m, 0.0, s);
  setup_scatter(h->sdt, h->n, h->p, h->t, h->d_part, h->d_blk, h->d_rowptr, h->d_col, h->d_val, h->d_tiles,
                h->d_spikes, h->tips_only ? h->d_rhs : nullptr, h->d_colnorm, h->d_flags, s);
  setup_mask(h->sdt, h->p, h->t, h->opt.drop_delta, h->d_blk, h->d_colnorm, h->d_mask, h->d_spikes,
             h->tips_only ? h->d_rhs : nullptr, s);
  return DDPS_OK;
}

int run_schedule(ddps_ctx* h, const std::vector<Launch>& S, int R, int64_t ldx, int64_t ldy, int tk_gemv,
                 hipStream_t s, int tk_all = -1) {
  for (const Launch& L : S) {
    const int tk = tk_all >= 0 ? tk_all : L.kind == LK_GEMM ? TK_GEMM : L.kind == LK_PANEL ? TK_PANEL : tk_gemv;
    run_launch(h, L, R, ldx, ldy, nullptr, nullptr, nullptr, tk, s);
  }
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}
int run_schedule(ddps_ctx* h, const std::vector<Launch>& S, int R, int64_t ldx, int64_t ldy, int tk_gemv) {
  return run_schedule(h, S, R, ldx, ldy, tk_gemv, h->stream);
}

// Stages 2 and 4 with incomplete factors: ILU(0) of every block, then the
// spikes batch by batch (only their tips kept), then the direct reduced
// solve's factorisation if asked for.
int enqueue_factor_ilu(ddps_ctx* h) {
  hipStream_t f = h->fstream;
  int rc = do_scatter(h, f);
  if (rc) return rc;
  ilu_factor(h->p, h->d_iblk, h->d_lrows, h->d_lptr, h->d_ilo, h->d_idg, h->d_ihi, h->d_col, h->d_val, h->d_fv,
             h->d_thresh, h->d_bad, f);
  if (h->tips_only)
    for (const auto& b : h->ilu_batches)
      ilu_spikes(h->sdt, b.second, h->d_iblk, h->d_ibatch + b.first, h->p, h->t, h->d_rhs, h->d_ilo, h->d_idg,
                 h->d_ihi, h->d_col, h->d_fv, h->d_iws, h->ilu_nmax * 2 * h->t, h->d_tipcm, f);
  if ((rc = run_schedule(h, h->sch_rfac, 1, 0, 0, TK_GEMM, f, TK_RFAC))) return rc;
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

// Stages 1-5 on the internal factor stream: scatter, then every group's
// schedule on its own stream (fork/join through events).
int enqueue_factor(ddps_ctx* h) {
  if (h->ilu) return enqueue_factor_ilu(h);
  hipStream_t f = h->fstream;
  int rc = do_scatter(h, f);
  if (rc) return rc;
  const int G = (int)h->sch_group.size();
  // with per-launch timing of the factor kernels the groups run one after
  // another on the factor stream, so that each launch's event interval holds
  // its own kernel only (same launches, no overlap between groups); a graph
  // being captured carries no events and keeps the concurrent form
  const bool serial = (h->tim_on[TK_GEMM] || h->tim_on[TK_PANEL]) && !h->capturing;
  if (G <= 1 || serial) {
    for (int g = 0; g < G; ++g)
      if ((rc = run_schedule(h, h->sch_group[g], 1, 0, 0, TK_GEMM, f))) return rc;
    if (h->tip_nseg > 0) pack_tips(h->sdt, h->p, h->t, h->d_blk, h->d_spikes, h->d_tips, f);
    if ((rc = run_schedule(h, h->sch_rfac, 1, 0, 0, TK_GEMM, f, TK_RFAC))) return rc;
    HIPCHK(hipGetLastError());
    return DDPS_OK;
  }
  hipEvent_t fork = h->capturing ? h->cap_fork : h->fork_ev;
  const std::vector<hipEvent_t>& gev = h->capturing ? h->cap_gevent : h->gevent;
  if (!fork || (int)gev.size() < G - 1) return DDPS_E_STATE;
  HIPCHK(hipEventRecord(fork, f));
  for (int g = 1; g < G; ++g) HIPCHK(hipStreamWaitEvent(h->gstream[g - 1], fork, 0));
  if ((rc = run_schedule(h, h->sch_group[0], 1, 0, 0, TK_GEMM, f))) return rc;
  for (int g = 1; g < G; ++g) {
    if ((rc = run_schedule(h, h->sch_group[g], 1, 0, 0, TK_GEMM, h->gstream[g - 1]))) return rc;
    HIPCHK(hipEventRecord(gev[g - 1], h->gstream[g - 1]));
  }
  for (int g = 1; g < G; ++g) HIPCHK(hipStreamWaitEvent(f, gev[g - 1], 0));
  if (h->tip_nseg > 0) pack_tips(h->sdt, h->p, h->t, h->d_blk, h->d_spikes, h->d_tips, f);
  if ((rc = run_schedule(h, h->sch_rfac, 1, 0, 0, TK_GEMM, f, TK_RFAC))) return rc;
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

// Blocks to groups, longest first (LPT: each block, in decreasing number of
// tile rows, goes to the group with the least work so far); then the
// factor schedules of all groups and the solve schedules, uploaded.
int build_schedules(ddps_ctx* h) {
  const int p = h->p;
  const int G = std::max(1, std::min<int>(h->groups, (int)std::min<int64_t>(p, h->nslots)));
  std::vector<int> order(p);
  for (int i = 0; i < p; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->blk[a].T > h->blk[b].T; });
  std::vector<int64_t> load(G, 0);
  h->group_of.assign(p, 0);
  for (int i : order) {
    int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    h->group_of[i] = g;
    load[g] += h->blk[i].T;
  }
  ScheduleBuilder sb;
  sb.h = h;
  h->mode_cursor = 0;
  h->sch_group.assign(G, {});
  h->wslot.assign(p, 0);
  if (h->ilu) {
    // incomplete factors: no factor schedule (the factor kernels run per
    // batch of ilu_batches), only the solve-phase launches below
  } else if (!h->tips_only) {
    for (int i = 0; i < p; ++i) h->wslot[i] = i;
    for (int g = 0; g < G; ++g) {
      std::vector<int> mem;
      for (int i = 0; i < p; ++i)
        if (h->group_of[i] == g) mem.push_back(i);
      build_factor_schedule(h, sb, mem, h->sch_group[g]);
    }
  } else {
    // Each group owns nslots / G workspace slots and runs its blocks in
    // batches of that many, longest first (a batch's launches last as long
    // as its longest block); a slot's scratch and spike matrix are reused by
    // the next batch of the group, which follows on the group's stream.
    const int64_t per = h->nslots / G;
    if (per < 1) return DDPS_E_ARG;
    const int64_t slot_elems = h->Nmax * 2 * h->t;
    for (int g = 0; g < G; ++g) {
      std::vector<int> mem;
      for (int i : order)
        if (h->group_of[i] == g) mem.push_back(i);
      for (size_t b0 = 0; b0 < mem.size(); b0 += (size_t)per) {
        std::vector<int> batch(mem.begin() + b0, mem.begin() + std::min(mem.size(), b0 + (size_t)per));
        std::sort(batch.begin(), batch.end());
        for (size_t j = 0; j < batch.size(); ++j) {
          const int64_t slot = (int64_t)g * per + (int64_t)j;
          h->wslot[batch[j]] = slot;
          h->blk[batch[j]].goff = slot * slot_elems;
        }
        build_batch_rhs(h, sb, batch, h->sch_group[g]);
        build_factor_schedule(h, sb, batch, h->sch_group[g]);
        build_batch_tips(h, sb, batch, h->sch_group[g]);
      }
    }
    HIPCHK(hipMemcpyAsync(h->d_blk, h->blk.data(), sizeof(BlockInfo) * p, hipMemcpyHostToDevice, h->stream));
  }
  h->sch_fwd.clear();
  h->sch_bwd.clear();
  h->sch_retr.clear();
  build_solve_schedules(h, sb);
  build_reduced_direct(h, sb);
  h->free_ptr(h->d_gemm);
  h->free_ptr(h->d_order);
  h->free_ptr(h->d_panel);
  h->free_ptr(h->d_gemv);
  h->d_gemm = nullptr;
  h->d_order = nullptr;
  h->d_panel = nullptr;
  h->d_gemv = nullptr;
  int rc;
  if ((rc = h->alloc(h->d_gemm, (int64_t)sb.gemm.size())) || (rc = h->alloc(h->d_order, (int64_t)sb.order.size())) ||
      (rc = h->alloc(h->d_panel, (int64_t)sb.panel.size())) ||
      (rc = h->alloc(h->d_gemv, (int64_t)sb.gemv.size())))
    return rc;
  hipStream_t s = h->stream;
  if (!sb.gemm.empty())
    HIPCHK(hipMemcpyAsync(h->d_gemm, sb.gemm.data(), sizeof(GemmProb) * sb.gemm.size(), hipMemcpyHostToDevice, s));
  if (!sb.order.empty())
    HIPCHK(hipMemcpyAsync(h->d_order, sb.order.data(), sizeof(int32_t) * sb.order.size(), hipMemcpyHostToDevice, s));
  if (!sb.panel.empty())
    HIPCHK(hipMemcpyAsync(h->d_panel, sb.panel.data(), sizeof(PanelProb) * sb.panel.size(), hipMemcpyHostToDevice, s));
  if (!sb.gemv.empty())
    HIPCHK(hipMemcpyAsync(h->d_gemv, sb.gemv.data(), sizeof(GemvProb) * sb.gemv.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  // streams and events of the groups
  while ((int)h->gstream.size() < G - 1) {
    hipStream_t gs;
    hipEvent_t ge;
    HIPCHK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ge, hipEventDisableTiming));
    h->gstream.push_back(gs);
    h->gevent.push_back(ge);
  }
  h->drop_graph();
  if ((int64_t)h->W1 * h->R * 2 > h->part_cap) return DDPS_E_ARG;
  return DDPS_OK;
}

// Step 6.1 on the padded vector d_ypad, in place (R columns): the tile
// sweeps of the exact factors, or the level-scheduled triangular solves of
// the incomplete ones.
int block_solves(ddps_ctx* h, int tk) {
  const int R = h->R;
  if (!h->ilu) {
    int rc = run_schedule(h, h->sch_fwd, R, h->Np, h->Np, tk);
    if (rc) return rc;
    return run_schedule(h, h->sch_bwd, R, h->Np, h->Np, tk);
  }
  hipEvent_t a;
  h->tim_begin(tk, a);
  ilu_solve(h->p, h->d_iblk, h->d_lrows, h->d_lptr, h->d_lq, h->d_urows, h->d_uptr, h->d_uq, h->d_col, h->d_fv,
            h->d_ypad, h->Np, R, h->d_vpad, h->stream);
  // both triangles once (values and column indices), each vector entry read and written per sweep
  h->tim_end(tk, a, 2.0 * (double)h->ilu_nnz * R, 12.0 * (double)h->ilu_nnz + 32.0 * (double)h->n * R);
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

// Inner BiCGStab on G^ z^ = g^ for R columns (k used).  z^ in d_zh.
int inner_solve(ddps_ctx* h, int k, int use_guess, double tol, int maxit, std::vector<int>& iters,
                std::vector<int>& status_out) {
  const int R = h->R;
  const int64_t m = h->m;
  hipStream_t s = h->stream;
  iters.assign(k, 0);
  status_out.assign(k, KS_CONVERGED);
  if (m == 0) {
    return DDPS_OK;
  }
  if (!h->sch_rsol.empty()) {
    // direct: block LU substitutions over the interfaces (no iterations)
    HIPCHK(hipMemcpyAsync(h->d_zh, h->d_gh, sizeof(double) * m * R, hipMemcpyDeviceToDevice, s));
    int rc = run_schedule(h, h->sch_rsol, R, m, m, TK_RSPMV);
    if (rc) return rc;
    vec_apply_mask(m, R, h->d_mask, h->d_zh, s);
    HIPCHK(hipGetLastError());
    return DDPS_OK;
  }
  const int W2 = vec_grid(m);
  const bool prec = h->opt.inner_prec == 1;
  double* S0 = h->d_sums;
  double* S1 = S0 + 2 * kMaxRhs;
  double* S2 = S1 + 2 * kMaxRhs;
  double* S3 = S2 + 2 * kMaxRhs;
  double* S4 = S3 + 2 * kMaxRhs;
  if (use_guess) {
    HIPCHK(hipMemcpyAsync(h->d_zh, h->d_guess, sizeof(double) * m * R, hipMemcpyDeviceToDevice, s));
    run_launch(h, h->l_zv, R, m, m, nullptr, nullptr, nullptr, TK_RSPMV);
  }
  bicg_init(R, m, use_guess, h->d_gh, h->d_zh, h->d_v, h->d_r, h->d_rt, h->d_p, h->d_part_buf, W2, s);
  reduce2(R, W2, h->d_part_buf, S0, nullptr, s);
  bicg_init_state(R, k, tol, S0, h->d_state, s);
  std::vector<int> restarts(k, 0);
  int it = 1;
  const int batch = 4;
  bool done = false;
  std::vector<int32_t> flags(kMaxRhs, 0);
  while (!done) {
    int last = std::min(maxit, it + batch - 1);
    for (; it <= last; ++it) {
      const int32_t* stop = &h->d_state->status[it & 1][0];
      // right preconditioning: v = G^ M^{-1} p, t = G^ M^{-1} s, x += a M^{-1} p + w M^{-1} s
      if (prec) run_launch(h, h->l_lp, R, m, m, nullptr, nullptr, stop, TK_RSPMV);
      run_launch(h, prec ? h->l_pvh : h->l_pv, R, m, m, h->d_rt, h->d_part_buf, stop, TK_RSPMV);
      reduce2(R, h->W1, h->d_part_buf, S1, stop, s, h->d_red1);
      bicg_s(R, it, m, S1, h->d_state, h->d_r, h->d_v, h->d_s, h->d_part_buf, W2, s);
      reduce2(R, W2, h->d_part_buf, S2, stop, s, h->d_red1);
      if (prec) run_launch(h, h->l_ls, R, m, m, nullptr, nullptr, stop, TK_RSPMV);
      run_launch(h, prec ? h->l_sth : h->l_st, R, m, m, h->d_s, h->d_part_buf, stop, TK_RSPMV);
      reduce2(R, h->W1, h->d_part_buf, S3, stop, s, h->d_red1);
      bicg_xr(R, it, m, tol, S1, S2, S3, h->d_state, h->d_zh, h->d_p, h->d_s, h->d_tv, h->d_r, h->d_rt,
              h->d_part_buf, W2, s, prec ? h->d_mp : nullptr, prec ? h->d_ms : nullptr);
      reduce2(R, W2, h->d_part_buf, S4, stop, s, h->d_red1);
      bicg_p(R, it, maxit, m, tol, S1, S2, S3, S4, h->d_state, h->d_r, h->d_p, h->d_v, W2, s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->h_state, h->d_state, sizeof(KState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // status of the next iteration (slot `it & 1`, it already advanced)
    const int32_t* stt = h->h_state->status[it & 1];
    bool any_running = false, any_restart = false;
    std::fill(flags.begin(), flags.end(), 0);
    for (int j = 0; j < k; ++j) {
      if (stt[j] == KS_RUNNING) any_running = true;
      if (stt[j] == KS_BREAKDOWN && restarts[j] == 0 && it <= maxit) {
        flags[j] = 1;
        restarts[j] = 1;
        any_restart = true;
      }
    }
    if (any_restart) {
      HIPCHK(hipMemcpyAsync(h->d_flag, flags.data(), sizeof(int32_t) * kMaxRhs, hipMemcpyHostToDevice, s));
      bicg_restart(R, it - 1, m, h->d_flag, h->d_r, h->d_rt, h->d_p, h->d_part_buf, W2, S0, h->d_state, s);
      any_running = true;
    }
    if (!any_running || it > maxit) done = true;
  }
  HIPCHK(hipMemcpyAsync(h->h_state, h->d_state, sizeof(KState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    iters[j] = h->h_state->iters2[j];
    status_out[j] = h->h_state->status[it & 1][j];
  }
  return DDPS_OK;
}

int dots(ddps_ctx* h, int64_t len, const double* a0, const double* b0, const double* a1, const double* b1,
         std::vector<double>& d0, std::vector<double>& d1);

// Learned starting vector of the reduced solve of one application (a network
// attached with ddps_set_guess_model).  Three candidates per column, judged
// by the reduced residual ||g^ - G^ z0||_2 on c: z0 = 0; z0 = g^ (G^ = I +
// G(c,c), so g^ is the zero-order approximation of z^); and the network's
// correction of g^, z0 = g^ + s_j net([r_j/s_j, g^_j/q_j, 0, 0]) per
// interface j, r = g^ - G^ g^ the residual of g^.  The smallest residual wins
// and is left in d_guess.  Two reduced products, one network pass and one
// host synchronisation.
int learned_start(ddps_ctx* h, int k) {
  const int R = h->R;
  const int64_t m = h->m;
  hipStream_t s = h->stream;
  const int nif = h->p - 1;
  Coef3 cf{};
  for (int j = 0; j < R; ++j) {
    cf.a[j] = 1.0;
    cf.b[j] = -1.0;
  }
  // residual of the zero-order candidate g^
  HIPCHK(hipMemcpyAsync(h->d_zh, h->d_gh, sizeof(double) * m * R, hipMemcpyDeviceToDevice, s));
  run_launch(h, h->l_zv, R, m, m, nullptr, nullptr, nullptr, TK_RSPMV);
  lincomb(R, m, cf, h->d_gh, h->d_v, nullptr, h->d_r, s);
  vec_apply_mask(m, R, h->d_mask, h->d_r, s);
  // the network's candidate
  guess_features(nif, k, 2 * h->t, h->gnet_din, h->d_r, h->d_gh, h->d_mask, 0.0, 0.0, h->d_gX, h->d_gS, s);
  int rc = ddps_mlp_forward(h->gnet, k * nif, h->d_gX, h->d_gY);
  if (rc) return rc;
  guess_compose(m * k, m, 2 * h->t, h->d_gh, h->d_gY, h->d_gS, h->d_mask, h->d_guess, s);
  HIPCHK(hipMemcpyAsync(h->d_zh, h->d_guess, sizeof(double) * m * k, hipMemcpyDeviceToDevice, s));
  run_launch(h, h->l_zv, R, m, m, nullptr, nullptr, nullptr, TK_RSPMV);
  lincomb(R, m, cf, h->d_gh, h->d_v, nullptr, h->d_rt, s);
  vec_apply_mask(m, R, h->d_mask, h->d_rt, s);
  std::vector<double> nb, nl, ng, unused;
  if ((rc = dots(h, m, h->d_r, h->d_r, h->d_rt, h->d_rt, nb, nl))) return rc;
  if ((rc = dots(h, m, h->d_gh, h->d_gh, nullptr, nullptr, ng, unused))) return rc;
  h->garm.assign(k, -1);
  for (int j = 0; j < k; ++j) {
    double* col = h->d_guess + (int64_t)j * m;
    if (!h->gtrial_done) {
      // trial: every other reduced solve leaves the network out
      h->garm[j] = (int)(h->gtrial_seq++ & 1);
      if (h->garm[j] == 0) nl[j] = std::numeric_limits<double>::infinity();
    }
    if (ng[j] <= nb[j] && ng[j] <= nl[j]) {
      fill_f64(col, m, 0.0, s);
      ++h->guess_counts[0];
    } else if (nb[j] <= nl[j]) {
      HIPCHK(hipMemcpyAsync(col, h->d_gh + (int64_t)j * m, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
      ++h->guess_counts[1];
    } else {
      ++h->guess_counts[2];
    }
    if (h->gtrial_done || h->garm[j] == 1)
      h->gnet_losses = (nl[j] < ng[j] && nl[j] < nb[j]) ? 0 : h->gnet_losses + 1;
  }
  if (k < R) fill_f64(h->d_guess + (int64_t)k * m, m * (R - k), 0.0, s);
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

// A network is retired (no candidates tried) once its candidate has lost
// kRetire reduced solves in a row, or lost the trial against its absence.
constexpr int kRetire = 8;

// z = P^{-1} y (k columns, device, leading dims ldy/ldz).  Reduced vectors
// are left in d_gh / d_zh.
int prec_apply(ddps_ctx* h, int k, const double* y, int64_t ldy, double* z, int64_t ldz, double inner_tol,
               int use_guess, std::vector<int>& iters, int* breakdown) {
  const int R = h->R;
  hipStream_t s = h->stream;
  vec_to_padded(h->Np, R, k, h->p, h->d_blk, y, ldy, h->d_ypad, s);
  int rc = block_solves(h, TK_SWEEP);
  if (rc) return rc;
  vec_gather_reduced(h->m, R, h->d_rrow, h->d_mask, h->d_ypad, h->Np, h->d_gh, s);
  if (h->gnet && h->m > 0 && h->sch_rsol.empty()) {
    // the network is retired (no candidates tried; the zero start of the
    // method) once it has lost kRetire reduced solves in a row, until a
    // network is attached again
    if (h->gnet_losses < kRetire) {
      if ((rc = learned_start(h, k))) return rc;
      use_guess = 1;
    } else {
      h->gnet_skipped += k;
    }
  }
  const bool trial = h->gnet && !h->gtrial_done && (int)h->garm.size() == k && use_guess;
  std::vector<int> st;
  rc = inner_solve(h, k, use_guess, inner_tol, h->opt.inner_maxit, iters, st);
  if (rc) return rc;
  if (trial) {
    // the network stays only if its solves take at least half an iteration
    // fewer on average than the solves without it (its candidate costs two
    // reduced products per application); otherwise it is retired
    constexpr int kTrial = 8;
    for (int j = 0; j < k; ++j) {
      const int a = h->garm[j];
      if (a < 0) continue;
      h->gtrial_n[a] += 1;
      h->gtrial_its[a] += iters[j];
    }
    h->garm.clear();
    if (h->gtrial_n[0] >= kTrial && h->gtrial_n[1] >= kTrial) {
      h->gtrial_done = true;
      // mean counts in half iterations (the inner solve's unit)
      const double m0 = (double)h->gtrial_its[0] / (double)h->gtrial_n[0];
      const double m1 = (double)h->gtrial_its[1] / (double)h->gtrial_n[1];
      if (!(m1 <= m0 - 1.0)) h->gnet_losses = kRetire;
    }
  }
  if (breakdown) {
    *breakdown = 0;
    for (int j = 0; j < k; ++j)
      if (st[j] == KS_BREAKDOWN) *breakdown = 1;
  }
  if (h->opt.retrieval == 1 && h->m > 0) {
    // 6.5 re-solved: z = D~^{-1}(y - R~ z^), the block sweeps once more
    coupling_rhs(h->Np, R, k, h->p, h->t, h->d_blk, h->d_rowptr, h->d_col, h->d_val, y, ldy, h->d_zh, h->m,
                 h->d_mask, h->d_ypad, s);
    rc = block_solves(h, TK_RETR);
    if (rc) return rc;
    vec_from_padded(h->Np, k, h->p, h->d_blk, h->d_ypad, z, ldz, s);
  } else {
    rc = run_schedule(h, h->sch_retr, R, h->m, h->Np, TK_RETR);
    if (rc) return rc;
    vec_from_padded(h->Np, k, h->p, h->d_blk, h->d_vpad, z, ldz, s);
  }
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

int resid(ddps_ctx* h, const double* x, double* r, std::vector<double>& rinf, std::vector<double>& r2,
          std::vector<double>& finf, std::vector<double>& f2) {
  const int R = h->R;
  const int W = vec_grid(h->n);
  hipEvent_t a;
  h->tim_begin(TK_CSR, a);
  csr_resid(R, h->n, h->d_rowptr, h->d_col, h->d_val, x, h->n, h->d_fo, h->n, r, h->n, h->d_part_buf, W,
            h->d_out, h->stream);
  h->tim_end(TK_CSR, a, 2.0 * h->nnz * R, 12.0 * h->nnz + 8.0 * h->n * (R * 3 + 2));
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->h_out, h->d_out, sizeof(double) * 4 * R, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  rinf.resize(R); r2.resize(R); finf.resize(R); f2.resize(R);
  for (int j = 0; j < R; ++j) {
    rinf[j] = h->h_out[4 * j];
    r2[j] = std::sqrt(h->h_out[4 * j + 1]);
    finf[j] = h->h_out[4 * j + 2];
    f2[j] = std::sqrt(h->h_out[4 * j + 3]);
  }
  return DDPS_OK;
}

// out = A x
int matvec(ddps_ctx* h, const double* x, double* out) {
  const int R = h->R;
  const int W = vec_grid(h->n);
  hipEvent_t a;
  h->tim_begin(TK_CSR, a);
  csr_resid(R, h->n, h->d_rowptr, h->d_col, h->d_val, x, h->n, nullptr, h->n, out, h->n, h->d_part_buf, W,
            h->d_out, h->stream);
  h->tim_end(TK_CSR, a, 2.0 * h->nnz * R, 12.0 * h->nnz + 8.0 * h->n * (R * 2 + 1));
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

int dots(ddps_ctx* h, int64_t len, const double* a0, const double* b0, const double* a1, const double* b1,
         std::vector<double>& d0, std::vector<double>& d1) {
  const int R = h->R;
  const int W = vec_grid(len);
  dot2(R, len, a0, b0, a1, b1, h->d_part_buf, W, h->d_out, h->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->h_out, h->d_out, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  d0.resize(R); d1.resize(R);
  for (int j = 0; j < R; ++j) {
    d0[j] = h->h_out[2 * j];
    d1[j] = h->h_out[2 * j + 1];
  }
  return DDPS_OK;
}

// max |v| (two = false) or ||v||_2 (two = true) per column (host)
int norm_of(ddps_ctx* h, const double* v, bool two, std::vector<double>& out) {
  const int R = h->R;
  const int W = vec_grid(h->n);
  csr_resid(R, h->n, nullptr, nullptr, nullptr, nullptr, h->n, v, h->n, nullptr, h->n, h->d_part_buf, W,
            h->d_out, h->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->h_out, h->d_out, sizeof(double) * 4 * R, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out.resize(R);
  for (int j = 0; j < R; ++j) out[j] = two ? std::sqrt(h->h_out[4 * j + 1]) : h->h_out[4 * j];
  return DDPS_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

void ddps_default_options(ddps_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(ddps_options);
  o->drop_delta = 0.0;
  o->factor_dtype = DDPS_F64;
  o->inner_tol = 1e-12;
  o->inner_maxit = 1000;
  o->outer_maxit = 1000;
  o->outer_method = 1;
  o->guess = 0;
  o->use_x0 = 0;
  o->max_rhs = 1;
  o->mem_budget = 0;
  o->stream = nullptr;
  o->factor_streams = 0;
  o->factor_graph = 0;
  o->inner_prec = 0;
  o->retrieval = 0;
  o->norm = 0;
  o->work_slots = 0;
  o->reduced_solve = 0;
  o->loosen_ratio = 0.0;
  o->gemv_sums = 0;
  o->block_factor = 0;
}

const char* ddps_last_hip_error(void) {
  hipError_t e = last_hip_error();
  if (e == hipSuccess) e = hipGetLastError();
  last_hip_error() = hipSuccess;
  return hipGetErrorString(e);
}

const char* ddps_status_string(int s) {
  switch (s) {
    case DDPS_OK: return "DDPS_OK";
    case DDPS_E_ARG: return "DDPS_E_ARG: invalid argument or unsupported matrix structure";
    case DDPS_E_NOMEM: return "DDPS_E_NOMEM: the plan does not fit the memory budget (F1)";
    case DDPS_E_NOCONV: return "DDPS_E_NOCONV: tolerance not met (F2)";
    case DDPS_E_SINGULAR: return "DDPS_E_SINGULAR: zero pivot in a diagonal-block LU";
    case DDPS_E_BREAKDOWN: return "DDPS_E_BREAKDOWN: BiCGStab breakdown";
    case DDPS_E_STATE: return "DDPS_E_STATE: call out of order";
    case DDPS_E_HIP: return "DDPS_E_HIP: HIP runtime error";
    default: return "unknown ddps status";
  }
}

void ddps_destroy(ddps_handle h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (int k = 0; k < TK_N; ++k)
    for (auto& r : h->tim[k]) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  h->drop_graph();
  if (h->fstream) (void)hipStreamSynchronize(h->fstream);
  for (auto gs : h->gstream) {
    (void)hipStreamSynchronize(gs);
    (void)hipStreamDestroy(gs);
  }
  for (auto ge : h->gevent) (void)hipEventDestroy(ge);
  if (h->fstream) (void)hipStreamDestroy(h->fstream);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  for (void* q : h->allocs) (void)hipFree(q);
  if (h->h_state) (void)hipHostFree(h->h_state);
  if (h->h_out) (void)hipHostFree(h->h_out);
  delete h;
}

extern "C++" {  // internal helpers: C++ linkage
namespace {

// Host plan of the incomplete-factor form: per row the CSR positions of its
// in-block lower part, pivot and end; each block's rows grouped into forward
// levels (level of r = 1 + the largest level among its lower-pattern rows)
// and backward levels (the same over the upper pattern); the block records.
struct IluPlan {
  std::vector<int64_t> lo, dg, hi, lptr, uptr;
  std::vector<int32_t> lrows, urows;
  std::vector<IluBlock> blk;
};

int ilu_plan(ddps_ctx* h, IluPlan& P) {
  const int64_t n = h->n, nnz = h->nnz;
  const int p = h->p;
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> cl(nnz);
  if (hipMemcpyAsync(rp.data(), h->d_rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, h->stream) !=
          hipSuccess ||
      hipMemcpyAsync(cl.data(), h->d_col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return DDPS_E_HIP;
  P.lo.assign(n, 0);
  P.dg.assign(n, -1);
  P.hi.assign(n, 0);
  P.lrows.assign(n, 0);
  P.urows.assign(n, 0);
  P.lptr.clear();
  P.uptr.clear();
  P.blk.assign(p, IluBlock{});
  std::vector<int64_t> lev(n, 0), cnt;
  h->ilu_nmax = 0;
  h->ilu_nnz = 0;
  h->ilu_levels = 0;
  for (int i = 0; i < p; ++i) {
    const BlockInfo& B = h->blk[i];
    const int64_t s0 = B.s, s1 = B.s + B.n;
    for (int64_t r = s0; r < s1; ++r) {
      int64_t q = rp[r];
      const int64_t e = rp[r + 1];
      for (int64_t u = q + 1; u < e; ++u)
        if (cl[u] <= cl[u - 1]) return DDPS_E_ARG;   // columns must be sorted, no repeats
      while (q < e && cl[q] < s0) ++q;
      P.lo[r] = q;
      while (q < e && cl[q] < s1) {
        if (cl[q] == r) P.dg[r] = q;
        ++q;
      }
      P.hi[r] = q;
      if (P.dg[r] < 0) return DDPS_E_ARG;   // no stored diagonal: a structurally zero pivot
      h->ilu_nnz += P.hi[r] - P.lo[r];
    }
    h->ilu_nmax = std::max<int64_t>(h->ilu_nmax, B.n);
    // levels over one triangle, rows visited in dependency order, then
    // bucketed by level (a counting sort keeps the row order within a level)
    auto levels = [&](bool fwd, std::vector<int32_t>& rows, std::vector<int64_t>& ptr, int64_t& beg,
                      int64_t& num) {
      int64_t top = 0;
      for (int64_t k = 0; k < B.n; ++k) {
        const int64_t r = fwd ? s0 + k : s1 - 1 - k;
        int64_t lv = 0;
        const int64_t a = fwd ? P.lo[r] : P.dg[r] + 1, e = fwd ? P.dg[r] : P.hi[r];
        for (int64_t q = a; q < e; ++q) lv = std::max(lv, lev[cl[q]] + 1);
        lev[r] = lv;
        top = std::max(top, lv + 1);
      }
      cnt.assign(top + 1, 0);
      for (int64_t r = s0; r < s1; ++r) ++cnt[lev[r] + 1];
      for (int64_t l = 0; l < top; ++l) cnt[l + 1] += cnt[l];
      beg = (int64_t)ptr.size();
      num = top;
      for (int64_t l = 0; l <= top; ++l) ptr.push_back(s0 + cnt[l]);
      for (int64_t k = 0; k < B.n; ++k) {
        const int64_t r = fwd ? s0 + k : s1 - 1 - k;
        rows[s0 + cnt[lev[r]]++] = (int32_t)r;
      }
    };
    IluBlock& I = P.blk[i];
    I.s = s0;
    I.n = B.n;
    I.vbase = B.voff + B.pad;
    I.left = i > 0;
    I.right = i < p - 1;
    levels(true, P.lrows, P.lptr, I.lbeg, I.lnum);
    levels(false, P.urows, P.uptr, I.ubeg, I.unum);
    h->ilu_levels = std::max<int64_t>(h->ilu_levels, I.lnum + I.unum);
  }
  return DDPS_OK;
}

size_t ilu_plan_bytes(const ddps_ctx* h, const IluPlan& P) {
  return (size_t)h->nnz * 8 + (size_t)h->n * (3 * 8 + 2 * 4 + 2 * 16) + (P.lptr.size() + P.uptr.size()) * 8 +
         (size_t)h->p * (sizeof(IluBlock) + 4);
}

int ilu_upload(ddps_ctx* h, const IluPlan& P) {
  int rc;
  const int64_t n = h->n, p = h->p;
  if ((rc = h->alloc(h->d_fv, h->nnz)) || (rc = h->alloc(h->d_ilo, n)) || (rc = h->alloc(h->d_idg, n)) ||
      (rc = h->alloc(h->d_ihi, n)) || (rc = h->alloc(h->d_lrows, n)) || (rc = h->alloc(h->d_urows, n)) ||
      (rc = h->alloc(h->d_lptr, (int64_t)P.lptr.size())) || (rc = h->alloc(h->d_uptr, (int64_t)P.uptr.size())) ||
      (rc = h->alloc(h->d_iblk, p)) || (rc = h->alloc(h->d_ibatch, p)) || (rc = h->alloc(h->d_lq, 2 * n)) ||
      (rc = h->alloc(h->d_uq, 2 * n)))
    return rc;
  {
    std::vector<int64_t> q(2 * n);
    for (int64_t j = 0; j < n; ++j) {
      q[2 * j] = P.lo[P.lrows[j]];
      q[2 * j + 1] = P.dg[P.lrows[j]];
    }
    HIPCHK(hipMemcpy(h->d_lq, q.data(), sizeof(int64_t) * 2 * n, hipMemcpyHostToDevice));
    for (int64_t j = 0; j < n; ++j) {
      q[2 * j] = P.dg[P.urows[j]] + 1;
      q[2 * j + 1] = P.hi[P.urows[j]];
    }
    HIPCHK(hipMemcpy(h->d_uq, q.data(), sizeof(int64_t) * 2 * n, hipMemcpyHostToDevice));
  }
  std::vector<int32_t> order(p);
  for (int i = 0; i < p; ++i) order[i] = i;
  hipStream_t s = h->stream;
  HIPCHK(hipMemcpyAsync(h->d_ilo, P.lo.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_idg, P.dg.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_ihi, P.hi.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_lrows, P.lrows.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_urows, P.urows.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_lptr, P.lptr.data(), sizeof(int64_t) * P.lptr.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_uptr, P.uptr.data(), sizeof(int64_t) * P.uptr.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_iblk, P.blk.data(), sizeof(IluBlock) * p, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_ibatch, order.data(), sizeof(int32_t) * p, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  h->ilu_batches.clear();
  const int64_t per = std::max<int64_t>(1, h->nslots);
  for (int64_t b0 = 0; b0 < p; b0 += per) h->ilu_batches.push_back({(int)b0, (int)std::min<int64_t>(per, p - b0)});
  return DDPS_OK;
}

}  // namespace
}  // extern "C++"

int ddps_setup(ddps_handle* out, int64_t n, int32_t p, const int64_t* part_ptr, const int64_t* row_ptr,
               const int32_t* col, const double* val, int64_t nnz, const ddps_options* opt) {
  if (!out) return DDPS_E_ARG;
  *out = nullptr;
  if (n <= 0 || p <= 0 || !part_ptr || !row_ptr || !col || !val || nnz <= 0) return DDPS_E_ARG;
  if (nnz > (int64_t)std::numeric_limits<int64_t>::max() / 16) return DDPS_E_ARG;
  if (part_ptr[0] != 0 || part_ptr[p] != n) return DDPS_E_ARG;
  for (int i = 0; i < p; ++i)
    if (part_ptr[i + 1] <= part_ptr[i]) return DDPS_E_ARG;
  ddps_ctx* h = new (std::nothrow) ddps_ctx();
  if (!h) return DDPS_E_NOMEM;
  ddps_default_options(&h->opt);
  if (opt) {
    if (opt->struct_size != (int32_t)sizeof(ddps_options)) {
      delete h;
      return DDPS_E_ARG;
    }
    h->opt = *opt;
  }
  const ddps_options& o = h->opt;
  if (!(o.drop_delta >= 0.0 && o.drop_delta <= 1.0) || fac_dtype_code(o.factor_dtype) < 0 || o.inner_maxit < 1 ||
      o.outer_maxit < 1 || o.max_rhs < 1 || o.max_rhs > kMaxRhs || !(o.inner_tol > 0.0) || o.inner_prec < 0 ||
      o.inner_prec > 1 || o.retrieval < 0 || o.retrieval > 1 || (o.norm != 0 && o.norm != 2) || o.work_slots < 0 ||
      o.reduced_solve < 0 || o.reduced_solve > 1 || std::isnan(o.loosen_ratio) || o.gemv_sums < 0 ||
      o.gemv_sums > 1 || o.block_factor < 0 || o.block_factor > 1 ||
      (o.block_factor == 1 && p > 1 && o.retrieval != 1)) {
    delete h;
    return DDPS_E_ARG;
  }
  auto fail = [&](int rc) {
    ddps_destroy(h);
    return rc;
  };
  h->stream = (hipStream_t)o.stream;
  h->n = n;
  h->nnz = nnz;
  h->p = p;
  h->part.assign(part_ptr, part_ptr + p + 1);
  h->gdt = fac_dtype_code(o.factor_dtype);
  h->sdt = h->gdt == 0 ? 0 : 1;
  h->elt = h->sdt == 0 ? 8 : 4;
  h->R = rhs_alloc(o.max_rhs);
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) return fail(DDPS_E_HIP);
  if (hipHostMalloc((void**)&h->h_state, sizeof(KState)) != hipSuccess) return fail(DDPS_E_HIP);
  if (hipHostMalloc((void**)&h->h_out, sizeof(double) * 4 * kMaxRhs) != hipSuccess) return fail(DDPS_E_HIP);
  (void)hipEventRecord(h->ev0, h->stream);

  // copy the CSR and scan it
  int rc;
  if ((rc = h->alloc(h->d_part, p + 1)) || (rc = h->alloc(h->d_rowptr, n + 1)) || (rc = h->alloc(h->d_col, nnz)) ||
      (rc = h->alloc(h->d_val, nnz)) || (rc = h->alloc(h->d_band, 1)) || (rc = h->alloc(h->d_flags, 1)) ||
      (rc = h->alloc(h->d_bad, 1)))
    return fail(rc);
  hipStream_t s = h->stream;
  if (hipMemcpyAsync(h->d_part, part_ptr, sizeof(int64_t) * (p + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->d_rowptr, row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->d_col, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->d_val, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(DDPS_E_HIP);
  fill_u64(h->d_band, 1, 0ull, s);
  {
    unsigned int* f = h->d_flags;
    fill_f32((float*)f, 1, 0.f, s);
  }
  setup_scan(n, p, h->d_part, h->d_rowptr, h->d_col, h->d_val, nnz, h->d_band, h->d_flags, s);
  unsigned long long band = 0;
  unsigned int flags = 0;
  if (hipMemcpyAsync(&band, h->d_band, sizeof(band), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&flags, h->d_flags, sizeof(flags), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(DDPS_E_HIP);
  if (flags) return fail(DDPS_E_ARG);
  h->b = (int32_t)std::max<unsigned long long>(band, 1ull);
  h->t = ((h->b + 63) / 64) * 64;
  const int t = h->t;
  // layout
  h->blk.resize(p);
  int64_t tiles = 0, goff = 0, voff = 0;
  h->Tmax = 0;
  h->Nmax = 0;
  const int64_t tt = (int64_t)t * t;
  for (int i = 0; i < p; ++i) {
    BlockInfo& B = h->blk[i];
    B.s = part_ptr[i];
    B.n = part_ptr[i + 1] - part_ptr[i];
    if (p > 1 && B.n < 2 * (int64_t)t) return fail(DDPS_E_ARG);
    B.T = (B.n + t - 1) / t;
    B.N = B.T * t;
    B.pad = B.N - B.n;
    if (B.N > std::numeric_limits<int32_t>::max()) return fail(DDPS_E_ARG);
    B.tiles = tiles;
    tiles += B.T * tt + (B.T - 1) * h->pair_elems();
    B.goff = goff;
    goff += p > 1 ? B.N * 2 * t : 0;
    B.voff = voff;
    voff += B.N;
    h->Tmax = std::max<int>(h->Tmax, (int)B.T);
    h->Nmax = std::max<int64_t>(h->Nmax, B.N);
  }
  h->ilu = o.block_factor == 1;
  h->tile_elems = h->ilu ? 0 : tiles;
  h->tips_only = o.retrieval == 1 && p > 1;
  h->Np = voff;
  h->m = p > 1 ? (int64_t)2 * t * (p - 1) : 0;
  h->scr_per_block = h->ilu ? 0 : ddps_ctx::scratch_elems(t);
  IluPlan iplan;
  if (h->ilu && (rc = ilu_plan(h, iplan))) return fail(rc);
  h->groups = o.factor_streams > 0 ? o.factor_streams : default_groups(h);
  // memory plan (F1 check before the large allocations)
  const int R = h->R;
  const int64_t m = h->m;
  const int64_t Wmax = std::max<int64_t>({(int64_t)kVecGrid, (int64_t)p * 2 * t / 64 + 1, 1});
  size_t need = 0;
  need += (size_t)h->tile_elems * h->elt;
  // packed tips (2(p-1) parts of t x 2t = m x 2t) for one or two right-hand
  // sides, or the column-major tips that are all the tips-only form keeps,
  // and that form's compact store of the coupling entries
  h->tip_nseg = (R <= 2 && p > 1 && !h->tips_only) ? tipmv_segments(h->sdt, t) : 0;
  if (h->tip_nseg > 0 || h->tips_only) need += (size_t)m * 2 * t * h->elt;
  if (h->tips_only) need += (size_t)p * h->pair_elems() * h->elt;
  const bool direct = o.reduced_solve == 1 && p > 1;
  const size_t rw_elems = 5 * (size_t)t * t + 2 * (size_t)t * (t / 2 + 64);
  if (direct) need += (2 * (size_t)(p - 1) * t * t + rw_elems) * h->elt;
  need += (size_t)p * 2 * t * 8 + (size_t)m * (8 + 8 + 8);
  need += (size_t)h->Np * R * 8 * 2 + (size_t)h->Np * 8;
  need += (size_t)m * R * 8 * 11;
  need += (size_t)n * R * 8 * 10;
  need += (size_t)Wmax * R * 4 * 8;
  if (h->ilu) need += ilu_plan_bytes(h, iplan);
  size_t budget = o.mem_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(DDPS_E_HIP);
    budget = fr > ((size_t)1 << 30) ? fr - ((size_t)1 << 30) : fr;
  }
  // workspace: a scratch area per block, and the whole spike array; with the
  // tips only, `nslots` slots of scratch + an Nmax x 2t spike matrix, as many
  // as the budget allows (at most p, or opt.work_slots)
  // (incomplete factors: a slot is one block's n x 2t spike workspace)
  const size_t slot_bytes = h->ilu ? (size_t)h->ilu_nmax * 2 * t * h->elt
                                   : (size_t)(h->scr_per_block + (p > 1 ? h->Nmax * 2 * t : 0)) * h->elt;
  if (!h->tips_only) {
    h->nslots = p;
    h->nspike = goff;
    need += (size_t)h->nspike * h->elt + (size_t)p * h->scr_per_block * h->elt;
    if (need > budget) return fail(DDPS_E_NOMEM);
  } else {
    if (need >= budget) return fail(DDPS_E_NOMEM);
    int64_t fit = (int64_t)((budget - need) / slot_bytes);
    // above 32 slots, a multiple of 32: the launch sequence (and so the
    // autotuner's cache key) then does not move with a few GB of free memory
    if (fit > 32) fit -= fit % 32;
    fit = std::min<int64_t>(fit, p);
    if (o.work_slots > 0) fit = std::min<int64_t>(fit, o.work_slots);
    if (fit < 1) return fail(DDPS_E_NOMEM);
    h->nslots = fit;
    h->groups = (int)std::min<int64_t>(h->groups, fit);
    h->nspike = h->ilu ? 0 : fit * h->Nmax * 2 * t;
    need += (size_t)fit * slot_bytes;
  }
  if (h->ilu && !h->tips_only) h->nspike = 0;
  int64_t nlu = 0;
  h->lu_off.assign(p, 0);
  for (int i = 0; i < p; ++i) {
    h->lu_off[i] = nlu;
    nlu += (h->blk[i].T - 1) * h->pair_elems();
  }
  const size_t lu_bytes = (size_t)nlu * h->elt;
  const bool sep_lu = !h->ilu && nlu > 0 && need + lu_bytes <= budget;
  void* vp;
  if (sep_lu) {
    if ((rc = h->alloc_raw(vp, lu_bytes))) return fail(rc);
    h->d_lu = vp;
  }
  if ((rc = h->alloc_raw(vp, (size_t)h->tile_elems * h->elt))) return fail(rc);
  h->d_tiles = vp;
  if ((rc = h->alloc_raw(vp, (size_t)std::max<int64_t>(h->nspike, 1) * h->elt))) return fail(rc);
  h->d_spikes = vp;
  h->spikes_zeroed = false;
  if (h->tip_nseg > 0) {
    if ((rc = h->alloc_raw(vp, (size_t)h->m * 2 * t * h->elt))) return fail(rc);
    h->d_tips = vp;
  }
  if (h->ilu) {
    if (h->tips_only) {
      if ((rc = h->alloc_raw(vp, (size_t)h->nslots * h->ilu_nmax * 2 * t * h->elt))) return fail(rc);
      h->d_iws = vp;
    }
    if ((rc = ilu_upload(h, iplan))) return fail(rc);
    iplan = IluPlan();
  }
  if (h->tips_only) {
    if ((rc = h->alloc_raw(vp, (size_t)h->m * 2 * t * h->elt))) return fail(rc);
    h->d_tipcm = vp;
    if ((rc = h->alloc_raw(vp, (size_t)p * h->pair_elems() * h->elt))) return fail(rc);
    h->d_rhs = vp;
  }
  if ((rc = h->alloc_raw(vp, (size_t)h->nslots * h->scr_per_block * h->elt))) return fail(rc);
  h->d_scratch = vp;
  if (direct) {
    if ((rc = h->alloc_raw(vp, (size_t)(p - 1) * t * t * h->elt))) return fail(rc);
    h->d_rP = vp;
    if ((rc = h->alloc_raw(vp, (size_t)(p - 1) * t * t * h->elt))) return fail(rc);
    h->d_rS = vp;
    if ((rc = h->alloc_raw(vp, rw_elems * h->elt))) return fail(rc);
    h->d_rW = vp;
    // the identity tile (fifth work tile), built on the host once
    if (h->sdt == 0) {
      std::vector<double> id((size_t)t * t, 0.0);
      for (int i = 0; i < t; ++i) id[(size_t)i * t + i] = 1.0;
      if (hipMemcpy((char*)vp + 4 * (size_t)t * t * 8, id.data(), id.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return fail(DDPS_E_HIP);
    } else {
      std::vector<float> id((size_t)t * t, 0.f);
      for (int i = 0; i < t; ++i) id[(size_t)i * t + i] = 1.f;
      if (hipMemcpy((char*)vp + 4 * (size_t)t * t * 4, id.data(), id.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(DDPS_E_HIP);
    }
  }
  if ((rc = h->alloc(h->d_colnorm, (int64_t)p * 2 * t)) || (rc = h->alloc(h->d_mask, std::max<int64_t>(m, 1))) ||
      (rc = h->alloc(h->d_c, std::max<int64_t>(m, 1))) || (rc = h->alloc(h->d_rrow, std::max<int64_t>(m, 1))) ||
      (rc = h->alloc(h->d_blk, p)) || (rc = h->alloc(h->d_ypad, h->Np * R)) || (rc = h->alloc(h->d_vpad, h->Np * R)) ||
      (rc = h->alloc(h->d_thresh, h->Np + t)))
    return fail(rc);
  const int64_t mR = std::max<int64_t>(m, 1) * R;
  if ((rc = h->alloc(h->d_gh, mR)) || (rc = h->alloc(h->d_zh, mR)) || (rc = h->alloc(h->d_r, mR)) ||
      (rc = h->alloc(h->d_rt, mR)) || (rc = h->alloc(h->d_p, mR)) || (rc = h->alloc(h->d_v, mR)) ||
      (rc = h->alloc(h->d_s, mR)) || (rc = h->alloc(h->d_tv, mR)) || (rc = h->alloc(h->d_guess, mR)) ||
      (rc = h->alloc(h->d_mp, mR)) || (rc = h->alloc(h->d_ms, mR)))
    return fail(rc);
  const int64_t nR = n * R;
  if ((rc = h->alloc(h->d_fo, nR)) || (rc = h->alloc(h->d_xo, nR)) || (rc = h->alloc(h->d_ro, nR)) ||
      (rc = h->alloc(h->d_z, nR)) || (rc = h->alloc(h->d_rto, nR)) || (rc = h->alloc(h->d_po, nR)) ||
      (rc = h->alloc(h->d_vo, nR)) || (rc = h->alloc(h->d_ph, nR)) || (rc = h->alloc(h->d_sh, nR)) ||
      (rc = h->alloc(h->d_to, nR)))
    return fail(rc);
  h->part_cap = Wmax * R * 4;
  if ((rc = h->alloc(h->d_part_buf, h->part_cap)) || (rc = h->alloc(h->d_sums, 5 * 2 * kMaxRhs)) ||
      (rc = h->alloc(h->d_red1, (int64_t)kReduceGroups * kMaxRhs * 2)) ||
      (rc = h->alloc(h->d_out, 4 * kMaxRhs)) || (rc = h->alloc(h->d_state, 1)) || (rc = h->alloc(h->d_flag, kMaxRhs)))
    return fail(rc);
  // zero every vector buffer once (unused RHS columns stay finite)
  for (double* q : {h->d_ypad, h->d_vpad}) fill_f64(q, h->Np * R, 0.0, s);
  for (double* q : {h->d_gh, h->d_zh, h->d_r, h->d_rt, h->d_p, h->d_v, h->d_s, h->d_tv, h->d_guess, h->d_mp, h->d_ms})
    fill_f64(q, mR, 0.0, s);
  for (double* q : {h->d_fo, h->d_xo, h->d_ro, h->d_z, h->d_rto, h->d_po, h->d_vo, h->d_ph, h->d_sh, h->d_to})
    fill_f64(q, nR, 0.0, s);
  // reduced-space index maps
  if (m > 0) {
    std::vector<int64_t> c(m), rrow(m);
    for (int j = 0; j < p - 1; ++j) {
      const BlockInfo& A = h->blk[j];
      const BlockInfo& B = h->blk[j + 1];
      for (int q = 0; q < 2 * t; ++q) {
        const int64_t idx = (int64_t)2 * j * t + q;
        c[idx] = B.s - t + q;
        rrow[idx] = q < t ? A.voff + A.N - t + q : B.voff + B.pad + (q - t);
      }
    }
    if (hipMemcpyAsync(h->d_c, c.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->d_rrow, rrow.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(DDPS_E_HIP);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(DDPS_E_HIP);
  }
  if (hipMemcpyAsync(h->d_blk, h->blk.data(), sizeof(BlockInfo) * p, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(DDPS_E_HIP);
  const double eps = h->sdt == 0 ? 2.220446049250313e-16 : 1.1920928955078125e-7;
  // the t entries after the padded rows stay 0: pivot thresholds of the
  // reduced system's tile LU (only a zero or non-finite pivot is reported)
  fill_f64(h->d_thresh + h->Np, t, 0.0, s);
  setup_row_thresh(n, p, h->Np, h->d_part, h->d_blk, h->d_rowptr, h->d_col, h->d_val, eps, h->d_thresh, s);
  // execution resources and schedules
  if (hipStreamCreateWithFlags(&h->fstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess)
    return fail(DDPS_E_HIP);
  h->use_graph = o.factor_graph != 0;
  if ((rc = build_schedules(h))) return fail(rc);
  (void)hipEventRecord(h->ev1, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(DDPS_E_HIP);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
  h->t_setup_ms = ms;
  *out = h;
  return DDPS_OK;
}

int ddps_factor(ddps_handle h) {
  if (!h) return DDPS_E_ARG;
  (void)hipEventRecord(h->ev0, h->stream);
  // the factorisation runs on the internal stream, ordered after the
  // caller's stream and joined back into it
  HIPCHK(hipEventRecord(h->fork_ev, h->stream));
  HIPCHK(hipStreamWaitEvent(h->fstream, h->fork_ev, 0));
  if (h->use_graph) {
    if (!h->graph_exec) {
      h->drop_capture_events();
      HIPCHK(hipEventCreateWithFlags(&h->cap_fork, hipEventDisableTiming));
      for (size_t g = 0; g < h->gstream.size(); ++g) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->cap_gevent.push_back(e);
      }
      h->capturing = true;
      hipError_t e = hipStreamBeginCapture(h->fstream, hipStreamCaptureModeThreadLocal);
      int rc = e == hipSuccess ? enqueue_factor(h) : DDPS_E_HIP;
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(h->fstream, &g);
      h->capturing = false;
      if (rc || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        last_hip_error() = e2;
        return rc ? rc : DDPS_E_HIP;
      }
      h->graph = g;
      HIPCHK(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(h->graph_exec, h->fstream));
  } else {
    int rc = enqueue_factor(h);
    if (rc) return rc;
  }
  HIPCHK(hipEventRecord(h->join_ev, h->fstream));
  HIPCHK(hipStreamWaitEvent(h->stream, h->join_ev, 0));
  (void)hipEventRecord(h->ev1, h->stream);
  unsigned long long bad = 0;
  unsigned int flags = 0;
  HIPCHK(hipMemcpyAsync(&bad, h->d_bad, sizeof(bad), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(&flags, h->d_flags, sizeof(flags), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
  h->t_factor_ms = ms;
  if (flags) return DDPS_E_ARG;
  if (bad != ~0ull) {
    h->bad_block = (int32_t)(bad >> 40);
    h->bad_row = (int64_t)(bad & ((1ull << 40) - 1));
    h->factored = false;
    return DDPS_E_SINGULAR;
  }
  h->bad_block = -1;
  h->bad_row = -1;
  h->factored = true;
  return DDPS_OK;
}

int ddps_refactor_values(ddps_handle h, const double* val) {
  if (!h || !val) return DDPS_E_ARG;
  HIPCHK(hipMemcpyAsync(h->d_val, val, sizeof(double) * h->nnz, hipMemcpyDeviceToDevice, h->stream));
  fill_u64(h->d_band, 1, 0ull, h->stream);
  fill_f32((float*)h->d_flags, 1, 0.f, h->stream);
  setup_scan(h->n, h->p, h->d_part, h->d_rowptr, h->d_col, h->d_val, h->nnz, h->d_band, h->d_flags, h->stream);
  const double eps = h->sdt == 0 ? 2.220446049250313e-16 : 1.1920928955078125e-7;
  setup_row_thresh(h->n, h->p, h->Np, h->d_part, h->d_blk, h->d_rowptr, h->d_col, h->d_val, eps, h->d_thresh,
                   h->stream);
  unsigned int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, h->d_flags, sizeof(flags), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->factored = false;
  return flags ? DDPS_E_ARG : DDPS_OK;
}

static int solve_impl(ddps_handle h, int k, const double* F, int64_t ldf, double* X, int64_t ldx, double tol,
                      ddps_info* info) {
  if (!h || !F || !X || k < 1 || k > h->opt.max_rhs || ldf < h->n || ldx < h->n || !(tol > 0.0)) return DDPS_E_ARG;
  if (!h->factored) return DDPS_E_STATE;
  hipStream_t s = h->stream;
  const int R = h->R;
  const int64_t n = h->n;
  (void)hipEventRecord(h->ev0, s);
  // internal copies with leading dimension n; unused columns are zero
  HIPCHK(hipMemcpy2DAsync(h->d_fo, n * 8, F, ldf * 8, n * 8, k, hipMemcpyDeviceToDevice, s));
  if (h->opt.use_x0)
    HIPCHK(hipMemcpy2DAsync(h->d_xo, n * 8, X, ldx * 8, n * 8, k, hipMemcpyDeviceToDevice, s));
  else
    fill_f64(h->d_xo, n * R, 0.0, s);
  const bool guess = h->opt.guess == 1 && h->guess_k > 0;
  std::vector<double> rinf, r2, finf, f2;
  int rc = resid(h, h->d_xo, h->d_ro, rinf, r2, finf, f2);
  if (rc) return rc;
  // the stopping norm: inf (Section 4) or 2 (opt.norm); `cur` picks the
  // residual norms of the chosen kind after each resid()
  const bool two = h->opt.norm == 2;
  std::vector<double> fnorm(two ? f2 : finf), f2n(f2.begin(), f2.end()), finfn(finf.begin(), finf.end());
  auto cur = [&]() -> const std::vector<double>& { return two ? r2 : rinf; };
  auto conv_col = [&](int j, double ri) { return ri <= tol * fnorm[j] || fnorm[j] == 0.0; };
  double outer = 0;
  int64_t inner_total = 0;
  int apps = 0;
  int undone = 0, loosened_n = 0;   // refinement steps undone / taken loosened
  bool breakdown = false;
  std::vector<int> its;
  int bk = 0;
  auto all_conv = [&](const std::vector<double>& ri) {
    for (int j = 0; j < k; ++j)
      if (!conv_col(j, ri[j])) return false;
    return true;
  };
  // inner tolerance of one application: opt.inner_tol, relaxed (never beyond
  // 1e-2) when the current residual is already small, since an application
  // then only has to reduce it by tol * ||f|| / ||r||
  double itol = h->opt.inner_tol;
  auto papply = [&](const double* y, double* z) -> int {
    // the guess seeds the reduced solve of the first application only; later
    // applications act on residuals, for which it is no approximation
    int r = prec_apply(h, k, y, n, z, n, itol, (guess && apps == 0) ? 1 : 0, its, &bk);
    if (r) return r;
    ++apps;
    for (int j = 0; j < k; ++j) inner_total += its[j];
    if (bk) breakdown = true;
    return DDPS_OK;
  };
  if (h->opt.outer_method == 1) {
    // iterative refinement: x += P^{-1} (f - A x).
    // A step's inner tolerance is inner_tol, or the end-game value
    // 0.1 tol ||f|| / ||r|| when larger (at most 1e-2).  rho_f is the
    // residual ratio of the last step taken at that tolerance.  When rho_f is
    // at most 1e-2 but far above the tolerance, the factors (not the inner
    // solve) limit a step, and later steps ask the inner solve for 0.1 rho_f
    // only.  Such a loosened step never updates rho_f.  If its ratio exceeds
    // guard * rho_f, x and its residual are restored from before the step,
    // loosening stops for the rest of the solve, and the step is redone at
    // the unloosened tolerance; so every loosened step that is kept cuts the
    // residual by at most guard * rho_f (the undone one still counts as an
    // outer iteration and an application).
    double rho_f = -1.0;
    bool loosen_off = h->opt.loosen_ratio < 0.0;
    undone = loosened_n = 0;
    const double guard = h->opt.loosen_ratio > 0.0 ? h->opt.loosen_ratio : 10.0;
    std::vector<double> rprev;
    while (!all_conv(cur()) && outer < h->opt.outer_maxit) {
      double worst = 0.0;   // largest ||r||/||f|| still above the tolerance
      for (int j = 0; j < k; ++j)
        if (fnorm[j] > 0) worst = std::max(worst, cur()[j] / fnorm[j]);
      itol = h->opt.inner_tol;
      const bool loosened = !loosen_off && rho_f > 0.0 && rho_f <= 1e-2 && 0.1 * rho_f > itol;
      if (loosened) itol = 0.1 * rho_f;
      if (worst > 0) itol = std::min(1e-2, std::max(itol, 0.1 * tol / worst));
      rprev = cur();
      // a loosened step may be undone: keep x (d_rto is free under refinement)
      if (loosened) HIPCHK(hipMemcpyAsync(h->d_rto, h->d_xo, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
      if ((rc = papply(h->d_ro, h->d_z))) return rc;
      // columns already converged keep their x
      Coef3 cf{};
      for (int j = 0; j < R; ++j) {
        cf.a[j] = 1.0;
        cf.b[j] = (j < k && !conv_col(j, cur()[j])) ? 1.0 : 0.0;
      }
      lincomb(R, n, cf, h->d_xo, h->d_z, nullptr, h->d_xo, s);
      if ((rc = resid(h, h->d_xo, h->d_ro, rinf, r2, finf, f2))) return rc;
      double rho = 0.0;
      for (int j = 0; j < k; ++j)
        if (rprev[j] > 0 && !conv_col(j, rprev[j])) rho = std::max(rho, cur()[j] / rprev[j]);
      outer += 1;
      if (!loosened) {
        rho_f = rho;
      } else if (rho > guard * rho_f) {
        loosen_off = true;
        HIPCHK(hipMemcpyAsync(h->d_xo, h->d_rto, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
        if ((rc = resid(h, h->d_xo, h->d_ro, rinf, r2, finf, f2))) return rc;
        ++undone;
      }
      if (loosened) ++loosened_n;
    }
  } else {
    // preconditioned BiCGStab (Templates form), convergence tested after
    // each half step on the inf-norm relative residual; per-column scalars
    std::vector<double> rho(R, 1.0), rho_old(R, 1.0), alpha(R, 0.0), omega(R, 1.0), d0, d1, nrm;
    std::vector<int> active(R, 0);
    for (int j = 0; j < k; ++j) active[j] = conv_col(j, cur()[j]) ? 0 : 1;
    HIPCHK(hipMemcpyAsync(h->d_rto, h->d_ro, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
    int restarts = 0;
    bool fresh = true;
    Coef3 cf{};
    for (int it = 1; it <= h->opt.outer_maxit; ++it) {
      bool any = false;
      for (int j = 0; j < k; ++j) any |= active[j] != 0;
      if (!any) break;
      if ((rc = dots(h, n, h->d_rto, h->d_ro, nullptr, nullptr, d0, d1))) return rc;
      bool brk = false;
      for (int j = 0; j < R; ++j) {
        rho[j] = d0[j];
        if (j < k && active[j] && rho[j] == 0.0) brk = true;
      }
      for (int j = 0; j < R; ++j) {
        const double beta = (!fresh && active[j]) ? (rho[j] / rho_old[j]) * (alpha[j] / omega[j]) : 0.0;
        cf.a[j] = 1.0; cf.b[j] = beta; cf.c[j] = -beta * omega[j];
      }
      lincomb(R, n, cf, h->d_ro, h->d_po, h->d_vo, h->d_po, s);
      fresh = false;
      if ((rc = papply(h->d_po, h->d_ph))) return rc;
      if ((rc = matvec(h, h->d_ph, h->d_vo))) return rc;
      if ((rc = dots(h, n, h->d_rto, h->d_vo, nullptr, nullptr, d0, d1))) return rc;
      for (int j = 0; j < R; ++j) {
        alpha[j] = 0.0;
        if (j >= k || !active[j]) continue;
        if (d0[j] == 0.0 || !std::isfinite(rho[j] / d0[j])) brk = true;
        else alpha[j] = rho[j] / d0[j];
      }
      // s = r - alpha v (d_sh); a column whose ||s|| meets the tolerance takes
      // x += alpha p^ and stops after this half step
      for (int j = 0; j < R; ++j) { cf.a[j] = 1.0; cf.b[j] = -alpha[j]; cf.c[j] = 0.0; }
      lincomb(R, n, cf, h->d_ro, h->d_vo, nullptr, h->d_sh, s);
      if ((rc = norm_of(h, h->d_sh, two, nrm))) return rc;
      std::vector<int> half(R, 0);
      bool anyh = false, anyfull = false;
      for (int j = 0; j < k; ++j)
        if (active[j] && alpha[j] != 0.0 && conv_col(j, nrm[j])) { half[j] = 1; anyh = true; }
      if (anyh) {
        for (int j = 0; j < R; ++j) { cf.a[j] = 1.0; cf.b[j] = half[j] ? alpha[j] : 0.0; cf.c[j] = 0.0; }
        lincomb(R, n, cf, h->d_xo, h->d_ph, nullptr, h->d_xo, s);
      }
      for (int j = 0; j < k; ++j) {
        if (half[j]) { active[j] = 0; outer = std::max(outer, it - 0.5); }
        anyfull |= active[j] != 0;
      }
      if (!anyfull) break;
      if ((rc = papply(h->d_sh, h->d_z))) return rc;   // s^ in d_z
      if ((rc = matvec(h, h->d_z, h->d_to))) return rc;
      if ((rc = dots(h, n, h->d_to, h->d_sh, h->d_to, h->d_to, d0, d1))) return rc;
      for (int j = 0; j < R; ++j) omega[j] = (j < k && active[j] && d1[j] != 0.0) ? d0[j] / d1[j] : 0.0;
      // x += alpha p^ + omega s^ ;  r = s - omega t   (inactive columns unchanged)
      for (int j = 0; j < R; ++j) {
        const bool a = j < k && active[j];
        cf.a[j] = 1.0; cf.b[j] = a ? alpha[j] : 0.0; cf.c[j] = a ? omega[j] : 0.0;
      }
      lincomb(R, n, cf, h->d_xo, h->d_ph, h->d_z, h->d_xo, s);
      for (int j = 0; j < R; ++j) {
        const bool a = j < k && active[j];
        cf.a[j] = a ? 1.0 : 0.0; cf.b[j] = a ? -omega[j] : 0.0; cf.c[j] = a ? 0.0 : 1.0;
      }
      lincomb(R, n, cf, h->d_sh, h->d_to, h->d_ro, h->d_ro, s);
      if ((rc = norm_of(h, h->d_ro, two, nrm))) return rc;
      for (int j = 0; j < k; ++j) {
        if (!active[j]) continue;
        outer = std::max(outer, (double)it);
        if (conv_col(j, nrm[j])) active[j] = 0;
        else if (omega[j] == 0.0) brk = true;
      }
      rho_old = rho;
      if (brk) {
        if (restarts >= 1) { breakdown = true; break; }
        ++restarts;
        HIPCHK(hipMemcpyAsync(h->d_rto, h->d_ro, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
        fresh = true;
      }
    }
  }
  // true residual of the final iterate
  if ((rc = resid(h, h->d_xo, h->d_ro, rinf, r2, finf, f2))) return rc;
  HIPCHK(hipMemcpy2DAsync(X, ldx * 8, h->d_xo, n * 8, n * 8, k, hipMemcpyDeviceToDevice, s));
  (void)hipEventRecord(h->ev1, s);
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
  h->t_solve_ms = ms;
  h->last_k = k;
  double worst_inf = 0, worst_2 = 0;
  bool ok = true;
  for (int j = 0; j < k; ++j) {
    const double ri = finfn[j] > 0 ? rinf[j] / finfn[j] : 0.0;
    const double rt = f2n[j] > 0 ? r2[j] / f2n[j] : 0.0;
    worst_inf = std::max(worst_inf, ri);
    worst_2 = std::max(worst_2, rt);
    if (!((two ? rt : ri) <= tol)) ok = false;
  }
  if (h->opt.outer_method == 1 && outer == 0 && ok) outer = 0;
  if (info) {
    info->outer_iters = outer;
    info->inner_iters_total = inner_total / 2;
    info->applications = apps;
    info->inner_iters_avg = apps ? (double)inner_total / 2.0 / ((double)apps * k) : 0.0;
    info->relres_inf = worst_inf;
    info->relres_2 = worst_2;
    info->t_setup_ms = h->t_setup_ms;
    info->t_factor_ms = h->t_factor_ms;
    info->t_solve_ms = h->t_solve_ms;
    info->bad_block = h->bad_block;
    info->bad_row = h->bad_row;
    info->loosened_steps = loosened_n;
    info->undone_steps = undone;
  }
  if (ok) return DDPS_OK;
  if (breakdown) return DDPS_E_BREAKDOWN;
  return DDPS_E_NOCONV;
}

int ddps_solve(ddps_handle h, const double* f, double* x, double tol, ddps_info* info) {
  if (!h) return DDPS_E_ARG;
  return solve_impl(h, 1, f, h->n, x, h->n, tol, info);
}

int ddps_solve_many(ddps_handle h, int32_t k, const double* F, int64_t ldf, double* X, int64_t ldx, double tol,
                    ddps_info* info) {
  return solve_impl(h, k, F, ldf, X, ldx, tol, info);
}

int ddps_set_guess(ddps_handle h, const double* zhat0, int32_t k) {
  if (!h || k < 0 || k > h->R) return DDPS_E_ARG;
  if (k == 0 || !zhat0) {
    h->guess_k = 0;
    return DDPS_OK;
  }
  if (h->m == 0) return DDPS_OK;
  fill_f64(h->d_guess, h->m * h->R, 0.0, h->stream);
  HIPCHK(hipMemcpyAsync(h->d_guess, zhat0, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  // entries outside c are not unknowns of the reduced system: zero them
  vec_apply_mask(h->m, h->R, h->d_mask, h->d_guess, h->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  h->guess_k = k;
  return DDPS_OK;
}

int ddps_set_guess_model(ddps_handle h, ddps_mlp net) {
  if (!h) return DDPS_E_ARG;
  if (!net) {
    h->gnet = nullptr;
    return DDPS_OK;
  }
  int din = 0, dout = 0, mb = 0;
  hipStream_t ns = nullptr;
  if (mlp_shape(net, &din, &dout, &mb, &ns) || din < 4 * h->t + 2 || dout != 2 * h->t ||
      (int64_t)mb < (int64_t)h->R * (h->p - 1) || ns != h->stream)
    return DDPS_E_ARG;
  if (h->m == 0) return DDPS_OK;
  if (din != h->gnet_din) {
    const int64_t rows = (int64_t)h->R * (h->p - 1);
    for (float* q : {h->d_gX, h->d_gS, h->d_gY}) h->free_ptr(q);
    h->d_gX = h->d_gS = h->d_gY = nullptr;
    int rc;
    if ((rc = h->alloc(h->d_gX, rows * din)) || (rc = h->alloc(h->d_gS, rows)) ||
        (rc = h->alloc(h->d_gY, rows * dout)))
      return rc;
    h->gnet_din = din;
  }
  h->gnet = net;
  h->gnet_losses = 0;
  h->gtrial_n[0] = h->gtrial_n[1] = h->gtrial_its[0] = h->gtrial_its[1] = 0;
  h->gtrial_seq = 0;
  h->gtrial_done = false;
  h->garm.clear();
  return DDPS_OK;
}

int ddps_guess_counts(ddps_handle h, int64_t* counts) {
  if (!h || !counts) return DDPS_E_ARG;
  for (int q = 0; q < 3; ++q) counts[q] = h->guess_counts[q];
  counts[3] = h->gnet_skipped;
  return DDPS_OK;
}

int ddps_guess_trial(ddps_handle h, int64_t* solves, double* mean_iters, int32_t* state) {
  if (!h || !solves || !mean_iters || !state) return DDPS_E_ARG;
  for (int a = 0; a < 2; ++a) {
    solves[a] = h->gtrial_n[a];
    // the inner solve counts half iterations
    mean_iters[a] = h->gtrial_n[a] ? 0.5 * (double)h->gtrial_its[a] / (double)h->gtrial_n[a] : 0.0;
  }
  *state = h->gnet_losses >= kRetire ? 2 : (h->gtrial_done ? 1 : 0);
  return DDPS_OK;
}

int ddps_reduced_layout(ddps_handle h, int64_t* m, int64_t* c, double* mask, int32_t* t, int32_t* b) {
  if (!h) return DDPS_E_ARG;
  if (mask && h->m && !h->factored) return DDPS_E_STATE;   // the dropping rule runs in ddps_factor
  if (m) *m = h->m;
  if (t) *t = h->t;
  if (b) *b = h->b;
  if (c && h->m) HIPCHK(hipMemcpyAsync(c, h->d_c, sizeof(int64_t) * h->m, hipMemcpyDeviceToDevice, h->stream));
  if (mask && h->m)
    HIPCHK(hipMemcpyAsync(mask, h->d_mask, sizeof(double) * h->m, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDPS_OK;
}

int ddps_last_reduced(ddps_handle h, double* ghat, double* zhat) {
  if (!h) return DDPS_E_ARG;
  const int k = std::max(1, h->last_k);
  if (ghat && h->m) HIPCHK(hipMemcpyAsync(ghat, h->d_gh, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  if (zhat && h->m) HIPCHK(hipMemcpyAsync(zhat, h->d_zh, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDPS_OK;
}

int ddps_apply_preconditioner(ddps_handle h, int32_t k, const double* y, double* z, double* ghat, double* zhat,
                              double* inner_iters) {
  if (!h || !y || !z || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (!h->factored) return DDPS_E_STATE;
  std::vector<int> its;
  int bk = 0;
  const bool guess = h->opt.guess == 1 && h->guess_k > 0;
  int rc = prec_apply(h, k, y, h->n, z, h->n, h->opt.inner_tol, guess ? 1 : 0, its, &bk);
  if (rc) return rc;
  if (ghat && h->m) HIPCHK(hipMemcpyAsync(ghat, h->d_gh, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  if (zhat && h->m) HIPCHK(hipMemcpyAsync(zhat, h->d_zh, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (inner_iters)
    for (int j = 0; j < k; ++j) inner_iters[j] = its[j] / 2.0;
  h->last_k = k;
  return bk ? DDPS_E_BREAKDOWN : DDPS_OK;
}

int ddps_block_solve(ddps_handle h, int32_t k, const double* y, double* g) {
  if (!h || !y || !g || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (!h->factored) return DDPS_E_STATE;
  const int R = h->R;
  vec_to_padded(h->Np, R, k, h->p, h->d_blk, y, h->n, h->d_ypad, h->stream);
  int rc = block_solves(h, TK_SWEEP);
  if (rc) return rc;
  vec_from_padded(h->Np, k, h->p, h->d_blk, h->d_ypad, g, h->n, h->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDPS_OK;
}

int ddps_reduced_matvec(ddps_handle h, int32_t k, const double* x, double* v) {
  if (!h || !x || !v || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (!h->factored) return DDPS_E_STATE;
  if (h->m == 0) return DDPS_OK;
  HIPCHK(hipMemcpyAsync(h->d_zh, x, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  run_launch(h, h->l_zv, h->R, h->m, h->m, nullptr, nullptr, nullptr, TK_RSPMV);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(v, h->d_v, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDPS_OK;
}


// ---------------------------------------------------------------- learned guess
int ddps_reduced_rhs(ddps_handle h, int32_t k, const double* y, double* ghat) {
  if (!h || !y || !ghat || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (!h->factored) return DDPS_E_STATE;
  if (h->m == 0) return DDPS_OK;
  const int R = h->R;
  hipStream_t s = h->stream;
  vec_to_padded(h->Np, R, k, h->p, h->d_blk, y, h->n, h->d_ypad, s);
  int rc = block_solves(h, TK_SWEEP);
  if (rc) return rc;
  vec_gather_reduced(h->m, R, h->d_rrow, h->d_mask, h->d_ypad, h->Np, h->d_r, s);
  HIPCHK(hipMemcpyAsync(ghat, h->d_r, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return DDPS_OK;
}

int ddps_reduced_restrict(ddps_handle h, int32_t k, const double* x, double* z) {
  if (!h || !x || !z || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (h->m == 0) return DDPS_OK;
  const int R = h->R;
  hipStream_t s = h->stream;
  vec_to_padded(h->Np, R, k, h->p, h->d_blk, x, h->n, h->d_ypad, s);
  vec_gather_reduced(h->m, R, h->d_rrow, h->d_mask, h->d_ypad, h->Np, h->d_r, s);
  HIPCHK(hipMemcpyAsync(z, h->d_r, sizeof(double) * h->m * k, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return DDPS_OK;
}

int ddps_reduced_residual(ddps_handle h, int32_t k, const double* ghat, const double* z, double* res, double* rvec) {
  if (!h || !ghat || !z || !res || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (!h->factored) return DDPS_E_STATE;
  const int R = h->R;
  const int64_t m = h->m;
  if (m == 0) {
    for (int j = 0; j < k; ++j) res[j] = 0.0;
    return DDPS_OK;
  }
  hipStream_t s = h->stream;
  fill_f64(h->d_zh, m * R, 0.0, s);
  fill_f64(h->d_r, m * R, 0.0, s);
  HIPCHK(hipMemcpyAsync(h->d_zh, z, sizeof(double) * m * k, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(h->d_r, ghat, sizeof(double) * m * k, hipMemcpyDeviceToDevice, s));
  vec_apply_mask(m, R, h->d_mask, h->d_zh, s);
  run_launch(h, h->l_zv, R, m, m, nullptr, nullptr, nullptr, TK_RSPMV);
  Coef3 cf{};
  for (int j = 0; j < R; ++j) {
    cf.a[j] = 1.0;
    cf.b[j] = -1.0;
  }
  lincomb(R, m, cf, h->d_r, h->d_v, nullptr, h->d_r, s);
  vec_apply_mask(m, R, h->d_mask, h->d_r, s);
  if (rvec) HIPCHK(hipMemcpyAsync(rvec, h->d_r, sizeof(double) * m * k, hipMemcpyDeviceToDevice, s));
  std::vector<double> d0, d1;
  int rc = dots(h, m, h->d_r, h->d_r, nullptr, nullptr, d0, d1);
  if (rc) return rc;
  for (int j = 0; j < k; ++j) res[j] = std::sqrt(d0[j]);
  return DDPS_OK;
}

int ddps_guess_features(ddps_handle h, int32_t k, const double* r, const double* zprev, double cos_t,
                        double sin_t, int32_t d_in, float* X, float* scale) {
  if (!h || !r || !zprev || !X || !scale || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (d_in < 4 * h->t + 2) return DDPS_E_ARG;
  if (h->m == 0) return DDPS_OK;
  const int nif = h->p - 1;
  guess_features(nif, k, 2 * h->t, d_in, r, zprev, h->d_mask, cos_t, sin_t, X, scale, h->stream);
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

int ddps_guess_compose(ddps_handle h, int32_t k, const double* zprev, const float* Y, const float* scale,
                       double* zhat0) {
  if (!h || !zprev || !Y || !scale || !zhat0 || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (h->m == 0) return DDPS_OK;
  guess_compose(h->m * k, h->m, 2 * h->t, zprev, Y, scale, h->d_mask, zhat0, h->stream);
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

int ddps_guess_target(ddps_handle h, int32_t k, const double* zhat, const double* zprev, const float* scale,
                      float* T) {
  if (!h || !zhat || !zprev || !scale || !T || k < 1 || k > h->opt.max_rhs) return DDPS_E_ARG;
  if (h->m == 0) return DDPS_OK;
  guess_target(h->m * k, h->m, 2 * h->t, zhat, zprev, scale, h->d_mask, T, h->stream);
  HIPCHK(hipGetLastError());
  return DDPS_OK;
}

int ddps_get_tile(ddps_handle h, int32_t blk, int32_t k, int32_t which, double* dst) {
  if (!h || !dst || blk < 0 || blk >= h->p || which < 0 || which > 2) return DDPS_E_ARG;
  if (h->ilu) return DDPS_E_STATE;   // incomplete factors keep no tiles
  const BlockInfo& B = h->blk[blk];
  if (k < 0 || k >= B.T || (which > 0 && k >= B.T - 1)) return DDPS_E_ARG;
  const int t = h->t;
  const int64_t tt = (int64_t)t * t;
  const char* src = which == 0 ? h->tile(blk, 0, k) : h->lu(blk, which, k);
  std::vector<double> out(tt);
  if (h->sdt == 0) {
    HIPCHK(hipMemcpyAsync(out.data(), src, sizeof(double) * tt, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  } else {
    std::vector<float> tmp(tt);
    HIPCHK(hipMemcpyAsync(tmp.data(), src, sizeof(float) * tt, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int64_t q = 0; q < tt; ++q) out[q] = tmp[q];
  }
  // the off-diagonal factors are halves of a pair: the other half holds the
  // other factor, so it is zeroed here (L_{k+1,k} is upper, U_{k,k+1} lower)
  if (which > 0)
    for (int64_t c = 0; c < t; ++c)
      for (int64_t r = 0; r < t; ++r)
        if (which == 1 ? r > c : r < c) out[c * t + r] = 0.0;
  HIPCHK(hipMemcpyAsync(dst, out.data(), sizeof(double) * tt, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDPS_OK;
}

int ddps_get_spikes(ddps_handle h, int32_t blk, double* dst) {
  if (!h || !dst || blk < 0 || blk >= h->p) return DDPS_E_ARG;
  if (h->tips_only) return DDPS_E_STATE;   // only the tips are kept
  const BlockInfo& B = h->blk[blk];
  const int t = h->t;
  if (h->p == 1) {
    fill_f64(dst, B.n * 2 * t, 0.0, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    return DDPS_OK;
  }
  const int64_t cnt = B.N * 2 * t;
  std::vector<double> full(cnt), outv(B.n * 2 * t);
  if (h->sdt == 0) {
    HIPCHK(hipMemcpyAsync(full.data(), h->spike(blk, 0, 0), sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  } else {
    std::vector<float> tmp(cnt);
    HIPCHK(hipMemcpyAsync(tmp.data(), h->spike(blk, 0, 0), sizeof(float) * cnt, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int64_t q = 0; q < cnt; ++q) full[q] = tmp[q];
  }
  for (int64_t c = 0; c < 2 * t; ++c)
    for (int64_t r = 0; r < B.n; ++r) outv[c * B.n + r] = full[c * B.N + B.pad + r];
  HIPCHK(hipMemcpyAsync(dst, outv.data(), sizeof(double) * outv.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DDPS_OK;
}

int ddps_block_shape(ddps_handle h, int32_t* t, int32_t* tiles, int32_t* pads) {
  if (!h) return DDPS_E_ARG;
  if (t) *t = h->t;
  for (int i = 0; i < h->p; ++i) {
    if (tiles) tiles[i] = (int32_t)h->blk[i].T;
    if (pads) pads[i] = (int32_t)h->blk[i].pad;
  }
  return DDPS_OK;
}

int ddps_last_singular(ddps_handle h, int32_t* block, int64_t* row) {
  if (!h) return DDPS_E_ARG;
  if (block) *block = h->bad_block;
  if (row) *row = h->bad_row;
  return DDPS_OK;
}

int ddps_set_execution(ddps_handle h, int32_t streams, int32_t graph, int32_t tile_policy) {
  if (!h || streams < 0 || tile_policy < 0 || tile_policy > 5) return DDPS_E_ARG;
  if (h->ilu) return DDPS_E_STATE;   // no factor schedule to arrange
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipStreamSynchronize(h->fstream));
  h->groups = streams > 0 ? streams : default_groups(h);
  h->use_graph = graph != 0;
  h->tile_policy = tile_policy;
  h->factored = false;   // the factors must be recomputed with the new form
  return build_schedules(h);
}

extern "C++" {  // internal helpers: C++ linkage
namespace {

std::string tune_key(ddps_ctx* h) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch = arch.substr(0, c);
  }
  static const char* dt[] = {"f64", "f32", "bf16x3", "bf16"};
  char buf[256];
  // the tips-only form's launch sequence depends on its workspace slots
  if (h->tips_only)
    std::snprintf(buf, sizeof(buf), "%s/%s/t%d/p%d/T%d/tips%lld", arch.c_str(), dt[h->gdt], h->t, h->p, h->Tmax,
                  (long long)h->nslots);
  else
    std::snprintf(buf, sizeof(buf), "%s/%s/t%d/p%d/T%d", arch.c_str(), dt[h->gdt], h->t, h->p, h->Tmax);
  return buf;
}

// The cache is a flat JSON object {"key": {"streams": s, "tile_policy": q,
// "factor_ms": ms, "modes": "..."}, ...}, one entry per line, written and
// read by this file only; "modes" (policy 3) holds the tile mode of each
// factor GEMM launch as one digit.
bool cache_lookup(const char* path, const std::string& key, int* streams, int* policy, double* ms,
                  std::string* modes) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string txt;
  char b[4096];
  size_t nr;
  while ((nr = std::fread(b, 1, sizeof(b), f)) > 0) txt.append(b, nr);
  std::fclose(f);
  const size_t at = txt.find("\"" + key + "\"");
  if (at == std::string::npos) return false;
  int s2 = 0, q2 = 0;
  double m2 = 0;
  const size_t br = txt.find('{', at);
  if (br == std::string::npos) return false;
  if (std::sscanf(txt.c_str() + br, "{\"streams\": %d, \"tile_policy\": %d, \"factor_ms\": %lf", &s2, &q2, &m2) != 3)
    return false;
  *streams = s2;
  *policy = q2;
  *ms = m2;
  modes->clear();
  const size_t end = txt.find('}', br);
  const std::string tag = "\"modes\": \"";
  const size_t mp = txt.find(tag, br);
  if (mp != std::string::npos && mp < end)
    for (size_t i = mp + tag.size(); i < txt.size() && txt[i] >= '0' && txt[i] <= '4'; ++i) modes->push_back(txt[i]);
  return true;
}

void cache_store(const char* path, const std::string& key, int streams, int policy, double ms,
                 const std::string& modes) {
  if (!path) return;
  std::vector<std::string> entries;
  if (FILE* f = std::fopen(path, "r")) {
    std::string txt;
    char b[4096];
    size_t nr;
    while ((nr = std::fread(b, 1, sizeof(b), f)) > 0) txt.append(b, nr);
    std::fclose(f);
    size_t pos = 0;
    while (pos < txt.size()) {
      size_t nl = txt.find('\n', pos);
      if (nl == std::string::npos) nl = txt.size();
      std::string l = txt.substr(pos, nl - pos);
      pos = nl + 1;
      if (l.find("\"streams\"") != std::string::npos && l.find("\"" + key + "\"") == std::string::npos) {
        while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
        entries.push_back(l);
      }
    }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf), "  \"%s\": {\"streams\": %d, \"tile_policy\": %d, \"factor_ms\": %.3f", key.c_str(),
                streams, policy, ms);
  std::string e = buf;
  if (policy == 3 && !modes.empty()) e += ", \"modes\": \"" + modes + "\"";
  e += "}";
  entries.push_back(e);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i) std::fprintf(f, "%s%s\n", entries[i].c_str(), i + 1 < entries.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

}  // namespace
}  // extern "C++"

extern "C++" {  // internal helpers: C++ linkage
namespace {
// Durations (ms) of the factor GEMM launches of one ddps_factor, in order.
int time_gemm_launches(ddps_ctx* h, std::vector<float>& out) {
  int rc;
  auto drain = [&]() {
    for (auto& r : h->tim[TK_GEMM]) {
      h->ev_pool.push_back(r.a);
      h->ev_pool.push_back(r.b);
    }
    h->tim[TK_GEMM].clear();
  };
  HIPCHK(hipDeviceSynchronize());
  drain();
  const bool was = h->tim_on[TK_GEMM];
  h->tim_on[TK_GEMM] = true;
  rc = ddps_factor(h);
  h->tim_on[TK_GEMM] = was;
  if (rc) return rc;
  HIPCHK(hipDeviceSynchronize());
  out.clear();
  for (auto& r : h->tim[TK_GEMM]) {
    float e = 0;
    HIPCHK(hipEventElapsedTime(&e, r.a, r.b));
    out.push_back(e);
  }
  drain();
  return DDPS_OK;
}

// Policy 3 for `groups` stream groups: time every factor GEMM launch under
// each fixed policy, keep per launch the tile of the fastest, and time the
// resulting schedule (*ms).  Leaves the handle factored with policy 3.
// Seconds since `t0` (host clock) for the autotuner's budget and progress.
double secs_since(const std::chrono::steady_clock::time_point& t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int tune_launch_modes(ddps_ctx* h, int groups, double* ms) {
  // fixed policies 0, 1, 2, 4 and 5 ask for tile modes 1, 0, 2, 3 and 4
  static const int8_t mode_of_policy[5] = {1, 0, 2, 3, 4};
  static const int policy_of[5] = {0, 1, 2, 4, 5};
  const int nq = h->gdt >= 2 ? 5 : 2;
  std::vector<std::vector<float>> t(nq);
  int rc;
  std::vector<float> t2;
  for (int q = 0; q < nq; ++q) {
    if ((rc = ddps_set_execution(h, groups, 0, policy_of[q]))) return rc;
    if ((rc = ddps_factor(h))) return rc;   // warm-up
    if ((rc = time_gemm_launches(h, t[q]))) return rc;
    if ((rc = time_gemm_launches(h, t2))) return rc;   // per launch, the faster of two runs
    if (t[q].size() != t[0].size() || t2.size() != t[q].size()) return DDPS_E_STATE;
    for (size_t i = 0; i < t2.size(); ++i) t[q][i] = std::min(t[q][i], t2[i]);
  }
  h->mode_choice.assign(t[0].size(), 1);
  for (size_t i = 0; i < t[0].size(); ++i) {
    int best = 0;
    for (int q = 1; q < nq; ++q)
      if (t[q][i] < t[best][i]) best = q;
    h->mode_choice[i] = mode_of_policy[best];
  }
  if ((rc = ddps_set_execution(h, groups, 0, 3))) return rc;
  if ((rc = ddps_factor(h))) return rc;   // warm-up
  if ((rc = ddps_factor(h))) return rc;
  *ms = h->t_factor_ms;
  return DDPS_OK;
}
}  // namespace
}  // extern "C++"

int ddps_autotune(ddps_handle h, const char* cache_path, double budget_s, int32_t* streams, int32_t* tile_policy,
                  double* factor_ms) {
  if (!h) return DDPS_E_ARG;
  if (h->ilu) return DDPS_E_STATE;
  const std::string key = tune_key(h);
  const auto t0 = std::chrono::steady_clock::now();
  // once the budget is spent no further form is timed: the best one so far
  // stands (the first form is always timed)
  auto over = [&]() { return budget_s > 0.0 && secs_since(t0) > budget_s; };
  int bs = 0, bq = 0;
  double bms = 0;
  int rc;
  std::string modes;
  const bool hit = cache_lookup(cache_path, key, &bs, &bq, &bms, &modes);
  // per-launch tiles tuned for group counts whose best fixed form is within
  // 10% of the fastest one (filled only without a cache hit)
  std::vector<int> cand;
  if (!hit) {
    // fewest stream groups within 3% of the fastest form: extra streams are
    // kept only for a clear gain (their launches then time as overlapping)
    std::vector<std::array<double, 3>> tried;   // groups, policy, ms
    double best = 1e300;
    std::vector<int> pols = {0, 1};
    if (h->gdt >= 2) pols = {0, 1, 2, 4, 5};
    for (int q : pols)
      for (int g : {1, 2, 3, 4, 6, 8}) {
        if (g > h->p || (h->tips_only && g > h->nslots)) continue;
        if (!tried.empty() && over()) break;
        if ((rc = ddps_set_execution(h, g, 0, q))) return rc;
        if ((rc = ddps_factor(h))) return rc;       // warm-up
        if ((rc = ddps_factor(h))) return rc;
        tried.push_back({(double)g, (double)q, h->t_factor_ms});
        best = std::min(best, h->t_factor_ms);
        std::fprintf(stderr, "ddps_autotune %s: %d groups, policy %d: %.2f ms (%.1f s)\n", key.c_str(), g, q,
                     h->t_factor_ms, secs_since(t0));
      }
    bms = 1e300;
    int bg = 1 << 30;
    for (auto& c : tried)
      if (c[2] <= 1.03 * best && ((int)c[0] < bg || ((int)c[0] == bg && c[2] < bms))) {
        bg = (int)c[0];
        bs = bg;
        bq = (int)c[1];
        bms = c[2];
      }
    for (int g : {1, 2, 3, 4, 6, 8}) {
      double gb = 1e300;
      for (auto& c : tried)
        if ((int)c[0] == g) gb = std::min(gb, c[2]);
      if (gb <= 1.10 * best) cand.push_back(g);
    }
  }
  bool stored = false;
  if (hit && bq == 3 && !modes.empty()) {
    // the cached per-launch tiles, if they fit this schedule
    h->mode_choice.assign(modes.size(), 1);
    for (size_t i = 0; i < modes.size(); ++i) h->mode_choice[i] = (int8_t)(modes[i] - '0');
    if ((rc = ddps_set_execution(h, bs, 0, 3))) return rc;
    stored = h->mode_cursor == (int)modes.size();
  }
  if (hit && bq == 3 && !stored) {
    // cached per-launch form whose tiles no longer fit: tune them again
    double ms3 = 0;
    if ((rc = tune_launch_modes(h, bs, &ms3))) return rc;
  } else if (!hit) {
    // per-launch tile choice: every factor GEMM launch is timed under each
    // policy (same launch sequence) and takes the tile of the policy under
    // which it ran fastest.  Done for each candidate group count; the fewest
    // groups within 3% of the fastest per-launch form win, if that beats the
    // fixed form.
    std::vector<std::pair<int, double>> per;
    std::vector<std::vector<int8_t>> choice;
    double best3 = 1e300;
    for (int g : cand) {
      if (over()) break;
      double ms3 = 0;
      if ((rc = tune_launch_modes(h, g, &ms3))) return rc;
      per.push_back({g, ms3});
      choice.push_back(h->mode_choice);
      best3 = std::min(best3, ms3);
      std::fprintf(stderr, "ddps_autotune %s: %d groups, per-launch tiles: %.2f ms (%.1f s)\n", key.c_str(), g, ms3,
                   secs_since(t0));
    }
    int pick = -1;
    for (size_t i = 0; i < per.size(); ++i)
      if (per[i].second <= 1.03 * best3 && (pick < 0 || per[i].first < per[pick].first)) pick = (int)i;
    if (pick >= 0 && per[pick].second < bms) {
      bs = per[pick].first;
      bq = 3;
      bms = per[pick].second;
      h->mode_choice = choice[pick];
    }
  }
  if (!hit || (bq == 3 && !stored)) {
    std::string ms_str;
    for (int8_t v : h->mode_choice) ms_str.push_back((char)('0' + v));
    cache_store(cache_path, key, bs, bq, bms, ms_str);
  }
  const int graph = h->use_graph ? 1 : 0;
  if ((rc = ddps_set_execution(h, bs, graph, bq))) return rc;
  if ((rc = ddps_factor(h))) return rc;
  if (streams) *streams = bs;
  if (tile_policy) *tile_policy = bq;
  if (factor_ms) *factor_ms = bms;
  return DDPS_OK;
}

int ddps_timing_enable(ddps_handle h, int32_t kind, int32_t on) {
  if (!h || kind < 0 || kind >= TK_N) return DDPS_E_ARG;
  h->tim_on[kind] = on != 0;
  return DDPS_OK;
}

int ddps_timing_read(ddps_handle h, int32_t kind, int64_t* launches, double* ms, double* flops, double* bytes) {
  if (!h || kind < 0 || kind >= TK_N) return DDPS_E_ARG;
  HIPCHK(hipStreamSynchronize(h->stream));
  double tot = 0, fl = 0, by = 0;
  for (auto& r : h->tim[kind]) {
    float e = 0;
    (void)hipEventElapsedTime(&e, r.a, r.b);
    tot += e;
    fl += r.flops;
    by += r.bytes;
    h->ev_pool.push_back(r.a);
    h->ev_pool.push_back(r.b);
  }
  if (launches) *launches = (int64_t)h->tim[kind].size();
  if (ms) *ms = tot;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  h->tim[kind].clear();
  return DDPS_OK;
}

int ddps_residual_norms(int64_t n, int32_t k, const int64_t* row_ptr, const int32_t* col, const double* val,
                        const double* X, int64_t ldx, const double* F, int64_t ldf, double* R, int64_t ldr,
                        double* norms, void* stream) {
  if (n <= 0 || k < 1 || k > kMaxRhs || !row_ptr || !col || !val || !X || !F || !norms || ldx < n || ldf < n ||
      (R && ldr < n))
    return DDPS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const size_t part_bytes = sizeof(double) * (size_t)kVecGrid * kMaxRhs * 4;
  void* buf = nullptr;
  if (hipMalloc(&buf, part_bytes + sizeof(double) * 4 * kMaxRhs) != hipSuccess) return DDPS_E_NOMEM;
  double* part = (double*)buf;
  double* out = part + (size_t)kVecGrid * kMaxRhs * 4;
  residual_norms_cols(n, k, row_ptr, col, val, X, ldx, F, ldf, R, ldr, part, out, s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(norms, out, sizeof(double) * 4 * k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) {
    last_hip_error() = e;
    return DDPS_E_HIP;
  }
  for (int j = 0; j < k; ++j) {
    norms[4 * j + 1] = std::sqrt(norms[4 * j + 1]);
    norms[4 * j + 3] = std::sqrt(norms[4 * j + 3]);
  }
  return DDPS_OK;
}

int ddps_memory(ddps_handle h, size_t* bytes) {
  if (!h || !bytes) return DDPS_E_ARG;
  *bytes = h->bytes;
  return DDPS_OK;
}

}  // extern "C"
