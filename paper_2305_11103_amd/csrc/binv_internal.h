// Internal declarations shared by the library's translation units: the
// argument records the kernels read and the launchers the host code calls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/binv.h"

namespace binv {

// One GEMM step problem (row panel or Schur update) of the blockwise sweep.
struct StepArgs {
  // operand A of the contraction, k-major (A[t][m]) or m-major (A[m][t])
  const double* A;
  int64_t lda;
  // operand B, k-major: B[t][j]
  const double* B;
  int64_t ldb;
  // output: row panel R (ld = ldw), or the working matrix W for the Schur update
  double* W;
  int64_t ldw;
  const double* Win;  // Schur update: matrix read before the update (== W in place)
  int64_t ldwin;
  const double* R;    // Schur update: row panel; row panel: the pivot inverse P
  int64_t ldr;
  int64_t M, N;       // output extent
  int K;              // contraction length (= b)
  int64_t o;          // first row of block p
  int b;              // order of block p
  int64_t oc;         // first column of block p (== o except where a panel of
                      // pivot rows is updated on its own)
  // tile subset (Schur update): 0 = every tile; 1 = the band of tile-rows
  // [tr0, tr1] and tile-columns [tc0, tc1] (the next block's rows and
  // columns); 2 = every tile outside that band.
  int region;
  int64_t tr0, tr1, tc0, tc1;
  int64_t ntiles;     // tiles enumerated by the region (before band skipping)
  // window of each XCD's tile range this launch covers: positions [w0, w1)
  // of the T8 = ceil(ntiles / 8) positions (w1 = 0: all of them)
  int64_t w0, w1;
};

// Column save fused into a Schur update: the elements of columns
// [c0, c0 + cb) are also stored transposed into p (p[(j - c0) ld + i]), the
// next block's saved column panel (p == nullptr: none).
struct ColSave {
  double* p;
  int64_t ld;
  int64_t c0;
  int cb;
};

// The next block of a fused nested sweep step (see launch_schur_leaf).
struct SchurLeafArgs {
  double* ct_next;    // q's saved column panel (qb x n, k-major)
  int64_t ldc_next;
  int64_t qo;         // q's first row/column (a multiple of 64)
  int qb;             // q's order (<= 64)
  double* p_next;     // q's leaf inverse (qb x qb, ld qb)
  int64_t row0;       // global row of W's first row (singular-row report)
  long long* info;
};

// One small matrix of a batch.
struct SmallMat {
  int64_t off;   // element offset of the matrix in A and X (row-major, ld = m)
  int32_t m;     // order
  int32_t nb;    // number of diagonal blocks
  int32_t bnd;   // blocks are [bounds[bnd + i], bounds[bnd + i + 1]), i < nb
  int32_t id;    // index of the matrix in the caller's batch (for info)
};

// One pivot block of a batch.
struct LeafJob {
  const double* A;
  int64_t lda;
  double* P;
  int64_t ldp;
  int b;
  int row0;   // first row of the block within its matrix (for info)
  int* info;  // the matrix's info word
};

// One step of one matrix of the batched sweep, done by one workgroup: the
// pivot block's inverse (leaf), the row panel, then the Schur update with the
// old column panel copied first.
struct SweptJob {
  LeafJob leaf;
  StepArgs row;
  StepArgs schur;
};


// kernels.hip
hipError_t launch_leaf_inverse(const double* A, int64_t lda, double* P, int64_t ldp, int b, int64_t row0,
                               long long* info, hipStream_t s);
hipError_t launch_col_save(const double* W, int64_t ldw, int64_t n, int64_t o, int b, double* Ct, int64_t ldc,
                           hipStream_t s);
hipError_t launch_copy2d(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                         hipStream_t s);
// The copy (S != D) or, in place (S == D), only the check: *info = -1 if any
// element of S is a NaN or an infinity.
hipError_t launch_copy2d_check(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                               long long* info, hipStream_t s);
hipError_t launch_zero_info(long long* p, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_iota_i32(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_row_panel(const double* P, int64_t ldp, const double* W, int64_t ldw, int64_t n, int64_t o, int b,
                            double* R, int64_t ldr, hipStream_t s, double* flops);
hipError_t launch_schur(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* W, int64_t ldw, int64_t n,
                        int64_t o, int b, int region, int64_t qo, int qb, hipStream_t s, double* flops,
                        int part = 0, double split = 1.0, const ColSave* cs = nullptr);
hipError_t launch_row_panel_rows(const double* P, int64_t ldp, const double* Wp, int64_t ldw, int64_t n, int64_t o,
                                 int b, double* R, int64_t ldr, hipStream_t s);
hipError_t launch_schur_rows(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* S, int64_t lds,
                             int64_t r0, int64_t h, int64_t n, int64_t o, int b, hipStream_t s);
hipError_t launch_schur_leaf(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* W, int64_t ldw,
                             const double* Win, int64_t ldwin, int64_t n, int64_t o, int b, const SchurLeafArgs& a,
                             hipStream_t s);
hipError_t launch_swept_step(const SweptJob* jobs, int64_t count, int bmax, hipStream_t s);

// block-row pivoting (kernels.hip): one level of the tournament that picks a
// strip's pivot rows (see k_tourn_node)
struct TournArgs {
  const double* T;     // the block's columns, k-major: T[col * ldt + row], rows global
  int64_t ldt;
  int64_t o, n;        // candidate rows [o, n)
  int c0, w;           // strip columns [c0, c0 + w), w <= 64
  const int32_t* used; // used[row] != 0: chosen by an earlier strip of this block
  const int32_t* in;   // merge levels: the children's picks (nin nodes x 64, -1 = none)
  int64_t nin;
  int32_t* out;        // this level's picks (nodes x 64, -1 = none)
  int32_t* chosen;     // root: chosen[c0 + t] = pick t
  int32_t* used_w;     // root: marks its picks in used
  long long* info;     // root: first exactly-zero pivot, reported as row0 + c + 1
  int64_t row0;
  int is_leaf, is_root;
};
constexpr int kTournRows = 256;   // candidate rows per node (leaf rows; 4 children x 64 picks)
constexpr int kTournArity = 4;
hipError_t launch_tourn_level(const TournArgs& a, int64_t nodes, hipStream_t s);
hipError_t launch_gather_kmajor(const double* T, int64_t ldt, int c0, int ncols, const int32_t* rows, int nrows,
                                double* S, int64_t lds, hipStream_t s);
hipError_t launch_gather_rows(const double* W, int64_t ldw, int64_t ncols, const int32_t* rows, int nrows, double* Y,
                              int64_t ldy, hipStream_t s);
hipError_t launch_moves(const int32_t* used, const int32_t* chosen, int64_t o, int b, int64_t n, int bmax,
                        int32_t* plan, int32_t* perm, double* W, int64_t ldw, double* Ct, int64_t ldc,
                        hipStream_t s);
hipError_t launch_unpermute_cols(double* W, int64_t ldw, int64_t n, const int32_t* perm, hipStream_t s);
hipError_t launch_gemm_rows(int mode, const double* A, int64_t lda, const double* B, int64_t ldb, double* W,
                            int64_t ldw, const double* Win, int64_t ldwin, const double* R, int64_t ldr, int64_t M,
                            int64_t N, int K, int64_t o, int64_t oc, int b, hipStream_t s);
constexpr int kModeRow = 0;    // W = A B with R in block p's columns
constexpr int kModeSchur = 1;  // W = Win - A B with R in block p's rows

hipError_t launch_gemm_f64(int mode, const double* A, int64_t lda, const double* B, int64_t ldb, const double* Cin,
                           int64_t ldcin, double* C, int64_t ldc, int64_t n, hipStream_t s, double* flops);
hipError_t launch_probe_residual(const double* A, int64_t lda, const double* X, int64_t ldx, int64_t n,
                                 double* work, uint64_t seed, double* part, int kParts, hipStream_t s);
// R = I - A X with an error-free split of A (by rows) and X (by columns):
// split_a and split_x hold 2 n^2 doubles each, exps 2 n ints; fresh_a = false
// reuses split_a from an earlier call with the same A.
hipError_t launch_resid_compensated(const double* A, int64_t lda, const double* X, int64_t ldx, int64_t n,
                                    double* R, double* split_a, double* split_x, int* exps, bool fresh_a,
                                    hipStream_t s, double* flops);
int split_bits(int64_t n);
constexpr int kModeResid = 2;  // C = I - A B
constexpr int kModeAdd = 3;    // C = Cin + A B

// mixed.hip
hipError_t launch_f64_to_f32(const double* S, int64_t lds, float* D, int64_t ldd, int64_t rows, int64_t cols,
                             hipStream_t s);
hipError_t launch_f32_to_f64(const float* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                             hipStream_t s);
hipError_t launch_col_save_f32(const float* W, int64_t ldw, int64_t n, int64_t o, int b, float* Ct, int64_t ldc,
                               hipStream_t s);
hipError_t launch_row_panel_f32(const float* P, int64_t ldp, const float* W, int64_t ldw, int64_t n, int64_t o, int b,
                                float* R, int64_t ldr, hipStream_t s);
hipError_t launch_schur_f32(const float* Ct, int64_t ldc, const float* R, int64_t ldr, float* W, int64_t ldw, int64_t n,
                            int64_t o, int b, hipStream_t s);
hipError_t launch_sumsq(const double* R, int64_t ldr, int64_t rows, int64_t cols, double* part, double* out,
                        hipStream_t s);
constexpr int kSumPartsHost = 1024;
hipError_t launch_sum_final(const double* part, int np, double* out, hipStream_t s);

// batched.hip
constexpr int kSmallVariants = 4;  // most launch shapes of a small tier (autotuned)
constexpr int kSmallTierCount = 6;  // register-resident tiers: orders up to 8, 16, 32, 64, 128, 192
constexpr int kSmallMaxOrder = 192; // largest order of the register-resident tiers
hipError_t launch_small_tier(int tier, const double* A, double* X, const SmallMat* mats, const int32_t* order,
                             int64_t count, const int32_t* bounds, int32_t* info, hipStream_t s);
hipError_t launch_small_tier(int tier, int variant, const double* A, double* X, const SmallMat* mats,
                             const int32_t* order, int64_t count, const int32_t* bounds, int32_t* info,
                             hipStream_t s);
void small_variant_shape(int tier, int variant, int shape[4]);
int small_variant_count(int tier);
int small_tier_limit(int tier);
// Residual (and optional Newton-Schulz refinement) of packed small matrices:
// one workgroup per listed matrix; work = 2 m^2 doubles per matrix at 2 * off
// (NULL: residual norm only); targets[id] (or `target` when NULL) per matrix.
hipError_t launch_small_refine(const double* A, double* X, const SmallMat* mats, const int32_t* order, int64_t count,
                               double* work, double target, const double* targets, int max_steps, double* rho,
                               int32_t* steps, hipStream_t s);

// levels.hip: the paper's parallel algorithm (§5) on packed small matrices,
// one workgroup per matrix.  Class c takes orders <= level_class_limit(c)
// (8, 16, 32, 45, 52, 64); a launch's dynamic LDS is lds_doubles (the
// largest a^2 + d^2 (the top-level halves' orders; m^2 where the class does
// not split) plus provisional sets of its matrices), at most
// kLevelLdsDoubles.
constexpr int kLevelClasses = 6;
constexpr size_t kLevelLdsDoubles = 19968;  // 156 KB of the CU's 160
int level_class_limit(int c);
// whether class c keeps only M_inv's top-level diagonal squares in LDS
bool level_class_split(int c);
hipError_t launch_level_class(int c, const double* A, double* X, const SmallMat* mats, const int32_t* order,
                              int64_t count, size_t lds_doubles, const int32_t* bounds, int32_t* info,
                              hipStream_t s);

// binv_api.hip: records the thread-local message returned by binv_last_error
void set_error(const std::string& msg);

// A growable device buffer, or (borrowed) a fixed slice of memory the
// library does not own, which never grows.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;
  void borrow(void* ptr, size_t n) {
    p = ptr;
    bytes = n;
    borrowed = true;
  }
  binv_status ensure(size_t want) {
    if (want <= bytes) return BINV_OK;
    if (borrowed) {
      binv::set_error("a fixed workspace slice of " + std::to_string(bytes) + " bytes cannot hold " +
                      std::to_string(want));
      return BINV_E_INVALID;
    }
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) {
        binv::set_error(std::string("hipFree: ") + hipGetErrorString(e));
        return BINV_E_HIP;
      }
    }
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      binv::set_error("hipMalloc of " + std::to_string(want) + " bytes failed");
      return BINV_E_NOMEM;
    }
    bytes = want;
    return BINV_OK;
  }
  void release() {
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
  }
};

// Workspace for one recursion level of the block sweep (two sets of panels:
// under lookahead the next block's panels are formed while the current ones
// are still being read).
struct Level {
  DevBuf ct[2];  // old column panel, k-major: b x n
  DevBuf r[2];   // row panel: b x n
  DevBuf p[2];   // pivot inverse: b x b
};

// Workspace of block-row pivoting (sized before a pivoted sweep starts).
struct PivWork {
  DevBuf T;       // bmax x n doubles: a block's columns, eliminated strip by strip to choose its pivot rows
  DevBuf used;    // n int32: rows chosen by earlier strips of the block
  DevBuf chosen;  // bmax int32: the block's pivot rows in pick order
  DevBuf lvl[2];  // tournament picks of consecutive levels: ceil(n / 256) x 64 int32 each
  DevBuf strip;   // 64 x bmax: the picked rows' strip and later columns
  DevBuf q;       // 64 x 64: inverse of the picked rows' strip block
  DevBuf g;       // 64 x bmax: that inverse times the picked rows' later columns
  DevBuf sel;     // bmax x bmax: the pivot block in pick order (inverted in place)
  DevBuf qs;      // (bmax / 64) x 64 x 64: the pivot block sweep's leaf inverses
  DevBuf cs;      // (bmax / 64) x 64 x bmax: its saved column panels
  DevBuf rj;      // 64 x n: one sub-step's row panel over the pivot rows
  DevBuf plan;    // 1 + 2 bmax int32: the row moves
  DevBuf perm;    // n int32: the original row at each position
  void release() {
    for (DevBuf* d : {&T, &used, &chosen, &lvl[0], &lvl[1], &strip, &q, &g, &sel, &qs, &cs, &rj, &plan, &perm})
      d->release();
  }
};

}  // namespace binv

// The library context (opaque to callers; see include/binv.h).
struct binv_ctx {
  int device = 0;
  int ncu = 256;  // compute units of the device
  binv::Level lv[2];
  binv::DevBuf info;  // scratch info word when the caller passes none
  binv::PivWork piv;  // block-row pivoting
  // lookahead: the trailing update runs on `gemm` (CU-masked to all but a few
  // CUs) while the next pivot inversion runs on `side` (masked to the rest)
  hipStream_t side = nullptr, gemm = nullptr;
  int side_cus = 0;  // CUs reserved for `side`; 0 if the device refused the masks
  bool cu_mask = true;  // false: lookahead on unmasked streams (a server's workers)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_gemm = nullptr;
  // autotuned launch shape of each small batched tier, by log2 of the
  // tier's matrix count (-1: not tuned yet)
  int8_t tuned_small[binv::kSmallTierCount][40];
  // mixed precision workspace
  binv::DevBuf mx_w32, mx_ct32, mx_r32, mx_p32, mx_p64a, mx_p64b, mx_res, mx_xn, mx_part;
  // compensated residual: the split parts of A and of X, and their exponents
  binv::DevBuf mx_split_a, mx_split_x, mx_exps;
  const double* split_a_of = nullptr;  // the A whose split mx_split_a holds (within one call)
  // optional per-phase event timing
  uint32_t timing_mask = 0;
  std::vector<hipEvent_t> ev_free;
  struct Pending { int phase; hipEvent_t a, b; double flops; };
  std::vector<Pending> pending;
  // binv_invert's launch sequences captured as HIP graphs (BINV_F_GRAPH),
  // keyed by the call; ws holds the workspace addresses baked into the graph
  struct GraphEntry {
    std::vector<int64_t> key;
    std::vector<const void*> ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  hipStream_t cap = nullptr;
  // out-of-core inversion (binv_invert_host): the pivot rows and the column
  // panel as copied from the host, two row slabs, and the slabs' streams
  binv::DevBuf oo_rows, oo_cols, oo_slab[2];
  hipStream_t oo_stream[2] = {nullptr, nullptr};
  hipEvent_t oo_ev[3] = {nullptr, nullptr, nullptr};
};

namespace binv {

// Brackets one top-level launch with events when its phase is being timed.
struct PhaseTimer {
  binv_ctx* c;
  int phase;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  double flops = 0.0;
  bool on() const { return a && b; }
  double* fl() { return on() ? &flops : nullptr; }
  PhaseTimer(binv_ctx* c_, int level, int phase_, hipStream_t s_) : c(c_), phase(phase_), s(s_) {
    if (level != 0 || !(c->timing_mask & (1u << phase))) return;
    a = take();
    b = take();
    if (a && b) (void)hipEventRecord(a, s);
  }
  hipEvent_t take() {
    if (!c->ev_free.empty()) {
      hipEvent_t e = c->ev_free.back();
      c->ev_free.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~PhaseTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      c->pending.push_back({phase, a, b, flops});
    } else {
      if (a) c->ev_free.push_back(a);
      if (b) c->ev_free.push_back(b);
    }
  }
};

constexpr int kLeafMax = 128;   // largest pivot block the register leaf kernel holds
constexpr int kSubBlock = 64;   // sub-block order of the nested sweep of a larger pivot block

// Device bytes a context's workspace holds (binv_api.hip).
size_t ctx_device_bytes(const binv_ctx* c);

}  // namespace binv
