// C ABI of the blockwise inversion library (declared in include/binv.h).
//
// The host side only plans and enqueues: it walks the diagonal blocks in
// order, one elimination step per block (Eq. (a) of §3 applied in place, as
// the in-place procedure of §4.2 does once its recursion is unrolled over the
// block grid), and launches the kernels of kernels.hip on the caller's
// stream.  A pivot block larger than the LDS leaf is itself inverted by the
// same block sweep on a private copy with 64-wide sub-blocks.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "binv_internal.h"

namespace {

thread_local std::string g_err = "";

binv_status fail(binv_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// Lookahead schedule of a call: BINV_F_NO_LOOKAHEAD forces it off,
// BINV_F_LOOKAHEAD on; otherwise it is used from order kLookaheadMinN up.
// Below that the serial schedule was measured as fast or faster (plain FP64,
// every block size from 128 to 512: 0.86-1.0 of the serial time's speed at
// n <= 1536, 0.98-1.06 at n = 2048, 1.01-1.16 from n = 3072).
constexpr int64_t kLookaheadMinN = 2048;
bool use_lookahead(uint32_t flags, int64_t n) {
  if (flags & BINV_F_NO_LOOKAHEAD) return false;
  if (flags & BINV_F_LOOKAHEAD) return true;
  // the pivoted sweep's selection chain does not hide under the trailing
  // update, and beside it both slow down: serial measured 2% faster at
  // n = 8192 and 16384
  if (flags & BINV_F_PIVOT) return false;
  return n >= kLookaheadMinN;
}

}  // namespace

void binv::set_error(const std::string& msg) { g_err = msg; }

size_t binv::ctx_device_bytes(const binv_ctx* c) {
  size_t t = c->info.bytes;
  for (const auto& L : c->lv)
    for (int h = 0; h < 2; ++h) t += L.ct[h].bytes + L.r[h].bytes + L.p[h].bytes;
  const binv::PivWork& P = c->piv;
  for (const binv::DevBuf* d : {&P.T, &P.used, &P.chosen, &P.lvl[0], &P.lvl[1], &P.strip, &P.q, &P.g, &P.sel, &P.qs,
                                &P.cs, &P.rj, &P.plan, &P.perm})
    t += d->bytes;
  for (const binv::DevBuf* d : {&c->mx_w32, &c->mx_ct32, &c->mx_r32, &c->mx_p32, &c->mx_p64a, &c->mx_p64b, &c->mx_res,
                                &c->mx_xn, &c->mx_part, &c->mx_split_a, &c->mx_split_x, &c->mx_exps, &c->oo_rows,
                                &c->oo_cols, &c->oo_slab[0], &c->oo_slab[1]})
    t += d->bytes;
  return t;
}

namespace {

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(BINV_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

}  // namespace

using binv::DevBuf;
using binv::Level;
using binv::PhaseTimer;

// Static device workspace of binv_invert_noalloc: the panels (saved column
// panel, row panel, pivot inverse) of its serial sweep and its info word, for
// callers that cannot allocate device memory.  Every device the library runs
// on holds one copy for the life of the process.  In host code `scratch`
// names a host-side stand-in, not device memory: the device address of each
// device's copy is looked up once (scratch_setup, called by binv_create with
// that device current) and only that address is handed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
std::string g_scratch_err[kScratchDevices];

// The device address of `device`'s copy of scratch (that device current).
void scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    (void)hipGetLastError();
    return;
  }
  g_scratch_ptr[device] = ptr;
}

void* scratch_ptr(int device, std::string& why) {
  if (device < 0 || device >= kScratchDevices) {
    why = "device index beyond the static workspace table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) why = g_scratch_err[device].empty() ? "static workspace not set up" : g_scratch_err[device];
  return g_scratch_ptr[device];
}

}  // namespace

namespace {

binv_status sweep(binv_ctx* c, int level, int64_t n, double* W, int64_t ldw, const std::vector<int32_t>& part,
                  hipStream_t s, long long* info, int64_t row0, bool lookahead, const double* src0 = nullptr,
                  int64_t ldsrc0 = 0, int p0 = 0, int p1 = -1);

// Order of the sub-blocks of the nested sweep that inverts a pivot block
// larger than one leaf (BINV_SUB_BLOCK may set 32, 64 or 128).
int sub_block() {
  static const int v = [] {
    const char* e = getenv("BINV_SUB_BLOCK");
    const int x = e ? atoi(e) : binv::kSubBlock;
    return (x == 32 || x == 64 || x == 128) ? x : binv::kSubBlock;
  }();
  return v;
}

// The sweep of a pivot block (n x n, n < 2048, read from Wpp with leading
// dimension ldwp) into P (n x n, ld n) with 64-wide sub-blocks, two launches
// per step: the fused Schur update of step p, which also inverts block p+1's
// leaf and saves its column panel, then block p+1's row panel.  Step 0 reads
// the block where it lies and writes every element of P, so no copy is made.
// The same arithmetic as sweep() on a copy; 2 k + 1 launches instead of 4 k + 1.
// keep_q / keep_c (optional): every sub-step's leaf inverse (slot p at
// keep_q + 4096 p, ld = its order) and saved column panel (slot p at
// keep_c + 64 n p, ld = n) are kept there instead of in alternating buffers,
// so that the same sub-steps can later be applied to other columns.
binv_status nested_sweep_fused(binv_ctx* c, int level, int64_t n, const double* Wpp, int64_t ldwp, double* P,
                               const std::vector<int32_t>& part, hipStream_t s, long long* info, int64_t row0,
                               double* keep_q = nullptr, double* keep_c = nullptr) {
  const int k = (int)part.size();
  if (k < 2) return fail(BINV_E_INVALID, "fused nested sweep needs two sub-blocks or more");
  Level& L = c->lv[level];
  binv_status st;
  for (int h = 0; h < 2; ++h) {
    if ((st = L.ct[h].ensure(sizeof(double) * 64 * (size_t)n)) != BINV_OK) return st;
    if ((st = L.r[h].ensure(sizeof(double) * 64 * (size_t)n)) != BINV_OK) return st;
    if ((st = L.p[h].ensure(sizeof(double) * 64 * 64)) != BINV_OK) return st;
  }
  auto pslot = [&](int p) { return keep_q ? keep_q + (size_t)4096 * p : (double*)L.p[p & 1].p; };
  auto cslot = [&](int p) { return keep_c ? keep_c + (size_t)64 * n * p : (double*)L.ct[p & 1].p; };
  std::vector<int64_t> off(k + 1, 0);
  for (int p = 0; p < k; ++p) off[p + 1] = off[p] + part[p];
  HIP_TRY(binv::launch_leaf_inverse(Wpp, ldwp, pslot(0), part[0], part[0], row0, info, s));
  HIP_TRY(binv::launch_col_save(Wpp, ldwp, n, 0, part[0], cslot(0), n, s));
  HIP_TRY(binv::launch_row_panel(pslot(0), part[0], Wpp, ldwp, n, 0, part[0], (double*)L.r[0].p, n, s, nullptr));
  for (int p = 0; p < k; ++p) {
    const int cur = p & 1;
    const double* Ct = cslot(p);
    const double* R = (const double*)L.r[cur].p;
    if (p + 1 == k) {
      HIP_TRY(binv::launch_schur(Ct, n, R, n, P, n, n, off[p], part[p], 0, 0, 0, s, nullptr));
      break;
    }
    binv::SchurLeafArgs a;
    a.ct_next = cslot(p + 1);
    a.ldc_next = n;
    a.qo = off[p + 1];
    a.qb = part[p + 1];
    a.p_next = pslot(p + 1);
    a.row0 = row0 + off[p + 1];
    a.info = info;
    const double* Win = p == 0 ? Wpp : P;
    const int64_t ldwin = p == 0 ? ldwp : n;
    HIP_TRY(binv::launch_schur_leaf(Ct, n, R, n, P, n, Win, ldwin, n, off[p], part[p], a, s));
    HIP_TRY(binv::launch_row_panel(a.p_next, a.qb, P, n, n, a.qo, a.qb, (double*)L.r[cur ^ 1].p, n, s, nullptr));
  }
  return BINV_OK;
}

binv_status invert_pivot(binv_ctx* c, int level, const double* Wpp, int64_t ldw, int b, double* P, hipStream_t s,
                         long long* info, int64_t row0) {
  if (b <= binv::kLeafMax) {
    HIP_TRY(binv::launch_leaf_inverse(Wpp, ldw, P, b, b, row0, info, s));
    return BINV_OK;
  }
  if (level + 1 >= 2) return fail(BINV_E_INVALID, "pivot block too large for the recursion depth");
  // the same sweep with 64-wide sub-blocks, into P
  std::vector<int32_t> sub;
  for (int off = 0; off < b; off += sub_block()) sub.push_back(std::min(sub_block(), b - off));
  if (sub_block() == 64 && b < 2048) return nested_sweep_fused(c, level + 1, b, Wpp, ldw, P, sub, s, info, row0);
  // generic: invert a copy in place
  HIP_TRY(binv::launch_copy2d(Wpp, ldw, P, b, b, b, s));
  return sweep(c, level + 1, b, P, b, sub, s, info, row0, false);
}

// Pivot inversion of block [o, o+b) into panel set `buf`, on stream s.
binv_status block_pivot(binv_ctx* c, int level, const double* W, int64_t ldw, int64_t o, int b, int buf,
                        hipStream_t s, long long* info, int64_t row0) {
  PhaseTimer t(c, level, BINV_PHASE_PIVOT, s);
  return invert_pivot(c, level, W + o * ldw + o, ldw, b, (double*)c->lv[level].p[buf].p, s, info, row0 + o);
}

// Column-panel save and row panel of block [o, o+b) into panel set `buf`.
// save_cols = false: the column panel was already saved by the Schur update
// that produced it.
binv_status block_panels(binv_ctx* c, int level, int64_t n, double* W, int64_t ldw, int64_t o, int b, int buf,
                         hipStream_t s, bool save_cols = true) {
  Level& L = c->lv[level];
  if (save_cols) {
    PhaseTimer t(c, level, BINV_PHASE_OTHER, s);
    HIP_TRY(binv::launch_col_save(W, ldw, n, o, b, (double*)L.ct[buf].p, n, s));
  }
  {
    PhaseTimer t(c, level, BINV_PHASE_ROW, s);
    HIP_TRY(binv::launch_row_panel((double*)L.p[buf].p, b, W, ldw, n, o, b, (double*)L.r[buf].p, n, s, t.fl()));
  }
  return BINV_OK;
}

// CUs left out of the trailing update's CU mask for the pivot chain: none by
// default (BINV_SIDE_NCU = 8..64 sets a multiple of 8).  Measured at b = 512:
// once the trailing update is enqueued ahead of the pivot chain, a mask costs
// the trailing update more than it gains the chain (n = 8192: 25.6 against
// 24.3 ms; 16384: 182.6 against 163.0 ms; 4096: 6.84 against 6.96 ms).
constexpr int kReserveCUs = 0;

// Fraction of every XCD's share of the trailing-update tiles launched on the
// trailing update's stream; the rest follows the pivot chain on the side
// stream.  0.75 with a CU mask, 1 (no tail launch) without; BINV_REST_SPLIT in
// (0, 1] overrides both.
double rest_split(bool masked) {
  static const double v = [] {
    const char* e = getenv("BINV_REST_SPLIT");
    const double x = e ? atof(e) : -1.0;
    return (x > 0.0 && x <= 1.0) ? x : -1.0;
  }();
  return v > 0.0 ? v : (masked ? 0.75 : 1.0);
}

binv_status ensure_side(binv_ctx* c) {
  if (c->side) return BINV_OK;
  const int words = (c->ncu + 31) / 32;
  std::vector<uint32_t> mg(words, 0u);
  // The driver deals a stream's CU-mask bits to the 8 XCDs in turn (bit i
  // goes to XCD i mod 8; measured: a mask whose bits all share one residue
  // mod 8 is refused, as it leaves the other XCDs without a CU for the
  // queue).  Workgroups are dealt to the XCDs round-robin too, so every XCD
  // must keep the same share of the trailing update's CUs: leaving the last
  // nres bits out of its mask reserves nres / 8 CUs on each XCD.
  // BINV_SIDE_NCU sets nres (a multiple of 8); by default there is no mask.
  static const int nres = [] {
    const char* e = getenv("BINV_SIDE_NCU");
    const int v = e ? atoi(e) : kReserveCUs;
    return (v >= 8 && v <= 64) ? v / 8 * 8 : 0;  // 0: no mask, every CU for both streams
  }();
  for (int cu = 0; cu < c->ncu - nres; ++cu) mg[cu / 32] |= 1u << (cu % 32);
  // With a mask, only the trailing update's stream is CU-masked: at the fork
  // the reserved CUs are the only free ones, so the pivot chain runs there,
  // and the rest of the trailing update that follows it on the side stream
  // takes any CU as the first part drains.  Plain streams without a mask or if
  // the device refuses it (binv_lookahead_cus then reports 0).
  c->side_cus = 0;
  if (c->cu_mask && nres > 0 && c->ncu > 2 * nres &&
      hipExtStreamCreateWithCUMask(&c->gemm, (uint32_t)words, mg.data()) == hipSuccess) {
    c->side_cus = nres;
  } else {
    if (c->gemm) (void)hipStreamDestroy(c->gemm);
    c->gemm = nullptr;
    (void)hipGetLastError();
    HIP_TRY(hipStreamCreateWithFlags(&c->gemm, hipStreamNonBlocking));
  }
  HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_gemm, hipEventDisableTiming));
  return BINV_OK;
}

// src0 (lookahead only): where the caller's out-of-place copy into W takes
// W from; block 0's pivot block is then read there, on the side stream,
// beside that copy (the caller recorded ev_fork on s before the copy).
// [p0, p1): the steps to run (p1 < 0: to the last block); W must hold the
// state after step p0 - 1.  The lookahead never reaches past p1 - 1, so a
// range ends with W holding exactly the state after step p1 - 1.
binv_status sweep(binv_ctx* c, int level, int64_t n, double* W, int64_t ldw, const std::vector<int32_t>& part,
                  hipStream_t s, long long* info, int64_t row0, bool lookahead, const double* src0,
                  int64_t ldsrc0, int p0, int p1) {
  int bmax = 0;
  for (int32_t b : part) bmax = std::max(bmax, (int)b);
  const int k = (int)part.size();
  if (p1 < 0 || p1 > k) p1 = k;
  if (p0 >= p1) return BINV_OK;
  if (p0 > 0) src0 = nullptr;
  lookahead = lookahead && level == 0 && p1 - p0 >= 2;
  Level& L = c->lv[level];
  binv_status st;
  for (int h = 0; h < (lookahead ? 2 : 1); ++h) {
    if ((st = L.ct[h].ensure(sizeof(double) * (size_t)bmax * (size_t)n)) != BINV_OK) return st;
    if ((st = L.r[h].ensure(sizeof(double) * (size_t)bmax * (size_t)n)) != BINV_OK) return st;
    if ((st = L.p[h].ensure(sizeof(double) * (size_t)bmax * (size_t)bmax)) != BINV_OK) return st;
  }
  if (lookahead && (st = ensure_side(c)) != BINV_OK) return st;
  std::vector<int64_t> off(k + 1, 0);
  for (int p = 0; p < k; ++p) off[p + 1] = off[p] + part[p];

  if (!lookahead) {
    for (int p = p0; p < p1; ++p) {
      if ((st = block_pivot(c, level, W, ldw, off[p], part[p], 0, s, info, row0)) != BINV_OK) return st;
      if ((st = block_panels(c, level, n, W, ldw, off[p], part[p], 0, s)) != BINV_OK) return st;
      PhaseTimer t(c, level, BINV_PHASE_SCHUR, s);
      HIP_TRY(binv::launch_schur((double*)L.ct[0].p, n, (double*)L.r[0].p, n, W, ldw, n, off[p], part[p], 0, 0, 0, s,
                                 t.fl(), 0));
    }
    return BINV_OK;
  }

  // Lookahead.  After block 0's panels every launch on the critical path runs
  // on the trailing update's stream g, so consecutive steps hand over nothing
  // but the pivot chain.  Step p: update block q = p+1's diagonal block; fork:
  // the trailing update on g and q's pivot inversion on the side stream, so
  // the chain is off the critical path whenever it is shorter than the
  // trailing update (its workgroups take CUs as the update's drain, or the CUs
  // a mask on g leaves free).  With split < 1 the last (1 - split) of every
  // XCD's share of the trailing-update tiles follows the chain on the side
  // stream, where it can use every CU, so reserved CUs do not idle once the
  // chain is done.  g waits for the side stream, then forms q's row panel;
  // q's column panel is saved by the launches that update it.
  const double split = rest_split(c->side_cus > 0);
  if (src0) {
    HIP_TRY(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    if ((st = block_pivot(c, level, src0, ldsrc0, off[0], part[0], 0, c->side, info, row0)) != BINV_OK) return st;
    HIP_TRY(hipEventRecord(c->ev_join, c->side));
    HIP_TRY(hipStreamWaitEvent(s, c->ev_join, 0));
  } else if ((st = block_pivot(c, level, W, ldw, off[p0], part[p0], p0 & 1, s, info, row0)) != BINV_OK) {
    return st;
  }
  if ((st = block_panels(c, level, n, W, ldw, off[p0], part[p0], p0 & 1, s)) != BINV_OK) return st;
  hipStream_t g = c->gemm;
  HIP_TRY(hipEventRecord(c->ev_fork, s));
  HIP_TRY(hipStreamWaitEvent(g, c->ev_fork, 0));
  for (int p = p0; p < p1; ++p) {
    const int cur = p & 1;
    const double* Ct = (const double*)L.ct[cur].p;
    const double* R = (const double*)L.r[cur].p;
    if (p + 1 == p1) {
      PhaseTimer t(c, level, BINV_PHASE_SCHUR, g);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 0, 0, 0, g, t.fl(), 0));
      break;
    }
    // block q's column panel is saved by the launches that update it
    const binv::ColSave cs{(double*)L.ct[cur ^ 1].p, n, off[p + 1], part[p + 1]};
    {
      // only block q's diagonal block must be current before its pivot
      // inversion starts; its row and column bands join the rest
      PhaseTimer t(c, level, BINV_PHASE_BAND, g);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 3, off[p + 1], part[p + 1], g, t.fl(), 0,
                                 1.0, &cs));
    }
    HIP_TRY(hipEventRecord(c->ev_fork, g));
    HIP_TRY(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    // the trailing update is enqueued first: enqueuing the pivot chain's
    // launches takes the host a few hundred microseconds, which the trailing
    // update would otherwise wait out
    {
      PhaseTimer t(c, level, BINV_PHASE_SCHUR, g);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 4, off[p + 1], part[p + 1], g, t.fl(),
                                 split < 1.0 ? 1 : 0, split, &cs));
    }
    if ((st = block_pivot(c, level, W, ldw, off[p + 1], part[p + 1], cur ^ 1, c->side, info, row0)) != BINV_OK)
      return st;
    if (split < 1.0) {
      PhaseTimer t(c, level, BINV_PHASE_TAIL, c->side);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 4, off[p + 1], part[p + 1], c->side,
                                 t.fl(), 2, split, &cs));
    }
    HIP_TRY(hipEventRecord(c->ev_join, c->side));
    HIP_TRY(hipStreamWaitEvent(g, c->ev_join, 0));
    if ((st = block_panels(c, level, n, W, ldw, off[p + 1], part[p + 1], cur ^ 1, g, false)) != BINV_OK) return st;
  }
  HIP_TRY(hipEventRecord(c->ev_gemm, g));
  HIP_TRY(hipStreamWaitEvent(s, c->ev_gemm, 0));
  return BINV_OK;
}

// ---------------------------------------------------------------------------
// Block-row pivoting (BINV_F_PIVOT).  Step p of the sweep becomes:
//   1. choose the b pivot rows among rows o..n-1 from the block's saved
//      columns Ct (k-major), strip by strip (tournament, then the strip
//      eliminated from the block's later columns);
//   2. gather the pivot block in pick order and sweep it with 64-wide
//      sub-blocks, keeping every sub-step's leaf inverse and column panel;
//   3. gather the pivot rows (all n columns) and apply those sub-steps to
//      them: the row panel R, with the pivot block's inverse in its p columns;
//   4. move the chosen rows to o..o+b-1 and the displaced rows to the vacated
//      positions (rows of W, entries of Ct, the row order perm);
//   5. the trailing update with Ct and R, as without pivoting.
// At the end column perm[c] of X is column c of W.
// ---------------------------------------------------------------------------
constexpr int kPivSub = 64;
constexpr int kPivMaxBlock = 2047;
constexpr int64_t kPivMaxN = 32768;

binv_status piv_ensure(binv_ctx* c, int64_t n, int bmax) {
  binv::PivWork& P = c->piv;
  const int64_t nodes = (n + binv::kTournRows - 1) / binv::kTournRows;
  const int nsub = (bmax + kPivSub - 1) / kPivSub;
  binv_status st;
  struct { binv::DevBuf* d; size_t bytes; } want[] = {
      {&P.T, sizeof(double) * (size_t)bmax * n},
      {&P.used, sizeof(int32_t) * (size_t)n},
      {&P.chosen, sizeof(int32_t) * (size_t)bmax},
      {&P.lvl[0], sizeof(int32_t) * 64 * (size_t)nodes},
      {&P.lvl[1], sizeof(int32_t) * 64 * (size_t)nodes},
      {&P.strip, sizeof(double) * 64 * (size_t)bmax},
      {&P.q, sizeof(double) * 64 * 64},
      {&P.g, sizeof(double) * 64 * (size_t)bmax},
      {&P.sel, sizeof(double) * (size_t)bmax * bmax},
      {&P.qs, sizeof(double) * 4096 * (size_t)nsub},
      {&P.cs, sizeof(double) * 64 * (size_t)bmax * nsub},
      {&P.rj, sizeof(double) * 64 * (size_t)n},
      {&P.plan, sizeof(int32_t) * (1 + 2 * (size_t)bmax)},
      {&P.perm, sizeof(int32_t) * (size_t)n},
  };
  for (auto& w : want)
    if ((st = w.d->ensure(w.bytes)) != BINV_OK) return st;
  return BINV_OK;
}

// 1. The pivot rows of block [o, o+b) from its saved columns Ct (b x n,
// k-major, ld n) into piv.chosen (and piv.used).
binv_status piv_select(binv_ctx* c, int64_t n, const double* Ct, int64_t o, int b, hipStream_t s, long long* info) {
  binv::PivWork& P = c->piv;
  double* T = (double*)P.T.p;
  int32_t* used = (int32_t*)P.used.p;
  int32_t* chosen = (int32_t*)P.chosen.p;
  HIP_TRY(binv::launch_copy2d(Ct + o, n, T + o, n, b, n - o, s));
  HIP_TRY(binv::launch_fill_i32(used + o, n - o, 0, s));
  for (int c0 = 0; c0 < b; c0 += kPivSub) {
    const int w = std::min(kPivSub, b - c0);
    int64_t nodes = (n - o + binv::kTournRows - 1) / binv::kTournRows;
    binv::TournArgs a;
    std::memset(&a, 0, sizeof(a));
    a.T = T; a.ldt = n; a.o = o; a.n = n; a.c0 = c0; a.w = w;
    a.used = used; a.in = nullptr; a.nin = 0;
    a.out = (int32_t*)P.lvl[0].p;
    a.chosen = chosen; a.used_w = used; a.info = info; a.row0 = o + c0;
    a.is_leaf = 1;
    a.is_root = nodes == 1;
    HIP_TRY(binv::launch_tourn_level(a, nodes, s));
    int cur = 0;
    while (nodes > 1) {
      const int64_t up = (nodes + binv::kTournArity - 1) / binv::kTournArity;
      a.is_leaf = 0;
      a.in = (const int32_t*)P.lvl[cur].p;
      a.nin = nodes;
      a.out = (int32_t*)P.lvl[cur ^ 1].p;
      a.is_root = up == 1;
      HIP_TRY(binv::launch_tourn_level(a, up, s));
      cur ^= 1;
      nodes = up;
    }
    const int rest = b - c0 - w;
    if (rest <= 0) continue;
    // eliminate the strip from the block's later columns of every row:
    // T[later] -= T[strip] (Q T[picked, later]), Q the picked strip block's inverse
    double* S = (double*)P.strip.p;
    double* Q = (double*)P.q.p;
    double* G = (double*)P.g.p;
    HIP_TRY(binv::launch_gather_kmajor(T, n, c0, b - c0, chosen + c0, w, S, b - c0, s));
    HIP_TRY(binv::launch_leaf_inverse(S, b - c0, Q, w, w, o + c0, info, s));
    HIP_TRY(binv::launch_gemm_rows(binv::kModeRow, Q, w, S + w, b - c0, G, rest, nullptr, 0, nullptr, 0, w, rest, w,
                                   0, 0, 0, s));
    HIP_TRY(binv::launch_gemm_rows(binv::kModeSchur, G, rest, T + (int64_t)c0 * n + o, n, T + (int64_t)(c0 + w) * n + o,
                                   n, T + (int64_t)(c0 + w) * n + o, n, nullptr, 0, rest, n - o, w, 0, 0, 0, s));
  }
  return BINV_OK;
}

// 2. The pivot block in pick order, swept with 64-wide sub-blocks into
// piv.qs / piv.cs (a single leaf when b <= 64).
binv_status piv_block_ops(binv_ctx* c, int64_t n, const double* Ct, int64_t o, int b, hipStream_t s,
                          long long* info) {
  binv::PivWork& P = c->piv;
  double* sel = (double*)P.sel.p;
  HIP_TRY(binv::launch_gather_kmajor(Ct, n, 0, b, (const int32_t*)P.chosen.p, b, sel, b, s));
  if (b <= kPivSub) {
    HIP_TRY(binv::launch_leaf_inverse(sel, b, (double*)P.qs.p, b, b, o, info, s));
    return BINV_OK;
  }
  std::vector<int32_t> sub;
  for (int off = 0; off < b; off += kPivSub) sub.push_back(std::min(kPivSub, b - off));
  return nested_sweep_fused(c, 1, b, sel, b, sel, sub, s, info, o, (double*)P.qs.p, (double*)P.cs.p);
}

// 3. R (b x n, ld n) = the pivot rows W[chosen, :] after the pivot block's
// sub-steps: R[:, o:o+b] = the block's inverse, elsewhere that inverse times
// the rows, formed by the same 64-wide row operations.
binv_status piv_row_panel(binv_ctx* c, int64_t n, const double* W, int64_t ldw, int64_t o, int b, double* R,
                          hipStream_t s) {
  binv::PivWork& P = c->piv;
  const int32_t* chosen = (const int32_t*)P.chosen.p;
  const double* qs = (const double*)P.qs.p;
  if (b <= kPivSub) {
    double* Y = (double*)P.T.p;  // free once the block's rows are chosen
    HIP_TRY(binv::launch_gather_rows(W, ldw, n, chosen, b, Y, n, s));
    HIP_TRY(binv::launch_gemm_rows(binv::kModeRow, qs, b, Y, n, R, n, nullptr, 0, qs, b, b, n, b, 0, o, b, s));
    return BINV_OK;
  }
  HIP_TRY(binv::launch_gather_rows(W, ldw, n, chosen, b, R, n, s));
  double* rj = (double*)P.rj.p;
  for (int s0 = 0, j = 0; s0 < b; s0 += kPivSub, ++j) {
    const int sb = std::min(kPivSub, b - s0);
    const double* q = qs + (size_t)4096 * j;
    const double* cj = (const double*)P.cs.p + (size_t)64 * b * j;
    HIP_TRY(binv::launch_gemm_rows(binv::kModeRow, q, sb, R + (int64_t)s0 * n, n, rj, n, nullptr, 0, q, sb, sb, n, sb,
                                   0, o + s0, sb, s));
    HIP_TRY(binv::launch_gemm_rows(binv::kModeSchur, cj, b, rj, n, R, n, R, n, rj, n, b, n, sb, s0, o + s0, sb, s));
  }
  return BINV_OK;
}

binv_status sweep_pivoted(binv_ctx* c, int64_t n, double* W, int64_t ldw, const std::vector<int32_t>& part,
                          hipStream_t s, long long* info, bool lookahead) {
  int bmax = 0;
  for (int32_t b : part) bmax = std::max(bmax, (int)b);
  const int k = (int)part.size();
  if (bmax > kPivMaxBlock || n > kPivMaxN)
    return fail(BINV_E_INVALID, "block-row pivoting needs blocks of order <= 2047 and n <= 32768");
  lookahead = lookahead && k >= 2;
  Level& L = c->lv[0];
  binv_status st;
  for (int h = 0; h < 2; ++h) {
    if ((st = L.ct[h].ensure(sizeof(double) * (size_t)bmax * (size_t)n)) != BINV_OK) return st;
    if ((st = L.r[h].ensure(sizeof(double) * (size_t)bmax * (size_t)n)) != BINV_OK) return st;
  }
  if ((st = piv_ensure(c, n, bmax)) != BINV_OK) return st;
  if (lookahead && (st = ensure_side(c)) != BINV_OK) return st;
  binv::PivWork& P = c->piv;
  int32_t* perm = (int32_t*)P.perm.p;
  std::vector<int64_t> off(k + 1, 0);
  for (int p = 0; p < k; ++p) off[p + 1] = off[p] + part[p];
  HIP_TRY(binv::launch_iota_i32(perm, n, s));

  // steps 1-4 of block p, whose columns are saved in Ct
  auto choose_and_panel = [&](int p, double* Ct, double* R, hipStream_t sc, hipStream_t sg) -> binv_status {
    binv_status e;
    {
      PhaseTimer t(c, 0, BINV_PHASE_PIVOT, sc);
      if ((e = piv_select(c, n, Ct, off[p], part[p], sc, info)) != BINV_OK) return e;
      if ((e = piv_block_ops(c, n, Ct, off[p], part[p], sc, info)) != BINV_OK) return e;
    }
    if (sc != sg) {
      HIP_TRY(hipEventRecord(c->ev_join, sc));
      HIP_TRY(hipStreamWaitEvent(sg, c->ev_join, 0));
    }
    {
      PhaseTimer t(c, 0, BINV_PHASE_ROW, sg);
      if ((e = piv_row_panel(c, n, W, ldw, off[p], part[p], R, sg)) != BINV_OK) return e;
    }
    PhaseTimer t(c, 0, BINV_PHASE_OTHER, sg);
    HIP_TRY(binv::launch_moves((const int32_t*)P.used.p, (const int32_t*)P.chosen.p, off[p], part[p], n, bmax,
                               (int32_t*)P.plan.p, perm, W, ldw, Ct, n, sg));
    return BINV_OK;
  };

  if (!lookahead) {
    double* Ct = (double*)L.ct[0].p;
    double* R = (double*)L.r[0].p;
    for (int p = 0; p < k; ++p) {
      {
        PhaseTimer t(c, 0, BINV_PHASE_OTHER, s);
        HIP_TRY(binv::launch_col_save(W, ldw, n, off[p], part[p], Ct, n, s));
      }
      if ((st = choose_and_panel(p, Ct, R, s, s)) != BINV_OK) return st;
      PhaseTimer t(c, 0, BINV_PHASE_SCHUR, s);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 0, 0, 0, s, t.fl(), 0));
    }
    PhaseTimer t(c, 0, BINV_PHASE_OTHER, s);
    HIP_TRY(binv::launch_unpermute_cols(W, ldw, n, perm, s));
    return BINV_OK;
  }

  // Lookahead: step p updates block q = p+1's whole column band first (every
  // row: q's pivot rows may come from anywhere below), saving q's columns;
  // then the rest of the trailing update on g while q's pivot rows are chosen
  // and its block swept on the side stream; g then forms q's row panel and
  // moves the rows.
  {
    PhaseTimer t(c, 0, BINV_PHASE_OTHER, s);
    HIP_TRY(binv::launch_col_save(W, ldw, n, off[0], part[0], (double*)L.ct[0].p, n, s));
  }
  if ((st = choose_and_panel(0, (double*)L.ct[0].p, (double*)L.r[0].p, s, s)) != BINV_OK) return st;
  hipStream_t g = c->gemm;
  HIP_TRY(hipEventRecord(c->ev_fork, s));
  HIP_TRY(hipStreamWaitEvent(g, c->ev_fork, 0));
  for (int p = 0; p < k; ++p) {
    const int cur = p & 1;
    double* Ct = (double*)L.ct[cur].p;
    double* R = (double*)L.r[cur].p;
    if (p + 1 == k) {
      PhaseTimer t(c, 0, BINV_PHASE_SCHUR, g);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 0, 0, 0, g, t.fl(), 0));
      break;
    }
    double* Ctq = (double*)L.ct[cur ^ 1].p;
    const binv::ColSave cs{Ctq, n, off[p + 1], part[p + 1]};
    {
      PhaseTimer t(c, 0, BINV_PHASE_BAND, g);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 5, off[p + 1], part[p + 1], g, t.fl(), 0,
                                 1.0, &cs));
    }
    HIP_TRY(hipEventRecord(c->ev_fork, g));
    HIP_TRY(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    {
      PhaseTimer t(c, 0, BINV_PHASE_SCHUR, g);
      HIP_TRY(binv::launch_schur(Ct, n, R, n, W, ldw, n, off[p], part[p], 6, off[p + 1], part[p + 1], g, t.fl(), 0));
    }
    if ((st = choose_and_panel(p + 1, Ctq, (double*)L.r[cur ^ 1].p, c->side, g)) != BINV_OK) return st;
  }
  {
    PhaseTimer t(c, 0, BINV_PHASE_OTHER, g);
    HIP_TRY(binv::launch_unpermute_cols(W, ldw, n, perm, g));
  }
  HIP_TRY(hipEventRecord(c->ev_gemm, g));
  HIP_TRY(hipStreamWaitEvent(s, c->ev_gemm, 0));
  return BINV_OK;
}

}  // namespace

extern "C" {

const char* binv_last_error(void) { return g_err.c_str(); }

const char* binv_version(void) { return "binv 0.1 (gfx950)"; }

binv_status binv_create(binv_ctx** ctx, int device) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  *ctx = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(BINV_E_INVALID, "device index out of range");
  binv_ctx* c = new (std::nothrow) binv_ctx();
  if (!c) return fail(BINV_E_NOMEM, "out of host memory");
  c->device = device;
  std::memset(c->tuned_small, -1, sizeof(c->tuned_small));
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->ncu = ncu;
  // the device address of this device's static workspace, once per device
  int prev = 0;
  if (hipGetDevice(&prev) == hipSuccess) {
    if (prev == device || hipSetDevice(device) == hipSuccess) {
      scratch_setup(device);
      if (prev != device) (void)hipSetDevice(prev);
    }
  }
  (void)hipGetLastError();
  *ctx = c;
  return BINV_OK;
}

binv_status binv_destroy(binv_ctx* ctx) {
  if (!ctx) return BINV_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  for (auto& L : ctx->lv)
    for (int h = 0; h < 2; ++h) {
      L.ct[h].release();
      L.r[h].release();
      L.p[h].release();
    }
  for (hipStream_t st : {ctx->side, ctx->gemm})
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  for (hipEvent_t e : {ctx->ev_fork, ctx->ev_join, ctx->ev_gemm})
    if (e) (void)hipEventDestroy(e);
  ctx->info.release();
  ctx->piv.release();
  for (binv::DevBuf* d : {&ctx->mx_w32, &ctx->mx_ct32, &ctx->mx_r32, &ctx->mx_p32, &ctx->mx_p64a, &ctx->mx_p64b,
                          &ctx->mx_res, &ctx->mx_xn, &ctx->mx_part, &ctx->mx_split_a, &ctx->mx_split_x,
                          &ctx->mx_exps})
    d->release();
  for (auto& p : ctx->pending) {
    (void)hipEventSynchronize(p.b);
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
  for (auto& g : ctx->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  for (binv::DevBuf* d : {&ctx->oo_rows, &ctx->oo_cols, &ctx->oo_slab[0], &ctx->oo_slab[1]}) d->release();
  for (hipStream_t st : ctx->oo_stream)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t e : ctx->oo_ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipSetDevice(prev);
  delete ctx;
  return BINV_OK;
}

binv_status binv_lookahead_cus(binv_ctx* ctx, int32_t* reserved) {
  if (!ctx || !reserved) return fail(BINV_E_INVALID, "NULL argument");
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  const binv_status st = ensure_side(ctx);
  if (prev != ctx->device) (void)hipSetDevice(prev);
  *reserved = ctx->side_cus;
  return st;
}

binv_status binv_set_timing(binv_ctx* ctx, uint32_t phase_mask) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  ctx->timing_mask = phase_mask & ((1u << BINV_NPHASE) - 1u);
  return BINV_OK;
}

binv_status binv_get_timing(binv_ctx* ctx, binv_timing* out) {
  if (!ctx || !out) return fail(BINV_E_INVALID, "NULL argument");
  binv_status st = BINV_OK;
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(p.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess && st == BINV_OK) st = fail(BINV_E_HIP, std::string("event timing: ") + hipGetErrorString(e));
    out->ms[p.phase] += ms;
    out->launches[p.phase] += 1;
    out->flops[p.phase] += p.flops;
    ctx->ev_free.push_back(p.a);
    ctx->ev_free.push_back(p.b);
  }
  ctx->pending.clear();
  return st;
}

}  // extern "C"

namespace {

binv_status parse_partition(int64_t n, const binv_opts* opts, std::vector<int32_t>& part) {
  part.clear();
  if (opts && opts->part) {
    if (opts->k <= 0) return fail(BINV_E_INVALID, "k must be positive when part is given");
    int64_t sum = 0;
    for (int32_t i = 0; i < opts->k; ++i) {
      if (opts->part[i] <= 0) return fail(BINV_E_INVALID, "non-positive block order in part");
      sum += opts->part[i];
      part.push_back(opts->part[i]);
    }
    if (sum != n) return fail(BINV_E_INVALID, "block orders do not sum to n");
  } else {
    if (opts && opts->block < 0) return fail(BINV_E_INVALID, "negative block order");
    int32_t blk = (opts && opts->block > 0) ? opts->block : 512;
    for (int64_t off = 0; off < n; off += blk) part.push_back((int32_t)std::min<int64_t>(blk, n - off));
  }
  for (int32_t b : part)
    if (b > 8192) return fail(BINV_E_INVALID, "diagonal block larger than 8192");
  return BINV_OK;
}

binv_status read_info(long long* info, hipStream_t s, long long* h) {
  HIP_TRY(hipMemcpyAsync(h, info, sizeof(*h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return BINV_OK;
}

// rho = ||I - A X||_F / sqrt(n) with the residual left in Res.  Plain: one
// FP64 GEMM.  Compensated: the error-free split of A and X (three FP64 GEMMs,
// see launch_resid_compensated), accurate to about the rounding of R itself
// rather than to u |A| |X|; A's split is reused while c->split_a_of == A.
binv_status residual_norm(binv_ctx* c, int64_t n, const double* A, int64_t lda, const double* X, int64_t ldx,
                          double* Res, hipStream_t s, double* rho, bool compensated = false) {
  if (compensated) {
    const size_t nn = (size_t)n * (size_t)n;
    binv_status st;
    if ((st = c->mx_split_a.ensure(sizeof(double) * 2 * nn)) != BINV_OK) return st;
    if ((st = c->mx_split_x.ensure(sizeof(double) * 2 * nn)) != BINV_OK) return st;
    if ((st = c->mx_exps.ensure(sizeof(int) * 2 * (size_t)n)) != BINV_OK) return st;
    const bool fresh = c->split_a_of != A;
    HIP_TRY(binv::launch_resid_compensated(A, lda, X, ldx, n, Res, (double*)c->mx_split_a.p,
                                           (double*)c->mx_split_x.p, (int*)c->mx_exps.p, fresh, s, nullptr));
    c->split_a_of = A;
  } else {
    HIP_TRY(binv::launch_gemm_f64(binv::kModeResid, A, lda, X, ldx, nullptr, 0, Res, n, n, s, nullptr));
  }
  double* part = (double*)c->mx_part.p;
  HIP_TRY(binv::launch_sumsq(Res, n, n, n, part, part + binv::kSumPartsHost, s));
  double h = 0.0;
  HIP_TRY(hipMemcpyAsync(&h, part + binv::kSumPartsHost, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *rho = std::sqrt(h / (double)n);
  return BINV_OK;
}

// rho estimated from kProbes random sign vectors z: the mean of
// ||(A X - I) z||^2 over the probes is an unbiased estimate of ||A X - I||_F^2
// with relative standard deviation at most sqrt(2 / kProbes) = 0.18 however
// the error is spread over the rows (a sample of rows is not: where a few rows
// carry most of the error it can miss them).  It costs two n x n x kProbes
// products (4 kProbes n^2 flops) instead of the full residual's 2 n^3.  Res
// (n^2 doubles) holds the probes and the products' partial slices once
// n >= kProbeMinN; below that the full residual is cheaper anyway.
constexpr int kProbes = 64;
constexpr int64_t kProbeMinN = 3 * kProbes;
constexpr uint64_t kProbeSeed = 0x243F6A8885A308D3ull;

binv_status probe_residual_norm(binv_ctx* c, int64_t n, const double* A, int64_t lda, const double* X, int64_t ldx,
                                double* Res, hipStream_t s, double* rho) {
  double* part = (double*)c->mx_part.p;
  HIP_TRY(binv::launch_probe_residual(A, lda, X, ldx, n, Res, kProbeSeed ^ (uint64_t)n, part, binv::kSumPartsHost, s));
  double h = 0.0;
  HIP_TRY(hipMemcpyAsync(&h, part + binv::kSumPartsHost, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *rho = std::sqrt(h / ((double)kProbes * (double)n));
  return BINV_OK;
}

// The blockwise sweep on an FP32 copy of A (pivot blocks inverted in FP64);
// leaves X = FP64(result).
binv_status sweep_f32(binv_ctx* c, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                      const std::vector<int32_t>& part, hipStream_t s, long long* info) {
  int bmax = 0;
  for (int32_t b : part) bmax = std::max(bmax, (int)b);
  binv_status st;
  const size_t nn = (size_t)n * (size_t)n;
  if ((st = c->mx_w32.ensure(sizeof(float) * nn)) != BINV_OK) return st;
  if ((st = c->mx_ct32.ensure(sizeof(float) * (size_t)bmax * n)) != BINV_OK) return st;
  if ((st = c->mx_r32.ensure(sizeof(float) * (size_t)bmax * n)) != BINV_OK) return st;
  if ((st = c->mx_p32.ensure(sizeof(float) * (size_t)bmax * bmax)) != BINV_OK) return st;
  if ((st = c->mx_p64a.ensure(sizeof(double) * (size_t)bmax * bmax)) != BINV_OK) return st;
  if ((st = c->mx_p64b.ensure(sizeof(double) * (size_t)bmax * bmax)) != BINV_OK) return st;
  float* W = (float*)c->mx_w32.p;
  float* Ct = (float*)c->mx_ct32.p;
  float* R = (float*)c->mx_r32.p;
  float* P32 = (float*)c->mx_p32.p;
  double* Pa = (double*)c->mx_p64a.p;
  double* Pb = (double*)c->mx_p64b.p;
  HIP_TRY(binv::launch_f64_to_f32(A, lda, W, n, n, n, s));
  int64_t o = 0;
  for (int32_t b : part) {
    HIP_TRY(binv::launch_f32_to_f64(W + o * n + o, n, Pa, b, b, b, s));
    const double* Pinv = Pb;
    {
      PhaseTimer t(c, 0, BINV_PHASE_PIVOT, s);
      if (b <= binv::kLeafMax) {
        HIP_TRY(binv::launch_leaf_inverse(Pa, b, Pb, b, b, o, info, s));
      } else {
        std::vector<int32_t> sub;
        for (int off = 0; off < b; off += sub_block()) sub.push_back(std::min(sub_block(), b - off));
        if ((st = sweep(c, 1, b, Pa, b, sub, s, info, o, false)) != BINV_OK) return st;
        Pinv = Pa;
      }
    }
    HIP_TRY(binv::launch_f64_to_f32(Pinv, b, P32, b, b, b, s));
    HIP_TRY(binv::launch_col_save_f32(W, n, n, o, b, Ct, n, s));
    {
      PhaseTimer t(c, 0, BINV_PHASE_ROW, s);
      if (t.on()) t.flops = 2.0 * b * (double)b * (double)(n - b);
      HIP_TRY(binv::launch_row_panel_f32(P32, b, W, n, n, o, b, R, n, s));
    }
    {
      PhaseTimer t(c, 0, BINV_PHASE_SCHUR, s);
      if (t.on()) t.flops = 2.0 * b * (double)(n - b) * (double)n;
      HIP_TRY(binv::launch_schur_f32(Ct, n, R, n, W, n, n, o, b, s));
    }
    o += b;
  }
  HIP_TRY(binv::launch_f32_to_f64(W, n, X, ldx, n, n, s));
  return BINV_OK;
}

}  // namespace

namespace {

// Every workspace address of a context (what a captured graph bakes in).
std::vector<const void*> workspace_addresses(const binv_ctx* c) {
  std::vector<const void*> a;
  a.push_back(c->info.p);
  for (const auto& L : c->lv)
    for (int h = 0; h < 2; ++h) {
      a.push_back(L.ct[h].p);
      a.push_back(L.r[h].p);
      a.push_back(L.p[h].p);
    }
  const binv::PivWork& P = c->piv;
  for (const binv::DevBuf* d : {&P.T, &P.used, &P.chosen, &P.lvl[0], &P.lvl[1], &P.strip, &P.q, &P.g, &P.sel, &P.qs,
                                &P.cs, &P.rj, &P.plan, &P.perm})
    a.push_back(d->p);
  return a;
}

// binv_invert's work on stream s: clear the info word, copy A into X checking
// that it is finite (in place: the check alone), then the sweep.
binv_status invert_enqueue(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                           const std::vector<int32_t>& part, uint32_t flags, hipStream_t s, long long* info) {
  const bool inplace = (A == X);
  {
    hipError_t e = binv::launch_zero_info(info, s);
    if (e != hipSuccess) return fail(BINV_E_HIP, std::string("zero info: ") + hipGetErrorString(e));
  }
  if (n == 0) return BINV_OK;
  const bool look = use_lookahead(flags, n) && part.size() >= 2;
  // out of place with the lookahead: block 0's pivot inversion reads A and
  // runs on the side stream beside the copy of A into X
  const bool early = look && !inplace && !(flags & BINV_F_PIVOT);
  binv_status st;
  if (early) {
    if ((st = ensure_side(ctx)) != BINV_OK) return st;
    hipError_t e = hipEventRecord(ctx->ev_fork, s);
    if (e != hipSuccess) return fail(BINV_E_HIP, std::string("fork: ") + hipGetErrorString(e));
  }
  {
    // the copy of A into X (out of place), checking that A is finite
    PhaseTimer t(ctx, 0, BINV_PHASE_OTHER, s);
    hipError_t e = binv::launch_copy2d_check(A, lda, X, ldx, n, n, info, s);
    if (e != hipSuccess) return fail(BINV_E_HIP, std::string("copy: ") + hipGetErrorString(e));
  }
  if (flags & BINV_F_PIVOT) return sweep_pivoted(ctx, n, X, ldx, part, s, info, use_lookahead(flags, n));
  return sweep(ctx, 0, n, X, ldx, part, s, info, 0, look, early ? A : nullptr, lda);
}

// Capture invert_enqueue's launches into a graph kept in the context (at
// most 16, the least recently used replaced).  Timing is off while capturing.
binv_status invert_capture(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                           const std::vector<int32_t>& part, uint32_t flags, long long* info,
                           const std::vector<int64_t>& key) {
  if (!ctx->cap) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
  if (ctx->graphs.size() >= 16) {
    auto old = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                [](const binv_ctx::GraphEntry& a, const binv_ctx::GraphEntry& b) { return a.used < b.used; });
    (void)hipGraphExecDestroy(old->exec);
    (void)hipGraphDestroy(old->graph);
    ctx->graphs.erase(old);
  }
  const uint32_t mask = ctx->timing_mask;
  ctx->timing_mask = 0;
  const std::vector<const void*> ws = workspace_addresses(ctx);
  HIP_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
  binv_status st = invert_enqueue(ctx, n, A, lda, X, ldx, part, flags, ctx->cap, info);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap, &g);
  ctx->timing_mask = mask;
  if (st != BINV_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(BINV_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  if (workspace_addresses(ctx) != ws) {
    (void)hipGraphDestroy(g);
    return fail(BINV_E_HIP, "the workspace grew while capturing");
  }
  binv_ctx::GraphEntry ent;
  ent.key = key;
  ent.ws = ws;
  ent.graph = g;
  hipError_t ie = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(BINV_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  }
  ent.used = ++ctx->graph_clock;
  ctx->graphs.push_back(ent);
  return BINV_OK;
}

}  // namespace

extern "C" {

binv_status binv_residual(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, const double* X, int64_t ldx,
                          uint32_t flags, void* stream, double* rho) {
  if (!ctx || !rho) return fail(BINV_E_INVALID, "ctx or rho is NULL");
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  if (flags & ~(BINV_RESID_ESTIMATE | BINV_RESID_COMPENSATED)) return fail(BINV_E_INVALID, "unknown flags");
  if ((flags & BINV_RESID_ESTIMATE) && (flags & BINV_RESID_COMPENSATED))
    return fail(BINV_E_INVALID, "the estimate has no compensated form");
  *rho = 0.0;
  if (n == 0) return BINV_OK;
  if (!A || !X) return fail(BINV_E_INVALID, "A or X is NULL");
  if (lda < n || ldx < n) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const bool estimate = (flags & BINV_RESID_ESTIMATE) && n >= kProbeMinN;
  binv_status st = ctx->mx_res.ensure(sizeof(double) * (size_t)n * (size_t)n);
  if (st == BINV_OK) st = ctx->mx_part.ensure(sizeof(double) * (binv::kSumPartsHost + 1));
  if (st == BINV_OK) {
    double* Res = (double*)ctx->mx_res.p;
    ctx->split_a_of = nullptr;
    st = estimate ? probe_residual_norm(ctx, n, A, lda, X, ldx, Res, s, rho)
                  : residual_norm(ctx, n, A, lda, X, ldx, Res, s, rho, (flags & BINV_RESID_COMPENSATED) != 0);
  }
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

binv_status binv_residual_matrix(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, const double* X,
                                 int64_t ldx, double* R, int64_t ldr, void* stream, double* rho) {
  if (!ctx || !rho) return fail(BINV_E_INVALID, "ctx or rho is NULL");
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  *rho = 0.0;
  if (n == 0) return BINV_OK;
  if (!A || !X || !R) return fail(BINV_E_INVALID, "A, X or R is NULL");
  if (lda < n || ldx < n || ldr < n) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  binv_status st = ctx->mx_res.ensure(sizeof(double) * (size_t)n * (size_t)n);
  if (st == BINV_OK) st = ctx->mx_part.ensure(sizeof(double) * (binv::kSumPartsHost + 1));
  if (st == BINV_OK) {
    ctx->split_a_of = nullptr;
    double* Res = (double*)ctx->mx_res.p;
    st = residual_norm(ctx, n, A, lda, X, ldx, Res, s, rho, true);
    if (st == BINV_OK) {
      hipError_t e = binv::launch_copy2d(Res, n, R, ldr, n, n, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = fail(BINV_E_HIP, hipGetErrorString(e));
    }
  }
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

binv_status binv_invert_mixed(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                              const binv_opts* opts, double target, int32_t max_refine, void* stream,
                              binv_info* info_out) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  if (n > 0 && (!A || !X)) return fail(BINV_E_INVALID, "A or X is NULL");
  if (n > 0 && (lda < n || ldx < n)) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  if (n > 0) {
    const char* a0 = (const char*)A;
    const char* a1 = (const char*)(A + (n - 1) * lda + n);
    const char* x0 = (const char*)X;
    const char* x1 = (const char*)(X + (n - 1) * ldx + n);
    if (a0 < x1 && x0 < a1) return fail(BINV_E_INVALID, "mixed precision needs X separate from A");
  }
  if (target <= 0) target = 1e-10;
  if (max_refine < 0) max_refine = 5;
  if (max_refine > 6) max_refine = 6;
  binv_info inf;
  std::memset(&inf, 0, sizeof(inf));
  std::vector<int32_t> part;
  binv_status st = parse_partition(n, opts, part);
  if (st != BINV_OK) return st;
  if (n == 0) {
    inf.converged = 1;
    if (info_out) *info_out = inf;
    return BINV_OK;
  }
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const size_t nn = (size_t)n * (size_t)n;
  long long hinfo = 0;
  double rho = 0.0;
  double* Res = nullptr;
  double* Xn = nullptr;
  long long* dinfo = nullptr;
  if ((st = ctx->info.ensure(sizeof(long long))) != BINV_OK) goto out;
  dinfo = (long long*)ctx->info.p;
  if ((st = ctx->mx_res.ensure(sizeof(double) * nn)) != BINV_OK) goto out;
  if ((st = ctx->mx_xn.ensure(sizeof(double) * nn)) != BINV_OK) goto out;
  if ((st = ctx->mx_part.ensure(sizeof(double) * (binv::kSumPartsHost + 1))) != BINV_OK) goto out;
  ctx->split_a_of = nullptr;  // A's split is formed afresh by this call
  Res = (double*)ctx->mx_res.p;
  Xn = (double*)ctx->mx_xn.p;
  {
    hipError_t e = binv::launch_zero_info(dinfo, s);
    if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
  }
  {
    const bool look = use_lookahead(opts ? opts->flags : 0u, n);
    const bool from64 = opts && (opts->flags & BINV_F_REFINE_FROM_FP64);
    const bool pivot = opts && (opts->flags & BINV_F_PIVOT);
    // small orders take the full residual, which is as cheap as the estimate there
    const bool sampled = opts && (opts->flags & BINV_F_SAMPLED_CHECK) && n >= kProbeMinN;
    {
      hipError_t e = binv::launch_copy2d_check(A, lda, const_cast<double*>(A), lda, n, n, dinfo, s);
      if (e == hipSuccess) e = hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
      if (hinfo < 0) { st = fail(BINV_E_INVALID, "A holds a NaN or an infinity"); goto out; }
    }
    if (from64) {
      hipError_t e = binv::launch_copy2d(A, lda, X, ldx, n, n, s);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
      if ((st = pivot ? sweep_pivoted(ctx, n, X, ldx, part, s, dinfo, look)
                      : sweep(ctx, 0, n, X, ldx, part, s, dinfo, 0, look)) != BINV_OK)
        goto out;
    } else {
      if ((st = sweep_f32(ctx, n, A, lda, X, ldx, part, s, dinfo)) != BINV_OK) goto out;
    }
    if ((st = read_info(dinfo, s, &hinfo)) != BINV_OK) goto out;
    if (hinfo != 0) { st = fail(BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(hinfo)); goto out; }
    if (sampled) {
      // accept the sweep on the estimate when it already meets the target
      double est = 0.0;
      if ((st = probe_residual_norm(ctx, n, A, lda, X, ldx, Res, s, &est)) != BINV_OK) goto out;
      if (est <= target) {
        inf.rho_steps[0] = est;
        inf.rho_count = 1;
        inf.rho = est;
        inf.sampled = 1;
        inf.converged = 1;
        goto out;
      }
    }
    if ((st = residual_norm(ctx, n, A, lda, X, ldx, Res, s, &rho, true)) != BINV_OK) goto out;
    if (!(rho < 0.5) && !from64) {
      // the FP32 sweep is too inaccurate for Newton-Schulz to converge: start
      // again from the FP64 sweep (and refine that)
      inf.fell_back = 1;
      inf.rho_steps[0] = rho;
      inf.rho_count = 1;
      hipError_t e = binv::launch_copy2d(A, lda, X, ldx, n, n, s);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
      if ((st = pivot ? sweep_pivoted(ctx, n, X, ldx, part, s, dinfo, look)
                      : sweep(ctx, 0, n, X, ldx, part, s, dinfo, 0, look)) != BINV_OK)
        goto out;
      if ((st = read_info(dinfo, s, &hinfo)) != BINV_OK) goto out;
      if (hinfo != 0) { st = fail(BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(hinfo)); goto out; }
      if ((st = residual_norm(ctx, n, A, lda, X, ldx, Res, s, &rho, true)) != BINV_OK) goto out;
    }
    int hk = inf.fell_back ? 1 : 0;  // next free slot of rho_steps
    if (hk < 8) inf.rho_steps[hk++] = rho;
    inf.rho_count = hk;
    for (int k = 0; rho > target && k < max_refine && rho < 0.5; ++k) {
      // Xn = X + X (I - A X); X takes Xn only if Xn's residual is smaller, so
      // a step that stagnates at the rounding floor (or diverges) leaves the
      // better iterate and its rho in place
      {
        PhaseTimer t(ctx, 0, BINV_PHASE_OTHER, s);
        hipError_t e = binv::launch_gemm_f64(binv::kModeAdd, X, ldx, Res, n, X, ldx, Xn, n, n, s, nullptr);
        if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
      }
      if (sampled) {
        double est = 0.0;
        if ((st = probe_residual_norm(ctx, n, A, lda, Xn, n, Res, s, &est)) != BINV_OK) goto out;
        if (est <= target) {
          hipError_t e = binv::launch_copy2d(Xn, n, X, ldx, n, n, s);
          if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
          inf.refine_steps = k + 1;
          if (hk < 8) inf.rho_steps[hk++] = est;
          inf.rho_count = hk;
          inf.rho = est;
          inf.sampled = 1;
          inf.converged = 1;
          goto out;
        }
      }
      double rho_n = 0.0;
      if ((st = residual_norm(ctx, n, A, lda, Xn, n, Res, s, &rho_n, true)) != BINV_OK) goto out;
      if (hk < 8) inf.rho_steps[hk++] = rho_n;
      inf.rho_count = hk;
      if (!(rho_n < rho)) break;  // rejected: X and rho stay
      {
        hipError_t e = binv::launch_copy2d(Xn, n, X, ldx, n, n, s);
        if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
      }
      rho = rho_n;
      inf.refine_steps = k + 1;
    }
    inf.converged = rho <= target;
    if (!inf.converged) {
      char msg[160];
      snprintf(msg, sizeof(msg), "rho %.3e above the target %.3e after %d Newton-Schulz steps", rho, target,
               inf.refine_steps);
      st = fail(BINV_E_NOCONVERGE, msg);
    }
  }
  inf.rho = rho;
out:
  if (info_out) *info_out = inf;
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

binv_status binv_invert(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                        const binv_opts* opts, void* stream, int64_t* d_info) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  if (n > 0 && (!A || !X)) return fail(BINV_E_INVALID, "A or X is NULL");
  if (n > 0 && (lda < n || ldx < n)) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  const bool inplace = (A == X);
  if (inplace && lda != ldx) return fail(BINV_E_INVALID, "in-place call needs lda == ldx");
  if (!inplace && n > 0) {
    const char* a0 = (const char*)A;
    const char* a1 = (const char*)(A + (n - 1) * lda + n);
    const char* x0 = (const char*)X;
    const char* x1 = (const char*)(X + (n - 1) * ldx + n);
    if (a0 < x1 && x0 < a1) return fail(BINV_E_INVALID, "A and X overlap without being the same matrix");
  }
  std::vector<int32_t> part;
  uint32_t flags = opts ? opts->flags : 0u;
  {
    binv_status pst = parse_partition(n, opts, part);
    if (pst != BINV_OK) return pst;
  }

  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  binv_status st = BINV_OK;
  long long* info = (long long*)d_info;
  if (!info) {
    if ((st = ctx->info.ensure(sizeof(long long))) != BINV_OK) goto out;
    info = (long long*)ctx->info.p;
  }
  if ((flags & BINV_F_GRAPH) && use_lookahead(flags, n) && part.size() >= 2) {
    // the first capture of the two-stream lookahead schedule ended the process
    // (a host-side crash during capture) and its cause is not known, so only
    // the one-stream schedule is captured
    st = fail(BINV_E_INVALID, "BINV_F_GRAPH needs the one-stream schedule (BINV_F_NO_LOOKAHEAD, or n < 2048 without BINV_F_LOOKAHEAD)");
    goto out;
  }
  if (flags & BINV_F_GRAPH) {
    // replay the call's captured launch sequence; capture it after an eager
    // run (which sizes the workspace) on first use, or when the workspace
    // moved since
    std::vector<int64_t> key = {n, lda, ldx, (int64_t)(uintptr_t)A, (int64_t)(uintptr_t)X,
                                (int64_t)(uintptr_t)info, (int64_t)(flags & ~(BINV_F_SYNC | BINV_F_GRAPH))};
    key.insert(key.end(), part.begin(), part.end());
    binv_ctx::GraphEntry* hit = nullptr;
    for (auto& g : ctx->graphs)
      if (g.key == key) hit = &g;
    if (hit && hit->ws != workspace_addresses(ctx)) {
      (void)hipGraphExecDestroy(hit->exec);
      (void)hipGraphDestroy(hit->graph);
      ctx->graphs.erase(ctx->graphs.begin() + (hit - ctx->graphs.data()));
      hit = nullptr;
    }
    if (hit) {
      hit->used = ++ctx->graph_clock;
      hipError_t e = hipGraphLaunch(hit->exec, s);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e)); goto out; }
    } else {
      if ((st = invert_enqueue(ctx, n, A, lda, X, ldx, part, flags, s, info)) != BINV_OK) goto out;
      if ((st = invert_capture(ctx, n, A, lda, X, ldx, part, flags, info, key)) != BINV_OK) goto out;
    }
  } else if ((st = invert_enqueue(ctx, n, A, lda, X, ldx, part, flags, s, info)) != BINV_OK) {
    goto out;
  }
  if (flags & BINV_F_SYNC) {
    long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, info, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("sync: ") + hipGetErrorString(e)); goto out; }
    if (h < 0) st = fail(BINV_E_INVALID, "A holds a NaN or an infinity");
    if (h > 0) st = fail(BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(h));
  }
out:
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

binv_status binv_sweep_steps(binv_ctx* ctx, int64_t n, double* W, int64_t ldw, const binv_opts* opts,
                             int32_t p_begin, int32_t p_end, void* stream, int64_t* d_info) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  if (n > 0 && !W) return fail(BINV_E_INVALID, "W is NULL");
  if (n > 0 && ldw < n) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  const uint32_t flags = opts ? opts->flags : 0u;
  if (flags & BINV_F_PIVOT)
    return fail(BINV_E_INVALID, "binv_sweep_steps does not pivot across blocks (the row order would be state)");
  std::vector<int32_t> part;
  {
    binv_status pst = parse_partition(n, opts, part);
    if (pst != BINV_OK) return pst;
  }
  const int k = (int)part.size();
  if (p_end < 0) p_end = k;
  if (p_begin < 0 || p_begin > p_end || p_end > k)
    return fail(BINV_E_INVALID, "step range outside 0 <= p_begin <= p_end <= " + std::to_string(k));
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  binv_status st = BINV_OK;
  long long* info = (long long*)d_info;
  if (!info) {
    if ((st = ctx->info.ensure(sizeof(long long))) != BINV_OK) goto out;
    info = (long long*)ctx->info.p;
  }
  if (p_begin == 0 || !d_info) {
    // the caller's word starts at step 0; the internal one at every call
    hipError_t e = binv::launch_zero_info(info, s);
    if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("zero info: ") + hipGetErrorString(e)); goto out; }
  }
  if (n > 0 && p_end > p_begin) {
    const bool look = use_lookahead(flags, n);
    if ((st = sweep(ctx, 0, n, W, ldw, part, s, info, 0, look, nullptr, 0, p_begin, p_end)) != BINV_OK) goto out;
  }
  if (flags & BINV_F_SYNC) {
    long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, info, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("sync: ") + hipGetErrorString(e)); goto out; }
    if (h > 0) st = fail(BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(h));
  }
out:
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

binv_status binv_invert_host(binv_ctx* ctx, int64_t n, double* W, int64_t ldw, const binv_opts* opts,
                             size_t device_bytes, void* stream, int64_t* singular_row) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  if (singular_row) *singular_row = 0;
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  if (n > 0 && !W) return fail(BINV_E_INVALID, "W is NULL");
  if (n > 0 && ldw < n) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  const uint32_t flags = opts ? opts->flags : 0u;
  if (flags & BINV_F_PIVOT) return fail(BINV_E_INVALID, "binv_invert_host does not pivot across blocks");
  std::vector<int32_t> part;
  {
    binv_status pst = parse_partition(n, opts, part);
    if (pst != BINV_OK) return pst;
  }
  if (n == 0) return BINV_OK;
  int bmax = 0;
  for (int32_t b : part) bmax = std::max(bmax, (int)b);
  if (bmax >= 2048) return fail(BINV_E_INVALID, "binv_invert_host needs diagonal blocks of order <= 2047");
  const size_t d = sizeof(double), nb = (size_t)bmax * (size_t)n;
  // fixed: the pivot rows, the column panel (as copied, then k-major), the
  // row panel, the pivot inverse, the nested pivot sweep's panels, info
  const size_t fixed = d * (4 * nb + (size_t)bmax * bmax + 4 * (64 * (size_t)bmax + 4096)) + 256;
  const size_t per_row = 2 * d * (size_t)n;  // one row in each of the two slabs
  if (device_bytes < fixed + per_row)
    return fail(BINV_E_INVALID, "binv_invert_host: device_bytes below the " + std::to_string(fixed + per_row) +
                                    " bytes one row slab needs for n = " + std::to_string(n));
  int64_t h = (int64_t)std::min<size_t>((device_bytes - fixed) / per_row, (size_t)n);
  if (h >= 128) h = h / 128 * 128;
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  binv_status st = BINV_OK;
  std::vector<int64_t> off(part.size() + 1, 0);
  for (size_t p = 0; p < part.size(); ++p) off[p + 1] = off[p] + part[p];
  Level& L = ctx->lv[0];
  long long hinfo = 0;
  {
    struct { binv::DevBuf* b; size_t bytes; } want[] = {
        {&ctx->oo_rows, d * nb}, {&ctx->oo_cols, d * nb}, {&L.ct[0], d * nb}, {&L.r[0], d * nb},
        {&L.p[0], d * (size_t)bmax * bmax}, {&ctx->oo_slab[0], d * (size_t)h * n}, {&ctx->oo_slab[1], d * (size_t)h * n},
        {&ctx->info, sizeof(long long)}};
    for (auto& w : want)
      if ((st = w.b->ensure(w.bytes)) != BINV_OK) goto out;
  }
  for (int i = 0; i < 2; ++i)
    if (!ctx->oo_stream[i]) {
      hipError_t e = hipStreamCreateWithFlags(&ctx->oo_stream[i], hipStreamNonBlocking);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
    }
  for (int i = 0; i < 3; ++i)
    if (!ctx->oo_ev[i]) {
      hipError_t e = hipEventCreateWithFlags(&ctx->oo_ev[i], hipEventDisableTiming);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, hipGetErrorString(e)); goto out; }
    }
  {
    long long* info = (long long*)ctx->info.p;
    double* rows = (double*)ctx->oo_rows.p;
    double* cols = (double*)ctx->oo_cols.p;
    double* Ct = (double*)L.ct[0].p;
    double* R = (double*)L.r[0].p;
    double* P = (double*)L.p[0].p;
#define OOC_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) { st = fail(BINV_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); goto out; } \
  } while (0)
    OOC_TRY(binv::launch_zero_info(info, s));
    for (size_t p = 0; p < part.size(); ++p) {
      const int64_t o = off[p];
      const int b = part[p];
      // block p's rows and its column panel, as the last step left them on the host
      OOC_TRY(hipMemcpy2DAsync(rows, d * n, W + o * ldw, d * ldw, d * n, b, hipMemcpyHostToDevice, s));
      OOC_TRY(hipMemcpy2DAsync(cols, d * b, W + o, d * ldw, d * b, n, hipMemcpyHostToDevice, s));
      OOC_TRY(binv::launch_col_save(cols, b, n, 0, b, Ct, n, s));
      if ((st = invert_pivot(ctx, 0, rows + o, n, b, P, s, info, o)) != BINV_OK) goto out;
      OOC_TRY(binv::launch_row_panel_rows(P, b, rows, n, n, o, b, R, n, s));
      // every row slab: in, trailing update (block p's rows take R), out;
      // the two slab streams alternate so copies overlap the other's update
      OOC_TRY(hipEventRecord(ctx->oo_ev[2], s));
      int64_t j = 0;
      for (int64_t r0 = 0; r0 < n; r0 += h, ++j) {
        const int64_t hr = std::min<int64_t>(h, n - r0);
        hipStream_t ss = ctx->oo_stream[j & 1];
        double* S = (double*)ctx->oo_slab[j & 1].p;
        OOC_TRY(hipStreamWaitEvent(ss, ctx->oo_ev[2], 0));
        OOC_TRY(hipMemcpy2DAsync(S, d * n, W + r0 * ldw, d * ldw, d * n, hr, hipMemcpyHostToDevice, ss));
        OOC_TRY(binv::launch_schur_rows(Ct, n, R, n, S, n, r0, hr, n, o, b, ss));
        OOC_TRY(hipMemcpy2DAsync(W + r0 * ldw, d * ldw, S, d * n, d * n, hr, hipMemcpyDeviceToHost, ss));
      }
      for (int i = 0; i < 2; ++i) {
        OOC_TRY(hipEventRecord(ctx->oo_ev[i], ctx->oo_stream[i]));
        OOC_TRY(hipStreamWaitEvent(s, ctx->oo_ev[i], 0));
      }
    }
    OOC_TRY(hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    OOC_TRY(hipStreamSynchronize(s));
#undef OOC_TRY
  }
  if (hinfo != 0) {
    if (singular_row) *singular_row = hinfo;
    st = fail(BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(hinfo));
  }
out:
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

binv_status binv_invert_noalloc(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                                const binv_opts* opts, void* stream, int64_t* d_info) {
  if (!ctx) return fail(BINV_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(BINV_E_INVALID, "n < 0");
  if (n > 0 && (!A || !X)) return fail(BINV_E_INVALID, "A or X is NULL");
  if (n > 0 && (lda < n || ldx < n)) return fail(BINV_E_INVALID, "leading dimension smaller than n");
  const bool inplace = (A == X);
  if (inplace && lda != ldx) return fail(BINV_E_INVALID, "in-place call needs lda == ldx");
  if (!inplace && n > 0) {
    const char* a0 = (const char*)A;
    const char* a1 = (const char*)(A + (n - 1) * lda + n);
    const char* x0 = (const char*)X;
    const char* x1 = (const char*)(X + (n - 1) * ldx + n);
    if (a0 < x1 && x0 < a1) return fail(BINV_E_INVALID, "A and X overlap without being the same matrix");
  }
  const uint32_t flags = opts ? opts->flags : 0u;
  if (flags & BINV_F_PIVOT) return fail(BINV_E_INVALID, "binv_invert_noalloc does not pivot across blocks");
  std::vector<int32_t> part;
  {
    binv_status pst = parse_partition(n, opts, part);
    if (pst != BINV_OK) return pst;
  }
  int bmax = 0;
  for (int32_t b : part) bmax = std::max(bmax, (int)b);
  if (bmax > 2047) return fail(BINV_E_INVALID, "binv_invert_noalloc needs diagonal blocks of order <= 2047");
  // workspace in doubles: the info word (padded to 32 doubles), the serial
  // sweep's column panel, row panel and pivot inverse, and two sets of the
  // nested pivot sweep's panels (sub-blocks of at most 128)
  const size_t nb = (size_t)bmax * (size_t)n, sub = 128 * (size_t)bmax;
  const size_t need = 32 + 2 * nb + (size_t)bmax * bmax + 4 * sub + 2 * 128 * 128;
  if (need * sizeof(double) > kScratchBytes)
    return fail(BINV_E_INVALID, "binv_invert_noalloc: n = " + std::to_string(n) + " with blocks of " +
                                    std::to_string(bmax) + " needs " + std::to_string(need * sizeof(double)) +
                                    " bytes of workspace; the static workspace holds " +
                                    std::to_string(kScratchBytes));
  std::string why;
  double* base = (double*)scratch_ptr(ctx->device, why);
  if (!base) return fail(BINV_E_HIP, "binv_invert_noalloc: " + why);

  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != ctx->device) HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  binv_status st = BINV_OK;
  long long* info = d_info ? (long long*)d_info : (long long*)base;
  {
    // a context of slices of the static workspace: the sweep's ensure() calls
    // find them large enough and never allocate; no timing, no side streams
    binv_ctx w;
    w.device = ctx->device;
    w.ncu = ctx->ncu;
    double* q = base + 32;
    auto take = [&](DevBuf& d, size_t doubles) {
      d.borrow(q, doubles * sizeof(double));
      q += doubles;
    };
    take(w.lv[0].ct[0], nb);
    take(w.lv[0].r[0], nb);
    take(w.lv[0].p[0], (size_t)bmax * bmax);
    for (int h = 0; h < 2; ++h) {
      take(w.lv[1].ct[h], sub);
      take(w.lv[1].r[h], sub);
      take(w.lv[1].p[h], 128 * 128);
    }
    hipError_t e = binv::launch_zero_info(info, s);
    if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("zero info: ") + hipGetErrorString(e)); goto out; }
    if (n > 0) {
      e = binv::launch_copy2d_check(A, lda, X, ldx, n, n, info, s);
      if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("copy: ") + hipGetErrorString(e)); goto out; }
      if ((st = sweep(&w, 0, n, X, ldx, part, s, info, 0, false)) != BINV_OK) goto out;
    }
  }
  if (flags & BINV_F_SYNC) {
    long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, info, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(BINV_E_HIP, std::string("sync: ") + hipGetErrorString(e)); goto out; }
    if (h < 0) st = fail(BINV_E_INVALID, "A holds a NaN or an infinity");
    if (h > 0) st = fail(BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(h));
  }
out:
  if (prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}

}  // extern "C"
