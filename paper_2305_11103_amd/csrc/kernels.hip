// HIP kernels (gfx950) for in-place blockwise inversion.
//
// One elimination step for diagonal block p (rows/columns [o, o+b)) of the
// working matrix W (row-major, leading dimension ldw) is, following Eq. (a)
// of §3 applied in place as in §4.2:
//
//   k_leaf_inverse   P = W_pp^-1 by Gauss-Jordan with partial pivoting inside
//                    the block, held in registers (b <= 128).
//   k_col_save       Ct = (W[:, o:o+b])^T, the old column panel, k-major.
//   k_gemm_step<ROW> R = P W[o:o+b, :] with R[:, o:o+b] = P  (row panel,
//                    "-A^-1 B" up to sign; the p columns carry P itself).
//   k_gemm_step<SCHUR>
//                    W[i, j] = (j in p ? 0 : W[i, j]) - sum_t Ct[t, i] R[t, j]
//                    for i outside p (Schur complement, assembly of the
//                    inverted region, and the column panel -W_ip P), and
//                    W[p rows, :] = R.
//
// The GEMM core uses the FP64 4x4x4 MFMA (v_mfma_f64_4x4x4_4b_f64), which on
// gfx950 sustains close to the FP64 matrix peak, unlike the 16x16x4 form.
// One instruction computes four independent 4x4 products.  Lane layout
// (measured): A lane l holds A_beta[l%4][l/16], B lane l holds
// B_beta[l/16][l%4], D lane l holds D_beta[l/16][l%4], beta = (l/4)%4.
// Feeding every beta the same A rows and 16 consecutive B columns makes one
// instruction a 4 x 16 x 4 product whose output lane l is (row l/16,
// column l%16) of that 4 x 16 tile.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <cstring>

#include "binv_internal.h"

namespace binv {

constexpr int kNT = 256;        // threads per workgroup in the GEMM and leaf kernels

// ---------------------------------------------------------------------------
// Leaf: Gauss-Jordan with partial pivoting on a b x b block held in registers.
// ---------------------------------------------------------------------------
// Layout: NWV waves; wave w owns columns [w*CPW, (w+1)*CPW); lane l owns
// rows l + 64 h (h < RPL).  Column c is eliminated in one pass:
//   - the owning wave finds the pivot (largest |value| among rows not yet used
//     as pivots, lowest row on ties), publishes it and the column of
//     multipliers through LDS (double-buffered, so one barrier per column);
//   - in every wave the pivot row is broadcast with readlane; every other row
//     does w_ij -= (f_i q) p_j with q = 1/pivot, the pivot row is scaled by q;
//     the column-c slot of the other rows becomes -f_i q and that of the
//     pivot row q.
// Rows are not physically swapped: row r_c used for column c stays where it
// is.  This is Gauss-Jordan on the row-permuted matrix B (B[c] = A[r_c]), so
// the stored result satisfies A^-1[c][r_m] = W[r_c][m], which the final store
// applies.
// A (lda): the block, read only.  P (ldp): receives the inverse.  info: set
// (first writer wins) to row0 + c + 1 when the pivot of column c is exactly
// zero; P is then undefined.
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ void record_singular(long long* info, long long row) {
  atomicCAS((unsigned long long*)info, 0ULL, (unsigned long long)row);
}
__device__ __forceinline__ void record_singular(int* info, long long row) { atomicCAS(info, 0, (int)row); }

// Pivot search of one column held as x[h] (row lane + 64 h) in every lane of
// a wave: for non-negative doubles the IEEE bit pattern orders like the value,
// so key = bits(|x|) + 1 (0 for rows already used) turns the search into one
// integer wave-max (two 32-bit DPP reductions); ties go to the lowest row.
// With `publish` the wave stores the column of multipliers and the pivot
// (row, value) into the LDS slot.
template <int RPL>
__device__ __forceinline__ void leaf_search(const double (&x)[RPL], const bool (&used)[RPL], bool publish,
                                            double* colbuf, int* s_r, double* s_pv, int lane) {
  unsigned long long key[RPL];
  unsigned long long kmax = 0;
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    key[h] = used[h] ? 0ULL : (unsigned long long)__double_as_longlong(fabs(x[h])) + 1ULL;
    kmax = key[h] > kmax ? key[h] : kmax;
  }
  const unsigned hi = __ockl_wfred_max_u32((unsigned)(kmax >> 32));
  const unsigned lo = __ockl_wfred_max_u32((unsigned)(kmax >> 32) == hi ? (unsigned)kmax : 0u);
  kmax = ((unsigned long long)hi << 32) | lo;
  int r = 64 * RPL;
#pragma unroll
  for (int h = RPL - 1; h >= 0; --h) {
    const unsigned long long mk = __ballot(key[h] == kmax);
    if (mk) r = 64 * h + __ffsll((long long)mk) - 1;
  }
  double pv = 0.0;
#pragma unroll
  for (int h = 0; h < RPL; ++h)
    if ((r >> 6) == h) pv = readlane_f64(x[h], r & 63);
  if (publish) {
#pragma unroll
    for (int h = 0; h < RPL; ++h) colbuf[lane + 64 * h] = x[h];
    if (lane == 0) {
      *s_r = r;
      *s_pv = pv;
    }
  }
}

// Rows are stored unscaled: when row r becomes the pivot of column c (value
// pv, q = 1/pv) its stored values stay, its column-c slot becomes 1 and its
// scale q.  A later update of any row subtracts (its stored multiplier) x
// (the true, scaled pivot row), which is the true update divided by that
// row's scale, so each element costs one fma per column and every row is
// rescaled once at the end.  The pivot of column c + 1 is searched as soon as
// that column has been updated for column c, before the rest of the update,
// so the search overlaps the other waves' work instead of following it.
template <int RPL, int CPW, int NWV, class InfoT>
__device__ __forceinline__ void leaf_body(const double* __restrict__ A, int64_t lda, double* __restrict__ P,
                                          int64_t ldp, int b, int64_t row0, InfoT* info) {
  constexpr int NB = NWV * CPW;  // the block is padded to NB x NB with an identity
  static_assert(NB <= 64 * RPL, "columns exceed rows");
  __shared__ double colbuf[2][64 * RPL];
  __shared__ int s_r[2];
  __shared__ double s_pv[2];
  __shared__ int piv_row[NB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cbase = wave * CPW;

  // diag(A, I) has inverse diag(A^-1, I): padding keeps the loop uniform.
  double v[RPL][CPW];
  double scale[RPL];
  bool used[RPL];
  int step_of[RPL];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int row = lane + 64 * h;
    used[h] = row >= NB;  // rows beyond the padded block never pivot
    step_of[h] = 0;
    scale[h] = 1.0;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int col = cbase + j;
      v[h][j] = (row < b && col < b) ? A[(int64_t)row * lda + col] : (row == col ? 1.0 : 0.0);
    }
  }
  {
    double x[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) x[h] = v[h][0];
    leaf_search<RPL>(x, used, wave == 0, colbuf[0], &s_r[0], &s_pv[0], lane);
  }

  // Columns b..NB-1 are identity padding: their rows hold zeros in the real
  // columns (never updated, never chosen over a real row) and eliminating
  // them would not touch the real block, so the loop stops at b (uniform).
  bool singular = false;
  for (int cw = 0; cw < NWV; ++cw) {
    if (cw * CPW >= b) break;
    const bool owner = (wave == cw);
#pragma unroll
    for (int t = 0; t < CPW; ++t) {
      const int c = cw * CPW + t;
      if (c >= b) continue;
      const int buf = c & 1;
      __syncthreads();
      const int r = s_r[buf];
      const double pv = s_pv[buf];
      if (pv == 0.0 && !singular) {
        // exactly-zero pivot: record it; the arithmetic runs on (inf/nan) and
        // the result is not stored
        if (tid == 0) record_singular(info, (long long)(row0 + c + 1));
        singular = true;
      }
      const double q = 1.0 / pv;
      // uniform: keep the pivot lane and row half in scalar registers
      const int rl = __builtin_amdgcn_readfirstlane(r & 63);
      const int rh = (RPL == 1) ? 0 : __builtin_amdgcn_readfirstlane(r >> 6);
      // the true pivot row p q (row r has scale 1: it has not pivoted yet);
      // column c's slot takes q, so the other rows' slot ends as -f q
      double sp[CPW];
      if (RPL == 1 || rh == 0) {
#pragma unroll
        for (int j = 0; j < CPW; ++j) sp[j] = readlane_f64(v[0][j], rl) * q;
      } else {
#pragma unroll
        for (int j = 0; j < CPW; ++j) sp[j] = readlane_f64(v[RPL - 1][j], rl) * q;
      }
      sp[t] = owner ? q : sp[t];
      double f[RPL];
#pragma unroll
      for (int h = 0; h < RPL; ++h) {
        const int row = lane + 64 * h;
        const bool isr = (row == r);
        f[h] = isr ? 0.0 : colbuf[buf][row];
        v[h][t] = owner ? (isr ? 1.0 : 0.0) : v[h][t];
        used[h] = used[h] || isr;
        step_of[h] = isr ? c : step_of[h];
        scale[h] = isr ? q : scale[h];
      }
      // column c + 1 first (slot s of wave (c + 1) / CPW), then its search
      const int s = (t + 1) % CPW;  // a constant once the t loop is unrolled
      const bool has_next = (c + 1 < b);
      const bool next_owner = (t + 1 < CPW) ? owner : (wave == cw + 1);
#pragma unroll
      for (int h = 0; h < RPL; ++h) v[h][s] = fma(-f[h], sp[s], v[h][s]);
      if (has_next && next_owner) {
        double x[RPL];
#pragma unroll
        for (int h = 0; h < RPL; ++h) x[h] = v[h][s];
        leaf_search<RPL>(x, used, true, colbuf[buf ^ 1], &s_r[buf ^ 1], &s_pv[buf ^ 1], lane);
      }
#pragma unroll
      for (int h = 0; h < RPL; ++h) {
#pragma unroll
        for (int j = 0; j < CPW; ++j)
          if (j != s) v[h][j] = fma(-f[h], sp[j], v[h][j]);
      }
      if (tid == 0) piv_row[c] = r;
    }
  }
  if (singular) return;
  __syncthreads();
  // A^-1[step_of(row)][piv_row[col]] = scale(row) W[row][col]
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int row = lane + 64 * h;
    if (row >= b) continue;
    double* dst = P + (int64_t)step_of[h] * ldp;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int col = cbase + j;
      if (col < b) dst[piv_row[col]] = v[h][j] * scale[h];
    }
  }
}

template <int RPL, int CPW, int NWV>
__global__ void __launch_bounds__(64 * NWV) k_leaf_inverse(const double* __restrict__ A, int64_t lda,
                                                           double* __restrict__ P, int64_t ldp, int b,
                                                           int64_t row0, long long* info) {
  // a leaf is on the pivot chain, which gates the next step
  __builtin_amdgcn_s_setprio(3);
  leaf_body<RPL, CPW, NWV>(A, lda, P, ldp, b, row0, info);
}


// ---------------------------------------------------------------------------
// Column panel save: Ct[t][i] = W[i][o + t], t < b, i < n (tiled transpose).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_col_save(const double* __restrict__ W, int64_t ldw, int64_t n,
                                                  int64_t o, int b, double* __restrict__ Ct, int64_t ldc) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;  // rows of W
  const int t0 = blockIdx.y * 32;                // columns within the panel
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int64_t i = i0 + r;
    int t = t0 + tx;
    tile[r][tx] = (i < n && t < b) ? W[i * ldw + o + t] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int t = t0 + r;
    int64_t i = i0 + tx;
    if (t < b && i < n) Ct[(int64_t)t * ldc + i] = tile[tx][r];
  }
}

// ---------------------------------------------------------------------------
// 2-D copy (out-of-place calls start from a copy of A).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_copy2d(const double* __restrict__ S, int64_t lds, double* __restrict__ D,
                                                int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t i = blockIdx.y;
  if (i >= rows) return;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < cols; j += (int64_t)gridDim.x * 256)
    D[i * ldd + j] = S[i * lds + j];
}

// Copy that also checks the input: any NaN or infinity sets *info to -1
// (unconditionally, so it wins over a singular row recorded by a pivot search
// that read the same input).
__global__ void __launch_bounds__(256) k_copy2d_check(const double* __restrict__ S, int64_t lds,
                                                      double* __restrict__ D, int64_t ldd, int64_t rows,
                                                      int64_t cols, long long* info) {
  const int64_t i = blockIdx.y;
  if (i >= rows) return;
  bool bad = false;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < cols; j += (int64_t)gridDim.x * 256) {
    const double v = S[i * lds + j];
    bad |= !isfinite(v);
    D[i * ldd + j] = v;
  }
  if (bad) atomicExch((unsigned long long*)info, (unsigned long long)-1LL);
}

// The check alone (in-place calls).
__global__ void __launch_bounds__(256) k_check_finite(const double* __restrict__ S, int64_t lds, int64_t rows,
                                                      int64_t cols, long long* info) {
  const int64_t i = blockIdx.y;
  if (i >= rows) return;
  bool bad = false;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < cols; j += (int64_t)gridDim.x * 256)
    bad |= !isfinite(S[i * lds + j]);
  if (bad) atomicExch((unsigned long long*)info, (unsigned long long)-1LL);
}

__global__ void k_zero_i64(long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void __launch_bounds__(256) k_iota_i32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = (int32_t)i;
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

// Random sign probes of the residual estimate: Z[e] = +-1 and Zn[e] = -Z[e]
// for e < count, the sign being the top bit of SplitMix64 (Steele, Lea and
// Flood, 2014) at position seed + e.
__global__ void __launch_bounds__(256) k_sign_probes(double* Z, double* Zn, int64_t count, uint64_t seed) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
    uint64_t x = seed + (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    const double v = (x >> 63) ? 1.0 : -1.0;
    Z[e] = v;
    Zn[e] = -v;
  }
}

// ---------------------------------------------------------------------------
// GEMM step kernel.
// ---------------------------------------------------------------------------
enum { MODE_ROW = 0, MODE_SCHUR = 1, MODE_RESID = 2, MODE_ADD = 3 };
// MODE_RESID: W = I - A B (refinement residual); MODE_ADD: W = Win + A B
// (refinement correction).  Both read A m-major (row-major A) and B k-major.

typedef double dbl;


// Tile order: the grid is 1-D and persistent.  Workgroups are dealt to the 8
// XCDs round-robin (workgroup g runs on XCD g % 8), so XCD x owns the
// contiguous tile range [x T8, (x+1) T8) and its workgroups stride through it.
// Inside the range tiles go in groups of GM tile-rows (column-major inside a
// group), so the workgroups resident on one XCD share row and column panels in
// that XCD's L2.  Region 1 enumerates only the band of tile-rows [tr0, tr1]
// and tile-columns [tc0, tc1]; region 2 skips that band.  A launch may cover
// a window [w0, w1) of positions inside every XCD's range (the trailing update
// split in two launches keeps each part spread over all XCDs).
template <int GM>
__host__ __device__ __forceinline__ bool tile_of(int64_t t, int64_t TM, int64_t TN, int64_t& tm, int64_t& tn, int region,
                                        int64_t tr0, int64_t tr1, int64_t tc0, int64_t tc1) {
  if (region == 1) {
    const int64_t nr = tr1 - tr0 + 1, nc = tc1 - tc0 + 1;
    const int64_t T1 = nr * TN;
    if (t < T1) {
      tm = tr0 + t / TN;
      tn = t % TN;
      return true;
    }
    const int64_t u = t - T1;
    if (u >= (TM - nr) * nc) return false;
    tn = tc0 + u % nc;
    const int64_t mi = u / nc;
    tm = (mi < tr0) ? mi : mi + nr;
    return true;
  }
  if (region == 5) {  // the tile-columns [tc0, tc1], every tile-row
    const int64_t nc = tc1 - tc0 + 1;
    if (t >= TM * nc) return false;
    tm = t / nc;
    tn = tc0 + t % nc;
    return true;
  }
  if (region == 3) {  // the diagonal tile block [tr0, tr1] x [tc0, tc1] only
    const int64_t nc = tc1 - tc0 + 1;
    if (t >= (tr1 - tr0 + 1) * nc) return false;
    tm = tr0 + t / nc;
    tn = tc0 + t % nc;
    return true;
  }
  if (t >= TM * TN) return false;
  const int64_t per_group = (int64_t)GM * TN;
  const int64_t group = t / per_group;
  const int64_t first = group * GM;
  const int64_t rows = (TM - first < GM) ? (TM - first) : GM;
  const int64_t r = t - group * per_group;
  tm = first + r % rows;
  tn = r / rows;
  if (region == 2 && ((tm >= tr0 && tm <= tr1) || (tn >= tc0 && tn <= tc1))) return false;
  if (region == 4 && tm >= tr0 && tm <= tr1 && tn >= tc0 && tn <= tc1) return false;
  if (region == 6 && tn >= tc0 && tn <= tc1) return false;
  return true;
}

// GEMM tile configuration.  NWM x NWN waves per workgroup, each owning a
// (BM/NWM) x (BN/NWN) sub-tile; K is consumed in LDS chunks of BK.
// VEC: every tile is interior, K is a multiple of BK and rows are 16-byte
// aligned, so global loads are unguarded double2 loads; otherwise loads are
// guarded element by element.
template <int BM_, int BN_, int NWM_, int NWN_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, NWM = NWM_, NWN = NWN_;
  // waves per SIMD the register budget is sized for (two workgroups per CU)
  static constexpr int WPE = (64 * NWM_ * NWN_ >= 512) ? 4 : 2;
  static constexpr int NT = 64 * NWM * NWN;
  static constexpr int BK = 16;
  static constexpr int PAD = 4;
  static constexpr int LA = BM + PAD;
  static constexpr int LB = BN + PAD;
};

typedef __attribute__((address_space(3))) void lds_void;

// Direct global -> LDS staging of one K-chunk of a 128 x 128 tile's operands
// (A k-major, B row-major, both full tiles): each wave instruction moves one
// 128-double row of the chunk, 64 lanes x 16 bytes, into its padded LDS row,
// so the chunk needs no staging registers and no LDS stores.  The transfer is
// written as inline assembly because the compiler's builtin for it makes every
// later LDS read wait for the transfer, which would serialize the prefetch
// with the multiply of the chunk before it.  The instruction writes no
// register; M0 (the LDS row address) is set one wait state ahead of it; the
// caller waits for the transfer (vmcnt) before the barrier that publishes the
// buffer, and reads the buffer only after that barrier.
template <class C>
__device__ __forceinline__ void dl_issue(double* __restrict__ an, double* __restrict__ bn, const StepArgs& g,
                                         int64_t m0, int64_t n0, int k0) {
  constexpr int NW = C::NT / 64;
  static_assert(C::BM == 128 && C::BN == 128 && C::BK % NW == 0, "one 128-double row per wave instruction");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < C::BK / NW; ++e) {
    const int kk = wave + e * NW;
    const uint32_t la = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)(an + kk * C::LA));
    const uint32_t lb = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)(bn + kk * C::LB));
    const double* pa = g.A + (int64_t)(k0 + kk) * g.lda + m0 + 2 * lane;
    const double* pb = g.B + (int64_t)(k0 + kk) * g.ldb + n0 + 2 * lane;
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(la), "v"(pa) : "memory", "m0");
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(lb), "v"(pb) : "memory", "m0");
  }
}

// One K-chunk with direct staging: start the next chunk's transfer into
// (an, bn), multiply the chunk in (as, bs), then wait for this wave's
// transfer and for the workgroup.
template <class C, int RG, int CG, int KU>
__device__ __forceinline__ void dl_chunk(const double* __restrict__ as, const double* __restrict__ bs,
                                         double* __restrict__ an, double* __restrict__ bn, const StepArgs& g,
                                         int64_t m0, int64_t n0, int k0next, bool more, double (&acc)[RG][CG]) {
  constexpr int LA = C::LA, LB = C::LB, BK = C::BK, NWN = C::NWN;
  constexpr int WM = C::BM / C::NWM, WN = C::BN / C::NWN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int lk = lane >> 4, lm = lane & 3, ln = lane & 15;
  if (more) dl_issue<C>(an, bn, g, m0, n0, k0next);
#pragma unroll KU
  for (int k4 = 0; k4 < BK / 4; ++k4) {
    double fb[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) fb[c] = bs[(k4 * 4 + lk) * LB + wn * WN + c * 16 + ln];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const double fa = as[(k4 * 4 + lk) * LA + wm * WM + r * 4 + lm];
#pragma unroll
      for (int c = 0; c < CG; ++c) acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa, fb[c], acc[r][c], 0, 0, 0);
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// One output tile (tm, tn) of a step GEMM.
// With CS (Schur update only), elements of columns [cs0, cs0 + csb) are also
// stored transposed into cs (cs[(j - cs0) ldcs + i]): the next block's saved
// column panel, written as its values are produced.
template <int MODE, class C, bool A_KMAJOR, bool VEC, bool CS = false>
__device__ __forceinline__ void gemm_tile(const StepArgs& g, int64_t tm, int64_t tn,
                                          double (&As)[2][C::BK * C::LA], double (&Bs)[2][C::BK * C::LB],
                                          double* cs = nullptr, int64_t ldcs = 0, int64_t cs0 = 0, int csb = 0) {
  constexpr int BM = C::BM, BN = C::BN, NWM = C::NWM, NWN = C::NWN, NT = C::NT, BK = C::BK;
  constexpr int LA = C::LA, LB = C::LB;
  constexpr int WM = BM / NWM, WN = BN / NWN;
  constexpr int RG = WM / 4, CG = WN / 16;  // 4x16 MFMA tiles per wave
  constexpr int A_V2 = BK * BM / 2 / NT;    // per-thread double2 loads per chunk
  constexpr int B_V2 = BK * BN / 2 / NT;
  static_assert(A_V2 * 2 * NT == BK * BM && B_V2 * 2 * NT == BK * BN, "tile/thread mismatch");
  static_assert(WM % 4 == 0 && WN % 16 == 0, "wave tile must be whole 4x16 MFMA tiles");
  // full unroll of the k4 loop hoists every fragment load; at 4 waves per SIMD
  // (<= 128 VGPRs) that spills, so the 8-wave form keeps it rolled
  constexpr int KU = (NWM * NWN >= 8) ? 1 : BK / 4;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int64_t m0 = tm * BM;
  const int64_t n0 = tn * BN;
  const int64_t o = g.o;
  const int b = g.b;

  // Does this tile need the contraction at all?
  bool need = true;
  if (MODE == MODE_RESID || MODE == MODE_ADD) {
  } else if (MODE == MODE_SCHUR) {
    if (m0 >= o && m0 + BM <= o + b) need = false;  // rows inside block p: copy of R
  } else {
    if (n0 >= g.oc && n0 + BN <= g.oc + b) need = false;  // columns inside block p: copy of P
  }

  double acc[RG][CG];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int c = 0; c < CG; ++c) acc[r][c] = 0.0;

  if (need) {
    const int K = g.K;
    const int nk = (K + BK - 1) / BK;
    // staged chunk: element pairs (x, y) of each double2 slot
    double rax[A_V2], ray[A_V2], rbx[B_V2], rby[B_V2];

    auto gload = [&](int kc) {
      const int k0 = kc * BK;
      if (VEC) {
#pragma unroll
        for (int e = 0; e < A_V2; ++e) {
          const int idx = tid + e * NT;
          double2 t;
          if (A_KMAJOR) {
            const int kk = idx / (BM / 2), mm = 2 * (idx % (BM / 2));
            t = *(const double2*)(g.A + (int64_t)(k0 + kk) * g.lda + m0 + mm);
          } else {
            const int mm = idx / (BK / 2), kk = 2 * (idx % (BK / 2));
            t = *(const double2*)(g.A + (m0 + mm) * g.lda + k0 + kk);
          }
          rax[e] = t.x;
          ray[e] = t.y;
        }
#pragma unroll
        for (int e = 0; e < B_V2; ++e) {
          const int idx = tid + e * NT;
          const int kk = idx / (BN / 2), nn = 2 * (idx % (BN / 2));
          const double2 t = *(const double2*)(g.B + (int64_t)(k0 + kk) * g.ldb + n0 + nn);
          rbx[e] = t.x;
          rby[e] = t.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < A_V2; ++e) {
          const int idx = tid + e * NT;
          int kk, mm, dk, dm;
          if (A_KMAJOR) { kk = idx / (BM / 2); mm = 2 * (idx % (BM / 2)); dk = 0; dm = 1; }
          else { mm = idx / (BK / 2); kk = 2 * (idx % (BK / 2)); dk = 1; dm = 0; }
          double x[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int64_t gm = m0 + mm + u * dm;
            const int gk = k0 + kk + u * dk;
            x[u] = (gm < g.M && gk < K) ? (A_KMAJOR ? g.A[(int64_t)gk * g.lda + gm] : g.A[gm * g.lda + gk]) : 0.0;
          }
          rax[e] = x[0];
          ray[e] = x[1];
        }
#pragma unroll
        for (int e = 0; e < B_V2; ++e) {
          const int idx = tid + e * NT;
          const int kk = idx / (BN / 2), nn = 2 * (idx % (BN / 2));
          const int gk = k0 + kk;
          double x[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int64_t gn = n0 + nn + u;
            x[u] = (gn < g.N && gk < K) ? g.B[(int64_t)gk * g.ldb + gn] : 0.0;
          }
          rbx[e] = x[0];
          rby[e] = x[1];
        }
      }
    };
    auto sstore = [&](int buf) {
#pragma unroll
      for (int e = 0; e < A_V2; ++e) {
        const int idx = tid + e * NT;
        if (A_KMAJOR) {
          const int kk = idx / (BM / 2), mm = 2 * (idx % (BM / 2));
          *(double2*)&As[buf][kk * LA + mm] = make_double2(rax[e], ray[e]);
        } else {
          const int mm = idx / (BK / 2), kk = 2 * (idx % (BK / 2));
          As[buf][kk * LA + mm] = rax[e];
          As[buf][(kk + 1) * LA + mm] = ray[e];
        }
      }
#pragma unroll
      for (int e = 0; e < B_V2; ++e) {
        const int idx = tid + e * NT;
        const int kk = idx / (BN / 2), nn = 2 * (idx % (BN / 2));
        *(double2*)&Bs[buf][kk * LB + nn] = make_double2(rbx[e], rby[e]);
      }
    };

    const int lk = lane >> 4;       // k row this lane feeds
    const int lm = lane & 3;        // A row within a 4-row group
    const int ln = lane & 15;       // B column within a 16-column group
    // the trailing update's 128 x 128 full tiles stage their operands
    // directly into LDS; the other shapes go through registers
    constexpr bool DL = VEC && A_KMAJOR && BM == 128 && BN == 128 && NT == 512;
    if constexpr (DL) {
      dl_issue<C>(&As[0][0], &Bs[0][0], g, m0, n0, 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      int kc = 0;
      for (; kc + 1 < nk; kc += 2) {
        dl_chunk<C, RG, CG, KU>(&As[0][0], &Bs[0][0], &As[1][0], &Bs[1][0], g, m0, n0, (kc + 1) * BK, true, acc);
        dl_chunk<C, RG, CG, KU>(&As[1][0], &Bs[1][0], &As[0][0], &Bs[0][0], g, m0, n0, (kc + 2) * BK, kc + 2 < nk,
                                acc);
      }
      if (kc < nk) dl_chunk<C, RG, CG, KU>(&As[0][0], &Bs[0][0], &As[1][0], &Bs[1][0], g, m0, n0, 0, false, acc);
    } else {
      gload(0);
      sstore(0);
      __syncthreads();
      for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) gload(kc + 1);
        const double* as = &As[buf][0];
        const double* bs = &Bs[buf][0];
#pragma unroll KU
        for (int k4 = 0; k4 < BK / 4; ++k4) {
          double fb[CG];
#pragma unroll
          for (int c = 0; c < CG; ++c) fb[c] = bs[(k4 * 4 + lk) * LB + wn * WN + c * 16 + ln];
#pragma unroll
          for (int r = 0; r < RG; ++r) {
            const double fa = as[(k4 * 4 + lk) * LA + wm * WM + r * 4 + lm];
#pragma unroll
            for (int c = 0; c < CG; ++c)
              acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa, fb[c], acc[r][c], 0, 0, 0);
          }
        }
        if (kc + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
      }
    }
  }

  // epilogue: acc[r][c] in lane l is row wm*WM + 4r + l/16, column wn*WN + 16c + l%16
  const int er = lane >> 4;
  const int ec = lane & 15;
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    const int64_t i = m0 + wm * WM + r * 4 + er;
    if (i >= g.M) continue;
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      const int64_t j = n0 + wn * WN + c * 16 + ec;
      if (j >= g.N) continue;
      const bool jp = (j >= g.oc && j < g.oc + b);
      if (MODE == MODE_RESID) {
        g.W[i * g.ldw + j] = (i == j ? 1.0 : 0.0) - acc[r][c];
      } else if (MODE == MODE_ADD) {
        g.W[i * g.ldw + j] = g.Win[i * g.ldwin + j] + acc[r][c];
      } else if (MODE == MODE_ROW) {
        // R[i][j] = P[i][j - o] for the block's own columns, else (P W_p)[i][j]
        g.W[i * g.ldw + j] = jp ? g.R[i * g.ldr + (j - g.oc)] : acc[r][c];
      } else {
        const bool ip = (i >= o && i < o + b);
        double val;
        if (ip) {
          val = g.R[(i - o) * g.ldr + j];
        } else {
          const double w = jp ? 0.0 : g.Win[i * g.ldwin + j];
          val = w - acc[r][c];
        }
        g.W[i * g.ldw + j] = val;
        if (CS && j >= cs0 && j < cs0 + csb) cs[(j - cs0) * ldcs + i] = val;
      }
    }
  }
}

template <int MODE, class C, bool A_KMAJOR, bool VEC, bool CS>
__global__ void __launch_bounds__(C::NT)
__attribute__((amdgpu_waves_per_eu(C::WPE, C::WPE))) k_gemm_step(StepArgs g, ColSave cs) {
  __shared__ double As[2][C::BK * C::LA];
  __shared__ double Bs[2][C::BK * C::LB];
  const int64_t TM = (g.M + C::BM - 1) / C::BM, TN = (g.N + C::BN - 1) / C::BN;
  const int64_t T8 = (g.ntiles + 7) / 8;
  const int64_t w0 = g.w1 ? g.w0 : 0, w1 = g.w1 ? g.w1 : T8;
  const int64_t xcd = blockIdx.x & 7, per = (int64_t)gridDim.x >> 3;
  for (int64_t tl = w0 + ((int64_t)blockIdx.x >> 3); tl < w1; tl += per) {
    int64_t tm, tn;
    if (!tile_of<8>(xcd * T8 + tl, TM, TN, tm, tn, g.region, g.tr0, g.tr1, g.tc0, g.tc1)) continue;
    gemm_tile<MODE, C, A_KMAJOR, VEC, CS>(g, tm, tn, As, Bs, cs.p, cs.ld, cs.c0, cs.cb);
  }
}

// One step of a pivot block's nested sweep with 64-wide sub-blocks, fused:
// the Schur update of step p on 64 x 64 tiles, where workgroup 0 updates the
// next block q's diagonal tile first and then inverts it (the leaf of step q)
// while the other workgroups update the remaining tiles, and every tile of
// block q's columns also stores its values into q's saved column panel.  The
// arithmetic is that of the separate Schur, leaf and column-save launches, in
// one launch instead of three, with the leaf overlapping the update.
template <bool VEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_schur_leaf(StepArgs g, SchurLeafArgs a) {
  // the nested sweep is the pivot chain that runs beside the trailing update
  // and gates the next step: its waves issue ahead of the update's on shared
  // CUs (a wave priority, not a stream priority)
  __builtin_amdgcn_s_setprio(3);
  using C = TileCfg<64, 64, 2, 2>;
  static_assert(C::NT == 256, "the leaf runs on the tile's 4 waves");
  __shared__ double As[2][C::BK * C::LA];
  __shared__ double Bs[2][C::BK * C::LB];
  const int64_t TM = (g.M + C::BM - 1) / C::BM, TN = (g.N + C::BN - 1) / C::BN;
  const int64_t tq = a.qo / C::BM;
  if (blockIdx.x == 0) {
    gemm_tile<MODE_SCHUR, C, true, VEC, true>(g, tq, tq, As, Bs, a.ct_next, a.ldc_next, a.qo, a.qb);
    __syncthreads();  // the tile's stores are visible to the whole workgroup
    leaf_body<1, 16, 4>(g.W + a.qo * g.ldw + a.qo, g.ldw, a.p_next, a.qb, a.qb, a.row0, a.info);
    return;
  }
  const int64_t skip = tq * TN + tq;
  for (int64_t t = (int64_t)blockIdx.x - 1; t < TM * TN - 1; t += (int64_t)gridDim.x - 1) {
    const int64_t u = t >= skip ? t + 1 : t;
    gemm_tile<MODE_SCHUR, C, true, VEC, true>(g, u / TN, u % TN, As, Bs, a.ct_next, a.ldc_next, a.qo, a.qb);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI implementation).
// ---------------------------------------------------------------------------
hipError_t launch_leaf_inverse(const double* A, int64_t lda, double* P, int64_t ldp, int b, int64_t row0,
                               long long* info, hipStream_t s) {
  if (b <= 8)
    hipLaunchKernelGGL((k_leaf_inverse<1, 2, 4>), dim3(1), dim3(256), 0, s, A, lda, P, ldp, b, row0, info);
  else if (b <= 16)
    hipLaunchKernelGGL((k_leaf_inverse<1, 4, 4>), dim3(1), dim3(256), 0, s, A, lda, P, ldp, b, row0, info);
  else if (b <= 32)
    hipLaunchKernelGGL((k_leaf_inverse<1, 8, 4>), dim3(1), dim3(256), 0, s, A, lda, P, ldp, b, row0, info);
  else if (b <= 64)
    hipLaunchKernelGGL((k_leaf_inverse<1, 16, 4>), dim3(1), dim3(256), 0, s, A, lda, P, ldp, b, row0, info);
  else
    hipLaunchKernelGGL((k_leaf_inverse<2, 16, 8>), dim3(1), dim3(512), 0, s, A, lda, P, ldp, b, row0, info);
  return hipGetLastError();
}

hipError_t launch_col_save(const double* W, int64_t ldw, int64_t n, int64_t o, int b, double* Ct, int64_t ldc,
                           hipStream_t s) {
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((b + 31) / 32));
  hipLaunchKernelGGL(k_col_save, grid, dim3(256), 0, s, W, ldw, n, o, b, Ct, ldc);
  return hipGetLastError();
}

hipError_t launch_copy2d(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                         hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  unsigned gx = (unsigned)((cols + 255) / 256);
  if (gx > 64) gx = 64;
  dim3 grid(gx, (unsigned)rows);
  hipLaunchKernelGGL(k_copy2d, grid, dim3(256), 0, s, S, lds, D, ldd, rows, cols);
  return hipGetLastError();
}

hipError_t launch_copy2d_check(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                               long long* info, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  unsigned gx = (unsigned)((cols + 255) / 256);
  if (gx > 64) gx = 64;
  dim3 grid(gx, (unsigned)rows);
  if (S == D && lds == ldd) {
    hipLaunchKernelGGL(k_check_finite, grid, dim3(256), 0, s, S, lds, rows, cols, info);
  } else {
    hipLaunchKernelGGL(k_copy2d_check, grid, dim3(256), 0, s, S, lds, D, ldd, rows, cols, info);
  }
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_iota_i32, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_info(long long* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

// Algorithmic flops of one step launch: 2 K per output element that needs the
// contraction (rows of block p are copies in the Schur update, columns of
// block p copies in the row panel), over the tiles the launch covers (the
// region, and the window of every XCD's range when g.w1 > 0).
template <int BM, int BN>
static double step_flops(const StepArgs& g, int mode) {
  const int64_t TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
  auto tile_elems = [&](int64_t tm, int64_t tn) {
    const int64_t r0 = tm * BM, r1 = (r0 + BM < g.M) ? r0 + BM : g.M;
    int64_t rows = r1 - r0;
    if (mode == MODE_SCHUR) {
      const int64_t a = (r0 > g.o) ? r0 : g.o, z = (r1 < g.o + g.b) ? r1 : g.o + g.b;
      if (z > a) rows -= z - a;
    }
    const int64_t c0 = tn * BN, c1 = (c0 + BN < g.N) ? c0 + BN : g.N;
    int64_t cols = c1 - c0;
    if (mode == MODE_ROW) {
      const int64_t a = (c0 > g.oc) ? c0 : g.oc, z = (c1 < g.oc + g.b) ? c1 : g.oc + g.b;
      if (z > a) cols -= z - a;
    }
    return (double)rows * (double)cols;
  };
  double cnt = 0;
  const int64_t T8 = (g.ntiles + 7) / 8;
  const int64_t w0 = g.w1 ? g.w0 : 0, w1 = g.w1 ? g.w1 : T8;
  for (int64_t x = 0; x < 8; ++x)
    for (int64_t tl = w0; tl < w1; ++tl) {
      int64_t tm, tn;
      if (tile_of<8>(x * T8 + tl, TM, TN, tm, tn, g.region, g.tr0, g.tr1, g.tc0, g.tc1)) cnt += tile_elems(tm, tn);
    }
  return 2.0 * g.K * cnt;
}

// part 0: every tile of the region; part 1 / part 2: the first `split` / the
// remaining 1 - `split` of the positions of every XCD's tile range.
template <int MODE, int BM, int BN, bool AK, int NWM = 2, int NWN = 2>
static hipError_t launch_step(StepArgs g, hipStream_t s, int region, int64_t qo, int qb, double* flops,
                              int part = 0, double split = 1.0, const ColSave* cs = nullptr) {
  using C = TileCfg<BM, BN, NWM, NWN>;
  constexpr int BK = C::BK;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int64_t TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
  g.region = region;
  g.tr0 = g.tr1 = g.tc0 = g.tc1 = -1;
  int64_t T = TM * TN;
  if (region != 0) {
    g.tr0 = qo / BM;
    g.tr1 = (qo + qb - 1) / BM;
    g.tc0 = qo / BN;
    g.tc1 = (qo + qb - 1) / BN;
    if (region == 1) T = (g.tr1 - g.tr0 + 1) * TN + (TM - (g.tr1 - g.tr0 + 1)) * (g.tc1 - g.tc0 + 1);
    if (region == 3) T = (g.tr1 - g.tr0 + 1) * (g.tc1 - g.tc0 + 1);
    if (region == 5) T = TM * (g.tc1 - g.tc0 + 1);
  }
  g.ntiles = T;
  const int64_t T8 = (T + 7) / 8;
  g.w0 = 0;
  g.w1 = 0;
  if (part != 0) {
    int64_t w = (int64_t)(split * (double)T8 + 0.5);
    w = w < 0 ? 0 : (w > T8 ? T8 : w);
    g.w0 = part == 1 ? 0 : w;
    g.w1 = part == 1 ? w : T8;
    if (g.w1 <= g.w0) {
      if (flops) *flops = 0.0;
      return hipSuccess;  // an empty part
    }
  }
  if (flops) *flops = step_flops<BM, BN>(g, MODE);
  int64_t G = 8 * (g.w1 ? g.w1 - g.w0 : T8);  // multiple of 8 for the XCD-aware tile order
  if (G < 8) G = 8;
  const bool vec = (g.M % BM == 0) && (g.N % BN == 0) && (g.K % BK == 0) && ((g.lda & 1) == 0) &&
                   ((g.ldb & 1) == 0) && ((((uintptr_t)g.A) & 15) == 0) && ((((uintptr_t)g.B) & 15) == 0);
  const ColSave none{nullptr, 0, 0, 0};
  if constexpr (MODE == MODE_SCHUR) {
    if (cs && cs->p) {
      if (vec)
        hipLaunchKernelGGL((k_gemm_step<MODE, C, AK, true, true>), dim3((unsigned)G), dim3(C::NT), 0, s, g, *cs);
      else
        hipLaunchKernelGGL((k_gemm_step<MODE, C, AK, false, true>), dim3((unsigned)G), dim3(C::NT), 0, s, g, *cs);
      return hipGetLastError();
    }
  }
  if (vec) {
    hipLaunchKernelGGL((k_gemm_step<MODE, C, AK, true, false>), dim3((unsigned)G), dim3(C::NT), 0, s, g, none);
  } else {
    hipLaunchKernelGGL((k_gemm_step<MODE, C, AK, false, false>), dim3((unsigned)G), dim3(C::NT), 0, s, g, none);
  }
  return hipGetLastError();
}

// Row panel: R (b x n, ldr) = P (b x b, m-major, ldp) * W[o:o+b, :], with R[:, o:o+b] = P.
hipError_t launch_row_panel(const double* P, int64_t ldp, const double* W, int64_t ldw, int64_t n, int64_t o, int b,
                            double* R, int64_t ldr, hipStream_t s, double* flops) {
  StepArgs g;
  g.A = P; g.lda = ldp;
  g.B = W + o * ldw; g.ldb = ldw;
  g.W = R; g.ldw = ldr;
  g.Win = nullptr; g.ldwin = 0;
  g.R = P; g.ldr = ldp;
  g.M = b; g.N = n; g.K = b; g.o = o; g.b = b; g.oc = o;
  // wide panels: 64 x 128 tiles on 8 waves (measured at n = 8192, b = 512:
  // 90 us per panel against 100 for 64 x 64, 95 for 128 x 64, 100 for 128 x 128)
  if (b >= 128 && n >= 2048) return launch_step<MODE_ROW, 64, 128, false, 2, 4>(g, s, 0, 0, 0, flops);
  return launch_step<MODE_ROW, 64, 64, false>(g, s, 0, 0, 0, flops);
}

// Schur trailing update in place on W using the saved column panel Ct (b x n,
// k-major) and the row panel R (b x n).  region 0: all tiles; 1: only the
// tile band covering rows/columns [qo, qo+qb) of the next block; 2: the rest;
// 3: only the tiles of the next block's diagonal block (rows and columns
// [qo, qo+qb)); 4: every tile but those; 5: the tile-columns covering the
// next block's columns, every row; 6: every tile but those.  part 1 / 2 with `split`: the first
// `split` / the rest of every XCD's share of the region's tiles.  cs: the
// next block's column panel saved as its elements are updated.
int schur_tile(int64_t n) { return n >= 2048 ? 128 : 64; }

hipError_t launch_schur(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* W, int64_t ldw, int64_t n,
                        int64_t o, int b, int region, int64_t qo, int qb, hipStream_t s, double* flops, int part,
                        double split, const ColSave* cs) {
  StepArgs g;
  g.A = Ct; g.lda = ldc;
  g.B = R; g.ldb = ldr;
  g.W = W; g.ldw = ldw;
  g.Win = W; g.ldwin = ldw;
  g.R = R; g.ldr = ldr;
  g.M = n; g.N = n; g.K = b; g.o = o; g.b = b; g.oc = o;
  if (region == 3) {
    // the next block's diagonal tiles of the trailing-update grid, updated
    // with 32 x 32 tiles (a 512-block gives 256 workgroups, one per CU, for
    // this short launch on the critical path) over exactly the element range
    // those grid tiles cover
    const int64_t tile = schur_tile(n);
    const int64_t a0 = qo / tile * tile;
    const int64_t a1 = std::min<int64_t>(n, ((qo + qb - 1) / tile + 1) * tile);
    return launch_step<MODE_SCHUR, 32, 32, true>(g, s, 3, a0, (int)(a1 - a0), flops, 0, 1.0, cs);
  }
  if (region == 5) {
    // the next block's whole column band (every row), before its pivot rows
    // are chosen: 64 x 64 tiles over exactly the columns the trailing-update
    // grid's tile-columns covering it span
    const int64_t tile = schur_tile(n);
    const int64_t a0 = qo / tile * tile;
    const int64_t a1 = std::min<int64_t>(n, ((qo + qb - 1) / tile + 1) * tile);
    return launch_step<MODE_SCHUR, 64, 64, true>(g, s, 5, a0, (int)(a1 - a0), flops, 0, 1.0, cs);
  }
  if (schur_tile(n) == 128)
    return launch_step<MODE_SCHUR, 128, 128, true, 4, 2>(g, s, region, qo, qb, flops, part, split, cs);
  return launch_step<MODE_SCHUR, 64, 64, true>(g, s, region, qo, qb, flops, part, split, cs);
}

// The row panel from the pivot rows held on their own (Wp: b x n, ld ldw):
// launch_row_panel's launch with its operand B at Wp instead of W + o ldw.
hipError_t launch_row_panel_rows(const double* P, int64_t ldp, const double* Wp, int64_t ldw, int64_t n, int64_t o,
                                 int b, double* R, int64_t ldr, hipStream_t s) {
  StepArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = P; g.lda = ldp;
  g.B = Wp; g.ldb = ldw;
  g.W = R; g.ldw = ldr;
  g.R = P; g.ldr = ldp;
  g.M = b; g.N = n; g.K = b; g.o = o; g.b = b; g.oc = o;
  if (b >= 128 && n >= 2048) return launch_step<MODE_ROW, 64, 128, false, 2, 4>(g, s, 0, 0, 0, nullptr);
  return launch_step<MODE_ROW, 64, 64, false>(g, s, 0, 0, 0, nullptr);
}

// The trailing update of rows [r0, r0 + h) held on their own (S: h x n, ld
// lds, in place), with the block's saved column panel Ct (b x n, k-major, ld
// ldc, global rows) and row panel R: rows of block p among them take R.
hipError_t launch_schur_rows(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* S, int64_t lds,
                             int64_t r0, int64_t h, int64_t n, int64_t o, int b, hipStream_t s) {
  StepArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = Ct + r0; g.lda = ldc;
  g.B = R; g.ldb = ldr;
  g.W = S; g.ldw = lds;
  g.Win = S; g.ldwin = lds;
  g.R = R; g.ldr = ldr;
  g.M = h; g.N = n; g.K = b; g.o = o - r0; g.b = b; g.oc = o;
  if (schur_tile(n) == 128) return launch_step<MODE_SCHUR, 128, 128, true, 4, 2>(g, s, 0, 0, 0, nullptr);
  return launch_step<MODE_SCHUR, 64, 64, true>(g, s, 0, 0, 0, nullptr);
}

// The fused nested step: Schur update of step p (block [o, o+b)) of Win
// (ld ldwin) into W (ld ldw; Win == W in place), n x n with n < 2048, with
// the leaf of block q = [qo, qo+qb) (qo a multiple of 64, qb <= 64) into
// p_next (ld qb) and q's column panel into ct_next.  Every element of W is
// written, so the first step can read the pivot block where it lies and write
// the working copy.
hipError_t launch_schur_leaf(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* W, int64_t ldw,
                             const double* Win, int64_t ldwin, int64_t n, int64_t o, int b, const SchurLeafArgs& a,
                             hipStream_t s) {
  if (n <= 0 || n >= 2048 || a.qo % 64 != 0 || a.qb <= 0 || a.qb > 64 || a.qo + a.qb > n || b <= 0)
    return hipErrorInvalidValue;
  StepArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = Ct; g.lda = ldc;
  g.B = R; g.ldb = ldr;
  g.W = W; g.ldw = ldw;
  g.Win = Win; g.ldwin = ldwin;
  g.R = R; g.ldr = ldr;
  g.M = n; g.N = n; g.K = b; g.o = o; g.b = b; g.oc = o;
  const int64_t TT = (n + 63) / 64;
  const unsigned G = (unsigned)(TT * TT);  // one workgroup per tile
  const bool vec = (n % 64 == 0) && (b % 16 == 0) && ((ldc & 1) == 0) && ((ldr & 1) == 0) &&
                   ((((uintptr_t)Ct) & 15) == 0) && ((((uintptr_t)R) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL(k_schur_leaf<true>, dim3(G), dim3(256), 0, s, g, a);
  else
    hipLaunchKernelGGL(k_schur_leaf<false>, dim3(G), dim3(256), 0, s, g, a);
  return hipGetLastError();
}

// Plain FP64 products for the refinement: C = I - A B (resid) or C = Cin + A B,
// all n x n row-major.
hipError_t launch_gemm_f64(int mode, const double* A, int64_t lda, const double* B, int64_t ldb, const double* Cin,
                           int64_t ldcin, double* C, int64_t ldc, int64_t n, hipStream_t s, double* flops) {
  StepArgs g;
  g.A = A; g.lda = lda;
  g.B = B; g.ldb = ldb;
  g.W = C; g.ldw = ldc;
  g.Win = Cin; g.ldwin = ldcin;
  g.R = nullptr; g.ldr = 0;
  g.M = n; g.N = n; g.K = (int)n; g.o = 0; g.b = 0; g.oc = 0;
  if (mode == MODE_RESID) return launch_step<MODE_RESID, 128, 128, false, 4, 2>(g, s, 0, 0, 0, flops);
  return launch_step<MODE_ADD, 128, 128, false, 4, 2>(g, s, 0, 0, 0, flops);
}

// Skinny product with the contraction split over workgroups: part s of the
// S slices is M[:, s kslice ..) (m-major, ld ldm) times V[s kslice .., :]
// (n x 64, ld 64), written to parts + s pstride (n x 64, ld 64).  Workgroup
// (t, s) computes row tile t of slice s.
template <bool VEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_skinny_splitk(const double* __restrict__ Mx, int64_t ldm, const double* __restrict__ V, int64_t n, int64_t kslice,
                double* __restrict__ parts, int64_t pstride) {
  using C = TileCfg<64, 64, 2, 2>;
  __shared__ double As[2][C::BK * C::LA];
  __shared__ double Bs[2][C::BK * C::LB];
  const int64_t TM = (n + 63) / 64;
  const int64_t t = blockIdx.x % TM, sl = blockIdx.x / TM;
  const int64_t k0 = sl * kslice;
  StepArgs g;
  g.A = Mx + k0; g.lda = ldm;
  g.B = V + k0 * 64; g.ldb = 64;
  g.W = parts + sl * pstride; g.ldw = 64;
  g.Win = nullptr; g.ldwin = 0;
  g.R = nullptr; g.ldr = 0;
  g.M = n; g.N = 64;
  g.K = (int)((n - k0 < kslice) ? n - k0 : kslice);
  g.o = 0; g.b = 0; g.oc = 0;
  gemm_tile<MODE_ROW, C, false, VEC>(g, t, 0, As, Bs);
}

// out[e] = sum over s of parts[s pstride + e], in the order s = 0, 1, ...
__global__ void __launch_bounds__(256) k_sum_slices(const double* __restrict__ parts, int S, int64_t pstride,
                                                    int64_t count, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int sl = 0; sl < S; ++sl) v += parts[sl * pstride + e];
    out[e] = v;
  }
}

// Per-workgroup partial sums of (Z[e] + sum over s of parts[s pstride + e])^2.
__global__ void __launch_bounds__(256) k_probe_sumsq(const double* __restrict__ Z, const double* __restrict__ parts,
                                                     int S, int64_t pstride, int64_t count, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
    double v = Z[e];
    for (int sl = 0; sl < S; ++sl) v += parts[sl * pstride + e];
    acc = fma(v, v, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ||Z - A X Z||_F^2 into *out for 64 random sign columns Z (the probed
// residual E = Z + A Y with Y = X Zn, Zn = -Z): Z and Zn are drawn into the
// workspace, Y = X Zn and A Y are formed with the contraction split over about
// 512 workgroups (both products have only n / 64 row tiles), the slices are
// summed in a fixed order, and E is reduced as it is formed.  Every row of
// A X - I contributes to every column of E, so ||E||_F^2 / 64 is an unbiased
// estimate of ||A X - I||_F^2 whatever the distribution of the error over the
// rows.  work: 3 * 64 n doubles with one slice, (3 + S) 64 n with S >= 2
// slices (S <= n / 64 - 3), so n^2 doubles suffice for n >= 192; part:
// kParts + 1 doubles, the result in part[kParts].
hipError_t launch_probe_residual(const double* A, int64_t lda, const double* X, int64_t ldx, int64_t n,
                                 double* work, uint64_t seed, double* part, int kParts, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  constexpr int k = 64;
  const int64_t count = n * k;
  double* Z = work;
  double* Zn = work + count;
  double* Y = work + 2 * count;
  double* parts = work + 3 * count;
  const int64_t TM = (n + 63) / 64;
  int64_t S = (512 + TM - 1) / TM;
  const int64_t smax = n / 64 - 3 > 1 ? n / 64 - 3 : 1;
  if (S > smax) S = smax;
  int64_t kslice = (n + S - 1) / S;
  kslice = (kslice + 63) / 64 * 64;
  S = (n + kslice - 1) / kslice;
  const int64_t gz = (count + 255) / 256;
  const unsigned gr = (unsigned)(gz < 1024 ? gz : 1024);
  hipLaunchKernelGGL(k_sign_probes, dim3(gr), dim3(256), 0, s, Z, Zn, count, seed);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool vec = (n % 64 == 0) && ((lda & 1) == 0) && ((ldx & 1) == 0) && ((((uintptr_t)A) & 15) == 0) &&
                   ((((uintptr_t)X) & 15) == 0);
  const dim3 grid((unsigned)(TM * S));
  // with one slice the products need no partial buffers: X Zn goes straight
  // to Y and A Y to Zn's place (3 * 64 n doubles in all)
  double* p1 = S == 1 ? Y : parts;
  double* p2 = S == 1 ? Zn : parts;
  // Y = X Zn
  if (vec)
    hipLaunchKernelGGL(k_skinny_splitk<true>, grid, dim3(256), 0, s, X, ldx, Zn, n, kslice, p1, count);
  else
    hipLaunchKernelGGL(k_skinny_splitk<false>, grid, dim3(256), 0, s, X, ldx, Zn, n, kslice, p1, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (S > 1) {
    hipLaunchKernelGGL(k_sum_slices, dim3(gr), dim3(256), 0, s, parts, (int)S, count, count, Y);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // A Y, then ||Z + A Y||^2
  if (vec)
    hipLaunchKernelGGL(k_skinny_splitk<true>, grid, dim3(256), 0, s, A, lda, Y, n, kslice, p2, count);
  else
    hipLaunchKernelGGL(k_skinny_splitk<false>, grid, dim3(256), 0, s, A, lda, Y, n, kslice, p2, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_probe_sumsq, dim3((unsigned)kParts), dim3(256), 0, s, Z, p2, (int)S, count, count, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_sum_final(part, kParts, part + kParts, s);
}

// ---------------------------------------------------------------------------
// One batched sweep step of one matrix per workgroup: P = W_pp^-1 (leaf), the
// row panel R = P W[p, :], the old column panel W[:, p] copied to Ct, then the
// Schur update of every tile.  The workgroup alone touches this matrix during
// the launch, so the phases only need workgroup barriers; the arithmetic is
// that of the separate leaf, row-panel and Schur launches.
// ---------------------------------------------------------------------------
template <int RPL, int CPW, int NWV, class C>
__global__ void __launch_bounds__(64 * NWV) k_swept_step(const SweptJob* __restrict__ jobs) {
  static_assert(64 * NWV == C::NT, "leaf and tile shapes must use the same workgroup");
  __shared__ double As[2][C::BK * C::LA];
  __shared__ double Bs[2][C::BK * C::LB];
  const SweptJob& J = jobs[blockIdx.x];
  leaf_body<RPL, CPW, NWV>(J.leaf.A, J.leaf.lda, J.leaf.P, J.leaf.ldp, J.leaf.b, (int64_t)J.leaf.row0, J.leaf.info);
  __syncthreads();
  {
    const StepArgs& g = J.row;
    const int64_t TM = (g.M + C::BM - 1) / C::BM, TN = (g.N + C::BN - 1) / C::BN;
    for (int64_t t = 0; t < TM * TN; ++t) gemm_tile<MODE_ROW, C, false, false>(g, t / TN, t % TN, As, Bs);
  }
  __syncthreads();
  {
    const StepArgs& g = J.schur;
    double* Cp = const_cast<double*>(g.A);
    const int total = (int)g.M * g.b;  // <= 256 x 128
    for (int e = threadIdx.x; e < total; e += C::NT) {
      const int i = e / g.b;
      const int t = e - i * g.b;
      Cp[(int64_t)i * g.lda + t] = g.Win[(int64_t)i * g.ldwin + g.o + t];
    }
    __syncthreads();
    const int64_t TM = (g.M + C::BM - 1) / C::BM, TN = (g.N + C::BN - 1) / C::BN;
    for (int64_t t = 0; t < TM * TN; ++t) gemm_tile<MODE_SCHUR, C, false, false>(g, t / TN, t % TN, As, Bs);
  }
}

hipError_t launch_swept_step(const SweptJob* jobs, int64_t count, int bmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  // pivot blocks above 64: 64 x 128 Schur tiles (each row's column-panel
  // slice read half as often; 18.4 against 18.9 ms per measured batch); at
  // most 64: 64 x 64 (the wider tile's registers halve the occupancy there)
  if (bmax <= 64)
    hipLaunchKernelGGL((k_swept_step<1, 16, 4, TileCfg<64, 64, 2, 2>>), dim3((unsigned)count), dim3(256), 0, s, jobs);
  else
    hipLaunchKernelGGL((k_swept_step<2, 16, 8, TileCfg<64, 128, 4, 2>>), dim3((unsigned)count), dim3(512), 0, s, jobs);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Block-row pivoting (the pivot rows of block p chosen among all rows below).
//
// The paper's method assumes that every pivot block and Schur complement is
// invertible and otherwise changes the blocking (§3); its counter-diagonal
// partition, Eqs. (b) and (c), is Eq. (a) applied to a block-row permuted
// matrix.  Here the rows that form each pivot block are chosen by tournament
// selection on the block's current columns: strips of 64 columns in turn;
// leaves of 256 consecutive rows (rows already chosen left out), each node
// keeping the 64 rows that Gauss elimination with partial pivoting picks among
// its candidates, four nodes merging into one, the root's picks (in pick
// order) being the strip's pivot rows, which are then eliminated from the
// block's later columns.  The chosen rows move to the block's position, the
// rows they displace take the vacated positions, and a final column
// permutation undoes the moves.
// ---------------------------------------------------------------------------

// Pivot search in one column held as x[h] (candidate lane + 64 h) by every
// lane of a wave: the largest |value| among rows not yet picked, the lowest
// candidate position on ties; kTournRows when every row is picked.
template <int RPL>
__device__ __forceinline__ int tourn_search(const double (&x)[RPL], const bool (&used)[RPL], double& pv) {
  unsigned long long key[RPL];
  unsigned long long kmax = 0;
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    key[h] = used[h] ? 0ULL : (unsigned long long)__double_as_longlong(fabs(x[h])) + 1ULL;
    kmax = key[h] > kmax ? key[h] : kmax;
  }
  const unsigned hi = __ockl_wfred_max_u32((unsigned)(kmax >> 32));
  const unsigned lo = __ockl_wfred_max_u32((unsigned)(kmax >> 32) == hi ? (unsigned)kmax : 0u);
  kmax = ((unsigned long long)hi << 32) | lo;
  pv = 0.0;
  if (kmax == 0ULL) return 64 * RPL;
  int r = 64 * RPL;
#pragma unroll
  for (int h = RPL - 1; h >= 0; --h) {
    const unsigned long long mk = __ballot(key[h] == kmax);
    if (mk) r = 64 * h + __ffsll((long long)mk) - 1;
  }
#pragma unroll
  for (int h = 0; h < RPL; ++h)
    if ((r >> 6) == h) pv = readlane_f64(x[h], r & 63);
  return r;
}

// One tournament node per workgroup: 4 waves, lane l holding candidates
// l + 64 h (h < 4), wave v holding strip columns [16 v, 16 v + 16).
// CPW strip columns per wave, 64 / CPW waves: fewer columns per wave shorten
// each wave's share of a column step (its updates and pivot-row reads).
template <int CPW>
__global__ void __launch_bounds__(64 * (64 / CPW)) k_tourn_node(TournArgs a) {
  // the selection gates the next step's row panel and runs beside the
  // trailing update: its waves issue ahead of the update's on shared CUs
  __builtin_amdgcn_s_setprio(3);
  constexpr int RPL = kTournRows / 64, NW = 64 / CPW;
  static_assert(NW * CPW == 64 && NW >= kTournArity && 64 * NW >= kTournRows, "waves must cover the strip and the candidates");
  __shared__ int cand[kTournRows];
  __shared__ int wcount[NW];
  __shared__ double colbuf[2][kTournRows];
  __shared__ int s_r[2];
  __shared__ double s_pv[2];
  __shared__ int picks[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t node = blockIdx.x;

  // candidates, in order: a leaf's rows not yet chosen, or the children's picks
  int row = -1;
  if (a.is_leaf) {
    const int64_t r = a.o + node * kTournRows + tid;
    if (tid < kTournRows && r < a.n && a.used[r] == 0) row = (int)r;
  } else {
    const int64_t child = node * kTournArity + (tid >> 6);
    if ((tid >> 6) < kTournArity && child < a.nin) row = a.in[child * 64 + lane];
  }
  const unsigned long long mk = __ballot(row >= 0);
  if (lane == 0) wcount[wave] = __popcll(mk);
  __syncthreads();
  int before = 0, nc = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    before += (v < wave) ? wcount[v] : 0;
    nc += wcount[v];
  }
  if (row >= 0) cand[before + __popcll(mk & ((1ULL << lane) - 1ULL))] = row;
  __syncthreads();

  const int w = a.w;
  // row half h of this wave's CPW columns (a vector, so that the next
  // column's slot, a uniform index, is one indexed register move)
  typedef double vcd __attribute__((ext_vector_type(CPW)));
  vcd v[RPL];
  bool used[RPL];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int i = lane + 64 * h;
    used[h] = i >= nc;
    const int ri = used[h] ? 0 : cand[i];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int col = wave * CPW + j;
      v[h][j] = (!used[h] && col < w) ? a.T[(int64_t)(a.c0 + col) * a.ldt + ri] : 0.0;
    }
  }
  if (wave == 0) {
    double x[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) x[h] = v[h][0];
    double pv;
    const int r = tourn_search<RPL>(x, used, pv);
#pragma unroll
    for (int h = 0; h < RPL; ++h) colbuf[0][lane + 64 * h] = x[h];
    if (lane == 0) {
      s_r[0] = r;
      s_pv[0] = pv;
    }
  }
  // Per column c: the multipliers, then column c + 1 by its owner wave and
  // its pivot search, then every slot of every wave with the pivot row's
  // values (read from lane r % 64 of row half r / 64, a uniform choice).
  // Columns up to c are never read again, so their slots are updated too (the
  // rows' values there no longer matter) and every register index is a
  // constant; only the next column's slot (a uniform index) is chosen at run
  // time.
  int got = 0, zero = -1;
  for (int c = 0; c < w; ++c) {
    const int buf = c & 1;
    __syncthreads();
    const int r = s_r[buf];
    if (r >= kTournRows) break;  // every candidate picked (uniform)
    const double pv = s_pv[buf];
    if (tid == 0) picks[c] = cand[r];
    got = c + 1;
    if (pv == 0.0 && zero < 0) zero = c;
    const double q = pv != 0.0 ? 1.0 / pv : 0.0;
    const int rl = __builtin_amdgcn_readfirstlane(r & 63);
    const int rh = __builtin_amdgcn_readfirstlane(r >> 6);
    double f[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int i = lane + 64 * h;
      const bool isr = (i == r);
      f[h] = (used[h] || isr) ? 0.0 : colbuf[buf][i] * q;
      used[h] = used[h] || isr;
    }
    const int cn = c + 1;
    const bool nowner = (cn < w) && (cn / CPW == wave);
    const int sn = cn % CPW;
    if (nowner) {
      // the pivot row's value in column c + 1 alone, read first: the search
      // does not wait for the rest of the row
      double t = v[0][sn];
#pragma unroll
      for (int h = 1; h < RPL; ++h) t = (h == rh) ? v[h][sn] : t;
      const double pj = readlane_f64(t, rl);
      double x[RPL];
#pragma unroll
      for (int h = 0; h < RPL; ++h) x[h] = fma(-f[h], pj, v[h][sn]);
      double pv2;
      const int r2 = tourn_search<RPL>(x, used, pv2);
#pragma unroll
      for (int h = 0; h < RPL; ++h) colbuf[buf ^ 1][lane + 64 * h] = x[h];
      if (lane == 0) {
        s_r[buf ^ 1] = r2;
        s_pv[buf ^ 1] = pv2;
      }
    }
    // the pivot row's values in this wave's columns, then every slot
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      double t = v[0][j];
#pragma unroll
      for (int h = 1; h < RPL; ++h) t = (h == rh) ? v[h][j] : t;
      const double sp = readlane_f64(t, rl);
#pragma unroll
      for (int h = 0; h < RPL; ++h) v[h][j] = fma(-f[h], sp, v[h][j]);
    }
  }
  __syncthreads();
  if (tid < 64) {
    const int pk = tid < got ? picks[tid] : -1;
    a.out[node * 64 + tid] = pk;
    if (a.is_root && tid < w) {
      a.chosen[a.c0 + tid] = pk;
      if (pk >= 0) a.used_w[pk] = 1;
    }
  }
  if (a.is_root && tid == 0 && (zero >= 0 || got < w)) record_singular(a.info, a.row0 + (zero >= 0 ? zero : got) + 1);
}

// S[k][t] = T[(c0 + t) ldt + rows[k]] for k < nrows, t < ncols (rows of a
// k-major panel gathered into a row-major block).
__global__ void __launch_bounds__(256) k_gather_kmajor(const double* __restrict__ T, int64_t ldt, int c0, int ncols,
                                                       const int32_t* __restrict__ rows, int nrows,
                                                       double* __restrict__ S, int64_t lds) {
  const int k = blockIdx.y;
  if (k >= nrows) return;
  const int64_t r = rows[k];
  for (int t = blockIdx.x * 256 + threadIdx.x; t < ncols; t += gridDim.x * 256)
    S[(int64_t)k * lds + t] = r >= 0 ? T[(int64_t)(c0 + t) * ldt + r] : 0.0;
}

// Y[k][:] = W[rows[k]][:] (whole rows gathered).
__global__ void __launch_bounds__(256) k_gather_rows(const double* __restrict__ W, int64_t ldw, int64_t ncols,
                                                     const int32_t* __restrict__ rows, double* __restrict__ Y,
                                                     int64_t ldy) {
  const int k = blockIdx.y;
  const int64_t r = rows[k];
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < ncols; j += (int64_t)gridDim.x * 256)
    Y[(int64_t)k * ldy + j] = r >= 0 ? W[r * ldw + j] : 0.0;
}

// The moves of block [o, o + b) once its pivot rows chosen[0..b) are known:
// D = the rows of [o, o + b) not chosen, V = the chosen rows at or after
// o + b, both ascending (|D| = |V| = m); row D_i moves to V_i and the chosen
// row chosen[k] to o + k.  One workgroup of 1024 threads: plan[0] = m,
// plan[1 + i] = D_i, plan[1 + bmax + i] = V_i; perm (the original row at each
// position) is updated to match.
__global__ void __launch_bounds__(1024) k_plan_moves(const int32_t* __restrict__ used,
                                                     const int32_t* __restrict__ chosen, int64_t o, int b,
                                                     int64_t n, int bmax, int32_t* __restrict__ plan,
                                                     int32_t* __restrict__ perm) {
  __shared__ int wsum[16];
  __shared__ int s_base;
  __shared__ int32_t pv_chosen[2048];
  __shared__ int32_t pv_disp[2048];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int32_t* D = plan + 1;
  int32_t* V = plan + 1 + bmax;
  // ordered compaction of the rows of [lo, hi) whose used flag equals want
  auto compact = [&](int64_t lo, int64_t hi, int want, int32_t* dst) -> int {
    __syncthreads();  // every thread has read the previous call's count
    if (tid == 0) s_base = 0;
    __syncthreads();
    for (int64_t r0 = lo; r0 < hi; r0 += 1024) {
      const int64_t r = r0 + tid;
      const bool ok = r < hi && (used[r] != 0) == (want != 0);
      const unsigned long long mk = __ballot(ok);
      if (lane == 0) wsum[wave] = __popcll(mk);
      __syncthreads();
      int before = 0, tot = 0;
      for (int v = 0; v < 16; ++v) {
        before += (v < wave) ? wsum[v] : 0;
        tot += wsum[v];
      }
      const int base = s_base;
      const int at = base + before + __popcll(mk & ((1ULL << lane) - 1ULL));
      if (ok && at < b) dst[at] = (int32_t)r;  // at most b rows qualify when the picks are consistent
      __syncthreads();
      if (tid == 0) s_base = base + tot;
      __syncthreads();
    }
    return s_base;
  };
  const int m1 = compact(o, o + b, 0, D);
  const int m2 = compact(o + b, n, 1, V);
  const int m = m1 < m2 ? m1 : m2;  // equal unless a pick was missing
  if (tid == 0) plan[0] = m;
  for (int k = tid; k < b; k += 1024) pv_chosen[k] = chosen[k] >= 0 ? perm[chosen[k]] : -1;
  for (int i = tid; i < m; i += 1024) pv_disp[i] = perm[D[i]];
  __syncthreads();
  for (int k = tid; k < b; k += 1024)
    if (pv_chosen[k] >= 0) perm[o + k] = pv_chosen[k];
  for (int i = tid; i < m; i += 1024) perm[V[i]] = pv_disp[i];
}

// Row D_i of W moves to row V_i (all n columns), and so does its entry in
// every row of the saved column panel Ct (b x n, k-major).
__global__ void __launch_bounds__(256) k_apply_moves(const int32_t* __restrict__ plan, int bmax, double* W,
                                                     int64_t ldw, int64_t n, double* Ct, int64_t ldc, int b) {
  const int i = blockIdx.y;
  if (i >= plan[0]) return;
  const int64_t d = plan[1 + i], v = plan[1 + bmax + i];
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    W[v * ldw + j] = W[d * ldw + j];
  for (int t = blockIdx.x * 256 + threadIdx.x; t < b; t += gridDim.x * 256)
    Ct[(int64_t)t * ldc + v] = Ct[(int64_t)t * ldc + d];
}

// X[i][perm[c]] = W[i][c] in place, one workgroup per row: every value of the
// row is read into registers before any is written.
template <int VPT>
__global__ void __launch_bounds__(1024) k_unpermute_cols(double* W, int64_t ldw, int64_t n,
                                                         const int32_t* __restrict__ perm) {
  const int64_t i = blockIdx.x;
  double v[VPT];
  int32_t dst[VPT];
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    const int64_t c = threadIdx.x + 1024 * u;
    const int32_t d = c < n ? perm[c] : -1;
    dst[u] = d < n ? d : -1;
    v[u] = c < n ? W[i * ldw + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < VPT; ++u)
    if (dst[u] >= 0) W[i * ldw + dst[u]] = v[u];
}

// ---- launchers ----
hipError_t launch_tourn_level(const TournArgs& a, int64_t nodes, hipStream_t s) {
  if (nodes <= 0 || a.w <= 0 || a.w > 64) return hipErrorInvalidValue;
  // 8 waves of 8 columns (measured: pivoted sweep 87 against 96 ms at
  // n = 8192 for 4 waves of 16, 88 for 16 waves of 4)
  hipLaunchKernelGGL(k_tourn_node<8>, dim3((unsigned)nodes), dim3(512), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_kmajor(const double* T, int64_t ldt, int c0, int ncols, const int32_t* rows, int nrows,
                                double* S, int64_t lds, hipStream_t s) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min(8, (ncols + 255) / 256);
  hipLaunchKernelGGL(k_gather_kmajor, dim3(gx, (unsigned)nrows), dim3(256), 0, s, T, ldt, c0, ncols, rows, nrows, S,
                     lds);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double* W, int64_t ldw, int64_t ncols, const int32_t* rows, int nrows, double* Y,
                              int64_t ldy, hipStream_t s) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min<int64_t>(16, (ncols + 255) / 256);
  hipLaunchKernelGGL(k_gather_rows, dim3(gx, (unsigned)nrows), dim3(256), 0, s, W, ldw, ncols, rows, Y, ldy);
  return hipGetLastError();
}

hipError_t launch_moves(const int32_t* used, const int32_t* chosen, int64_t o, int b, int64_t n, int bmax,
                        int32_t* plan, int32_t* perm, double* W, int64_t ldw, double* Ct, int64_t ldc,
                        hipStream_t s) {
  if (b <= 0) return hipSuccess;
  if (b > 2048 || bmax < b) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plan_moves, dim3(1), dim3(1024), 0, s, used, chosen, o, b, n, bmax, plan, perm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gx = (unsigned)std::min<int64_t>(16, (n + 255) / 256);
  hipLaunchKernelGGL(k_apply_moves, dim3(gx, (unsigned)b), dim3(256), 0, s, plan, bmax, W, ldw, n, Ct, ldc, b);
  return hipGetLastError();
}

hipError_t launch_unpermute_cols(double* W, int64_t ldw, int64_t n, const int32_t* perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n <= 8192)
    hipLaunchKernelGGL(k_unpermute_cols<8>, dim3((unsigned)n), dim3(1024), 0, s, W, ldw, n, perm);
  else if (n <= 16384)
    hipLaunchKernelGGL(k_unpermute_cols<16>, dim3((unsigned)n), dim3(1024), 0, s, W, ldw, n, perm);
  else if (n <= 32768)
    hipLaunchKernelGGL(k_unpermute_cols<32>, dim3((unsigned)n), dim3(1024), 0, s, W, ldw, n, perm);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// General step GEMMs on 64 x 64 tiles, for panels the sweep does not cover:
// MODE_ROW: W = A B (A m-major), with W[:, oc:oc+b] = R (b columns);
// MODE_SCHUR: W = Win - A B (A k-major), rows [o, o+b) taking R and columns
// [oc, oc+b) starting from zero.  b = 0 disables both special cases.
hipError_t launch_gemm_rows(int mode, const double* A, int64_t lda, const double* B, int64_t ldb, double* W,
                            int64_t ldw, const double* Win, int64_t ldwin, const double* R, int64_t ldr, int64_t M,
                            int64_t N, int K, int64_t o, int64_t oc, int b, hipStream_t s) {
  StepArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.lda = lda;
  g.B = B; g.ldb = ldb;
  g.W = W; g.ldw = ldw;
  g.Win = Win; g.ldwin = ldwin;
  g.R = R; g.ldr = ldr;
  g.M = M; g.N = N; g.K = K; g.o = o; g.b = b; g.oc = oc;
  if (mode == MODE_ROW) return launch_step<MODE_ROW, 64, 64, false>(g, s, 0, 0, 0, nullptr);
  return launch_step<MODE_SCHUR, 64, 64, true>(g, s, 0, 0, 0, nullptr);
}


// ---------------------------------------------------------------------------
// Compensated residual R = I - A X by an error-free split of the operands
// (Ozaki, Ogita, Oishi and Rump, 2012): A = A1 + A2 row by row and
// X = X1 + X2 column by column, where A1 keeps `bits` bits of each row's
// largest magnitude and X1 likewise per column.  With 2 bits + ceil(log2 n)
// <= 52 every product of A1 X1 and every partial sum of a row-by-column dot
// product lies on one grid of at most 53 bits, so the FP64 product A1 X1 is
// exact whatever the summation order, and so is I - A1 X1.  Then
// R = (I - A1 X1) - A2 X1 - A X2, where the last two terms are about 2^-bits
// of |A||X| and their rounding errors 2^-bits times smaller than that of a
// plain FP64 residual.
// ---------------------------------------------------------------------------

// exps[i] = the binary exponent E with max_k |M[i][k]| < 2^E (0 for a zero row).
__global__ void __launch_bounds__(256) k_row_exponent(const double* __restrict__ M, int64_t ldm, int64_t n,
                                                      int* __restrict__ exps) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) m = fmax(m, fabs(M[i * ldm + k]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    (void)frexp(red[0], &e);
    exps[i] = e;
  }
}

// exps[j] = the binary exponent F with max_k |M[k][j]| < 2^F, one thread per column.
__global__ void __launch_bounds__(256) k_col_exponent(const double* __restrict__ M, int64_t ldm, int64_t n,
                                                      int* __restrict__ exps) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double m = 0.0;
  for (int64_t k = 0; k < n; ++k) m = fmax(m, fabs(M[k * ldm + j]));
  int e = 0;
  (void)frexp(m, &e);
  exps[j] = e;
}

// Hi = M rounded to `bits` bits below 2^exp (exp of the row when by_row, of
// the column otherwise), NegLo = Hi - M (exact): both n x n, ld n.
__global__ void __launch_bounds__(256) k_split(const double* __restrict__ M, int64_t ldm, int64_t n,
                                               const int* __restrict__ exps, int by_row, int bits,
                                               double* __restrict__ Hi, double* __restrict__ NegLo) {
  const int64_t i = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const int e = by_row ? exps[i] : exps[j];
    const double x = M[i * ldm + j];
    const double h = ldexp(rint(ldexp(x, bits - e)), e - bits);
    Hi[i * n + j] = h;
    NegLo[i * n + j] = h - x;
  }
}

hipError_t launch_split(const double* M, int64_t ldm, int64_t n, int by_row, int bits, int* exps, double* Hi,
                        double* NegLo, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (by_row)
    hipLaunchKernelGGL(k_row_exponent, dim3((unsigned)n), dim3(256), 0, s, M, ldm, n, exps);
  else
    hipLaunchKernelGGL(k_col_exponent, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, ldm, n, exps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gx = (unsigned)std::min<int64_t>(64, (n + 255) / 256);
  hipLaunchKernelGGL(k_split, dim3(gx, (unsigned)n), dim3(256), 0, s, M, ldm, n, exps, by_row, bits, Hi, NegLo);
  return hipGetLastError();
}

// Bits kept per part so that two parts' products summed over n terms stay on
// a 53-bit grid: 2 bits + ceil(log2 n) <= 52.
int split_bits(int64_t n) {
  int lg = 0;
  while ((int64_t(1) << lg) < n) ++lg;
  return (52 - lg) / 2;
}

// R (n x n, ld n) = I - A X, compensated: split A by rows into A1 and -A2
// (split_a = {A1, -A2}, computed when fresh_a), X by columns into X1 and -X2
// (split_x), then R = I - A1 X1 (exact), R += (-A2) X1, R += A (-X2).
hipError_t launch_resid_compensated(const double* A, int64_t lda, const double* X, int64_t ldx, int64_t n,
                                    double* R, double* split_a, double* split_x, int* exps, bool fresh_a,
                                    hipStream_t s, double* flops) {
  const int bits = split_bits(n);
  const size_t nn = (size_t)n * (size_t)n;
  hipError_t e = hipSuccess;
  if (fresh_a) e = launch_split(A, lda, n, 1, bits, exps, split_a, split_a + nn, s);
  if (e == hipSuccess) e = launch_split(X, ldx, n, 0, bits, exps + n, split_x, split_x + nn, s);
  if (e == hipSuccess) e = launch_gemm_f64(MODE_RESID, split_a, n, split_x, n, nullptr, 0, R, n, n, s, nullptr);
  if (e == hipSuccess) e = launch_gemm_f64(MODE_ADD, split_a + nn, n, split_x, n, R, n, R, n, n, s, nullptr);
  if (e == hipSuccess) e = launch_gemm_f64(MODE_ADD, A, lda, split_x + nn, n, R, n, R, n, n, s, nullptr);
  if (flops) *flops = 3 * 2.0 * (double)n * (double)n * (double)n;
  return e;
}



}  // namespace binv
