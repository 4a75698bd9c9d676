// Batched inversion of many small, uneven matrices (orders up to 256).
//
// Every matrix keeps its own partition into diagonal blocks.  Eliminating the
// columns of diagonal block p one at a time, with the pivot of each column
// searched only among the not-yet-used rows of block p, performs exactly the
// row operations of one step of the blockwise sweep (Eq. (a) of §3 applied in
// place, §4.2): the Gauss-Jordan inversion of the pivot block P = W_pp^-1
// (pivoting inside the block), then W_pj <- P W_pj and the Schur update
// W_ij <- W_ij - W_ip P W_pj.  So a matrix of order <= 128 is inverted by one
// register-resident kernel pass with that block-restricted pivoting.
//
// Register layout per matrix (as in the leaf kernel of kernels.hip): NWV waves,
// wave w owns columns [w CPW, (w+1) CPW), lane l owns rows l + 64 h (h < RPL);
// a workgroup holds SUB independent matrices, one per group of NWV waves.  The
// matrix is padded with an identity to NB = NWV*CPW (the padding forms a last
// diagonal block of its own).
//
// Pivot rows are stored unscaled: when row r becomes the pivot of column c
// (value pv, q = 1/pv), its stored values stay as they are and its scale
// becomes q (its column-c slot is set to 1, i.e. q / q).  Any later update of
// a row subtracts (its stored multiplier) x (true scaled pivot row), which is
// the true update divided by that row's scale, so every row is rescaled once
// at the end.  This saves one multiply per element per column.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "binv_internal.h"

namespace binv {


__device__ __forceinline__ double bread_f64(double x, int l) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Pivot search of one column x[h] (row lane + 64 h) among the rows of [bs, be)
// not used yet: key = bits(|x|) + 1 orders like |x| (0 excludes a row), one
// 64-bit wave max as two 32-bit DPP reductions, lowest row on ties.  With
// `publish` the wave stores the multipliers and the pivot into the LDS slot.
template <int RPL>
__device__ __forceinline__ void small_search(const double (&x)[RPL], const bool (&used)[RPL], int bs, int be,
                                             bool publish, double* colbuf, int* s_r, double* s_pv, int lane) {
  unsigned long long key[RPL];
  unsigned long long kmax = 0;
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int row = lane + 64 * h;
    const bool cand = !used[h] && row >= bs && row < be;
    key[h] = cand ? (unsigned long long)__double_as_longlong(fabs(x[h])) + 1ULL : 0ULL;
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
    if ((r >> 6) == h) pv = bread_f64(x[h], r & 63);
  if (publish) {
#pragma unroll
    for (int h = 0; h < RPL; ++h) colbuf[lane + 64 * h] = x[h];
    if (lane == 0) {
      *s_r = r;
      *s_pv = pv;
    }
  }
}

// MINW: waves per SIMD the register budget must allow (1 = no constraint;
// 4 lets two 8-wave workgroups share a CU at the cost of a few spilled bytes).
template <int RPL, int CPW, int NWV, int SUB, int MINW = 1>
__global__ void __launch_bounds__(64 * NWV * SUB) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
k_small_inverse(const double* __restrict__ A, double* __restrict__ X, const SmallMat* __restrict__ mats,
                const int32_t* __restrict__ order, int64_t count, const int32_t* __restrict__ bounds,
                int32_t* __restrict__ info) {
  constexpr int NB = NWV * CPW;
  static_assert(NB <= 64 * RPL, "columns exceed rows");
  __shared__ double colbuf[SUB][2][64 * RPL];
  __shared__ int s_r[SUB][2];
  __shared__ double s_pv[SUB][2];
  __shared__ int piv_row[SUB][NB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int gwave = tid >> 6;
  const int sub = gwave / NWV;          // which matrix of the workgroup
  const int wave = gwave % NWV;         // wave within the matrix group
  const int64_t slot = (int64_t)blockIdx.x * SUB + sub;
  const bool active = slot < count;     // uniform per wave group
  SmallMat mt;
  mt.off = 0; mt.m = 0; mt.nb = 0; mt.bnd = 0; mt.id = 0;
  if (active) mt = mats[order[slot]];
  const int m = mt.m;
  const int cbase = wave * CPW;

  double v[RPL][CPW];
  double scale[RPL];
  bool used[RPL];
  int step_of[RPL];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int row = lane + 64 * h;
    used[h] = row >= NB;
    step_of[h] = 0;
    scale[h] = 1.0;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int col = cbase + j;
      v[h][j] = (row < m && col < m) ? A[mt.off + (int64_t)row * m + col] : (row == col ? 1.0 : 0.0);
    }
  }

  // columns at or beyond every matrix's order are identity padding of all
  // the workgroup's matrices and are not eliminated (see the leaf kernel);
  // the loop bound must be uniform over the workgroup because of the barriers
  __shared__ int s_m[SUB];
  if (wave == 0 && lane == 0) s_m[sub] = m;
  __syncthreads();
  int mmax = 0;
#pragma unroll
  for (int q = 0; q < SUB; ++q) mmax = s_m[q] > mmax ? s_m[q] : mmax;

  // current diagonal block [bs, be) of the column being eliminated (the
  // padding beyond m forms a last block of its own)
  int blk = 0;
  int bs = 0;
  int be = (mt.nb > 0) ? bounds[mt.bnd + 1] : NB;
  {
    double x[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) x[h] = v[h][0];
    small_search<RPL>(x, used, bs, be, wave == 0, colbuf[sub][0], &s_r[sub][0], &s_pv[sub][0], lane);
  }
  bool singular = false;
  for (int cw = 0; cw < NWV; ++cw) {
    if (cw * CPW >= mmax) break;
    const bool owner = (wave == cw);
#pragma unroll
    for (int t = 0; t < CPW; ++t) {
      const int c = cw * CPW + t;
      if (c >= mmax) continue;
      const int buf = c & 1;
      __syncthreads();
      const int r = s_r[sub][buf];
      const double pv = s_pv[sub][buf];
      if (pv == 0.0 && !singular) {
        if (active && wave == 0 && lane == 0 && c < m) info[mt.id] = c + 1;
        singular = true;
      }
      const double q = 1.0 / pv;
      const int rl = __builtin_amdgcn_readfirstlane(r & 63);
      const int rh = (RPL == 1) ? 0 : __builtin_amdgcn_readfirstlane(r >> 6);
      double sp[CPW];
      static_assert(RPL <= 3, "the pivot row's half is chosen among at most three");
      if (RPL == 1 || rh == 0) {
#pragma unroll
        for (int j = 0; j < CPW; ++j) sp[j] = bread_f64(v[0][j], rl) * q;
      } else if (RPL == 3 && rh == 1) {
#pragma unroll
        for (int j = 0; j < CPW; ++j) sp[j] = bread_f64(v[1 % RPL][j], rl) * q;
      } else {
#pragma unroll
        for (int j = 0; j < CPW; ++j) sp[j] = bread_f64(v[RPL - 1][j], rl) * q;
      }
      sp[t] = owner ? q : sp[t];
      double f[RPL];
#pragma unroll
      for (int h = 0; h < RPL; ++h) {
        const int row = lane + 64 * h;
        const bool isr = (row == r);
        f[h] = isr ? 0.0 : colbuf[sub][buf][row];
        v[h][t] = owner ? (isr ? 1.0 : 0.0) : v[h][t];
        used[h] = used[h] || isr;
        step_of[h] = isr ? c : step_of[h];
        scale[h] = isr ? q : scale[h];
      }
      // the block of column c + 1 (uniform)
      if (c + 1 == be) {
        bs = be;
        ++blk;
        be = (blk < mt.nb) ? bounds[mt.bnd + blk + 1] : NB;
      }
      // column c + 1 first (slot s of wave (c + 1) / CPW), then its search
      const int s = (t + 1) % CPW;  // a constant once the t loop is unrolled
      const bool next_owner = (t + 1 < CPW) ? owner : (wave == cw + 1);
#pragma unroll
      for (int h = 0; h < RPL; ++h) v[h][s] = fma(-f[h], sp[s], v[h][s]);
      if (c + 1 < mmax && next_owner) {
        double x[RPL];
#pragma unroll
        for (int h = 0; h < RPL; ++h) x[h] = v[h][s];
        small_search<RPL>(x, used, bs, be, true, colbuf[sub][buf ^ 1], &s_r[sub][buf ^ 1], &s_pv[sub][buf ^ 1],
                          lane);
      }
#pragma unroll
      for (int h = 0; h < RPL; ++h) {
#pragma unroll
        for (int j = 0; j < CPW; ++j)
          if (j != s) v[h][j] = fma(-f[h], sp[j], v[h][j]);
      }
      if (wave == 0 && lane == 0) piv_row[sub][c] = r;
    }
  }
  __syncthreads();
  if (!active) return;
  if (!singular && wave == 0 && lane == 0) info[mt.id] = 0;
  if (singular) return;
  // X^-1[step_of(row)][piv_row[col]] = scale(row) * W[row][col]
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int row = lane + 64 * h;
    if (row >= m) continue;
    double* dst = X + mt.off + (int64_t)step_of[h] * m;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int col = cbase + j;
      if (col < m) dst[piv_row[sub][col]] = v[h][j] * scale[h];
    }
  }
}

// ---------------------------------------------------------------------------
// Residual and Newton-Schulz refinement of small matrices (one workgroup per
// matrix): R = I - A X and rho = ||R||_F / sqrt(m); while rho > target (at
// most max_steps times) X <- X + X R and R, rho again; a step that does not
// lower rho ends the loop.  Products are 64 x 64 output tiles over 16-deep
// LDS chunks, each thread owning a 4 x 4 block.
// ---------------------------------------------------------------------------
constexpr int kRefThreads = 256;

// Out = I - L M (MODE 0; also returns sum Out^2 over the workgroup) or
// Out = Add + L M (MODE 1); all m x m row-major, ld = m.  Out may be NULL in
// MODE 0 (norm only).
template <int MODE>
__device__ double small_product(const double* __restrict__ L, const double* __restrict__ M,
                                const double* __restrict__ Add, double* __restrict__ Out, int m, double* red) {
  __shared__ double Ls[64][17];
  __shared__ double Ms[16][65];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const int tiles = (m + 63) / 64;
  double ss = 0.0;
  for (int tile = 0; tile < tiles * tiles; ++tile) {
    const int i0 = (tile / tiles) * 64, j0 = (tile % tiles) * 64;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k0 = 0; k0 < m; k0 += 16) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = tid + e * kRefThreads;  // 0..1023
        const int li = idx >> 4, lk = idx & 15;
        Ls[li][lk] = (i0 + li < m && k0 + lk < m) ? L[(int64_t)(i0 + li) * m + k0 + lk] : 0.0;
        const int mk = idx >> 6, mj = idx & 63;
        Ms[mk][mj] = (k0 + mk < m && j0 + mj < m) ? M[(int64_t)(k0 + mk) * m + j0 + mj] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        double lv[4], mv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) lv[a] = Ls[ty * 4 + a][kk];
#pragma unroll
        for (int b = 0; b < 4; ++b) mv[b] = Ms[kk][tx * 4 + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(lv[a], mv[b], acc[a][b]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + ty * 4 + a;
      if (i >= m) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = j0 + tx * 4 + b;
        if (j >= m) continue;
        if (MODE == 0) {
          const double r = (i == j ? 1.0 : 0.0) - acc[a][b];
          ss = fma(r, r, ss);
          if (Out) Out[(int64_t)i * m + j] = r;
        } else {
          Out[(int64_t)i * m + j] = Add[(int64_t)i * m + j] + acc[a][b];
        }
      }
    }
  }
  // workgroup sum (fixed order: deterministic)
  red[tid] = ss;
  __syncthreads();
  for (int w = kRefThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double tot = red[0];
  __syncthreads();
  return tot;
}

// Matrix `i` of the list: A, X at mats[idx].off (ld = m); work holds 2 m^2
// doubles per matrix at 2 * off (refinement only).  rho[id], steps[id]
// (either may be NULL) receive the final rho and the number of steps.
__global__ void __launch_bounds__(kRefThreads)
k_small_refine(const double* __restrict__ A, double* __restrict__ X, const SmallMat* __restrict__ mats,
               const int32_t* __restrict__ order, double* __restrict__ work, double target,
               const double* __restrict__ targets, int max_steps, double* __restrict__ rho,
               int32_t* __restrict__ steps) {
  __shared__ double red[kRefThreads];
  const SmallMat mt = mats[order ? order[blockIdx.x] : blockIdx.x];
  const int m = mt.m;
  const double tgt = targets ? targets[mt.id] : target;
  const double* a = A + mt.off;
  double* x = X + mt.off;
  double* R = work ? work + 2 * mt.off : nullptr;
  double* Xn = R ? R + (int64_t)m * m : nullptr;
  double r = sqrt(small_product<0>(a, x, nullptr, R, m, red) / m);
  int k = 0;
  for (; R && k < max_steps && r > tgt; ++k) {
    small_product<1>(x, R, x, Xn, m, red);  // Xn = X + X R
    __syncthreads();
    const double rn = sqrt(small_product<0>(a, Xn, nullptr, R, m, red) / m);  // R of Xn
    if (!(rn < r)) break;  // rounding floor: keep X
    for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += kRefThreads) x[e] = Xn[e];
    __syncthreads();
    r = rn;
  }
  if (threadIdx.x == 0) {
    if (rho) rho[mt.id] = r;
    if (steps) steps[mt.id] = k;
  }
}

hipError_t launch_small_refine(const double* A, double* X, const SmallMat* mats, const int32_t* order, int64_t count,
                               double* work, double target, const double* targets, int max_steps, double* rho,
                               int32_t* steps, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_refine, dim3((unsigned)count), dim3(kRefThreads), 0, s, A, X, mats, order, work, target,
                     targets, max_steps, rho, steps);
  return hipGetLastError();
}

// Launch shapes of the register kernel, per tier.  Every shape runs the same
// per-element arithmetic in the same order (the pivot search is exact and each
// update is one fma of the same operands), so all shapes of a tier give
// bitwise-identical results; the autotuner picks among them by time alone.
// {rows per lane, columns per wave, waves per matrix, matrices per workgroup}
struct TierShape {
  int rpl, cpw, nwv, sub;
};
static const TierShape kShapes[kSmallTierCount][kSmallVariants] = {
    {{1, 8, 1, 4}, {1, 8, 1, 8}, {1, 8, 1, 2}, {1, 8, 1, 16}},      // m <= 8
    {{1, 16, 1, 4}, {1, 16, 1, 8}, {1, 8, 2, 4}, {1, 8, 2, 2}},     // m <= 16
    {{1, 32, 1, 4}, {1, 16, 2, 2}, {1, 8, 4, 1}, {1, 32, 1, 8}},    // m <= 32
    {{1, 16, 4, 1}, {1, 32, 2, 2}, {1, 8, 8, 1}, {1, 16, 4, 2}},    // m <= 64
    {{2, 16, 8, 1}, {2, 8, 16, 1}, {2, 16, 8, 1}, {0, 0, 0, 0}},    // m <= 128 (wider shapes spill;
                                                                    // shape 2 = shape 0 at two workgroups per CU)
    {{3, 16, 12, 1}, {3, 24, 8, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}},    // m <= 192 (one workgroup per CU)
};
static const int kShapeCount[kSmallTierCount] = {4, 4, 4, 4, 3, 2};

template <int RPL, int CPW, int NWV, int SUB, int MINW = 1>
hipError_t launch_shape(const double* A, double* X, const SmallMat* mats, const int32_t* order, int64_t count,
                        const int32_t* bounds, int32_t* info, hipStream_t s) {
  const unsigned g = (unsigned)((count + SUB - 1) / SUB);
  hipLaunchKernelGGL((k_small_inverse<RPL, CPW, NWV, SUB, MINW>), dim3(g), dim3(64 * NWV * SUB), 0, s, A, X, mats,
                     order, count, bounds, info);
  return hipGetLastError();
}

hipError_t launch_small_tier(int tier, int variant, const double* A, double* X, const SmallMat* mats,
                             const int32_t* order, int64_t count, const int32_t* bounds, int32_t* info,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (tier < 0 || tier >= kSmallTierCount || variant < 0 || variant >= kShapeCount[tier]) return hipErrorInvalidValue;
#define BINV_SHAPE(T, V, R, C, N, S) \
  if (tier == T && variant == V) return launch_shape<R, C, N, S>(A, X, mats, order, count, bounds, info, s);
  BINV_SHAPE(0, 0, 1, 8, 1, 4) BINV_SHAPE(0, 1, 1, 8, 1, 8) BINV_SHAPE(0, 2, 1, 8, 1, 2) BINV_SHAPE(0, 3, 1, 8, 1, 16)
  BINV_SHAPE(1, 0, 1, 16, 1, 4) BINV_SHAPE(1, 1, 1, 16, 1, 8) BINV_SHAPE(1, 2, 1, 8, 2, 4) BINV_SHAPE(1, 3, 1, 8, 2, 2)
  BINV_SHAPE(2, 0, 1, 32, 1, 4) BINV_SHAPE(2, 1, 1, 16, 2, 2) BINV_SHAPE(2, 2, 1, 8, 4, 1) BINV_SHAPE(2, 3, 1, 32, 1, 8)
  BINV_SHAPE(3, 0, 1, 16, 4, 1) BINV_SHAPE(3, 1, 1, 32, 2, 2) BINV_SHAPE(3, 2, 1, 8, 8, 1) BINV_SHAPE(3, 3, 1, 16, 4, 2)
  BINV_SHAPE(4, 0, 2, 16, 8, 1) BINV_SHAPE(4, 1, 2, 8, 16, 1)
  if (tier == 4 && variant == 2) return launch_shape<2, 16, 8, 1, 4>(A, X, mats, order, count, bounds, info, s);
  if (tier == 5 && variant == 0) return launch_shape<3, 16, 12, 1>(A, X, mats, order, count, bounds, info, s);
  if (tier == 5 && variant == 1) return launch_shape<3, 24, 8, 1>(A, X, mats, order, count, bounds, info, s);
#undef BINV_SHAPE
  return hipErrorInvalidValue;
}

hipError_t launch_small_tier(int tier, const double* A, double* X, const SmallMat* mats, const int32_t* order,
                             int64_t count, const int32_t* bounds, int32_t* info, hipStream_t s) {
  return launch_small_tier(tier, 0, A, X, mats, order, count, bounds, info, s);
}

int small_variant_count(int tier) { return (tier >= 0 && tier < kSmallTierCount) ? kShapeCount[tier] : 0; }

void small_variant_shape(int tier, int variant, int shape[4]) {
  const TierShape& t = kShapes[tier][variant];
  shape[0] = t.rpl;
  shape[1] = t.cpw;
  shape[2] = t.nwv;
  shape[3] = t.sub;
}

// Largest order handled by each small tier.
int small_tier_limit(int tier) {
  static const int lim[kSmallTierCount] = {8, 16, 32, 64, 128, 192};
  return (tier >= 0 && tier < kSmallTierCount) ? lim[tier] : 0;
}

}  // namespace binv
