// The paper's parallel algorithm (§5) for batches of small matrices: each
// matrix, partitioned into a power-of-two number N_k of diagonal blocks of
// orders 1..4 (Table 2's scheme gives orders 2..4), is inverted bottom-up by
// Eq. (ad) over N_s = 2 N_k - 1 steps.  The step number (stepid) alone fixes
// what a step does (§5.3-§5.4, Tables 4 and 5): with z the 1-based position
// of its lowest set bit and p that of the next set bit above it,
//   z > 1: →, ← and ∼ (R = -A^-1 B, L = -D^-1 C, S_A = D + C R,
//          S_D = A + B L) on every level-(z-1) unit of the source, into the
//          provisional set T_(z-1);
//   z = 1: ◊ (closed-form inverse) of every diagonal block of the source,
//          then ↑↓ (X12 = R S_A^-1, X21 = L S_D^-1) with T_1, T_2, ... for as
//          many levels as the step's trailing one bits continue;
// the source being the matrix itself when stepid is a power of two and the
// Schur complements held in T_(p-1) otherwise.  A level-l unit is 2^l
// consecutive diagonal blocks; its halves A (first 2^(l-1) blocks) and D.
//
// One workgroup inverts one matrix with everything on chip: M_inv (the
// inverted matrix, whose diagonal band also holds every ◊ and ↑↓ result) and
// the provisional sets T_1..T_K in LDS, each T_l stored compactly as the
// squares of its level-l units, [[S_D, R], [L, S_A]] (the Schur complements
// at the halves' diagonal positions, where their inverses belong).  The input
// is read from HBM where a step takes it as its source.  Every step's
// operations are independent across units and output elements, so the
// workgroup's threads share them; a barrier separates dependent phases, the
// role the paper gives stepid in its thread barriers.
#include <hip/hip_runtime.h>

#include "binv_internal.h"

namespace binv {

namespace {

// det of the b x b (b <= 4) matrix a (row stride 4) by Laplace expansion
// along the first row.
__device__ __forceinline__ double det2(double a, double b, double c, double d) { return a * d - b * c; }

__device__ __forceinline__ double det3(const double (&a)[4][4], int r0, int r1, int r2, int c0, int c1, int c2) {
  return a[r0][c0] * det2(a[r1][c1], a[r1][c2], a[r2][c1], a[r2][c2]) -
         a[r0][c1] * det2(a[r1][c0], a[r1][c2], a[r2][c0], a[r2][c2]) +
         a[r0][c2] * det2(a[r1][c0], a[r1][c1], a[r2][c0], a[r2][c1]);
}

// Closed-form inverse (adjugate over determinant) of a block of order b <= 4
// into inv; returns false when the determinant is exactly zero.
__device__ bool leaf_closed_form(const double (&a)[4][4], int b, double (&inv)[4][4]) {
  if (b == 1) {
    if (a[0][0] == 0.0) return false;
    inv[0][0] = 1.0 / a[0][0];
    return true;
  }
  if (b == 2) {
    const double d = det2(a[0][0], a[0][1], a[1][0], a[1][1]);
    if (d == 0.0) return false;
    inv[0][0] = a[1][1] / d;
    inv[0][1] = -a[0][1] / d;
    inv[1][0] = -a[1][0] / d;
    inv[1][1] = a[0][0] / d;
    return true;
  }
  // cofactor C[i][j] = (-1)^(i+j) det(a without row i and column j);
  // inv[j][i] = C[i][j] / det
  int rows[4][3], cols[4][3];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    int q = 0;
#pragma unroll
    for (int y = 0; y < 4; ++y)
      if (y != x) {
        rows[x][q] = y;
        cols[x][q] = y;
        ++q;
      }
  }
  if (b == 3) {
    double cof[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int i0 = i == 0 ? 1 : 0, i1 = i == 2 ? 1 : 2;
        const int j0 = j == 0 ? 1 : 0, j1 = j == 2 ? 1 : 2;
        const double m = det2(a[i0][j0], a[i0][j1], a[i1][j0], a[i1][j1]);
        cof[i][j] = ((i + j) & 1) ? -m : m;
      }
    const double d = a[0][0] * cof[0][0] + a[0][1] * cof[0][1] + a[0][2] * cof[0][2];
    if (d == 0.0) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) inv[j][i] = cof[i][j] / d;
    return true;
  }
  double cof[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double m = det3(a, rows[i][0], rows[i][1], rows[i][2], cols[j][0], cols[j][1], cols[j][2]);
      cof[i][j] = ((i + j) & 1) ? -m : m;
    }
  const double d = a[0][0] * cof[0][0] + a[0][1] * cof[0][1] + a[0][2] * cof[0][2] + a[0][3] * cof[0][3];
  if (d == 0.0) return false;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) inv[j][i] = cof[i][j] / d;
  return true;
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

}  // namespace

// MMAX: largest order of the launch's matrices; NT threads.  Dynamic LDS:
// M_inv (MMAX^2 doubles, row stride MMAX) then the compact provisional sets
// (tmax doubles, checked on the host).
template <int MMAX, int NT>
__global__ void __launch_bounds__(NT) k_level_scheme(const double* __restrict__ A, double* __restrict__ X,
                                                     const SmallMat* __restrict__ mats,
                                                     const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ bounds, int32_t* __restrict__ info) {
  constexpr int KMAX = ilog2c(MMAX);
  extern __shared__ double lds[];
  double* Minv = lds;
  double* T = lds + MMAX * MMAX;
  __shared__ int bs[MMAX + 1];          // first row of each diagonal block, then m
  __shared__ int rb[MMAX];              // diagonal block of each row
  __shared__ int toff[KMAX + 1][MMAX];  // offset of level-l unit v's square in T
  __shared__ int sing;

  const SmallMat mt = mats[order[blockIdx.x]];
  const int m = mt.m, nk = mt.nb;
  const double* __restrict__ M = A + mt.off;
  const int tid = threadIdx.x;
  if (tid == 0) {
    for (int j = 0; j <= nk; ++j) bs[j] = bounds[mt.bnd + j];
    for (int j = 0; j < nk; ++j)
      for (int r = bs[j]; r < bs[j + 1]; ++r) rb[r] = j;
    int off = 0;
    for (int l = 1; (1 << l) <= nk; ++l)
      for (int v = 0; v < (nk >> l); ++v) {
        toff[l][v] = off;
        const int s = bs[(v + 1) << l] - bs[v << l];
        off += s * s;
      }
    sing = 0x7fffffff;
  }
  __syncthreads();

  // element (r, c) of a step's source: the input matrix (src 0) or the Schur
  // complements held in T_src (r and c lie in one level-src unit)
  auto src_el = [&](int src, int r, int c) -> double {
    if (src == 0) return M[r * m + c];
    const int v = rb[r] >> src;
    const int u0 = bs[v << src];
    const int s = bs[(v + 1) << src] - u0;
    return T[toff[src][v] + (r - u0) * s + (c - u0)];
  };
  // the slot of (r, c) in T_l (r and c in one level-l unit)
  auto t_at = [&](int l, int r, int c) -> double& {
    const int v = rb[r] >> l;
    const int u0 = bs[v << l];
    const int s = bs[(v + 1) << l] - u0;
    return T[toff[l][v] + (r - u0) * s + (c - u0)];
  };
  // The square holding the level-l unit of row (or column) x: element (i, j)
  // of the unit is at base[i * ld + j] for the unit's rows and columns i, j
  // (global indices).  l = 0 names the input matrix itself.  A product's
  // inner index stays inside one unit, so its terms take the unit's square
  // once instead of looking up the unit per term.
  struct Sq {
    const double* base;
    int ld;
  };
  auto square = [&](int l, int x) -> Sq {
    if (l == 0) return Sq{M, m};
    const int v = rb[x] >> l;
    const int u0 = bs[v << l];
    const int s = bs[(v + 1) << l] - u0;
    return Sq{T + toff[l][v] - (int64_t)u0 * s - u0, s};
  };

  const int ns = 2 * nk - 1;
  for (int step = 1; step <= ns; ++step) {
    const int z = __builtin_ctz(step) + 1;  // last non-zero loopid entry
    const int hi = step >> z;
    const int src = hi ? __builtin_ctz(hi) + z : 0;  // T_(p-1), or the input
    if (z > 1) {
      const int l = z - 1;
      // → and ←: R = -A^-1 B (rows of A, columns of D), L = -D^-1 C
      for (int idx = tid; idx < m * m; idx += NT) {
        const int r = idx / m, c = idx - (idx / m) * m;
        const int br = rb[r], bc = rb[c];
        if ((br >> l) != (bc >> l)) continue;
        const int hr = (br >> (l - 1)) & 1, hc = (bc >> (l - 1)) & 1;
        if (hr == hc) continue;
        const int v = br >> l;
        const int k0 = hr == 0 ? bs[v << l] : bs[(v << l) + (1 << (l - 1))];
        const int k1 = hr == 0 ? bs[(v << l) + (1 << (l - 1))] : bs[(v + 1) << l];
        // (k, c) lie in one level-src unit (src > l, or the input)
        const Sq q = square(src, c);
        const double* sc = q.base + c;
        const double* mi = Minv + r * MMAX;
        double acc = 0.0;
        for (int k = k0; k < k1; ++k) acc = fma(mi[k], sc[(int64_t)k * q.ld], acc);
        t_at(l, r, c) = -acc;
      }
      __syncthreads();
      // ∼: S_A = D + C R (rows and columns of D), S_D = A + B L (of A)
      for (int idx = tid; idx < m * m; idx += NT) {
        const int r = idx / m, c = idx - (idx / m) * m;
        const int br = rb[r], bc = rb[c];
        if ((br >> (l - 1)) != (bc >> (l - 1))) continue;
        const int hr = (br >> (l - 1)) & 1;
        const int v = br >> l;
        const int k0 = hr == 1 ? bs[v << l] : bs[(v << l) + (1 << (l - 1))];
        const int k1 = hr == 1 ? bs[(v << l) + (1 << (l - 1))] : bs[(v + 1) << l];
        // (r, k) in one level-src unit, (k, c) in the level-l unit
        const Sq qs = square(src, r);
        const Sq qt = square(l, c);
        const double* sr = qs.base + (int64_t)r * qs.ld;
        const double* tc = qt.base + c;
        double acc = sr[c];
        for (int k = k0; k < k1; ++k) acc = fma(sr[k], tc[(int64_t)k * qt.ld], acc);
        t_at(l, r, c) = acc;
      }
      __syncthreads();
    } else {
      // ◊: every diagonal block of the source, closed form, into M_inv
      for (int j = tid; j < nk; j += NT) {
        const int o = bs[j], b = bs[j + 1] - bs[j];
        double a[4][4], inv[4][4] = {};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) a[i][k] = (i < b && k < b) ? src_el(src, o + i, o + k) : 0.0;
        // a zero determinant: the earliest step, then the lowest block, wins
        if (!leaf_closed_form(a, b, inv)) atomicMin(&sing, step * 65536 + o + 1);
        for (int i = 0; i < b; ++i)
          for (int k = 0; k < b; ++k) Minv[(o + i) * MMAX + o + k] = inv[i][k];
      }
      __syncthreads();
      // ↑↓ with T_1 .. T_(r-1), r the number of trailing one bits of stepid
      const int ones = __builtin_ctz(~step);
      for (int l = 1; l < ones; ++l) {
        for (int idx = tid; idx < m * m; idx += NT) {
          const int r = idx / m, c = idx - (idx / m) * m;
          const int br = rb[r], bc = rb[c];
          if ((br >> l) != (bc >> l)) continue;
          const int hr = (br >> (l - 1)) & 1, hc = (bc >> (l - 1)) & 1;
          if (hr == hc) continue;
          const int v = br >> l;
          // X12 = R S_A^-1 (k over D), X21 = L S_D^-1 (k over A)
          const int k0 = hr == 0 ? bs[(v << l) + (1 << (l - 1))] : bs[v << l];
          const int k1 = hr == 0 ? bs[(v + 1) << l] : bs[(v << l) + (1 << (l - 1))];
          const Sq qt = square(l, r);
          const double* tr = qt.base + (int64_t)r * qt.ld;
          double acc = 0.0;
          for (int k = k0; k < k1; ++k) acc = fma(tr[k], Minv[k * MMAX + c], acc);
          Minv[r * MMAX + c] = acc;
        }
        __syncthreads();
      }
    }
  }
  for (int idx = tid; idx < m * m; idx += NT) {
    const int r = idx / m, c = idx - (idx / m) * m;
    X[mt.off + idx] = Minv[r * MMAX + c];
  }
  if (tid == 0) info[mt.id] = sing == 0x7fffffff ? 0 : (sing & 65535);
}

int level_tier_limit(int t) { return 8 << t; }

size_t level_tier_tmax(int t) {
  const size_t mm = (size_t)level_tier_limit(t) * level_tier_limit(t);
  return mm * 5 / 2;
}

size_t level_tier_lds(int t) { return sizeof(double) * ((size_t)level_tier_limit(t) * level_tier_limit(t) + level_tier_tmax(t)); }

hipError_t launch_level_tier(int tier, const double* A, double* X, const SmallMat* mats, const int32_t* order,
                             int64_t count, const int32_t* bounds, int32_t* info, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t lds = level_tier_lds(tier);
  const dim3 grid((unsigned)count);
  switch (tier) {
    case 0: hipLaunchKernelGGL((k_level_scheme<8, 64>), grid, dim3(64), lds, s, A, X, mats, order, bounds, info); break;
    case 1: hipLaunchKernelGGL((k_level_scheme<16, 64>), grid, dim3(64), lds, s, A, X, mats, order, bounds, info); break;
    case 2: hipLaunchKernelGGL((k_level_scheme<32, 128>), grid, dim3(128), lds, s, A, X, mats, order, bounds, info); break;
    case 3: {
      // more than 64 KB of dynamic LDS: raise the kernel's limit once
      static const hipError_t attr = hipFuncSetAttribute(
          reinterpret_cast<const void*>(&k_level_scheme<64, 256>), hipFuncAttributeMaxDynamicSharedMemorySize,
          (int)level_tier_lds(3));
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL((k_level_scheme<64, 256>), grid, dim3(256), lds, s, A, X, mats, order, bounds, info);
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace binv
