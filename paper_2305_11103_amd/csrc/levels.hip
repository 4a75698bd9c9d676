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
//
// Work sharing: each row of the matrix has a group of threads, and in every
// product phase a row's outputs form one contiguous column range (the other
// half, or its own half, of the row's unit at the phase's level), so a group
// walks only the outputs that exist.  The closed-form inverses take one
// thread per block element.  M_inv's two off-diagonal blocks of the top
// level are written once, by the last step's ↑↓, and never read, so they go
// straight to the output and LDS holds only its two top-level diagonal
// squares (in the classes above order 32, where LDS bounds the occupancy).
// A launch's LDS is the largest a^2 + d^2 + |T_1..T_K| of its matrices (a,
// d the top-level halves' orders; m^2 + |T| without the split), and orders
// are launched in classes whose LDS lets 4, 3 or 2 workgroups share a CU.
#include <hip/hip_runtime.h>

#include "binv_internal.h"

namespace binv {

namespace {

__device__ __forceinline__ double det2(double a, double b, double c, double d) { return a * d - b * c; }

// det of the 3 x 3 matrix with elements e(x, y), expanded along its first row
template <class E>
__device__ __forceinline__ double det3(E e) {
  return e(0, 0) * det2(e(1, 1), e(1, 2), e(2, 1), e(2, 2)) - e(0, 1) * det2(e(1, 0), e(1, 2), e(2, 0), e(2, 2)) +
         e(0, 2) * det2(e(1, 0), e(1, 1), e(2, 0), e(2, 1));
}

// Element (i, k) of the closed-form inverse (adjugate over determinant) of
// the block of order b <= 4 whose element (r, c) is el(r, c): the cofactor of
// (k, i) over the determinant, which is expanded along the block's first row.
// *d receives the determinant (every element's thread computes the same one;
// a zero determinant leaves the element undefined).
template <class El>
__device__ double leaf_element(El el, int b, int i, int k, double* d) {
  if (b == 1) {
    *d = el(0, 0);
    return 1.0 / el(0, 0);
  }
  if (b == 2) {
    const double dd = det2(el(0, 0), el(0, 1), el(1, 0), el(1, 1));
    *d = dd;
    // [[a11, -a01], [-a10, a00]] / d
    const double num = i == k ? el(1 - i, 1 - i) : -el(i, k);
    return num / dd;
  }
  if (b == 3) {
    // cofactor (p, q): the signed det of the rows other than p and the
    // columns other than q, in ascending order
    auto cof = [&](int p, int q) {
      const int p0 = p == 0 ? 1 : 0, p1 = p == 2 ? 1 : 2;
      const int q0 = q == 0 ? 1 : 0, q1 = q == 2 ? 1 : 2;
      const double mnr = det2(el(p0, q0), el(p0, q1), el(p1, q0), el(p1, q1));
      return ((p + q) & 1) ? -mnr : mnr;
    };
    const double dd = el(0, 0) * cof(0, 0) + el(0, 1) * cof(0, 1) + el(0, 2) * cof(0, 2);
    *d = dd;
    return cof(k, i) / dd;
  }
  auto cof = [&](int p, int q) {
    const int p0 = p == 0 ? 1 : 0, p1 = p <= 1 ? 2 : 1, p2 = p <= 2 ? 3 : 2;
    const int q0 = q == 0 ? 1 : 0, q1 = q <= 1 ? 2 : 1, q2 = q <= 2 ? 3 : 2;
    const double mnr = det3([&](int x, int y) {
      return el(x == 0 ? p0 : x == 1 ? p1 : p2, y == 0 ? q0 : y == 1 ? q1 : q2);
    });
    return ((p + q) & 1) ? -mnr : mnr;
  };
  const double dd = el(0, 0) * cof(0, 0) + el(0, 1) * cof(0, 1) + el(0, 2) * cof(0, 2) + el(0, 3) * cof(0, 3);
  *d = dd;
  return cof(k, i) / dd;
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

}  // namespace

// MMAX: largest order of the launch's matrices; NT threads; at least WPE
// waves per SIMD (bounds the registers so that the class's workgroups fit a
// CU together); SPLIT: M_inv's top-level off-diagonal blocks go straight to
// the output.  Dynamic LDS: M_inv's top-level diagonal squares (a^2 then d^2
// doubles; the whole m^2 without SPLIT) and the compact provisional sets
// (sized on the host from the launch's partitions).
template <int MMAX, int NT, int WPE, bool SPLIT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) k_level_scheme(const double* __restrict__ A, double* __restrict__ X,
                                                     const SmallMat* __restrict__ mats,
                                                     const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ bounds, int32_t* __restrict__ info) {
  constexpr int KMAX = ilog2c(MMAX);
  constexpr int UMAX = MMAX / 2 > 0 ? MMAX / 2 : 1;  // units per level (levels >= 1)
  extern __shared__ double lds[];
  __shared__ int bs[MMAX + 1];          // first row of each diagonal block, then m
  __shared__ int rb[MMAX];              // diagonal block of each row
  __shared__ int toff[KMAX + 1][UMAX];  // offset of level-l unit v's square in T
  __shared__ int sing;

  const SmallMat mt = mats[order[blockIdx.x]];
  const int m = mt.m, nk = mt.nb;
  const double* __restrict__ M = A + mt.off;
  double* __restrict__ Xm = X + mt.off;
  const int tid = threadIdx.x;
  for (int j = tid; j <= nk; j += NT) bs[j] = bounds[mt.bnd + j];
  if (tid == 0) sing = 0x7fffffff;
  __syncthreads();
  for (int j = tid; j < nk; j += NT)
    for (int r = bs[j]; r < bs[j + 1]; ++r) rb[r] = j;
  if (tid == 0) {
    int off = 0;
    for (int l = 1; (1 << l) <= nk; ++l)
      for (int v = 0; v < (nk >> l); ++v) {
        toff[l][v] = off;
        const int s = bs[(v + 1) << l] - bs[v << l];
        off += s * s;
      }
  }
  __syncthreads();

  // Each row r < m has G threads (lane g of them).
  const int G = NT / m;
  const int r = tid / G, g = tid - r * G;
  const bool row = r < m;

  // M_inv: the top level's halves [0, ha) and [ha, m) (one square if N_k =
  // 1 or without SPLIT); for x in one half, minv(x)[y] is element (x, y)
  // with y in that half.  K: the level whose ↑↓ goes to the output (none
  // without SPLIT).
  const int K = SPLIT ? 31 - __builtin_clz(nk) : -1;
  const int ha = (SPLIT && nk >= 2) ? bs[nk >> 1] : m, hd = m - ha;
  double* MinvA = lds;
  double* MinvD = lds + ha * ha;
  double* T = MinvD + hd * hd;
  auto minv = [&](int x) -> double* { return x < ha ? MinvA + x * ha : MinvD + (x - ha) * hd - ha; };

  // The square holding the level-l unit of row (or column) x: element (i, j)
  // of the unit is at base[i * ld + j] for the unit's rows and columns i, j
  // (global indices).  l = 0 names the input matrix itself.
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
  // Row r's level-l unit (l >= 1): its rows u0..u1-1, halves A = u0..uh-1
  // and D = uh..u1-1, and its square in T_l (element (i, j) at sq[i * s + j]).
  struct Unit {
    int u0, uh, u1, s;
    bool inA;
    double* sq;
  };
  auto unit = [&](int l) -> Unit {
    const int v = rb[r] >> l;
    Unit u;
    u.u0 = bs[v << l];
    u.uh = bs[(v << l) + (1 << (l - 1))];
    u.u1 = bs[(v + 1) << l];
    u.s = u.u1 - u.u0;
    u.inA = r < u.uh;
    u.sq = T + toff[l][v] - (int64_t)u.u0 * u.s - u.u0;
    return u;
  };

  const int ns = 2 * nk - 1;
  for (int step = 1; step <= ns; ++step) {
    const int z = __builtin_ctz(step) + 1;  // last non-zero loopid entry
    const int hi = step >> z;
    const int src = hi ? __builtin_ctz(hi) + z : 0;  // T_(p-1), or the input
    if (z > 1) {
      const int l = z - 1;
      if (row) {
        // → and ←: R = -A^-1 B (rows of A, columns of D), L = -D^-1 C; the
        // sum runs over the row's own half, whose inverse M_inv holds
        const Unit u = unit(l);
        const int c0 = u.inA ? u.uh : u.u0, c1 = u.inA ? u.u1 : u.uh;
        const int k0 = u.inA ? u.u0 : u.uh, k1 = u.inA ? u.uh : u.u1;
        // B and C lie in the row's level-src unit (src > l), or the input
        const Sq q = square(src, r);
        const double* mi = minv(r);
        double* out = u.sq + (int64_t)r * u.s;
        for (int c = c0 + g; c < c1; c += G) {
          const double* sc = q.base + c;
          double acc = 0.0;
          for (int k = k0; k < k1; ++k) acc = fma(mi[k], sc[(int64_t)k * q.ld], acc);
          out[c] = -acc;
        }
      }
      __syncthreads();
      if (row) {
        // ∼: S_A = D + C R (rows and columns of D), S_D = A + B L (of A);
        // the sum runs over the other half
        const Unit u = unit(l);
        const int c0 = u.inA ? u.u0 : u.uh, c1 = u.inA ? u.uh : u.u1;
        const int k0 = u.inA ? u.uh : u.u0, k1 = u.inA ? u.u1 : u.uh;
        const Sq q = square(src, r);
        const double* sr = q.base + (int64_t)r * q.ld;
        double* out = u.sq + (int64_t)r * u.s;
        for (int c = c0 + g; c < c1; c += G) {
          const double* tc = u.sq + c;
          double acc = sr[c];
          for (int k = k0; k < k1; ++k) acc = fma(sr[k], tc[(int64_t)k * u.s], acc);
          out[c] = acc;
        }
      }
      __syncthreads();
    } else {
      // ◊: every diagonal block of the source, closed form, into M_inv, one
      // thread per block element
      for (int slot = tid; slot < nk * 16; slot += NT) {
        const int j = slot >> 4, i = (slot >> 2) & 3, k = slot & 3;
        const int o = bs[j], b = bs[j + 1] - o;
        if (i >= b || k >= b) continue;
        const Sq q = square(src, o);
        const double* blk = q.base + (int64_t)o * q.ld + o;
        const int ld = q.ld;
        double d;
        const double x = leaf_element([&](int y, int w) { return blk[(int64_t)y * ld + w]; }, b, i, k, &d);
        // a zero determinant: the earliest step, then the lowest block, wins
        if (d == 0.0) {
          if (i == 0 && k == 0) atomicMin(&sing, step * 65536 + o + 1);
        } else {
          minv(o + i)[o + k] = x;
        }
      }
      __syncthreads();
      // ↑↓ with T_1 .. T_(r-1), r the number of trailing one bits of stepid:
      // X12 = R S_A^-1, X21 = L S_D^-1, the sum over the other half; the top
      // level's (last step only) goes to the output
      const int ones = __builtin_ctz(~step);
      for (int l = 1; l < ones; ++l) {
        if (row) {
          const Unit u = unit(l);
          const int c0 = u.inA ? u.uh : u.u0, c1 = u.inA ? u.u1 : u.uh;
          const double* tr = u.sq + (int64_t)r * u.s;
          double* dst = l == K ? Xm + (int64_t)r * m : minv(r);
          for (int c = c0 + g; c < c1; c += G) {
            double acc = 0.0;
            for (int k = c0; k < c1; ++k) acc = fma(tr[k], minv(k)[c], acc);
            dst[c] = acc;
          }
        }
        // nothing reads the top level's blocks: no barrier (and no wait for
        // their stores) after them
        if (l != K) __syncthreads();
      }
    }
  }
  // the top-level diagonal squares (the off-diagonal blocks are written)
  if (row) {
    const int c0 = r < ha ? 0 : ha, c1 = r < ha ? ha : m;
    const double* src_row = minv(r);
    for (int c = c0 + g; c < c1; c += G) Xm[(int64_t)r * m + c] = src_row[c];
  }
  if (tid == 0) info[mt.id] = sing == 0x7fffffff ? 0 : (sing & 65535);
}

namespace {

// Launch classes: orders <= kLimit[c].  The classes above 32 split orders
// 33..64 where their LDS (a^2 + d^2 + |T|, about 2.4 m^2 doubles with Table
// 2's partitions) lets 4, 3 and 2 workgroups share a CU.  Threads and the
// register bound per class are the measured best (a bound that makes the
// kernel spill cost more than the occupancy it buys at orders <= 8 and
// 53..64).
constexpr int kLimit[kLevelClasses] = {8, 16, 32, 45, 52, 64};

template <int MMAX, int NT, int WPE, bool SPLIT>
hipError_t launch_one(dim3 grid, size_t lds, hipStream_t s, const double* A, double* X, const SmallMat* mats,
                      const int32_t* order, const int32_t* bounds, int32_t* info) {
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_level_scheme<MMAX, NT, WPE, SPLIT>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(kLevelLdsDoubles * sizeof(double)));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_level_scheme<MMAX, NT, WPE, SPLIT>), grid, dim3(NT), lds, s, A, X, mats, order, bounds, info);
  return hipSuccess;
}

}  // namespace

int level_class_limit(int c) { return kLimit[c]; }

bool level_class_split(int c) { return kLimit[c] > 32; }

hipError_t launch_level_class(int c, const double* A, double* X, const SmallMat* mats, const int32_t* order,
                              int64_t count, size_t lds_doubles, const int32_t* bounds, int32_t* info,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (lds_doubles > kLevelLdsDoubles) return hipErrorInvalidValue;
  const size_t lds = lds_doubles * sizeof(double);
  const dim3 grid((unsigned)count);
  hipError_t e;
  switch (c) {
    case 0: e = launch_one<8, 64, 4, false>(grid, lds, s, A, X, mats, order, bounds, info); break;
    case 1: e = launch_one<16, 128, 8, false>(grid, lds, s, A, X, mats, order, bounds, info); break;
    case 2: e = launch_one<32, 256, 8, false>(grid, lds, s, A, X, mats, order, bounds, info); break;
    case 3: e = launch_one<64, 512, 8, true>(grid, lds, s, A, X, mats, order, bounds, info); break;
    case 4: e = launch_one<64, 512, 6, true>(grid, lds, s, A, X, mats, order, bounds, info); break;
    case 5: e = launch_one<64, 512, 4, true>(grid, lds, s, A, X, mats, order, bounds, info); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace binv
