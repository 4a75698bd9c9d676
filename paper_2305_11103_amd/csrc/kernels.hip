// HIP kernels (gfx950) for in-place blockwise inversion.
//
// One elimination step for diagonal block p (rows/columns [o, o+b)) of the
// working matrix W (row-major, leading dimension ldw) is, following Eq. (a)
// of §3 applied in place as in §4.2:
//
//   k_leaf_inverse   P = W_pp^-1 by Gauss-Jordan with partial pivoting inside
//                    the block, held entirely in LDS (b <= 128).
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

namespace binv {

constexpr int kNT = 256;        // threads per workgroup in the GEMM and leaf kernels
constexpr int kLeafMax = 128;   // largest pivot block the LDS leaf kernel holds

// ---------------------------------------------------------------------------
// Leaf: Gauss-Jordan with partial pivoting on a b x b block in LDS.
// ---------------------------------------------------------------------------
// A (lda): the block, read only.  P (ldp): receives the inverse.
// info: set (first writer wins) to row0 + c + 1 when the pivot of column c is
// exactly zero; the block's output is then undefined.
template <int BMAX>
__global__ void __launch_bounds__(kNT) k_leaf_inverse(const double* __restrict__ A, int64_t lda,
                                                      double* __restrict__ P, int64_t ldp, int b,
                                                      int64_t row0, long long* info) {
  constexpr int LD = BMAX + 1;
  __shared__ double W[BMAX * LD];
  __shared__ double fcol[BMAX];
  __shared__ int perm[BMAX];
  __shared__ int colmap[BMAX];
  __shared__ int s_piv;
  __shared__ double s_pval;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int NW = kNT / 64;

  for (int e = tid; e < b * b; e += kNT) {
    int i = e / b, j = e - i * b;
    W[i * LD + j] = A[(int64_t)i * lda + j];
  }
  __syncthreads();

  bool singular = false;
  for (int c = 0; c < b; ++c) {
    // pivot search on column c, rows c..b-1: wave 0, lowest row wins ties
    if (wave == 0) {
      double best = -1.0;
      int bi = BMAX;
      for (int i = c + lane; i < b; i += 64) {
        double v = fabs(W[i * LD + c]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(best, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (lane == 0) {
        s_piv = bi;
        s_pval = W[bi * LD + c];
        perm[c] = bi;
      }
    }
    __syncthreads();
    const int r = s_piv;
    const double pv = s_pval;
    if (pv == 0.0) {
      if (tid == 0) atomicCAS((unsigned long long*)info, 0ULL, (unsigned long long)(row0 + c + 1));
      singular = true;
      break;
    }
    if (r != c) {
      for (int j = tid; j < b; j += kNT) {
        double t = W[c * LD + j];
        W[c * LD + j] = W[r * LD + j];
        W[r * LD + j] = t;
      }
      __syncthreads();
    }
    const double q = 1.0 / pv;
    // save column c (multipliers) and scale the pivot row; its column-c slot becomes q
    for (int i = tid; i < b; i += kNT) fcol[i] = (i == c) ? 0.0 : W[i * LD + c];
    for (int j = tid; j < b; j += kNT) W[c * LD + j] = (j == c ? 1.0 : W[c * LD + j]) * q;
    __syncthreads();
    // eliminate column c from every other row; column c receives -f q
    for (int i = wave; i < b; i += NW) {
      if (i == c) continue;
      const double f = fcol[i];
      for (int j = lane; j < b; j += 64) {
        double w = (j == c) ? 0.0 : W[i * LD + j];
        W[i * LD + j] = w - f * W[c * LD + j];
      }
    }
    __syncthreads();
  }
  if (singular) return;
  // undo the row interchanges as column interchanges in reverse order:
  // final[:, j] = W[:, colmap[j]]
  if (tid == 0) {
    for (int j = 0; j < b; ++j) colmap[j] = j;
    for (int c = b - 1; c >= 0; --c) {
      int r = perm[c];
      int t = colmap[c];
      colmap[c] = colmap[r];
      colmap[r] = t;
    }
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += kNT) {
    int i = e / b, j = e - i * b;
    P[(int64_t)i * ldp + j] = W[i * LD + colmap[j]];
  }
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

__global__ void k_zero_i64(long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// ---------------------------------------------------------------------------
// GEMM step kernel.
// ---------------------------------------------------------------------------
enum { MODE_ROW = 0, MODE_SCHUR = 1 };

typedef double dbl;

struct StepArgs {
  // operand A of the contraction, k-major (A_km[t][m]) or m-major (A_mm[m][t])
  const double* A;
  int64_t lda;
  // operand B, k-major: B[t][j]
  const double* B;
  int64_t ldb;
  // output: MODE_ROW -> R (ldr); MODE_SCHUR -> W in place (ldw) and copy rows from R
  double* W;
  int64_t ldw;
  const double* R;   // row panel (MODE_SCHUR) or pivot inverse P (MODE_ROW, ld = ldp)
  int64_t ldr;
  int64_t M, N;      // output extent
  int K;             // contraction length (= b)
  int64_t o;         // first row/column of block p
  int b;             // order of block p
};

template <int MODE, int BM, int BN, bool A_KMAJOR>
__global__ void __launch_bounds__(kNT, (BM * BN >= 128 * 128) ? 1 : 2) k_gemm_step(StepArgs g) {
  constexpr int BK = 16;
  constexpr int PAD = 4;
  constexpr int LA = BM + PAD;
  constexpr int LB = BN + PAD;
  constexpr int WM = BM / 2, WN = BN / 2;   // 2 x 2 waves
  constexpr int RG = WM / 4, CG = WN / 16;  // 4x16 MFMA tiles per wave
  constexpr int A_ELEMS = BK * BM / kNT;    // per-thread global loads per chunk
  constexpr int B_ELEMS = BK * BN / kNT;
  __shared__ double As[2][BK * LA];
  __shared__ double Bs[2][BK * LB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  const int64_t o = g.o;
  const int b = g.b;

  // Does this tile need the contraction at all?
  bool need = true;
  if (MODE == MODE_SCHUR) {
    // rows entirely inside block p are a pure copy of R
    if (m0 >= o && m0 + BM <= o + b) need = false;
  } else {
    // columns entirely inside block p are a copy of P
    if (n0 >= o && n0 + BN <= o + b) need = false;
  }

  dbl acc[RG][CG];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int c = 0; c < CG; ++c) acc[r][c] = 0.0;

  if (need) {
    double ra[A_ELEMS], rb[B_ELEMS];
    const int K = g.K;
    const int nk = (K + BK - 1) / BK;

    auto gload = [&](int kc) {
      const int k0 = kc * BK;
#pragma unroll
      for (int e = 0; e < A_ELEMS; ++e) {
        const int idx = tid + e * kNT;
        int kk, mm;
        if (A_KMAJOR) { kk = idx / BM; mm = idx % BM; }
        else { mm = idx / BK; kk = idx % BK; }
        const int64_t gm = m0 + mm;
        const int gk = k0 + kk;
        double v = 0.0;
        if (gm < g.M && gk < K)
          v = A_KMAJOR ? g.A[(int64_t)gk * g.lda + gm] : g.A[gm * g.lda + gk];
        ra[e] = v;
      }
#pragma unroll
      for (int e = 0; e < B_ELEMS; ++e) {
        const int idx = tid + e * kNT;
        const int kk = idx / BN, nn = idx % BN;
        const int64_t gn = n0 + nn;
        const int gk = k0 + kk;
        rb[e] = (gn < g.N && gk < K) ? g.B[(int64_t)gk * g.ldb + gn] : 0.0;
      }
    };
    auto sstore = [&](int buf) {
#pragma unroll
      for (int e = 0; e < A_ELEMS; ++e) {
        const int idx = tid + e * kNT;
        int kk, mm;
        if (A_KMAJOR) { kk = idx / BM; mm = idx % BM; }
        else { mm = idx / BK; kk = idx % BK; }
        As[buf][kk * LA + mm] = ra[e];
      }
#pragma unroll
      for (int e = 0; e < B_ELEMS; ++e) {
        const int idx = tid + e * kNT;
        const int kk = idx / BN, nn = idx % BN;
        Bs[buf][kk * LB + nn] = rb[e];
      }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    const int lk = lane >> 4;       // k row this lane feeds
    const int lm = lane & 3;        // A row within a 4-row group
    const int ln = lane & 15;       // B column within a 16-column group
    for (int kc = 0; kc < nk; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nk) gload(kc + 1);
      const double* as = &As[buf][0];
      const double* bs = &Bs[buf][0];
#pragma unroll
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
      const bool jp = (j >= o && j < o + b);
      if (MODE == MODE_ROW) {
        // R[i][j] = P[i][j - o] for the block's own columns, else (P W_p)[i][j]
        g.W[i * g.ldw + j] = jp ? g.R[i * g.ldr + (j - o)] : acc[r][c];
      } else {
        const bool ip = (i >= o && i < o + b);
        double* dst = &g.W[i * g.ldw + j];
        if (ip) {
          *dst = g.R[(i - o) * g.ldr + j];
        } else {
          const double w = jp ? 0.0 : *dst;
          *dst = w - acc[r][c];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C ABI implementation).
// ---------------------------------------------------------------------------
hipError_t launch_leaf_inverse(const double* A, int64_t lda, double* P, int64_t ldp, int b, int64_t row0,
                               long long* info, hipStream_t s) {
  if (b <= 64)
    hipLaunchKernelGGL((k_leaf_inverse<64>), dim3(1), dim3(kNT), 0, s, A, lda, P, ldp, b, row0, info);
  else
    hipLaunchKernelGGL((k_leaf_inverse<kLeafMax>), dim3(1), dim3(kNT), 0, s, A, lda, P, ldp, b, row0, info);
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

hipError_t launch_zero_info(long long* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

template <int MODE, int BM, int BN, bool AK>
static hipError_t launch_step(const StepArgs& g, hipStream_t s) {
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM));
  hipLaunchKernelGGL((k_gemm_step<MODE, BM, BN, AK>), grid, dim3(kNT), 0, s, g);
  return hipGetLastError();
}

// Row panel: R (b x n, ldr) = P (b x b, m-major, ldp) * W[o:o+b, :], with R[:, o:o+b] = P.
hipError_t launch_row_panel(const double* P, int64_t ldp, const double* W, int64_t ldw, int64_t n, int64_t o, int b,
                            double* R, int64_t ldr, hipStream_t s) {
  StepArgs g;
  g.A = P; g.lda = ldp;
  g.B = W + o * ldw; g.ldb = ldw;
  g.W = R; g.ldw = ldr;
  g.R = P; g.ldr = ldp;
  g.M = b; g.N = n; g.K = b; g.o = o; g.b = b;
  if (n >= 2048) return launch_step<MODE_ROW, 128, 128, false>(g, s);
  return launch_step<MODE_ROW, 64, 64, false>(g, s);
}

// Schur trailing update in place on W using the saved column panel Ct (b x n,
// k-major) and the row panel R (b x n).
hipError_t launch_schur(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* W, int64_t ldw, int64_t n,
                        int64_t o, int b, hipStream_t s) {
  StepArgs g;
  g.A = Ct; g.lda = ldc;
  g.B = R; g.ldb = ldr;
  g.W = W; g.ldw = ldw;
  g.R = R; g.ldr = ldr;
  g.M = n; g.N = n; g.K = b; g.o = o; g.b = b;
  if (n >= 2048) return launch_step<MODE_SCHUR, 128, 128, true>(g, s);
  return launch_step<MODE_SCHUR, 64, 64, true>(g, s);
}

}  // namespace binv
