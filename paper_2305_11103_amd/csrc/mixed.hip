// Mixed-precision blockwise inversion: the Schur-complement sweep (Eq. (a) of
// §3, applied in place block by block as in §4.2) on an FP32 working copy,
// with every pivot block inverted in FP64, followed by FP64 Newton-Schulz
// refinement X <- X + X (I - A X) on the original FP64 matrix.
//
// Kernels here: FP64 <-> FP32 conversion, the FP32 column-panel save, the
// FP32 step GEMM (row panel and Schur update on MFMA v_mfma_f32_16x16x4_f32
// with FP32 accumulation) and a deterministic sum of squares for the residual
// norm.  v_mfma_f32_16x16x4_f32 lane layout (measured): A lane l holds
// A[l%16][l/16], B lane l holds B[l/16][l%16], and output register q of lane l
// holds D[F32_ROW(l, q)][l%16].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "binv_internal.h"

#ifndef F32_ROW
#define F32_ROW(l, q) (4 * ((l) >> 4) + (q))
#endif

namespace binv {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_f64_to_f32(const double* __restrict__ S, int64_t lds, float* __restrict__ D,
                                                    int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t i = blockIdx.y;
  if (i >= rows) return;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < cols; j += (int64_t)gridDim.x * 256)
    D[i * ldd + j] = (float)S[i * lds + j];
}

__global__ void __launch_bounds__(256) k_f32_to_f64(const float* __restrict__ S, int64_t lds, double* __restrict__ D,
                                                    int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t i = blockIdx.y;
  if (i >= rows) return;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < cols; j += (int64_t)gridDim.x * 256)
    D[i * ldd + j] = (double)S[i * lds + j];
}

// Ct[t][i] = W[i][o + t] (FP32 column panel, k-major)
__global__ void __launch_bounds__(256) k_col_save_f32(const float* __restrict__ W, int64_t ldw, int64_t n, int64_t o,
                                                      int b, float* __restrict__ Ct, int64_t ldc) {
  __shared__ float tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int t0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r;
    const int t = t0 + tx;
    tile[r][tx] = (i < n && t < b) ? W[i * ldw + o + t] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int t = t0 + r;
    const int64_t i = i0 + tx;
    if (t < b && i < n) Ct[(int64_t)t * ldc + i] = tile[tx][r];
  }
}

struct StepArgs32 {
  const float* A;  // row panel: P (m-major, lda); Schur: Ct (k-major, lda)
  int64_t lda;
  const float* B;  // k-major rows
  int64_t ldb;
  float* W;        // output (R for the row panel, W in place for the Schur update)
  int64_t ldw;
  const float* R;  // Schur: row panel; row panel: P
  int64_t ldr;
  int64_t M, N;
  int K;
  int64_t o;
  int b;
};

enum { M32_ROW = 0, M32_SCHUR = 1 };

// 128 x 128 tile, 4 waves of 64 x 64, K chunks of 16 double-buffered in LDS.
template <int MODE, bool A_KMAJOR>
__global__ void __launch_bounds__(256, 2) k_gemm_step_f32(StepArgs32 g) {
  constexpr int BM = 128, BN = 128, BK = 16, PAD = 4, LA = BM + PAD, LB = BN + PAD;
  constexpr int WM = 64, WN = 64, TR = WM / 16, TC = WN / 16;
  constexpr int NT = 256;
  constexpr int AE = BK * BM / NT, BE = BK * BN / NT;  // floats per thread per chunk
  __shared__ float As[2][BK * LA];
  __shared__ float Bs[2][BK * LB];
  const int64_t TM = (g.M + BM - 1) / BM, TN = (g.N + BN - 1) / BN;
  const int64_t T = TM * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
    const int64_t tm = t / TN, tn = t % TN;
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int64_t o = g.o;
    const int b = g.b;
    bool need = true;
    if (MODE == M32_SCHUR) {
      if (m0 >= o && m0 + BM <= o + b) need = false;
    } else {
      if (n0 >= o && n0 + BN <= o + b) need = false;
    }
    f32x4 acc[TR][TC];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
      for (int c = 0; c < TC; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (need) {
      const int K = g.K;
      const int nk = (K + BK - 1) / BK;
      float ra[AE], rb[BE];
      auto gload = [&](int kc) {
        const int k0 = kc * BK;
#pragma unroll
        for (int e = 0; e < AE; ++e) {
          const int idx = tid + e * NT;
          int kk, mm;
          if (A_KMAJOR) { kk = idx / BM; mm = idx % BM; }
          else { mm = idx / BK; kk = idx % BK; }
          const int64_t gm = m0 + mm;
          const int gk = k0 + kk;
          ra[e] = (gm < g.M && gk < K) ? (A_KMAJOR ? g.A[(int64_t)gk * g.lda + gm] : g.A[gm * g.lda + gk]) : 0.f;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
          const int idx = tid + e * NT;
          const int kk = idx / BN, nn = idx % BN;
          const int64_t gn = n0 + nn;
          const int gk = k0 + kk;
          rb[e] = (gn < g.N && gk < K) ? g.B[(int64_t)gk * g.ldb + gn] : 0.f;
        }
      };
      auto sstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
          const int idx = tid + e * NT;
          int kk, mm;
          if (A_KMAJOR) { kk = idx / BM; mm = idx % BM; }
          else { mm = idx / BK; kk = idx % BK; }
          As[buf][kk * LA + mm] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
          const int idx = tid + e * NT;
          const int kk = idx / BN, nn = idx % BN;
          Bs[buf][kk * LB + nn] = rb[e];
        }
      };
      gload(0);
      sstore(0);
      __syncthreads();
      const int lk = lane >> 4, lr = lane & 15;
      for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) gload(kc + 1);
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
          float fa[TR], fb[TC];
#pragma unroll
          for (int r = 0; r < TR; ++r) fa[r] = As[buf][(k4 * 4 + lk) * LA + wm * WM + r * 16 + lr];
#pragma unroll
          for (int c = 0; c < TC; ++c) fb[c] = Bs[buf][(k4 * 4 + lk) * LB + wn * WN + c * 16 + lr];
#pragma unroll
          for (int r = 0; r < TR; ++r)
#pragma unroll
            for (int c = 0; c < TC; ++c) acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[r], fb[c], acc[r][c], 0, 0, 0);
        }
        if (kc + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
      }
    }
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
      for (int c = 0; c < TC; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t i = m0 + wm * WM + r * 16 + F32_ROW(lane, q);
          const int64_t j = n0 + wn * WN + c * 16 + (lane & 15);
          if (i >= g.M || j >= g.N) continue;
          const bool jp = (j >= o && j < o + b);
          if (MODE == M32_ROW) {
            g.W[i * g.ldw + j] = jp ? g.R[i * g.ldr + (j - o)] : acc[r][c][q];
          } else {
            const bool ip = (i >= o && i < o + b);
            float* dst = &g.W[i * g.ldw + j];
            if (ip) *dst = g.R[(i - o) * g.ldr + j];
            else *dst = (jp ? 0.f : *dst) - acc[r][c][q];
          }
        }
  }
}

// Deterministic sum of squares: fixed-size partials, then one final sum.
__global__ void __launch_bounds__(256) k_sumsq_partial(const double* __restrict__ R, int64_t ldr, int64_t rows,
                                                       int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t total = rows * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e - i * n;
    const double x = R[i * ldr + j];
    acc = fma(x, x, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_final(const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

constexpr int kSumParts = 1024;

hipError_t launch_sum_final(const double* part, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part, np, out);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* S, int64_t lds, float* D, int64_t ldd, int64_t rows, int64_t cols,
                             hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  unsigned gx = (unsigned)((cols + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(gx, (unsigned)rows), dim3(256), 0, s, S, lds, D, ldd, rows, cols);
  return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                             hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  unsigned gx = (unsigned)((cols + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_f32_to_f64, dim3(gx, (unsigned)rows), dim3(256), 0, s, S, lds, D, ldd, rows, cols);
  return hipGetLastError();
}

hipError_t launch_col_save_f32(const float* W, int64_t ldw, int64_t n, int64_t o, int b, float* Ct, int64_t ldc,
                               hipStream_t s) {
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((b + 31) / 32));
  hipLaunchKernelGGL(k_col_save_f32, grid, dim3(256), 0, s, W, ldw, n, o, b, Ct, ldc);
  return hipGetLastError();
}

static unsigned grid_for(int64_t M, int64_t N) {
  const int64_t T = ((M + 127) / 128) * ((N + 127) / 128);
  return (unsigned)(T < 4096 ? (T > 0 ? T : 1) : 4096);
}

// R (b x n) = P (b x b, m-major) * W[o:o+b, :], R[:, o:o+b] = P  (FP32)
hipError_t launch_row_panel_f32(const float* P, int64_t ldp, const float* W, int64_t ldw, int64_t n, int64_t o, int b,
                                float* R, int64_t ldr, hipStream_t s) {
  StepArgs32 g{P, ldp, W + o * ldw, ldw, R, ldr, P, ldp, (int64_t)b, n, b, o, b};
  hipLaunchKernelGGL((k_gemm_step_f32<M32_ROW, false>), dim3(grid_for(b, n)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// W (n x n, in place) Schur update from Ct (b x n, k-major) and R (b x n)  (FP32)
hipError_t launch_schur_f32(const float* Ct, int64_t ldc, const float* R, int64_t ldr, float* W, int64_t ldw, int64_t n,
                            int64_t o, int b, hipStream_t s) {
  StepArgs32 g{Ct, ldc, R, ldr, W, ldw, R, ldr, n, n, b, o, b};
  hipLaunchKernelGGL((k_gemm_step_f32<M32_SCHUR, true>), dim3(grid_for(n, n)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// out = sum of squares of the n x n matrix R (part: kSumParts doubles of scratch)
hipError_t launch_sumsq(const double* R, int64_t ldr, int64_t rows, int64_t cols, double* part, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_partial, dim3(kSumParts), dim3(256), 0, s, R, ldr, rows, cols, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part, kSumParts, out);
  return hipGetLastError();
}

}  // namespace binv
