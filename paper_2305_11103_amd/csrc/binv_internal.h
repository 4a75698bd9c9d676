// Internal declarations shared by the library's translation units: the
// argument records the kernels read and the launchers the host code calls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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
  int64_t o;          // first row/column of block p
  int b;              // order of block p
  // tile subset (Schur update): 0 = every tile; 1 = the band of tile-rows
  // [tr0, tr1] and tile-columns [tc0, tc1] (the next block's rows and
  // columns); 2 = every tile outside that band.
  int region;
  int64_t tr0, tr1, tc0, tc1;
  int64_t ntiles;     // tiles enumerated by the region (before band skipping)
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

// One column-panel save of a batch.
struct ColJob {
  const double* W;
  int64_t ldw;
  int64_t n;
  int64_t o;
  int b;
  double* Ct;
  int64_t ldc;
};

// kernels.hip
hipError_t launch_leaf_inverse(const double* A, int64_t lda, double* P, int64_t ldp, int b, int64_t row0,
                               long long* info, hipStream_t s);
hipError_t launch_col_save(const double* W, int64_t ldw, int64_t n, int64_t o, int b, double* Ct, int64_t ldc,
                           hipStream_t s);
hipError_t launch_copy2d(const double* S, int64_t lds, double* D, int64_t ldd, int64_t rows, int64_t cols,
                         hipStream_t s);
hipError_t launch_zero_info(long long* p, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_row_panel(const double* P, int64_t ldp, const double* W, int64_t ldw, int64_t n, int64_t o, int b,
                            double* R, int64_t ldr, hipStream_t s, double* flops);
hipError_t launch_schur(const double* Ct, int64_t ldc, const double* R, int64_t ldr, double* W, int64_t ldw, int64_t n,
                        int64_t o, int b, int region, int64_t qo, int qb, hipStream_t s, double* flops, int slots);
hipError_t launch_leaf_batched(const LeafJob* jobs, int64_t count, int bmax, hipStream_t s);
hipError_t launch_col_save_batched(const ColJob* jobs, int64_t count, hipStream_t s);
hipError_t launch_row_panel_batched(const StepArgs* args, int64_t count, hipStream_t s);
hipError_t launch_schur_batched(const StepArgs* args, int64_t count, hipStream_t s);

// batched.hip
hipError_t launch_small_tier(int tier, const double* A, double* X, const SmallMat* mats, const int32_t* order,
                             int64_t count, const int32_t* bounds, int32_t* info, hipStream_t s);
int small_tier_limit(int tier);

// binv_api.hip: records the thread-local message returned by binv_last_error
void set_error(const std::string& msg);

constexpr int kLeafMax = 128;   // largest pivot block the register leaf kernel holds
constexpr int kSubBlock = 64;   // sub-block order of the nested sweep of a larger pivot block

}  // namespace binv
