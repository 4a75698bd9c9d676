// Sustained FP64 rates of the instructions a trailing update can be built on,
// the figures the choice of the GEMM core rests on:
//   v_mfma_f64_4x4x4_4b_f64 (four independent 4x4x4 blocks): 512 flops per
//     wave instruction;
//   v_mfma_f64_16x16x4_f64: 2048 flops per wave instruction;
//   v_fma_f64 (vector): 128 flops per wave instruction.
// Every wave issues a long run of independent instructions (kAcc accumulator
// chains, more issue slots than an instruction's latency), and each launch
// is exactly one round of as many workgroups as fit on every CU at once
// (no partial last round); the launch's time on its stream (HIP events)
// gives flops per second.  Prints one JSON object per instruction.  Standalone
// measurement program, not part of the library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                      \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));             \
      std::exit(1);                                                                   \
    }                                                                                 \
  } while (0)

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kAcc = 8;
constexpr int kThreads = 256;  // four waves per workgroup

__global__ void __launch_bounds__(kThreads) k_rate_mfma4(int iters, double* out) {
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - blockIdx.x * 1e-9;
  double acc[kAcc];
#pragma unroll
  for (int i = 0; i < kAcc; ++i) acc[i] = i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kAcc; ++i) s += acc[i];
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_rate_mfma16(int iters, double* out) {
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - blockIdx.x * 1e-9;
  d4 acc[kAcc];
#pragma unroll
  for (int i = 0; i < kAcc; ++i) acc[i] = d4{(double)i, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kAcc; ++i) s += acc[i].x + acc[i].y + acc[i].z + acc[i].w;
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) k_rate_fma(int iters, double* out) {
  const double a = 1.0 + threadIdx.x * 1e-12, b = 1e-9 * blockIdx.x;
  double acc[kAcc];
#pragma unroll
  for (int i = 0; i < kAcc; ++i) acc[i] = i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = fma(acc[i], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kAcc; ++i) s += acc[i];
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

struct Case {
  const char* name;
  void (*kernel)(int, double*);
  double flops_per_wave_instr;
  int iters;
};

}  // namespace

int main(int argc, char** argv) {
  const int reps = argc > 1 ? std::atoi(argv[1]) : 5;
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  constexpr int kMaxPerCU = 8;  // 32 waves per CU
  double* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(double) * (size_t)cus * kMaxPerCU * kThreads));
  hipStream_t s;
  CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const Case cases[] = {
      {"v_mfma_f64_4x4x4_4b_f64", k_rate_mfma4, 512.0, 20000},
      {"v_mfma_f64_16x16x4_f64", k_rate_mfma16, 2048.0, 4000},
      {"v_fma_f64", k_rate_fma, 128.0, 80000},
  };
  std::printf("{\"device\": \"%s\", \"compute_units\": %d, \"max_clock_mhz\": %d, \"threads\": %d, "
              "\"accumulators_per_wave\": %d}\n",
              prop.gcnArchName, cus, prop.clockRate / 1000, kThreads, kAcc);
  for (const Case& c : cases) {
    int per_cu = 0;
    CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(c.kernel), kThreads, 0));
    per_cu = std::min(std::max(per_cu, 1), kMaxPerCU);
    const int grid = cus * per_cu;
    hipLaunchKernelGGL(c.kernel, dim3(grid), dim3(kThreads), 0, s, c.iters, out);  // warm-up
    CHECK(hipGetLastError());
    CHECK(hipStreamSynchronize(s));
    std::vector<double> ms;
    for (int r = 0; r < reps; ++r) {
      CHECK(hipEventRecord(e0, s));
      hipLaunchKernelGGL(c.kernel, dim3(grid), dim3(kThreads), 0, s, c.iters, out);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(e1, s));
      CHECK(hipEventSynchronize(e1));
      float t = 0.0f;
      CHECK(hipEventElapsedTime(&t, e0, e1));
      ms.push_back(t);
    }
    std::sort(ms.begin(), ms.end());
    const double waves = (double)grid * (kThreads / 64);
    const double flops = waves * (double)c.iters * kAcc * c.flops_per_wave_instr;
    std::printf("{\"instruction\": \"%s\", \"flops_per_wave_instruction\": %.0f, \"waves_per_simd\": %d, "
                "\"workgroups\": %d, \"flops_per_launch\": %.6e, \"ms_best\": %.4f, \"ms_median\": %.4f, "
                "\"tflops_best\": %.3f, \"tflops_median\": %.3f}\n",
                c.name, c.flops_per_wave_instr, per_cu * (kThreads / 64) / 4, grid, flops, ms.front(),
                ms[ms.size() / 2], flops / (ms.front() * 1e9), flops / (ms[ms.size() / 2] * 1e9));
    std::fflush(stdout);
  }
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  CHECK(hipStreamDestroy(s));
  CHECK(hipFree(out));
  return 0;
}
