// wts_ubench.hip -- VALU issue-rate microbenchmark for the roofline of the
// sweeps (not part of the C ABI of the hot path; built as libwts_ubench.so).
//
// Every lane runs eight independent dependency chains of one instruction
// kind, with enough resident waves that the chains' latency is hidden, so the
// kernel time measures the issue rate of that instruction.  The rates are
// compared with the float64 add: a transcendental that costs tau add slots is
// counted as tau lane-operations in the sweeps' algorithmic floors.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

enum Op {
  kAddF64 = 0,     // v_add_f64
  kFmaF64 = 1,     // v_fma_f64
  kExpLogF32 = 2,  // v_exp_f32 then v_log_f32 (two transcendentals per step)
  kAddF32 = 3,     // v_add_f32
  kCvt = 4,        // v_cvt_f32_f64 then v_cvt_f64_f32 (two conversions per step)
  kRcpF64 = 5,     // v_rcp_f64
  kNumOps = 6
};

constexpr int kChains = 8;

template <int OP>
__global__ __launch_bounds__(256) void ubench_kernel(double* out, int iters, double seed) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double xd[kChains];
  float xf[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    xd[c] = seed + 1e-3 * (double)(t + c);
    xf[c] = (float)(0.5 + 1e-4 * (double)((t + c) & 1023));
  }
  const double k1 = seed * 1e-9, k2 = 1.0 - seed * 1e-12;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == kAddF64) xd[c] = xd[c] + k1;
      if constexpr (OP == kFmaF64) xd[c] = __builtin_fma(xd[c], k2, k1);
      if constexpr (OP == kExpLogF32) xf[c] = __builtin_amdgcn_logf(__builtin_amdgcn_exp2f(xf[c]));
      if constexpr (OP == kAddF32) xf[c] = xf[c] + (float)k1;
      if constexpr (OP == kCvt) xd[c] = (double)(float)xd[c];
      if constexpr (OP == kRcpF64) xd[c] = __builtin_amdgcn_rcp(xd[c]);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += xd[c] + (double)xf[c];
  out[t] = s;
}

template <int OP>
hipError_t run(double* out, int blocks, int iters, hipStream_t st) {
  hipLaunchKernelGGL(ubench_kernel<OP>, dim3(blocks), dim3(256), 0, st, out, iters, 1.25);
  return hipGetLastError();
}

}  // namespace

extern "C" {

// Operations (lane-level instructions of the measured kind) one launch of
// `op` performs per lane and step: 2 for the pairs, 1 otherwise.
int wts_ubench_ops_per_step(int op) { return (op == kExpLogF32 || op == kCvt) ? 2 : 1; }
int wts_ubench_chains(void) { return kChains; }
int wts_ubench_num_ops(void) { return kNumOps; }

// Runs `reps` launches of the microbenchmark `op` with `blocks` workgroups of
// 256 threads and `iters` steps each, and returns the mean launch time in
// milliseconds (HIP events on the null stream) in *ms.  out: a device buffer
// of blocks * 256 doubles.  Returns 0, or -1 on a bad argument / HIP error.
int wts_ubench_run(int op, double* out, int blocks, int iters, int reps, double* ms) {
  if (!out || !ms || blocks < 1 || iters < 1 || reps < 1 || op < 0 || op >= kNumOps) return -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1;
  }
  auto launch = [&]() -> hipError_t {
    switch (op) {
      case kAddF64: return run<kAddF64>(out, blocks, iters, nullptr);
      case kFmaF64: return run<kFmaF64>(out, blocks, iters, nullptr);
      case kExpLogF32: return run<kExpLogF32>(out, blocks, iters, nullptr);
      case kAddF32: return run<kAddF32>(out, blocks, iters, nullptr);
      case kCvt: return run<kCvt>(out, blocks, iters, nullptr);
      default: return run<kRcpF64>(out, blocks, iters, nullptr);
    }
  };
  int rc = 0;
  if (launch() != hipSuccess) rc = -1;   // warm-up
  if (rc == 0 && hipEventRecord(e0, nullptr) != hipSuccess) rc = -1;
  for (int r = 0; rc == 0 && r < reps; ++r)
    if (launch() != hipSuccess) rc = -1;
  if (rc == 0 && hipEventRecord(e1, nullptr) != hipSuccess) rc = -1;
  float t = 0.f;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -1;
  *ms = (double)t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
