// wts_aux.hip -- small kernels around the sweeps: input validation (the
// paper drops samples with missing values before any DTW, Sec. III-A, so the
// dynamic programs assume finite inputs), the plan's status word, and the
// Eq. 7 objective.
#include "wts_device.h"
#include "wts_kernels.h"

namespace wts {

namespace {

constexpr int kMaxScanSegs = 3;

struct ScanArgs {
  ScanSeg seg[kMaxScanSegs];
  int nseg;
  int* flag;     // the call's skip flag: set to 1 when a value is not finite
  int* status;   // the plan's sticky status word
};

// Exponent field all ones: an infinity or a NaN (float32 and float64).
__device__ __forceinline__ bool bad32(uint32_t u) { return (u & 0x7f800000u) == 0x7f800000u; }
__device__ __forceinline__ bool bad64(uint64_t u) {
  return (u & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
}

__global__ void finite_scan_kernel(ScanArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool bad = false;
  for (int q = 0; q < a.nseg; ++q) {
    const ScanSeg sg = a.seg[q];
    if (sg.p == nullptr) continue;
    if (sg.f32) {
      const uint32_t* v = static_cast<const uint32_t*>(sg.p);
      for (int64_t k = t0; k < sg.n; k += stride) bad |= bad32(v[k]);
    } else {
      const uint64_t* v = static_cast<const uint64_t*>(sg.p);
      for (int64_t k = t0; k < sg.n; k += stride) bad |= bad64(v[k]);
    }
  }
  if (__any(bad) && (threadIdx.x % kWave) == 0) {
    atomicOr(a.flag, 1);
    atomicOr(a.status, kStatusNonFinite);
  }
}

// out = the status word, which is cleared (one atomic exchange, so a bit set
// concurrently is either returned now or kept for the next read).
__global__ void status_take_kernel(int* status, int* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = atomicExch(status, 0);
}

// Eq. 7 objective: out = [out +] sum_{k ascending} w_k value_k (w = 1 if null).
__global__ void objective_kernel(const double* __restrict__ v, const double* __restrict__ w,
                                 int n, int accumulate, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = accumulate ? *out : 0.0;
  for (int k = 0; k < n; ++k) s = s + (w ? w[k] : 1.0) * v[k];
  *out = s;
}

}  // namespace

hipError_t launch_finite_scan(const ScanSeg* segs, int nseg, int* flag, int* status,
                              hipStream_t st) {
  if (nseg < 1 || nseg > kMaxScanSegs) return hipErrorInvalidValue;
  ScanArgs a{};
  int64_t tot = 0;
  for (int q = 0; q < nseg; ++q) {
    a.seg[q] = segs[q];
    if (segs[q].p) tot += segs[q].n;
  }
  a.nseg = nseg;
  a.flag = flag;
  a.status = status;
  // 8 values per thread at least, at most 4096 workgroups (grid-stride)
  int64_t blocks = (tot + 256 * 8 - 1) / (256 * 8);
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(finite_scan_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_status_take(int* status, int* out, hipStream_t st) {
  hipLaunchKernelGGL(status_take_kernel, dim3(1), dim3(64), 0, st, status, out);
  return hipGetLastError();
}

hipError_t launch_objective(const double* values, const double* weights, int n, int accumulate,
                            double* out, hipStream_t st) {
  hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(64), 0, st, values, weights, n, accumulate,
                     out);
  return hipGetLastError();
}

}  // namespace wts
