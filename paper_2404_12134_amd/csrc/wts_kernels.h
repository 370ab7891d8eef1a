// wts_kernels.h -- host-side launchers of the WETSAND kernels (wts_dtw.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wts_device.h"

namespace wts {

struct WalkArgs {
  const PairDesc* pairs;
  const int2* items;
  const int2* seg;          // per item: (bottom-row column, top-row column) of the path
  int2* seg_out;            // the same, written by the path walk
  int2* runs;               // [out][L]: the columns [lo, hi] of each row's path run
  const uint32_t* codes;
  const void* y;
  double* psum;             // [out][L][d] per-cycle row sums, or nullptr
  int* pcnt;                // [out][L] per-cycle row counts
  int64_t L;
  int* seg_len;             // per item: cells of the path inside the strip
  const int* seg_off;       // per item: offset of the strip's segment in the pair's path
  const int64_t* path_base; // per pair slot: first path row
  int32_t* paths;           // [rows][2]
  int* status;              // device status word
  const int* skip;          // validation flag of the call (or null)
};

// fp32: the float32-decision instances (float32 cycles, squared cost only).
hipError_t launch_fwd(int d, int rho, int mode, bool euc, bool x_is_cycle, int ydtype, bool fp32,
                      const FwdArgs& a, int grid, hipStream_t st);
hipError_t launch_fwd32(int d, int rho, int mode, bool euc, bool x_is_cycle, int ydtype,
                        const FwdArgs& a, int grid, hipStream_t st);
// Path recovery after a PATHT sweep: the strip chain (segments from the
// entry tags), then walks of all strips at once (emit = false: row runs,
// segment lengths and DBA partial sums; emit = true: the path list).
hipError_t launch_walk(int d, int rho, int ydtype, bool emit, const WalkArgs& a, int n_items,
                       hipStream_t st);
hipError_t launch_chain(const PairDesc* pairs, int n_pairs, const int* bnd_aux,
                        const int* out_aux, int2* seg, int* status, const int* skip,
                        hipStream_t st);
// Path recovery after a PATH sweep: one workgroup per pair walks its strips
// in turn (segments, their lengths, the row runs).
hipError_t launch_path_walk(int rho, const WalkArgs& a, int n_pairs, hipStream_t st);
// DBA partial sums per (cycle, barycenter row) from the pair walk's runs.
hipError_t launch_run_sum(int d, int ydtype, const int2* runs, const int64_t* off, const void* y,
                          int n, int64_t L, double* psum, int* pcnt, const int* skip,
                          hipStream_t st);
hipError_t launch_zero(int* p, int64_t n, hipStream_t st);
hipError_t launch_fill_sentinels(double* r, int64_t nr, int* x, int64_t nx, hipStream_t st);
hipError_t launch_seg_prefix(const PairDesc* pairs, int n_pairs, const int* seg_len,
                             int* seg_off, int64_t* path_len, hipStream_t st);
hipError_t launch_dba_reduce(const double* psum, const int* pcnt, const double* w, int n,
                             int64_t L, int d, double* bout, int64_t* counts, hipStream_t st);
hipError_t launch_score(const double* dist, const int* len, int n, double* score,
                        int64_t* path_len, hipStream_t st);
hipError_t launch_sub_out(const int* start, const int* end, int n, int64_t* a_star,
                          int64_t* b_star, hipStream_t st);
hipError_t launch_medoid(const double* pair_dist, const int2* pair_ab, int n_pairs, int n,
                         double* Dm, double* totals, int32_t* medoid, hipStream_t st);
hipError_t launch_soft(int d, int ydtype, bool bwd, const SoftArgs& a, int grid, hipStream_t st);
hipError_t launch_soft_rows_scale(const double* g, const int64_t* off, int n, int64_t rows, int d,
                                  const double* w, double* out, hipStream_t st);
hipError_t launch_soft_reduce(const double* gsum, const double* hsum, const double* w, int n,
                              int64_t L, int d, double* grad, double* mass, int accumulate,
                              hipStream_t st);

// wts_aux.hip: input validation, the status word, the Eq. 7 objective.
struct ScanSeg {
  const void* p;   // values to check (or null)
  int64_t n;       // number of values
  int f32;         // 1: float32, 0: float64
};
hipError_t launch_finite_scan(const ScanSeg* segs, int nseg, int* flag, int* status,
                              hipStream_t st);
hipError_t launch_status_take(int* status, int* out, hipStream_t st);
hipError_t launch_objective(const double* values, const double* weights, int n, int accumulate,
                            double* out, hipStream_t st);
hipError_t launch_precond_step(double* bary, const double* grad, const double* mass, int64_t L,
                               int d, double eta, hipStream_t st);
hipError_t launch_init(int ydtype, const void* Y, const int64_t* off, int n, int d, int src,
                       int64_t Nsrc, int64_t L, int euclid, double* out, hipStream_t st);

}  // namespace wts
