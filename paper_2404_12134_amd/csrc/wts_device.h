// wts_device.h -- device-side definitions shared by the WETSAND HIP kernels.
//
// Layout of the dynamic program on gfx950 (one wavefront = 64 lanes):
//  * a "strip" is 64*RHO consecutive rows of X (the barycenter, or the
//    shorter cycle for the medoid); lane k owns rows i0 + k*RHO .. + RHO-1 and
//    keeps them in registers as float64;
//  * the wave sweeps the columns (samples of Y) in a skewed order: at step t
//    lane k works on column j = t - k, so the cells a lane needs from the
//    rows above (lane k-1) were produced one step earlier and arrive through
//    a DPP wave_shr:1 move; lane 0 takes them from the previous strip's
//    bottom row;
//  * strips of one pair run on different workgroups and hand their bottom
//    row over through device memory.  The DTW sweeps give every strip its own
//    row, filled with a sentinel before the launch: the strip below polls
//    the values themselves (device-scope loads) until no sentinel is left,
//    so the producer needs neither a counter nor a store drain.  The
//    Soft-DTW sweeps publish a per-strip progress counter (columns written
//    so far) after their device-scope row stores, ordered by s_waitcnt; in
//    both cases no L2 writeback is needed;
//  * workgroups pop (pair, strip) items from a queue in which the strips of
//    one pair are consecutive and pairs are sorted by decreasing size: a
//    strip only ever waits for an item popped earlier by a running
//    workgroup, so the sweep cannot deadlock.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wts {

constexpr int kWave = 64;

struct PairDesc {
  int64_t x_off;      // first row of X in the x buffer (row units)
  int64_t y_off;      // first row of Y in the cycle buffer (row units)
  int64_t code_base;  // first code word (uint32 units) of this pair
  int64_t bnd_base;   // first element of this pair's boundary rows
  int32_t M, N;       // rows of X, columns (samples of Y)
  int32_t S;          // strips
  int32_t out;        // output slot (cycle index, or pair index for the medoid)
  int32_t flag_base;  // progress counter of strip 0
  int32_t WT;         // code words per (strip, row, lane): ceil((N + 63) / 16) rounded
  int32_t item_base;  // index of this pair's strip 0 in the item list
  int32_t pad;
  int64_t aux_base;   // first element of this pair's per-strip rows (S * N)
  int64_t state_base; // first double of this pair's Soft-DTW sweep states
  int64_t row_base;   // DTW sweeps: first element of this pair's strip rows (S * RS)
};

// Wave-uniform copies (scalar registers) of values every lane holds alike:
// addresses built from them stay scalar, so buffer resources need no
// per-lane waterfall loop.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ PairDesc uniform(const PairDesc& p) {
  PairDesc q;
  q.x_off = uni(p.x_off);
  q.y_off = uni(p.y_off);
  q.code_base = uni(p.code_base);
  q.bnd_base = uni(p.bnd_base);
  q.M = uni(p.M);
  q.N = uni(p.N);
  q.S = uni(p.S);
  q.out = uni(p.out);
  q.flag_base = uni(p.flag_base);
  q.WT = uni(p.WT);
  q.item_base = uni(p.item_base);
  q.pad = 0;
  q.aux_base = uni(p.aux_base);
  q.state_base = uni(p.state_base);
  q.row_base = uni(p.row_base);
  return q;
}

// Rows per lane of the Soft-DTW sweeps (the backward keeps 3 weights per cell
// for 16 steps in registers).
constexpr int kSoftRho = 2;

// DIST: value only; DIST_LEN: value and path length; PATH: value and argmin
// codes; SUB: Sub-DTW (free start; lowest-column minimum of the last row and
// the start column of its path).
// MODE_PATH keeps the argmin codes only (the path is then walked pair by
// pair); MODE_PATHT also tags every cell with the top-row cell through which
// its path enters the strip, so that all strips can be walked at once.
enum Mode { MODE_DIST = 0, MODE_DIST_LEN = 1, MODE_PATH = 2, MODE_SUB = 3, MODE_PATHT = 4 };

struct FwdArgs {
  const PairDesc* pairs;
  const int2* items;     // (pair, strip)
  int n_items;
  int* queue;            // item counter, zeroed before the launch
  int* status;           // device status word (bit 0: a boundary wait gave up)
  const void* x;         // X rows (float64 barycenter, or cycles for the medoid)
  const void* y;         // cycle values
  double* bnd_r;         // strip rows (S * RS per pair, sentinel-filled): cumulative cost
  int* bnd_aux;          // strip rows: path length (DIST_LEN) or entry code (PATH)
  uint32_t* codes;       // 2-bit argmin codes (PATH)
  double* out_dist;      // [pair slot] r(M-1, N-1)
  int* out_aux;          // [pair slot] |pi| (DIST_LEN), entry code of (M-1, N-1) (PATH) or a* (SUB)
  int* out_end;          // [pair slot] b* (SUB)
  int cost_kind;         // 0 squared, 1 Euclidean (sqrt)
  int relaxed_wait;      // 1: far more items than resident wavefronts; wait with long sleeps
  const int* skip;       // non-zero flag: the call's inputs failed validation, do nothing (or null)
  int zero_skip;         // backward: 1 = tiles whose e is exactly zero are not swept
  unsigned long long* tiles;   // backward: += tiles swept, tiles of the strips' ranges (or null)
};

struct SoftArgs {
  const PairDesc* pairs;
  const int2* items;     // (pair, strip); strips descending within a pair for the backward
  int n_items;
  int* queue;
  int* status;
  int* progress;
  const double* x;       // row series: the barycenter [L][d], or packed float64 cycles (x_off)
  const void* y;         // column series: cycle values, or the barycenter
  double* rows;          // bottom row of every strip, scaled units (S * N per pair)
  double* states;        // sweep state every 16 steps (RHO + 1 values per lane)
  double kscale;         // log2(e) / gamma
  double* value;         // [n] Soft-DTW values (forward)
  float* push_up;        // rolling top-row pushes between strips (backward, float32 e)
  float* push_dg;
  double* gsum;          // per-pair gradient rows ([n][L][d], or packed [sum M][d])
  double* hsum;          // per-pair row mass ([n][L], or packed [sum M])
  int64_t L;
  int relaxed_wait;      // 1: far more items than resident wavefronts; wait with long sleeps
  double band;           // Sakoe-Chiba bandwidth as a fraction of the longer length (0: none)
  int rows_packed;       // 0: gsum/hsum rows at out * L + i; 1: at x_off + i (X rows packed)
  const int* skip;       // non-zero flag: the call's inputs failed validation, do nothing (or null)
  int zero_skip;         // backward: 1 = tiles whose e is exactly zero are not swept
  unsigned long long* tiles;   // backward: += tiles swept, tiles of the strips' ranges (or null)
};

__device__ __forceinline__ double inf_d() { return __builtin_huge_val(); }

// Status bits of a plan's device status word (sticky until wts_plan_status
// reads and clears it).
constexpr int kStatusSpinTimeout = 1;   // a strip gave up waiting for its predecessor
constexpr int kStatusBadPath = 2;       // path recovery left the strip (inconsistent tags)
constexpr int kStatusNonFinite = 4;     // a validated call found a NaN or an infinity in its inputs

// A validated call whose inputs hold a non-finite value sets its skip flag;
// every sweep and path-recovery kernel of the call then returns at once.
__device__ __forceinline__ bool skipped(const int* skip) { return skip != nullptr && *skip != 0; }
// Sleep between two polls of a strip that waits for its neighbour: two quick
// polls, then short sleeps, or long ones when far more items than resident
// wavefronts keep the SIMD busy meanwhile (each poll costs issue slots).
__device__ __forceinline__ void poll_backoff(int polls, int relaxed) {
  if (polls < 2) __builtin_amdgcn_s_sleep(2);
  else if (!relaxed) __builtin_amdgcn_s_sleep(8);
  else __builtin_amdgcn_s_sleep(64);
}

// Polls of a progress counter before a strip gives up (about a second);
// a legitimate wait is bounded by one chunk of the predecessor strip.
constexpr int kSpinLimit = 1 << 20;

// DPP wave_shr:1 -- lane k receives v from lane k-1; lane 0 receives `old`.
__device__ __forceinline__ int shr1_i32(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ double shr1_f64(double v, double old) {
  const long long s = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = shr1_i32((int)s, (int)o);
  const int hi = shr1_i32((int)(s >> 32), (int)(o >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Device-scope relaxed accesses for data exchanged between workgroups.
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ float ld_dev(const float* p) {
  return __builtin_bit_cast(float, __hip_atomic_load(reinterpret_cast<const unsigned*>(p),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_dev(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_dev(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}
// Device-scope (sc1) buffer accesses: stores write through to the point of
// coherence for all CUs of the device.  Every lane issues the instruction; a
// lane that must not access memory passes kDrop, an offset past the buffer's
// record count, and the hardware range check discards its access (a load
// returns 0).  No branch around the access is needed.
constexpr int kDrop = 0x7ffffff0;   // > any row these kernels address (< 2^28 bytes)
typedef unsigned int u2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_dev(__amdgpu_buffer_rsrc_t r, int byte_off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_t, v), r, byte_off, 0, 16);
}
__device__ __forceinline__ double ld_dev(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 16));
}
__device__ __forceinline__ void st_dev(__amdgpu_buffer_rsrc_t r, int byte_off, int v) {
  __builtin_amdgcn_raw_buffer_store_b32((unsigned)v, r, byte_off, 0, 16);
}
__device__ __forceinline__ void st_dev(__amdgpu_buffer_rsrc_t r, int byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, 0, 16);
}
__device__ __forceinline__ float ld_dev_f32(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 16));
}
// Wait for every outstanding memory operation of this wave (orders the
// relaxed stores above before a following progress-counter store).
__device__ __forceinline__ void mem_drain() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// Wait for every outstanding vector memory operation (vmcnt 0) but not for
// LDS or scalar memory.
__device__ __forceinline__ void mem_wait_vm0() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// Wait until at most the most recent vector memory operation of this wave is
// outstanding (vmcnt 1).
__device__ __forceinline__ void mem_wait_all_but_1() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F71);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// Wait until at most the two most recent vector memory operations of this
// wave are outstanding (gfx9 s_waitcnt: vmcnt 2, expcnt and lgkmcnt not
// waited on).  Vector loads and stores share one in-order counter, so every
// older access is complete.
__device__ __forceinline__ void mem_wait_all_but_2() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F72);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

}  // namespace wts
