// wts_sweep.h -- the DTW wavefront sweep of gfx950 (value, value + path
// length, argmin codes, Sub-DTW) and its launchers, shared by the float64
// instances (wts_dtw.hip) and the float32-decision instances (wts_dtw32.hip).
//
// The recurrence (Eq. 5 with gamma = 0, i.e. Eq. 1 by dynamic programming):
//   r(-1,-1) = 0, r(i,-1) = r(-1,j) = +inf,
//   r(i,j) = delta(x_i, y_j) + min(r(i-1,j-1), r(i-1,j), r(i,j-1)),
// all in float64 (the float32-decision instances: all in float32), delta =
// e_0*e_0 then fma(e_c, e_c, s) (Def. 3, squared Euclidean).  The argmin of a cell is the first of diag, up, left that
// attains the minimum, kept as two bits (diagonal chosen; else up chosen);
// following them back from (M-1, N-1) gives the optimal path that Eq. 8
// divides by.
#pragma once
#include <climits>
#include <type_traits>

#include "wts_device.h"
#include "wts_kernels.h"

namespace wts {

namespace {

// One IEEE operation each, in the compute type of the sweep (float64, or
// float32 for the float32-decision variant).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double min_t(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float min_t(float a, float b) { return __builtin_fminf(a, b); }

template <typename T, int D>
__device__ __forceinline__ T sq_cost(const T (&x)[D], const T (&y)[D]) {
  T e = x[0] - y[0];
  T s = e * e;
#pragma unroll
  for (int c = 1; c < D; ++c) {
    e = x[c] - y[c];
    s = fma_t(e, e, s);
  }
  return s;
}

constexpr int kChunk = 64;          // sweep steps per Y staging round
constexpr int kRing = 128;          // Y columns kept in LDS (>= kChunk + 63, power of 2)

// Strip boundary rows.  Strip s writes the bottom row of its rows into its own
// row of the pair's boundary block, column j at index j + 63 (the 16 columns
// lane 63 produces in the steps tg .. tg+15 land at indices tg .. tg+15),
// after the whole block was filled with sentinels.  The strip below polls the values
// themselves: a value is ready once it is no longer the sentinel, so no
// progress counter, fence or store drain is needed between strips.
// The sentinel is a NaN that no arithmetic makes, read as one float64 or as
// two float32 words (the float32-decision sweeps keep float32 rows in the
// same buffer); both halves are the float32 sentinel.
constexpr unsigned long long kSentR = 0xFFF4DEADFFF4DEADull;
constexpr unsigned kSentR32 = 0xFFF4DEADu;
constexpr int kSentX = INT_MIN;
__device__ __forceinline__ int row_stride(int N) { return (N + 63 + 3) & ~3; }

// acc * 2 + b in one instruction: the carry-in of v_addc is the lane mask of
// the comparison that produced b.
__device__ __forceinline__ uint32_t push_bit(uint32_t acc, bool b) {
  uint32_t r;
  unsigned long long carry_out;
  const unsigned long long m = __builtin_amdgcn_ballot_w64(b);
  __asm__("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(acc), "s"(m));
  return r;
}
__device__ __forceinline__ bool is_sent(double v) {
  return (unsigned long long)__double_as_longlong(v) == kSentR;
}
__device__ __forceinline__ bool is_sent(float v) { return __builtin_bit_cast(unsigned, v) == kSentR32; }

// Strip-row accesses in the compute type.
__device__ __forceinline__ double shr1_t(double v, double old) { return shr1_f64(v, old); }
__device__ __forceinline__ float shr1_t(float v, float old) {
  return __builtin_bit_cast(float, shr1_i32(__builtin_bit_cast(int, v), __builtin_bit_cast(int, old)));
}
template <typename T>
__device__ __forceinline__ T ld_row(__amdgpu_buffer_rsrc_t r, int byte_off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 16));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 16));
}

// Waves per sweep workgroup.  Each wave works alone (own items, own LDS);
// grouping four of them makes the dispatcher place one wave on each SIMD of a
// compute unit, which one-wave workgroups do not get reliably.
constexpr int kSweepWaves = 4;
// Orders a wave's own LDS accesses around a point of the program; a wave's
// LDS operations execute in order, so no hardware barrier is needed.
__device__ __forceinline__ void wave_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One wavefront sweeps one strip of one pair.  State per lane: RHO rows of X
// (registers of the compute type TC), the cumulative cost of those rows at
// the previous column (`left`) and, for the row above its first row, the
// value received one step earlier (`upprev`, the diagonal predecessor).
// TC = double is the float64 recurrence; TC = float runs the same steps in
// float32 (X rounded to float32 once, float32 cycles as they are): the
// float32-decision variant.
// The value sweep (medoid) runs on many items at once and is held to five
// resident wavefronts per SIMD; the other modes keep their registers.
template <typename TX, typename TY, typename TC, int D, int RHO, int MODE, bool EUC>
__global__ __launch_bounds__(kWave * kSweepWaves, MODE == MODE_DIST && D <= 4 ? 5 : 1)
void dtw_fwd_kernel(FwdArgs a) {
  constexpr int H = kWave * RHO;
  // tags carried along the argmin: the path length (DIST_LEN), the start
  // column (SUB) or the strip entry (PATHT); PATH keeps only its codes
  constexpr bool kAux = MODE == MODE_DIST_LEN || MODE == MODE_SUB || MODE == MODE_PATHT;
  constexpr bool kCodes = MODE == MODE_PATH || MODE == MODE_PATHT;
  // Y ring; slots kRing .. kRing+15 mirror slots 0 .. 15, so a group of 16
  // steps reads consecutive slots from one base without wrapping
  static_assert(!EUC || sizeof(TC) == 8, "the l2 cost is evaluated in float64 only");
  __shared__ TC ys_[kSweepWaves][D][kRing + 16];
  __shared__ TC binr_[kSweepWaves][16];   // strip above, this group's 16 columns
  __shared__ int binx_[kSweepWaves][16];
  // lane 63's bottom row of the last group; the other lanes write the same
  // steps into a scratch area (no exec-mask switch around the write)
  __shared__ TC stg_r_[kSweepWaves][16 + kWave + 16];
  __shared__ int stg_x_[kSweepWaves][16 + kWave + 16];
  __shared__ int s_item_[kSweepWaves];

  // Every wave of the workgroup is an independent sweeper with its own LDS.
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  auto& ys = ys_[wv];
  auto& binr = binr_[wv];
  auto& binx = binx_[wv];
  auto& stg_r = stg_r_[wv];
  auto& stg_x = stg_x_[wv];
  int& s_item = s_item_[wv];
  const TX* __restrict__ X = static_cast<const TX*>(a.x);
  const TY* __restrict__ Y = static_cast<const TY*>(a.y);
  const TC INF = (TC)inf_d();
  if (skipped(a.skip)) return;   // every wave of every workgroup: no strip waits for another

  for (;;) {
    if (lane == 0) s_item = atomicAdd(a.queue, 1);
    wave_sync();
    const int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: scalar loads below
    wave_sync();
    if (item >= a.n_items) break;
    const int2 it = a.items[item];
    const PairDesc pd = uniform(a.pairs[uni(it.x)]);
    const int s = uni(it.y);
    const int M = pd.M, N = pd.N;
    const int i0 = s * H;
    const int ib = i0 + lane * RHO;
    const bool has_prev = s > 0;
    const bool has_next = s + 1 < pd.S;
    const int Tend = pd.WT * 16;
    const int RS = row_stride(N);

    const TC* r_in = reinterpret_cast<const TC*>(a.bnd_r) + pd.row_base + (int64_t)(s - 1) * RS;
    TC* r_out = reinterpret_cast<TC*>(a.bnd_r) + pd.row_base + (int64_t)s * RS;   // via rr_out
    const int* x_in = a.bnd_aux + pd.row_base + (int64_t)(s - 1) * RS;
    int* x_out = a.bnd_aux + pd.row_base + (int64_t)s * RS;
    constexpr int kB = (int)sizeof(TC);
    const __amdgpu_buffer_rsrc_t rr_out = rsrc(r_out, RS * kB);
    const __amdgpu_buffer_rsrc_t rx_out = rsrc(x_out, RS * 4);

    TC xr[RHO][D];
#pragma unroll
    for (int r = 0; r < RHO; ++r) {
      const int i = ib + r;
#pragma unroll
      for (int c = 0; c < D; ++c)
        xr[r][c] = (i < M) ? static_cast<TC>(X[(pd.x_off + i) * D + c]) : (TC)0;
    }
    TC left[RHO];
    int lx[RHO];
    uint32_t acc[RHO];
#pragma unroll
    for (int r = 0; r < RHO; ++r) { left[r] = INF; lx[r] = 0; acc[r] = 0u; }
    TC upprev = (s == 0 && lane == 0) ? (TC)0 : INF;   // r(-1,-1) = 0 at the origin
    // Sub-DTW: running minimum of the last row (lowest column on ties)
    const bool last_strip = s + 1 == pd.S;
    const int rl_last = M - 1 - ib;
    TC sub_best = INF;
    int sub_end = 0, sub_start = 0;
    int upprevx = 0;
    TC bot = INF;
    int botx = 0;
    bool gave_up = false;   // set once a wait times out: the strip never waits again

    // The strip above's bottom row, 16 columns at a time: lanes 0..15 hold the
    // next group's values in (pr, px) -- loaded one group ahead -- and wait
    // until none of them is a sentinel any more.  The prefetch is one
    // unconditional buffer load per value (lanes without a value read past
    // the record count and get 0; strip 0 has no records at all), so the
    // only wait for it is the check after the group's sweep steps.
    const __amdgpu_buffer_rsrc_t rr_in = rsrc(r_in, has_prev ? RS * kB : 0);
    const __amdgpu_buffer_rsrc_t rx_in = rsrc(x_in, has_prev ? RS * 4 : 0);
    TC pr = (TC)0;
    int px = 0;
    auto fetch = [&](int tg) {
      const int j = tg + lane;
      const bool want = lane < 16 && j < N;
      pr = ld_row<TC>(rr_in, want ? (j + 63) * kB : kDrop);
      if (kAux)
        px = (int)__builtin_amdgcn_raw_buffer_load_b32(rx_in, want ? (j + 63) * 4 : kDrop, 0, 16);
    };
    auto settle = [&](int tg) {
      if (!has_prev || gave_up) return;
      const int j = tg + lane;
      auto ready = [&]() {
        return lane >= 16 || j >= N || (!is_sent(pr) && (!kAux || px != kSentX));
      };
      if (__all(ready())) return;   // the usual case: the prefetch found every value
      int polls = 0;
      do {
        // a strip that has caught up with the one above waits for up to a
        // group of the other strip's steps
        poll_backoff(polls, a.relaxed_wait);
        if (++polls > kSpinLimit) {   // never expected: report and carry on
          if (lane == 0) atomicOr(a.status, kStatusSpinTimeout);
          gave_up = true;
          break;
        }
        if (!ready()) {
          pr = ld_dev(r_in + j + 63);
          if (kAux) px = ld_dev(x_in + j + 63);
        }
      } while (!__all(ready()));
    };
    // Stores of group tg: lane 63's bottom row (columns tg-63 .. tg-48, at
    // indices tg .. tg+15 of the strip's row, by lanes 0..15 in one
    // coalesced store) and, for PATH, the group's argmin code words.
    auto publish = [&](int tg) {
      const int j = tg - 63 + lane;
      const bool w = has_next && lane < 16 && j >= 0 && j < N;
      st_dev(rr_out, w ? (tg + lane) * kB : kDrop, stg_r[lane & 15]);
      if (kAux) st_dev(rx_out, w ? (tg + lane) * 4 : kDrop, stg_x[lane & 15]);
      if (kCodes) {
        const int64_t cw = pd.code_base + (int64_t)(s * pd.WT + (tg >> 4)) * RHO * kWave + lane;
#pragma unroll
        for (int r = 0; r < RHO; ++r) a.codes[cw + r * kWave] = acc[r];
      }
    };
    fetch(0);
    settle(0);

    // Y values are read from a clamped column (always in bounds) and zeroed
    // past N, so the loads are unconditional
    TC yv[D];
    {
      const int j = lane;
      const int64_t row = (pd.y_off + min(j, N - 1)) * D;
#pragma unroll
      for (int c = 0; c < D; ++c) yv[c] = static_cast<TC>(Y[row + c]);
#pragma unroll
      for (int c = 0; c < D; ++c) yv[c] = j < N ? yv[c] : (TC)0;
#pragma unroll
      for (int c = 0; c < D; ++c) ys[c][j & (kRing - 1)] = yv[c];
      if ((j & (kRing - 1)) < 16) {
#pragma unroll
        for (int c = 0; c < D; ++c) ys[c][(j & (kRing - 1)) + kRing] = yv[c];
      }
    }

    for (int t0 = 0; t0 < Tend; t0 += kChunk) {
      const int tcnt = min(kChunk, Tend - t0);
      const bool more = t0 + kChunk < Tend;
      if (more) {   // next chunk of Y into registers; stored to LDS after this sweep
        const int j = t0 + kChunk + lane;
        const int64_t row = (pd.y_off + min(j, N - 1)) * D;
#pragma unroll
        for (int c = 0; c < D; ++c) yv[c] = static_cast<TC>(Y[row + c]);
#pragma unroll
        for (int c = 0; c < D; ++c) yv[c] = j < N ? yv[c] : (TC)0;
      }

      // 16 sweep steps; FULL: every lane is inside the grid (no masking)
      auto group16 = [&](auto full_tag, int tb) {
        constexpr bool FULL = decltype(full_tag)::value;
        const int tg = t0 + tb;
        // LDS operands of step u+1 are read during step u (software pipelining)
        TC yn[D];
        TC bn;
        int bxn = 0;
        const int yb = (tg - lane) & (kRing - 1);   // slot of step 0's column
        const int sb = lane == kWave - 1 ? 0 : 16 + lane;   // staging slot of step 0
#pragma unroll
        for (int c = 0; c < D; ++c) yn[c] = ys[c][yb];
        bn = binr[0];
        if (MODE == MODE_DIST_LEN || MODE == MODE_SUB) bxn = binx[0];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = tg + u;
          const int j = t - lane;
          TC y[D];
#pragma unroll
          for (int c = 0; c < D; ++c) y[c] = yn[c];
          const TC bval = bn;
          const int bxv = bxn;
          if (u + 1 < 16) {
#pragma unroll
            for (int c = 0; c < D; ++c) yn[c] = ys[c][yb + u + 1];
            bn = binr[u + 1];
            if (MODE == MODE_DIST_LEN || MODE == MODE_SUB) bxn = binx[u + 1];
          }
          const TC upin = shr1_t(bot, bval);
          int upinx = 0, dgx0 = 0;
          if (MODE == MODE_DIST_LEN) {
            upinx = shr1_i32(botx, bxv);
            dgx0 = upprevx;
          } else if (MODE == MODE_PATHT) {
            // top row of the strip (lane 0): entered from above at column j,
            // coded 2j (up) or 2j+1 (diagonal)
            upinx = shr1_i32(botx, 2 * t);
            dgx0 = lane == 0 ? upinx + 1 : upprevx;
          } else if (MODE == MODE_SUB) {
            // tags are start columns; a path entering the first row at
            // column j (from above or diagonally) starts at j
            upinx = shr1_i32(botx, s == 0 ? t : bxv);
            dgx0 = s == 0 && lane == 0 ? upinx : upprevx;
          }
          const TC dg0 = upprev;
          upprev = upin;
          upprevx = upinx;
          bool isd_r[RHO], isu_r[RHO];   // argmin of each row's cell (PATH, PATHT)
#pragma unroll
          for (int r = 0; r < RHO; ++r) { isd_r[r] = false; isu_r[r] = false; }
          if (FULL || (j >= 0 && j < N)) {
            TC dg = dg0, up = upin;
            int dgx = dgx0, upx = upinx;
#pragma unroll
            for (int r = 0; r < RHO; ++r) {
              const TC lf = left[r];
              const TC m1 = min_t(up, lf);
              const TC m = min_t(dg, m1);
              TC delta = sq_cost<TC, D>(xr[r], y);
              if constexpr (EUC) delta = __builtin_sqrt(delta);
              const TC rv = delta + m;
              int rxv = 0;
              if (MODE != MODE_DIST) {
                const bool isd = dg <= m1;
                const bool isu = up <= lf;
                if (kAux) {
                  // keep these as lane selects (v_cndmask), not branches
                  const int t1 = __builtin_unpredictable(isu) ? upx : lx[r];
                  const int sel = __builtin_unpredictable(isd) ? dgx : t1;
                  rxv = MODE == MODE_DIST_LEN ? sel + 1 : sel;
                }
                isd_r[r] = isd;
                isu_r[r] = isu;
              }
              dg = lf;
              dgx = lx[r];
              up = rv;
              upx = rxv;
              left[r] = rv;
              lx[r] = rxv;
            }
            bot = left[RHO - 1];
            botx = lx[RHO - 1];
            if (MODE == MODE_SUB && last_strip) {
              // the lane holding row M-1 keeps the lowest column of minimal
              // cost, and the start column of its path
              TC v = left[0];
              int vx = lx[0];
#pragma unroll
              for (int r = 1; r < RHO; ++r)
                if (r == rl_last) { v = left[r]; vx = lx[r]; }
              const bool better = v < sub_best;
              sub_best = better ? v : sub_best;
              sub_end = better ? j : sub_end;
              sub_start = better ? vx : sub_start;
            }
          }
          if (kCodes) {
            // every step of every lane shifts two bits into the row's code
            // word (cells outside the grid shift in don't-care bits)
#pragma unroll
            for (int r = 0; r < RHO; ++r) acc[r] = push_bit(push_bit(acc[r], isd_r[r]), isu_r[r]);
          }
          stg_r[sb + u] = bot;   // staged in LDS, stored at the next group's start
          if (kAux) stg_x[sb + u] = botx;
        }
      };

      // Memory order within a group: the previous group's stores, then the
      // next group's loads, then 16 sweep steps with no global memory access,
      // then the check of the loads.  Loads and stores share one in-order
      // counter, so a store issued after a load would have to complete
      // before the load's value may be used.
      for (int tb = 0; tb < tcnt; tb += 16) {
        const int tg = t0 + tb;
        if (lane < 16) {   // this group's upper input, ready and checked
          // above the first strip: +inf, or 0 for Sub-DTW (free start)
          binr[lane] = has_prev ? (tg + lane < N ? pr : INF) : (MODE == MODE_SUB ? (TC)0 : INF);
          if (kAux) binx[lane] = has_prev ? px : 0;
        }
        wave_sync();
        if (tg > 0) publish(tg - 16);
        fetch(tg + 16);                // next group's input, in flight during the sweep
        if (tg >= kWave - 1 && tg + 16 <= N) group16(std::true_type{}, tb);
        else group16(std::false_type{}, tb);
        if (tg + 16 < Tend) settle(tg + 16);
      }
      if (more) {
        const int j = t0 + kChunk + lane;
#pragma unroll
        for (int c = 0; c < D; ++c) ys[c][j & (kRing - 1)] = yv[c];
        if ((j & (kRing - 1)) < 16) {
#pragma unroll
          for (int c = 0; c < D; ++c) ys[c][(j & (kRing - 1)) + kRing] = yv[c];
        }
      }
      wave_sync();
    }
    publish(Tend - 16);
    // every lane ends with left[r] = r(ib + r, N - 1)
    if (ib <= M - 1 && M - 1 < ib + RHO) {
      const int rl = M - 1 - ib;
      TC v = left[0];
      int vx = lx[0];
#pragma unroll
      for (int r = 1; r < RHO; ++r)
        if (r == rl) { v = left[r]; vx = lx[r]; }
      if (MODE == MODE_SUB) {
        a.out_dist[pd.out] = sub_best;
        a.out_aux[pd.out] = sub_start;
        a.out_end[pd.out] = sub_end;
      } else {
        a.out_dist[pd.out] = v;
        if (kAux) a.out_aux[pd.out] = vx;
      }
    }
    wave_sync();
  }
}

// ------------------------------------------------------------------ dispatch

// `grid` counts sweep waves; the launch uses workgroups of kSweepWaves waves.
inline unsigned sweep_groups(int grid) {
  return (unsigned)((grid + kSweepWaves - 1) / kSweepWaves);
}

#define WTS_D_SWITCH(d, RHO, CALL)   \
  switch (d) {                       \
    case 1: return CALL(1, RHO);     \
    case 2: return CALL(2, RHO);     \
    case 3: return CALL(3, RHO);     \
    case 4: return CALL(4, RHO);     \
    case 5: return CALL(5, RHO);     \
    case 6: return CALL(6, RHO);     \
    case 7: return CALL(7, RHO);     \
    case 8: return CALL(8, RHO);     \
    default: return hipErrorInvalidValue; \
  }

template <typename TX, typename TY, typename TC, int D, int RHO, int MODE, bool EUC>
hipError_t launch_one(const FwdArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((dtw_fwd_kernel<TX, TY, TC, D, RHO, MODE, EUC>), dim3(sweep_groups(grid)),
                     dim3(kWave * kSweepWaves), 0, st, a);
  return hipGetLastError();
}

// The modes for one (X, Y, compute) type triple; the l2 cost is a
// float64 instance only.
template <typename TX, typename TY, typename TC, int D, int RHO>
hipError_t launch_fwd_t(int mode, bool euc, const FwdArgs& a, int grid, hipStream_t st) {
  if (mode == MODE_DIST) return launch_one<TX, TY, TC, D, RHO, MODE_DIST, false>(a, grid, st);
  if (mode == MODE_PATH) return launch_one<TX, TY, TC, D, RHO, MODE_PATH, false>(a, grid, st);
  if (mode == MODE_PATHT) return launch_one<TX, TY, TC, D, RHO, MODE_PATHT, false>(a, grid, st);
  if (mode == MODE_SUB) {
    if (euc) return hipErrorInvalidValue;
    return launch_one<TX, TY, TC, D, RHO, MODE_SUB, false>(a, grid, st);
  }
  if (euc) {
    if constexpr (sizeof(TC) == 8) return launch_one<TX, TY, TC, D, RHO, MODE_DIST_LEN, true>(a, grid, st);
    return hipErrorInvalidValue;
  }
  return launch_one<TX, TY, TC, D, RHO, MODE_DIST_LEN, false>(a, grid, st);
}

// rho 2 and 4: every mode; X is the float64 barycenter, or a cycle (the
// medoid's value sweep).  The float32 compute type needs float32 cycles.
template <typename TC, int D, int RHO>
hipError_t launch_fwd_d(int mode, bool euc, bool x_is_cycle, int ydtype, const FwdArgs& a,
                        int grid, hipStream_t st) {
  if (ydtype == 0) {
    if (x_is_cycle) {
      if (mode != MODE_DIST) return hipErrorInvalidValue;
      return launch_one<float, float, TC, D, RHO, MODE_DIST, false>(a, grid, st);
    }
    return launch_fwd_t<double, float, TC, D, RHO>(mode, euc, a, grid, st);
  }
  if constexpr (sizeof(TC) == 8) {
    if (x_is_cycle && mode != MODE_DIST) return hipErrorInvalidValue;
    return launch_fwd_t<double, double, TC, D, RHO>(mode, euc, a, grid, st);
  }
  return hipErrorInvalidValue;
}

// rho = 5 serves barycenter plans only (value+length, path and Sub-DTW sweeps).
template <typename TC, int D, int RHO>
hipError_t launch_fwd_bary(int mode, bool euc, bool x_is_cycle, int ydtype, const FwdArgs& a,
                           int grid, hipStream_t st) {
  if (x_is_cycle || mode == MODE_DIST) return hipErrorInvalidValue;
  if (ydtype == 0) return launch_fwd_t<double, float, TC, D, RHO>(mode, euc, a, grid, st);
  if constexpr (sizeof(TC) == 8) return launch_fwd_t<double, double, TC, D, RHO>(mode, euc, a, grid, st);
  return hipErrorInvalidValue;
}

// rho = 5 for the medoid: the value sweep between two cycles.
template <typename TC, int D, int RHO>
hipError_t launch_fwd_med(int mode, int ydtype, const FwdArgs& a, int grid, hipStream_t st) {
  if (mode != MODE_DIST) return hipErrorInvalidValue;
  if (ydtype == 0) return launch_one<float, float, TC, D, RHO, MODE_DIST, false>(a, grid, st);
  if constexpr (sizeof(TC) == 8) return launch_one<double, double, TC, D, RHO, MODE_DIST, false>(a, grid, st);
  return hipErrorInvalidValue;
}

template <typename TC>
hipError_t launch_fwd_impl(int d, int rho, int mode, bool euc, bool x_is_cycle, int ydtype,
                           const FwdArgs& a, int grid, hipStream_t st) {
#define CALLF(D, R) launch_fwd_d<TC, D, R>(mode, euc, x_is_cycle, ydtype, a, grid, st)
#define CALLB(D, R) launch_fwd_bary<TC, D, R>(mode, euc, x_is_cycle, ydtype, a, grid, st)
#define CALLM(D, R) launch_fwd_med<TC, D, R>(mode, ydtype, a, grid, st)
  if (rho == 4) { WTS_D_SWITCH(d, 4, CALLF) }
  if (rho == 2) { WTS_D_SWITCH(d, 2, CALLF) }
  if (rho == 5 && x_is_cycle) { WTS_D_SWITCH(d, 5, CALLM) }
  if (rho == 5) { WTS_D_SWITCH(d, 5, CALLB) }
#undef CALLM
#undef CALLB
#undef CALLF
  return hipErrorInvalidValue;
}

}  // namespace

}  // namespace wts
