// wts_dtw.hip -- DTW forward sweep, path recovery, DBA update, scores, medoid
// and barycenter initialisation for gfx950.
//
// The recurrence (Eq. 5 with gamma = 0, i.e. Eq. 1 by dynamic programming):
//   r(-1,-1) = 0, r(i,-1) = r(-1,j) = +inf,
//   r(i,j) = delta(x_i, y_j) + min(r(i-1,j-1), r(i-1,j), r(i,j-1)),
// all in float64, delta = e_0*e_0 then fma(e_c, e_c, s) (Def. 3, squared
// Euclidean).  The argmin of a cell is the first of diag, up, left that
// attains the minimum, kept as two bits (diagonal chosen; else up chosen);
// following them back from (M-1, N-1) gives the optimal path that Eq. 8
// divides by.
#include <climits>
#include <type_traits>

#include "wts_device.h"
#include "wts_kernels.h"

namespace wts {

namespace {

template <int D>
__device__ __forceinline__ double sq_cost(const double (&x)[D], const double (&y)[D]) {
  double e = x[0] - y[0];
  double s = e * e;
#pragma unroll
  for (int c = 1; c < D; ++c) {
    e = x[c] - y[c];
    s = __builtin_fma(e, e, s);
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
constexpr unsigned long long kSentR = 0xFFF4DEADBEEF0000ull;   // a NaN no arithmetic makes
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
// (float64 registers), the cumulative cost of those rows at the previous
// column (`left`) and, for the row above its first row, the value received
// one step earlier (`upprev`, the diagonal predecessor).
// The value sweep (medoid) runs on many items at once and is held to five
// resident wavefronts per SIMD; the other modes keep their registers.
template <typename TX, typename TY, int D, int RHO, int MODE, bool EUC>
__global__ __launch_bounds__(kWave * kSweepWaves, MODE == MODE_DIST && D <= 4 ? 5 : 1)
void dtw_fwd_kernel(FwdArgs a) {
  constexpr int H = kWave * RHO;
  constexpr bool kAux = MODE != MODE_DIST;
  // Y ring; slots kRing .. kRing+15 mirror slots 0 .. 15, so a group of 16
  // steps reads consecutive slots from one base without wrapping
  __shared__ double ys_[kSweepWaves][D][kRing + 16];
  __shared__ double binr_[kSweepWaves][16];   // strip above, this group's 16 columns
  __shared__ int binx_[kSweepWaves][16];
  // lane 63's bottom row of the last group; the other lanes write the same
  // steps into a scratch area (no exec-mask switch around the write)
  __shared__ double stg_r_[kSweepWaves][16 + kWave + 16];
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
  const double INF = inf_d();
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

    const double* r_in = a.bnd_r + pd.row_base + (int64_t)(s - 1) * RS;
    double* r_out = a.bnd_r + pd.row_base + (int64_t)s * RS;   // written via rr_out
    const int* x_in = a.bnd_aux + pd.row_base + (int64_t)(s - 1) * RS;
    int* x_out = a.bnd_aux + pd.row_base + (int64_t)s * RS;
    const __amdgpu_buffer_rsrc_t rr_out = rsrc(r_out, RS * 8);
    const __amdgpu_buffer_rsrc_t rx_out = rsrc(x_out, RS * 4);

    double xr[RHO][D];
#pragma unroll
    for (int r = 0; r < RHO; ++r) {
      const int i = ib + r;
#pragma unroll
      for (int c = 0; c < D; ++c)
        xr[r][c] = (i < M) ? static_cast<double>(X[(pd.x_off + i) * D + c]) : 0.0;
    }
    double left[RHO];
    int lx[RHO];
    uint32_t acc[RHO];
#pragma unroll
    for (int r = 0; r < RHO; ++r) { left[r] = INF; lx[r] = 0; acc[r] = 0u; }
    double upprev = (s == 0 && lane == 0) ? 0.0 : INF;   // r(-1,-1) = 0 at the origin
    // Sub-DTW: running minimum of the last row (lowest column on ties)
    const bool last_strip = s + 1 == pd.S;
    const int rl_last = M - 1 - ib;
    double sub_best = INF;
    int sub_end = 0, sub_start = 0;
    int upprevx = 0;
    double bot = INF;
    int botx = 0;
    bool gave_up = false;   // set once a wait times out: the strip never waits again

    // The strip above's bottom row, 16 columns at a time: lanes 0..15 hold the
    // next group's values in (pr, px) -- loaded one group ahead -- and wait
    // until none of them is a sentinel any more.  The prefetch is one
    // unconditional buffer load per value (lanes without a value read past
    // the record count and get 0; strip 0 has no records at all), so the
    // only wait for it is the check after the group's sweep steps.
    const __amdgpu_buffer_rsrc_t rr_in = rsrc(r_in, has_prev ? RS * 8 : 0);
    const __amdgpu_buffer_rsrc_t rx_in = rsrc(x_in, has_prev ? RS * 4 : 0);
    double pr = 0.0;
    int px = 0;
    auto fetch = [&](int tg) {
      const int j = tg + lane;
      const bool want = lane < 16 && j < N;
      pr = __builtin_bit_cast(
          double, __builtin_amdgcn_raw_buffer_load_b64(rr_in, want ? (j + 63) * 8 : kDrop, 0, 16));
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
      st_dev(rr_out, w ? (tg + lane) * 8 : kDrop, stg_r[lane & 15]);
      if (kAux) st_dev(rx_out, w ? (tg + lane) * 4 : kDrop, stg_x[lane & 15]);
      if (MODE == MODE_PATH) {
        const int64_t cw = pd.code_base + (int64_t)(s * pd.WT + (tg >> 4)) * RHO * kWave + lane;
#pragma unroll
        for (int r = 0; r < RHO; ++r) a.codes[cw + r * kWave] = acc[r];
      }
    };
    fetch(0);
    settle(0);

    // Y values are read from a clamped column (always in bounds) and zeroed
    // past N, so the loads are unconditional
    double yv[D];
    {
      const int j = lane;
      const int64_t row = (pd.y_off + min(j, N - 1)) * D;
#pragma unroll
      for (int c = 0; c < D; ++c) yv[c] = static_cast<double>(Y[row + c]);
#pragma unroll
      for (int c = 0; c < D; ++c) yv[c] = j < N ? yv[c] : 0.0;
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
        for (int c = 0; c < D; ++c) yv[c] = static_cast<double>(Y[row + c]);
#pragma unroll
        for (int c = 0; c < D; ++c) yv[c] = j < N ? yv[c] : 0.0;
      }

      // 16 sweep steps; FULL: every lane is inside the grid (no masking)
      auto group16 = [&](auto full_tag, int tb) {
        constexpr bool FULL = decltype(full_tag)::value;
        const int tg = t0 + tb;
        // LDS operands of step u+1 are read during step u (software pipelining)
        double yn[D];
        double bn;
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
          double y[D];
#pragma unroll
          for (int c = 0; c < D; ++c) y[c] = yn[c];
          const double bval = bn;
          const int bxv = bxn;
          if (u + 1 < 16) {
#pragma unroll
            for (int c = 0; c < D; ++c) yn[c] = ys[c][yb + u + 1];
            bn = binr[u + 1];
            if (MODE == MODE_DIST_LEN || MODE == MODE_SUB) bxn = binx[u + 1];
          }
          const double upin = shr1_f64(bot, bval);
          int upinx = 0, dgx0 = 0;
          if (MODE == MODE_DIST_LEN) {
            upinx = shr1_i32(botx, bxv);
            dgx0 = upprevx;
          } else if (MODE == MODE_PATH) {
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
          const double dg0 = upprev;
          upprev = upin;
          upprevx = upinx;
          bool isd_r[RHO], isu_r[RHO];   // argmin of each row's cell (PATH)
#pragma unroll
          for (int r = 0; r < RHO; ++r) { isd_r[r] = false; isu_r[r] = false; }
          if (FULL || (j >= 0 && j < N)) {
            double dg = dg0, up = upin;
            int dgx = dgx0, upx = upinx;
#pragma unroll
            for (int r = 0; r < RHO; ++r) {
              const double lf = left[r];
              const double m1 = __builtin_fmin(up, lf);
              const double m = __builtin_fmin(dg, m1);
              double delta = sq_cost<D>(xr[r], y);
              if (EUC) delta = __builtin_sqrt(delta);
              const double rv = delta + m;
              int rxv = 0;
              if (MODE != MODE_DIST) {
                const bool isd = dg <= m1;
                const bool isu = up <= lf;
                // keep these as lane selects (v_cndmask), not branches
                const int t1 = __builtin_unpredictable(isu) ? upx : lx[r];
                const int sel = __builtin_unpredictable(isd) ? dgx : t1;
                rxv = MODE == MODE_DIST_LEN ? sel + 1 : sel;
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
              double v = left[0];
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
          if (MODE == MODE_PATH) {
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
          binr[lane] = has_prev ? (tg + lane < N ? pr : INF) : (MODE == MODE_SUB ? 0.0 : INF);
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
      double v = left[0];
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
        if (MODE != MODE_DIST) a.out_aux[pd.out] = vx;
      }
    }
    wave_sync();
  }
}

// Strip-level path recovery.  The forward sweep tagged every cell with the
// top-row cell through which its optimal path enters the strip (code 2j for
// "from (i0-1, j)", 2j+1 for "from (i0-1, j-1)"), and kept that tag for the
// bottom row of every strip.  Walking the tags from (M-1, N-1) gives, per
// strip, where the path crosses its bottom row and its top row.
__global__ void chain_kernel(const PairDesc* __restrict__ pairs, int n_pairs,
                             const int* __restrict__ bnd_aux, const int* __restrict__ out_aux,
                             int2* __restrict__ seg, int* __restrict__ status,
                             const int* __restrict__ skip) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs || skipped(skip)) return;
  const PairDesc pd = pairs[p];
  int e = out_aux[pd.out];
  int jx = pd.N - 1;
  for (int s = pd.S - 1; s >= 0; --s) {
    const int jtop = e >> 1;
    if (jtop < 0 || jtop > jx) {   // inconsistent tags: mark every strip left empty
      atomicOr(status, kStatusBadPath);
      for (int q = s; q >= 0; --q) seg[pd.item_base + q] = make_int2(-1, -1);
      return;
    }
    seg[pd.item_base + s] = make_int2(jx, jtop);
    if (s == 0) break;
    const int jp = jtop - (e & 1);
    if (jp < 0) {
      atomicOr(status, kStatusBadPath);
      for (int q = s - 1; q >= 0; --q) seg[pd.item_base + q] = make_int2(-1, -1);
      return;
    }
    e = bnd_aux[pd.row_base + (int64_t)(s - 1) * row_stride(pd.N) + jp + 63];
    jx = jp;
  }
}

constexpr int kWalkWords = 16;   // code words (per row and lane) staged in LDS at a time

// Walks the optimal path through one strip, from its bottom-row crossing to
// its top-row cell, with the strip's argmin codes staged in LDS.  All 64
// lanes walk in lockstep (identical state), so the staging loads are
// cooperative and the LDS reads are broadcasts.
//   EMIT = false: per-row runs -> DBA partial sums (psum != nullptr) and the
//                 strip's segment length;
//   EMIT = true:  writes the segment's (i, j) pairs into the path list.
template <typename TY, int D, int RHO, bool EMIT>
__global__ __launch_bounds__(kWave) void walk_kernel(WalkArgs a) {
  constexpr int H = kWave * RHO;
  __shared__ uint32_t blk[kWalkWords][RHO][kWave];
  __shared__ int run_lo[H];
  __shared__ int run_hi[H];
  const int lane = threadIdx.x;
  const int item = blockIdx.x;
  if (skipped(a.skip)) return;
  const int2 it = a.items[item];
  const PairDesc pd = a.pairs[it.x];
  const int s = it.y;
  const int i0 = s * H;
  const int iend = min(pd.M, i0 + H) - 1;
  const int2 sg = a.seg[item];
  const uint32_t* codes = a.codes + pd.code_base + (int64_t)s * pd.WT * RHO * kWave;

  int i = iend, j = sg.x, hi = sg.x;
  const int jstop = sg.y;
  // An inconsistent path (the chain reported one, or the walk leaves the
  // strip) is flagged in the status word; the strip then contributes empty
  // row runs, so no later access depends on the bad path.
  bool bad = sg.x < 0 || sg.x >= pd.N || sg.y < 0 || sg.y > sg.x;
  if (bad && lane == 0) atomicOr(a.status, kStatusBadPath);
  int wlo = 1 << 30, whi = -1;
  uint32_t cw[RHO];
  int ck = -1, cwk = -1;
  int cnt = 0;
  int32_t* out = nullptr;
  int seg_len = 0;
  if (EMIT) {
    out = a.paths + 2 * (a.path_base[pd.out] + a.seg_off[item]);
    seg_len = a.seg_len[item];
  }
  while (!bad) {
    if (i < i0 || j < 0 || (EMIT && cnt >= seg_len)) {   // left the strip: inconsistent tags
      if (lane == 0) atomicOr(a.status, kStatusBadPath);
      bad = true;
      break;
    }
    if (EMIT && lane == 0) {
      out[2 * (seg_len - 1 - cnt)] = i;
      out[2 * (seg_len - 1 - cnt) + 1] = j;
    }
    ++cnt;
    if (i == i0 && j == jstop) {
      if (!EMIT && lane == 0) { run_lo[0] = j; run_hi[0] = hi; }
      break;
    }
    const int q = i - i0;
    const int k = q / RHO, r = q - k * RHO;
    const int t = j + k;
    const int w = t >> 4;
    if (k != ck || w != cwk) {   // the RHO words of (lane k, word w) into registers
      if (w < wlo || w > whi) {
        __syncthreads();
        wlo = max(0, w - kWalkWords + 1);
        whi = w;
        for (int ww = wlo; ww <= whi; ++ww)
#pragma unroll
          for (int rr = 0; rr < RHO; ++rr)
            blk[ww - wlo][rr][lane] = codes[((int64_t)ww * RHO + rr) * kWave + lane];
        __syncthreads();
      }
#pragma unroll
      for (int rr = 0; rr < RHO; ++rr) cw[rr] = blk[w - wlo][rr][k];
      ck = k;
      cwk = w;
    }
    uint32_t word = cw[0];
#pragma unroll
    for (int rr = 1; rr < RHO; ++rr) word = r == rr ? cw[rr] : word;
    // step u of a word: bit 31-2u = diagonal chosen, bit 30-2u = up chosen
    const int u = t & 15;
    const uint32_t code = (word >> (30 - 2 * u)) & 3u;
    if (code == 0u) {   // left
      --j;
      if (!EMIT && u > 0) {
        // the cells (i, j), (i, j-1), ... of this word that are left moves
        // too: their fields (steps u-1, u-2, ...) sit above this one
        const uint32_t rest = word >> (32 - 2 * u);
        int more = rest == 0u ? u : (int)(__builtin_ctz(rest) >> 1);
        if (i == i0) more = min(more, j - jstop);   // the run ends at the entry cell
        j -= more;
        cnt += more;
      }
    } else {
      if (!EMIT && lane == 0) { run_lo[q] = j; run_hi[q] = hi; }
      --i;
      if (code & 2u) --j;   // diagonal
      hi = j;
    }
  }
  if (EMIT) return;
  if (lane == 0) a.seg_len[item] = bad ? 0 : cnt;
  if (a.psum == nullptr) return;
  __syncthreads();
  const TY* __restrict__ Y = static_cast<const TY*>(a.y);
  const int nrows = iend - i0 + 1;
  for (int q = lane; q < nrows; q += kWave) {
    const int lo = bad ? 0 : run_lo[q], h = bad ? -1 : run_hi[q];
    const int64_t o = ((int64_t)pd.out * a.L + i0 + q);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double acc = 0.0;
      for (int jj = h; jj >= lo; --jj) acc = acc + static_cast<double>(Y[(pd.y_off + jj) * D + c]);
      a.psum[o * D + c] = acc;
    }
    a.pcnt[o] = h - lo + 1;
  }
}

}  // namespace

// --------------------------------------------------------------- small kernels

__global__ void zero_i32_kernel(int* p, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = 0;
}

// Sentinel fill of the strip boundary rows before a sweep.
__global__ void fill_sent_kernel(unsigned long long* r, int64_t nr, int* x, int64_t nx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nr; k += stride)
    r[k] = kSentR;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nx; k += stride)
    x[k] = kSentX;
}

// Segment offsets in forward path order (strip 0 first) and |pi| per pair.
__global__ void seg_prefix_kernel(const PairDesc* __restrict__ pairs, int n_pairs,
                                  const int* __restrict__ seg_len, int* __restrict__ seg_off,
                                  int64_t* __restrict__ path_len) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const PairDesc pd = pairs[p];
  int off = 0;
  for (int s = 0; s < pd.S; ++s) {
    seg_off[pd.item_base + s] = off;
    off += seg_len[pd.item_base + s];
  }
  if (path_len) path_len[pd.out] = off;
}

// B'_l = S_l / C_l with S_l, C_l folded over cycles in ascending order.
__global__ void dba_reduce_kernel(const double* __restrict__ psum, const int* __restrict__ pcnt,
                                  const double* __restrict__ w, int n, int64_t L, int d,
                                  double* __restrict__ bout, int64_t* __restrict__ counts) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= L * d) return;
  const int64_t l = idx / d;
  const int c = (int)(idx - l * d);
  double S = 0.0, C = 0.0;
  int64_t K = 0;
  for (int p = 0; p < n; ++p) {
    const double wp = w ? w[p] : 1.0;
    S = S + wp * psum[((int64_t)p * L + l) * d + c];
  }
  for (int p = 0; p < n; ++p) {
    const double wp = w ? w[p] : 1.0;
    const int k = pcnt[(int64_t)p * L + l];
    C = C + wp * (double)k;
    K += k;
  }
  bout[idx] = S / C;
  if (c == 0 && counts) counts[l] = K;
}

__global__ void score_kernel(const double* __restrict__ dist, const int* __restrict__ len, int n,
                             double* __restrict__ score, int64_t* __restrict__ path_len) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double dv = dist[p];
  const int lv = len[p];
  if (score) score[p] = dv / (double)lv;
  if (path_len) path_len[p] = lv;
}

// Medoid: D[a][b] = D[b][a] = DTW of pair (a, b); totals in ascending order.
__global__ void medoid_fill_kernel(const double* __restrict__ pair_dist,
                                   const int2* __restrict__ pair_ab, int n_pairs, int n,
                                   double* __restrict__ Dm) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n_pairs) {
    const int2 ab = pair_ab[k];
    Dm[(int64_t)ab.x * n + ab.y] = pair_dist[k];
    Dm[(int64_t)ab.y * n + ab.x] = pair_dist[k];
  }
  if (k < n) Dm[k * n + k] = 0.0;
}

__global__ void medoid_total_kernel(const double* __restrict__ Dm, int n,
                                    double* __restrict__ totals) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s = s + Dm[(int64_t)k * n + i];
  totals[k] = s;
}

__global__ void medoid_argmin_kernel(const double* __restrict__ totals, int n,
                                     int32_t* __restrict__ medoid) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int best = 0;
  double bv = inf_d();
  for (int k = 0; k < n; ++k)
    if (totals[k] < bv) { bv = totals[k]; best = k; }
  *medoid = best;
}

// Resampling at t_l = l (N-1)/(L-1); source = one cycle, or (euclid = true)
// the per-index mean of all cycles padded with their last sample.
template <typename TY>
__global__ void init_kernel(const TY* __restrict__ Y, const int64_t* __restrict__ off, int n,
                            int d, int src, int64_t Nsrc, int64_t L, int euclid,
                            double* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= L * d) return;
  const int64_t l = idx / d;
  const int c = (int)(idx - l * d);
  auto sample = [&](int64_t tt) -> double {
    if (!euclid) return static_cast<double>(Y[(off[src] + tt) * d + c]);
    double s = 0.0;
    for (int p = 0; p < n; ++p) {
      const int64_t Np = off[p + 1] - off[p];
      const int64_t q = tt < Np ? tt : Np - 1;
      s = s + static_cast<double>(Y[(off[p] + q) * d + c]);
    }
    return s / (double)n;
  };
  const double pos = L == 1 ? 0.0 : ((double)l * (double)(Nsrc - 1)) / (double)(L - 1);
  const int64_t a0 = (int64_t)__builtin_floor(pos);
  double v;
  if (a0 >= Nsrc - 1) {
    v = sample(Nsrc - 1);
  } else {
    const double f = pos - (double)a0;
    const double ya = sample(a0), yb = sample(a0 + 1);
    v = ya + f * (yb - ya);
  }
  out[idx] = v;
}

// ------------------------------------------------------------------ dispatch

// `grid` counts sweep waves; the launch uses workgroups of kSweepWaves waves.
static inline unsigned sweep_groups(int grid) {
  return (unsigned)((grid + kSweepWaves - 1) / kSweepWaves);
}

template <typename TX, typename TY, int D, int RHO>
static hipError_t launch_fwd_t(int mode, bool euc, const FwdArgs& a, int grid, hipStream_t st) {
  if (mode == MODE_DIST) {
    hipLaunchKernelGGL((dtw_fwd_kernel<TX, TY, D, RHO, MODE_DIST, false>), dim3(sweep_groups(grid)),
                       dim3(kWave * kSweepWaves), 0, st, a);
  } else if (mode == MODE_DIST_LEN) {
    if (euc)
      hipLaunchKernelGGL((dtw_fwd_kernel<TX, TY, D, RHO, MODE_DIST_LEN, true>), dim3(sweep_groups(grid)),
                         dim3(kWave * kSweepWaves), 0, st, a);
    else
      hipLaunchKernelGGL((dtw_fwd_kernel<TX, TY, D, RHO, MODE_DIST_LEN, false>), dim3(sweep_groups(grid)),
                         dim3(kWave * kSweepWaves), 0, st, a);
  } else if (mode == MODE_PATH) {
    hipLaunchKernelGGL((dtw_fwd_kernel<TX, TY, D, RHO, MODE_PATH, false>), dim3(sweep_groups(grid)),
                       dim3(kWave * kSweepWaves), 0, st, a);
  } else {
    if (euc) return hipErrorInvalidValue;
    hipLaunchKernelGGL((dtw_fwd_kernel<TX, TY, D, RHO, MODE_SUB, false>), dim3(sweep_groups(grid)),
                       dim3(kWave * kSweepWaves), 0, st, a);
  }
  return hipGetLastError();
}

template <int D, int RHO>
static hipError_t launch_fwd_d(int mode, bool euc, bool x_is_cycle, int ydtype,
                               const FwdArgs& a, int grid, hipStream_t st) {
  if (ydtype == 0) {
    if (x_is_cycle) {
      if (mode != MODE_DIST) return hipErrorInvalidValue;
      hipLaunchKernelGGL((dtw_fwd_kernel<float, float, D, RHO, MODE_DIST, false>), dim3(sweep_groups(grid)),
                         dim3(kWave * kSweepWaves), 0, st, a);
      return hipGetLastError();
    }
    return launch_fwd_t<double, float, D, RHO>(mode, euc, a, grid, st);
  }
  if (x_is_cycle && mode != MODE_DIST) return hipErrorInvalidValue;
  return launch_fwd_t<double, double, D, RHO>(mode, euc, a, grid, st);
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

// rho = 5 serves barycenter plans only (value+length, path and Sub-DTW sweeps).
template <int D, int RHO>
static hipError_t launch_fwd_bary(int mode, bool euc, bool x_is_cycle, int ydtype,
                                  const FwdArgs& a, int grid, hipStream_t st) {
  if (x_is_cycle || mode == MODE_DIST) return hipErrorInvalidValue;
  const dim3 g(sweep_groups(grid)), b(kWave * kSweepWaves);
  if (mode == MODE_SUB && euc) return hipErrorInvalidValue;
  if (ydtype == 0) {
    if (mode == MODE_SUB)
      hipLaunchKernelGGL((dtw_fwd_kernel<double, float, D, RHO, MODE_SUB, false>), g, b, 0, st, a);
    else if (mode == MODE_PATH)
      hipLaunchKernelGGL((dtw_fwd_kernel<double, float, D, RHO, MODE_PATH, false>), g, b, 0, st, a);
    else if (euc)
      hipLaunchKernelGGL((dtw_fwd_kernel<double, float, D, RHO, MODE_DIST_LEN, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((dtw_fwd_kernel<double, float, D, RHO, MODE_DIST_LEN, false>), g, b, 0, st, a);
  } else {
    if (mode == MODE_SUB)
      hipLaunchKernelGGL((dtw_fwd_kernel<double, double, D, RHO, MODE_SUB, false>), g, b, 0, st, a);
    else if (mode == MODE_PATH)
      hipLaunchKernelGGL((dtw_fwd_kernel<double, double, D, RHO, MODE_PATH, false>), g, b, 0, st, a);
    else if (euc)
      hipLaunchKernelGGL((dtw_fwd_kernel<double, double, D, RHO, MODE_DIST_LEN, true>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((dtw_fwd_kernel<double, double, D, RHO, MODE_DIST_LEN, false>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

// rho = 5 for the medoid: the value sweep between two cycles.
template <int D, int RHO>
static hipError_t launch_fwd_med(int mode, int ydtype, const FwdArgs& a, int grid, hipStream_t st) {
  if (mode != MODE_DIST) return hipErrorInvalidValue;
  const dim3 g(sweep_groups(grid)), b(kWave * kSweepWaves);
  if (ydtype == 0)
    hipLaunchKernelGGL((dtw_fwd_kernel<float, float, D, RHO, MODE_DIST, false>), g, b, 0, st, a);
  else
    hipLaunchKernelGGL((dtw_fwd_kernel<double, double, D, RHO, MODE_DIST, false>), g, b, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fwd(int d, int rho, int mode, bool euc, bool x_is_cycle, int ydtype,
                      const FwdArgs& a, int grid, hipStream_t st) {
#define CALLF(D, R) launch_fwd_d<D, R>(mode, euc, x_is_cycle, ydtype, a, grid, st)
#define CALLB(D, R) launch_fwd_bary<D, R>(mode, euc, x_is_cycle, ydtype, a, grid, st)
#define CALLM(D, R) launch_fwd_med<D, R>(mode, ydtype, a, grid, st)
  if (rho == 4) { WTS_D_SWITCH(d, 4, CALLF) }
  if (rho == 2) { WTS_D_SWITCH(d, 2, CALLF) }
  if (rho == 5 && x_is_cycle) { WTS_D_SWITCH(d, 5, CALLM) }
  if (rho == 5) { WTS_D_SWITCH(d, 5, CALLB) }
#undef CALLM
#undef CALLB
#undef CALLF
  return hipErrorInvalidValue;
}

template <typename TY, int D, int RHO>
static hipError_t launch_walk_t(bool emit, const WalkArgs& a, int n_items, hipStream_t st) {
  if (emit)
    hipLaunchKernelGGL((walk_kernel<TY, D, RHO, true>), dim3(n_items), dim3(kWave), 0, st, a);
  else
    hipLaunchKernelGGL((walk_kernel<TY, D, RHO, false>), dim3(n_items), dim3(kWave), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_walk(int d, int rho, int ydtype, bool emit, const WalkArgs& a, int n_items,
                       hipStream_t st) {
#define CALLW(D, R) (ydtype == 0 ? launch_walk_t<float, D, R>(emit, a, n_items, st) \
                                 : launch_walk_t<double, D, R>(emit, a, n_items, st))
  if (rho == 4) { WTS_D_SWITCH(d, 4, CALLW) }
  if (rho == 2) { WTS_D_SWITCH(d, 2, CALLW) }
  if (rho == 5) { WTS_D_SWITCH(d, 5, CALLW) }
#undef CALLW
  return hipErrorInvalidValue;
}

hipError_t launch_chain(const PairDesc* pairs, int n_pairs, const int* bnd_aux,
                        const int* out_aux, int2* seg, int* status, const int* skip,
                        hipStream_t st) {
  hipLaunchKernelGGL(chain_kernel, dim3((n_pairs + 63) / 64), dim3(64), 0, st, pairs, n_pairs,
                     bnd_aux, out_aux, seg, status, skip);
  return hipGetLastError();
}

hipError_t launch_zero(int* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256),
                     0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_sentinels(double* r, int64_t nr, int* x, int64_t nx, hipStream_t st) {
  const int64_t n = nr > nx ? nr : nx;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_sent_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0,
                     st, reinterpret_cast<unsigned long long*>(r), nr, x, nx);
  return hipGetLastError();
}

hipError_t launch_seg_prefix(const PairDesc* pairs, int n_pairs, const int* seg_len,
                             int* seg_off, int64_t* path_len, hipStream_t st) {
  hipLaunchKernelGGL(seg_prefix_kernel, dim3((n_pairs + 63) / 64), dim3(64), 0, st, pairs,
                     n_pairs, seg_len, seg_off, path_len);
  return hipGetLastError();
}

hipError_t launch_dba_reduce(const double* psum, const int* pcnt, const double* w, int n,
                             int64_t L, int d, double* bout, int64_t* counts, hipStream_t st) {
  const int64_t tot = L * d;
  hipLaunchKernelGGL(dba_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     psum, pcnt, w, n, L, d, bout, counts);
  return hipGetLastError();
}

hipError_t launch_score(const double* dist, const int* len, int n, double* score,
                        int64_t* path_len, hipStream_t st) {
  hipLaunchKernelGGL(score_kernel, dim3((n + 255) / 256), dim3(256), 0, st, dist, len, n, score,
                     path_len);
  return hipGetLastError();
}

// Sub-DTW columns (a*, b*) as int64.
__global__ void sub_out_kernel(const int* __restrict__ start, const int* __restrict__ end, int n,
                               int64_t* __restrict__ a_star, int64_t* __restrict__ b_star) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  a_star[p] = start[p];
  b_star[p] = end[p];
}

hipError_t launch_sub_out(const int* start, const int* end, int n, int64_t* a_star,
                          int64_t* b_star, hipStream_t st) {
  hipLaunchKernelGGL(sub_out_kernel, dim3((n + 255) / 256), dim3(256), 0, st, start, end, n,
                     a_star, b_star);
  return hipGetLastError();
}

hipError_t launch_medoid(const double* pair_dist, const int2* pair_ab, int n_pairs, int n,
                         double* Dm, double* totals, int32_t* medoid, hipStream_t st) {
  const int64_t m = n_pairs > n ? n_pairs : n;
  hipLaunchKernelGGL(medoid_fill_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                     pair_dist, pair_ab, n_pairs, n, Dm);
  hipLaunchKernelGGL(medoid_total_kernel, dim3((n + 255) / 256), dim3(256), 0, st, Dm, n, totals);
  hipLaunchKernelGGL(medoid_argmin_kernel, dim3(1), dim3(64), 0, st, totals, n, medoid);
  return hipGetLastError();
}

hipError_t launch_init(int ydtype, const void* Y, const int64_t* off, int n, int d, int src,
                       int64_t Nsrc, int64_t L, int euclid, double* out, hipStream_t st) {
  const int64_t tot = L * d;
  const dim3 g((unsigned)((tot + 255) / 256));
  if (ydtype == 0)
    hipLaunchKernelGGL(init_kernel<float>, g, dim3(256), 0, st, static_cast<const float*>(Y), off,
                       n, d, src, Nsrc, L, euclid, out);
  else
    hipLaunchKernelGGL(init_kernel<double>, g, dim3(256), 0, st, static_cast<const double*>(Y),
                       off, n, d, src, Nsrc, L, euclid, out);
  return hipGetLastError();
}

}  // namespace wts
