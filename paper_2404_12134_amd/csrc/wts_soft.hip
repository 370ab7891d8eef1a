// wts_soft.hip -- Soft-DTW forward (Eq. 3-5) and its gradient (Eq. 6) for gfx950.
//
// Units.  The cumulative costs are kept scaled, R' = R * k with
// k = log2(e) / gamma, so the soft-min of Eq. 3 becomes
//   min'(a, b, c) = m - log2(2^(m-a) + 2^(m-b) + 2^(m-c)),  m = min(a, b, c),
// evaluated with float64 differences and the hardware base-2 exponential and
// logarithm (v_exp_f32 / v_log_f32).  Every cost delta enters as delta * k:
// the kernels take the series multiplied by sqrt(k) when they load them, so
// the squared differences come out scaled with no multiply per cell (the
// gradient's sums are scaled back once per row).  The Soft-DTW value is
// r'(M-1, N-1) / k.
//
// Forward.  Same skewed wavefront sweep as the DTW kernels (one wave per strip
// of 64*RHO rows, strips of a pair chained through device memory).  It keeps
// every strip's bottom row and, every 16 sweep steps, the sweep state of each
// lane (its RHO cumulative costs at the previous column and the diagonal
// input from the row above): enough to replay any 16-step tile.
//
// Backward.  E of Eq. 6 follows from Eq. 5 by the chain rule:
//   e(i, j) = sum over the successors s of (i, j) of e(s) * w_s(i, j),
// where w_s(i, j) = 2^(m_s - r'(i, j)) / sum_s is the normalised weight of
// (i, j) in the soft-min of its successor s, and e(M-1, N-1) = 1 (the cell
// that closes the path).  The kernel walks each strip's tiles from the last
// column to the first: it replays the tile forward, keeping the normalised
// weights of the up and left predecessors of every cell in registers
// (float32), then sweeps the tile backwards in "push" form -- each finished
// cell splits its e over its three predecessors with its own weights, the
// diagonal taking what the other two do not, so that the split conserves e
// up to the rounding of one float32 subtraction -- and no cell ever needs a
// neighbour's weights.  e lies in [0, 1] and travels in float32 (registers,
// lane shifts, LDS and the push rows between strips).  The pushes of a
// strip's top row feed the strip above, so strips are pipelined from the
// bottom up.  Per row l of the barycenter the kernel accumulates, in
// float64, sum_j e(l, j) and sum_j e(l, j) y_j, and the gradient is
//   d Soft-DTW / d b_l = 2 (b_l * sum_j e(l, j) - sum_j e(l, j) y_j).
#include <type_traits>

#include "wts_device.h"
#include "wts_kernels.h"

namespace wts {

namespace {


__device__ __forceinline__ double shl1_f64(double v, double old) {
  // DPP wave_shl:1 -- lane k receives v from lane k+1; lane 63 receives `old`.
  const long long s = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x130, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float shl1_f32(float v, float old) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, v), 0x130,
                                                               0xf, 0xf, false));
}

constexpr int kRing = 128;   // Y columns in LDS (>= 16 + 63 for a tile, power of 2)
// The ring holds kRing + 16 slots: slots kRing .. kRing + 15 mirror slots
// 0 .. 15, so the 16 steps of a group read consecutive slots yb .. yb + 15
// from one base (immediate LDS offsets, no wrap-around per step).
__device__ __forceinline__ void ring_put(double* row, int slot, double v) {
  row[slot] = v;
  if (slot < 16) row[slot + kRing] = v;
}
constexpr int kTile = 16;    // sweep steps per checkpoint / replay tile

// Def. 3's squared cost in the scaled units of these kernels, k |x - y|^2,
// in d + 1 operations per cell: the rows carry x' = sk (x - mu) and
// |x'|^2, the columns y' = sk (y - mu) as -2 y' and |y'|^2, and
// k |x - y|^2 = |x'|^2 + |y'|^2 + x' . (-2 y').  mu, the first row of the
// pair's row series, keeps the three terms of the order of the series'
// spread, so cancellation costs no more than a few roundings of that size.
template <int D>
__device__ __forceinline__ double sq_cost(const double (&x)[D], double xx, const double (&ym2)[D],
                                          double yy) {
  double s = xx + yy;
#pragma unroll
  for (int c = 0; c < D; ++c) s = __builtin_fma(x[c], ym2[c], s);
  return s;
}
template <int D>
__device__ __forceinline__ double sq_norm(const double (&v)[D]) {
  double q = v[0] * v[0];
#pragma unroll
  for (int c = 1; c < D; ++c) q = __builtin_fma(v[c], v[c], q);
  return q;
}
// One column into the Y ring: -2 y' per channel and |y'|^2.
template <int D>
__device__ __forceinline__ void ring_col(double (*ys)[kRing + 16], double* yq, int slot,
                                         const double (&yc)[D]) {
#pragma unroll
  for (int c = 0; c < D; ++c) ring_put(ys[c], slot, -2.0 * yc[c]);
  ring_put(yq, slot, sq_norm<D>(yc));
}

// Soft-min of the three predecessors in scaled units.  Returns the soft-min
// value and the three (unnormalised) base-2 exponentials.
struct SoftMin {
  double v;
  float ed, eu, el, s;
};
__device__ __forceinline__ SoftMin softmin3(double dg, double up, double lf) {
  const double m = __builtin_fmin(__builtin_fmin(dg, up), lf);
  SoftMin o;
  o.ed = __builtin_amdgcn_exp2f((float)(m - dg));
  o.eu = __builtin_amdgcn_exp2f((float)(m - up));
  o.el = __builtin_amdgcn_exp2f((float)(m - lf));
  o.s = (o.ed + o.eu) + o.el;
  o.v = m - (double)__builtin_amdgcn_logf(o.s);
  return o;
}

// Sakoe-Chiba band (the bandwidth of Table I, a fraction w of the longer
// length): cell (i, j) of an M x N pair lies in the band iff
//   |i (N-1) - j (M-1)| <= B,   B = R min(M-1, N-1),
//   R = max(ceil(w max(M, N)), ceil(max(M-1, N-1) / min(M-1, N-1))),
// a band of radius R around the diagonal from (0, 0) to (M-1, N-1) along
// the longer side; the lower bound on R keeps a predecessor in the band for
// every cell of the band but (0, 0).  Returns B, or +inf (every cell) when
// w = 0 or a side has length 1.  The test is done in float64, exact for
// M, N < 2^26 (checked at plan time).
__device__ __forceinline__ double band_halfwidth(int M, int N, double w) {
  if (!(w > 0.0) || M == 1 || N == 1) return __builtin_huge_val();
  const int64_t am = M - 1, bn = N - 1;
  const int64_t mn = am < bn ? am : bn, mx = am < bn ? bn : am;
  int64_t R = (int64_t)__builtin_ceil(w * (double)(M > N ? M : N));
  const int64_t Rmin = (mx + mn - 1) / mn;
  if (R < Rmin) R = Rmin;
  return (double)(R * mn);
}

// Columns of the band over rows i_first .. i_last (the band's left edge is
// non-decreasing in i, so the range runs from row i_first's left edge to row
// i_last's right edge), in exact integer arithmetic: a 16-step group whose
// cells all lie outside it can skip its cell arithmetic.
__device__ __forceinline__ void band_strip_cols(int M, int N, double w, int i_first, int i_last,
                                                int* jlo, int* jhi) {
  *jlo = 0;
  *jhi = N - 1;
  if (!(w > 0.0) || M == 1 || N == 1) return;
  const int64_t am = M - 1, bn = N - 1;
  const int64_t B = (int64_t)band_halfwidth(M, N, w);
  // left edge of row i: ceil((i bn - B) / am); right edge: floor((i bn + B) / am)
  auto floor_div = [](int64_t x, int64_t y) { return x / y - ((x % y != 0) && (x < 0)); };
  const int64_t lo = -floor_div(B - (int64_t)i_first * bn, am);
  const int64_t hi = floor_div((int64_t)i_last * bn + B, am);
  if (lo > 0) *jlo = (int)(lo < bn ? lo : bn);
  if (hi < bn) *jhi = (int)(hi > 0 ? hi : 0);
}

// softmin3 for a cell that may lie outside the band: there every input may
// be +inf, so the shift m is replaced by 0 to keep the arithmetic free of
// inf - inf (the caller discards the result of such a cell).
__device__ __forceinline__ SoftMin softmin3_band(double dg, double up, double lf, bool inb) {
  double m = __builtin_fmin(__builtin_fmin(dg, up), lf);
  m = inb ? m : 0.0;
  SoftMin o;
  o.ed = __builtin_amdgcn_exp2f((float)(m - dg));
  o.eu = __builtin_amdgcn_exp2f((float)(m - up));
  o.el = __builtin_amdgcn_exp2f((float)(m - lf));
  o.s = (o.ed + o.eu) + o.el;
  o.v = m - (double)__builtin_amdgcn_logf(o.s);
  return o;
}

// --------------------------------------------------------------- forward

template <typename TY, int D, int RHO, bool BAND>
__global__ __launch_bounds__(kWave) void soft_fwd_kernel(SoftArgs a) {
  constexpr int H = kWave * RHO;
  constexpr int kChunk = 64;
  __shared__ double ys[D][kRing + 16];   // -2 y' of the columns (see sq_cost)
  __shared__ double yq[kRing + 16];      // |y'|^2
  __shared__ double binr[kChunk];       // the strip above's bottom row (+inf for the top strip)
  __shared__ double bor[kRing];
  __shared__ int s_item;
  const int lane = threadIdx.x;
  const TY* __restrict__ Y = static_cast<const TY*>(a.y);
  const double INF = inf_d();
  const double k = a.kscale;
  const double sk = __builtin_sqrt(k);   // x and y enter as sqrt(k) (x - mu), sqrt(k) (y - mu)
  if (skipped(a.skip)) return;   // every workgroup: no strip waits for another

  for (;;) {
    if (lane == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: scalar loads below
    __syncthreads();
    if (item >= a.n_items) break;
    const int2 it = a.items[item];
    const PairDesc pd = uniform(a.pairs[uni(it.x)]);
    const int s = uni(it.y);
    const int M = pd.M, N = pd.N;
    double mu[D];
#pragma unroll
    for (int c = 0; c < D; ++c) mu[c] = a.x[pd.x_off * D + c];
    const int i0 = s * H;
    const int ib = i0 + lane * RHO;
    const double band_b = BAND ? band_halfwidth(M, N, a.band) : 0.0;
    int band_jlo = 0, band_jhi = N - 1;
    if (BAND) band_strip_cols(M, N, a.band, i0, min(i0 + H, M) - 1, &band_jlo, &band_jhi);
    // columns inside the band on every row of the strip (from the last row's
    // left edge to the first row's right edge; empty when they cross): a
    // group whose columns all lie there needs no band test.  The rows past
    // M - 1 of the last strip count too: the band test keeps them at +inf
    // where the band's formula puts them outside, and the unbanded arithmetic
    // would turn three +inf inputs into NaN.
    int band_in_lo = 0, band_in_hi = -1;
    if (BAND) band_strip_cols(M, N, a.band, i0 + H - 1, i0, &band_in_lo, &band_in_hi);
    const bool has_prev = s > 0;
    const bool has_next = s + 1 < pd.S;
    const int Tend = pd.WT * 16;
    const double* row_in = a.rows + pd.aux_base + (int64_t)(s - 1) * N;
    double* row_out = a.rows + pd.aux_base + (int64_t)s * N;
    double* st = a.states + pd.state_base + (int64_t)s * pd.WT * (RHO + 1) * kWave;
    int* prog_in = a.progress + pd.flag_base + s - 1;
    int* prog_out = a.progress + pd.flag_base + s;

    double xr[RHO][D], xx[RHO];
#pragma unroll
    for (int r = 0; r < RHO; ++r) {
#pragma unroll
      for (int c = 0; c < D; ++c)
        xr[r][c] = (ib + r < M) ? (a.x[(pd.x_off + ib + r) * D + c] - mu[c]) * sk : 0.0;
      xx[r] = sq_norm<D>(xr[r]);
    }
    double left[RHO];
#pragma unroll
    for (int r = 0; r < RHO; ++r) left[r] = INF;
    double upprev = (s == 0 && lane == 0) ? 0.0 : INF;
    double bot = INF;
    bool gave_up = false;       // wave-uniform
    int seen_prev = 0;          // last progress read from the strip above (uniform)
    bool have_next = false;     // pr_next holds the next chunk's upper input (uniform)
    double pr_next = INF;
    const __amdgpu_buffer_rsrc_t ro = rsrc(row_out, has_next ? N * 8 : 0);

    {
      double yc[D];
#pragma unroll
      for (int c = 0; c < D; ++c)
        yc[c] = lane < N ? (static_cast<double>(Y[(pd.y_off + lane) * D + c]) - mu[c]) * sk : 0.0;
      ring_col<D>(ys, yq, lane, yc);
    }
    __syncthreads();

    for (int t0 = 0; t0 < Tend; t0 += kChunk) {
      const int tcnt = min(kChunk, Tend - t0);
      const bool more = t0 + kChunk < Tend;
      // next chunk's Y columns: unconditional loads from a clamped column,
      // kept in the storage type until they are written to LDS after this
      // chunk (a conditional load would be waited for on the spot)
      TY yraw[D];
      {
        const int j = min(t0 + kChunk + lane, N - 1);
#pragma unroll
        for (int c = 0; c < D; ++c) yraw[c] = Y[(pd.y_off + j) * D + c];
      }
      if (has_prev) {
        // the strip above's bottom row for this chunk: prefetched during the
        // previous chunk when its counter already covered it, else read now
        // (one read of the counter usually covers many chunks)
        double pr = pr_next;
        if (!have_next) {
          const int need = min(N, t0 + kChunk);
          if (need > seen_prev && !gave_up) {
            int got = 0, quit = 0;
            if (lane == 0) {
              int polls = 0;
              got = ld_dev(prog_in);
              while (got < need) {
                poll_backoff(polls, a.relaxed_wait);
                if (++polls > kSpinLimit) {
                  atomicOr(a.status, kStatusSpinTimeout);
                  quit = 1;
                  break;
                }
                got = ld_dev(prog_in);
              }
            }
            seen_prev = __builtin_amdgcn_readfirstlane(got);
            gave_up = __builtin_amdgcn_readfirstlane(quit) != 0;
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          const int j = t0 + lane;
          pr = j < N ? ld_dev(row_in + j) : INF;
        }
        binr[lane] = pr;
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int jn = t0 + kChunk + lane;
        have_next = more && seen_prev >= min(N, t0 + 2 * kChunk);
        if (have_next) pr_next = jn < N ? ld_dev(row_in + jn) : INF;
      } else {
        binr[lane] = INF;
      }
      __syncthreads();

      // FULL: every lane is inside the grid (no masking); INSIDE: every cell
      // is inside the band as well (the unbanded arithmetic, which gives an
      // in-band cell the same bits as the band test's path)
      auto group16 = [&](auto full_tag, auto inside_tag, int tb) {
        constexpr bool FULL = decltype(full_tag)::value;
        constexpr bool TEST = BAND && !decltype(inside_tag)::value;
        const int tg = t0 + tb;
        {   // checkpoint: the sweep state at the start of these 16 steps
          double* p = st + (int64_t)(tg >> 4) * (RHO + 1) * kWave + lane;
#pragma unroll
          for (int r = 0; r < RHO; ++r) p[r * kWave] = left[r];
          p[RHO * kWave] = upprev;
        }
        const int yb = (tg - lane) & (kRing - 1);   // ring slot of step 0's column
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = tg + u;
          const int j = t - lane;
          const double bval = binr[tb + u];
          const double upin = shr1_f64(bot, bval);
          const double dg0 = upprev;
          upprev = upin;
          if (FULL || (j >= 0 && j < N)) {
            double y[D];
#pragma unroll
            for (int c = 0; c < D; ++c) y[c] = ys[c][yb + u];
            const double yy = yq[yb + u];
            double dg = dg0, up = upin;
            // band coordinate of row ib at column j (exact in float64)
            const double bd0 = (double)ib * (double)(N - 1) - (double)j * (double)(M - 1);
#pragma unroll
            for (int r = 0; r < RHO; ++r) {
              const double lf = left[r];
              double rv;
              if constexpr (TEST) {
                const bool inb = __builtin_fabs(bd0 + (double)r * (double)(N - 1)) <= band_b;
                const SoftMin sm = softmin3_band(dg, up, lf, inb);
                rv = inb ? sq_cost<D>(xr[r], xx[r], y, yy) + sm.v : INF;
              } else {
                const SoftMin sm = softmin3(dg, up, lf);
                rv = sq_cost<D>(xr[r], xx[r], y, yy) + sm.v;
              }
              dg = lf;
              up = rv;
              left[r] = rv;
            }
            bot = left[RHO - 1];
            if (has_next && lane == kWave - 1) bor[j & (kRing - 1)] = bot;
          }
        }
      };
      // a group whose columns (tg - 63 .. tg + 15 over the lanes) all lie
      // outside the strip's band keeps only its bookkeeping: checkpoint,
      // +inf state and bottom row, and lane 0's diagonal input of the next step
      auto skip16 = [&](int tb) {
        const int tg = t0 + tb;
        double* p = st + (int64_t)(tg >> 4) * (RHO + 1) * kWave + lane;
#pragma unroll
        for (int r = 0; r < RHO; ++r) p[r * kWave] = left[r];
        p[RHO * kWave] = upprev;
        // lanes with cells in the grid during the group end it at +inf; a lane
        // already past column N-1 keeps its values (as the sweep would)
        if (tg + 15 - lane >= 0 && tg - lane <= N - 1) {
#pragma unroll
          for (int r = 0; r < RHO; ++r) left[r] = INF;
          bot = INF;
        }
        upprev = (lane == 0 && has_prev) ? binr[tb + 15] : INF;
        if (has_next && lane < 16) {
          const int j = tg - (kWave - 1) + lane;
          if (j >= 0 && j < N) bor[j & (kRing - 1)] = INF;
        }
      };
      for (int tb = 0; tb < tcnt; tb += 16) {
        const int tg = t0 + tb;
        if (BAND && (tg + 15 < band_jlo || tg - (kWave - 1) > band_jhi)) {
          skip16(tb);
        } else if (tg >= kWave - 1 && tg + 16 <= N) {
          if (BAND && tg - (kWave - 1) >= band_in_lo && tg + 15 <= band_in_hi)
            group16(std::true_type{}, std::true_type{}, tb);
          else
            group16(std::true_type{}, std::false_type{}, tb);
        } else {
          group16(std::false_type{}, std::false_type{}, tb);
        }
      }
      __syncthreads();
      if (has_next) {
        // this chunk's columns of the bottom row (one store, dropped outside
        // the row), then the previous chunk's columns are announced: waiting
        // until at most this store is outstanding completes every older one
        const int jend = t0 + tcnt - (kWave - 1);
        const int j = t0 - (kWave - 1) + lane;
        const bool w = j >= 0 && j < N && j < jend;
        st_dev(ro, w ? j * 8 : kDrop, bor[j & (kRing - 1)]);
        mem_wait_all_but_1();
        if (lane == 0) st_dev(prog_out, min(N, max(0, t0 - (kWave - 1))));
      }
      if (more) {
        const int j = t0 + kChunk + lane;
        double yc[D];
#pragma unroll
        for (int c = 0; c < D; ++c) yc[c] = j < N ? (static_cast<double>(yraw[c]) - mu[c]) * sk : 0.0;
        ring_col<D>(ys, yq, j & (kRing - 1), yc);
      }
      __syncthreads();
    }
    if (has_next) {   // the last chunk's columns
      mem_drain();
      if (lane == 0) st_dev(prog_out, N);
    }
    if (ib <= M - 1 && M - 1 < ib + RHO) {
      const int rl = M - 1 - ib;
      double v = left[0];
#pragma unroll
      for (int r = 1; r < RHO; ++r)
        if (r == rl) v = left[r];
      a.value[pd.out] = v / k;
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- backward

// Occupancy: the unbanded instance is held to three resident waves per SIMD
// (168 VGPRs; a few values of the tile setup spill), measured 5 % faster than
// two waves without spills; the band test needs more registers, so the
// banded instance is held to two.
template <typename TY, int D, int RHO, bool BAND>
__global__ __launch_bounds__(kWave, 2) void soft_bwd_kernel(SoftArgs a) {
  constexpr int H = kWave * RHO;
  __shared__ double ys[D][kRing + 16];     // -2 y' of the columns (see sq_cost)
  __shared__ double yq[kRing + 16];        // |y'|^2
  __shared__ double bin_fwd[kTile];        // lane 0's upper input for the replay
  __shared__ float bin_up[kTile];          // lane 63's pushes from the strip below
  __shared__ float bin_dg[kTile];
  // lane 0's pushes for the strip above in slots 0..15; slots 16 + lane + u
  // take the other lanes' writes
  __shared__ float bout_up[kTile + kWave + kTile];
  __shared__ float bout_dg[kTile + kWave + kTile];
  __shared__ int s_item;
  const int lane = threadIdx.x;
  const int bsl = lane == 0 ? 0 : kTile + lane;
  const TY* __restrict__ Y = static_cast<const TY*>(a.y);
  const double INF = inf_d();
  const double k = a.kscale;
  const double sk = __builtin_sqrt(k);   // x and y enter as sqrt(k) (x - mu), sqrt(k) (y - mu)
  if (skipped(a.skip)) return;   // every workgroup: no strip waits for another

  for (;;) {
    if (lane == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: scalar loads below
    __syncthreads();
    if (item >= a.n_items) break;
    const int2 it = a.items[item];
    const PairDesc pd = uniform(a.pairs[uni(it.x)]);
    double mu[D];
#pragma unroll
    for (int c = 0; c < D; ++c) mu[c] = a.x[pd.x_off * D + c];
    // first gradient row of this pair (per-cycle blocks of L rows, or the packed X rows)
    const int64_t grow = uni(a.rows_packed ? pd.x_off : (int64_t)pd.out * a.L);
    const int s = uni(it.y);
    const int M = pd.M, N = pd.N;
    const int i0 = s * H;
    const int ib = i0 + lane * RHO;
    const double band_b = BAND ? band_halfwidth(M, N, a.band) : 0.0;
    const bool has_above = s > 0;            // a strip above consumes our top-row pushes
    const bool has_below = s + 1 < pd.S;     // the strip below feeds our bottom row
    const int G = pd.WT;                     // 16-step tiles
    // Sakoe-Chiba band: a tile whose columns (tg - 63 .. tg + 15 over the
    // lanes) all lie outside the band of the strip's rows has e = 0 in every
    // cell (a cell outside the band gets nothing from its successors: their
    // weight towards a +inf cell is 0), so the sweep runs tiles g_lo .. g_hi
    // only.  The strip above never reads pushes right of our tiles (the
    // band's right edge moves right from row to row); the columns left of
    // them are published as zeros at the end.
    int g_lo = 0, g_hi = G - 1;
    if (BAND) {
      int jlo_b, jhi_b;
      band_strip_cols(M, N, a.band, i0, min(i0 + H, M) - 1, &jlo_b, &jhi_b);
      g_hi = min(G - 1, (jhi_b + kWave - 1) / 16);   // last tile with tg - 63 <= jhi_b
      g_lo = min(g_hi, jlo_b / 16);                  // first tile with tg + 15 >= jlo_b
    }
    const double* row_fwd = a.rows + pd.aux_base + (int64_t)(s - 1) * N;
    const double* st = a.states + pd.state_base + (int64_t)s * G * (RHO + 1) * kWave;
    const __amdgpu_buffer_rsrc_t rf_in = rsrc(row_fwd, has_above ? N * 8 : 0);
    // rolling push rows: the strip below wrote them for us, we overwrite them
    // for the strip above after reading
    float* pu_row = a.push_up + pd.bnd_base;
    float* pd_row = a.push_dg + pd.bnd_base;
    int* prog_below = a.progress + pd.flag_base + s + 1;
    int* prog_self = a.progress + pd.flag_base + s;
    // the cell that closes the path, (M-1, N-1), receives e = 1: it is
    // pending as a left push into that cell before the sweep starts (lane
    // k_last computes no cell of its rows to the right of column N-1)
    const bool last = s + 1 == pd.S;
    const int k_last = (M - 1 - i0) / RHO;
    const int r_last = (M - 1 - i0) - k_last * RHO;

    double xr[RHO][D], xx[RHO];
#pragma unroll
    for (int r = 0; r < RHO; ++r) {
#pragma unroll
      for (int c = 0; c < D; ++c)
        xr[r][c] = (ib + r < M) ? (a.x[(pd.x_off + ib + r) * D + c] - mu[c]) * sk : 0.0;
      xx[r] = sq_norm<D>(xr[r]);
    }

    // float64 row accumulators: sum_j e and sum_j e (-2 y'_j)
    double acc_e[RHO], acc_ey[RHO][D];
    float pl[RHO], pdg[RHO];                  // pending left / diagonal pushes into each row
#pragma unroll
    for (int r = 0; r < RHO; ++r) {
      acc_e[r] = 0.0;
      pl[r] = (last && lane == k_last && r == r_last) ? 1.0f : 0.0f;
      pdg[r] = 0.0f;
#pragma unroll
      for (int c = 0; c < D; ++c) acc_ey[r][c] = 0.0;
    }
    float up0 = 0.0f, dg0 = 0.0f;             // this lane's row-0 pushes, sent up next step
    float recv_dg = 0.0f;                     // diagonal push received last step
    bool gave_up = false;                     // wave-uniform
    int seen_below = 0;                       // last progress read from the strip below (uniform)
    const __amdgpu_buffer_rsrc_t pu_out = rsrc(pu_row, N * 4);
    const __amdgpu_buffer_rsrc_t pd_out = rsrc(pd_row, N * 4);
    const __amdgpu_buffer_rsrc_t pu_in = rsrc(pu_row, has_below ? N * 4 : 0);
    const __amdgpu_buffer_rsrc_t pd_in = rsrc(pd_row, has_below ? N * 4 : 0);
    // a tile's replay inputs: the forward's sweep state at its first step and
    // (lanes 0..15) the strip above's bottom row at its 16 columns (the top
    // strip reads an empty buffer and uses +inf; columns past N are never used)
    double st_n[RHO + 1];
    double rf_n;
    auto load_tile_inputs = [&](int gg) {
#pragma unroll
      for (int r = 0; r <= RHO; ++r) st_n[r] = st[((int64_t)gg * (RHO + 1) + r) * kWave + lane];
      const int j = 16 * gg + lane;
      rf_n = __builtin_bit_cast(
          double, __builtin_amdgcn_raw_buffer_load_b64(rf_in, lane < kTile && j < N ? j * 8 : kDrop, 0, 0));
    };
    // the Y columns of tile gg (63 + 16 of them, through the ring)
    auto fill_ring = [&](int gg) {
      const int jlo = 16 * gg - (kWave - 1);
      for (int q = lane; q < 16 + kWave - 1; q += kWave) {
        const int j = jlo + q;
        double yc[D];
#pragma unroll
        for (int c = 0; c < D; ++c)
          yc[c] = (j >= 0 && j < N) ? (static_cast<double>(Y[(pd.y_off + j) * D + c]) - mu[c]) * sk
                                    : 0.0;
        ring_col<D>(ys, yq, j & (kRing - 1), yc);
      }
    };
    // any push still travelling inside the strip (wave-uniform)
    auto pending = [&]() {
      bool p = up0 != 0.0f || dg0 != 0.0f || recv_dg != 0.0f;
#pragma unroll
      for (int r = 0; r < RHO; ++r) p = p || pl[r] != 0.0f || pdg[r] != 0.0f;
      return __builtin_amdgcn_ballot_w64(p) != 0;
    };
    // waits until the strip below has published every column >= jlo
    auto wait_below = [&](int jlo) {
      const int need = N - max(0, jlo);
      if (need > seen_below && !gave_up) {
        int got = 0, quit = 0;
        if (lane == 0) {
          int polls = 0;
          got = ld_dev(prog_below);
          while (got < need) {
            poll_backoff(polls, a.relaxed_wait);
            if (++polls > kSpinLimit) {
              atomicOr(a.status, kStatusSpinTimeout);
              quit = 1;
              break;
            }
            got = ld_dev(prog_below);
          }
        }
        seen_below = __builtin_amdgcn_readfirstlane(got);
        gave_up = __builtin_amdgcn_readfirstlane(quit) != 0;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    };

    load_tile_inputs(g_hi);
    fill_ring(g_hi);

    // Zero tiles.  e reaches a cell only through the pushes of its
    // successors, so a tile entered with no push travelling inside the strip
    // and no non-zero push from the strip below has e = 0 in every cell and
    // pushes nothing on.  With zero_skip such tiles are not swept; the strip
    // checks the pushes from below for up to 16 tiles at a time (as far as
    // the strip below has published) and moves on.  The result is the same
    // bit for bit: a swept zero tile only adds +0 to the row sums and pushes
    // 0 * w = 0.  Its top-row pushes are zero: they are stored unless the
    // shared push row is known to hold zero there already, which is the case
    // for every column this strip read as zero while skipping (the strip
    // below left a zero there; the bottom strip, which reads nothing, stores
    // them all).
    bool idle = a.zero_skip && !pending();
    int n_swept = 0;
    for (int g = g_hi; g >= g_lo; --g) {
      if (idle) {
        // columns at or below clean_hi read as zero from below in this run of skips
        const int clean_hi = has_below ? 16 * g - (kWave - 1) + 15 : -1;
        int hit = -1;   // first tile (from the right) fed a non-zero push from below
        for (;;) {
          int ge = max(g_lo, g - 15);   // this round: tiles g .. ge
          if (has_below) {
            wait_below(16 * g - (kWave - 1));   // tile g's inputs, at least
            if (!gave_up && seen_below < N - max(0, 16 * ge - (kWave - 1))) {
              int got = 0;   // one more read of the counter, without waiting
              if (lane == 0) got = ld_dev(prog_below);
              seen_below = max(seen_below, __builtin_amdgcn_readfirstlane(got));
            }
            // tile t takes columns >= 16 t - 63, all published once
            // 16 t - 63 >= N - seen_below (any t once every column is)
            if (!gave_up && seen_below < N) ge = max(ge, (N - seen_below + (kWave - 1) + 15) >> 4);
            // the pushes tiles g .. ge take in: columns 16 ge - 63 .. 16 g - 48
            const int jlo = 16 * ge - (kWave - 1);
            const int cnt = 16 * (g - ge + 1);
            float u[4], v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int q = lane + kWave * k;
              const int c = jlo + q;
              const int off = q < cnt && c >= 0 && c < N ? c * 4 : kDrop;
              u[k] = ld_dev_f32(pu_in, off);
              v[k] = ld_dev_f32(pd_in, off);
            }
#pragma unroll
            for (int k = 3; k >= 0; --k) {
              const unsigned long long m = __builtin_amdgcn_ballot_w64(u[k] != 0.0f || v[k] != 0.0f);
              if (hit < 0 && m != 0) hit = ge + ((kWave * k + 63 - __builtin_clzll(m)) >> 4);
            }
          }
          const int gz = hit >= 0 ? hit + 1 : ge;   // tiles g .. gz are zero
          if (has_above && gz <= g) {
            // their top-row pushes: columns 16 gz .. 16 g + 15, announced
            // once every older store is complete
            const int cnt = 16 * (g - gz + 1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int q = lane + kWave * k;
              const int c = 16 * gz + q;
              if (q < cnt && c < N && c > clean_hi) {
                st_dev(pu_out, c * 4, 0.0f);
                st_dev(pd_out, c * 4, 0.0f);
              }
            }
            mem_drain();
            if (lane == 0) st_dev(prog_self, N - min(N, 16 * gz));
          }
          g = gz - 1;
          if (hit >= 0 || g < g_lo) break;
        }
        if (g < g_lo) break;
        // sweep tile g: its replay inputs and Y columns were not kept up
        idle = false;
        load_tile_inputs(g);
        fill_ring(g);
      }
      ++n_swept;
      const int tg = 16 * g;
      const int yb = (tg - lane) & (kRing - 1);   // ring slot of step 0's column
      // next tile's 16 new Y columns, stored after this tile
      // (unconditional loads from a clamped column, kept in the storage type
      // until the store: a conditional load would be waited for on the spot)
      TY yraw[D];
      const int jn = tg - 16 - (kWave - 1) + lane;
      {
        const int jc = min(max(jn, 0), N - 1);
#pragma unroll
        for (int c = 0; c < D; ++c) yraw[c] = Y[(pd.y_off + jc) * D + c];
      }
      // lane 0's upper input for the replay (bottom row of the strip above),
      // loaded during the previous tile
      if (lane < kTile) bin_fwd[lane] = has_above ? rf_n : INF;
      // lane 63's inputs: pushes of the strip below's top row at columns
      // tg-63 ..  The strip below usually runs far ahead: one read of its
      // counter covers many tiles, and only a counter short of what this
      // tile needs is read again.
      if (has_below) wait_below(tg - (kWave - 1));
      // the pushes are only needed by the backward half: loaded now (one
      // unconditional load each, zero outside the row or without a strip
      // below) and written to LDS after the replay
      float in_up, in_dg;
      {
        const int j = tg - (kWave - 1) + lane;
        const int off = lane < kTile && j >= 0 && j < N ? j * 4 : kDrop;
        in_up = ld_dev_f32(pu_in, off);
        in_dg = ld_dev_f32(pd_in, off);
      }
      __syncthreads();

      // ---- replay the tile forward, keeping the soft-min weights
      double left[RHO];
#pragma unroll
      for (int r = 0; r < RHO; ++r) left[r] = st_n[r];
      double upprev = st_n[RHO];
      double bot = left[RHO - 1];
      // normalised soft-min weights of the up and left predecessors (the
      // diagonal takes the rest of the cell's e, so every cell passes on
      // exactly what it received)
      float wu[16][RHO], wl[16][RHO];
      const bool full = tg >= kWave - 1 && tg + 16 <= N;
      // The banded instances (two waves per SIMD, less latency hidden by
      // the other waves) read the LDS inputs of the lane shifts one step ahead.
      double bf_n = bin_fwd[0];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int t = tg + u;
        const int j = t - lane;
        double bf;
        if constexpr (BAND) {
          bf = bf_n;
          if (u + 1 < 16) bf_n = bin_fwd[u + 1];
        } else {
          bf = bin_fwd[u];
        }
        const double upin = shr1_f64(bot, bf);
        const double dgi = upprev;
        upprev = upin;
        if (full || (j >= 0 && j < N)) {
          double y[D];
#pragma unroll
          for (int c = 0; c < D; ++c) y[c] = ys[c][yb + u];
          const double yy = yq[yb + u];
          double dg = dgi, up = upin;
          const double bd0 = (double)ib * (double)(N - 1) - (double)j * (double)(M - 1);
#pragma unroll
          for (int r = 0; r < RHO; ++r) {
            const double lf = left[r];
            if constexpr (BAND) {
              // outside the band: cost +inf and weights (1, 0, 0), so the cell
              // receives and passes on exactly nothing
              const bool inb = __builtin_fabs(bd0 + (double)r * (double)(N - 1)) <= band_b;
              const SoftMin sm = softmin3_band(dg, up, lf, inb);
              const double rv = inb ? sq_cost<D>(xr[r], xx[r], y, yy) + sm.v : INF;
              const float rs = __builtin_amdgcn_rcpf(inb ? sm.s : 1.0f);
              wu[u][r] = inb ? sm.eu * rs : 0.0f;
              wl[u][r] = inb ? sm.el * rs : 0.0f;
              dg = lf;
              up = rv;
              left[r] = rv;
            } else {
              const SoftMin sm = softmin3(dg, up, lf);
              const double rv = sq_cost<D>(xr[r], xx[r], y, yy) + sm.v;
              const float rs = __builtin_amdgcn_rcpf(sm.s);   // s >= 1: the minimum's term is 1
              wu[u][r] = sm.eu * rs;
              wl[u][r] = sm.el * rs;
              dg = lf;
              up = rv;
              left[r] = rv;
            }
          }
          bot = left[RHO - 1];
        }
      }

      if (lane < kTile) {
        bin_up[lane] = in_up;
        bin_dg[lane] = in_dg;
      }
      // the next tile's replay inputs, in flight during the backward half
      // (unconditional: the last tile reloads its own)
      load_tile_inputs(max(g - 1, 0));
      __syncthreads();

      // ---- backward over the tile
      float bu_n = bin_up[15], bd_n = bin_dg[15];
#pragma unroll
      for (int u = 15; u >= 0; --u) {
        const int t = tg + u;
        const int j = t - lane;
        float bu, bd;
        if constexpr (BAND) {
          bu = bu_n;
          bd = bd_n;
          if (u > 0) {
            bu_n = bin_up[u - 1];
            bd_n = bin_dg[u - 1];
          }
        } else {
          bu = bin_up[u];
          bd = bin_dg[u];
        }
        // pushes of the lane below (rows i+1): its up push for column j now,
        // its diagonal push for column j-1 next step
        const float recv_up = shl1_f32(up0, bu);
        const float recv_dg_next = shl1_f32(dg0, bd);
        if (full || (j >= 0 && j < N)) {
          double y[D];
#pragma unroll
          for (int c = 0; c < D; ++c) y[c] = ys[c][yb + u];
          float below_up = recv_up;          // push up from (i+1, j)
          float new_pdg[RHO];
#pragma unroll
          for (int r = RHO - 1; r >= 0; --r) {
            const float din = (r == RHO - 1) ? recv_dg : pdg[r];
            const float e = (below_up + pl[r]) + din;
            // e in [0, 1] is carried in float32; the row sums take it in
            // float64.  Split e over the three predecessors: up and left by
            // their weights, the diagonal takes the rest, so the three pushes
            // add up to e up to one rounding of each subtraction (unbiased,
            // where weights that summed to 1 only to float32 rounding would
            // drain or add ~1e-8 of the mass at every cell, systematically)
            const float pu_ = e * wu[u][r];
            const float pl_ = e * wl[u][r];
            const float dpush = (e - pu_) - pl_;
            below_up = pu_;
            pl[r] = pl_;
            if (r > 0) new_pdg[r - 1] = dpush;
            else dg0 = dpush;
            const double e64 = e;
            acc_e[r] += e64;
#pragma unroll
            for (int c = 0; c < D; ++c) acc_ey[r][c] = __builtin_fma(e64, y[c], acc_ey[r][c]);
          }
          up0 = below_up;
#pragma unroll
          for (int r = 0; r + 1 < RHO; ++r) pdg[r] = new_pdg[r];
        }
        // lane 0's pushes into slot u (a column past N holds a stale value,
        // never published), the other lanes' into scratch slots: no branch
        bout_up[bsl + u] = up0;
        bout_dg[bsl + u] = dg0;
        recv_dg = recv_dg_next;
      }
      idle = a.zero_skip && !pending();
      __syncthreads();
      if (has_above) {
        // publish the top row's pushes for columns tg .. tg+15 (two stores,
        // issued by every lane, dropped past the row), then announce the
        // previous tile's columns: waiting until at most these two stores are
        // outstanding completes every older store without waiting for them
        const int j = tg + lane;
        const bool w = lane < kTile && j < N;
        st_dev(pu_out, w ? j * 4 : kDrop, bout_up[lane & (kTile - 1)]);
        st_dev(pd_out, w ? j * 4 : kDrop, bout_dg[lane & (kTile - 1)]);
        mem_wait_all_but_2();
        if (lane == 0) st_dev(prog_self, N - min(N, tg + 16));
      }
      if (g > 0 && lane < 16) {
        const bool in = jn >= 0 && jn < N;
        double yc[D];
#pragma unroll
        for (int c = 0; c < D; ++c) yc[c] = in ? (static_cast<double>(yraw[c]) - mu[c]) * sk : 0.0;
        ring_col<D>(ys, yq, jn & (kRing - 1), yc);
      }
      __syncthreads();
    }
    if (has_above) {   // the last tile's columns
      if (BAND && g_lo > 0) {
        // columns 0 .. 16 g_lo - 1 of the top row push nothing: zeros, written
        // once the strip below has finished with the shared row (it writes
        // its own pushes for us there)
        if (has_below && !gave_up) {
          int got = 0, quit = 0;
          if (lane == 0) {
            int polls = 0;
            got = ld_dev(prog_below);
            while (got < N) {
              poll_backoff(polls, a.relaxed_wait);
              if (++polls > kSpinLimit) {
                atomicOr(a.status, kStatusSpinTimeout);
                quit = 1;
                break;
              }
              got = ld_dev(prog_below);
            }
          }
          gave_up = __builtin_amdgcn_readfirstlane(quit) != 0;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        for (int j = lane; j < 16 * g_lo; j += kWave) {
          st_dev(pu_out, j * 4, 0.0f);
          st_dev(pd_out, j * 4, 0.0f);
        }
      }
      mem_drain();
      if (lane == 0) st_dev(prog_self, N);
    }
    if (a.tiles != nullptr && lane == 0) {
      atomicAdd(a.tiles, (unsigned long long)n_swept);
      atomicAdd(a.tiles + 1, (unsigned long long)(g_hi - g_lo + 1));
    }
    // per-row sums of this cycle: gradient 2 (b sum_j e - sum_j e y_j), which
    // is (2 x' sum_j e + sum_j e (-2 y'_j)) / sk, and mass
#pragma unroll
    for (int r = 0; r < RHO; ++r) {
      const int i = ib + r;
      if (i < M) {
        const int64_t o = grow + i;
#pragma unroll
        for (int c = 0; c < D; ++c)
          a.gsum[o * D + c] = (2.0 * xr[r][c] * acc_e[r] + acc_ey[r][c]) / sk;
        a.hsum[o] = acc_e[r];
      }
    }
    __syncthreads();
  }
}

// G_l = sum_k w_k * grad_k(l), h_l = sum_k w_k * mass_k(l), ascending k,
// starting from 0 or (accumulate) from the values already in grad / mass.
// Calls over consecutive cycle groups with accumulate = 1 after the first
// therefore perform the very additions of one call over all cycles.
__global__ void soft_reduce_kernel(const double* __restrict__ gsum, const double* __restrict__ hsum,
                                   const double* __restrict__ w, int n, int64_t L, int d,
                                   double* __restrict__ grad, double* __restrict__ mass,
                                   int accumulate) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= L * d) return;
  const int64_t l = idx / d;
  const int c = (int)(idx - l * d);
  double g = accumulate ? grad[idx] : 0.0;
  for (int p = 0; p < n; ++p) g = g + (w ? w[p] : 1.0) * gsum[((int64_t)p * L + l) * d + c];
  grad[idx] = g;
  if (c == 0 && mass) {
    double h = accumulate ? mass[l] : 0.0;
    for (int p = 0; p < n; ++p) h = h + (w ? w[p] : 1.0) * hsum[(int64_t)p * L + l];
    mass[l] = h;
  }
}

// Rows of a packed [sum N][d] gradient scaled by their cycle's weight:
// out[row] = w[k] * g[row] for the cycle k holding the row (offsets off[n+1]).
__global__ void soft_rows_scale_kernel(const double* __restrict__ g, const int64_t* __restrict__ off,
                                       int n, int d, const double* __restrict__ w,
                                       double* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t rows = off[n];
  if (idx >= rows * d) return;
  const int64_t row = idx / d;
  int lo = 0, hi = n - 1;   // the cycle k with off[k] <= row < off[k + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= row) lo = mid;
    else hi = mid - 1;
  }
  out[idx] = w ? w[lo] * g[idx] : g[idx];
}

// One preconditioned gradient step on the barycenter:
//   b_l <- b_l - eta * G_l / (2 h_l)
// With eta = 1 this is the soft-DBA update b_l = sum_j e y_j / sum_j e.
__global__ void precond_step_kernel(double* __restrict__ bary, const double* __restrict__ grad,
                                    const double* __restrict__ mass, int64_t L, int d,
                                    double eta) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= L * d) return;
  const int64_t l = idx / d;
  bary[idx] = bary[idx] - eta * grad[idx] / (2.0 * mass[l]);
}

}  // namespace

hipError_t launch_precond_step(double* bary, const double* grad, const double* mass, int64_t L,
                               int d, double eta, hipStream_t st) {
  const int64_t tot = L * d;
  hipLaunchKernelGGL(precond_step_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     bary, grad, mass, L, d, eta);
  return hipGetLastError();
}

#define WTS_SOFT_D_SWITCH(d, CALL) \
  switch (d) {                     \
    case 1: return CALL(1);        \
    case 2: return CALL(2);        \
    case 3: return CALL(3);        \
    case 4: return CALL(4);        \
    case 5: return CALL(5);        \
    case 6: return CALL(6);        \
    case 7: return CALL(7);        \
    case 8: return CALL(8);        \
    default: return hipErrorInvalidValue; \
  }

template <typename TY, int D>
static hipError_t launch_soft_t(bool bwd, const SoftArgs& a, int grid, hipStream_t st) {
  const bool band = a.band > 0.0;
  if (bwd) {
    if (band)
      hipLaunchKernelGGL((soft_bwd_kernel<TY, D, kSoftRho, true>), dim3(grid), dim3(kWave), 0, st, a);
    else
      hipLaunchKernelGGL((soft_bwd_kernel<TY, D, kSoftRho, false>), dim3(grid), dim3(kWave), 0, st, a);
  } else {
    if (band)
      hipLaunchKernelGGL((soft_fwd_kernel<TY, D, kSoftRho, true>), dim3(grid), dim3(kWave), 0, st, a);
    else
      hipLaunchKernelGGL((soft_fwd_kernel<TY, D, kSoftRho, false>), dim3(grid), dim3(kWave), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_soft(int d, int ydtype, bool bwd, const SoftArgs& a, int grid, hipStream_t st) {
#define CALLS(D) (ydtype == 0 ? launch_soft_t<float, D>(bwd, a, grid, st) \
                              : launch_soft_t<double, D>(bwd, a, grid, st))
  WTS_SOFT_D_SWITCH(d, CALLS)
#undef CALLS
}

hipError_t launch_soft_rows_scale(const double* g, const int64_t* off, int n, int64_t rows, int d,
                                  const double* w, double* out, hipStream_t st) {
  const int64_t tot = rows * d;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(soft_rows_scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     g, off, n, d, w, out);
  return hipGetLastError();
}

hipError_t launch_soft_reduce(const double* gsum, const double* hsum, const double* w, int n,
                              int64_t L, int d, double* grad, double* mass, int accumulate,
                              hipStream_t st) {
  const int64_t tot = L * d;
  hipLaunchKernelGGL(soft_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     gsum, hsum, w, n, L, d, grad, mass, accumulate);
  return hipGetLastError();
}

}  // namespace wts
