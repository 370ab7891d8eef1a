// wts_dtw.hip -- path recovery, DBA update, scores, medoid and barycenter
// initialisation for gfx950, and the float64 instances of the DTW sweep
// (wts_sweep.h).
#include "wts_sweep.h"

namespace wts {

namespace {

// Strip-level path recovery after a PATHT sweep.  That sweep tagged every
// cell with the top-row cell through which its optimal path enters the strip (code 2j for
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

// Path recovery, one pair per workgroup.  From (M-1, N-1) the walk follows
// the argmin codes strip by strip, the bottom strip first: in each strip
// from the column where the path crosses the strip's bottom row up to the
// cell of its top row whose code leaves the strip (an up or diagonal move
// out of row i0), which gives the column where the path crosses the bottom
// row of the strip above.  Per strip it records the segment (bottom-row
// column, top-row column) and its length, for the path list, and per row
// the run of columns [lo, hi] the path occupies (for the DBA sums, which
// run_sum_kernel forms in parallel).  All 64 lanes walk in lockstep
// (identical state): the code-word staging is cooperative, and the words
// read back from LDS are moved to scalar registers, so the walk itself runs
// on the scalar unit.  A walk that leaves its strip marks the status word,
// and every strip from there up gets empty runs.
template <int RHO>
__global__ __launch_bounds__(kWave) void path_walk_kernel(WalkArgs a) {
  constexpr int H = kWave * RHO;
  __shared__ uint32_t blk[kWalkWords][RHO][kWave];
  const int lane = threadIdx.x;
  if (skipped(a.skip)) return;
  const PairDesc pd = a.pairs[blockIdx.x];
  int2* runs = a.runs ? a.runs + (int64_t)pd.out * a.L : nullptr;   // null: no DBA sums wanted
  bool bad = false;
  int jx = pd.N - 1;   // where the path crosses the current strip's bottom row
  for (int s = pd.S - 1; s >= 0; --s) {
    const int item = pd.item_base + s;
    const int i0 = s * H;
    const int iend = min(pd.M, i0 + H) - 1;
    const uint32_t* codes = a.codes + pd.code_base + (int64_t)s * pd.WT * RHO * kWave;
    if (jx < 0 || jx >= pd.N) bad = true;
    int i = iend, j = jx, hi = jx, jtop = -1, jnext = -1, cnt = 0;
    int k = (iend - i0) / RHO, r = (iend - i0) - k * RHO;   // lane and row of row i
    int wlo = 1 << 30, whi = -1;
    uint32_t cw[RHO];
    int ck = -1, cwk = -1;
    while (!bad) {
      if (j < 0) {   // walked out of the strip: inconsistent codes
        bad = true;
        break;
      }
      ++cnt;
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
        // the same words in every lane: scalar registers, so the walk's
        // arithmetic and branches below stay on the scalar unit
#pragma unroll
        for (int rr = 0; rr < RHO; ++rr) cw[rr] = __builtin_amdgcn_readfirstlane(blk[w - wlo][rr][k]);
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
        if (u > 0) {
          // the cells (i, j), (i, j-1), ... of this word that are left moves
          // too: their fields (steps u-1, u-2, ...) sit above this one
          const uint32_t rest = word >> (32 - 2 * u);
          const int more = rest == 0u ? u : (int)(__builtin_ctz(rest) >> 1);
          j -= more;
          cnt += more;
        }
      } else {
        if (runs && lane == 0) runs[i] = make_int2(j, hi);
        if (i == i0) {   // the move out of the strip
          jtop = j;
          jnext = j - ((code & 2u) ? 1 : 0);
          break;
        }
        --i;
        if (--r < 0) {
          r = RHO - 1;
          --k;
        }
        if (code & 2u) --j;   // diagonal
        hi = j;
      }
    }
    if (bad) {
      if (lane == 0) atomicOr(a.status, kStatusBadPath);
      if (runs)
        for (int q = i0 + lane; q <= iend; q += kWave) runs[q] = make_int2(0, -1);
    }
    if (lane == 0) {
      a.seg_out[item] = bad ? make_int2(-1, -1) : make_int2(jx, jtop);
      a.seg_len[item] = bad ? 0 : cnt;
    }
    if (s > 0 && !bad && jnext < 0) bad = true;   // the path left row 0 before strip 0
    jx = jnext;
  }
}

// Per (cycle, barycenter row): the sum of the cycle's samples over the run
// [lo, hi] of the row's path, in descending column order, and its length.
template <typename TY, int D>
__global__ void run_sum_kernel(const int2* __restrict__ runs, const int64_t* __restrict__ off,
                               const void* y, int n, int64_t L, double* __restrict__ psum,
                               int* __restrict__ pcnt, const int* skip) {
  if (skipped(skip)) return;
  const TY* __restrict__ Y = static_cast<const TY*>(y);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < (int64_t)n * L; o += stride) {
    const int2 rn = runs[o];
    const int64_t base = off[o / L];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double acc = 0.0;
      for (int jj = rn.y; jj >= rn.x; --jj) acc = acc + static_cast<double>(Y[(base + jj) * D + c]);
      psum[o * D + c] = acc;
    }
    pcnt[o] = rn.y - rn.x + 1;
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

hipError_t launch_fwd(int d, int rho, int mode, bool euc, bool x_is_cycle, int ydtype, bool fp32,
                      const FwdArgs& a, int grid, hipStream_t st) {
  if (fp32) return launch_fwd32(d, rho, mode, euc, x_is_cycle, ydtype, a, grid, st);
  return launch_fwd_impl<double>(d, rho, mode, euc, x_is_cycle, ydtype, a, grid, st);
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

hipError_t launch_path_walk(int rho, const WalkArgs& a, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (rho == 4) hipLaunchKernelGGL(path_walk_kernel<4>, dim3(n_pairs), dim3(kWave), 0, st, a);
  else if (rho == 2) hipLaunchKernelGGL(path_walk_kernel<2>, dim3(n_pairs), dim3(kWave), 0, st, a);
  else if (rho == 5) hipLaunchKernelGGL(path_walk_kernel<5>, dim3(n_pairs), dim3(kWave), 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename TY, int D>
static hipError_t launch_run_sum_t(const int2* runs, const int64_t* off, const void* y, int n,
                                   int64_t L, double* psum, int* pcnt, const int* skip,
                                   hipStream_t st) {
  const int64_t rows = (int64_t)n * L;
  const unsigned blocks = (unsigned)std::min<int64_t>((rows + 255) / 256, 65536);
  hipLaunchKernelGGL((run_sum_kernel<TY, D>), dim3(blocks), dim3(256), 0, st, runs, off, y, n, L,
                     psum, pcnt, skip);
  return hipGetLastError();
}

hipError_t launch_run_sum(int d, int ydtype, const int2* runs, const int64_t* off, const void* y,
                          int n, int64_t L, double* psum, int* pcnt, const int* skip,
                          hipStream_t st) {
  if ((int64_t)n * L <= 0) return hipSuccess;
#define CALLS(D, R) (ydtype == 0 ? launch_run_sum_t<float, D>(runs, off, y, n, L, psum, pcnt, skip, st) \
                                 : launch_run_sum_t<double, D>(runs, off, y, n, L, psum, pcnt, skip, st))
  WTS_D_SWITCH(d, 0, CALLS)
#undef CALLS
  return hipErrorInvalidValue;
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
