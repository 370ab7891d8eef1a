// wts_abi.hip -- the C ABI of include/wetsand_mi.h: plans, argument checks,
// workspace layout and the launch sequences of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/wetsand_mi.h"
#include "wts_kernels.h"
#include "wts_order.h"

using wts::PairDesc;

namespace {

thread_local std::string g_err;

wts_status fail(wts_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wts_status fail(wts_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(WTS_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));              \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Pairs of one kind (barycenter vs cycles, or cycle vs cycle) with their
// sweep items and the sizes of the buffers the sweep needs.
struct PairSet {
  std::vector<PairDesc> pairs;
  std::vector<int2> items;         // pair-major, strips ascending (walk, chain, segments)
  std::vector<int2> sweep_items;   // pop order of the forward sweeps
  std::vector<int2> items_rev;     // pop order of the Soft-DTW backward (strips descending)
  PairDesc* d_pairs = nullptr;
  int2* d_items = nullptr;
  int2* d_sweep_items = nullptr;
  int2* d_items_rev = nullptr;
  int n_pairs = 0, n_items = 0, n_flags = 0;
  int64_t code_words = 0, bnd_elems = 0, aux_strip_elems = 0, state_elems = 0, row_elems = 0;
  int64_t max_rows = 0;
  int rho = 4;   // barycenter rows per lane of this set's sweeps
  bool walk_pairs = false;   // path recovery one pair at a time (PATH sweep, no entry tags)
};

struct Job {
  int64_t x_off, y_off;
  int32_t M, N, out;
};

void build_set(PairSet& ps, std::vector<Job> jobs, int rho) {
  const int H = wts::kWave * rho;
  ps.rho = rho;
  std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) {
    return (int64_t)a.M * a.N > (int64_t)b.M * b.N;
  });
  ps.pairs.clear();
  ps.items.clear();
  int64_t code = 0, bnd = 0, aux = 0, state = 0, rows = 0;
  int flags = 0;
  for (size_t p = 0; p < jobs.size(); ++p) {
    const Job& jb = jobs[p];
    PairDesc d{};
    d.x_off = jb.x_off;
    d.y_off = jb.y_off;
    d.M = jb.M;
    d.N = jb.N;
    d.S = (jb.M + H - 1) / H;
    d.out = jb.out;
    d.WT = (jb.N + wts::kWave - 1 + 15) / 16;
    d.code_base = code;
    d.bnd_base = bnd;
    d.aux_base = aux;
    d.state_base = state;
    d.row_base = rows;
    d.flag_base = flags;
    d.item_base = (int)ps.items.size();
    code += (int64_t)d.S * d.WT * rho * wts::kWave;
    bnd += jb.N;
    aux += (int64_t)d.S * jb.N;
    state += (int64_t)d.S * d.WT * (rho + 1) * wts::kWave;
    flags += d.S;
    rows += (int64_t)d.S * ((jb.N + wts::kWave - 1 + 3) & ~3);   // strip row stride RS
    for (int s = 0; s < d.S; ++s) ps.items.push_back(make_int2((int)p, s));
    ps.pairs.push_back(d);
    ps.max_rows = std::max<int64_t>(ps.max_rows, jb.M);
  }
  std::vector<int64_t> cols(ps.pairs.size());
  std::vector<int> strips(ps.pairs.size());
  for (size_t q = 0; q < ps.pairs.size(); ++q) {
    cols[q] = (int64_t)ps.pairs[q].N + wts::kWave;
    strips[q] = ps.pairs[q].S;
  }
  ps.sweep_items.clear();
  ps.items_rev.clear();
  wts::pop_order(cols, strips, false, [&](int q, int s) { ps.sweep_items.push_back(make_int2(q, s)); });
  wts::pop_order(cols, strips, true, [&](int q, int s) { ps.items_rev.push_back(make_int2(q, s)); });
  ps.n_pairs = (int)ps.pairs.size();
  ps.n_items = (int)ps.items.size();
  ps.n_flags = flags;
  ps.code_words = code;
  ps.bnd_elems = bnd;
  ps.aux_strip_elems = aux;
  ps.state_elems = state;
  ps.row_elems = rows;
}

// Workspace: every region 256-byte aligned, in this order.
struct Layout {
  size_t queue = 0, progress = 0, bnd_r = 0, bnd_aux = 0, codes = 0, out_dist = 0, out_aux = 0;
  size_t seg = 0, seg_len = 0, seg_off = 0, runs = 0, psum = 0, pcnt = 0, dm = 0, totals = 0;
  size_t rows = 0, states = 0, push_up = 0, push_dg = 0, gsum = 0, hsum = 0, out_end = 0;
  size_t total = 0;
};

// Scratch of wts_anomaly_score_noalloc: the score sweep's workspace for
// callers that cannot allocate.  `scratch` (below) is a static device array;
// each GPU the library runs on holds its own copy, at its own address, until
// the process ends.  Host code never uses the array's name as an address:
// wts_plan_create resolves the device address once per GPU (with that GPU
// current) into g_scratch.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Rows per lane of the barycenter sweeps when the caller leaves it open.
// With about one strip per SIMD, a strip that shares its SIMD slows its whole
// chain, and the dispatcher does not spread workgroups perfectly once they
// cover nearly every compute unit: such batches take 5 rows per lane when
// that brings them under ~80 % of the SIMDs.  Small batches (one strip per
// SIMD or less) and large ones (several per SIMD) keep 4.
int bary_rho(int64_t L, int n, int cus) {
  auto items = [&](int r) { return (int64_t)n * ((L + 64 * r - 1) / (64 * r)); };
  const int64_t simds = 4 * (int64_t)cus;
  const int64_t cap = simds * 13 / 16;
  const int64_t i4 = items(4);
  if (i4 > cap && i4 <= 2 * simds && items(5) <= cap) return 5;
  return 4;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Resolves this GPU's address of `scratch` (the device must be current).
wts_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return WTS_OK;   // the no-alloc call refuses it
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device] != nullptr) return WTS_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(WTS_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_scratch[device] = ptr;
  return WTS_OK;
}

}  // namespace

struct wts_plan {
  int device = 0, n = 0, d = 0, dtype = 0, cus = 256;
  int64_t L = 0;
  wts_opts opts{};
  int rho = 4;
  std::vector<int64_t> off;
  int64_t* d_off = nullptr;
  int64_t* d_path_base = nullptr;
  int2* d_med_ab = nullptr;
  PairSet bary, med, soft;
  PairSet softT;   // Soft-DTW with the roles swapped: the cycles on the rows, B on the columns
  int64_t nmax = 0;
  // device words: [0] sticky status bits (wts_plan_status reads and clears
  // them), [1] the current call's validation flag, [2] read-out slot
  int* d_status = nullptr;
  unsigned long long* d_tiles = nullptr;   // Soft-DTW backward: tiles swept, tiles in range
  // optional sweep timing: pool of (start, stop) event pairs, one per sweep launch
  std::vector<hipEvent_t> ev;
  size_t ev_next = 0;
  std::vector<int> ev_op;     // op tag of each used pair (-1 = unused)
};

namespace {

Layout layout(const wts_plan* p, int op) {
  Layout l;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1)); return at; };
  const PairSet& ps = op == WTS_OP_MEDOID ? p->med
                      : (op == WTS_OP_SOFT_FWD || op == WTS_OP_SOFT_BWD) ? p->soft
                      : op == WTS_OP_SOFT_GRAD_C ? p->softT : p->bary;
  if (op == WTS_OP_SOFT_GRAD_C) {   // the transposed forward and backward in one buffer
    const int64_t rows = p->off[p->n];
    l.queue = take(2 * sizeof(int));
    l.progress = take(sizeof(int) * (size_t)ps.n_flags);
    l.rows = take(sizeof(double) * (size_t)ps.aux_strip_elems);
    l.states = take(sizeof(double) * (size_t)ps.state_elems);
    l.push_up = take(sizeof(float) * (size_t)ps.bnd_elems);
    l.push_dg = take(sizeof(float) * (size_t)ps.bnd_elems);
    l.gsum = take(sizeof(double) * (size_t)rows * (size_t)p->d);
    l.hsum = take(sizeof(double) * (size_t)rows);
    l.out_dist = take(sizeof(double) * (size_t)p->n);
    l.total = o;
    return l;
  }
  if (op == WTS_OP_SOFT_FWD || op == WTS_OP_SOFT_BWD) {
    l.queue = take(2 * sizeof(int));
    l.progress = take(sizeof(int) * (size_t)ps.n_flags);
    if (op == WTS_OP_SOFT_FWD) {
      l.rows = take(sizeof(double) * (size_t)ps.aux_strip_elems);
      l.states = take(sizeof(double) * (size_t)ps.state_elems);
    } else {
      l.push_up = take(sizeof(float) * (size_t)ps.bnd_elems);
      l.push_dg = take(sizeof(float) * (size_t)ps.bnd_elems);
      l.gsum = take(sizeof(double) * (size_t)p->n * (size_t)p->L * (size_t)p->d);
      l.hsum = take(sizeof(double) * (size_t)p->n * (size_t)p->L);
    }
    l.total = o;
    return l;
  }
  const bool paths = op == WTS_OP_ALIGN_PATHS || op == WTS_OP_DBA;
  l.queue = take(2 * sizeof(int));   // [0] item counter, [1] status word
  l.bnd_r = take(sizeof(double) * (size_t)ps.row_elems);
  l.bnd_aux = take(sizeof(int) * (size_t)(op == WTS_OP_MEDOID ? 0 : ps.row_elems));
  if (paths) l.codes = take(sizeof(uint32_t) * (size_t)ps.code_words);
  l.out_dist = take(sizeof(double) * (size_t)ps.n_pairs);
  l.out_aux = take(sizeof(int) * (size_t)ps.n_pairs);
  if (op == WTS_OP_SUBDTW) l.out_end = take(sizeof(int) * (size_t)ps.n_pairs);
  if (paths) {
    l.seg = take(sizeof(int2) * (size_t)ps.n_items);
    l.seg_len = take(sizeof(int) * (size_t)ps.n_items);
    l.seg_off = take(sizeof(int) * (size_t)ps.n_items);
  }
  if (op == WTS_OP_DBA) {
    if (ps.walk_pairs) l.runs = take(sizeof(int2) * (size_t)p->n * (size_t)p->L);
    l.psum = take(sizeof(double) * (size_t)p->n * (size_t)p->L * (size_t)p->d);
    l.pcnt = take(sizeof(int) * (size_t)p->n * (size_t)p->L);
  }
  if (op == WTS_OP_MEDOID) {
    l.dm = take(sizeof(double) * (size_t)p->n * (size_t)p->n);
    l.totals = take(sizeof(double) * (size_t)p->n);
  }
  l.total = o;
  return l;
}

template <typename T>
T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

// Path recovery.  Tagging every cell with its strip entry (PATHT) costs the
// sweep about a tenth of its time (two selects of about 22 operations per
// cell) and lets all strips be walked at once; without the tags (PATH) each
// pair walks its strips in turn, about 85 us per strip on gfx950.  The pair
// walk pays when the tags' tenth, about 1e-13 s per cell on 256 CUs, exceeds
// the longest pair's walk.
bool walk_pairs_pays(const PairSet& ps) {
  double cells = 0.0;
  int smax = 0;
  for (const PairDesc& d : ps.pairs) {
    cells += (double)d.M * (double)d.N;
    smax = std::max(smax, d.S);
  }
  return cells * 1e-13 > smax * 85e-6;
}

int default_grid(const wts_plan* p, const PairSet& ps) {
  // 24 one-wave workgroups per CU: enough resident waves for the value sweep
  // (6 per SIMD); the path sweep's register budget caps it lower by itself.
  const int g = p->opts.grid > 0 ? p->opts.grid : p->cus * 24;
  return std::max(1, std::min(g, ps.n_items));
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

wts_status check_ws(const wts_plan* p, int op, void* ws, size_t ws_bytes) {
  const size_t need = layout(p, op).total;
  if (ws == nullptr) return fail(WTS_E_ARG, "workspace pointer is null");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
    return fail(WTS_E_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(WTS_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  return WTS_OK;
}

wts_status check_bary_plan(const wts_plan* p) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  if (p->L <= 0) return fail(WTS_E_ARG, "plan was created with L = 0 (medoid/init only)");
  return WTS_OK;
}

const int* skip_of(const wts_plan* p) { return p->opts.validate ? p->d_status + 1 : nullptr; }

// opts.validate: clear the call's flag, then scan its inputs; a value that is
// not finite sets the flag (every sweep and path-recovery kernel of the call
// then returns at once) and the sticky WTS_E_NONFINITE bit.
wts_status validate_inputs(const wts_plan* p, hipStream_t st, wts::ScanSeg a, wts::ScanSeg b = {},
                           wts::ScanSeg c = {}) {
  if (!p->opts.validate) return WTS_OK;
  const wts::ScanSeg segs[3] = {a, b, c};
  HIP_TRY(wts::launch_zero(p->d_status + 1, 1, st));
  HIP_TRY(wts::launch_finite_scan(segs, 3, p->d_status + 1, p->d_status, st));
  return WTS_OK;
}
wts::ScanSeg seg_f64(const void* ptr, int64_t n) { return wts::ScanSeg{ptr, n, 0}; }
wts::ScanSeg seg_cycles(const wts_plan* p, const void* ptr) {
  return wts::ScanSeg{ptr, p->off[p->n] * p->d, p->dtype == WTS_F32 ? 1 : 0};
}

// Sweep timing (off unless wts_plan_timing enabled it): records a pair of
// events around the sweep kernel of operation `op` on its stream.
int timing_begin(const wts_plan* p, int op, hipStream_t st) {
  wts_plan* q = const_cast<wts_plan*>(p);
  if (q->ev.empty()) return -1;
  const size_t pairs = q->ev.size() / 2;
  const size_t k = q->ev_next % pairs;
  q->ev_next++;
  q->ev_op[k] = op;
  (void)hipEventRecord(q->ev[2 * k], st);
  return (int)k;
}
void timing_end(const wts_plan* p, int k, hipStream_t st) {
  if (k >= 0) (void)hipEventRecord(p->ev[2 * k + 1], st);
}

// Zero the queue, fill the strip rows with sentinels, then run the
// persistent sweep.
wts_status run_sweep(const wts_plan* p, const PairSet& ps, int mode, bool euc, bool x_is_cycle,
                     const void* x, const void* y, void* ws, const Layout& l, double* out_dist,
                     hipStream_t st) {
  HIP_TRY(wts::launch_zero(at<int>(ws, l.queue), 2, st));
  HIP_TRY(wts::launch_fill_sentinels(at<double>(ws, l.bnd_r), ps.row_elems, at<int>(ws, l.bnd_aux),
                                     mode == wts::MODE_DIST_LEN || mode == wts::MODE_SUB ||
                                             mode == wts::MODE_PATHT
                                         ? ps.row_elems : 0, st));
  wts::FwdArgs a{};
  a.pairs = ps.d_pairs;
  a.items = ps.d_sweep_items;
  a.n_items = ps.n_items;
  a.queue = at<int>(ws, l.queue);
  a.status = p->d_status;
  a.skip = skip_of(p);
  a.x = x;
  a.y = y;
  a.bnd_r = at<double>(ws, l.bnd_r);
  a.bnd_aux = at<int>(ws, l.bnd_aux);
  a.codes = mode == wts::MODE_PATH || mode == wts::MODE_PATHT ? at<uint32_t>(ws, l.codes) : nullptr;
  a.out_dist = out_dist ? out_dist : at<double>(ws, l.out_dist);
  a.out_aux = at<int>(ws, l.out_aux);
  a.out_end = mode == wts::MODE_SUB ? at<int>(ws, l.out_end) : nullptr;
  a.cost_kind = euc ? 1 : 0;
  a.relaxed_wait = ps.n_items > 16 * p->cus ? 1 : 0;   // > 4 items per SIMD
  const int tk = timing_begin(p, x_is_cycle ? WTS_OP_MEDOID
                                 : mode == wts::MODE_PATH || mode == wts::MODE_PATHT ? WTS_OP_DBA
                                 : mode == wts::MODE_SUB ? WTS_OP_SUBDTW : WTS_OP_SCORE, st);
  HIP_TRY(wts::launch_fwd(p->d, ps.rho, mode, euc, x_is_cycle, p->dtype,
                          p->opts.decision == WTS_DECISION_FP32, a, default_grid(p, ps), st));
  timing_end(p, tk, st);
  return WTS_OK;
}

// The path sweep, then path recovery: segments, segment lengths and, with
// psum, the DBA partial sums.  Pair walks: a PATH sweep, one walk per pair
// (row runs), the row sums in parallel.  Strip walks: a PATHT sweep, the
// strip chain from the entry tags, one walk per strip (row runs and sums).
wts_status run_paths(const wts_plan* p, const double* bary, const void* cycles, void* ws,
                     const Layout& l, double* out_dist, double* psum, int* pcnt, hipStream_t st) {
  const PairSet& ps = p->bary;
  const int mode = ps.walk_pairs ? wts::MODE_PATH : wts::MODE_PATHT;
  wts_status rc = run_sweep(p, ps, mode, false, false, bary, cycles, ws, l, out_dist, st);
  if (rc != WTS_OK) return rc;
  wts::WalkArgs w{};
  w.pairs = ps.d_pairs;
  w.items = ps.d_items;
  w.codes = at<uint32_t>(ws, l.codes);
  w.y = cycles;
  w.L = p->L;
  w.seg_len = at<int>(ws, l.seg_len);
  w.status = p->d_status;
  w.skip = skip_of(p);
  if (ps.walk_pairs) {
    w.seg_out = at<int2>(ws, l.seg);
    w.runs = psum ? at<int2>(ws, l.runs) : nullptr;
    HIP_TRY(wts::launch_path_walk(ps.rho, w, ps.n_pairs, st));
    if (psum)
      HIP_TRY(wts::launch_run_sum(p->d, p->dtype, w.runs, p->d_off, cycles, p->n, p->L, psum,
                                  pcnt, skip_of(p), st));
    return WTS_OK;
  }
  HIP_TRY(wts::launch_chain(ps.d_pairs, ps.n_pairs, at<int>(ws, l.bnd_aux),
                            at<int>(ws, l.out_aux), at<int2>(ws, l.seg), p->d_status,
                            skip_of(p), st));
  w.seg = at<int2>(ws, l.seg);
  w.psum = psum;
  w.pcnt = pcnt;
  HIP_TRY(wts::launch_walk(p->d, ps.rho, p->dtype, false, w, ps.n_items, st));
  return WTS_OK;
}

}  // namespace

extern "C" {

const char* wts_last_error(void) { return g_err.c_str(); }

wts_status wts_plan_create(wts_plan** out, int device, int32_t n, int32_t d, int32_t dtype,
                           const int64_t* offsets_host, int64_t L, const wts_opts* opts) {
  if (!out) return fail(WTS_E_ARG, "out is null");
  *out = nullptr;
  if (!offsets_host) return fail(WTS_E_ARG, "offsets_host is null");
  if (n < 1) return fail(WTS_E_SHAPE, "n = %d: need at least one cycle", n);
  if (d < 1 || d > 8) return fail(d < 1 ? WTS_E_SHAPE : WTS_E_UNSUPPORTED, "d = %d: 1..8 supported", d);
  if (dtype != WTS_F32 && dtype != WTS_F64) return fail(WTS_E_DTYPE, "dtype %d", dtype);
  if (L < 0) return fail(WTS_E_SHAPE, "L = %lld out of range", (long long)L);
  if (offsets_host[0] != 0) return fail(WTS_E_SHAPE, "offsets_host[0] must be 0");
  if (L > (1 << 24)) return fail(WTS_E_CAPACITY, "L = %lld: at most 2^24 rows", (long long)L);
  for (int k = 0; k < n; ++k) {
    const int64_t len = offsets_host[k + 1] - offsets_host[k];
    if (len < 1) return fail(WTS_E_SHAPE, "cycle %d has length %lld", k, (long long)len);
    if (len > (1 << 24))
      return fail(WTS_E_CAPACITY, "cycle %d has %lld samples: at most 2^24", k, (long long)len);
  }
  wts_opts o{};
  if (opts) o = *opts;
  if (o.cost != WTS_COST_SQEUCLID && o.cost != WTS_COST_EUCLID) return fail(WTS_E_ARG, "opts.cost");
  if (o.rho != 0 && o.rho != 2 && o.rho != 4 && o.rho != 5)
    return fail(WTS_E_UNSUPPORTED, "opts.rho = %d: 2, 4 or 5 supported", o.rho);
  if (o.grid < 0) return fail(WTS_E_ARG, "opts.grid = %d", o.grid);
  if (o.validate != 0 && o.validate != 1) return fail(WTS_E_ARG, "opts.validate = %d: 0 or 1", o.validate);
  if (o.dense_e != 0 && o.dense_e != 1) return fail(WTS_E_ARG, "opts.dense_e = %d: 0 or 1", o.dense_e);
  if (o.walk != WTS_WALK_AUTO && o.walk != WTS_WALK_STRIPS && o.walk != WTS_WALK_PAIRS)
    return fail(WTS_E_ARG, "opts.walk = %d: 0, 1 or 2", o.walk);
  if (o.decision != WTS_DECISION_FP64 && o.decision != WTS_DECISION_FP32)
    return fail(WTS_E_ARG, "opts.decision = %d: 0 or 1", o.decision);
  if (o.decision == WTS_DECISION_FP32 && (dtype != WTS_F32 || o.cost != WTS_COST_SQEUCLID))
    return fail(WTS_E_UNSUPPORTED, "float32 decisions need float32 cycles and the squared cost");
  if (!(o.band >= 0.0) || !std::isfinite(o.band)) return fail(WTS_E_ARG, "opts.band must be finite and >= 0");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(WTS_E_ARG, "device %d of %d", device, ndev);

  wts_plan* p = new wts_plan();
  p->device = device;
  p->n = n;
  p->d = d;
  p->dtype = dtype;
  p->L = L;
  p->opts = o;
  p->rho = o.rho ? o.rho : 4;   // medoid sweeps: 2, 4 or 5 (4 when automatic)
  p->off.assign(offsets_host, offsets_host + n + 1);
  for (int k = 0; k < n; ++k) p->nmax = std::max(p->nmax, p->off[k + 1] - p->off[k]);
  if (o.band > 0.0 && (L >= (int64_t(1) << 26) || p->nmax >= (int64_t(1) << 26))) {
    delete p;
    return fail(WTS_E_SHAPE, "a Sakoe-Chiba band needs L and every cycle length below 2^26");
  }

  DeviceGuard g(device);
  if (scratch_setup(device) != WTS_OK) {
    delete p;
    return WTS_E_HIP;
  }
  auto cleanup_fail = [&](hipError_t e, const char* what) {
    wts_plan_destroy(p);
    return fail(WTS_E_HIP, "%s failed: %s", what, hipGetErrorString(e));
  };
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    p->cus = cus;

  std::vector<Job> jobs;
  if (L > 0) {
    for (int k = 0; k < n; ++k)
      jobs.push_back(Job{0, p->off[k], (int32_t)L, (int32_t)(p->off[k + 1] - p->off[k]), k});
    build_set(p->bary, jobs, o.rho ? o.rho : bary_rho(L, n, p->cus));
    p->bary.walk_pairs = o.walk == WTS_WALK_PAIRS ||
                         (o.walk == WTS_WALK_AUTO && walk_pairs_pays(p->bary));
    build_set(p->soft, jobs, wts::kSoftRho);
    std::vector<Job> tjobs;
    for (int k = 0; k < n; ++k)
      tjobs.push_back(Job{p->off[k], 0, (int32_t)(p->off[k + 1] - p->off[k]), (int32_t)L, k});
    build_set(p->softT, tjobs, wts::kSoftRho);
    std::vector<int64_t> base(n);
    for (int k = 0; k < n; ++k) base[k] = (int64_t)k * (L - 1) + p->off[k];
    hipError_t e;
    if ((e = hipMalloc(&p->d_path_base, sizeof(int64_t) * n)) != hipSuccess) return cleanup_fail(e, "hipMalloc");
    if ((e = hipMemcpy(p->d_path_base, base.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup_fail(e, "hipMemcpy");
  } else {
    // all pairs a < b, the shorter cycle on the rows (DTW is symmetric)
    std::vector<int2> ab;
    for (int a = 0; a < n; ++a)
      for (int b = a + 1; b < n; ++b) {
        const int64_t la = p->off[a + 1] - p->off[a], lb = p->off[b + 1] - p->off[b];
        const int slot = (int)ab.size();
        ab.push_back(make_int2(a, b));
        if (la <= lb) jobs.push_back(Job{p->off[a], p->off[b], (int32_t)la, (int32_t)lb, slot});
        else jobs.push_back(Job{p->off[b], p->off[a], (int32_t)lb, (int32_t)la, slot});
      }
    build_set(p->med, jobs, p->rho);
    if (!ab.empty()) {
      hipError_t e;
      if ((e = hipMalloc(&p->d_med_ab, sizeof(int2) * ab.size())) != hipSuccess) return cleanup_fail(e, "hipMalloc");
      if ((e = hipMemcpy(p->d_med_ab, ab.data(), sizeof(int2) * ab.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup_fail(e, "hipMemcpy");
    }
  }
  for (PairSet* ps : {&p->bary, &p->med, &p->soft, &p->softT}) {
    if (ps->pairs.empty()) continue;
    hipError_t e;
    if ((e = hipMalloc(&ps->d_pairs, sizeof(PairDesc) * ps->pairs.size())) != hipSuccess) return cleanup_fail(e, "hipMalloc");
    if ((e = hipMalloc(&ps->d_items, sizeof(int2) * ps->items.size())) != hipSuccess) return cleanup_fail(e, "hipMalloc");
    if ((e = hipMalloc(&ps->d_items_rev, sizeof(int2) * ps->items_rev.size())) != hipSuccess) return cleanup_fail(e, "hipMalloc");
    if ((e = hipMalloc(&ps->d_sweep_items, sizeof(int2) * ps->sweep_items.size())) != hipSuccess) return cleanup_fail(e, "hipMalloc");
    if ((e = hipMemcpy(ps->d_sweep_items, ps->sweep_items.data(), sizeof(int2) * ps->sweep_items.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(ps->d_items_rev, ps->items_rev.data(), sizeof(int2) * ps->items_rev.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(ps->d_pairs, ps->pairs.data(), sizeof(PairDesc) * ps->pairs.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup_fail(e, "hipMemcpy");
    if ((e = hipMemcpy(ps->d_items, ps->items.data(), sizeof(int2) * ps->items.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup_fail(e, "hipMemcpy");
  }
  for (PairSet* ps : {&p->bary, &p->med, &p->soft, &p->softT})
    if (ps->items.size() > (size_t(1) << 30)) {
      wts_plan_destroy(p);
      return fail(WTS_E_CAPACITY, "more than 2^30 sweep items (pairs x strips)");
    }
  hipError_t e;
  if ((e = hipMalloc(&p->d_status, 4 * sizeof(int))) != hipSuccess) return cleanup_fail(e, "hipMalloc");
  if ((e = hipMemset(p->d_status, 0, 4 * sizeof(int))) != hipSuccess) return cleanup_fail(e, "hipMemset");
  if ((e = hipMalloc(&p->d_tiles, 2 * sizeof(unsigned long long))) != hipSuccess)
    return cleanup_fail(e, "hipMalloc");
  if ((e = hipMemset(p->d_tiles, 0, 2 * sizeof(unsigned long long))) != hipSuccess)
    return cleanup_fail(e, "hipMemset");
  if ((e = hipMalloc(&p->d_off, sizeof(int64_t) * (n + 1))) != hipSuccess) return cleanup_fail(e, "hipMalloc");
  if ((e = hipMemcpy(p->d_off, p->off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup_fail(e, "hipMemcpy");
  *out = p;
  return WTS_OK;
}

wts_status wts_plan_timing(wts_plan* p, int32_t max_launches) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  if (max_launches < 0 || max_launches > 4096) return fail(WTS_E_ARG, "max_launches %d", max_launches);
  DeviceGuard g(p->device);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->ev_op.clear();
  p->ev_next = 0;
  for (int k = 0; k < 2 * max_launches; ++k) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    p->ev.push_back(e);
  }
  p->ev_op.assign(max_launches, -1);
  return WTS_OK;
}

int32_t wts_plan_walk(const wts_plan* p) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  if (p->L == 0) return fail(WTS_E_ARG, "a medoid plan recovers no paths");
  return p->bary.walk_pairs ? WTS_WALK_PAIRS : WTS_WALK_STRIPS;
}

wts_status wts_plan_bwd_tiles(wts_plan* p, int64_t* swept, int64_t* in_range) {
  if (!p || !swept || !in_range) return fail(WTS_E_ARG, "null argument");
  DeviceGuard g(p->device);
  unsigned long long t[2] = {0, 0};
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(t, p->d_tiles, sizeof(t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(p->d_tiles, 0, sizeof(t)));
  *swept = (int64_t)t[0];
  *in_range = (int64_t)t[1];
  return WTS_OK;
}

wts_status wts_plan_sweep_ms(wts_plan* p, int op, double* total_ms, int32_t* launches) {
  if (!p || !total_ms || !launches) return fail(WTS_E_ARG, "null argument");
  DeviceGuard g(p->device);
  double tot = 0.0;
  int cnt = 0;
  for (size_t k = 0; k < p->ev_op.size(); ++k) {
    if (p->ev_op[k] != op) continue;
    float ms = 0.f;
    HIP_TRY(hipEventSynchronize(p->ev[2 * k + 1]));
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]));
    tot += ms;
    ++cnt;
    p->ev_op[k] = -1;
  }
  *total_ms = tot;
  *launches = cnt;
  return WTS_OK;
}

int32_t wts_plan_rho(const wts_plan* p, int op) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  switch (op) {
    case WTS_OP_ALIGN:
    case WTS_OP_ALIGN_PATHS:
    case WTS_OP_DBA:
    case WTS_OP_SCORE:
    case WTS_OP_SUBDTW:
      if (p->L <= 0) return fail(WTS_E_ARG, "plan was created with L = 0 (medoid/init only)");
      return p->bary.rho;
    case WTS_OP_SOFT_FWD:
    case WTS_OP_SOFT_BWD:
    case WTS_OP_SOFT_GRAD_C:
      if (p->L <= 0) return fail(WTS_E_ARG, "plan was created with L = 0 (medoid/init only)");
      return op == WTS_OP_SOFT_GRAD_C ? p->softT.rho : p->soft.rho;
    case WTS_OP_MEDOID:
      if (p->L != 0) return fail(WTS_E_ARG, "medoid needs a plan with L = 0");
      return p->med.rho;
    default:
      return fail(WTS_E_ARG, "unknown op %d", op);
  }
}

void wts_plan_destroy(wts_plan* p) {
  if (!p) return;
  DeviceGuard g(p->device);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  for (PairSet* ps : {&p->bary, &p->med, &p->soft, &p->softT}) {
    if (ps->d_pairs) (void)hipFree(ps->d_pairs);
    if (ps->d_items) (void)hipFree(ps->d_items);
    if (ps->d_items_rev) (void)hipFree(ps->d_items_rev);
    if (ps->d_sweep_items) (void)hipFree(ps->d_sweep_items);
  }
  if (p->d_off) (void)hipFree(p->d_off);
  if (p->d_status) (void)hipFree(p->d_status);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  if (p->d_path_base) (void)hipFree(p->d_path_base);
  if (p->d_med_ab) (void)hipFree(p->d_med_ab);
  delete p;
}

size_t wts_workspace_bytes(const wts_plan* p, int op) {
  if (!p) return 0;
  switch (op) {
    case WTS_OP_ALIGN:
    case WTS_OP_ALIGN_PATHS:
    case WTS_OP_DBA:
    case WTS_OP_SCORE:
    case WTS_OP_SOFT_FWD:
    case WTS_OP_SOFT_BWD:
    case WTS_OP_SUBDTW:
    case WTS_OP_SOFT_GRAD_C:
      return p->L > 0 ? layout(p, op).total : 0;
    case WTS_OP_MEDOID:
      return p->L == 0 ? layout(p, op).total : 0;
    default:
      return 0;
  }
}

wts_status wts_dtw_align(const wts_plan* p, const double* bary, const void* cycles, double* dist,
                         int64_t* path_len, int32_t* paths, void* ws, size_t ws_bytes,
                         void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!bary || !cycles || !dist || !path_len) return fail(WTS_E_ARG, "null bary/cycles/dist/path_len");
  if (paths && p->opts.cost != WTS_COST_SQEUCLID)
    return fail(WTS_E_UNSUPPORTED, "paths are recovered for the squared cost only");
  const int op = paths ? WTS_OP_ALIGN_PATHS : WTS_OP_ALIGN;
  if ((rc = check_ws(p, op, ws, ws_bytes)) != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(bary, p->L * p->d), seg_cycles(p, cycles))) != WTS_OK)
    return rc;
  const Layout l = layout(p, op);
  if (!paths) {
    rc = run_sweep(p, p->bary, wts::MODE_DIST_LEN, p->opts.cost == WTS_COST_EUCLID, false, bary,
                   cycles, ws, l, dist, st);
    if (rc != WTS_OK) return rc;
    HIP_TRY(wts::launch_score(dist, at<int>(ws, l.out_aux), p->n, nullptr, path_len, st));
    return WTS_OK;
  }
  rc = run_paths(p, bary, cycles, ws, l, dist, nullptr, nullptr, st);
  if (rc != WTS_OK) return rc;
  const PairSet& ps = p->bary;
  HIP_TRY(wts::launch_seg_prefix(ps.d_pairs, ps.n_pairs, at<int>(ws, l.seg_len),
                                 at<int>(ws, l.seg_off), path_len, st));
  wts::WalkArgs w{};
  w.pairs = ps.d_pairs;
  w.items = ps.d_items;
  w.seg = at<int2>(ws, l.seg);
  w.codes = at<uint32_t>(ws, l.codes);
  w.y = cycles;
  w.L = p->L;
  w.seg_len = at<int>(ws, l.seg_len);
  w.seg_off = at<int>(ws, l.seg_off);
  w.path_base = p->d_path_base;
  w.paths = paths;
  w.status = p->d_status;
  w.skip = skip_of(p);
  HIP_TRY(wts::launch_walk(p->d, ps.rho, p->dtype, true, w, ps.n_items, st));
  return WTS_OK;
}

wts_status wts_dba_iterate(const wts_plan* p, const double* bary_in, const void* cycles,
                           const double* weights, double* bary_out, int64_t* counts, double* dist,
                           void* ws, size_t ws_bytes, void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!bary_in || !cycles || !bary_out || !counts) return fail(WTS_E_ARG, "null bary/cycles/out/counts");
  if (bary_in == bary_out) return fail(WTS_E_ARG, "bary_out must not alias bary_in");
  if ((rc = check_ws(p, WTS_OP_DBA, ws, ws_bytes)) != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(bary_in, p->L * p->d), seg_cycles(p, cycles),
                            seg_f64(weights, p->n))) != WTS_OK)
    return rc;
  const Layout l = layout(p, WTS_OP_DBA);
  rc = run_paths(p, bary_in, cycles, ws, l, dist, at<double>(ws, l.psum), at<int>(ws, l.pcnt), st);
  if (rc != WTS_OK) return rc;
  HIP_TRY(wts::launch_dba_reduce(at<double>(ws, l.psum), at<int>(ws, l.pcnt), weights, p->n,
                                 p->L, p->d, bary_out, counts, st));
  return WTS_OK;
}

wts_status wts_anomaly_score(const wts_plan* p, const double* bary, const void* cycles,
                             double* score, double* dist, int64_t* path_len, void* ws,
                             size_t ws_bytes, void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!bary || !cycles || !score) return fail(WTS_E_ARG, "null bary/cycles/score");
  if ((rc = check_ws(p, WTS_OP_SCORE, ws, ws_bytes)) != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(bary, p->L * p->d), seg_cycles(p, cycles))) != WTS_OK)
    return rc;
  const Layout l = layout(p, WTS_OP_SCORE);
  double* dv = dist ? dist : at<double>(ws, l.out_dist);
  rc = run_sweep(p, p->bary, wts::MODE_DIST_LEN, p->opts.cost == WTS_COST_EUCLID, false, bary,
                 cycles, ws, l, dv, st);
  if (rc != WTS_OK) return rc;
  HIP_TRY(wts::launch_score(dv, at<int>(ws, l.out_aux), p->n, score, path_len, st));
  return WTS_OK;
}

wts_status wts_anomaly_score_noalloc(const wts_plan* p, const double* bary, const void* cycles,
                                     double* score, double* dist, int64_t* path_len,
                                     void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  const size_t need = layout(p, WTS_OP_SCORE).total;
  if (need > kScratchBytes)
    return fail(WTS_E_CAPACITY, "the score sweep of this plan needs %zu bytes of workspace; "
                "the static scratch holds %zu", need, kScratchBytes);
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (p->device >= 0 && p->device < kMaxDevices) ws = g_scratch[p->device];
  }
  if (ws == nullptr) return fail(WTS_E_HIP, "no scratch address for device %d", p->device);
  return wts_anomaly_score(p, bary, cycles, score, dist, path_len, ws, kScratchBytes, stream);
}

wts_status wts_subdtw(const wts_plan* p, const double* x, const void* windows, double* value,
                      int64_t* a_star, int64_t* b_star, void* ws, size_t ws_bytes, void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!x || !windows || !value || !a_star || !b_star)
    return fail(WTS_E_ARG, "null x/windows/value/a_star/b_star");
  if (p->opts.cost == WTS_COST_EUCLID)
    return fail(WTS_E_UNSUPPORTED, "Sub-DTW is built for the squared cost only");
  if ((rc = check_ws(p, WTS_OP_SUBDTW, ws, ws_bytes)) != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(x, p->L * p->d), seg_cycles(p, windows))) != WTS_OK)
    return rc;
  const Layout l = layout(p, WTS_OP_SUBDTW);
  rc = run_sweep(p, p->bary, wts::MODE_SUB, false, false, x, windows, ws, l, value, st);
  if (rc != WTS_OK) return rc;
  HIP_TRY(wts::launch_sub_out(at<int>(ws, l.out_aux), at<int>(ws, l.out_end), p->n, a_star,
                              b_star, st));
  return WTS_OK;
}

wts_status wts_softdtw_forward(const wts_plan* p, const double* bary, const void* cycles,
                               double gamma, double* value, void* ckpt, size_t ckpt_bytes,
                               void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!bary || !cycles || !value) return fail(WTS_E_ARG, "null bary/cycles/value");
  if (!(gamma > 0) || !(gamma < INFINITY)) return fail(WTS_E_ARG, "gamma must be finite and > 0");
  if ((rc = check_ws(p, WTS_OP_SOFT_FWD, ckpt, ckpt_bytes)) != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(bary, p->L * p->d), seg_cycles(p, cycles))) != WTS_OK)
    return rc;
  const Layout l = layout(p, WTS_OP_SOFT_FWD);
  const PairSet& ps = p->soft;
  HIP_TRY(wts::launch_zero(at<int>(ckpt, l.queue), 2, st));
  HIP_TRY(wts::launch_zero(at<int>(ckpt, l.progress), ps.n_flags, st));
  wts::SoftArgs a{};
  a.pairs = ps.d_pairs;
  a.items = ps.d_sweep_items;
  a.n_items = ps.n_items;
  a.queue = at<int>(ckpt, l.queue);
  a.status = p->d_status;
  a.skip = skip_of(p);
  a.relaxed_wait = ps.n_items > 16 * p->cus ? 1 : 0;   // > 4 items per SIMD
  a.progress = at<int>(ckpt, l.progress);
  a.x = bary;
  a.y = cycles;
  a.rows = at<double>(ckpt, l.rows);
  a.states = at<double>(ckpt, l.states);
  a.kscale = 1.0 / (gamma * 0.69314718055994530942);
  a.band = p->opts.band;
  a.value = value;
  a.L = p->L;
  const int tk = timing_begin(p, WTS_OP_SOFT_FWD, st);
  HIP_TRY(wts::launch_soft(p->d, p->dtype, false, a, default_grid(p, ps), st));
  timing_end(p, tk, st);
  return WTS_OK;
}

wts_status wts_softdtw_backward(const wts_plan* p, const double* bary, const void* cycles,
                                double gamma, const void* ckpt, size_t ckpt_bytes,
                                const double* grad_value, double* grad_bary, double* row_mass,
                                int32_t accumulate, void* ws, size_t ws_bytes, void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!bary || !cycles || !grad_bary) return fail(WTS_E_ARG, "null bary/cycles/grad_bary");
  if (!(gamma > 0) || !(gamma < INFINITY)) return fail(WTS_E_ARG, "gamma must be finite and > 0");
  if ((rc = check_ws(p, WTS_OP_SOFT_FWD, const_cast<void*>(ckpt), ckpt_bytes)) != WTS_OK) return rc;
  if ((rc = check_ws(p, WTS_OP_SOFT_BWD, ws, ws_bytes)) != WTS_OK) return rc;
  if (accumulate != 0 && accumulate != 1) return fail(WTS_E_ARG, "accumulate = %d: 0 or 1", accumulate);
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(bary, p->L * p->d), seg_cycles(p, cycles),
                            seg_f64(grad_value, p->n))) != WTS_OK)
    return rc;
  const Layout lc = layout(p, WTS_OP_SOFT_FWD);
  const Layout l = layout(p, WTS_OP_SOFT_BWD);
  const PairSet& ps = p->soft;
  void* ck = const_cast<void*>(ckpt);
  HIP_TRY(wts::launch_zero(at<int>(ws, l.queue), 2, st));
  HIP_TRY(wts::launch_zero(at<int>(ws, l.progress), ps.n_flags, st));
  wts::SoftArgs a{};
  a.pairs = ps.d_pairs;
  a.items = ps.d_items_rev;
  a.n_items = ps.n_items;
  a.queue = at<int>(ws, l.queue);
  a.status = p->d_status;
  a.skip = skip_of(p);
  a.relaxed_wait = ps.n_items > 16 * p->cus ? 1 : 0;   // > 4 items per SIMD
  a.progress = at<int>(ws, l.progress);
  a.x = bary;
  a.y = cycles;
  a.rows = at<double>(ck, lc.rows);
  a.states = at<double>(ck, lc.states);
  a.kscale = 1.0 / (gamma * 0.69314718055994530942);
  a.band = p->opts.band;
  a.push_up = at<float>(ws, l.push_up);
  a.push_dg = at<float>(ws, l.push_dg);
  a.gsum = at<double>(ws, l.gsum);
  a.hsum = at<double>(ws, l.hsum);
  a.L = p->L;
  a.zero_skip = p->opts.dense_e ? 0 : 1;
  a.tiles = p->d_tiles;
  const int tk = timing_begin(p, WTS_OP_SOFT_BWD, st);
  HIP_TRY(wts::launch_soft(p->d, p->dtype, true, a, default_grid(p, ps), st));
  timing_end(p, tk, st);
  HIP_TRY(wts::launch_soft_reduce(a.gsum, a.hsum, grad_value, p->n, p->L, p->d, grad_bary,
                                  row_mass, accumulate, st));
  return WTS_OK;
}

wts_status wts_softdtw_grad_cycles(const wts_plan* p, const double* bary, const double* cycles64,
                                   double gamma, const double* grad_value, double* grad_cycles,
                                   void* ws, size_t ws_bytes, void* stream) {
  wts_status rc = check_bary_plan(p);
  if (rc != WTS_OK) return rc;
  if (!bary || !cycles64 || !grad_cycles) return fail(WTS_E_ARG, "null bary/cycles64/grad_cycles");
  if (!(gamma > 0) || !(gamma < INFINITY)) return fail(WTS_E_ARG, "gamma must be finite and > 0");
  if ((rc = check_ws(p, WTS_OP_SOFT_GRAD_C, ws, ws_bytes)) != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_f64(bary, p->L * p->d), seg_f64(cycles64, p->off[p->n] * p->d),
                            seg_f64(grad_value, p->n))) != WTS_OK)
    return rc;
  const Layout l = layout(p, WTS_OP_SOFT_GRAD_C);
  const PairSet& ps = p->softT;
  wts::SoftArgs a{};
  a.pairs = ps.d_pairs;
  a.n_items = ps.n_items;
  a.queue = at<int>(ws, l.queue);
  a.status = p->d_status;
  a.skip = skip_of(p);
  a.relaxed_wait = ps.n_items > 16 * p->cus ? 1 : 0;   // > 4 items per SIMD
  a.progress = at<int>(ws, l.progress);
  a.x = cycles64;          // rows: every cycle, at its own offset (PairDesc.x_off)
  a.y = bary;              // columns: the barycenter, shared by all pairs
  a.rows = at<double>(ws, l.rows);
  a.states = at<double>(ws, l.states);
  a.kscale = 1.0 / (gamma * 0.69314718055994530942);
  a.band = p->opts.band;   // the band is symmetric in the two series
  a.value = at<double>(ws, l.out_dist);
  a.push_up = at<float>(ws, l.push_up);
  a.push_dg = at<float>(ws, l.push_dg);
  a.gsum = at<double>(ws, l.gsum);
  a.hsum = at<double>(ws, l.hsum);
  a.L = p->L;
  a.rows_packed = 1;
  HIP_TRY(wts::launch_zero(a.queue, 2, st));
  HIP_TRY(wts::launch_zero(a.progress, ps.n_flags, st));
  a.items = ps.d_sweep_items;
  HIP_TRY(wts::launch_soft(p->d, WTS_F64, false, a, default_grid(p, ps), st));
  HIP_TRY(wts::launch_zero(a.queue, 2, st));
  HIP_TRY(wts::launch_zero(a.progress, ps.n_flags, st));
  a.items = ps.d_items_rev;
  a.zero_skip = p->opts.dense_e ? 0 : 1;
  a.tiles = p->d_tiles;
  HIP_TRY(wts::launch_soft(p->d, WTS_F64, true, a, default_grid(p, ps), st));
  HIP_TRY(wts::launch_soft_rows_scale(a.gsum, p->d_off, p->n, p->off[p->n], p->d, grad_value,
                                      grad_cycles, st));
  return WTS_OK;
}

wts_status wts_precond_step(double* bary, const double* grad, const double* row_mass, int64_t L,
                            int32_t d, double eta, void* stream) {
  if (!bary || !grad || !row_mass) return fail(WTS_E_ARG, "null bary/grad/row_mass");
  if (L < 1 || d < 1) return fail(WTS_E_SHAPE, "L = %lld, d = %d", (long long)L, d);
  if (!(eta == eta)) return fail(WTS_E_ARG, "eta is NaN");
  HIP_TRY(wts::launch_precond_step(bary, grad, row_mass, L, d, eta,
                                   static_cast<hipStream_t>(stream)));
  return WTS_OK;
}

wts_status wts_medoid(const wts_plan* p, const void* cycles, double* dist_matrix, double* totals,
                      int32_t* medoid, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  if (p->L != 0) return fail(WTS_E_ARG, "wts_medoid needs a plan created with L = 0");
  if (!cycles || !medoid) return fail(WTS_E_ARG, "null cycles/medoid");
  wts_status rc = check_ws(p, WTS_OP_MEDOID, ws, ws_bytes);
  if (rc != WTS_OK) return rc;
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = validate_inputs(p, st, seg_cycles(p, cycles))) != WTS_OK) return rc;
  const Layout l = layout(p, WTS_OP_MEDOID);
  double* Dm = dist_matrix ? dist_matrix : at<double>(ws, l.dm);
  double* tot = totals ? totals : at<double>(ws, l.totals);
  double* pair_dist = at<double>(ws, l.out_dist);
  if (p->med.n_pairs > 0) {
    rc = run_sweep(p, p->med, wts::MODE_DIST, false, true, cycles, cycles, ws, l, pair_dist, st);
    if (rc != WTS_OK) return rc;
  }
  HIP_TRY(wts::launch_medoid(pair_dist, p->d_med_ab, p->med.n_pairs, p->n, Dm, tot, medoid, st));
  return WTS_OK;
}

wts_status wts_init_barycenter(const wts_plan* p, const void* cycles, int32_t kind, int32_t index,
                               double* bary_out, int32_t* chosen_host, void* stream) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  if (p->L <= 0) return fail(WTS_E_ARG, "wts_init_barycenter needs a plan with L > 0");
  if (!cycles || !bary_out) return fail(WTS_E_ARG, "null cycles/bary_out");
  int src = 0;
  int64_t Nsrc = 0;
  int euclid = 0;
  if (kind == WTS_INIT_EUCLID_MEAN) {
    euclid = 1;
    Nsrc = p->nmax;
  } else if (kind == WTS_INIT_NEAREST) {
    int64_t best = INT64_MAX;
    for (int k = 0; k < p->n; ++k) {
      const int64_t N = p->off[k + 1] - p->off[k];
      const int64_t dd = N > p->L ? N - p->L : p->L - N;
      if (dd < best) { best = dd; src = k; }
    }
    Nsrc = p->off[src + 1] - p->off[src];
  } else if (kind == WTS_INIT_COPY) {
    if (index < 0 || index >= p->n) return fail(WTS_E_ARG, "index %d out of range", index);
    src = index;
    Nsrc = p->off[src + 1] - p->off[src];
  } else {
    return fail(WTS_E_ARG, "init kind %d", kind);
  }
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const wts_status rc = validate_inputs(p, st, seg_cycles(p, cycles));
  if (rc != WTS_OK) return rc;
  HIP_TRY(wts::launch_init(p->dtype, cycles, p->d_off, p->n, p->d, src, Nsrc, p->L, euclid,
                           bary_out, st));
  if (chosen_host) *chosen_host = euclid ? -1 : src;
  return WTS_OK;
}

wts_status wts_plan_status(const wts_plan* p, void* stream) {
  if (!p) return fail(WTS_E_ARG, "plan is null");
  DeviceGuard g(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(wts::launch_status_take(p->d_status, p->d_status + 2, st));
  int word = 0;
  HIP_TRY(hipMemcpyAsync(&word, p->d_status + 2, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (word & wts::kStatusNonFinite)
    return fail(WTS_E_NONFINITE, "a validated call found a NaN or an infinity in its inputs; "
                "the sweeps of that call were skipped and its outputs are undefined");
  if (word & wts::kStatusSpinTimeout)
    return fail(WTS_E_DEVICE, "a strip gave up waiting for its neighbour; the results of the "
                "calls since the last status read are undefined");
  if (word & wts::kStatusBadPath)
    return fail(WTS_E_DEVICE, "path recovery found inconsistent strip tags; the paths and DBA "
                "updates since the last status read are undefined");
  return WTS_OK;
}

wts_status wts_barycenter_objective(const double* values, const double* weights, int32_t n,
                                    int32_t accumulate, double* out, void* stream) {
  if (!values || !out) return fail(WTS_E_ARG, "null values/out");
  if (n < 1) return fail(WTS_E_SHAPE, "n = %d", n);
  if (accumulate != 0 && accumulate != 1) return fail(WTS_E_ARG, "accumulate = %d: 0 or 1", accumulate);
  HIP_TRY(wts::launch_objective(values, weights, n, accumulate, out,
                                static_cast<hipStream_t>(stream)));
  return WTS_OK;
}

}  // extern "C"
