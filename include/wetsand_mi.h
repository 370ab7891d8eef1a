/*
 * wetsand_mi.h -- C ABI of the WETSAND hot path on AMD MI355X (gfx950).
 *
 * WETSAND (warped time-series anomaly detection) builds a prototype cycle
 * (a barycenter B) from many unevenly long cycles and scores every cycle by
 * its DTW distance to B.  This library runs the dynamic programs behind that
 * on one GPU:
 *
 *   wts_dtw_align        DTW value, path length and optional warping path of
 *                        every (B, C_k) pair                 (Sec. III-B, Eq. 1)
 *   wts_dba_iterate      one DTW-barycenter-averaging update of B     (Sec. II,
 *                        Sec. V-B: the DBA barycenter the paper compares with)
 *   wts_softdtw_forward  Soft-DTW values of every (B, C_k) pair  (Eq. 3-5)
 *   wts_softdtw_backward gradient of sum_k w_k Soft-DTW(B, C_k) w.r.t. B
 *                        through the E matrix                  (Eq. 6, Eq. 7)
 *   wts_anomaly_score    d_score = DTW(B, C_k) / |pi_k|        (Sec. III-D, Eq. 8)
 *   wts_subdtw           Sub-DTW of a reference cycle X against many windows,
 *                        with the first and last matched window columns
 *                        (Sec. III-B, Eq. 2: the segmentation step)
 *   wts_precond_step     one preconditioned gradient step on B (Eq. 7 driver)
 *   wts_barycenter_objective  sum_k w_k Soft-DTW(B, C_k), the Eq. 7 objective
 *   wts_medoid           all-pairs DTW and the medoid cycle (barycenter init)
 *   wts_init_barycenter  Euclidean-mean (Table I "Init", Sec. V-D) /
 *                        nearest-length / copy initialisation
 *   wts_plan_status      reads the device status word of a plan's calls
 *
 * Conventions
 *  - Every pointer argument is DEVICE memory unless its name ends in _host.
 *    The caller owns every buffer; compute calls never allocate and never
 *    synchronise: they enqueue work on `stream` (a hipStream_t, NULL = the
 *    null stream) and return.
 *  - Series are time-major: sample t of a d-channel series occupies d
 *    consecutive values.  The cycles of a batch are packed back to back in
 *    one buffer; offsets_host[k] .. offsets_host[k+1] is cycle k.  Cycle
 *    values are float32 (WTS_F32) or float64 (WTS_F64) as fixed at plan time
 *    and are widened exactly to float64 on load.  Barycenters, distances,
 *    scores and gradients are always float64.
 *  - Cost: delta(b, y) = sum_c (b_c - y_c)^2 computed as e_0*e_0 followed by
 *    fma(e_c, e_c, s) (squared Euclidean, Def. 3); WTS_COST_EUCLID takes its
 *    correctly rounded square root (DTW values and scores only).
 *  - Optimal path: the backtrack from (L, N) takes, at every cell, the first
 *    predecessor in the order diagonal, up (i-1, j), left (i, j-1) whose
 *    cumulative cost equals the minimum.  Distances, paths, path lengths and
 *    alignment counts are bitwise identical to a float64 CPU evaluation of
 *    the same definitions.
 *  - Inputs must be finite: the paper drops samples with missing values
 *    before any DTW (Sec. III-A).  A plan created with opts.validate = 1
 *    checks this on the device at the start of every compute call (one pass
 *    over the call's input values); a call that finds a NaN or an infinity
 *    skips its sweeps and leaves its outputs undefined, and the next
 *    wts_plan_status returns WTS_E_NONFINITE.  Without validation,
 *    non-finite inputs give unspecified results.
 *  - Errors: a non-zero wts_status is returned before anything is enqueued;
 *    wts_last_error() gives a message (thread-local).  WTS_E_HIP reports a
 *    failed HIP call (for instance a launch failure).  What the kernels find
 *    while they run (non-finite inputs, a strip that gave up waiting for its
 *    neighbour, inconsistent path tags) goes into the plan's device status
 *    word, which wts_plan_status reads.
 */
#ifndef WETSAND_MI_H
#define WETSAND_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wts_plan wts_plan;

typedef enum {
  WTS_OK = 0,
  WTS_E_ARG = -1,          /* null pointer where one is required, bad enum, gamma <= 0 ... */
  WTS_E_SHAPE = -2,        /* n, d, L or a cycle length out of range */
  WTS_E_DTYPE = -3,        /* dtype is not WTS_F32 / WTS_F64 */
  WTS_E_WORKSPACE = -4,    /* ws_bytes (or ckpt_bytes) smaller than required */
  WTS_E_CAPACITY = -5,     /* a size beyond a fixed limit of this library: L or a cycle longer
                              than 2^24 samples, more than 2^30 sweep items (pairs x strips) */
  WTS_E_HIP = -6,          /* a HIP runtime call failed */
  WTS_E_NONFINITE = -7,    /* (wts_plan_status) a validated call found a NaN or an infinity */
  WTS_E_UNSUPPORTED = -8,  /* valid request this library does not implement */
  WTS_E_DEVICE = -9        /* (wts_plan_status) a kernel reported an inconsistency: a strip
                              gave up waiting for its neighbour (about a second), or path
                              recovery met inconsistent tags; results are undefined        */
} wts_status;

enum { WTS_F32 = 0, WTS_F64 = 1 };
enum { WTS_COST_SQEUCLID = 0, WTS_COST_EUCLID = 1 };

/* Operation selectors for wts_workspace_bytes. */
enum {
  WTS_OP_ALIGN = 0,        /* wts_dtw_align without paths           */
  WTS_OP_ALIGN_PATHS = 1,  /* wts_dtw_align with paths              */
  WTS_OP_DBA = 2,          /* wts_dba_iterate                       */
  WTS_OP_SCORE = 3,        /* wts_anomaly_score                     */
  WTS_OP_SOFT_FWD = 4,     /* checkpoint buffer of the Soft-DTW pair */
  WTS_OP_SOFT_BWD = 5,     /* workspace of wts_softdtw_backward      */
  WTS_OP_MEDOID = 6,       /* wts_medoid                            */
  WTS_OP_SUBDTW = 7,       /* wts_subdtw                            */
  WTS_OP_SOFT_GRAD_C = 8   /* wts_softdtw_grad_cycles               */
};

enum { WTS_INIT_EUCLID_MEAN = 0, WTS_INIT_NEAREST = 1, WTS_INIT_COPY = 2 };

enum { WTS_DECISION_FP64 = 0, WTS_DECISION_FP32 = 1 };
enum { WTS_WALK_AUTO = 0, WTS_WALK_STRIPS = 1, WTS_WALK_PAIRS = 2 };

typedef struct {
  int32_t cost;       /* WTS_COST_* for wts_dtw_align / wts_anomaly_score; DBA, Soft-DTW and
                         the medoid always use the squared cost                              */
  int32_t rho;        /* rows per lane in the wavefront sweeps: 0 = automatic (4, or 5 for
                         barycenter plans whose strips would just about fill every SIMD);
                         2, 4 or 5 for any plan (Soft-DTW sweeps always use 2); other
                         values return WTS_E_UNSUPPORTED                                     */
  int32_t grid;       /* workgroups of the persistent sweep (0 = tuned default)              */
  int32_t validate;   /* 1: every compute call first checks its inputs for NaN / infinity on
                         the device (see Conventions); 0: no check                           */
  int32_t decision;   /* precision of the hard-DTW sweeps (wts_dtw_align, wts_dba_iterate,
                         wts_anomaly_score[_noalloc], wts_medoid, wts_subdtw):
                         WTS_DECISION_FP64 (0, default): cost, minima and argmins in
                         float64, bit for bit the float64 definitions (Def. 3, Eq. 1, Eq. 2);
                         WTS_DECISION_FP32 (1): the same operations in float32 on the
                         float32 cycles and the barycenter rounded to float32 -- about
                         twice the arithmetic rate, with values, paths and codes bit for
                         bit those of the float32 evaluation of the same definitions
                         (near-ties may resolve differently from float64).  Needs
                         WTS_F32 cycles and the squared cost (else WTS_E_UNSUPPORTED).
                         Path sums, DBA means and scores stay float64; the Soft-DTW
                         calls do not read this field                                   */
  double band;        /* Soft-DTW only: Sakoe-Chiba bandwidth as a fraction w of the longer
                         length (Table I: 0.6); 0 = no band.  Cell (i, j) of an M x N pair
                         is kept iff |i (N-1) - j (M-1)| <= R min(M-1, N-1) with
                         R = max(ceil(w max(M, N)), ceil(max(M-1,N-1) / min(M-1,N-1)))
                         (computed in float64 from this value); the Soft-DTW values and
                         gradients are those over the paths inside the band.  Must be
                         finite and >= 0; a band needs L and every cycle length below
                         2^26                                                            */
  int32_t dense_e;    /* Soft-DTW backward (Eq. 6): 0 (default) skips every 16-column tile
                         of a strip whose E entries are exactly zero in the float32 e
                         arithmetic: e reaches a cell only through its successors'
                         pushes, so a tile with no push entering it is zero throughout.
                         Gradients and row masses are bit for bit those of a sweep over
                         every tile; only the time changes (E is non-zero in a band
                         around the soft alignment, a few hundred columns wide on long
                         similar series).  1: sweep every tile                            */
  int32_t walk;       /* path recovery of wts_dba_iterate / wts_dtw_align with paths:
                         WTS_WALK_STRIPS (1): the path sweep tags every cell with the cell
                         through which its path enters the strip, and all strips are then
                         walked at once; WTS_WALK_PAIRS (2): the sweep keeps only the argmin
                         codes (about a tenth faster) and each pair walks its strips in turn;
                         WTS_WALK_AUTO (0, default): pairs when the batch's cells outweigh
                         its longest pair's walk (large batches), else strips.  Paths,
                         counts and sums are the same bits either way                      */
} wts_opts;

/* Create a plan for a batch of n cycles of d channels (1 <= d <= 8) stored as
 * `dtype`, with cycle k spanning offsets_host[k] .. offsets_host[k+1]
 * (host array of n+1 non-decreasing int64, offsets_host[0] == 0, every
 * cycle at least one sample long), against a barycenter of L rows.
 * L = 0 makes a plan for wts_medoid only (all n(n-1)/2 cycle pairs); the
 * barycenter operations need L > 0.
 * The plan binds the lengths, L and the device; cycle and barycenter VALUES
 * may change between calls.  It allocates small device tables and the
 * plan's status word (hipMalloc) here, never in the compute calls.  opts may
 * be NULL (defaults).  Errors: WTS_E_ARG (null out or offsets_host, bad opts,
 * no such device), WTS_E_SHAPE (n < 1, d < 1, L < 0, offsets_host[0] != 0,
 * an empty cycle), WTS_E_UNSUPPORTED (d > 8, rho not 0/2/4/5), WTS_E_DTYPE,
 * WTS_E_CAPACITY (L or a cycle longer than 2^24, more than 2^30 sweep items),
 * WTS_E_HIP.  Calls on one plan share its status word: run them on one
 * stream, or read the status after synchronising all of them. */
wts_status wts_plan_create(wts_plan** out, int device, int32_t n, int32_t d, int32_t dtype,
                           const int64_t* offsets_host, int64_t L, const wts_opts* opts);
void wts_plan_destroy(wts_plan* plan);

/* Bytes of workspace (device memory, any content, 256-byte aligned) an
 * operation needs; 0 for an operation the plan cannot run. */
size_t wts_workspace_bytes(const wts_plan* plan, int op);

/* Sweep timing, for profiling.  wts_plan_timing(plan, k) creates k pairs of
 * HIP events (k = 0 switches timing off); afterwards every sweep kernel the
 * plan launches (the dynamic-programming kernel of an operation, not its
 * small helper kernels) is bracketed by an event pair recorded on the call's
 * stream, reusing the pairs round-robin.  Not for use under graph capture.
 * wts_plan_sweep_ms(plan, op, &total_ms, &launches) waits for the recorded
 * launches of `op` (WTS_OP_DBA for the path sweep of wts_dba_iterate and of
 * wts_dtw_align with paths, WTS_OP_SCORE for the value+length sweep,
 * WTS_OP_MEDOID, WTS_OP_SOFT_FWD, WTS_OP_SOFT_BWD), sums their durations and
 * forgets them. */
wts_status wts_plan_timing(wts_plan* plan, int32_t max_launches);
wts_status wts_plan_sweep_ms(wts_plan* plan, int op, double* total_ms, int32_t* launches);

/* The path recovery this plan's barycenter operations use (opts.walk, or the
 * automatic choice): WTS_WALK_STRIPS or WTS_WALK_PAIRS; WTS_E_ARG for a null
 * plan or a medoid plan (L = 0). */
int32_t wts_plan_walk(const wts_plan* plan);

/* Tiles of the Soft-DTW backward, for profiling: *swept receives the 16-column
 * strip tiles the backward kernels of this plan (wts_softdtw_backward,
 * wts_softdtw_grad_cycles) swept since the plan was created or last read, and
 * *in_range the tiles their strips spanned (inside the band, if any); the
 * difference is the tiles skipped as exactly zero (opts.dense_e = 0).  Waits
 * for the device, then resets both counts.  WTS_E_ARG for null arguments,
 * WTS_E_HIP if a HIP call fails.  Not for use under graph capture. */
wts_status wts_plan_bwd_tiles(wts_plan* plan, int64_t* swept, int64_t* in_range);

/* Rows per lane (rho) of the wavefront sweeps that operation `op` runs on this
 * plan, as chosen at plan creation (opts.rho, or the automatic choice); it
 * names the kernel instance a profiler shows.  Returns a value >= 1, or
 * WTS_E_ARG for a null plan or an operation the plan cannot run. */
int32_t wts_plan_rho(const wts_plan* plan, int op);

/* Message describing the last non-OK status returned on this thread. */
const char* wts_last_error(void);

/* Synchronises `stream`, then reads and clears the plan's device status word
 * (one atomic exchange on `stream`, so a bit set by a call still running on
 * another stream is reported by the next read, never lost).  The word
 * collects what every kernel of every call on this plan reported since the
 * last read: WTS_E_NONFINITE if a validated call found a NaN or an infinity
 * (that call skipped its sweeps), else WTS_E_DEVICE if a strip gave up
 * waiting for its neighbour or path recovery met inconsistent tags (the
 * results of those calls are undefined), else WTS_OK.  WTS_E_ARG for a null
 * plan, WTS_E_HIP if a HIP call fails.  It synchronises, so it cannot be
 * captured into a graph. */
wts_status wts_plan_status(const wts_plan* plan, void* stream);

/* Eq. 1 (DTW) and the optimal path of every (B, C_k).
 *   bary      [L][d] float64
 *   cycles    packed cycle values, plan dtype
 *   dist      [n] float64 out: DTW(B, C_k) = r_{L, N_k}
 *   path_len  [n] int64 out: |pi_k|, number of index pairs on the path
 *   paths     NULL, or int32 [n (L-1) + offsets_host[n]][2] out: the (i, j)
 *             pairs of pi_k (0-based, forward order from (0, 0)) in rows
 *             k (L-1) + offsets_host[k] .. + path_len[k] - 1 (each cycle owns
 *             L + N_k - 1 rows, the longest possible path; rows past
 *             path_len[k] are left untouched).  Squared cost only.
 *   ws        workspace of wts_workspace_bytes(WTS_OP_ALIGN[_PATHS]) bytes */
wts_status wts_dtw_align(const wts_plan* plan, const double* bary, const void* cycles,
                         double* dist, int64_t* path_len, int32_t* paths, void* ws,
                         size_t ws_bytes, void* stream);

/* One DBA update.  With pi_k the optimal path of (B, C_k):
 *   S_l = sum_{k ascending} w_k * sum_{j: (l, j) in pi_k, descending j} y_kj
 *   C_l = sum_{k ascending} w_k * |{j: (l, j) in pi_k}|
 *   bary_out_l = S_l / C_l,   counts_l = sum_k |{j: (l, j) in pi_k}|
 * (sums start from +0.0, left to right).  weights [n] float64 or NULL (all 1).
 * bary_out [L][d] float64, counts [L] int64, dist [n] float64 or NULL
 * (DTW(B, C_k) of the input barycenter).  bary_out must not alias bary_in. */
wts_status wts_dba_iterate(const wts_plan* plan, const double* bary_in, const void* cycles,
                           const double* weights, double* bary_out, int64_t* counts,
                           double* dist, void* ws, size_t ws_bytes, void* stream);

/* Eq. 8: score_k = DTW(B, C_k) / |pi_k| (plan cost).  score [n] float64;
 * dist [n] float64 and path_len [n] int64 may be NULL. */
wts_status wts_anomaly_score(const wts_plan* plan, const double* bary, const void* cycles,
                             double* score, double* dist, int64_t* path_len, void* ws,
                             size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops such as online scoring of new cycles, harnesses that forbid
 * hipMalloc): wts_anomaly_score with the library's own scratch as the
 * workspace -- a static device array of 32 MiB that each GPU the library
 * runs on holds until the process ends (its address on a GPU is resolved by
 * wts_plan_create on that GPU).  Arguments, results and errors are those of
 * wts_anomaly_score; WTS_E_CAPACITY when the plan's score workspace
 * (wts_workspace_bytes(plan, WTS_OP_SCORE)) exceeds 32 MiB.  It calls no
 * allocating routine.  Every call on one GPU uses that GPU's one scratch:
 * calls that overlap on a GPU (two streams, two host threads) race and give
 * undefined results; the scratch keeps the last call's contents, and each
 * call clears what must start at zero. */
wts_status wts_anomaly_score_noalloc(const wts_plan* plan, const double* bary, const void* cycles,
                                     double* score, double* dist, int64_t* path_len,
                                     void* stream);

/* Sec. III-B, Eq. 2: Sub-DTW of the reference X (the plan's L rows, float64
 * [L][d], passed where the other calls take the barycenter) against every
 * window C_k of the batch: the minimum over alignment paths that cover all
 * rows of X and any run of columns of C_k,
 *   value_k = min_{a <= b} DTW(X, C_k[a..b])   (squared cost only),
 * b*_k = the lowest column of C_k where the last row of X reaches that
 * minimum, a*_k = the column at which the optimal path ending there (the
 * diag > up > left backtrack) enters the first row.  value [n] float64,
 * a_star / b_star [n] int64 (0-based columns of window k).  Plans created
 * with cost WTS_COST_EUCLID return WTS_E_UNSUPPORTED.  ws: workspace of
 * wts_workspace_bytes(WTS_OP_SUBDTW) bytes. */
wts_status wts_subdtw(const wts_plan* plan, const double* x, const void* windows, double* value,
                      int64_t* a_star, int64_t* b_star, void* ws, size_t ws_bytes, void* stream);

/* Eq. 3-5 with gamma > 0: value_k = Soft-DTW^gamma(B, C_k) (squared cost).
 * ckpt: checkpoint buffer of wts_workspace_bytes(WTS_OP_SOFT_FWD) bytes that
 * wts_softdtw_backward consumes (the forward must precede the backward with
 * the same bary, cycles and gamma). */
wts_status wts_softdtw_forward(const wts_plan* plan, const double* bary, const void* cycles,
                               double gamma, double* value, void* ckpt, size_t ckpt_bytes,
                               void* stream);

/* Eq. 6-7: grad_bary = sum_{k ascending} grad_value_k * d Soft-DTW^gamma(B, C_k) / d B,
 * with E from the chain rule on Eq. 5 (E(L, N) = 1 and zero outside the grid).
 * grad_value [n] float64 (the upstream gradient, e.g. lambda_k / m_k for Eq. 7;
 * NULL = all 1); grad_bary [L][d] float64 out; row_mass [L] float64 out or
 * NULL: row_mass_l = sum_k grad_value_k * sum_j E^k_{lj}.
 * accumulate = 0: the sums start from 0 (grad_bary and row_mass are
 * overwritten); accumulate = 1: they start from the values already in
 * grad_bary and row_mass.  A batch split into consecutive cycle groups (one
 * plan each, for instance so that each group's checkpoints fit in memory),
 * run in order with accumulate = 1 after the first group, gives bitwise the
 * result of one call over the whole batch: the same additions in the same
 * order.  WTS_E_ARG also for accumulate not 0 or 1. */
wts_status wts_softdtw_backward(const wts_plan* plan, const double* bary, const void* cycles,
                                double gamma, const void* ckpt, size_t ckpt_bytes,
                                const double* grad_value, double* grad_bary, double* row_mass,
                                int32_t accumulate, void* ws, size_t ws_bytes, void* stream);

/* Eq. 6 for the other argument: the gradient of sum_k w_k Soft-DTW^gamma(B, C_k)
 * with respect to the cycle values,
 *   d/dc_kj = w_k sum_i e_ij 2 (c_kj - b_i),
 * computed as the row gradient of Soft-DTW(C_k, B) (the measure is symmetric in
 * its two series, and so is the plan's band): one forward and one backward
 * sweep with the cycles on the rows.  cycles64: the cycle values as float64
 * [sum N][d]; grad_value [n] float64 or NULL (all 1); grad_cycles [sum N][d]
 * float64, overwritten.  ws: workspace of wts_workspace_bytes(WTS_OP_SOFT_GRAD_C)
 * bytes (it holds this call's own checkpoints; no wts_softdtw_forward is
 * needed first).  WTS_E_ARG for a null pointer, a ws not 256-byte aligned, gamma
 * not finite and > 0, or a plan created with L = 0; WTS_E_WORKSPACE for a short ws. */
wts_status wts_softdtw_grad_cycles(const wts_plan* plan, const double* bary, const double* cycles64,
                                   double gamma, const double* grad_value, double* grad_cycles,
                                   void* ws, size_t ws_bytes, void* stream);

/* One step of the gradient descent that approximates the Soft-DTW barycenter
 * of Eq. 7 (Sec. III-C computes it by gradient descent):
 *   bary_l <- bary_l - eta * grad_l / (2 row_mass_l)
 * using the gradient and row mass of wts_softdtw_backward (eta = 1 gives the
 * soft-DBA average sum_j E_lj y_j / sum_j E_lj).  bary [L][d] float64 updated
 * in place; grad [L][d], row_mass [L] float64.  No plan needed. */
wts_status wts_precond_step(double* bary, const double* grad, const double* row_mass, int64_t L,
                            int32_t d, double eta, void* stream);

/* Eq. 7 objective of a batch: out = sum_{k ascending} weights_k value_k (weights
 * NULL = all 1), for instance the Soft-DTW values of wts_softdtw_forward
 * with weights lambda_k / m_k.  accumulate = 1 adds to the value already in
 * out (cycle groups, as for wts_softdtw_backward).  values [n], weights [n]
 * float64, out [1] float64.  No plan needed.  WTS_E_ARG for a null values or
 * out, or accumulate not 0 or 1; WTS_E_SHAPE for n < 1. */
wts_status wts_barycenter_objective(const double* values, const double* weights, int32_t n,
                                    int32_t accumulate, double* out, void* stream);

/* Medoid initialisation (the workload recipes' barycenter init for DTW
 * barycenter averaging; the paper itself starts the Soft-DTW barycenter from
 * the Euclidean mean): D[k][i] = DTW(C_k, C_i) (squared cost, D[k][k] = 0),
 * total_k = sum_{i ascending} D[k][i], medoid = argmin_k total_k (lowest k on
 * ties).  dist_matrix [n][n] float64 or NULL, totals [n] float64 or NULL,
 * medoid [1] int32 out. */
wts_status wts_medoid(const wts_plan* plan, const void* cycles, double* dist_matrix,
                      double* totals, int32_t* medoid, void* ws, size_t ws_bytes, void* stream);

/* Barycenter initialisation into bary_out [L][d] float64 (plan L > 0):
 *   WTS_INIT_EUCLID_MEAN: pad every cycle with its last sample to the longest
 *     length Nmax (Sec. IV-A pads cycles this way), average per index
 *     (ascending k, then / n), resample to L: the "Euclidean barycenter"
 *     Table I starts from (Sec. V-D finds it the best start);
 *   WTS_INIT_NEAREST: the cycle whose length is closest to L (lowest k on
 *     ties), resampled to L (a choice of the workload recipes, not the
 *     paper's);
 *   WTS_INIT_COPY: cycle `index` resampled to L (a copy when its length is L).
 * Resampling: t_l = l (N-1) / (L-1), value = y[a] + f (y[a+1] - y[a]) with
 * a = floor(t_l), f = t_l - a.  chosen_host: HOST int32 out (the cycle used,
 * -1 for the mean) or NULL. */
wts_status wts_init_barycenter(const wts_plan* plan, const void* cycles, int32_t kind,
                               int32_t index, double* bary_out, int32_t* chosen_host,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WETSAND_MI_H */
