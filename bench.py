#!/usr/bin/env python3
"""Benchmark of the WETSAND hot path on one MI355X.

Headline workload: 256 cycles x 6 channels, float32, lengths 40,000..50,000
with 1 % of the samples dropped in gaps of 1..50 (the irregular workload the
paper's robots produce: missing samples are dropped, Sec. III-A), barycenter
of L = max N = 49,454 rows, nearest-length initialisation.  One step is one
barycenter iteration of the paper's prototype computation on all cycles:

  * one DTW barycenter averaging (DBA) iteration: DTW of every cycle against
    the barycenter with argmin codes, path backtrack, accumulate-and-average;
  * one Soft-DTW refinement step (gamma 0.1, Eq. 7 weights 1/m_k) on the DBA
    result: forward with checkpoints and E-matrix backward over cycle groups
    whose checkpoints fit in HBM, then the preconditioned update.

The whole step (every kernel of both halves) is captured once in a HIP graph
and replayed; inputs are resident in HBM before timing starts.

Metric: DTW cell updates per second (GCUPS): cells = L * sum_k N_k per
dynamic-programming pass, one pass for DBA and two (forward + backward) for
the Soft-DTW step; recomputation inside the backward is time, not cells.
Also reported: seconds per barycenter iteration, the roofline of the dominant
sweep kernel against the VALU lane-op peak with the algorithmic op floors
(tau, the cost of a transcendental in add slots, measured live by a
microbenchmark), the FP64 CPU oracle on a bounded sample, and extra sections
on the other workloads (64 x 4-6k DBA + scores with the medoid; 512 x 1-20k
graph-replayed DBA; 128 x 20k Soft-DTW descent, finite-difference check and
L-BFGS; segmentation of robot-scale streams).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# gfx950 (MI355X): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz; FP64 add/mul/fma/min
# issue at one per lane per clock (78.6 TFLOP/s FP64 vector counts an FMA as 2).
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9          # 39.32e12 lane-ops/s
# float32 and 32-bit integer VALU operations issue at twice that rate (157.3
# TFLOP/s FP32 vector counts an FMA as 2): the peak of the float32-decision sweeps
VALU_LANE_OPS_PEAK_F32 = 2 * VALU_LANE_OPS_PEAK  # 78.64e12 lane-ops/s
HBM_PEAK_GBS = 8000.0


# ------------------------------------------------------------ op floors
# Algorithmic VALU operations per DP cell (add/sub/mul/fma/min/cmp/select/cvt
# count 1, a transcendental counts tau; loads, LDS and cross-lane moves are
# not counted, and neither is recomputation).

def c_dba(d: int) -> int:
    """DTW with a 2-bit argmin code per cell (the DBA path sweep): the value
    recursion (d subtractions, 1 multiply, d-1 FMAs, 2 minima, 1 add) plus
    the two comparisons that decide the code."""
    return 2 * d + 5


def c_score(d: int) -> int:
    """DTW value carrying the path length (scores): the value recursion, two
    comparisons and the carried length's update."""
    return 2 * d + 6


def c_medoid(d: int) -> int:
    """DTW value only (all pairs of the medoid): the value recursion; no path
    length and no code are needed for the medoid's totals."""
    return 2 * d + 3


def c_sub(d: int) -> int:
    """Sub-DTW sweep: the value recursion and the two comparisons that decide
    which start column a cell inherits (as the DBA sweep decides its code)."""
    return 2 * d + 5


def c_soft_fwd(d: int, tau: float) -> float:
    """Soft-DTW forward: cost (2d), three shifted differences, their
    exponentials (3 tau) and sum, the logarithm (tau), min of three, scaling
    and conversions: 2d + 13 + 4 tau."""
    return 2 * d + 13 + 4 * tau


def c_soft_bwd(d: int, tau: float) -> float:
    """Soft-DTW backward: the three soft-min weights of the cell (3 tau and
    their arguments), the E recursion (3 products, 2 sums), the gradient sums
    (d FMAs + 1) and the cost terms it needs: 3d + 11 + 3 tau.  The
    replayed forward of the checkpointed tiles is recomputation, not counted."""
    return 3 * d + 11 + 3 * tau


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("wts_sweep.h", "wts_dtw.hip", "wts_dtw32.hip", "wts_soft.hip", "wts_device.h"):
        with open(os.path.join(ROOT, "paper_2404_12134_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNELS = {   # sweep -> rocprofv3 kernel name ({rho}: rows per lane of the plan;
              # {mode}: the path sweep's mode, 2 without entry tags, 4 with them)
    "medoid": "void wts::(anonymous namespace)::dtw_fwd_kernel<float, float, double, 3, {rho}, 0, false>",
    "dba": "void wts::(anonymous namespace)::dtw_fwd_kernel<double, float, double, 3, {rho}, {mode}, false>",
    "score": "void wts::(anonymous namespace)::dtw_fwd_kernel<double, float, double, 3, {rho}, 1, false>",
    "c5_dba": "void wts::(anonymous namespace)::dtw_fwd_kernel<double, float, double, 6, {rho}, {mode}, false>",
    "c5_soft_fwd": "void wts::(anonymous namespace)::soft_fwd_kernel<float, 6, {rho}, false>",
    "c5_soft_bwd": "void wts::(anonymous namespace)::soft_bwd_kernel<float, 6, {rho}, false>",
}


def traffic_from_profiles(kernel: str, name: str = None):
    """HBM bytes per launch measured with rocprofv3 PMC counters, if the
    committed measurement was taken on the current kernel source (and, when
    `name` is given, on that kernel instance)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p)).get(kernel)
    except Exception:
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    inst = rec.get("instances", {})
    if name is None:
        name = rec.get("kernel", "").replace("void ", "")
    hit = inst.get("void " + name) or inst.get(name)
    return None if hit is None else hit.get("bytes_per_launch")


def ingest_traffic(root: str):
    """Reads rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE passes (CSV) found under
    `root` and writes profiles/traffic.json: HBM bytes per launch of every sweep
    kernel, scaled by what the same counters read for the 1 GiB copy of
    `bench.py --only copy` (bytes_read / FETCH_SIZE_KiB, and the same for
    writes), tagged with the current kernel source hash.  Each pass lives in a
    directory named <phase>_<counter>, so launches of one kernel instance on
    different workloads are told apart by the phase that ran them."""
    import csv
    import glob
    hashes = set()
    used = {}              # sweep key -> the kernel instance its phase ran
    last = {}              # kernel instance -> count of its final dispatches that count
    for f in glob.glob(os.path.join(root, "**", "*.out"), recursive=True):
        for line in open(f, errors="replace"):
            if line.startswith("{") and '"phase"' in line:
                rec = json.loads(line)
                hashes.add(rec.get("source_hash"))
                for k, v in (rec.get("kernels") or {}).items():
                    used[k] = v
                for k, v in (rec.get("last_dispatches") or {}).items():
                    if k in (rec.get("kernels") or {}):
                        last[rec["kernels"][k].replace("void ", "")] = v
    if hashes != {kernel_source_hash()}:
        raise SystemExit("counter passes under %s ran kernel sources %s, not the current %s"
                         % (root, sorted(map(str, hashes)), kernel_source_hash()))
    per_dispatch = {}      # counters come in several rows per dispatch: sum them
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        phase = os.path.relpath(f, root).split(os.sep)[0].split("_")[0]
        for r in csv.DictReader(open(f)):
            key = (phase, r["Kernel_Name"], r["Counter_Name"], f, int(r["Dispatch_Id"]))
            per_dispatch[key] = per_dispatch.get(key, 0.0) + float(r["Counter_Value"])
    # a phase that tunes first (the sweep-shape candidates run the same kernel
    # instances) names how many of each kernel's final dispatches are its own
    if last:
        keep = {}
        for (phase, kn, cname, f, dsp), v in per_dispatch.items():
            keep.setdefault((phase, kn.split("(wts::")[0], cname, f), []).append((dsp, v))
        per_dispatch = {}
        for (phase, kn, cname, f), lst in keep.items():
            lst.sort()
            n_last = last.get(kn.replace("void ", ""))
            if n_last:
                lst = lst[-n_last:]
            for dsp, v in lst:
                per_dispatch[(phase, kn, cname, f, dsp)] = v
    vals = {}
    for (phase, kn, cname, _, _), v in per_dispatch.items():
        vals.setdefault((phase, kn.split("(wts::")[0], cname), []).append(v)
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    gib = float(1 << 30)
    f_cal = max(v for k, vs in vals.items() if "copyBuffer" in k[1] and k[2] == "FETCH_SIZE"
                for v in vs)
    w_cal = max(v for k, vs in vals.items() if "copyBuffer" in k[1] and k[2] == "WRITE_SIZE"
                for v in vs)
    f_scale, w_scale = gib / f_cal, gib / w_cal        # bytes per counted KiB
    out = {"_calibration": {"copy_bytes": int(gib), "fetch_kib": f_cal, "write_kib": w_cal,
                            "fetch_scale": f_scale, "write_scale": w_scale}}
    for key, pattern in KERNELS.items():
        phase = "c5" if key.startswith("c5") else key
        pre = _pattern_re(pattern)
        inst = {}
        for (ph, kn, cname), v in avg.items():
            if ph != phase or not pre.match(kn):
                continue
            if cname not in ("FETCH_SIZE", "WRITE_SIZE"):
                continue
            rec = inst.setdefault(kn, {})
            rec["fetch_bytes" if cname == "FETCH_SIZE" else "write_bytes"] = v * (
                f_scale if cname == "FETCH_SIZE" else w_scale)
        inst = {k: dict(v, bytes_per_launch=v["fetch_bytes"] + v["write_bytes"])
                for k, v in inst.items() if "fetch_bytes" in v and "write_bytes" in v}
        if inst:
            out[key] = {"kernel": used.get(key, sorted(inst)[0]),
                        "source_hash": kernel_source_hash(), "instances": inst}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    # issued VALU instructions per cell (SQ_INSTS_VALU counts wave
    # instructions: x 64 lanes / cells), from a pass over one iteration of
    # the headline ('c5' phase, --steps 1): the launches of one kernel cover
    # one DP pass together
    # the backward sweeps only its non-zero tiles: its cells are the swept share
    cells = {}
    swept = 1.0
    for f in glob.glob(os.path.join(root, "**", "*.out"), recursive=True):
        for line in open(f, errors="replace"):
            if line.startswith("{") and '"phase": "c5"' in line:
                rec = json.loads(line)
                cells["c5"] = rec["cells_per_pass"]
                swept = rec.get("bwd_tiles_swept_frac", swept)
    per_cell = {}
    if "c5" in cells:
        tot = {}
        for (phase, kn, cname, _, _), v in per_dispatch.items():
            if phase == "c5" and cname == "SQ_INSTS_VALU":
                tot[kn.split("(wts::")[0]] = tot.get(kn.split("(wts::")[0], 0.0) + v
        for key, pattern in KERNELS.items():
            if not key.startswith("c5"):
                continue
            pre = _pattern_re(pattern)
            for kn, v in tot.items():
                if pre.match(kn):
                    c = cells["c5"] * (swept if key == "c5_soft_bwd" else 1.0)
                    per_cell[key] = {"kernel": kn.replace("void ", ""),
                                     "per_cell": round(v * 64 / c, 2)}
    if per_cell:
        rec = {"source_hash": kernel_source_hash(), "per_cell": per_cell,
               "bwd_tiles_swept_frac": swept,
               "note": "SQ_INSTS_VALU x 64 / cells of one pass, headline workload (the "
                       "backward: the cells of the tiles it swept)"}
        with open(os.path.join(ROOT, "profiles", "valu_issued.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))


def progress(msg: str):
    """A progress line on stderr (long phases print one every so often)."""
    print("[bench %s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


def guarded(fn, *a, **kw):
    """Runs an optional section; an error is reported in its record instead of
    ending the run before the JSON line.  Device memory is released after it."""
    import torch
    try:
        return fn(*a, **kw)
    except Exception as exc:   # noqa: BLE001 -- reported, not hidden
        print("section %s failed: %r" % (fn.__name__, exc), file=sys.stderr)
        return {"error": repr(exc)}
    finally:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


# ------------------------------------------------------------ VALU rates

UBENCH_NAMES = ["add_f64", "fma_f64", "exp_log_f32", "add_f32", "cvt_f64_f32", "rcp_f64"]


def valu_rates(reps: int = 5):
    """Issue rates of single VALU instruction kinds (libwts_ubench.so: eight
    independent chains per lane, 32 resident waves per CU), in lane-ops/s,
    and tau = add_f64 rate / transcendental rate."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2404_12134_amd", "libwts_ubench.so"))
    lib.wts_ubench_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    blocks, iters = 256 * 8, 4096
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    chains = lib.wts_ubench_chains()
    rates = {}
    for op, name in enumerate(UBENCH_NAMES):
        ms = ctypes.c_double(0.0)
        if lib.wts_ubench_run(op, ctypes.c_void_p(out.data_ptr()), blocks, iters, reps,
                              ctypes.byref(ms)) != 0:
            raise RuntimeError("microbenchmark %s failed" % name)
        lane_ops = blocks * 256 * iters * chains * lib.wts_ubench_ops_per_step(op)
        rates[name] = {"ms": round(ms.value, 4), "lane_ops_per_s": lane_ops / (ms.value * 1e-3)}
    tau_meas = rates["add_f64"]["lane_ops_per_s"] / rates["exp_log_f32"]["lane_ops_per_s"]
    return {"rates": {k: {"ms": v["ms"], "T_lane_ops_per_s": round(v["lane_ops_per_s"] / 1e12, 3),
                          "frac_of_peak": round(v["lane_ops_per_s"] / VALU_LANE_OPS_PEAK, 3)}
                      for k, v in rates.items()},
            "tau_measured": round(tau_meas, 3), "tau": max(1, int(round(tau_meas))),
            "setup": "%d workgroups x 256 threads, %d steps x %d chains per lane"
                     % (blocks, iters, chains)}


# ------------------------------------------------------------ CPU baselines

def cpu_baseline_c5(w, B, gamma: float, n_sample: int = 16, rows: int = 3072, seed: int = 5):
    """The FP64 oracle (as it stands) on a bounded sample of the headline
    workload: n_sample seeded cycles (full length) against the first `rows`
    rows of the barycenter, one DBA iteration and one Soft-DTW forward +
    backward (the oracle keeps square-root checkpoints of R), OpenMP across
    the cycles.  Cells count as in the metric (DBA 1 pass, Soft-DTW 2)."""
    import numpy as np
    import oracle
    r = np.random.Generator(np.random.PCG64(seed))
    pick = np.sort(r.choice(w.n, size=n_sample, replace=False))
    cyc = [np.asarray(w.cycles[k], dtype=np.float64) for k in pick]
    Bs = np.ascontiguousarray(B[:rows])
    wv = 1.0 / w.lengths[pick].astype(np.float64)
    t0 = time.perf_counter()
    oracle.dba_iterate(Bs, cyc)
    t1 = time.perf_counter()
    oracle.softdtw_batch(Bs, cyc, gamma, wv)
    t2 = time.perf_counter()
    cells = rows * int(sum(c.shape[0] for c in cyc))
    return {"value": round(3 * cells / (t2 - t0) / 1e9, 4), "unit": "GCUPS",
            "cores": oracle.num_threads(), "kind": "oracle", "seconds": round(t2 - t0, 3),
            "dba_gcups": round(cells / (t1 - t0) / 1e9, 4),
            "soft_fwd_bwd_gcups": round(2 * cells / (t2 - t1) / 1e9, 4),
            "sample": "%d seeded cycles of the workload (full length) against the first %d "
                      "barycenter rows: one DBA iteration + one Soft-DTW gamma=%g forward and "
                      "backward, %d cells per pass, rate extrapolated linearly in cells"
                      % (n_sample, rows, gamma, cells)}


def cpu_baseline_c2(w, n_sample: int = 40):
    """The FP64 oracle on the first n_sample cycles of the 64-cycle workload:
    all-pairs medoid, one DBA iteration from it and the scores."""
    import numpy as np
    import oracle
    cyc = [np.asarray(c, dtype=np.float64) for c in w.cycles[:n_sample]]
    lens = np.array([c.shape[0] for c in cyc], dtype=np.int64)
    t0 = time.perf_counter()
    k, _ = oracle.medoid(cyc)
    B = cyc[k]
    Bn, _, _, _ = oracle.dba_iterate(B, cyc)
    oracle.score_batch(Bn, cyc)
    dt = time.perf_counter() - t0
    n = len(cyc)
    cells = int(sum(int(lens[a]) * int(lens[b]) for a in range(n) for b in range(n) if a != b))
    cells += 2 * int(B.shape[0]) * int(lens.sum())
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": "first %d of %d cycles: all-pairs medoid (both orders, as the oracle "
                      "computes them), 1 DBA iteration, scores; %d cells" % (n, w.n, cells)}


# ------------------------------------------------------------ helpers

def band_cells(L: int, lengths, w: float) -> int:
    """Cells inside the Sakoe-Chiba band of every (L x N) pair (the band the
    Soft-DTW kernels apply for bandwidth w), counted row by row."""
    import numpy as np
    tot = 0
    for N in np.asarray(lengths, dtype=np.int64):
        N = int(N)
        if w <= 0 or L == 1 or N == 1:
            tot += L * N
            continue
        a, b = L - 1, N - 1
        mn, mx = min(a, b), max(a, b)
        R = max(int(np.ceil(w * max(L, N))), -(-mx // mn))
        B = R * mn
        i = np.arange(L, dtype=np.int64)
        lo = np.maximum(-((B - i * b) // a), 0)
        hi = np.minimum((i * b + B) // a, N - 1)
        tot += int((hi - lo + 1).sum())
    return tot


def kname(key: str, rho: int, mode: int = 2) -> str:
    return KERNELS[key].format(rho=rho, mode=mode).replace("void ", "")


def path_mode(plan) -> int:
    """The sweep mode of a barycenter plan's path sweep: 2 (codes only) when
    it recovers paths pair by pair, 4 (with entry tags) strip by strip."""
    return 2 if plan.walk() == "pairs" else 4


def _pattern_re(pattern: str):
    import re
    return re.compile(re.escape(pattern).replace(r"\{rho\}", r"\d+").replace(r"\{mode\}", r"\d+")
                      + "$")


def issued_per_cell(key: str, name: str):
    """Issued VALU instructions per cell of one sweep kernel instance
    (rocprofv3 SQ_INSTS_VALU / cells), from the committed counter summary, if
    it was taken on the current kernel source and on that instance."""
    p = os.path.join(ROOT, "profiles", "valu_issued.json")
    try:
        rec = json.load(open(p))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    hit = rec.get("per_cell", {}).get(key)
    if not isinstance(hit, dict) or hit.get("kernel") != name.replace("void ", ""):
        return None
    return hit.get("per_cell")


def roofline(key: str, rho: int, ops: float, seconds: float, launches: int, cells: float,
             ops_per_cell: float, name: str = None):
    """Roofline record of one sweep kernel: `ops` algorithmic lane-ops over
    `launches` launches taking `seconds` in total (HIP events around each
    launch, on its stream)."""
    name = name or kname(key, rho)
    achieved = ops / seconds / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    tr = traffic_from_profiles(key, name)
    rec = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
           "peak": round(peak, 3), "unit": "TOP/s", "frac": round(achieved / peak, 4),
           "traffic": None if tr is None else round(tr, 1), "ops_per_cell": ops_per_cell,
           "cells_per_launch": int(cells / launches),
           "launch_ms": round(seconds / launches * 1e3, 3)}
    iss = issued_per_cell(key, name)
    if iss is not None:
        rec["issued_valu_per_cell"] = iss
    return rec


# ------------------------------------------------------------ headline

class BarycenterIteration:
    """One barycenter iteration of the headline: a DBA iteration A -> D, then
    a Soft-DTW descent step on D (in place), then A <- D.  All buffers are
    allocated at construction (the DBA workspace and the Soft-DTW checkpoints
    share one arena: the two halves run one after the other on one stream),
    so run() allocates nothing and can be captured into a graph."""

    def __init__(self, wts, plan, groups, Y, off, B0, gamma, gv, eta, arena):
        import torch
        self.wts, self.plan = wts, plan
        self.Y = Y
        self.A = B0.clone()
        self.D = torch.empty_like(B0)
        self.counts = torch.empty(plan.L, dtype=torch.int64, device=B0.device)
        self.dist = torch.empty(plan.n, dtype=torch.float64, device=B0.device)
        self.soft = wts.SoftDescent(groups, Y, off, plan.L, plan.d, gamma, gv, eta, ckpt=arena)
        self.ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def run(self, mark: bool = False):
        wts = self.wts
        if mark:
            self.ev[0].record()
        wts.dba_iterate(self.plan, self.A, self.Y, bary_out=self.D, counts=self.counts,
                        dist=self.dist)
        if mark:
            self.ev[1].record()
        self.soft.step(self.D)
        self.A.copy_(self.D)
        if mark:
            self.ev[2].record()

    def halves_s(self):
        return (self.ev[0].elapsed_time(self.ev[1]) / 1e3,
                self.ev[1].elapsed_time(self.ev[2]) / 1e3)


def c5_setup(wts, dev, gamma: float = 0.1, max_group_gib: float = 215.0, tune: bool = False,
             tune_cache=None):
    """The headline's plans, arena and iteration.  tune=True first times the
    sweep shapes on the workload itself (DBA: 4 or 5 rows per lane x grid
    candidates; Soft-DTW: grid candidates on the first checkpoint group),
    every candidate using the arena as its workspace."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import autotune, synth
    w = synth.make(5)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, w.L)
    groups = wts.subset_plans(off, w.d, dt, w.L, int(max_group_gib * 2 ** 30))
    arena_bytes = max(plan.workspace_bytes(wts.OP_DBA), wts.SoftDescent.ckpt_bytes(groups))
    arena = wts.aligned_buffer(arena_bytes, dev)
    B0, _ = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    tuned = None
    if tune:
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        shapes = [(r, g) for r in (4, 5) for g in autotune.grid_candidates("dba", cus)]
        td = autotune.tune(off, w.d, dt, w.L, op="dba", cycles=Y, bary=B0, reps=1,
                           cache_path=tune_cache, shapes=shapes, workspace=arena)
        a, b, _ = groups[0]
        ts = autotune.tune(off[a:b + 1] - off[a], w.d, dt, w.L, op="soft",
                           cycles=Y[int(off[a]):int(off[b])], bary=B0, reps=1,
                           cache_path=tune_cache, workspace=arena)
        for _, _, gp in groups:
            gp.close()
        plan.close()
        plan = wts.Plan(off, w.d, dt, w.L, rho=td["rho"], grid=td["grid"])
        groups = wts.subset_plans(off, w.d, dt, w.L, int(max_group_gib * 2 ** 30),
                                  grid=ts["grid"])
        tuned = {"dba": {k: td[k] for k in ("rho", "grid", "table")},
                 "soft": {k: ts[k] for k in ("rho", "grid", "table")}}
    plan.set_workspace(wts.OP_DBA, arena)
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).to(dev)   # Eq. 7: lambda / m
    it = BarycenterIteration(wts, plan, groups, Y, off, B0, gamma, gv, 0.5, arena)
    it.tuned = tuned
    return w, Y, off, dt, plan, groups, arena, it


def c5_kernel_times(wts, it, groups):
    """One eager iteration with HIP events around every sweep launch (on the
    launch stream): (DBA path sweep s, [soft fwd s per group], [soft bwd s per
    group], DBA iteration s, Soft-DTW step s)."""
    import torch
    it.plan.enable_timing(4)
    for _, _, gp in groups:
        gp.enable_timing(4)
        gp.bwd_tiles()   # forget the counts of earlier iterations
    it.run(mark=True)
    torch.cuda.synchronize()
    dba_ms, _ = it.plan.sweep_ms(wts.OP_DBA)
    fwd = [gp.sweep_ms(wts.OP_SOFT_FWD)[0] / 1e3 for _, _, gp in groups]
    bwd = [gp.sweep_ms(wts.OP_SOFT_BWD)[0] / 1e3 for _, _, gp in groups]
    tiles = [gp.bwd_tiles() for _, _, gp in groups]
    it.plan.enable_timing(0)
    for _, _, gp in groups:
        gp.enable_timing(0)
    t_dba, t_soft = it.halves_s()
    swept = sum(t[0] for t in tiles) / max(1, sum(t[1] for t in tiles))
    return dba_ms / 1e3, fwd, bwd, t_dba, t_soft, swept


def c5_headline(wts, dev, steps: int, warmup: int, tau: float, gamma: float = 0.1,
                speedup: bool = True, cpu: bool = True, tune_cache=None, fp32: bool = True):
    import torch
    progress("headline: generating the 256-cycle workload, tuning the sweep shapes")
    w, Y, off, dt, plan, groups, arena, it = c5_setup(wts, dev, gamma, tune=True,
                                                      tune_cache=tune_cache)
    L, d = w.L, w.d
    cells = L * int(w.lengths.sum())
    progress("headline: %d Soft-DTW groups, arena %.1f GiB; capturing the iteration"
             % (len(groups), arena.numel() / 2 ** 30))
    # capture the whole iteration once (every allocation was made above)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        it.run()
    torch.cuda.current_stream(dev).wait_stream(s)
    torch.cuda.synchronize()

    for _ in range(warmup):
        graph.replay()
        torch.cuda.synchronize()
        progress("headline: warm-up iteration done")
    torch.cuda.synchronize()      # one GPU: the barrier of the multi-rank contract is a no-op
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress("headline: %d timed iterations, %.3f s each" % (steps, (t1 - t0) / steps))
    plan.check()
    for _, _, gp in groups:
        gp.check()
    sec = (t1 - t0) / steps
    counted = 3 * cells
    value = counted / sec / 1e9

    # per-kernel launch times: one eager iteration with HIP events per sweep
    dba_s, fwd, bwd, t_dba, t_soft, swept = c5_kernel_times(wts, it, groups)
    plan.check()
    # the backward sweeps only the tiles whose E entries are not all zero:
    # its algorithmic work is that of the swept share of the cells
    kern = {   # name: (seconds per step, launches, cells, floor, KERNELS key, rho, mode)
        "dba_path_sweep": (dba_s, 1, cells, c_dba(d), "c5_dba", plan.rho(wts.OP_DBA),
                           path_mode(plan)),
        "soft_fwd": (sum(fwd), len(groups), cells, c_soft_fwd(d, tau), "c5_soft_fwd", 2, 0),
        "soft_bwd": (sum(bwd), len(groups), cells * swept, c_soft_bwd(d, tau), "c5_soft_bwd", 2,
                     0),
    }
    dom = max(kern, key=lambda k: kern[k][0])
    ksec, kl, kcells, kc, kkey, krho, kmode = kern[dom]
    roof = roofline(kkey, krho, kcells * kc, ksec, kl, kcells, kc, name=kname(kkey, krho, kmode))
    roof["per_kernel_ms_per_step"] = {k: round(v[0] * 1e3, 2) for k, v in kern.items()}
    roof["per_kernel_alu_frac"] = {k: round(v[2] * v[3] / v[0] / VALU_LANE_OPS_PEAK, 4)
                                   for k, v in kern.items()}
    roof["per_kernel_issued_valu_per_cell"] = {k: issued_per_cell(v[4], kname(v[4], v[5], v[6]))
                                               for k, v in kern.items()}
    roof["dba_path_recovery"] = plan.walk()
    roof["ops_per_cell_floors"] = {k: v[3] for k, v in kern.items()}
    roof["step_alu_frac"] = round(sum(v[2] * v[3] for v in kern.values()) / sec /
                                  VALU_LANE_OPS_PEAK, 4)
    roof["soft_group_launch_ms"] = {"fwd": [round(x * 1e3, 2) for x in fwd],
                                    "bwd": [round(x * 1e3, 2) for x in bwd]}
    progress("headline: the Soft-DTW backward with every tile swept (dense_e)")
    skip_rec = dense_e_compare(wts, it, groups, off, d, dt, L, Y, gamma, swept)

    # the anomaly scores of all cycles (after the iterations)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wts.anomaly_score(plan, it.A, Y)
    torch.cuda.synchronize()
    e0.record()
    wts.anomaly_score(plan, it.A, Y)
    e1.record()
    torch.cuda.synchronize()
    plan.check()
    t_score = e0.elapsed_time(e1) / 1e3
    fp32_rec = None
    if fp32:
        progress("headline: the DBA iteration with float32 decisions")
        fp32_rec = fp32_dba_compare(wts, plan, off, d, dt, L, Y, it.A, arena, cells, sec, t_dba)
    speed = None
    if speedup:
        progress("headline: one-cycle-per-launch DBA comparison")
        speed = dba_per_cycle_speedup(wts, plan, off, d, dt, L, Y, it.A, sequential=True)
    Bhost = it.A.cpu().numpy()
    rec = {
        "value": round(value, 3), "ms_per_step": round(sec * 1e3, 3),
        "config": {"workload": w.name + ": one barycenter iteration per step = 1 DBA iteration "
                                        "+ 1 Soft-DTW gamma=%g descent step (forward + backward "
                                        "over %d checkpoint groups, eta 0.5, weights 1/m_k), the "
                                        "whole step one captured hipGraph" % (gamma, len(groups)),
                   "n": w.n, "d": d, "L": L, "cells_per_pass": cells,
                   "counted_cells_per_step": counted, "soft_groups": len(groups),
                   "arena_gib": round(arena.numel() / 2 ** 30, 1)},
        "s_per_iteration": round(sec, 4),
        "halves_s": {"dba_iteration": round(t_dba, 4), "soft_step": round(t_soft, 4)},
        "phase_gcups": {"dba": round(cells / t_dba / 1e9, 2),
                        "soft_fwd_bwd": round(2 * cells / t_soft / 1e9, 2)},
        "score_s": round(t_score, 4),
        "workload_s": round(w.dba_iters * t_dba + 10 * t_soft + t_score, 2),
        "roofline": roof,
        "autotune": it.tuned,
        "batched_vs_per_cycle": speed,
        "fp32_decisions": fp32_rec,
        "soft_bwd_zero_tiles": skip_rec,
    }
    del graph, it, arena
    for _, _, gp in groups:
        gp.close()
    plan.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if cpu:
        progress("headline: oracle on the CPU")
        rec["cpu_baseline"] = cpu_baseline_c5(w, Bhost, gamma)
    return rec


def dense_e_compare(wts, it, groups, off, d, dt, L, Y, gamma, swept):
    """The Soft-DTW backward of the first checkpoint group with the zero
    tiles skipped (the headline's plans) and with every tile swept (a plan
    with dense_e), on the same checkpoints: launch times and whether the
    gradients and row masses agree bit for bit."""
    import torch
    gp, Yg, gv, a, b = it.soft.parts[0]
    offs = off[a:b + 1] - off[a]
    B = it.A
    ck = it.soft.ckpt[:gp.workspace_bytes(wts.OP_SOFT_FWD)]
    wts.softdtw_forward(gp, B, Yg, gamma, ckpt=ck)
    grid = it.tuned["soft"]["grid"] if it.tuned else 0
    pdense = wts.Plan(offs, d, dt, L, grid=grid, dense_e=True)
    out = {}
    for lab, pl in (("skipped", gp), ("dense", pdense)):
        pl.enable_timing(4)
        pl.bwd_tiles()
        g_, m_ = wts.softdtw_backward(pl, B, Yg, gamma, ck, gv, with_mass=True)
        torch.cuda.synchronize()
        ms, nl = pl.sweep_ms(wts.OP_SOFT_BWD)
        sw, tot = pl.bwd_tiles()
        pl.enable_timing(0)
        pl.check()
        out[lab] = (g_.clone(), m_.clone(), ms / max(nl, 1), sw / max(tot, 1))
    pdense.close()
    same = bool(torch.equal(out["skipped"][0], out["dense"][0])
                and torch.equal(out["skipped"][1], out["dense"][1]))
    return {"tiles_swept_frac_step": round(swept, 5),
            "group_cycles": int(b - a),
            "launch_ms_skipped": round(out["skipped"][2], 2),
            "launch_ms_dense": round(out["dense"][2], 2),
            "tiles_swept_frac_group": round(out["skipped"][3], 5),
            "speedup": round(out["dense"][2] / out["skipped"][2], 2),
            "bitwise_equal_grad_and_mass": same}


# ------------------------------------------------------------ extra sections

def fp32_dba_compare(wts, plan, off, d, dt, L, Y, B, arena, cells, sec, t_dba):
    """The DBA iteration of the headline workload with float32 decisions
    (plan option decision = fp32; 4 and 5 rows per lane at three grids tried)
    against the
    float64 one on the same barycenter: sweep and iteration times, the path
    sweep's roofline against the float32 VALU peak, and how the results
    differ (distances, path lengths, counts, the new barycenter).  Both plans
    use the headline's arena as their DBA workspace, one after the other."""
    import numpy as np
    import torch
    n = len(off) - 1
    out64 = (torch.empty_like(B), torch.empty(L, dtype=torch.int64, device=B.device),
             torch.empty(n, dtype=torch.float64, device=B.device))
    out32 = tuple(torch.empty_like(t) for t in out64)
    wts.dba_iterate(plan, B, Y, bary_out=out64[0], counts=out64[1], dist=out64[2])
    sc64, d64, l64 = wts.anomaly_score(plan, B, Y)
    from paper_2404_12134_amd import autotune
    cus = torch.cuda.get_device_properties(B.device).multi_processor_count
    best = None
    tried = {}
    for rho, grid in [(r, g) for r in (4, 5) for g in autotune.grid_candidates("dba", cus)]:
        p32 = wts.Plan(off, d, dt, L, decision="fp32", rho=rho, grid=grid)
        p32.set_workspace(wts.OP_DBA, arena)
        wts.dba_iterate(p32, B, Y, bary_out=out32[0], counts=out32[1], dist=out32[2])
        torch.cuda.synchronize()
        p32.enable_timing(4)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wts.dba_iterate(p32, B, Y, bary_out=out32[0], counts=out32[1], dist=out32[2])
        e1.record()
        torch.cuda.synchronize()
        ms, nl = p32.sweep_ms(wts.OP_DBA)
        p32.check()
        tried[(rho, grid)] = (ms / nl / 1e3, e0.elapsed_time(e1) / 1e3)
        if best is None or tried[(rho, grid)][1] < tried[best][1]:
            best = (rho, grid)
        if best == (rho, grid):
            sc32, d32, l32 = wts.anomaly_score(p32, B, Y)
        p32.close()
    torch.cuda.synchronize()
    sweep_s, iter_s = tried[best]
    ops = cells * c_dba(d)
    ach = ops / sweep_s / 1e12
    peak = VALU_LANE_OPS_PEAK_F32 / 1e12
    d64h, d32h = out64[2].cpu().numpy(), out32[2].cpu().numpy()
    l64h, l32h = l64.cpu().numpy(), l32.cpu().numpy()
    B64, B32 = out64[0].cpu().numpy(), out32[0].cpu().numpy()
    return {
        "rows_per_lane": best[0], "grid": best[1],
        "candidates_s": [[k[0], k[1], round(v[0], 4), round(v[1], 4)] for k, v in tried.items()],
        "dba_iteration_s": round(iter_s, 4), "dba_gcups": round(cells / iter_s / 1e9, 2),
        "path_sweep": {"bound": "alu", "achieved": round(ach, 3), "peak": round(peak, 3),
                       "unit": "TOP/s", "frac": round(ach / peak, 4),
                       "launch_ms": round(sweep_s * 1e3, 3), "ops_per_cell": c_dba(d)},
        "fp64_dba_iteration_s": round(t_dba, 4),
        "s_per_iteration_with_fp32_dba": round(sec - t_dba + iter_s, 4),
        "vs_fp64": {
            "max_rel_dist_diff": float(np.max(np.abs(d32h - d64h) / np.maximum(d64h, 1e-300))),
            "cycles_with_other_path_length": int((l32h != l64h).sum()),
            "rows_with_other_count": int((out32[1] != out64[1]).sum().item()),
            "max_abs_bary_diff": float(np.max(np.abs(B32 - B64))),
            "max_rel_score_diff": float(np.max(np.abs(sc32.cpu().numpy() - sc64.cpu().numpy())
                                               / np.maximum(sc64.cpu().numpy(), 1e-300))),
        },
    }


def dba_per_cycle_speedup(wts, plan, off, d, dt, L, Y, B, sequential=False):
    """Batched vs one-cycle-per-launch DBA iteration: the same kernels, run
    once on the batched plan and once per cycle on a one-cycle plan.  With
    sequential=True the one-cycle plans are built, run and freed one at a
    time (for batches whose workspaces do not fit side by side) and their
    launch times, taken with HIP events, are summed; otherwise the n calls run
    back to back between two events.  Workspaces are allocated before timing."""
    import torch
    n = len(off) - 1
    Bo = torch.empty_like(B)
    counts = torch.empty(L, dtype=torch.int64, device=B.device)
    dist = torch.empty(n, dtype=torch.float64, device=B.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wts.dba_iterate(plan, B, Y, bary_out=Bo, counts=counts, dist=dist)
    torch.cuda.synchronize()
    e0.record()
    wts.dba_iterate(plan, B, Y, bary_out=Bo, counts=counts, dist=dist)
    e1.record()
    torch.cuda.synchronize()
    batched = e0.elapsed_time(e1) / 1e3
    Ys = [Y[int(off[k]):int(off[k + 1])] for k in range(n)]
    d1 = torch.empty(1, dtype=torch.float64, device=B.device)
    per = 0.0
    if sequential:
        for k in range(n):
            one = wts.Plan(off[k:k + 2] - off[k], d, dt, L)
            wts.dba_iterate(one, B, Ys[k], bary_out=Bo, counts=counts, dist=d1)
            e0.record()
            wts.dba_iterate(one, B, Ys[k], bary_out=Bo, counts=counts, dist=d1)
            e1.record()
            torch.cuda.synchronize()
            per += e0.elapsed_time(e1) / 1e3
            one.close()
    else:
        single = [wts.Plan(off[k:k + 2] - off[k], d, dt, L) for k in range(n)]
        for k in range(n):
            wts.dba_iterate(single[k], B, Ys[k], bary_out=Bo, counts=counts, dist=d1)
        torch.cuda.synchronize()
        e0.record()
        for k in range(n):
            wts.dba_iterate(single[k], B, Ys[k], bary_out=Bo, counts=counts, dist=d1)
        e1.record()
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / 1e3
        for one in single:
            one.close()
    plan.check()
    return {"op": "dba_iterate", "one_cycle_per_launch_s": round(per, 5),
            "batched_s": round(batched, 5), "speedup": round(per / batched, 2),
            "per_cycle_timing": "sum of per-launch events" if sequential else "back to back"}


def c2_section(wts, dev, steps: int = 3, speedup: bool = True):
    """64 x 3 ch, 4000..6000 (3 cycles with an injected drift): medoid
    initialisation (all 2016 pairs), 10 DBA iterations from the medoid, the
    anomaly scores, and detection of the drifted cycles (Sec. V-C
    thresholds)."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import autotune, detect, synth
    w = synth.make(2)
    lens = w.lengths
    Y, off, dt = wts.pack_cycles(w.cycles)
    mplan, mtuned = autotune.tuned_plan(off, w.d, dt, 0, op="medoid", cycles=Y, cache_path=None)
    k0 = int(wts.medoid(mplan, Y, with_matrix=False)[0].item())
    L = int(lens[k0])
    B0, _ = wts.init_barycenter(wts.Plan(off, w.d, dt, L), Y, wts.INIT_COPY, k0)
    plan, tuned = autotune.tuned_plan(off, w.d, dt, L, op="dba", cycles=Y, bary=B0,
                                      cache_path=None)
    n = w.n
    Ba = torch.empty((L, w.d), dtype=torch.float64, device=dev)
    Bb = torch.empty_like(Ba)
    counts = torch.empty(L, dtype=torch.int64, device=dev)
    dist = torch.empty(n, dtype=torch.float64, device=dev)
    cells_medoid = int(sum(int(lens[a]) * int(lens[b]) for a in range(n) for b in range(a + 1, n)))
    cells_bary = L * int(lens.sum())
    iters = w.dba_iters
    cells_step = cells_medoid + iters * cells_bary + cells_bary
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("medoid", "dba", "score")}
    times = {k: [] for k in ev}

    def step(record: bool):
        e = ev["medoid"]
        e[0].record()
        kk, _, _ = wts.medoid(mplan, Y, with_matrix=False)
        e[1].record()
        Bi, _ = wts.init_barycenter(plan, Y, wts.INIT_COPY, k0)
        Ba.copy_(Bi)
        src, dst = Ba, Bb
        ev["dba"][0].record()
        for _ in range(iters):
            wts.dba_iterate(plan, src, Y, bary_out=dst, counts=counts, dist=dist)
            src, dst = dst, src
        ev["dba"][1].record()
        ev["score"][0].record()
        out = wts.anomaly_score(plan, src, Y)
        ev["score"][1].record()
        if record:
            torch.cuda.synchronize()
            if int(kk.item()) != k0:
                raise RuntimeError("medoid changed between steps")
            for key, (a, b) in ev.items():
                times[key].append(a.elapsed_time(b) / 1e3)
        return out

    step(False)
    torch.cuda.synchronize()
    mplan.enable_timing(4 * steps)
    plan.enable_timing(16 * steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        last = step(True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    mplan.check()
    plan.check()
    t_med = float(np.mean(times["medoid"]))
    t_dba = float(np.mean(times["dba"])) / iters
    t_score = float(np.mean(times["score"]))
    sweeps = {"medoid": (mplan, wts.OP_MEDOID, cells_medoid, c_medoid(w.d)),
              "dba": (plan, wts.OP_DBA, cells_bary, c_dba(w.d)),
              "score": (plan, wts.OP_SCORE, cells_bary, c_score(w.d))}
    per = {}
    for key, (pl, op, cells, cm) in sweeps.items():
        tot, cnt = pl.sweep_ms(op)
        per[key] = roofline(key, pl.rho(op), cells * cm * cnt, tot / 1e3, cnt, cells * cnt, cm,
                            name=kname(key, pl.rho(op), path_mode(pl) if key == "dba" else 2))
        per[key]["ms_per_step"] = round(tot / steps, 3)
    mplan.enable_timing(0)
    plan.enable_timing(0)
    sc = last[0].cpu().numpy()
    truth = np.zeros(n, dtype=bool)
    truth[w.meta["drift"]] = True
    detection = {"drifted_cycles": [int(i) for i in w.meta["drift"]],
                 "top_scores": [int(i) for i in np.argsort(-sc)[:len(w.meta["drift"])]]}
    for name, thr in (("two_sigma", detect.two_sigma_threshold(sc)),
                      ("boxplot", detect.boxplot_threshold(sc))):
        tp, fn, fp, tn = detect.confusion(detect.flag(sc, thr), truth)
        detection[name] = {"threshold": round(thr, 6), "tp": tp, "fn": fn, "fp": fp, "tn": tn,
                           "f2": round(detect.f_beta(tp, fn, fp), 3)}
    speed = dba_per_cycle_speedup(wts, plan, off, w.d, dt, L, Y, Ba) if speedup else None
    return {"workload": w.name + ": medoid init + %d DBA iterations + anomaly scores" % iters,
            "n": n, "d": w.d, "L": L, "cells_per_step": cells_step,
            "gcups": round(cells_step / sec / 1e9, 2), "ms_per_step": round(sec * 1e3, 3),
            "s_per_dba_iteration": round(t_dba, 6),
            "phase_gcups": {"medoid": round(cells_medoid / t_med / 1e9, 2),
                            "dba_iteration": round(cells_bary / t_dba / 1e9, 2),
                            "score": round(cells_bary / t_score / 1e9, 2)},
            "sweeps": per,
            "autotune": {"dba": {"rows_per_lane": tuned["rho"], "grid": tuned["grid"],
                                 "candidates_ms": tuned["table"]},
                         "medoid": {"rows_per_lane": mtuned["rho"], "grid": mtuned["grid"],
                                    "candidates_ms": mtuned["table"]}},
            "batched_vs_per_cycle": speed, "detection": detection}


def c3_section(wts, dev, iters: int = 10, speedup: bool = True):
    """512 x 6 ch, lengths log-uniform 1000..20000, L = 10000, nearest-length
    init: `iters` DBA iterations replayed from a captured hipGraph (two
    iterations per graph), plus the path sweep's own launch time."""
    import torch
    from paper_2404_12134_amd import synth
    from paper_2404_12134_amd import autotune
    w = synth.make(3)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan0 = wts.Plan(off, w.d, dt, w.L)
    B0, _ = wts.init_barycenter(plan0, Y, wts.INIT_NEAREST)
    plan0.close()
    plan, tuned = autotune.tuned_plan(off, w.d, dt, w.L, op="dba", cycles=Y, bary=B0, reps=2,
                                      cache_path=None)
    cells = w.L * int(w.lengths.sum())
    plan.enable_timing(8)
    for _ in range(3):
        wts.dba_iterate(plan, B0, Y)
    torch.cuda.synchronize()
    plan.sweep_ms(wts.OP_DBA)
    for _ in range(3):
        wts.dba_iterate(plan, B0, Y)
    tot, cnt = plan.sweep_ms(wts.OP_DBA)
    plan.enable_timing(0)
    plan.check()
    runner = wts.DBARunner(plan, Y, B0, graph=True)
    runner.run(2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    runner.run(iters, check=False)
    e1.record()
    torch.cuda.synchronize()
    plan.check()
    it_s = e0.elapsed_time(e1) / 1e3 / iters
    del runner
    speed = dba_per_cycle_speedup(wts, plan, off, w.d, dt, w.L, Y, B0) if speedup else None
    cm = c_dba(w.d)
    rho = plan.rho(wts.OP_DBA)
    rf = roofline("c5_dba", rho, cells * cm * cnt, tot / 1e3, cnt, cells * cnt, cm,
                  name=kname("c5_dba", rho, path_mode(plan)))
    rf["path_recovery"] = plan.walk()
    rf["traffic"] = None          # the committed counters are those of the headline workload
    rf.pop("issued_valu_per_cell", None)
    return {"workload": w.name + ": %d DBA iterations replayed from a hipGraph, nearest-length "
                                 "init" % iters,
            "s_per_dba_iteration": round(it_s, 5), "gcups": round(cells / it_s / 1e9, 2),
            "cells_per_iteration": cells, "rows_per_lane": rho,
            "autotune": {k: tuned[k] for k in ("rho", "grid", "table")},
            "path_sweep": rf, "batched_vs_per_cycle": speed}


def c4_section(wts, dev, tau: float, steps: int = 50, lbfgs: bool = True):
    """128 x 6 ch, 18000..22000, L = 20000, Euclidean-mean init (Table I):
    for gamma in (0.1, 1): `steps` preconditioned Soft-DTW descent steps
    (eta 0.5, Eq. 7 weights 1/m_k) with the objective trajectory, and at
    step 0 a directional finite-difference check of the GPU gradient on the
    whole batch; the forward and backward launch times and their roofline;
    the gradient with respect to the cycles; the Table I band (0.6); and
    Table I's L-BFGS (gamma 1, 40 iterations, 200 evaluations at most)."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    from paper_2404_12134_amd import autotune
    w = synth.make(4)
    Y, off, dt = wts.pack_cycles(w.cycles)
    L, d = w.L, w.d
    plan0 = wts.Plan(off, d, dt, L)
    B0, _ = wts.init_barycenter(plan0, Y, wts.INIT_EUCLID_MEAN)
    plan0.close()
    plan, tuned = autotune.tuned_plan(off, d, dt, L, op="soft", cycles=Y, bary=B0, reps=1,
                                      cache_path=None)
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).to(dev)   # Eq. 7: lambda / m
    cells = L * int(w.lengths.sum())
    cf, cb = c_soft_fwd(d, tau), c_soft_bwd(d, tau)
    rec = {"workload": w.name + ": Soft-DTW barycenter, Euclidean-mean init, weights 1/m_k",
           "cells_per_pass": cells, "ops_per_cell": {"fwd": cf, "bwd": cb},
           "autotune": {k: tuned[k] for k in ("rho", "grid", "table")}}
    groups = [(0, w.n, plan)]
    for gamma in (0.1, 1.0):
        sd = wts.SoftDescent(groups, Y, off, L, d, gamma, gv, 0.5)
        B = B0.clone()
        # directional finite differences at step 0 on the whole batch:
        # (f(B + hV) - f(B - hV)) / 2h against <G, V> for V = G / |G| and a
        # seeded random unit direction; h moves f by about 1e-5 of itself
        v0, ck = wts.softdtw_forward(plan, B, Y, gamma)
        G = wts.softdtw_backward(plan, B, Y, gamma, ck, gv)
        del ck
        f0 = wts.barycenter_objective(v0, gv).item()
        g = G.cpu().numpy()
        r = np.random.Generator(np.random.PCG64(11))
        fd = {}
        for name, V in (("gradient_direction", g), ("random_direction",
                                                    r.standard_normal(g.shape))):
            V = V / np.linalg.norm(V)
            dd = float(np.sum(g * V))
            h = 1e-5 * abs(f0) / max(abs(dd), 1e-30)
            Vt = torch.from_numpy(V).to(dev)
            fp = wts.barycenter_objective(wts.softdtw_forward(plan, B + h * Vt, Y, gamma)[0],
                                          gv).item()
            fm = wts.barycenter_objective(wts.softdtw_forward(plan, B - h * Vt, Y, gamma)[0],
                                          gv).item()
            est = (fp - fm) / (2 * h)
            fd[name] = {"h": h, "directional_derivative": dd, "finite_difference": est,
                        "rel_err": abs(est - dd) / abs(dd)}
        plan.check()
        traj = torch.empty(steps, dtype=torch.float64, device=dev)
        sd.step(B)
        torch.cuda.synchronize()
        B.copy_(B0)
        plan.enable_timing(2 * steps)
        plan.bwd_tiles()
        t0 = time.perf_counter()
        for s in range(steps):
            sd.step(B)
            traj[s:s + 1].copy_(sd.objective)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        tf, nf = plan.sweep_ms(wts.OP_SOFT_FWD)
        tb, nb = plan.sweep_ms(wts.OP_SOFT_BWD)
        sw, tot = plan.bwd_tiles()
        swept = sw / max(tot, 1)
        plan.enable_timing(0)
        plan.check()
        tr = traj.cpu().numpy()
        # the backward's algorithmic work: the cells of the tiles it swept
        fwd = roofline("c5_soft_fwd", 2, cells * cf * nf, tf / 1e3, nf, cells * nf, cf)
        bwd = roofline("c5_soft_bwd", 2, cells * swept * cb * nb, tb / 1e3, nb,
                       cells * swept * nb, cb)
        bwd["tiles_swept_frac"] = round(swept, 5)
        for rf in (fwd, bwd):
            rf["traffic"] = None   # the committed counters are those of the headline workload
            rf.pop("issued_valu_per_cell", None)
        pair_s = (tf / nf + tb / nb) / 1e3
        rec["gamma_%g" % gamma] = {
            "steps": steps, "s_per_step": round(sec, 4),
            "gcups_fwd_bwd": round(2 * cells / sec / 1e9, 2),
            "objective_trajectory": {"step_%d" % k: round(float(tr[k]), 8)
                                     for k in sorted({0, 1, 9, 19, 29, 39, steps - 1})
                                     if k < steps},
            "objective_non_increasing": bool(np.all(np.diff(tr) <= 1e-12 * np.abs(tr[:-1]))),
            "fd_check_step0": fd,
            "forward": fwd, "backward": bwd,
            "alu_frac_fwd_bwd": round(cells * (cf + swept * cb) / pair_s / VALU_LANE_OPS_PEAK,
                                      4),
        }
        del sd
    # the gradient with respect to the cycles (gamma 0.1)
    Y64 = Y.to(torch.float64)
    wts.softdtw_grad_cycles(plan, B0, Y64, 0.1, gv)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    wts.softdtw_grad_cycles(plan, B0, Y64, 0.1, gv)
    e1.record()
    torch.cuda.synchronize()
    plan.check()
    tg = e0.elapsed_time(e1) / 1e3
    rec["grad_cycles"] = {"ms": round(1e3 * tg, 2),
                          "gcups_fwd_bwd": round(2 * cells / tg / 1e9, 2)}
    del Y64
    # the Table I band (0.6), gamma 0.1, its own tuned grid
    bplan, btuned = autotune.tuned_plan(off, d, dt, L, op="soft", cycles=Y, bary=B0, reps=1,
                                        cache_path=None, band=0.6)
    bcells = band_cells(L, w.lengths, 0.6)
    sdb = wts.SoftDescent([(0, w.n, bplan)], Y, off, L, d, 0.1, gv, 0.5)
    B = B0.clone()
    sdb.step(B)
    torch.cuda.synchronize()
    bplan.enable_timing(8)
    bplan.bwd_tiles()
    t0 = time.perf_counter()
    for _ in range(3):
        sdb.step(B)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / 3
    tf, nf = bplan.sweep_ms(wts.OP_SOFT_FWD)
    tb, nb = bplan.sweep_ms(wts.OP_SOFT_BWD)
    bsw, btot = bplan.bwd_tiles()
    bplan.enable_timing(0)
    bplan.check()
    rec["band_0.6"] = {"cells_in_band_per_pass": bcells,
                       "band_fraction": round(bcells / cells, 4), "s_per_step": round(sec, 4),
                       "gcups_fwd_bwd_in_band": round(2 * bcells / sec / 1e9, 2),
                       "forward_ms": round(tf / nf, 2), "backward_ms": round(tb / nb, 2),
                       "backward_tiles_swept_frac_of_band": round(bsw / max(btot, 1), 5),
                       "autotune": {k: btuned[k] for k in ("rho", "grid", "table")}}
    del sdb
    bplan.close()
    if lbfgs:
        # Table I: gamma 1, L-BFGS, max_iter 40, max_fun 200, gtol 1e-8, tol 1e-5
        wts.lbfgs_barycenter(plan, Y, B0, 1.0, gv, max_iter=1, max_eval=2)   # loads torch kernels
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist = wts.lbfgs_barycenter(plan, Y, B0, 1.0, gv, max_iter=40, max_eval=200)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        s_step = rec["gamma_1"]["s_per_step"]
        rec["lbfgs_table1"] = {"gamma": 1.0, "max_iter": 40, "max_eval": 200,
                               "evaluations": len(hist), "seconds": round(tl, 2),
                               "s_per_evaluation": round(tl / len(hist), 4),
                               "objective_first_last": [round(hist[0], 8), round(hist[-1], 8)],
                               "sweep_share": round(min(1.0, len(hist) * s_step / tl), 3)}
    plan.close()
    return rec


# The paper's Soft-DTW barycenter timings (its computation-time table,
# Sec. V-B): signals of 18,385 time steps, 5 / 10 / 25 training cycles, on a
# cloud instance with an NVIDIA A10G GPU and an 8-core AMD EPYC 7R32 (Sec. IV);
# minutes for its GPU implementation and for TSLearn's CPU one.
PAPER_SOFT_MINUTES = {5: (40.3, 777.0), 10: (64.0, 1217.0), 25: (128.0, 3933.0)}


def paper_table_section(wts, dev, length: int = 18385):
    """The workload of the paper's computation-time table, run on this path
    with the Table I settings: Soft-DTW barycenters (gamma 1, Sakoe-Chiba
    band 0.6, Euclidean-mean init, L-BFGS with at most 40 iterations and 200
    evaluations, weights 1/m_k) of 5, 10 and 25 seeded cycles of `length`
    samples, one univariate barycenter per joint for three joints (the
    first three channels of the 128-cycle workload's generator), timed end
    to end (they stop on the L-BFGS tolerances, so the time 200 evaluations
    per joint would take is given too); the paper's minutes on its hardware
    beside them as context, not as a baseline of the same run."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    out = {"length": length, "gamma": 1.0, "band": 0.6, "max_iter": 40, "max_eval": 200,
           "hardware_of_the_paper": "NVIDIA A10G + 8-core AMD EPYC 7R32 (TSLearn on the CPU)"}
    for n, (gpu_min, tsl_min) in PAPER_SOFT_MINUTES.items():
        w = synth.make(4, n=n, len_range=(length, length), L=length, seed=400 + n)
        total, evals = 0.0, []
        for c in range(3):
            cyc = [np.ascontiguousarray(x[:, c:c + 1]) for x in w.cycles]
            Y, off, dt = wts.pack_cycles(cyc)
            plan = wts.Plan(off, 1, dt, length, band=0.6)
            B0, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
            gv = torch.from_numpy(1.0 / np.asarray([x.shape[0] for x in cyc], np.float64)).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B, hist = wts.lbfgs_barycenter(plan, Y, B0, 1.0, gv)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            plan.check()
            evals.append(len(hist))
            plan.close()
        per_eval = total / sum(evals)
        # the run stops on its tolerances; the bound of 200 evaluations per
        # barycenter is the most the Table I settings allow
        at_max = 3 * 200 * per_eval
        out["cycles_%d" % n] = {
            "seconds_three_joints": round(total, 2), "evaluations_per_joint": evals,
            "s_per_evaluation": round(per_eval, 4),
            "seconds_at_200_evaluations_three_joints": round(at_max, 2),
            "paper_gpu_minutes": gpu_min, "paper_tslearn_minutes": tsl_min,
            "ratio_to_paper_gpu_at_200_evaluations": round(gpu_min * 60.0 / at_max, 1)}
        torch.cuda.empty_cache()
    return out


def segmentation_section(wts, dev, n_streams: int = 16, n_cycles: int = 37,
                         speedup: bool = True):
    """The segmentation step (Sec. III-B) at the scale the paper reports for
    its robot (Sec. V-A: a reference cycle of about 16,300 samples, streams
    of about 6e5 samples): a reference of 15,500..16,500 samples, 3 channels,
    float32 streams of `n_cycles` cycles each.  `n_streams` streams are
    segmented together (one Sub-DTW launch per round over their windows),
    then the same streams one at a time."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    lr = (15500, 16500)
    X, _, _ = synth.make_stream(500, 1, lr, 3, template_seed=31)
    streams = [synth.make_stream(600 + k, n_cycles, lr, 3, template_seed=31)[1]
               for k in range(n_streams)]
    M = X.shape[0]
    Xt = torch.from_numpy(X.astype(np.float64)).to(dev)
    St = [torch.from_numpy(np.ascontiguousarray(Y)).to(dev) for Y in streams]
    al = wts.segment_alpha(M)

    def cells_of(segs, N):
        # replay the window starts of the loop: cells = M x window length
        ws, tot = 0, 0
        for a, b, _ in segs:
            tot += M * (min(ws + 2 * M, N) - ws)
            bq = b - ws
            ws = ws + bq - al if bq - al > 0 else ws + bq + 1
        return tot

    wts.segment(Xt, St[:1], "f32")                # warm-up: code paths, allocator
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    segs = wts.segment(Xt, St, "f32")
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    cells = sum(cells_of(sg, Y.shape[0]) for sg, Y in zip(segs, streams))
    rounds = max(len(sg) for sg in segs)
    rec = {"workload": "segmentation: %d streams x %d cycles (3 ch f32, %d..%d samples per "
                       "cycle, ~%d samples per stream), reference of %d samples"
                       % (n_streams, n_cycles, lr[0], lr[1],
                          int(np.mean([Y.shape[0] for Y in streams])), M),
           "segments_per_stream": [len(sg) for sg in segs][:4], "rounds": rounds,
           "cells": cells, "batched_s": round(t_batch, 4),
           "gcups": round(cells / t_batch / 1e9, 2), "ops_per_cell": c_sub(3),
           "loop_alu_frac": round(cells * c_sub(3) / t_batch / VALU_LANE_OPS_PEAK, 4)}
    if speedup:
        t0 = time.perf_counter()
        one = [wts.segment(Xt, [y], "f32")[0] for y in St]
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t0
        if one != segs:
            raise RuntimeError("segmentation differs between batched and one-stream runs")
        rec["one_stream_per_launch_s"] = round(t_one, 4)
        rec["s_per_stream_alone"] = round(t_one / n_streams, 4)
        rec["speedup"] = round(t_one / t_batch, 2)
    return rec


# ------------------------------------------------------------ profiling phases

def only_phase(args, wts, dev):
    """One phase, --steps times, for rocprofv3 passes.  'copy' is a plain
    1 GiB device-to-device copy: the reference for scaling FETCH_SIZE /
    WRITE_SIZE to bytes.  'c5' runs the headline iteration eagerly."""
    import torch
    from paper_2404_12134_amd import synth
    if args.only == "copy":
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"phase": "copy", "bytes_read": a.numel() * 8,
                          "bytes_written": b.numel() * 8, "source_hash": kernel_source_hash()}))
        return
    if args.only == "valu":
        print(json.dumps({"phase": "valu", "source_hash": kernel_source_hash(),
                          "valu": valu_rates()}))
        return
    if args.only == "c5":
        w, Y, off, dt, plan, groups, arena, it = c5_setup(wts, dev, tune=True,
                                                          tune_cache=args.tune_cache)
        for _, _, gp in groups:
            gp.bwd_tiles()
        for _ in range(args.steps):
            it.run()
        torch.cuda.synchronize()
        plan.check()
        tiles = [gp.bwd_tiles() for _, _, gp in groups]
        swept = sum(t[0] for t in tiles) / max(1, sum(t[1] for t in tiles))
        print(json.dumps({"phase": "c5", "source_hash": kernel_source_hash(),
                          "kernels": {"c5_dba": KERNELS["c5_dba"].format(rho=plan.rho(wts.OP_DBA),
                                                                         mode=path_mode(plan)),
                                      "c5_soft_fwd": KERNELS["c5_soft_fwd"].format(rho=2),
                                      "c5_soft_bwd": KERNELS["c5_soft_bwd"].format(rho=2)},
                          "cells_per_pass": w.L * int(w.lengths.sum()),
                          "bwd_tiles_swept_frac": swept,
                          "soft_groups": [[a, b] for a, b, _ in groups],
                          "last_dispatches": {"c5_dba": args.steps,
                                              "c5_soft_fwd": args.steps * len(groups),
                                              "c5_soft_bwd": args.steps * len(groups)},
                          "autotune": it.tuned}))
        return
    if args.only in ("c3", "segment", "paper"):
        fn = {"c3": c3_section, "segment": segmentation_section,
              "paper": paper_table_section}[args.only]
        rec = fn(wts, dev) if args.only == "paper" else fn(wts, dev, speedup=False)
        print(json.dumps({"phase": args.only, "source_hash": kernel_source_hash(),
                          args.only: rec}))
        return
    if args.only == "c4":
        rec = c4_section(wts, dev, 2.0, steps=args.steps, lbfgs=False)
        print(json.dumps({"phase": "c4", "source_hash": kernel_source_hash(), "c4": rec}))
        return
    from paper_2404_12134_amd import autotune
    w = synth.make(2)
    Y, off, dt = wts.pack_cycles(w.cycles)
    mplan, _ = autotune.tuned_plan(off, w.d, dt, 0, op="medoid", cycles=Y, cache_path=None)
    k0 = int(wts.medoid(mplan, Y, with_matrix=False)[0].item())
    L = int(w.lengths[k0])
    B, _ = wts.init_barycenter(wts.Plan(off, w.d, dt, L), Y, wts.INIT_COPY, k0)
    plan, _ = autotune.tuned_plan(off, w.d, dt, L, op="dba", cycles=Y, bary=B, cache_path=None)
    Bo = torch.empty_like(B)
    counts = torch.empty(L, dtype=torch.int64, device=dev)
    dist = torch.empty(w.n, dtype=torch.float64, device=dev)
    for _ in range(args.steps):
        if args.only == "medoid":
            wts.medoid(mplan, Y, with_matrix=False)
        elif args.only == "dba":
            wts.dba_iterate(plan, B, Y, bary_out=Bo, counts=counts, dist=dist)
        else:
            wts.anomaly_score(plan, B, Y)
    torch.cuda.synchronize()
    used = {"medoid": mplan.rho(wts.OP_MEDOID), "dba": plan.rho(wts.OP_DBA),
            "score": plan.rho(wts.OP_SCORE)}[args.only]
    print(json.dumps({"phase": args.only, "L": L, "source_hash": kernel_source_hash(),
                      "kernels": {args.only: KERNELS[args.only].format(rho=used,
                                                                       mode=path_mode(plan))}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the float32-decision DBA comparison of the headline")
    ap.add_argument("--tune-cache", metavar="JSON", default=None,
                    help="keep the headline's tuned sweep shapes in this file: a later run "
                         "with the same file (e.g. under a profiler) reuses them untimed")
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the batched vs one-cycle-per-launch comparisons")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline (no 64-, 512- and 128-cycle or segmentation sections)")
    ap.add_argument("--soft-steps", type=int, default=50,
                    help="Soft-DTW descent steps per gamma in the 128-cycle section")
    ap.add_argument("--only", choices=["medoid", "dba", "score", "copy", "valu", "c5", "c3", "c4",
                                       "segment", "paper"],
                    help="run only one phase --steps times (for hardware-counter passes)")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="write profiles/traffic.json from rocprofv3 FETCH/WRITE_SIZE passes")
    args = ap.parse_args()
    if args.traffic_from:
        ingest_traffic(args.traffic_from)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_12134_amd import wetsand as wts

    wts.load()
    dev = torch.device("cuda:0")
    if args.only:
        only_phase(args, wts, dev)
        return
    valu = valu_rates()
    tau = valu["tau"]
    progress("valu rates measured (tau %s)" % tau)
    head = c5_headline(wts, dev, args.steps, args.warmup, tau, speedup=not args.no_speedup,
                       cpu=not args.no_cpu_baseline, tune_cache=args.tune_cache,
                       fp32=not args.no_fp32)
    progress("headline done: %.1f GCUPS" % head["value"])
    extras = {}
    if not args.no_extras:
        for key, fn, kw in (("c4_soft_dtw", c4_section, {"tau": tau, "steps": args.soft_steps}),
                            ("c3_dba_large", c3_section, {"speedup": not args.no_speedup}),
                            ("c2_medoid_dba_scores", c2_section,
                             {"speedup": not args.no_speedup}),
                            ("segmentation", segmentation_section,
                             {"speedup": not args.no_speedup}),
                            ("paper_soft_dtw_timing_table", paper_table_section, {})):
            progress("section %s" % key)
            extras[key] = guarded(fn, wts, dev, **kw)
        if not args.no_cpu_baseline:
            from paper_2404_12134_amd import synth
            extras["c2_cpu_baseline"] = cpu_baseline_c2(synth.make(2))
    line = {
        "metric": "DTW cell updates/s (GCUPS): batched DBA iteration + Soft-DTW forward and "
                  "backward, one barycenter iteration per step",
        "value": head["value"], "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": head["config"],
        "s_per_iteration": head["s_per_iteration"],
        "halves_s": head["halves_s"], "phase_gcups": head["phase_gcups"],
        "score_s": head["score_s"], "workload_s": head["workload_s"],
        "roofline": head["roofline"],
        "autotune": head["autotune"],
        "cpu_baseline": head.get("cpu_baseline"),
        "batched_vs_per_cycle": head["batched_vs_per_cycle"],
        "fp32_decisions": head.get("fp32_decisions"),
        "soft_bwd_zero_tiles": head.get("soft_bwd_zero_tiles"),
        "valu": valu,
        "extras": extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
