#!/usr/bin/env python3
"""Benchmark of the WETSAND hot path on one MI355X.

Workload (default): 64 cycles x 3 channels, float32, lengths U{4000..6000},
random-Fourier template with random time warps, N(0, 0.05) noise and three
cycles carrying a gradual drift.  One step is the whole DTW path over that
batch: medoid initialisation (all-pairs DTW), 10 DBA iterations from the
medoid, then the anomaly score of every cycle.  Inputs are resident in HBM
before timing starts.

Metric: DTW cell updates per second (GCUPS), cells = M * N per dynamic
program (all pairs of the medoid, L * N_k per DBA iteration and for the
scores).  Also reported: seconds per DBA iteration, per-phase GCUPS, the
roofline fraction of the dominant kernel, and the FP64 CPU oracle timed on a
bounded sample of the same workload.

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
HBM_PEAK_GBS = 8000.0


def c_min_dist(d: int) -> int:
    """Algorithmic VALU ops per cell of the DTW value sweep (squared cost):
    d subtractions, 1 multiply, d-1 FMAs, 2 minima, 1 add."""
    return 2 * d + 3


def c_min_path(d: int) -> int:
    """Algorithmic VALU ops per cell of a DTW sweep that also decides the argmin
    (path code or carried path length): the value recursion (2d + 3), two
    compares, two selects and one pack/add."""
    return 2 * d + 8


def c_min_soft(d: int, tau: int = 2) -> int:
    """Algorithmic VALU ops per cell of one Soft-DTW forward + backward pass pair,
    counted per DP pass (two passes per gradient step).  Forward: cost (2d),
    scale (1), min of three (2), three differences, conversions and base-2
    exponentials (3 + 3 + 3 tau), sum (2), logarithm (tau), conversion, two
    adds.  Backward: the replayed forward plus the three weights (reciprocal
    tau + 3 mul), the E recursion (3 conversions, 3 multiplies, 2 adds) and the
    gradient sums (d FMAs + 1 add).  tau = 2: a transcendental costs two FP64
    issue slots (measured)."""
    fwd = 2 * d + 1 + 2 + 3 + 3 + 3 * tau + 2 + tau + 1 + 2
    bwd = fwd + tau + 3 + 3 + 3 + 2 + d + 1
    return (fwd + bwd + 1) // 2


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("wts_dtw.hip", "wts_soft.hip", "wts_device.h"):
        with open(os.path.join(ROOT, "paper_2404_12134_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


KERNELS = {   # sweep -> rocprofv3 kernel name, by rows per lane (rho) of the plan
    "medoid": "void wts::(anonymous namespace)::dtw_fwd_kernel<float, float, 3, {rho}, 0, false>",
    "dba": "void wts::(anonymous namespace)::dtw_fwd_kernel<double, float, 3, {rho}, 2, false>",
    "score": "void wts::(anonymous namespace)::dtw_fwd_kernel<double, float, 3, {rho}, 1, false>",
}


def ingest_traffic(root: str):
    """Reads rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE passes (CSV) found under
    `root` and writes profiles/traffic.json: HBM bytes per launch of every sweep
    kernel, scaled by what the same counters read for the 1 GiB copy of
    `bench.py --only copy` (bytes_read / FETCH_SIZE_KiB, and the same for
    writes), tagged with the current kernel source hash."""
    import csv
    import glob
    # every pass must have run the current kernel source (its --only line says which)
    hashes = set()
    used = {}              # phase -> the sweep kernel instance its timed steps ran
    for f in glob.glob(os.path.join(root, "**", "*.out"), recursive=True):
        for line in open(f, errors="replace"):
            if line.startswith("{") and '"phase"' in line:
                rec = json.loads(line)
                hashes.add(rec.get("source_hash"))
                if rec.get("kernel"):
                    used[rec["phase"]] = rec["kernel"]
    if hashes != {kernel_source_hash()}:
        raise SystemExit("counter passes under %s ran kernel sources %s, not the current %s"
                         % (root, sorted(map(str, hashes)), kernel_source_hash()))
    per_dispatch = {}      # counters come in several rows per dispatch: sum them
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            key = (r["Kernel_Name"], r["Counter_Name"], f, r["Dispatch_Id"])
            per_dispatch[key] = per_dispatch.get(key, 0.0) + float(r["Counter_Value"])
    vals = {}
    for (kname, cname, _, _), v in per_dispatch.items():
        vals.setdefault((kname, cname), []).append(v)
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    gib = float(1 << 30)
    # the 1 GiB copies are the largest copyBuffer dispatches of all passes
    f_cal = max(v for k, vs in vals.items() if "copyBuffer" in k[0] and k[1] == "FETCH_SIZE"
                for v in vs)
    w_cal = max(v for k, vs in vals.items() if "copyBuffer" in k[0] and k[1] == "WRITE_SIZE"
                for v in vs)
    f_scale, w_scale = gib / f_cal, gib / w_cal        # bytes per counted KiB
    out = {"_calibration": {"copy_bytes": int(gib), "fetch_kib": f_cal, "write_kib": w_cal,
                            "fetch_scale": f_scale, "write_scale": w_scale}}
    for key in KERNELS:
        # every instance of this sweep that ran a complete launch in the
        # passes (the sweep-shape tuner at the start of each phase launches
        # all candidates); `kernel` is the one the phase itself chose
        pre, post = KERNELS[key].split("{rho}")
        names = sorted({k[0].split("(wts::")[0] for k in avg
                        if k[0].startswith(pre) and k[0].split("(wts::")[0].endswith(post)})
        inst = {}
        for name in names:
            fk = [avg[k] for k in avg if k[0].split("(wts::")[0] == name and k[1] == "FETCH_SIZE"]
            wk = [avg[k] for k in avg if k[0].split("(wts::")[0] == name and k[1] == "WRITE_SIZE"]
            if fk and wk:
                inst[name] = {"fetch_bytes": fk[0] * f_scale, "write_bytes": wk[0] * w_scale,
                              "bytes_per_launch": fk[0] * f_scale + wk[0] * w_scale}
        if inst:
            out[key] = {"kernel": used.get(key, names[0]), "source_hash": kernel_source_hash(),
                        "instances": inst}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def guarded(fn, *a, **kw):
    """Runs an optional section; an error is reported in its record instead of
    ending the run before the JSON line."""
    try:
        return fn(*a, **kw)
    except Exception as exc:   # noqa: BLE001 -- reported, not hidden
        print("section %s failed: %r" % (fn.__name__, exc), file=sys.stderr)
        return {"error": repr(exc)}


def cpu_baseline(w, n_sample: int = 40):
    """The FP64 oracle on the first n_sample cycles: all-pairs medoid, one DBA
    iteration from it and the scores.  Returns the record for the JSON line."""
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
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": "first %d of %d cycles: all-pairs medoid (both orders, as the oracle "
                      "computes them), 1 DBA iteration, scores; %d cells" % (n, w.n, cells)}


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


def soft_section(wts, dev, steps: int = 2, gamma: float = 0.1, band: float = 0.0):
    """Soft-DTW barycenter gradient steps on the full 128-cycle workload:
    forward (with checkpoints) + E-matrix backward + preconditioned step;
    band > 0 restricts them to the Sakoe-Chiba band of Table I (every cell is
    still swept, those outside the band masked; only cells inside count)."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    w = synth.make(4)
    Y, off, dt = wts.pack_cycles(w.cycles)
    L = w.L
    plan = wts.Plan(off, w.d, dt, L, band=band)
    B, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).to(dev)   # Eq. 7: lambda / m
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tf, tb = [], []

    def step(record):
        ev[0].record()
        val, ck = wts.softdtw_forward(plan, B, Y, gamma)
        ev[1].record()
        g, h = wts.softdtw_backward(plan, B, Y, gamma, ck, gv, with_mass=True)
        ev[2].record()
        wts.precond_step(B, g, h, 0.5)
        ev[3].record()
        if record:
            torch.cuda.synchronize()
            tf.append(ev[0].elapsed_time(ev[1]) / 1e3)
            tb.append(ev[1].elapsed_time(ev[2]) / 1e3)
        return val

    step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    for op in (wts.OP_SOFT_BWD,):
        st = wts.device_status(plan, op)
        if st != 0:
            raise RuntimeError("device status %d after the Soft-DTW backward" % st)
    cells = band_cells(L, w.lengths, band)
    counted = 2 * cells
    gcups = counted / sec / 1e9
    cm = c_min_soft(w.d)
    frac = gcups * 1e9 * cm / VALU_LANE_OPS_PEAK
    rec = {"workload": w.name + ": Soft-DTW gamma=%g, forward + backward + preconditioned "
                                "step (eta 0.5), weights 1/m_k%s"
                                % (gamma, ", Sakoe-Chiba band %g" % band if band else ""),
           "gcups_fwd_bwd": round(gcups, 2), "s_per_gradient_step": round(sec, 4),
           "forward_ms": round(1e3 * float(np.mean(tf)), 2),
           "backward_ms": round(1e3 * float(np.mean(tb)), 2),
           "cells_per_pass": cells, "ops_per_cell": cm, "alu_frac": round(frac, 4)}
    if band == 0.0:
        # the gradient with respect to the cycles: one more forward and
        # backward over the same cells, with the cycles on the rows
        Y64 = Y.to(torch.float64)
        wts.softdtw_grad_cycles(plan, B, Y64, gamma, gv)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            wts.softdtw_grad_cycles(plan, B, Y64, gamma, gv)
        ev[1].record()
        torch.cuda.synchronize()
        if wts.device_status(plan, wts.OP_SOFT_GRAD_C) != 0:
            raise RuntimeError("device status after the cycles gradient")
        tg = ev[0].elapsed_time(ev[1]) / 1e3 / steps
        gg = 2 * cells / tg / 1e9
        rec["grad_cycles"] = {"ms": round(1e3 * tg, 2), "gcups_fwd_bwd": round(gg, 2),
                              "alu_frac": round(gg * 1e9 * cm / VALU_LANE_OPS_PEAK, 4)}
        # Table I's optimizer, bounded to 3 iterations / 8 evaluations: the
        # host L-BFGS share is the wall time beyond the evaluations' sweeps.
        # A first run loads the optimizer's own torch kernels (once per process).
        wts.lbfgs_barycenter(plan, Y, B, gamma, gv, max_iter=3, max_eval=8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist = wts.lbfgs_barycenter(plan, Y, B, gamma, gv, max_iter=3, max_eval=8)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        rec["lbfgs"] = {"iterations_max": 3, "evaluations": len(hist),
                        "s_per_evaluation": round(tl / len(hist), 4),
                        "objective_first_last": [round(hist[0], 6), round(hist[-1], 6)],
                        "sweep_share": round(len(hist) * sec / tl, 3)}
    return rec


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
    return {"op": "dba_iterate", "one_cycle_per_launch_s": round(per, 5),
            "batched_s": round(batched, 5), "speedup": round(per / batched, 2),
            "per_cycle_timing": "sum of per-launch events" if sequential else "back to back"}


def dba_large_section(wts, dev, iters: int = 10, speedup: bool = True):
    """DBA on the 512-cycle workload (6 channels, lengths log-uniform
    1000..20000, L = 10000, nearest-length init): `iters` iterations replayed
    from a captured hipGraph (two iterations per graph), plus the path
    sweep's own launch time measured eagerly for its ALU fraction."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    w = synth.make(3)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, w.L)
    B0, _ = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    cells = w.L * int(w.lengths.sum())
    plan.enable_timing(8)
    for _ in range(3):
        wts.dba_iterate(plan, B0, Y)
    torch.cuda.synchronize()
    plan.sweep_ms(wts.OP_DBA)
    for _ in range(3):
        wts.dba_iterate(plan, B0, Y)
    tot, cnt = plan.sweep_ms(wts.OP_DBA)
    sweep_s = tot / max(cnt, 1) / 1e3
    plan.enable_timing(0)
    st = wts.device_status(plan, wts.OP_DBA)
    if st != 0:
        raise RuntimeError("device status %d after the large DBA" % st)
    runner = wts.DBARunner(plan, Y, B0, graph=True)
    runner.run(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    runner.run(iters)
    e1.record()
    torch.cuda.synchronize()
    it_s = e0.elapsed_time(e1) / 1e3 / iters
    del runner
    speed = dba_per_cycle_speedup(wts, plan, off, w.d, dt, w.L, Y, B0) if speedup else None
    cm = c_min_path(w.d)
    return {"workload": w.name + ": %d DBA iterations replayed from a hipGraph, nearest-length "
                                 "init" % iters,
            "s_per_dba_iteration": round(it_s, 5), "gcups": round(cells / it_s / 1e9, 2),
            "cells_per_iteration": cells, "rows_per_lane": plan.rho(wts.OP_DBA),
            "path_sweep_ms": round(sweep_s * 1e3, 3), "ops_per_cell": cm,
            "path_sweep_alu_frac": round(cells * cm / sweep_s / VALU_LANE_OPS_PEAK, 4),
            "batched_vs_per_cycle": speed}


def irregular_section(wts, dev, dba_iters: int = 10, soft_steps: int = 10, gamma: float = 0.1,
                      max_ckpt_gib: float = 96.0, speedup: bool = True):
    """The 256-cycle workload (6 channels, lengths 40000..50000 with 1 % of the
    samples dropped in gaps, L = max N): nearest-length init, `dba_iters` DBA
    iterations replayed from a hipGraph, then `soft_steps` preconditioned
    Soft-DTW (gamma) descent steps over checkpoint-bounded cycle groups, then
    the anomaly scores of all cycles.  Each phase is timed on its own."""
    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    w = synth.make(5)
    Y, off, dt = wts.pack_cycles(w.cycles)
    L = w.L
    cells = L * int(w.lengths.sum())
    plan = wts.Plan(off, w.d, dt, L)
    B0, _ = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    plan.enable_timing(4)
    wts.dba_iterate(plan, B0, Y)
    torch.cuda.synchronize()
    plan.sweep_ms(wts.OP_DBA)
    wts.dba_iterate(plan, B0, Y)
    tot, cnt = plan.sweep_ms(wts.OP_DBA)
    sweep_s = tot / max(cnt, 1) / 1e3
    plan.enable_timing(0)
    st = wts.device_status(plan, wts.OP_DBA)
    if st != 0:
        raise RuntimeError("device status %d after the DBA iteration" % st)
    dba_ws_gib = plan.workspace_bytes(wts.OP_DBA) / 2 ** 30
    speed = dba_per_cycle_speedup(wts, plan, off, w.d, dt, L, Y, B0, sequential=True) \
        if speedup else None
    runner = wts.DBARunner(plan, Y, B0, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = runner.run(dba_iters).clone()
    torch.cuda.synchronize()
    t_dba = (time.perf_counter() - t0) / dba_iters
    del runner
    plan.close()
    torch.cuda.empty_cache()

    groups = wts.subset_plans(off, w.d, dt, L, int(max_ckpt_gib * 2 ** 30))
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).to(dev)   # Eq. 7: lambda / m
    t_soft = []
    for _ in range(soft_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wts.softdtw_descent_step(groups, Y, off, B, gamma, gv, 0.5)
        torch.cuda.synchronize()
        t_soft.append(time.perf_counter() - t0)
    for a, b, gp in groups:
        st = wts.device_status(gp, wts.OP_SOFT_BWD)
        if st != 0:
            raise RuntimeError("device status %d after the Soft-DTW backward" % st)
        gp.close()
    torch.cuda.empty_cache()

    splan = wts.Plan(off, w.d, dt, L)
    wts.anomaly_score(splan, B, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wts.anomaly_score(splan, B, Y)
    torch.cuda.synchronize()
    t_score = time.perf_counter() - t0
    splan.close()
    torch.cuda.empty_cache()
    s_soft = float(np.median(t_soft))
    cm = c_min_path(w.d)
    return {"workload": w.name + ": nearest-length init, %d DBA iterations (hipGraph), %d "
                                 "Soft-DTW gamma=%g descent steps in %d checkpoint groups, "
                                 "scores" % (dba_iters, soft_steps, gamma, len(groups)),
            "cells_per_pass": cells,
            "s_per_dba_iteration": round(t_dba, 4), "dba_gcups": round(cells / t_dba / 1e9, 2),
            "path_sweep_ms": round(sweep_s * 1e3, 2), "ops_per_cell": cm,
            "path_sweep_alu_frac": round(cells * cm / sweep_s / VALU_LANE_OPS_PEAK, 4),
            "dba_workspace_gib": round(dba_ws_gib, 1),
            "s_per_soft_step": round(s_soft, 3),
            "soft_gcups_fwd_bwd": round(2 * cells / s_soft / 1e9, 2),
            "soft_alu_frac": round(2 * cells * c_min_soft(w.d) / s_soft / VALU_LANE_OPS_PEAK, 4),
            "score_s": round(t_score, 4),
            "workload_s": round(dba_iters * t_dba + float(np.sum(t_soft)) + t_score, 2),
            "batched_vs_per_cycle": speed}


def c_min_sub(d: int) -> int:
    """Sub-DTW sweep: the value recursion (2d + 3), two compares and two
    selects of the carried start column."""
    return 2 * d + 7


def segmentation_section(wts, dev, n_streams: int = 16, n_cycles: int = 37,
                         speedup: bool = True):
    """The segmentation step (Sec. III-A) at the scale the paper reports for
    its robot (Sec. IV-B: a reference cycle of about 16,300 samples, streams
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
                       % (n_streams, n_cycles, lr[0], lr[1], int(np.mean([Y.shape[0] for Y in streams])), M),
           "segments_per_stream": [len(sg) for sg in segs][:4], "rounds": rounds,
           "cells": cells, "batched_s": round(t_batch, 4),
           "gcups": round(cells / t_batch / 1e9, 2), "ops_per_cell": c_min_sub(3),
           "loop_alu_frac": round(cells * c_min_sub(3) / t_batch / VALU_LANE_OPS_PEAK, 4)}
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


def only_phase(args, wts, dev):
    """One phase of the step, --steps times, for rocprofv3 counter passes.  The
    'copy' phase is a plain 1 GiB device-to-device copy: the reference for
    scaling FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    from paper_2404_12134_amd import synth
    if args.only == "copy":
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"phase": "copy", "bytes_read": a.numel() * 8, "bytes_written": b.numel() * 8,
                          "source_hash": kernel_source_hash()}))
        return
    if args.only in ("large", "irregular", "segment"):
        fn = {"large": dba_large_section, "irregular": irregular_section,
              "segment": segmentation_section}[args.only]
        rec = fn(wts, dev, speedup=not args.no_speedup)
        print(json.dumps({"phase": args.only, "source_hash": kernel_source_hash(),
                          args.only: rec}))
        return
    if args.only == "soft":
        rec = soft_section(wts, dev, args.steps)
        torch.cuda.synchronize()
        print(json.dumps({"phase": "soft", "source_hash": kernel_source_hash(), "soft_dtw": rec}))
        return
    from paper_2404_12134_amd import autotune
    w = synth.make(2)
    Y, off, dt = wts.pack_cycles(w.cycles)
    # the same tuned sweep shapes as the full bench
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
                      "kernel": KERNELS[args.only].format(rho=used)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the batched vs one-cycle-per-launch comparison")
    ap.add_argument("--no-soft", action="store_true", help="skip the Soft-DTW section")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 512-cycle DBA section")
    ap.add_argument("--no-irregular", action="store_true",
                    help="skip the 256-cycle 40k..50k section (DBA, Soft-DTW, scores)")
    ap.add_argument("--no-segment", action="store_true",
                    help="skip the Sub-DTW segmentation section")
    ap.add_argument("--soft-steps", type=int, default=2)
    ap.add_argument("--only", choices=["medoid", "dba", "score", "soft", "copy", "large",
                                       "irregular", "segment"],
                    help="run only one phase --steps times (for hardware-counter passes)")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="write profiles/traffic.json from rocprofv3 FETCH/WRITE_SIZE passes")
    args = ap.parse_args()
    if args.traffic_from:
        ingest_traffic(args.traffic_from)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2404_12134_amd import synth
    from paper_2404_12134_amd import wetsand as wts

    wts.load()
    dev = torch.device("cuda:0")
    if args.only:
        only_phase(args, wts, dev)
        return
    w = synth.make(2)
    lens = w.lengths
    Y, off, dt = wts.pack_cycles(w.cycles)
    # sweep shapes of the medoid and barycenter plans: picked by timing the
    # candidates on this batch (outside the timed region)
    from paper_2404_12134_amd import autotune
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
        if int(kk.item()) != k0:
            raise RuntimeError("medoid changed between steps")
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
            for k, (a, b) in ev.items():
                times[k].append(a.elapsed_time(b) / 1e3)
        return out

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    mplan.enable_timing(4 * args.steps)
    plan.enable_timing(16 * args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for op in (wts.OP_MEDOID, wts.OP_DBA, wts.OP_SCORE):
        st = wts.device_status(mplan if op == wts.OP_MEDOID else plan, op)
        if st != 0:
            raise RuntimeError("device status %d after op %d" % (st, op))

    sec = (t1 - t0) / args.steps
    value = cells_step / sec / 1e9
    t_med = float(np.mean(times["medoid"]))
    t_dba = float(np.mean(times["dba"])) / iters
    t_score = float(np.mean(times["score"]))

    # roofline of the dominant sweep kernel (largest total time over the timed
    # steps), timed with HIP events around each launch on its stream
    sweeps = {
        "medoid": (mplan, wts.OP_MEDOID, cells_medoid, c_min_dist(w.d)),
        "dba": (plan, wts.OP_DBA, cells_bary, c_min_path(w.d)),
        "score": (plan, wts.OP_SCORE, cells_bary, c_min_path(w.d)),
    }
    kt = {}
    for key, (pl, op, cells, cm) in sweeps.items():
        tot, cnt = pl.sweep_ms(op)
        kt[key] = (tot, cnt)
    dom = max(kt, key=lambda k: kt[k][0])
    pl, op, cells, cm = sweeps[dom]
    launch_s = kt[dom][0] / max(1, kt[dom][1]) / 1e3
    achieved = cells * cm / launch_s / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    kname = KERNELS[dom].format(rho=pl.rho(op)).replace("void ", "")
    roofline = {"bound": "alu", "kernel": kname,
                "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic_from_profiles(dom, kname),
                "ops_per_cell": cm, "cells_per_launch": cells,
                "launch_ms": round(launch_s * 1e3, 3),
                "per_kernel_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in kt.items()},
                "per_kernel_alu_frac": {k: round(sweeps[k][2] * sweeps[k][3] /
                                                 (kt[k][0] / max(1, kt[k][1]) / 1e3) /
                                                 VALU_LANE_OPS_PEAK, 4) for k in kt}}

    # detection on the step's scores (Sec. IV-D thresholds), against the
    # cycles that carry an injected drift (a sanity check, not a gate)
    from paper_2404_12134_amd import detect
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

    speed = None
    if not args.no_speedup:
        # same kernels, one launch per cycle vs one batched launch
        single = [wts.Plan(off[k:k + 2] - off[k], w.d, dt, L) for k in range(n)]
        Ys = [Y[int(off[k]):int(off[k + 1])] for k in range(n)]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for k in range(n):
            wts.dba_iterate(single[k], Ba, Ys[k])
        torch.cuda.synchronize()
        tb = time.perf_counter()
        wts.dba_iterate(plan, Ba, Y, bary_out=Bb, counts=counts, dist=dist)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        speed = {"op": "dba_iterate", "one_cycle_per_launch_s": round(tb - ta, 5),
                 "batched_s": round(tc - tb, 5), "speedup": round((tb - ta) / (tc - tb), 2)}

    soft = None if args.no_soft else guarded(soft_section, wts, dev, args.soft_steps)
    soft_band = None if args.no_soft else guarded(soft_section, wts, dev, args.soft_steps,
                                                  band=0.6)
    large = None if args.no_large else guarded(dba_large_section, wts, dev,
                                               speedup=not args.no_speedup)
    irregular = None if args.no_irregular else guarded(irregular_section, wts, dev,
                                                       speedup=not args.no_speedup)
    segment = None if args.no_segment else guarded(segmentation_section, wts, dev,
                                                   speedup=not args.no_speedup)
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)

    line = {
        "metric": "DTW cell updates/s (GCUPS): medoid init + 10 DBA iterations + anomaly scores",
        "value": round(value, 3), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name + ": medoid init + %d DBA iterations + anomaly scores" % iters,
                   "n": n, "d": w.d, "L": L, "cells_per_step": cells_step},
        "s_per_dba_iteration": round(t_dba, 6),
        "phase_gcups": {"medoid": round(cells_medoid / t_med / 1e9, 2),
                        "dba_iteration": round(cells_bary / t_dba / 1e9, 2),
                        "score": round(cells_bary / t_score / 1e9, 2)},
        "roofline": roofline,
        "autotune": {"dba": {"rows_per_lane": tuned["rho"], "grid": tuned["grid"],
                             "candidates_ms": tuned["table"]},
                     "medoid": {"rows_per_lane": mtuned["rho"], "grid": mtuned["grid"],
                                "candidates_ms": mtuned["table"]}},
        "batched_vs_per_cycle": speed,
        "detection": detection,
        "soft_dtw": soft,
        "soft_dtw_band": soft_band,
        "dba_large": large,
        "irregular": irregular,
        "segmentation": segment,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
