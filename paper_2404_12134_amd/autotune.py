"""Autotuner for the sweep shape of a plan.

A plan's wavefront sweeps have two shape parameters (`wts_opts`): the rows per
lane of a strip (rho: 2, 4 or 5 for the DTW sweeps; the Soft-DTW sweeps are
built for 2 rows per lane only -- one row per lane was measured slower on the
128 x 20k workload, three do not fit the backward's registers) and the
number of persistent sweep wavefronts (grid).  Which shape is fastest depends
on the batch: with few long pairs the chain fill and the one-wave-per-SIMD
issue rate dominate, with many pairs the per-cell instruction count does.
`tune` times every candidate shape on the batch (the caller's cycles, or
seeded random values of the same lengths) and keeps the fastest; results are
cached in a JSON file keyed by (GPU architecture, compute units, operation,
d, dtype, L, n, length buckets, and the Sakoe-Chiba band and decision
precision when they are set).

Every shape computes bit-identical results (each pair's dynamic program runs
the same operations whatever the strip-to-wave assignment), so the choice
only changes speed.
"""

from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

OPS = ("dba", "score", "align", "medoid", "soft")

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "wetsand_mi", "autotune.json")


def length_signature(lengths: Sequence[int]) -> Tuple[int, int, int, int]:
    """n and the 10th / 50th / 90th length percentiles, rounded to two
    significant digits: batches that differ only in detail share an entry."""
    x = np.asarray(lengths, dtype=np.float64)

    def r2(v: float) -> int:
        if v <= 0:
            return 0
        e = int(np.floor(np.log10(v))) - 1
        return int(round(v / 10 ** e) * 10 ** e)

    return (int(x.size), r2(np.percentile(x, 10)), r2(np.percentile(x, 50)),
            r2(np.percentile(x, 90)))


def cache_key(device_name: str, op: str, d: int, dtype: str, L: int,
              lengths: Sequence[int]) -> str:
    n, p10, p50, p90 = length_signature(lengths)
    return "%s|%s|d%d|%s|L%d|n%d|%d-%d-%d" % (device_name, op, d, dtype, L, n, p10, p50, p90)


def load_cache(path: str) -> Dict[str, dict]:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: str, key: str, entry: dict) -> None:
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def grid_candidates(op: str, cus: int) -> Tuple[int, ...]:
    """Persistent sweep waves to try: 0 is the library's default (24 per
    compute unit); fewer waves leave each SIMD fewer strips to interleave but
    start fewer strips that then wait on their neighbours.  The Soft-DTW
    backward holds three waves per SIMD (12 per compute unit)."""
    if op == "soft":
        return (0, 12 * cus, 6 * cus)
    return (0, 16 * cus, 8 * cus)


def candidates(op: str, cus: int = 256) -> Iterable[Tuple[int, int]]:
    """(rho, grid) shapes to try for `op` on a GPU with `cus` compute units."""
    rhos = (2,) if op == "soft" else (2, 4, 5)
    for rho in rhos:
        for grid in grid_candidates(op, cus):
            yield rho, grid


def _run_op(wts, plan, op: str, bary, Y, outs):
    if op == "soft":   # one forward (checkpoints in outs[0] if given) and backward
        _, ck = wts.softdtw_forward(plan, bary, Y, 0.1, ckpt=outs[0])
        return wts.softdtw_backward(plan, bary, Y, 0.1, ck)
    if op == "dba":
        return wts.dba_iterate(plan, bary, Y, bary_out=outs[0], counts=outs[1], dist=outs[2])
    if op == "score":
        return wts.anomaly_score(plan, bary, Y)
    if op == "align":
        return wts.dtw_align(plan, bary, Y, paths=True)
    return wts.medoid(plan, Y, with_matrix=False)


def tune(offsets, d: int, dtype: str, L: int, op: str = "dba", cycles=None, bary=None,
         reps: int = 3, device: int = 0, cache_path: Optional[str] = DEFAULT_CACHE,
         refresh: bool = False, shapes=None, workspace=None, band: float = 0.0,
         decision: str = "fp64") -> dict:
    """Times every candidate shape for `op` on this batch and returns
    {"rho": .., "grid": .., "ms": .., "table": [[rho, grid, ms], ...], "key": ..}.

    offsets: int64[n+1] cycle offsets; cycles: the packed device buffer
    ([ΣN][d], `dtype`), or None for seeded random values of the same shape;
    bary: [L][d] float64 device tensor (barycenter ops), or None for random
    rows.  L = 0 with op = "medoid".  shapes: the (rho, grid) candidates
    (default `candidates(op, cus)`); workspace: a caller-owned 256-byte
    aligned uint8 buffer used as the DBA workspace or the Soft-DTW
    checkpoints of every candidate (for batches whose buffers are large);
    band, decision: plan options of the candidates (a banded Soft-DTW sweep
    and the float32-decision DTW sweeps have shapes of their own)."""
    import torch
    from . import wetsand as wts

    if op not in OPS:
        raise ValueError("op must be one of %s" % (OPS,))
    if (op == "medoid") != (L == 0):
        raise ValueError("the medoid is tuned on L = 0 plans, the other operations on L > 0")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    lengths = np.diff(off)
    dev = torch.device("cuda", device)
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", torch.cuda.get_device_name(device)).split(":")[0]
    cus = int(props.multi_processor_count)
    shapes = list(candidates(op, cus) if shapes is None else shapes)
    key = cache_key("%s-%dcu" % (arch, cus), op, d, dtype, L, lengths)
    if band:
        key += "|band%g" % band
    if decision != "fp64":
        key += "|" + decision
    if cache_path and not refresh:
        hit = load_cache(cache_path).get(key)
        if hit:
            return dict(hit, key=key, cached=True)

    g = np.random.Generator(np.random.PCG64(12134))
    tdt = torch.float32 if dtype == "f32" else torch.float64
    Y = cycles
    if Y is None:
        Y = torch.from_numpy(g.standard_normal((int(off[-1]), d))).to(device=dev, dtype=tdt)
    B = bary
    if B is None and L > 0:
        B = torch.from_numpy(g.standard_normal((L, d))).to(dev)
    outs = None
    if op == "soft":
        outs = (workspace,)
    if op == "dba":
        outs = (torch.empty((L, d), dtype=torch.float64, device=dev),
                torch.empty(L, dtype=torch.int64, device=dev),
                torch.empty(len(lengths), dtype=torch.float64, device=dev))

    table = []
    for rho, grid in shapes:
        plan = wts.Plan(off, d, dtype, L, device=device, rho=rho, grid=grid, band=band,
                        decision=decision)
        if workspace is not None and op == "dba":
            plan.set_workspace(wts.OP_DBA, workspace)
        _run_op(wts, plan, op, B, Y, outs)            # warm-up: workspace, code paths
        torch.cuda.synchronize(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(max(1, reps)):
            e0.record()
            _run_op(wts, plan, op, B, Y, outs)
            e1.record()
            torch.cuda.synchronize(dev)
            best = min(best, e0.elapsed_time(e1))
        table.append([rho, grid, round(best, 4)])
        plan.close()
    rho, grid, ms = min(table, key=lambda r: r[2])
    entry = {"rho": rho, "grid": grid, "ms": ms, "table": table, "arch": arch, "cus": cus}
    if cache_path:
        store_cache(cache_path, key, entry)
    return dict(entry, key=key, cached=False)


def tuned_plan(offsets, d: int, dtype: str, L: int, op: str = "dba", **kw):
    """A plan with the shape `tune` picks for `op` on this batch."""
    from . import wetsand as wts
    t = tune(offsets, d, dtype, L, op=op, **kw)
    return wts.Plan(offsets, d, dtype, L, device=kw.get("device", 0), rho=t["rho"],
                    grid=t["grid"], band=kw.get("band", 0.0),
                    decision=kw.get("decision", "fp64")), t
