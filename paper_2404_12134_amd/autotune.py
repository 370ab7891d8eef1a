"""Autotuner for the sweep shape of a plan.

A plan's wavefront sweeps have two shape parameters (`wts_opts`): the rows per
lane of a strip (rho: 2, 4 or 5) and the number of
persistent sweep wavefronts (grid).  Which shape is fastest depends on the
batch: with few long pairs the chain fill and the one-wave-per-SIMD issue rate
dominate, with many pairs the per-cell instruction count does.  `tune` times
every candidate shape on the batch (the caller's cycles, or seeded random
values of the same lengths) and keeps the fastest; results are cached in a
JSON file keyed by (device, operation, d, dtype, L, n, length buckets).

Every shape computes bit-identical results, so the choice only changes speed.
"""

from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

OPS = ("dba", "score", "align", "medoid")

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


def candidates(op: str) -> Iterable[Tuple[int, int]]:
    """(rho, grid) shapes to try; grid 0 is the library's default."""
    rhos = (2, 4, 5)
    for rho in rhos:
        yield rho, 0


def _run_op(wts, plan, op: str, bary, Y, outs):
    if op == "dba":
        return wts.dba_iterate(plan, bary, Y, bary_out=outs[0], counts=outs[1], dist=outs[2])
    if op == "score":
        return wts.anomaly_score(plan, bary, Y)
    if op == "align":
        return wts.dtw_align(plan, bary, Y, paths=True)
    return wts.medoid(plan, Y, with_matrix=False)


def tune(offsets, d: int, dtype: str, L: int, op: str = "dba", cycles=None, bary=None,
         reps: int = 3, device: int = 0, cache_path: Optional[str] = DEFAULT_CACHE,
         refresh: bool = False) -> dict:
    """Times every candidate shape for `op` on this batch and returns
    {"rho": .., "grid": .., "ms": .., "table": [[rho, grid, ms], ...], "key": ..}.

    offsets: int64[n+1] cycle offsets; cycles: the packed device buffer
    ([ΣN][d], `dtype`), or None for seeded random values of the same shape;
    bary: [L][d] float64 device tensor (barycenter ops), or None for random
    rows.  L = 0 with op = "medoid"."""
    import torch
    from . import wetsand as wts

    if op not in OPS:
        raise ValueError("op must be one of %s" % (OPS,))
    if (op == "medoid") != (L == 0):
        raise ValueError("the medoid is tuned on L = 0 plans, the other operations on L > 0")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    lengths = np.diff(off)
    dev = torch.device("cuda", device)
    key = cache_key(torch.cuda.get_device_name(device), op, d, dtype, L, lengths)
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
    if op == "dba":
        outs = (torch.empty((L, d), dtype=torch.float64, device=dev),
                torch.empty(L, dtype=torch.int64, device=dev),
                torch.empty(len(lengths), dtype=torch.float64, device=dev))

    table = []
    for rho, grid in candidates(op):
        plan = wts.Plan(off, d, dtype, L, device=device, rho=rho, grid=grid)
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
    entry = {"rho": rho, "grid": grid, "ms": ms, "table": table}
    if cache_path:
        store_cache(cache_path, key, entry)
    return dict(entry, key=key, cached=False)


def tuned_plan(offsets, d: int, dtype: str, L: int, op: str = "dba", **kw):
    """A plan with the shape `tune` picks for `op` on this batch."""
    from . import wetsand as wts
    t = tune(offsets, d, dtype, L, op=op, **kw)
    return wts.Plan(offsets, d, dtype, L, device=kw.get("device", 0), rho=t["rho"],
                    grid=t["grid"]), t
