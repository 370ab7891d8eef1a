"""Path recovery by strips (entry tags, all strips walked at once) and by
pairs (argmin codes only, each pair walking its strips in turn) give the
same bits: distances, path lengths, paths, DBA barycenters, counts, for
float64 and float32 decisions, on ragged shapes across several strips and
on tie-heavy integer series; and both match the oracle's paths."""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(wts, X, cycles, walk, rho, decision="fp64"):
    import torch
    Y, off, dt = wts.pack_cycles(cycles)
    plan = wts.Plan(off, X.shape[1], dt, X.shape[0], rho=rho, walk=walk, decision=decision)
    assert plan.walk() == walk
    B = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).cuda()
    dist, plen, paths = wts.dtw_align(plan, B, Y, paths=True)
    Bo, counts, d2 = wts.dba_iterate(plan, B, Y)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    out = {k: v.cpu().numpy() for k, v in (("dist", dist), ("plen", plen), ("bary", Bo),
                                           ("counts", counts), ("dba_dist", d2))}
    ph = paths.cpu().numpy()
    L = X.shape[0]
    out["paths"] = [ph[k * (L - 1) + off[k]:k * (L - 1) + off[k] + out["plen"][k]]
                    for k in range(len(cycles))]
    plan.close()
    return out


SHAPES = [(300, [1, 5, 299, 700], 3), (700, [690, 1200], 1), (1030, [64, 2100, 1029], 6),
          (129, [128, 130, 1], 8)]


@pytest.mark.parametrize("rho", [2, 4, 5])
@pytest.mark.parametrize("L,lens,d", SHAPES)
def test_walk_modes_same_bits(wts, rho, L, lens, d):
    r = np.random.Generator(np.random.PCG64(L * 13 + rho))
    ints = L % 2 == 1   # odd L: small integers, where ties decide the path
    X = r.integers(0, 3, (L, d)).astype(np.float64) if ints else r.standard_normal((L, d))
    cyc = [(r.integers(0, 3, (N, d)) if ints else r.standard_normal((N, d))).astype(np.float32)
           for N in lens]
    say("case walk modes L=%d lens=%s d=%d rho=%d" % (L, lens, d, rho))
    a = run(wts, X, cyc, "strips", rho)
    b = run(wts, X, cyc, "pairs", rho)
    for k in ("dist", "plen", "bary", "counts", "dba_dist"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for pa, pb in zip(a["paths"], b["paths"]):
        np.testing.assert_array_equal(pa, pb)
    for k, c in enumerate(cyc):   # and the oracle's optimal path
        _, n_o, po, _ = oracle.dtw(X, c.astype(np.float64))
        np.testing.assert_array_equal(np.asarray(b["paths"][k]), po)


def test_walk_modes_same_bits_fp32_decisions(wts):
    w = synth.make(3, n=12, len_range=(900, 3000), L=1500, seed=9)
    k, X = oracle.nearest_init(w.cycles, w.L)
    say("case walk modes fp32 decisions: 12 x 900-3000, L 1500")
    a = run(wts, X, w.cycles, "strips", 4, decision="fp32")
    b = run(wts, X, w.cycles, "pairs", 4, decision="fp32")
    for key in ("dist", "plen", "bary", "counts", "dba_dist"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


def test_auto_walk_picks_pairs_for_large_batches_only(wts):
    small = synth.make(2, n=4, len_range=(400, 500), seed=3)
    Y, off, dt = wts.pack_cycles(small.cycles)
    p = wts.Plan(off, small.d, dt, 450)
    assert p.walk() == "strips"
    p.close()
