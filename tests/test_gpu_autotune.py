"""The sweep-shape autotuner on the GPU: it picks one of the candidate shapes,
caches the choice, and the tuned plan computes the same bits as the default."""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import autotune, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_tune_dba_picks_a_candidate_and_caches(wts, tmp_path):
    import torch
    w = synth.make(3, n=12, len_range=(100, 1500), L=900)
    Y, off, dt = wts.pack_cycles(w.cycles)
    _, B0 = oracle.nearest_init([np.asarray(c, np.float64) for c in w.cycles], 900)
    Bt = torch.from_numpy(B0).cuda()
    cache = str(tmp_path / "tune.json")
    say("case autotune dba")
    t = autotune.tune(off, w.d, dt, 900, op="dba", cycles=Y, bary=Bt, cache_path=cache)
    assert not t["cached"]
    assert sorted(r for r, _, _ in t["table"]) == [2, 4, 5]
    assert t["rho"] in (2, 4, 5) and t["ms"] == min(ms for _, _, ms in t["table"])
    t2 = autotune.tune(off, w.d, dt, 900, op="dba", cycles=Y, bary=Bt, cache_path=cache)
    assert t2["cached"] and t2["rho"] == t["rho"]
    plan, _ = autotune.tuned_plan(off, w.d, dt, 900, op="dba", cycles=Y, bary=Bt, cache_path=cache)
    assert plan.rho(wts.OP_DBA) == t["rho"]
    B1, K1, d1 = wts.dba_iterate(plan, Bt, Y)
    ref = wts.Plan(off, w.d, dt, 900)
    B2, K2, d2 = wts.dba_iterate(ref, Bt, Y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(B1.cpu().numpy(), B2.cpu().numpy())
    np.testing.assert_array_equal(K1.cpu().numpy(), K2.cpu().numpy())
    np.testing.assert_array_equal(d1.cpu().numpy(), d2.cpu().numpy())


def test_tune_medoid_on_random_values(wts, tmp_path):
    w = synth.make(2, n=6, len_range=(300, 700))
    _, off, dt = wts.pack_cycles(w.cycles)
    say("case autotune medoid")
    t = autotune.tune(off, w.d, dt, 0, op="medoid", cache_path=str(tmp_path / "m.json"))
    assert sorted(r for r, _, _ in t["table"]) == [2, 4, 5]
