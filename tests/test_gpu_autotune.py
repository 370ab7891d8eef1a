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
    assert sorted({r for r, _, _ in t["table"]}) == [2, 4, 5]
    assert len(t["table"]) == 9 and t["cus"] > 0
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
    assert sorted({r for r, _, _ in t["table"]}) == [2, 4, 5]


def test_tune_soft_grids_give_the_same_bits(wts, tmp_path):
    """The Soft-DTW shape candidates (grids) are timed, one is picked, and
    every candidate's plan gives bitwise the same values, gradient and row
    mass (each pair's sweep runs the same operations whatever the grid),
    within the Soft-DTW bar of the oracle."""
    import torch
    w = synth.make(4, n=9, len_range=(300, 900), L=600)
    cyc = [np.asarray(c, np.float64) for c in w.cycles]
    Y, off, dt = wts.pack_cycles(w.cycles)
    B0 = torch.from_numpy(oracle.euclid_mean(cyc, 600)).cuda()
    say("case autotune soft")
    t = autotune.tune(off, w.d, dt, 600, op="soft", cycles=Y, bary=B0,
                      cache_path=str(tmp_path / "s.json"))
    assert {r for r, _, _ in t["table"]} == {2} and len(t["table"]) == 3
    assert t["ms"] == min(ms for _, _, ms in t["table"])
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    outs = []
    for _, grid, _ in t["table"]:
        plan = wts.Plan(off, w.d, dt, 600, grid=grid)
        v, ck = wts.softdtw_forward(plan, B0, Y, 0.3)
        g, h = wts.softdtw_backward(plan, B0, Y, 0.3, ck, gv, with_mass=True)
        assert plan.status() == wts.OK
        outs.append([x.cpu().numpy() for x in (v, g, h)])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            np.testing.assert_array_equal(a, b)
    ov, og, oh = oracle.softdtw_batch(B0.cpu().numpy(), cyc, 0.3, gv.cpu().numpy())
    np.testing.assert_allclose(outs[0][0], ov, rtol=1e-4)
    assert np.linalg.norm(outs[0][1] - og) <= 1e-4 * np.linalg.norm(og)
    np.testing.assert_allclose(outs[0][2], oh, rtol=1e-4)
