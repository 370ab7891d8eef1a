"""Iteration drivers: graph-replayed DBA loop and grouped Soft-DTW descent."""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_dba_runner_graph_trajectory_bitwise(wts):
    import torch
    w = synth.make(3, n=8, len_range=(100, 1200), L=600)
    cyc64 = [np.asarray(c, np.float64) for c in w.cycles]
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, 600)
    _, B0 = oracle.nearest_init(cyc64, 600)
    for graph in (True, False):
        say("case dba runner graph=%s" % graph)
        run = wts.DBARunner(plan, Y, torch.from_numpy(B0).cuda(), graph=graph)
        Bo = B0
        done = 0
        for chunk in (2, 3, 2):          # odd chunk exercises the eager tail
            Bg = run.run(chunk).cpu().numpy()
            for _ in range(chunk):
                Bo, _, _, _ = oracle.dba_iterate(Bo, cyc64)
            done += chunk
            np.testing.assert_array_equal(Bg, Bo, err_msg="after %d iterations" % done)


def test_grouped_soft_descent_matches_single_group(wts):
    import torch
    w = synth.make(4, n=6, len_range=(300, 500), L=400)
    cyc64 = [np.asarray(c, np.float64) for c in w.cycles]
    Y, off, dt = wts.pack_cycles(w.cycles)
    B0 = oracle.euclid_mean(cyc64, 400)
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    one = wts.subset_plans(off, w.d, dt, 400, 1 << 40)
    per_cycle = wts.Plan(off[0:2] - off[0], w.d, dt, 400).workspace_bytes(wts.OP_SOFT_FWD)
    many = wts.subset_plans(off, w.d, dt, 400, int(2.5 * per_cycle))
    assert len(one) == 1 and len(many) >= 3
    say("case grouped soft: %d groups" % len(many))
    Ba = torch.from_numpy(B0.copy()).cuda()
    Bb = torch.from_numpy(B0.copy()).cuda()
    sa = wts.SoftDescent(one, Y, off, 400, w.d, 0.1, gv, 0.5)
    sb = wts.SoftDescent(many, Y, off, 400, w.d, 0.1, gv, 0.5)
    va = sa.step(Ba, check=True)
    vb = sb.step(Bb, check=True)
    # the groups accumulate into one gradient, row mass and objective with the
    # additions of the single group, in the same order: bitwise equal
    np.testing.assert_array_equal(vb.cpu().numpy(), va.cpu().numpy())
    np.testing.assert_array_equal(sb.objective.cpu().numpy(), sa.objective.cpu().numpy())
    np.testing.assert_array_equal(Bb.cpu().numpy(), Ba.cpu().numpy())
    # and the step itself against the oracle
    ov, og, oh = oracle.softdtw_batch(B0, cyc64, 0.1, 1.0 / w.lengths)
    expect = B0 - 0.5 * og / (2.0 * oh[:, None])
    np.testing.assert_allclose(va.cpu().numpy(), ov, rtol=1e-4)
    f = float(np.dot(1.0 / w.lengths, ov))
    assert abs(sa.objective.item() - f) <= 1e-4 * abs(f)
    d = np.abs(Ba.cpu().numpy() - expect)
    assert d.max() <= 1e-4 * np.abs(expect).max()


def test_soft_descent_step_replays_from_a_graph(wts):
    """The grouped descent step allocates nothing once built, so it can be
    captured: three replays, each against an eager step from the same bary
    (with eager work and synchronisations between the replays)."""
    import torch
    w = synth.make(4, n=5, len_range=(200, 400), L=300)
    Y, off, dt = wts.pack_cycles(w.cycles)
    per_cycle = wts.Plan(off[0:2] - off[0], w.d, dt, 300).workspace_bytes(wts.OP_SOFT_FWD)
    groups = wts.subset_plans(off, w.d, dt, 300, int(2.5 * per_cycle))
    assert len(groups) >= 2
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    B0, _ = wts.init_barycenter(wts.Plan(off, w.d, dt, 300), Y, wts.INIT_EUCLID_MEAN)
    eager = wts.SoftDescent(groups, Y, off, 300, w.d, 0.1, gv, 0.5)
    cap = wts.SoftDescent(groups, Y, off, 300, w.d, 0.1, gv, 0.5)
    Bg = B0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cap.step(Bg)
    torch.cuda.current_stream().wait_stream(s)
    Be = B0.clone()
    for rep in range(3):
        say("case soft descent graph replay %d" % rep)
        g.replay()
        eager.step(Be, check=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Bg.cpu().numpy(), Be.cpu().numpy())
        np.testing.assert_array_equal(cap.values.cpu().numpy(), eager.values.cpu().numpy())
        np.testing.assert_array_equal(cap.objective.cpu().numpy(),
                                      eager.objective.cpu().numpy())
    for _, _, plan in groups:
        assert plan.status() == wts.OK
