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
    va = wts.softdtw_descent_step(one, Y, off, Ba, 0.1, gv, 0.5)
    vb = wts.softdtw_descent_step(many, Y, off, Bb, 0.1, gv, 0.5)
    torch.cuda.synchronize()
    np.testing.assert_allclose(vb.cpu().numpy(), va.cpu().numpy(), rtol=1e-12)
    np.testing.assert_allclose(Bb.cpu().numpy(), Ba.cpu().numpy(), rtol=1e-9, atol=1e-12)
    # and the step itself against the oracle
    ov, og, oh = oracle.softdtw_batch(B0, cyc64, 0.1, 1.0 / w.lengths)
    expect = B0 - 0.5 * og / (2.0 * oh[:, None])
    np.testing.assert_allclose(va.cpu().numpy(), ov, rtol=1e-4)
    d = np.abs(Ba.cpu().numpy() - expect)
    assert d.max() <= 1e-4 * np.abs(expect).max()
