"""The score entry point that allocates nothing (its workspace is the
library's static device scratch), against the allocating wts_anomaly_score:
bit for bit on two calls in a row, the second with a smaller input, and
against the FP64 oracle."""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_scores_match_the_allocating_entry_point(wts):
    import torch
    for case, (n, lo, hi, L) in enumerate(((12, 300, 2500, 1500), (5, 100, 700, 400))):
        say("case no-alloc scores %d: n=%d lengths %d..%d L=%d" % (case, n, lo, hi, L))
        w = synth.make(3, n=n, len_range=(lo, hi), L=L)
        cyc = [np.asarray(c, np.float64) for c in w.cycles]
        Y, off, dt = wts.pack_cycles(w.cycles)
        plan = wts.Plan(off, w.d, dt, L)
        B, _ = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
        sc, dist, plen = wts.anomaly_score(plan, B, Y)
        s2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        d2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        p2 = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        wts.anomaly_score_noalloc(plan, B, Y, s2, d2, p2)
        assert plan.status() == wts.OK
        np.testing.assert_array_equal(s2.cpu().numpy(), sc.cpu().numpy())
        np.testing.assert_array_equal(d2.cpu().numpy(), dist.cpu().numpy())
        np.testing.assert_array_equal(p2.cpu().numpy(), plen.cpu().numpy())
        os_, od, ol = oracle.score_batch(B.cpu().numpy(), cyc)
        np.testing.assert_array_equal(s2.cpu().numpy(), os_)
        np.testing.assert_array_equal(p2.cpu().numpy(), ol)
        plan.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch(wts):
    """A plan whose score workspace exceeds the 32 MiB scratch gets
    WTS_E_CAPACITY before anything is enqueued."""
    import torch
    n, N, L = 64, 6000, 6000
    off = np.arange(n + 1, dtype=np.int64) * N
    plan = wts.Plan(off, 1, "f32", L)
    assert plan.workspace_bytes(wts.OP_SCORE) > (32 << 20)
    B = torch.zeros((L, 1), dtype=torch.float64, device="cuda")
    Y = torch.zeros((n * N, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(wts.WtsError) as ei:
        wts.anomaly_score_noalloc(plan, B, Y)
    assert ei.value.status == wts.E_CAPACITY
