"""The boundary's error surface on the GPU: input validation (the paper drops
samples with missing values before any DTW, Sec. III-A), the plan's status
word, the accumulating Soft-DTW backward and the Eq. 7 objective."""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small(n=5, L=300):
    w = synth.make(3, n=n, len_range=(150, 700), L=L)
    return w, [np.asarray(c, np.float64) for c in w.cycles]


def test_validate_flags_a_nan_sample_and_skips_the_sweeps(wts):
    """A NaN in the cycles (or an infinity in the barycenter) of a validated
    plan: the call is enqueued, its sweeps are skipped, and the status read
    reports WTS_E_NONFINITE once; the next clean call is bit-exact again."""
    import torch
    w, cyc = _small()
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, 300, validate=True)
    B0, _ = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    assert plan.status() == wts.OK
    bad = Y.clone()
    bad[int(off[2]) + 7, 1] = float("nan")
    say("case validate: NaN in cycle 2, dba_iterate")
    wts.dba_iterate(plan, B0, bad)
    assert plan.status() == wts.E_NONFINITE
    assert plan.status() == wts.OK            # read and cleared
    say("case validate: inf in the barycenter, anomaly_score and Soft-DTW forward")
    Binf = B0.clone()
    Binf[299, 0] = float("inf")
    wts.anomaly_score(plan, Binf, Y)
    assert plan.status() == wts.E_NONFINITE
    wts.softdtw_forward(plan, Binf, Y, 0.5)
    assert plan.status() == wts.E_NONFINITE
    say("case validate: clean call after the flagged ones")
    B1, counts, dist = wts.dba_iterate(plan, B0, Y)
    assert plan.status() == wts.OK
    Bn, K, od, _ = oracle.dba_iterate(B0.cpu().numpy(), cyc)
    np.testing.assert_array_equal(B1.cpu().numpy(), Bn)
    np.testing.assert_array_equal(counts.cpu().numpy(), K)
    np.testing.assert_array_equal(dist.cpu().numpy(), od)
    with pytest.raises(wts.WtsError):
        wts.anomaly_score(plan, Binf, Y)
        plan.check()


def test_validated_and_plain_plans_agree_bitwise(wts):
    """Validation only reads the inputs: results are the same bits."""
    import torch
    w, cyc = _small(n=4)
    Y, off, dt = wts.pack_cycles(w.cycles)
    pv = wts.Plan(off, w.d, dt, 300, validate=True)
    pp = wts.Plan(off, w.d, dt, 300)
    B0, _ = wts.init_barycenter(pp, Y, wts.INIT_EUCLID_MEAN)
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    out = []
    for plan in (pv, pp):
        b, _, _ = wts.dba_iterate(plan, B0, Y)
        s, _, _ = wts.anomaly_score(plan, B0, Y)
        v, ck = wts.softdtw_forward(plan, B0, Y, 0.3)
        g, h = wts.softdtw_backward(plan, B0, Y, 0.3, ck, gv, with_mass=True)
        out.append([t.cpu().numpy() for t in (b, s, v, g, h)])
        assert plan.status() == wts.OK
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_backward_accumulate_over_groups_is_bitwise_one_call(wts):
    """Two cycle groups with accumulate=1 on the second give the very
    additions of one call over the batch: bitwise equal gradient and mass."""
    import torch
    w, cyc = _small(n=6)
    Y, off, dt = wts.pack_cycles(w.cycles)
    whole = wts.Plan(off, w.d, dt, 300)
    B0, _ = wts.init_barycenter(whole, Y, wts.INIT_EUCLID_MEAN)
    gv = torch.from_numpy(np.linspace(0.5, 2.0, w.n)).cuda()
    v, ck = wts.softdtw_forward(whole, B0, Y, 0.2)
    g1, h1 = wts.softdtw_backward(whole, B0, Y, 0.2, ck, gv, with_mass=True)
    G = torch.empty_like(g1)
    H = torch.empty_like(h1)
    for q, (a, b) in enumerate(((0, 2), (2, 6))):
        part = wts.Plan(off[a:b + 1] - off[a], w.d, dt, 300)
        Yg = Y[int(off[a]):int(off[b])]
        _, ckg = wts.softdtw_forward(part, B0, Yg, 0.2)
        wts.softdtw_backward(part, B0, Yg, 0.2, ckg, gv[a:b], grad=G, mass=H,
                             accumulate=q > 0)
        assert part.status() == wts.OK
    np.testing.assert_array_equal(G.cpu().numpy(), g1.cpu().numpy())
    np.testing.assert_array_equal(H.cpu().numpy(), h1.cpu().numpy())
    # and against the oracle (Soft-DTW tolerance)
    _, og, oh = oracle.softdtw_batch(B0.cpu().numpy(), cyc, 0.2, gv.cpu().numpy())
    np.testing.assert_allclose(H.cpu().numpy(), oh, rtol=1e-4)
    assert np.linalg.norm(G.cpu().numpy() - og) <= 1e-4 * np.linalg.norm(og)


def test_objective_is_the_ordered_weighted_sum(wts):
    """Eq. 7: sum_k w_k value_k folded in ascending k (bitwise the same fold
    on the host), and within the Soft-DTW tolerance of the oracle's values."""
    import torch
    w, cyc = _small(n=7)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, 300)
    B0, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    wv = 1.0 / w.lengths.astype(np.float64)
    v, _ = wts.softdtw_forward(plan, B0, Y, 0.5)
    f = wts.barycenter_objective(v, torch.from_numpy(wv).cuda())
    vh = v.cpu().numpy()
    s = 0.0
    for k in range(w.n):
        s = s + wv[k] * vh[k]
    assert f.item() == s
    ov = oracle.softdtw_batch(B0.cpu().numpy(), cyc, 0.5, grad=False)
    assert abs(f.item() - float(np.dot(wv, ov))) <= 1e-4 * abs(float(np.dot(wv, ov)))
    # accumulate = 1 continues the fold from the value in out (here: in place)
    f2 = wts.barycenter_objective(v, None, out=f, accumulate=True)
    s2 = s
    for k in range(w.n):
        s2 = s2 + 1.0 * vh[k]
    assert f2.item() == s2
