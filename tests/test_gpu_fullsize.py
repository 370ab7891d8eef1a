"""Parity at the full workload sizes, on outputs the oracle can afford.

The GPU runs the whole batch in the bench's launch configuration; the oracle
checks sampled cycles one by one.  Whole-batch reductions are sampled through
the weights: with w_k = 0 for every cycle but a few, the fixed-order fold of
DBA (and of the Soft-DTW gradient) equals the fold over those few cycles
alone, so the comparison stays bit-exact (DBA) or within 1e-4 (Soft-DTW).
"""

import functools
import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f64(cycles):
    return [np.asarray(c, dtype=np.float64) for c in cycles]


def check_vec(a, b, rtol=1e-4):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    scale = np.maximum(np.abs(b), 1e-2 * np.abs(b).max())
    assert (np.abs(a - b) <= rtol * scale).all(), np.max(np.abs(a - b) / scale)
    assert np.linalg.norm(a - b) <= rtol * np.linalg.norm(b)


@pytest.mark.timeout(600)
def test_config2_full_step(wts):
    """64 x 3 ch, 4000..6000: medoid (sampled entries), one DBA iteration and
    the scores of all 64 cycles, bit-exact."""
    import torch
    w = synth.make(2)
    Y, off, dt = wts.pack_cycles(w.cycles)
    say("c2: medoid on the GPU")
    mplan = wts.Plan(off, 3, dt, 0)
    k, Dm, tot = wts.medoid(mplan, Y)
    Dm = Dm.cpu().numpy()
    cyc = f64(w.cycles)
    r = np.random.Generator(np.random.PCG64(0))
    for a, b in r.integers(0, w.n, (8, 2)):
        if a == b:
            continue
        od, _, _, _ = oracle.dtw(cyc[a], cyc[b], with_path=False)
        assert Dm[a, b] == od and Dm[b, a] == od
    assert (np.diag(Dm) == 0).all()
    k = int(k.item())
    tot_o = np.array([sum(Dm[q, i] for i in range(w.n)) for q in range(w.n)])
    np.testing.assert_array_equal(tot.cpu().numpy(), tot_o)
    assert k == int(np.argmin(tot_o))
    L = w.lengths[k]
    plan = wts.Plan(off, 3, dt, int(L))
    B0, _ = wts.init_barycenter(plan, Y, wts.INIT_COPY, k)
    say("c2: DBA iteration + scores, oracle on all 64 cycles")
    B1, counts, dist = wts.dba_iterate(plan, B0, Y)
    score, sdist, plen = wts.anomaly_score(plan, B1, Y)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    Bn, K, od, _ = oracle.dba_iterate(cyc[k], cyc)
    np.testing.assert_array_equal(B1.cpu().numpy(), Bn)
    np.testing.assert_array_equal(counts.cpu().numpy(), K)
    np.testing.assert_array_equal(dist.cpu().numpy(), od)
    os_, osd, ol = oracle.score_batch(Bn, cyc)
    np.testing.assert_array_equal(score.cpu().numpy(), os_)
    np.testing.assert_array_equal(plen.cpu().numpy(), ol)
    # the drifted cycles carry the largest scores (sanity, not a parity gate)
    top3 = set(np.argsort(-os_)[:3].tolist())
    say("c2: drift cycles", w.meta["drift"], "top-3 scores", sorted(top3))


@pytest.mark.timeout(600)
def test_config3_full_sampled(wts):
    """512 x 6 ch, log-uniform 1000..20000, L = 10000: paths of sampled cycles
    and a DBA update weighted onto them, bit-exact."""
    import torch
    w = synth.make(3)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 6, dt, w.L)
    cyc = f64(w.cycles)
    lens = w.lengths
    pick = sorted({int(np.argmin(lens)), int(np.argmax(lens)), 7, 301})
    say("c3: nearest-length init, full alignment with paths")
    B0, kn = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    ko, Bo = oracle.nearest_init(cyc, w.L)
    assert kn == ko
    np.testing.assert_array_equal(B0.cpu().numpy(), Bo)
    dist, plen, paths = wts.dtw_align(plan, B0, Y, paths=True)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    for q in pick:
        say("c3: oracle on cycle", q, "N =", lens[q])
        od, ol, op, _ = oracle.dtw(Bo, cyc[q])
        assert dist[q].item() == od and plen[q].item() == ol
        np.testing.assert_array_equal(wts.path_of(plan, paths, plen, q), op)
    wv = np.zeros(w.n)
    wv[pick] = [1.0, 2.0, 0.5, 1.5][:len(pick)]
    say("c3: weighted DBA update")
    B1, counts, d2 = wts.dba_iterate(plan, B0, Y, torch.from_numpy(wv).cuda())
    Bn, _, _, _ = oracle.dba_iterate(Bo, [cyc[q] for q in pick], wv[pick])
    np.testing.assert_array_equal(B1.cpu().numpy(), Bn)
    assert int(counts.sum().item()) == int(plen.sum().item())


@functools.lru_cache(maxsize=1)
def _config4():
    return synth.make(4)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("gamma,band", [(0.1, 0.0), (1.0, 0.0), (0.1, 0.6)])
def test_config4_full_soft_sampled(wts, gamma, band):
    """128 x 6 ch, 18000..22000, L = 20000, gamma in {0.1, 1}, and the Table I
    band of 0.6: values of sampled cycles and the gradient weighted onto
    them, within 1e-4."""
    import torch
    w = _config4()
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 6, dt, w.L, band=band)
    cyc = f64(w.cycles)
    pick = [5, 77]
    say("c4: Euclidean-mean init")
    B, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    Bo = oracle.euclid_mean(cyc, w.L)
    np.testing.assert_array_equal(B.cpu().numpy(), Bo)
    wv = np.zeros(w.n)
    wv[pick] = [1.0 / lens for lens in w.lengths[pick]]
    say("c4: Soft-DTW forward + backward on all 128 cycles, gamma", gamma)
    val, ck = wts.softdtw_forward(plan, B, Y, gamma)
    g, h = wts.softdtw_backward(plan, B, Y, gamma, ck, torch.from_numpy(wv).cuda(), with_mass=True)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    del ck
    say("c4: oracle on cycles", pick)
    ov, og, oh = oracle.softdtw_batch(Bo, [cyc[q] for q in pick], gamma, wv[pick], band=band)
    check_vec(val.cpu().numpy()[pick], ov)
    check_vec(g.cpu().numpy(), og)
    check_vec(h.cpu().numpy(), oh)


@pytest.mark.timeout(900)
def test_config4_full_grad_cycles_sampled(wts):
    """The gradient with respect to the cycles on all 128 cycles of the
    20000-sample workload (gamma 0.1, weights 1/m_k, the bench's call); the
    rows of two cycles checked against the oracle within 1e-4."""
    import torch
    w = _config4()
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 6, dt, w.L)
    cyc = f64(w.cycles)
    B, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    Bo = oracle.euclid_mean(cyc, w.L)
    wv = 1.0 / w.lengths.astype(np.float64)
    say("c4: gradient w.r.t. the cycles, all 128 cycles")
    g = wts.softdtw_grad_cycles(plan, B, Y.to(torch.float64), 0.1, torch.from_numpy(wv).cuda())
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    g = g.cpu().numpy()
    for q in (5, 77):
        say("c4: oracle gradient for cycle", q)
        _, want = oracle.softdtw_grad_y(Bo, cyc[q], 0.1)
        check_vec(g[off[q]:off[q + 1]], wv[q] * want)


@functools.lru_cache(maxsize=1)
def _config5():
    return synth.make(5)


@pytest.mark.timeout(900)
def test_config5_full_scores_sampled(wts):
    """256 x 6 ch, 40000..50000 with 1 % gaps, L = max N: scores of all cycles
    on the GPU, two of them checked against the oracle bit for bit."""
    import torch
    w = _config5()
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 6, dt, w.L)
    cyc = f64(w.cycles)
    pick = [3, int(np.argmin(w.lengths))]
    say("c5: nearest-length init + scores of 256 cycles")
    B, kn = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    score, dist, plen = wts.anomaly_score(plan, B, Y)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    ko, Bo = oracle.nearest_init(cyc, w.L)
    assert kn == ko
    say("c5: oracle on cycles", pick)
    os_, od, ol = oracle.score_batch(Bo, [cyc[q] for q in pick])
    np.testing.assert_array_equal(score.cpu().numpy()[pick], os_)
    np.testing.assert_array_equal(plen.cpu().numpy()[pick], ol)


@pytest.mark.timeout(900)
def test_config5_full_dba_and_soft(wts):
    """256 x 6 ch, 40000..50000 with 1 % gaps, L = max N (the DBA workspace is
    about 160 GB): one DBA iteration on all cycles weighted onto three of
    them, bit-exact against the oracle on those three; then one Soft-DTW
    (gamma 0.1) pass over checkpoint-bounded cycle groups, checked by
    properties that hold at any size: each value is at most the hard DTW of
    its cycle, each row mass is at least the sum of the weights (every path
    visits every row), and the eta = 1 update is a convex combination of
    samples."""
    import torch
    w = _config5()
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 6, dt, w.L)
    cyc = f64(w.cycles)
    lens = w.lengths
    pick = sorted({int(np.argmin(lens)), int(np.argmax(lens)), 100})
    B0, kn = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    say("c5: DBA iteration on 256 cycles, workspace %.1f GiB"
        % (plan.workspace_bytes(wts.OP_DBA) / 2 ** 30))
    wv = np.zeros(w.n)
    wv[pick] = [1.0, 0.5, 2.0][:len(pick)]
    B1, counts, dist = wts.dba_iterate(plan, B0, Y, torch.from_numpy(wv).cuda())
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    B1, counts, hard = B1.cpu().numpy(), counts.cpu().numpy(), dist.cpu().numpy()
    plan.close()
    torch.cuda.empty_cache()
    aplan = wts.Plan(off, 6, dt, w.L)
    _, plen, _ = wts.dtw_align(aplan, B0, Y, paths=False)
    plen = plen.cpu().numpy()
    assert aplan.status() == wts.OK
    aplan.close()
    assert int(counts.sum()) == int(plen.sum())
    assert (counts >= w.n).all()
    ko, Bo = oracle.nearest_init(cyc, w.L)
    assert kn == ko
    say("c5: oracle DBA on cycles", pick)
    Bn, _, od, _ = oracle.dba_iterate(Bo, [cyc[q] for q in pick], wv[pick])
    np.testing.assert_array_equal(B1, Bn)
    np.testing.assert_array_equal(hard[pick], od)
    torch.cuda.empty_cache()

    gamma = 0.1
    groups = wts.subset_plans(off, 6, dt, w.L, 48 << 30)
    say("c5: Soft-DTW forward + backward in %d groups" % len(groups))
    gv = torch.from_numpy(1.0 / lens.astype(np.float64)).cuda()
    sd = wts.SoftDescent(groups, Y, off, w.L, 6, gamma, gv, 1.0)
    B2 = B0.clone()
    sd.step(B2, check=True)
    for _, _, gp in groups:
        gp.close()
    v = sd.values.cpu().numpy()
    assert np.isfinite(v).all()
    assert (v <= hard + 1e-12 * np.abs(hard)).all(), np.max(v - hard)
    h = sd.H.cpu().numpy()
    assert (h >= (1.0 - 1e-4) * gv.sum().item()).all(), h.min()
    B2 = B2.cpu().numpy()
    yall = np.concatenate(cyc)
    lo, hi = yall.min(axis=0), yall.max(axis=0)
    tol = 1e-9 * (hi - lo)
    assert ((B2 >= lo - tol) & (B2 <= hi + tol)).all()


@pytest.mark.timeout(600)
def test_segmentation_robot_scale_sampled(wts):
    """The segmentation step at the scale of the paper's robot (reference of
    ~16k samples, a stream of 37 cycles, ~6e5 samples, 3 channels): the whole
    loop on the GPU, two of its rounds recomputed by the oracle bit for bit."""
    import torch
    lr = (15500, 16500)
    X, _, _ = synth.make_stream(500, 1, lr, 3, template_seed=31)
    _, Y, bounds = synth.make_stream(600, 37, lr, 3, template_seed=31)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    M, N = X.shape[0], Y.shape[0]
    say("segment: M = %d, N = %d" % (M, N))
    segs = wts.segment(torch.from_numpy(X64).cuda(),
                       [torch.from_numpy(np.ascontiguousarray(Y)).cuda()], "f32")[0]
    al = oracle.segment_alpha(M)
    ws = [0]
    for a, b, _ in segs[:-1]:
        bq = b - ws[-1]
        ws.append(ws[-1] + bq - al if bq - al > 0 else ws[-1] + bq + 1)
    for k in (0, len(segs) // 2):
        w0 = ws[k]
        say("segment: oracle on round", k, "window start", w0)
        v, a, b = oracle.subdtw(X64, Y64[w0:min(w0 + 2 * M, N)])
        assert segs[k] == (w0 + a, w0 + b, v)
    # sanity (not a parity gate): how many cycles were delimited within 2 %
    hits = sum(any(abs(a - lo) <= 0.02 * M and abs(b - hi) <= 0.02 * M for a, b, _ in segs)
               for lo, hi in bounds)
    say("segment: %d rounds, %d of %d cycles delimited within 2 %%" % (len(segs), hits, len(bounds)))


@pytest.mark.timeout(300)
def test_config5_longest_pair_softdtw_against_the_oracle(wts):
    """One full-size Soft-DTW pair of the 256-cycle workload against the
    oracle (gamma 0.1, no band): the Euclidean-mean barycenter at L = max N
    against the longest cycle, 49454 x 49454 cells -- the regime where the
    checkpointed backward has to carry E through tens of thousands of rows.
    The oracle's value, gradient and row mass (square-root checkpointing of
    R) are stored by tests/golden/make_c5_pair.py; the inputs are regenerated
    here from the seeded workload and checked against the stored hashes.
    Tolerances: 1e-4 relative (value), the vector bar on the gradient and
    the row mass."""
    import hashlib
    import os
    import torch
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden",
                               "c5_longest_pair_softdtw.npz"))
    w = _config5()
    k = int(ref["cycle"][0])
    assert k == int(np.argmax(w.lengths))
    Yk = np.asarray(w.cycles[k], dtype=np.float64)
    B = oracle.euclid_mean(f64(w.cycles), w.L)

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()
    assert sha(B) == str(ref["sha_b"]) and sha(Yk) == str(ref["sha_y"])
    gamma = float(ref["gamma"][0])
    Y, off, dt = wts.pack_cycles([w.cycles[k]])
    plan = wts.Plan(off, 6, dt, w.L)
    Bt = torch.from_numpy(B).cuda()
    say("c5 pair: Soft-DTW forward + backward, %d x %d" % (w.L, Yk.shape[0]))
    v, ck = wts.softdtw_forward(plan, Bt, Y, gamma)
    g, h = wts.softdtw_backward(plan, Bt, Y, gamma, ck, with_mass=True)
    assert plan.status() == wts.OK
    v = v.item()
    rv = float(ref["value"][0])
    assert abs(v - rv) <= 1e-4 * abs(rv), (v, rv)
    check_vec(g.cpu().numpy(), ref["grad"])
    check_vec(h.cpu().numpy(), ref["rowmass"])
