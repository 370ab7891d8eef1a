"""GPU parity of the float32-decision sweeps (plan decision "fp32") against
the oracle's float32 program, through the C ABI.

With decision = fp32 the sweeps evaluate the cost, the minima and the argmin
codes in float32 on the float32 cycles and the barycenter rounded to float32
(one rounding, to nearest), in the same operation order as the oracle's
float32 program (the same C source as its float64 one).  Distances, path
lengths, paths, DBA barycenters (whose sums stay float64), counts, scores,
medoid matrices and Sub-DTW (value, a*, b*) must match it BIT FOR BIT.
Against the float64 decisions the values are gated by a float32 rounding
bound, and the paths that differ (near-ties that float32 resolves the other
way) are counted and reported.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def as64(cycles):
    return [np.asarray(c, dtype=np.float64) for c in cycles]


def plan_of(wts, cycles, d, L, **kw):
    Y, off, dt = wts.pack_cycles(cycles, dtype="f32")
    return wts.Plan(off, d, dt, L, decision="fp32", **kw), Y


SHAPES = [  # (L, lengths): ragged tails, one and several strips, one-sample series
    (1, [1, 5, 64]),
    (63, [17, 200]),
    (65, [300, 1]),
    (257, [513, 40]),
    (700, [1, 1000, 333, 64]),
]


@pytest.mark.parametrize("rho", [2, 4, 5])
@pytest.mark.parametrize("d", [1, 3, 6, 8])
@pytest.mark.parametrize("L,lens", SHAPES)
def test_fp32_align_paths_bitwise(wts, d, rho, L, lens):
    import torch
    r = rng(L * 17 + d * 3 + rho)
    B = r.standard_normal((L, d))
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
    plan, Y = plan_of(wts, cyc, d, L, rho=rho)
    say("case fp32 align d=%d rho=%d L=%d lens=%s" % (d, rho, L, lens))
    dist, plen, pth = wts.dtw_align(plan, torch.from_numpy(B).cuda(), Y, paths=True)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    dist, plen = dist.cpu().numpy(), plen.cpu().numpy()
    for k, c in enumerate(cyc):
        od, ol, op, _ = oracle.dtw32(B, c)
        assert dist[k] == od and plen[k] == ol, (k, dist[k], od)
        np.testing.assert_array_equal(wts.path_of(plan, pth, torch.from_numpy(plen), k), op)


@pytest.mark.parametrize("rho", [2, 4, 5])
def test_fp32_dba_and_scores_bitwise(wts, rho):
    import torch
    w = synth.make(3, n=9, len_range=(60, 1500), L=700)
    cyc = [np.asarray(c, np.float32) for c in w.cycles]
    _, B0 = oracle.nearest_init(as64(cyc), 700)
    plan, Y = plan_of(wts, cyc, w.d, 700, rho=rho)
    wt = np.linspace(0.5, 2.0, w.n)
    Bg = torch.from_numpy(B0).cuda()
    Bo = B0
    for it, weights in enumerate((None, wt, None)):
        say("case fp32 dba rho=%d iteration %d" % (rho, it))
        Wt = None if weights is None else torch.from_numpy(weights).cuda()
        Bg, counts, dist = wts.dba_iterate(plan, Bg, Y, Wt)
        Bn, K, od, _ = oracle.dba_iterate(Bo, as64(cyc), weights, fp32=True)
        np.testing.assert_array_equal(Bg.cpu().numpy(), Bn)
        np.testing.assert_array_equal(counts.cpu().numpy(), K)
        np.testing.assert_array_equal(dist.cpu().numpy(), od)
        Bo, Bg = Bn, Bg.clone()
    say("case fp32 scores rho=%d" % rho)
    score, dist, plen = wts.anomaly_score(plan, torch.from_numpy(Bo).cuda(), Y)
    os_, od, ol = oracle.score_batch(Bo, as64(cyc), fp32=True)
    np.testing.assert_array_equal(score.cpu().numpy(), os_)
    np.testing.assert_array_equal(dist.cpu().numpy(), od)
    np.testing.assert_array_equal(plen.cpu().numpy(), ol)
    assert plan.status() == wts.OK


@pytest.mark.parametrize("rho", [0, 2, 5])
def test_fp32_medoid_bitwise(wts, rho):
    w = synth.make(2, n=9, len_range=(200, 700))
    cyc = [np.asarray(c, np.float32) for c in w.cycles]
    plan, Y = plan_of(wts, cyc, 3, 0, rho=rho)
    say("case fp32 medoid rho", rho)
    k, Dm, tot = wts.medoid(plan, Y)
    ko, Do = oracle.medoid(as64(cyc), fp32=True)
    np.testing.assert_array_equal(Dm.cpu().numpy(), Do)
    assert int(k.item()) == ko


@pytest.mark.parametrize("d", [1, 3, 6, 8])
def test_fp32_subdtw_bitwise(wts, d):
    import torch
    r = rng(60 + d)
    for M, lens in [(5, [1, 2, 40, 65]), (200, [400, 399, 1, 64]), (257, [514, 600])]:
        X = r.standard_normal((M, d))
        wins = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
        plan, Y = plan_of(wts, wins, d, M)
        say("case fp32 subdtw d=%d M=%d" % (d, M))
        v, a, b = wts.subdtw(plan, torch.from_numpy(X).cuda(), Y)
        torch.cuda.synchronize()
        ov, oa, ob = oracle.subdtw_batch(X, as64(wins), fp32=True)
        np.testing.assert_array_equal(v.cpu().numpy(), ov)
        np.testing.assert_array_equal(a.cpu().numpy(), oa)
        np.testing.assert_array_equal(b.cpu().numpy(), ob)


def test_fp32_ties_equal_fp64_on_exact_inputs(wts):
    """Small integers (every cost and sum exact in float32, many tied paths):
    the float32 sweeps reproduce the float64 ones bit for bit."""
    import torch
    r = rng(71)
    for L, lens in [(9, [7, 13, 1]), (300, [290, 310, 64, 600])]:
        B = r.integers(0, 3, (L, 2)).astype(np.float64)
        cyc = [r.integers(0, 3, (N, 2)).astype(np.float32) for N in lens]
        Y, off, dt = wts.pack_cycles(cyc, dtype="f32")
        out = []
        for dec in ("fp64", "fp32"):
            plan = wts.Plan(off, 2, dt, L, decision=dec)
            dist, plen, pth = wts.dtw_align(plan, torch.from_numpy(B).cuda(), Y, paths=True)
            Bo, K, _ = wts.dba_iterate(plan, torch.from_numpy(B).cuda(), Y)
            torch.cuda.synchronize()
            paths = [wts.path_of(plan, pth, plen, k) for k in range(len(cyc))]
            out.append((dist.cpu().numpy(), plen.cpu().numpy(), Bo.cpu().numpy(),
                        K.cpu().numpy()) + tuple(paths))
        say("case fp32 = fp64 on exact inputs L=%d" % L)
        for u, v in zip(*out):
            np.testing.assert_array_equal(u, v)


def test_fp32_against_fp64_rounding_bound_and_path_flips(wts):
    """Against float64 decisions: each value is within the float32 rounding
    of the float64 one -- a path sum of |pi| cells, each cost of d channels,
    carries at most (|pi| + 2d + 2) float32 roundings of at most 2^-24 of the
    running magnitude -- and the share of paths that float32 resolves
    differently is reported (not gated)."""
    import torch
    w = synth.make(2, n=64, len_range=(800, 1200))
    cyc = [np.asarray(c, np.float32) for c in w.cycles]
    r = rng(72)
    B = oracle.resample(np.asarray(cyc[0], np.float64), 1000) + 0.01 * r.standard_normal((1000, 3))
    Y, off, dt = wts.pack_cycles(cyc, dtype="f32")
    res = {}
    for dec in ("fp64", "fp32"):
        plan = wts.Plan(off, 3, dt, 1000, decision=dec)
        dist, plen, pth = wts.dtw_align(plan, torch.from_numpy(B).cuda(), Y, paths=True)
        torch.cuda.synchronize()
        res[dec] = (dist.cpu().numpy(), plen.cpu().numpy(),
                    [wts.path_of(plan, pth, plen, k) for k in range(len(cyc))])
    d64, l64, p64 = res["fp64"]
    d32, l32, p32 = res["fp32"]
    bound = (np.maximum(l64, l32) + 2 * 3 + 2) * 2.0 ** -24 * d64
    assert (np.abs(d32 - d64) <= bound).all(), np.max(np.abs(d32 - d64) / np.maximum(d64, 1e-30))
    flips = sum(not np.array_equal(a, b) for a, b in zip(p64, p32))
    say("fp32 vs fp64: max rel diff %.3g, paths that differ %d of %d"
        % (np.max(np.abs(d32 - d64) / d64), flips, len(cyc)))


def test_fp32_sampled_at_the_512_cycle_size(wts):
    """The 512-cycle workload (log-uniform 1k..20k samples, L = 10000): one
    float32-decision DBA iteration; three cycles, the longest included,
    checked against the oracle's float32 program (distance, path length, and
    the rows' sums through the scores), the rest by properties."""
    import torch
    w = synth.make(3)
    cyc = [np.asarray(c, np.float32) for c in w.cycles]
    k0, B0 = oracle.nearest_init(as64(cyc), w.L)
    plan, Y = plan_of(wts, cyc, w.d, w.L)
    say("case fp32 512-cycle dba")
    Bg, counts, dist = wts.dba_iterate(plan, torch.from_numpy(B0).cuda(), Y)
    score, d2, plen = wts.anomaly_score(plan, torch.from_numpy(B0).cuda(), Y)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    dist, d2, plen = dist.cpu().numpy(), d2.cpu().numpy(), plen.cpu().numpy()
    np.testing.assert_array_equal(dist, d2)
    longest = int(np.argmax(w.lengths))
    for k in sorted({0, 257, longest}):
        say("  cycle", k, "N =", int(w.lengths[k]))
        od, ol = oracle.dtw_batch(B0, [cyc[k].astype(np.float64)], fp32=True)
        assert dist[k] == od[0] and plen[k] == ol[0]
    K = counts.cpu().numpy()
    assert (K >= w.n).all() and K.sum() == plen.sum()
    assert np.isfinite(Bg.cpu().numpy()).all()


def test_fp32_segmentation_matches_the_float32_oracle_loop(wts):
    """The segmentation loop of Sec. III-B with float32-decision plans: the
    same cycles, in the same order, with the same costs as the oracle's loop
    run with its float32 Sub-DTW on each stream alone."""
    import torch
    X, _, _ = synth.make_stream(11, 1, (190, 210), 3, dtype="f32", template_seed=7)
    Xd = X.astype(np.float64)
    streams = [synth.make_stream(seed, n, (190, 210), 3, dtype="f32", template_seed=7)[1]
               for seed, n in ((31, 8), (32, 11))]
    say("case fp32 segmentation")
    dev = [torch.from_numpy(np.ascontiguousarray(Y)).cuda() for Y in streams]
    got = wts.segment(torch.from_numpy(Xd).cuda(), dev, "f32", decision="fp32")
    for Y, g in zip(streams, got):
        assert g == oracle.segment(Xd, Y.astype(np.float64), fp32=True)
        assert len(g) >= 3


@pytest.mark.timeout(900)
def test_fp32_dba_at_the_256_cycle_size_sampled(wts):
    """The 256-cycle workload (40k..50k samples, 1 % gaps, L = max N) in the
    launch configuration the bench times for float32 decisions (4 rows per
    lane): one DBA iteration weighted onto two cycles (the shortest and the
    longest), bit for bit the oracle's float32 program on those two; the
    unweighted counts match the float32 path lengths of all cycles."""
    import torch
    w = synth.make(5)
    cyc = [np.asarray(c, np.float32) for c in w.cycles]
    lens = w.lengths
    pick = sorted({int(np.argmin(lens)), int(np.argmax(lens))})
    plan, Y = plan_of(wts, cyc, w.d, w.L, rho=4)
    B0, kn = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    wv = np.zeros(w.n)
    wv[pick] = [1.0, 0.5][:len(pick)]
    say("case fp32 256-cycle DBA, workspace %.1f GiB" % (plan.workspace_bytes(wts.OP_DBA) / 2 ** 30))
    B1, counts, dist = wts.dba_iterate(plan, B0, Y, torch.from_numpy(wv).cuda())
    score, d2, plen = wts.anomaly_score(plan, B0, Y)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    B1, counts, dist = B1.cpu().numpy(), counts.cpu().numpy(), dist.cpu().numpy()
    plen = plen.cpu().numpy()
    np.testing.assert_array_equal(dist, d2.cpu().numpy())
    assert int(counts.sum()) == int(plen.sum()) and (counts >= w.n).all()
    plan.close()
    torch.cuda.empty_cache()
    ko, Bo = oracle.nearest_init(as64(cyc), w.L)
    assert kn == ko
    say("case fp32 256-cycle DBA: oracle on cycles", pick)
    Bn, _, od, ol = oracle.dba_iterate(Bo, [as64(cyc)[q] for q in pick], wv[pick], fp32=True)
    np.testing.assert_array_equal(B1, Bn)
    np.testing.assert_array_equal(dist[pick], od)
    np.testing.assert_array_equal(plen[pick], ol)


def test_fp32_graph_replay_noalloc_and_validation(wts):
    """The float32-decision sweeps under the other call forms: a DBA
    iteration and the scores captured in one HIP graph and replayed three
    times between eager calls (bit for bit), the scratch-buffer score entry
    point against the allocating one, and a validated plan that refuses a
    NaN sample before any sweep."""
    import torch
    r = rng(80)
    B = r.standard_normal((300, 3))
    cyc = [r.standard_normal((N, 3)).astype(np.float32) for N in (257, 129, 400, 1)]
    plan, Y = plan_of(wts, cyc, 3, 300)
    Bt = torch.from_numpy(B).cuda()
    Bo = torch.empty_like(Bt)
    K = torch.empty(300, dtype=torch.int64, device="cuda")
    dd = torch.empty(4, dtype=torch.float64, device="cuda")

    def calls():
        wts.dba_iterate(plan, Bt, Y, bary_out=Bo, counts=K, dist=dd)
        return wts.anomaly_score(plan, Bt, Y)

    say("case fp32 graph: eager")
    ref = [t.clone() for t in (Bo, K, dd) + tuple(calls())]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        outs = calls()
    torch.cuda.synchronize()
    for rep in range(3):
        say("case fp32 graph: replay", rep)
        calls()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((Bo, K, dd) + tuple(outs), ref):
            assert torch.equal(a, b)
    Bn, Kn, od, _ = oracle.dba_iterate(B, as64(cyc), fp32=True)
    np.testing.assert_array_equal(Bo.cpu().numpy(), Bn)
    say("case fp32 noalloc")
    s1, d1, l1 = wts.anomaly_score(plan, Bt, Y)
    s2, d2, l2 = wts.anomaly_score_noalloc(plan, Bt, Y, dist=torch.empty_like(d1),
                                           path_len=torch.empty_like(l1))
    torch.cuda.synchronize()
    assert torch.equal(s1, s2) and torch.equal(d1, d2) and torch.equal(l1, l2)
    say("case fp32 validate")
    bad = [c.copy() for c in cyc]
    bad[2][17, 1] = np.nan
    vplan, Yb = plan_of(wts, bad, 3, 300, validate=True)
    wts.anomaly_score(vplan, Bt, Yb)
    torch.cuda.synchronize()
    assert vplan.status() == wts.E_NONFINITE
    assert vplan.status() == wts.OK          # the status word is cleared by the read
