"""GPU parity of the DTW path (dtw_align, dba_iterate, anomaly_score, medoid,
init) against the FP64 oracle, through the C ABI.

The decision arithmetic on both sides is float64 with the same operation
order, so distances, path lengths, paths, alignment counts, DBA barycenters,
scores and medoid matrices must match BIT FOR BIT (paths and integer counts
must be exact and values within 1e-4 relative; these are held to 0 ulp).
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


def run_align(wts, B, cycles, dtype=None, paths=False, **kw):
    import torch
    Y, off, dt = wts.pack_cycles(cycles, dtype=dtype)
    plan = wts.Plan(off, B.shape[1], dt, B.shape[0], **kw)
    Bt = torch.from_numpy(np.ascontiguousarray(B, dtype=np.float64)).cuda()
    dist, plen, pth = wts.dtw_align(plan, Bt, Y, paths=paths)
    torch.cuda.synchronize()
    out = dist.cpu().numpy(), plen.cpu().numpy()
    if paths:
        out = out + ([wts.path_of(plan, pth, plen, k) for k in range(len(cycles))],)
    return out


# ------------------------------------------------------------------ DTW values

SHAPES = [  # (L, lengths): ragged tails, several strips (256 rows each at rho 4)
    (1, [1, 5, 64]),
    (5, [1, 2, 63, 64, 65]),
    (63, [17, 200]),
    (64, [64, 128]),
    (65, [300, 1]),
    (255, [256, 257]),
    (256, [100, 700]),
    (257, [513, 40]),
    (700, [1, 1000, 333, 64]),
]


@pytest.mark.parametrize("d", [1, 3, 6])
@pytest.mark.parametrize("L,lens", SHAPES)
def test_dtw_align_bitwise(wts, d, L, lens):
    r = rng(L * 131 + d)
    B = r.standard_normal((L, d))
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
    say("case dtw_align d=%d L=%d lens=%s" % (d, L, lens))
    dist, plen = run_align(wts, B, cyc)
    od, ol = oracle.dtw_batch(B, as64(cyc))
    np.testing.assert_array_equal(dist, od)
    np.testing.assert_array_equal(plen, ol)


@pytest.mark.parametrize("d", [1, 2, 6])
def test_dtw_paths_bitwise_with_ties(wts, d):
    # small integers: many tied optimal paths, the tie-break decides
    r = rng(7 + d)
    for L, lens in [(9, [7, 13, 1]), (300, [290, 310, 64, 600]), (520, [530])]:
        B = r.integers(0, 3, (L, d)).astype(np.float64)
        cyc = [r.integers(0, 3, (N, d)).astype(np.float64) for N in lens]
        say("case dtw_paths ties d=%d L=%d lens=%s" % (d, L, lens))
        dist, plen, paths = run_align(wts, B, cyc, dtype="f64", paths=True)
        for k, Y in enumerate(cyc):
            od, ol, op, _ = oracle.dtw(B, Y)
            assert dist[k] == od and plen[k] == ol
            np.testing.assert_array_equal(paths[k], op)


def test_dtw_paths_random_reals(wts):
    r = rng(11)
    B = r.standard_normal((777, 3))
    lens = [1, 64, 500, 777, 1500]
    cyc = [r.standard_normal((N, 3)).astype(np.float32) for N in lens]
    say("case dtw_paths reals")
    dist, plen, paths = run_align(wts, B, cyc, paths=True)
    for k, Y in enumerate(cyc):
        od, ol, op, _ = oracle.dtw(B, np.asarray(Y, np.float64))
        assert dist[k] == od and plen[k] == ol
        np.testing.assert_array_equal(paths[k], op)


def test_euclid_cost_bitwise(wts):
    r = rng(12)
    B = r.standard_normal((300, 3))
    cyc = [r.standard_normal((N, 3)) for N in (1, 100, 450)]
    say("case euclid")
    dist, plen = run_align(wts, B, cyc, dtype="f64", cost="euclid")
    od, ol = oracle.dtw_batch(B, cyc, kind=oracle.EUCLID)
    np.testing.assert_array_equal(dist, od)
    np.testing.assert_array_equal(plen, ol)


@pytest.mark.parametrize("rho,grid", [(2, 0), (4, 1), (4, 3), (2, 7), (5, 0), (5, 3)])
def test_tile_shape_and_grid_invariance(wts, rho, grid):
    r = rng(13)
    B = r.standard_normal((600, 2))
    cyc = [r.standard_normal((N, 2)).astype(np.float32) for N in (50, 900, 601, 2)]
    say("case invariance rho=%d grid=%d" % (rho, grid))
    d1, l1, p1 = run_align(wts, B, cyc, paths=True, rho=rho, grid=grid)
    d0, l0, p0 = run_align(wts, B, cyc, paths=True)
    np.testing.assert_array_equal(d1, d0)
    np.testing.assert_array_equal(l1, l0)
    for a, b in zip(p1, p0):
        np.testing.assert_array_equal(a, b)


def test_batch_order_and_single_launch_invariance(wts):
    r = rng(14)
    B = r.standard_normal((400, 3))
    cyc = [r.standard_normal((int(N), 3)).astype(np.float32) for N in r.integers(1, 900, 12)]
    say("case batch order")
    d0, l0 = run_align(wts, B, cyc)
    perm = r.permutation(len(cyc))
    d1, l1 = run_align(wts, B, [cyc[k] for k in perm])
    np.testing.assert_array_equal(d1, d0[perm])
    np.testing.assert_array_equal(l1, l0[perm])
    for k in (0, 5):
        ds, ls = run_align(wts, B, [cyc[k]])
        assert ds[0] == d0[k] and ls[0] == l0[k]


def test_repeat_runs_bitwise_identical(wts):
    r = rng(15)
    B = r.standard_normal((1000, 6))
    cyc = [r.standard_normal((N, 6)).astype(np.float32) for N in (1200, 800, 1000, 3)]
    say("case determinism")
    runs = [run_align(wts, B, cyc, paths=True) for _ in range(3)]
    for rr in runs[1:]:
        np.testing.assert_array_equal(rr[0], runs[0][0])
        for a, b in zip(rr[2], runs[0][2]):
            np.testing.assert_array_equal(a, b)


# -------------------------------------------------------------------- scores

def test_anomaly_score_bitwise(wts):
    import torch
    w = synth.make(2, n=6, len_range=(300, 500))
    B = np.asarray(w.cycles[0], np.float64)[:400] if w.cycles[0].shape[0] >= 400 else None
    r = rng(16)
    B = r.standard_normal((410, 3))
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 3, dt, 410)
    say("case score")
    score, dist, plen = wts.anomaly_score(plan, torch.from_numpy(B).cuda(), Y)
    os_, od, ol = oracle.score_batch(B, as64(w.cycles))
    np.testing.assert_array_equal(score.cpu().numpy(), os_)
    np.testing.assert_array_equal(dist.cpu().numpy(), od)
    np.testing.assert_array_equal(plen.cpu().numpy(), ol)


# ----------------------------------------------------------------------- DBA

def _dba_case(wts, w, B0, iters, weights=None, rho=0):
    import torch
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, B0.shape[0], rho=rho)
    Bg = torch.from_numpy(np.ascontiguousarray(B0)).cuda()
    Wt = None if weights is None else torch.from_numpy(np.asarray(weights, np.float64)).cuda()
    Bo = np.ascontiguousarray(B0)
    for it in range(iters):
        say("  dba iteration", it)
        Bg, counts, dist = wts.dba_iterate(plan, Bg, Y, Wt)
        Bn, K, od, ol = oracle.dba_iterate(Bo, as64(w.cycles), weights)
        np.testing.assert_array_equal(Bg.cpu().numpy(), Bn)
        np.testing.assert_array_equal(counts.cpu().numpy(), K)
        np.testing.assert_array_equal(dist.cpu().numpy(), od)
        Bo = Bn
        Bg = Bg.clone()


def test_dba_config1_full_medoid_init(wts):
    import torch
    w = synth.make(1)                      # 8 cycles, 200..256 samples, d = 1, f64
    Y, off, dt = wts.pack_cycles(w.cycles)
    mplan = wts.Plan(off, 1, dt, 0)
    say("case dba c1 medoid")
    k, Dm, tot = wts.medoid(mplan, Y)
    ko, Do = oracle.medoid(as64(w.cycles))
    assert int(k.item()) == ko
    np.testing.assert_array_equal(Dm.cpu().numpy(), Do)
    B0 = np.asarray(w.cycles[ko], np.float64)
    _dba_case(wts, w, B0, w.dba_iters)


def test_dba_uneven_several_strips_weighted(wts):
    w = synth.make(3, n=10, len_range=(60, 1500), L=700)
    _, B0 = oracle.nearest_init(as64(w.cycles), 700)
    say("case dba c3-like")
    _dba_case(wts, w, B0, 3)
    say("case dba c3-like weighted")
    _dba_case(wts, w, B0, 2, weights=np.linspace(0.5, 2.0, w.n))


def test_dba_and_score_five_rows_per_lane(wts):
    """5 rows per lane (320-row strips), the layout the plan picks by itself
    for batches whose strips would just about fill every SIMD."""
    import torch
    w = synth.make(3, n=7, len_range=(40, 1400), L=970)
    _, B0 = oracle.nearest_init(as64(w.cycles), 970)
    say("case dba rho 5")
    _dba_case(wts, w, B0, 2, rho=5)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, 970, rho=5)
    assert plan.rho(wts.OP_SCORE) == 5 and plan.rho(wts.OP_DBA) == 5
    say("case score rho 5")
    score, dist, plen = wts.anomaly_score(plan, torch.from_numpy(B0).cuda(), Y)
    os_, od, ol = oracle.score_batch(B0, as64(w.cycles))
    np.testing.assert_array_equal(score.cpu().numpy(), os_)
    np.testing.assert_array_equal(plen.cpu().numpy(), ol)


def test_dba_fixed_point(wts):
    import torch
    x = synth.dyadic(rng(17), (300, 3))
    Y, off, dt = wts.pack_cycles([x, x, x], dtype="f64")
    plan = wts.Plan(off, 3, dt, 300)
    say("case dba fixed point")
    Bo, K, dist = wts.dba_iterate(plan, torch.from_numpy(x).cuda(), Y)
    np.testing.assert_array_equal(Bo.cpu().numpy(), x)
    assert (K.cpu().numpy() == 3).all() and (dist.cpu().numpy() == 0).all()


# --------------------------------------------------------------------- init

def test_init_kinds_bitwise(wts):
    w = synth.make(4, n=5, len_range=(90, 140), L=120)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, 120)
    say("case init")
    b, k = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    np.testing.assert_array_equal(b.cpu().numpy(), oracle.euclid_mean(as64(w.cycles), 120))
    assert k == -1
    b, k = wts.init_barycenter(plan, Y, wts.INIT_NEAREST)
    ko, bo = oracle.nearest_init(as64(w.cycles), 120)
    assert k == ko
    np.testing.assert_array_equal(b.cpu().numpy(), bo)
    b, k = wts.init_barycenter(plan, Y, wts.INIT_COPY, 3)
    np.testing.assert_array_equal(b.cpu().numpy(), oracle.resample(as64(w.cycles)[3], 120))


@pytest.mark.parametrize("rho", [0, 2, 5])
def test_medoid_sampled_bitwise(wts, rho):
    w = synth.make(2, n=9, len_range=(200, 700))
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, 3, dt, 0, rho=rho)
    assert plan.rho(wts.OP_MEDOID) == (rho or 4)
    say("case medoid rho", rho)
    k, Dm, tot = wts.medoid(plan, Y)
    ko, Do = oracle.medoid(as64(w.cycles))
    np.testing.assert_array_equal(Dm.cpu().numpy(), Do)
    assert int(k.item()) == ko


# ----------------------------------------------------------- channel counts

@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_channel_count(wts, d):
    """Every kernel instance a plan can select (d = 1..8): paths, one DBA
    iteration, scores and the medoid bit for bit, on float32 cycles with a
    ragged tail and a one-sample cycle."""
    import torch
    r = rng(900 + d)
    L = 150
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in (1, 90, 300)]
    B = r.standard_normal((L, d))
    say("case channels d=%d" % d)
    dist, plen, paths = run_align(wts, B, cyc, paths=True)
    for k, Y in enumerate(cyc):
        od, ol, op, _ = oracle.dtw(B, np.asarray(Y, np.float64))
        assert dist[k] == od and plen[k] == ol
        np.testing.assert_array_equal(paths[k], op)
    Y, off, dt = wts.pack_cycles(cyc)
    plan = wts.Plan(off, d, dt, L)
    Bt = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    Bg, counts, dist = wts.dba_iterate(plan, Bt, Y)
    Bn, K, od, _ = oracle.dba_iterate(B, as64(cyc))
    np.testing.assert_array_equal(Bg.cpu().numpy(), Bn)
    np.testing.assert_array_equal(counts.cpu().numpy(), K)
    score, _, plen = wts.anomaly_score(plan, Bt, Y)
    os_, _, ol = oracle.score_batch(B, as64(cyc))
    np.testing.assert_array_equal(score.cpu().numpy(), os_)
    np.testing.assert_array_equal(plen.cpu().numpy(), ol)
    mplan = wts.Plan(off, d, dt, 0)
    k, Dm, _ = wts.medoid(mplan, Y)
    ko, Do = oracle.medoid(as64(cyc))
    np.testing.assert_array_equal(Dm.cpu().numpy(), Do)
    assert int(k.item()) == ko


# ------------------------------------------------------------------- graphs

def test_graph_replay_matches_eager(wts):
    import torch
    w = synth.make(3, n=6, len_range=(100, 900), L=500)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, 500)
    _, B0 = oracle.nearest_init(as64(w.cycles), 500)
    Bin = torch.from_numpy(B0).cuda()
    Bout = torch.empty_like(Bin)
    counts = torch.empty(500, dtype=torch.int64, device="cuda")
    dist = torch.empty(w.n, dtype=torch.float64, device="cuda")
    say("case graph: eager")
    wts.dba_iterate(plan, Bin, Y, bary_out=Bout, counts=counts, dist=dist)
    torch.cuda.synchronize()
    ref = Bout.clone(), counts.clone(), dist.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    say("case graph: capture")
    with torch.cuda.graph(g, stream=s):
        wts.dba_iterate(plan, Bin, Y, bary_out=Bout, counts=counts, dist=dist)
    for rep in range(3):
        say("case graph: replay", rep)
        Bout.zero_()
        counts.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Bout, ref[0]) and torch.equal(counts, ref[1])
        assert torch.equal(dist, ref[2])


def test_medoid_scores_and_paths_replay_from_a_captured_graph(wts):
    """The medoid, the scores and the path alignment captured in one HIP
    graph: every replay, with eager calls in between, matches the oracle bit
    for bit."""
    import torch
    w = synth.make(2, n=7, len_range=(150, 400))
    Y, off, dt = wts.pack_cycles(w.cycles)
    cyc = as64(w.cycles)
    ko, Do = oracle.medoid(cyc)
    L = int(w.lengths[ko])
    mplan = wts.Plan(off, 3, dt, 0)
    plan = wts.Plan(off, 3, dt, L)
    B = torch.from_numpy(np.ascontiguousarray(cyc[ko])).cuda()
    os_, od, ol = oracle.score_batch(cyc[ko], cyc)

    def calls():
        k, Dm, _ = wts.medoid(mplan, Y)
        score, _, plen = wts.anomaly_score(plan, B, Y)
        dist, plen2, pth = wts.dtw_align(plan, B, Y, paths=True)
        return k, Dm, score, plen, dist, plen2, pth

    def check(out):
        k, Dm, score, plen, dist, plen2, pth = out
        assert int(k.item()) == ko
        np.testing.assert_array_equal(Dm.cpu().numpy(), Do)
        np.testing.assert_array_equal(score.cpu().numpy(), os_)
        np.testing.assert_array_equal(plen.cpu().numpy(), ol)
        np.testing.assert_array_equal(dist.cpu().numpy(), od)
        np.testing.assert_array_equal(plen2.cpu().numpy(), ol)
        for q in (0, ko, w.n - 1):
            _, _, op, _ = oracle.dtw(cyc[ko], cyc[q])
            np.testing.assert_array_equal(wts.path_of(plan, pth, plen2, q), op)

    say("case graph dtw: eager")
    check(calls())
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    say("case graph dtw: capture")
    with torch.cuda.graph(g, stream=s):
        out = calls()
    torch.cuda.synchronize()
    for rep in range(3):
        say("case graph dtw: replay", rep)
        for t in out:
            t.fill_(-1)
        eager = calls()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(out)
        check(eager)
