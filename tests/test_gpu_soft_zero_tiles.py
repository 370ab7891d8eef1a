"""The Soft-DTW backward's zero-tile skip (plan option dense_e = 0, the
default) against sweeping every tile (dense_e = 1): the same gradients, row
masses and cycle gradients bit for bit, on workloads whose E matrix is
mostly exactly zero (long similar cycles, small gamma) and on small random
ones, with and without a Sakoe-Chiba band; and parity with the oracle on a
case where most tiles are skipped.  E (Eq. 6) reaches a cell only through
its successors, so a tile that receives no push has e = 0 throughout."""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_vec(a, b, rtol=1e-4):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    scale = np.maximum(np.abs(b), 1e-2 * np.abs(b).max())
    assert (np.abs(a - b) <= rtol * scale).all(), np.max(np.abs(a - b) / scale)
    assert np.linalg.norm(a - b) <= rtol * np.linalg.norm(b)


def both(wts, off, d, dt, L, B, Y, gamma, gv, band=0.0, grid=0):
    """(values, grad, mass) of the skipping and the dense plan, and their tile counts."""
    import torch
    out = []
    for dense in (False, True):
        plan = wts.Plan(off, d, dt, L, band=band, grid=grid, dense_e=dense)
        v, ck = wts.softdtw_forward(plan, B, Y, gamma)
        plan.bwd_tiles()
        g, h = wts.softdtw_backward(plan, B, Y, gamma, ck, gv, with_mass=True)
        torch.cuda.synchronize()
        tiles = plan.bwd_tiles()
        assert plan.status() == wts.OK
        out.append((v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy(), tiles))
        plan.close()
        del ck
    return out


@pytest.mark.parametrize("gamma", [0.1, 1.0])
@pytest.mark.parametrize("band", [0.0, 0.6])
def test_skip_is_bitwise_dense_on_similar_cycles(wts, gamma, band):
    import torch
    w = synth.make(4, n=6, len_range=(2500, 3300), L=3000, seed=11)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, w.L)
    B, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    plan.close()
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    say("case zero tiles: 6 x 2500-3300, L 3000, gamma %g, band %g" % (gamma, band))
    (v0, g0, h0, t0), (v1, g1, h1, t1) = both(wts, off, w.d, dt, w.L, B, Y, gamma, gv, band)
    np.testing.assert_array_equal(v0, v1)
    np.testing.assert_array_equal(g0, g1)
    np.testing.assert_array_equal(h0, h1)
    assert t1[0] == t1[1] > 0                    # dense: every tile of every strip
    assert t0[1] == t1[1] and 0 < t0[0] < t0[1] // 2, (t0, t1)   # most tiles skipped


@pytest.mark.parametrize("L,lens,d", [(1, [1, 7], 1), (130, [1, 64, 300], 3),
                                      (257, [256, 129, 700], 6), (700, [500, 900], 8)])
def test_skip_is_bitwise_dense_on_random_series(wts, L, lens, d):
    import torch
    r = np.random.Generator(np.random.PCG64(L + 17 * d))
    Bn = r.standard_normal((L, d))
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
    Y, off, dt = wts.pack_cycles(cyc)
    B = torch.from_numpy(Bn).cuda()
    gv = torch.from_numpy(r.uniform(0.5, 2.0, len(lens))).cuda()
    for gamma in (0.01, 1.0):
        say("case zero tiles random L=%d lens=%s d=%d gamma=%g" % (L, lens, d, gamma))
        (v0, g0, h0, t0), (v1, g1, h1, t1) = both(wts, off, d, dt, L, B, Y, gamma, gv)
        np.testing.assert_array_equal(g0, g1)
        np.testing.assert_array_equal(h0, h1)
        assert t0[0] <= t0[1] == t1[1] == t1[0]


def test_skip_cycle_gradient_is_bitwise_dense(wts):
    import torch
    w = synth.make(4, n=4, len_range=(1800, 2400), L=2000, seed=5)
    Y, off, dt = wts.pack_cycles(w.cycles)
    Y64 = Y.to(torch.float64)
    gv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    outs = []
    for dense in (False, True):
        plan = wts.Plan(off, w.d, dt, w.L, dense_e=dense)
        B, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
        say("case zero tiles: cycle gradient dense_e=%d" % dense)
        plan.bwd_tiles()
        gy = wts.softdtw_grad_cycles(plan, B, Y64, 0.1, gv)
        torch.cuda.synchronize()
        outs.append((gy.cpu().numpy(), plan.bwd_tiles()))
        assert plan.status() == wts.OK
        plan.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    assert outs[0][1][0] < outs[0][1][1] == outs[1][1][0]


def test_skip_matches_the_oracle_where_most_tiles_are_zero(wts):
    import torch
    w = synth.make(4, n=2, len_range=(1500, 1800), L=1600, seed=23)
    Y, off, dt = wts.pack_cycles(w.cycles)
    plan = wts.Plan(off, w.d, dt, w.L)
    B, _ = wts.init_barycenter(plan, Y, wts.INIT_EUCLID_MEAN)
    wv = np.array([0.7, 1.3])
    say("case zero tiles vs oracle: 2 x 1500-1800, L 1600, gamma 0.1")
    v, ck = wts.softdtw_forward(plan, B, Y, 0.1)
    plan.bwd_tiles()
    g, h = wts.softdtw_backward(plan, B, Y, 0.1, ck, torch.from_numpy(wv).cuda(), with_mass=True)
    torch.cuda.synchronize()
    sw, tot = plan.bwd_tiles()
    assert plan.status() == wts.OK
    assert sw < tot // 2, (sw, tot)
    Bh = B.cpu().numpy()
    ov, og, oh = oracle.softdtw_batch(Bh, [np.asarray(c, np.float64) for c in w.cycles], 0.1, wv)
    check_vec(v.cpu().numpy(), ov)
    check_vec(g.cpu().numpy(), og)
    check_vec(h.cpu().numpy(), oh)
    plan.close()
