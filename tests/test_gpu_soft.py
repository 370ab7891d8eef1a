"""GPU parity of Soft-DTW forward and backward (Eq. 3-7) against the FP64 oracle.

Soft-DTW uses float32 base-2 exponentials/logarithms on float64 differences,
so it is not bit-exact: scalars must satisfy |a - b| <= 1e-4 |b| and vectors
both |a_k - b_k| <= 1e-4 max(|b_k|, 1e-2 ||b||_inf) per element and
||a - b||_2 <= 1e-4 ||b||_2 (a 1e-4 relative bar).
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2404_12134_amd import synth

pytestmark = pytest.mark.gpu
RTOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def check_vec(a, b, rtol=RTOL):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    scale = np.maximum(np.abs(b), 1e-2 * np.abs(b).max())
    assert (np.abs(a - b) <= rtol * scale).all(), np.max(np.abs(a - b) / scale)
    assert np.linalg.norm(a - b) <= rtol * np.linalg.norm(b)


def setup(wts, B, cycles, dtype=None, band=0.0):
    import torch
    Y, off, dt = wts.pack_cycles(cycles, dtype=dtype)
    plan = wts.Plan(off, B.shape[1], dt, B.shape[0], band=band)
    return plan, torch.from_numpy(np.ascontiguousarray(B, dtype=np.float64)).cuda(), Y


SHAPES = [(1, [1, 7]), (5, [1, 64, 130]), (127, [128, 129]), (129, [300, 1]),
          (300, [257, 64, 500])]


@pytest.mark.parametrize("gamma", [0.1, 1.0])
@pytest.mark.parametrize("d", [1, 3, 6, 8])
@pytest.mark.parametrize("L,lens", SHAPES)
def test_soft_forward_and_gradient(wts, gamma, d, L, lens):
    import torch
    r = rng(L * 7 + d)
    B = r.standard_normal((L, d))
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
    w = r.uniform(0.5, 2.0, len(cyc))
    plan, Bt, Y = setup(wts, B, cyc)
    say("case soft d=%d L=%d lens=%s gamma=%g" % (d, L, lens, gamma))
    val, ckpt = wts.softdtw_forward(plan, Bt, Y, gamma)
    grad, mass = wts.softdtw_backward(plan, Bt, Y, gamma, ckpt,
                                      torch.from_numpy(w).cuda(), with_mass=True)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    ov, og, oh = oracle.softdtw_batch(B, [c.astype(np.float64) for c in cyc], gamma, w)
    check_vec(val.cpu().numpy(), ov)
    check_vec(grad.cpu().numpy(), og)
    check_vec(mass.cpu().numpy(), oh)


def test_soft_config4_shaped(wts):
    # the C4 recipe at reduced size: 6 channels, Euclidean-mean barycenter
    import torch
    w = synth.make(4, n=4, len_range=(900, 1100), L=1000)
    cyc64 = [c.astype(np.float64) for c in w.cycles]
    B = oracle.euclid_mean(cyc64, 1000)
    plan, Bt, Y = setup(wts, B, w.cycles)
    for gamma in w.gammas:
        say("case soft c4-shaped gamma=%g" % gamma)
        val, ckpt = wts.softdtw_forward(plan, Bt, Y, gamma)
        wv = np.array([1.0 / c.shape[0] for c in w.cycles])   # Eq. 7: lambda_k / m_k
        grad, mass = wts.softdtw_backward(plan, Bt, Y, gamma, ckpt, torch.from_numpy(wv).cuda(),
                                          with_mass=True)
        ov, og, oh = oracle.softdtw_batch(B, cyc64, gamma, wv)
        check_vec(val.cpu().numpy(), ov)
        check_vec(grad.cpu().numpy(), og)
        check_vec(mass.cpu().numpy(), oh)


def test_soft_limits_match_dtw(wts):
    # single-row series: Soft-DTW equals the sum of costs; tiny gamma -> DTW
    import torch
    r = rng(3)
    b, Y1 = r.standard_normal((1, 2)), r.standard_normal((40, 2))
    plan, Bt, Y = setup(wts, b, [Y1], dtype="f64")
    val, _ = wts.softdtw_forward(plan, Bt, Y, 0.5)
    d0, _, _, _ = oracle.dtw(b, Y1, with_path=False)
    assert abs(val.item() - d0) <= 1e-12 * d0
    B2, Y2 = r.standard_normal((200, 3)), r.standard_normal((180, 3))
    plan, Bt, Y = setup(wts, B2, [Y2], dtype="f64")
    val, _ = wts.softdtw_forward(plan, Bt, Y, 1e-3)
    d2, _, _, _ = oracle.dtw(B2, Y2, with_path=False)
    assert abs(val.item() - d2) <= 1e-3 * 20 + 1e-4 * d2


def test_autograd_function_and_finite_differences(wts):
    import torch
    r = rng(4)
    B = r.standard_normal((150, 2))
    cyc = [r.standard_normal((N, 2)) for N in (140, 170)]
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64")
    Bp = Bt.clone().requires_grad_(True)
    wv = torch.tensor([0.7, 1.3], dtype=torch.float64, device="cuda")
    vals = wts.SoftDTW.apply(Bp, plan, Y, 1.0)
    (vals * wv).sum().backward()
    _, og, _ = oracle.softdtw_batch(B, cyc, 1.0, wv.cpu().numpy())
    check_vec(Bp.grad.cpu().numpy(), og)
    # directional finite difference of the GPU forward (loose: float32 exponentials)
    V = torch.from_numpy(r.standard_normal(B.shape)).cuda()
    h = 1e-3
    fp = (wts.softdtw_forward(plan, Bt + h * V, Y, 1.0)[0] * wv).sum().item()
    fm = (wts.softdtw_forward(plan, Bt - h * V, Y, 1.0)[0] * wv).sum().item()
    dd = (fp - fm) / (2 * h)
    an = float((Bp.grad * V).sum().item())
    assert abs(dd - an) <= 1e-3 * abs(an) + 1e-6


def test_soft_repeat_deterministic(wts):
    import torch
    r = rng(5)
    B = r.standard_normal((400, 3))
    cyc = [r.standard_normal((N, 3)).astype(np.float32) for N in (350, 420, 60)]
    plan, Bt, Y = setup(wts, B, cyc)
    outs = []
    for _ in range(2):
        v, ck = wts.softdtw_forward(plan, Bt, Y, 0.3)
        g = wts.softdtw_backward(plan, Bt, Y, 0.3, ck)
        torch.cuda.synchronize()
        outs.append((v.cpu().numpy(), g.cpu().numpy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_precond_step_is_the_soft_dba_update(wts):
    # b <- b - eta G / (2h); with eta = 1 this is sum_j e y_j / sum_j e per row
    import torch
    r = rng(6)
    B = r.standard_normal((260, 3))
    cyc = [r.standard_normal((N, 3)) for N in (250, 270)]
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64")
    for eta in (1.0, 0.5):
        Bg = Bt.clone()
        val, ck = wts.softdtw_forward(plan, Bg, Y, 0.5)
        g, h = wts.softdtw_backward(plan, Bg, Y, 0.5, ck, with_mass=True)
        wts.precond_step(Bg, g, h, eta)
        _, og, oh = oracle.softdtw_batch(B, cyc, 0.5)
        expect = B - eta * og / (2.0 * oh[:, None])
        check_vec(Bg.cpu().numpy(), expect)


def test_lbfgs_barycenter_converges_on_the_oracle_objective(wts):
    """Table I optimizer (L-BFGS, 40 iterations, 200 evaluations) driven by the
    GPU forward/backward: the objective it reports is the oracle's at the
    same points (1e-4), it decreases, and the oracle gradient at the result is
    far below the one at the start (a stationary point of the true
    objective)."""
    import torch
    w = synth.make(2, n=6, len_range=(90, 130), seed=8)
    cyc = [np.asarray(c, dtype=np.float64) for c in w.cycles]
    L = 110
    Bo = oracle.euclid_mean(cyc, L)
    plan, Bt, Y = setup(wts, Bo, cyc, dtype="f64")
    wv = torch.from_numpy(1.0 / w.lengths.astype(np.float64)).cuda()
    B, hist = wts.lbfgs_barycenter(plan, Y, Bt, 1.0, weights=wv)
    wn = wv.cpu().numpy()
    f0, g0, _ = oracle.softdtw_batch(Bo, cyc, 1.0, wn)
    f1, g1, _ = oracle.softdtw_batch(B.cpu().numpy(), cyc, 1.0, wn)
    F0, F1 = float(np.dot(wn, f0)), float(np.dot(wn, f1))
    assert abs(hist[0] - F0) <= 1e-4 * abs(F0)
    assert F1 < F0
    assert abs(min(hist) - F1) <= 1e-3 * abs(F1)
    # (the same optimizer on the oracle's own objective reduces the gradient
    # max-norm about 56-fold on this problem)
    assert np.abs(g1).max() <= 5e-2 * np.abs(g0).max()
    assert len(hist) <= 200 + 25



BAND_SHAPES = [  # (L, lengths): one and several strips, L above and below N, one-row /
    (1, [1, 9]),    # one-column pairs (the band keeps every cell)
    (37, [1, 64]),
    (40, [40, 25, 90]),
    (300, [260, 420, 7]),
    (700, [500, 900]),
]


@pytest.mark.parametrize("w", [0.6, 0.2, 0.03])
@pytest.mark.parametrize("L,lens", BAND_SHAPES)
def test_soft_band_matches_oracle(wts, w, L, lens):
    """Sakoe-Chiba band (Table I): values, gradient and row mass of the paths
    inside the band, within 1e-4 of the oracle."""
    import torch
    r = rng(int(1000 * w) + L)
    B = r.standard_normal((L, 3))
    cyc = [r.standard_normal((N, 3)) for N in lens]
    wv = r.uniform(0.5, 1.5, len(lens))
    for gamma, dtype in ((0.1, "f32"), (1.0, "f64")):
        say("soft band w=%g L=%d lens=%s gamma=%g %s" % (w, L, lens, gamma, dtype))
        cs = [np.asarray(c, dtype=np.float32 if dtype == "f32" else np.float64) for c in cyc]
        plan, Bt, Y = setup(wts, B, cs, dtype=dtype, band=w)
        val, ck = wts.softdtw_forward(plan, Bt, Y, gamma)
        g, h = wts.softdtw_backward(plan, Bt, Y, gamma, ck, torch.from_numpy(wv).cuda(),
                                    with_mass=True)
        torch.cuda.synchronize()
        assert plan.status() == wts.OK
        c64 = [np.asarray(c, dtype=np.float64) for c in cs]
        ov, og, oh = oracle.softdtw_batch(B, c64, gamma, wv, band=w)
        check_vec(val.cpu().numpy(), ov)
        check_vec(g.cpu().numpy(), og)
        check_vec(h.cpu().numpy(), oh)


@pytest.mark.parametrize("d,L,lens", [(2, 300, (280, 333)), (6, 1200, (1100, 1500, 640))])
def test_soft_wide_band_is_bitwise_unbanded(wts, d, L, lens):
    """A band wider than every pair keeps every cell: the banded kernels then
    compute exactly the unbanded bits (the forward's groups inside the band
    take the unbanded arithmetic, the others the band test's)."""
    import torch
    r = rng(71 + d)
    B = r.standard_normal((L, d))
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
    outs = []
    for band in (0.0, 10.0):
        say("soft wide band d=%d L=%d lens=%s band=%g" % (d, L, lens, band))
        plan, Bt, Y = setup(wts, B, cyc, band=band)
        v, ck = wts.softdtw_forward(plan, Bt, Y, 0.5)
        g, h = wts.softdtw_backward(plan, Bt, Y, 0.5, ck, with_mass=True)
        torch.cuda.synchronize()
        outs.append((v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy()))
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("w", [0.3, 0.05])
def test_soft_band_six_channels_matches_oracle(wts, w):
    """The six-channel banded instance over several strips, with groups
    inside, across and outside the band: values, gradient and row mass
    within 1e-4 of the oracle."""
    import torch
    r = rng(int(1000 * w) + 6)
    B = r.standard_normal((900, 6))
    cyc = [r.standard_normal((N, 6)).astype(np.float32) for N in (800, 1000, 450)]
    wv = r.uniform(0.5, 1.5, 3)
    say("soft band six channels w=%g" % w)
    plan, Bt, Y = setup(wts, B, cyc, band=w)
    val, ck = wts.softdtw_forward(plan, Bt, Y, 0.1)
    g, h = wts.softdtw_backward(plan, Bt, Y, 0.1, ck, torch.from_numpy(wv).cuda(), with_mass=True)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    ov, og, oh = oracle.softdtw_batch(B, [np.asarray(c, np.float64) for c in cyc], 0.1, wv, band=w)
    check_vec(val.cpu().numpy(), ov)
    check_vec(g.cpu().numpy(), og)
    check_vec(h.cpu().numpy(), oh)


@pytest.mark.parametrize("offset", [1e3, 1e6])
def test_soft_large_offset_matches_oracle(wts, offset):
    """Series far from the origin: the kernels form the cost as an expanded
    square around the pair's first row, so a common offset of 1e6 (where
    |x|^2 would be 1e12 times the costs) still meets the 1e-4 bar."""
    import torch
    r = rng(int(offset) % 1000 + 3)
    B = offset + r.standard_normal((200, 3))
    cyc = [offset + r.standard_normal((N, 3)) for N in (180, 233)]
    wv = np.array([1.0, 0.5])
    say("soft offset %g" % offset)
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64")
    val, ck = wts.softdtw_forward(plan, Bt, Y, 0.5)
    g, h = wts.softdtw_backward(plan, Bt, Y, 0.5, ck, torch.from_numpy(wv).cuda(), with_mass=True)
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    ov, og, oh = oracle.softdtw_batch(B, cyc, 0.5, wv)
    check_vec(val.cpu().numpy(), ov)
    check_vec(g.cpu().numpy(), og)
    check_vec(h.cpu().numpy(), oh)
