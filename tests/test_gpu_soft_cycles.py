"""GPU parity of the Soft-DTW gradient with respect to the cycles (Eq. 6 for
the second series) against the FP64 oracle, through the C ABI.

The library computes it as the row gradient of Soft-DTW(C_k, B) (one forward
and one backward sweep with the cycles on the rows), the oracle as
sum_i e_ij 2 (c_kj - b_i) from its own E matrix of Soft-DTW(B, C_k).  The bar
is the Soft-DTW one: float32 base-2 exponentials on float64 differences, so
|a_k - b_k| <= 1e-4 max(|b_k|, 1e-2 ||b||_inf) per element and
||a - b||_2 <= 1e-4 ||b||_2.
"""

import sys

import numpy as np
import pytest

import oracle

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


def oracle_grad_cycles(B, cycles, gamma, w=None, band=0.0):
    """Packed [sum N][d]: w_k dSoft-DTW(B, C_k)/dC_k, cycle after cycle."""
    out = []
    for k, c in enumerate(cycles):
        _, g = oracle.softdtw_grad_y(B, c.astype(np.float64), gamma, band=band)
        out.append(g * (1.0 if w is None else w[k]))
    return np.concatenate(out, axis=0)


def setup(wts, B, cycles, dtype=None, band=0.0):
    import torch
    Y, off, dt = wts.pack_cycles(cycles, dtype=dtype)
    plan = wts.Plan(off, B.shape[1], dt, B.shape[0], band=band)
    return plan, torch.from_numpy(np.ascontiguousarray(B, dtype=np.float64)).cuda(), Y


# (L, cycle lengths): one and several strips of cycle rows (128 per strip),
# ragged tails, length-1 series on either side
SHAPES = [(1, [1, 7]), (7, [1, 64, 130]), (128, [127, 129]), (300, [129, 1]),
          (257, [300, 64, 513])]


@pytest.mark.parametrize("gamma", [0.1, 1.0])
@pytest.mark.parametrize("d", [1, 3, 6, 8])
@pytest.mark.parametrize("L,lens", SHAPES)
def test_grad_cycles_matches_oracle(wts, gamma, d, L, lens):
    import torch
    r = rng(L * 11 + d)
    B = r.standard_normal((L, d))
    cyc = [r.standard_normal((N, d)).astype(np.float32) for N in lens]
    w = r.uniform(0.5, 2.0, len(cyc))
    plan, Bt, Y = setup(wts, B, cyc)
    say("case grad-cycles d=%d L=%d lens=%s gamma=%g" % (d, L, lens, gamma))
    g = wts.softdtw_grad_cycles(plan, Bt, Y, gamma, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    assert plan.status() == wts.OK
    assert g.shape == (sum(lens), d) and g.dtype == torch.float64
    check_vec(g.cpu().numpy(), oracle_grad_cycles(B, cyc, gamma, w))


@pytest.mark.parametrize("band", [0.1, 0.3])
@pytest.mark.parametrize("L,lens", [(9, [1, 12, 40]), (200, [130, 260, 199]),
                                    (513, [300, 700])])
def test_grad_cycles_band_matches_oracle(wts, band, L, lens):
    r = rng(L + int(100 * band))
    B = r.standard_normal((L, 3))
    cyc = [r.standard_normal((N, 3)) for N in lens]
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64", band=band)
    say("case grad-cycles band=%g L=%d lens=%s" % (band, L, lens))
    g = wts.softdtw_grad_cycles(plan, Bt, Y, 0.5)
    check_vec(g.cpu().numpy(), oracle_grad_cycles(B, cyc, 0.5, band=band))


def test_grad_cycles_sums_with_bary_gradient_to_zero(wts):
    """Shifting the barycenter and every cycle by one vector leaves each value
    unchanged, so the barycenter gradient and the summed cycle gradients
    cancel (an identity between the two GPU backward paths)."""
    import torch
    r = rng(3)
    B = r.standard_normal((180, 4))
    cyc = [r.standard_normal((N, 4)) for N in (150, 210, 333)]
    w = np.array([0.7, 1.0, 1.9])
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64")
    wt = torch.from_numpy(w).cuda()
    _, ckpt = wts.softdtw_forward(plan, Bt, Y, 0.3)
    gb = wts.softdtw_backward(plan, Bt, Y, 0.3, ckpt, wt).cpu().numpy()
    gc = wts.softdtw_grad_cycles(plan, Bt, Y, 0.3, wt).cpu().numpy()
    tot = gb.sum(axis=0) + gc.sum(axis=0)
    # each side meets the 1e-4 relative bar, so the sum cancels to within it
    bound = RTOL * (np.abs(gb).sum(axis=0) + np.abs(gc).sum(axis=0))
    assert (np.abs(tot) <= bound).all(), (tot, bound)


def test_autograd_gradients_for_both_arguments(wts):
    import torch
    r = rng(4)
    B = r.standard_normal((70, 2))
    cyc = [r.standard_normal((N, 2)).astype(np.float32) for N in (50, 91)]
    plan, Bt, Y = setup(wts, B, cyc)
    b = Bt.clone().requires_grad_(True)
    y = Y.clone().requires_grad_(True)
    w = torch.tensor([1.5, 0.25], dtype=torch.float64, device="cuda")
    (wts.SoftDTW.apply(b, plan, y, 0.8) * w).sum().backward()
    assert y.grad.dtype == torch.float32 and y.grad.shape == Y.shape
    _, og, _ = oracle.softdtw_batch(B, [c.astype(np.float64) for c in cyc], 0.8, w.cpu().numpy())
    check_vec(b.grad.cpu().numpy(), og)
    check_vec(y.grad.cpu().numpy().astype(np.float64),
              oracle_grad_cycles(B, cyc, 0.8, w.cpu().numpy()), rtol=2e-4)
    # the cycles alone: no barycenter gradient is asked for
    y2 = Y.clone().requires_grad_(True)
    wts.SoftDTW.apply(Bt, plan, y2, 0.8).sum().backward()
    check_vec(y2.grad.cpu().numpy().astype(np.float64), oracle_grad_cycles(B, cyc, 0.8),
              rtol=2e-4)


def test_grad_cycles_repeat_and_workspace_reuse(wts):
    """Two calls on one plan (the workspace is reused, its queue and counters
    cleared by the call) give the same result, and a second plan with
    smaller inputs on the same device is unaffected."""
    import torch
    r = rng(5)
    B = r.standard_normal((260, 3))
    cyc = [r.standard_normal((N, 3)) for N in (400, 129, 257, 1)]
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64")
    a = wts.softdtw_grad_cycles(plan, Bt, Y, 1.0)
    b = wts.softdtw_grad_cycles(plan, Bt, Y, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan2, Bt2, Y2 = setup(wts, B[:40], cyc[1:3], dtype="f64")
    c = wts.softdtw_grad_cycles(plan2, Bt2, Y2, 1.0)
    check_vec(c.cpu().numpy(), oracle_grad_cycles(B[:40], cyc[1:3], 1.0))


def test_grad_cycles_many_cycles_sampled(wts):
    """64 cycles of 1.5k..2.5k samples against L = 2000 (many strips per
    cycle, more items than resident waves); three cycles checked in full."""
    import torch
    r = rng(6)
    lens = r.integers(1500, 2501, 64)
    B = r.standard_normal((2000, 6))
    cyc = [r.standard_normal((int(N), 6)).astype(np.float32) for N in lens]
    plan, Bt, Y = setup(wts, B, cyc)
    say("case grad-cycles 64 x 1.5k..2.5k, L=2000")
    g = wts.softdtw_grad_cycles(plan, Bt, Y, 1.0).cpu().numpy()
    off = np.concatenate([[0], np.cumsum(lens)])
    for k in (0, 31, 63):
        _, want = oracle.softdtw_grad_y(B, cyc[k].astype(np.float64), 1.0)
        check_vec(g[off[k]:off[k + 1]], want)


def test_grad_cycles_rejects_bad_arguments(wts):
    import torch
    B = np.zeros((4, 2))
    plan, Bt, Y = setup(wts, B, [np.zeros((5, 2))], dtype="f64")
    with pytest.raises(wts.WtsError):
        wts.softdtw_grad_cycles(plan, Bt, Y, 0.0)
    with pytest.raises(wts.WtsError):
        wts.softdtw_grad_cycles(plan, Bt, Y, float("inf"))
    mplan = wts.Plan([0, 5], 2, "f64", 0)   # medoid-only plan: no barycenter
    with pytest.raises(ValueError):         # the binding: a [0][2] barycenter is expected
        wts.softdtw_grad_cycles(mplan, Bt, Y, 1.0)
    # the C ABI itself refuses the plan before any launch
    import ctypes
    out = torch.empty_like(Y)
    ws = wts.aligned_buffer(1 << 16, "cuda:0")
    rc = wts.load().wts_softdtw_grad_cycles(mplan.handle, wts._ptr(Bt), wts._ptr(Y),
                                            ctypes.c_double(1.0), None, wts._ptr(out),
                                            wts._ptr(ws), ws.numel(), None)
    assert rc == wts.E_ARG
    assert torch.isfinite(wts.softdtw_grad_cycles(plan, Bt, Y, 1.0)).all()
    assert plan.rho(wts.OP_SOFT_GRAD_C) == plan.rho(wts.OP_SOFT_FWD) == 2
    assert plan.workspace_bytes(wts.OP_SOFT_GRAD_C) > 0
    assert mplan.workspace_bytes(wts.OP_SOFT_GRAD_C) == 0


def test_soft_calls_replay_from_a_captured_graph(wts):
    """Forward, backward and the cycles gradient captured in one HIP graph:
    every replay, with eager work on the same buffers in between, gives the
    eager results bit for bit (the sweeps are deterministic)."""
    import torch
    r = rng(8)
    B = r.standard_normal((300, 3))
    cyc = [r.standard_normal((N, 3)) for N in (257, 129, 400)]
    plan, Bt, Y = setup(wts, B, cyc, dtype="f64")
    wv = torch.tensor([0.5, 1.0, 2.0], dtype=torch.float64, device="cuda")

    def calls():
        v, ck = wts.softdtw_forward(plan, Bt, Y, 0.5)
        gb = wts.softdtw_backward(plan, Bt, Y, 0.5, ck, wv)
        gc = wts.softdtw_grad_cycles(plan, Bt, Y, 0.5, wv)
        return v, gb, gc

    say("case graph: eager")
    ref = [t.clone() for t in calls()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    say("case graph: capture")
    with torch.cuda.graph(g, stream=s):
        out = calls()
    torch.cuda.synchronize()
    for rep in range(3):
        say("case graph: replay", rep)
        for t in out:
            t.fill_(-1.0)
        eager = calls()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b, e in zip(out, ref, eager):
            assert torch.equal(a, b) and torch.equal(e, b)
