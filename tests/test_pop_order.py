"""The persistent sweeps' pop order (csrc/wts_order.h), built with the host
compiler and checked on the CPU: every strip exactly once, every strip after
the neighbour it waits on (no deadlock whatever the completion order), keys
non-increasing (the critical-path list schedule), and hand-derived orders."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2404_12134_amd", "csrc")
SPACING = 800   # kStripSpacing


@pytest.fixture(scope="module")
def pop_bin(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("pop") / "pop_order")
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "pop_order_main.cpp"),
                    "-o", exe], check=True)
    return exe


def order(exe, cols, strips, reverse):
    inp = "%d %d\n%s\n%s\n" % (len(cols), int(reverse), " ".join(map(str, cols)),
                               " ".join(map(str, strips)))
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [tuple(map(int, ln.split())) for ln in out.splitlines()]


def key(cols, strips, q, s, reverse):
    k = (strips[q] - 1 - s) if reverse else s   # position in the pair's own order
    return cols[q] + (strips[q] - 1 - k) * SPACING


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("reverse", [False, True])
def test_complete_ordered_and_keyed(pop_bin, seed, reverse):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 200))
    cols = rng.integers(64, 30000, n).tolist()
    strips = rng.integers(0, 50, n).tolist()
    if seed % 3 == 0:          # many equal pairs: ties everywhere
        cols = [20064] * n
    got = order(pop_bin, cols, strips, reverse)
    assert sorted(got) == sorted((q, s) for q in range(n) for s in range(strips[q]))
    nxt = [strips[q] - 1 if reverse else 0 for q in range(n)]
    for q, s in got:           # each pair's strips in its own sweep order
        assert s == nxt[q]
        nxt[q] += -1 if reverse else 1
    keys = [key(cols, strips, q, s, reverse) for q, s in got]
    assert all(a >= b for a, b in zip(keys, keys[1:]))


def test_long_pair_first_then_interleave(pop_bin):
    # A 20k-column pair heads chains longer than any strip of the 1k pairs:
    # all three of its strips go first, then the two equal short pairs
    # interleave strip by strip (ties: earlier strip, then lower pair).
    cols, strips = [1064, 20064, 1064], [3, 3, 3]
    assert order(pop_bin, cols, strips, False) == [
        (1, 0), (1, 1), (1, 2), (0, 0), (2, 0), (0, 1), (2, 1), (0, 2), (2, 2)]
    assert order(pop_bin, cols, strips, True) == [
        (1, 2), (1, 1), (1, 0), (0, 2), (2, 2), (0, 1), (2, 1), (0, 0), (2, 0)]


def test_spacing_lets_a_longer_chain_lead(pop_bin):
    # Pair 0: 2000 columns, 4 strips (chain keys 4400, 3600, 2800, 2000);
    # pair 1: 3000 columns, 1 strip (key 3000) lands between 3600 and 2800.
    assert order(pop_bin, [2000, 3000], [4, 1], False) == [(0, 0), (0, 1), (1, 0), (0, 2), (0, 3)]


def test_empty(pop_bin):
    assert order(pop_bin, [], [], False) == []
    assert order(pop_bin, [500, 700], [0, 0], True) == []
