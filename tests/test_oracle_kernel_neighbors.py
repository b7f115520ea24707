"""Pins of the oracle's kernel, random numbers and neighbour search.

Every expected value here comes from mathematics (normalisation, finite
differences, brute force) or from a published reference sequence; none is
produced by the code under test.
"""
import os

import numpy as np
import pytest
from scipy import integrate

from tests.helpers import block_case

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("h", [0.013, 0.37, 2.1])
def test_kernel_is_normalised(ora, dim, h):
    # Sec. 2.2: W is a smoothing kernel, so its integral over its support is 1.
    if dim == 2:
        f = lambda r: 2.0 * np.pi * r * ora.kernel_W(r, h, 2)
    else:
        f = lambda r: 4.0 * np.pi * r * r * ora.kernel_W(r, h, 3)
    val, _ = integrate.quad(f, 0.0, 2.0 * h, epsabs=0.0, epsrel=1e-13, limit=400)
    assert abs(val - 1.0) < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_derivative_matches_finite_differences(ora, dim):
    h = 0.5
    for r in np.linspace(0.03, 0.97, 17):
        e = 1e-6
        fd = (ora.kernel_W(r + e, h, dim) - ora.kernel_W(r - e, h, dim)) / (2 * e)
        dW = ora.kernel_dW(r, h, dim)
        assert abs(dW - fd) <= 1e-7 * max(1.0, abs(fd))
        assert dW < 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_compact_support_and_smoothness(ora, dim):
    h = 0.5
    assert ora.kernel_W(2 * h, h, dim) == 0.0
    assert ora.kernel_W(3 * h, h, dim) == 0.0
    assert ora.kernel_dW(2 * h, h, dim) == 0.0
    # C2 at the cut-off: W ~ (2h - r)^4 and W' ~ (2h - r)^3 on approach
    e = 1e-3
    r1, r2 = 2 * h - e, 2 * h - 2 * e
    ratio = ora.kernel_W(r2, h, dim) / ora.kernel_W(r1, h, dim)
    assert abs(ratio - 16.0) < 0.1
    ratio_d = ora.kernel_dW(r2, h, dim) / ora.kernel_dW(r1, h, dim)
    assert abs(ratio_d - 8.0) < 0.05
    # dW/dr vanishes at r = 0 (smooth peak)
    assert abs(ora.kernel_dW(0.0, h, dim)) == 0.0


def test_splitmix64_reference_sequence(ora):
    vals = [int(l) for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    g = 0x9E3779B97F4A7C15
    got = [ora.splitmix64((1234567 + k * g) % 2 ** 64) for k in range(5)]
    assert got == vals


def test_uniform_counter_rng_range_and_moments(ora):
    u = np.array([ora.uniform(42, pid, step, 0) for pid in range(200)
                  for step in range(50)])
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.03
    assert abs(u.var() - 1.0 / 3.0) < 0.02
    # counter-based: same counter, same number; any counter field changes it
    assert ora.uniform(1, 2, 3, 0) == ora.uniform(1, 2, 3, 0)
    assert ora.uniform(1, 2, 3, 0) != ora.uniform(1, 2, 3, 1)
    assert ora.uniform(1, 2, 3, 0) != ora.uniform(1, 2, 4, 0)
    assert ora.uniform(1, 2, 3, 0) != ora.uniform(1, 3, 3, 0)
    assert ora.uniform(1, 2, 3, 0) != ora.uniform(2, 2, 3, 0)


def _sets(off, idx):
    return [set(idx[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1)]


@pytest.mark.parametrize("dim,n_side,jit", [(2, 14, 0.0), (2, 14, 0.45),
                                             (3, 7, 0.0), (3, 7, 0.45)])
def test_cell_list_equals_brute_force(ora, dim, n_side, jit):
    c = block_case(dim=dim, n_side=n_side, jitter=jit, seed=3, walls=True)
    ob, ib = ora.neighbors(c.params, c.x, brute=True)
    oc, ic = ora.neighbors(c.params, c.x, brute=False)
    assert _sets(ob, ib) == _sets(oc, ic)
    assert len(ib) > 0
    # symmetric relation, no self pairs
    S = _sets(ob, ib)
    for i, s in enumerate(S):
        assert i not in s
        for j in s:
            assert i in S[j]


def test_cutoff_is_strict(ora):
    # two particles exactly 2h apart are not neighbours (r^2 < (2h)^2)
    c = block_case(dim=2, n_side=4, dp=0.25)
    p = dict(c.params)
    p["h"] = 0.5
    p["cell_size"] = 1.25
    x = np.array([[2.25, 2.0, 0.0], [3.25, 2.0, 0.0], [3.2499999999999996, 2.0, 0.0]])
    p["lo"], p["hi"] = (-2.0, -2.0, -1.0), (8.0, 8.0, 1.0)
    off, idx = ora.neighbors(p, x)
    S = _sets(off, idx)
    assert 1 not in S[0]
    assert 2 in S[0]          # one ulp inside the cut-off
