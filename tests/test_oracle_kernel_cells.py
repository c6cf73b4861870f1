"""Pins of the oracle's kernel, cell sort and neighbour search.

Each test checks the oracle against something other than itself: the
kernel's integral and derivative, textbook stable sorting, and brute-force
neighbour sets.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import integrate

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def golden():
    out = {}
    for line in open(GOLD):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split("=")
            out[k.strip()] = float(v)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_integrates_to_one(orc, dim):
    # A smoothing kernel has unit integral over its support (Eq. (4) with a
    # uniform particle distribution); this fixes the normalisation constant.
    h = 0.37
    f = (lambda r: orc.W(r, h, dim)[0] * 2 * math.pi * r) if dim == 2 else \
        (lambda r: orc.W(r, h, dim)[0] * 4 * math.pi * r * r)
    val, err = integrate.quad(f, 0.0, 2.0 * h, epsabs=1e-13, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_support_and_derivative(orc, dim):
    h = 0.013
    g = golden()
    support = g["support_radius_over_dx"] / g["smoothing_length_over_dx"]  # kappa = 2
    assert orc.W(support * h, h, dim)[0] == 0.0
    assert orc.W(support * h * 1.0000001, h, dim)[0] == 0.0
    assert orc.W(support * h * 0.999, h, dim)[0] > 0.0
    assert orc.dW(0.0, h, dim)[0] == 0.0
    r = np.linspace(0.01 * h, 1.99 * h, 57)
    eps = 1e-6 * h
    fd = (orc.W(r + eps, h, dim) - orc.W(r - eps, h, dim)) / (2 * eps)
    an = orc.dW(r, h, dim)
    scale = np.abs(an).max()
    assert np.abs(fd - an).max() < 1e-6 * scale
    assert np.all(an < 0.0)  # monotone decreasing inside the support


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_sum_converges_to_integral(orc, dim):
    # sigma0 dx^d is a Riemann sum of the unit-integral kernel: close to 1 at
    # the paper's h = 1.3 dx and converging as h/dx grows.
    e13 = abs(orc.sigma0_lattice(dim, 1.0, 1.3) - 1.0)
    e4 = abs(orc.sigma0_lattice(dim, 1.0, 4.0) - 1.0)
    assert e13 < 0.02
    assert e4 < 2e-4
    assert e4 < e13 / 20


def test_counting_sort_is_stable_sort(orc):
    rng = np.random.default_rng(1)
    for n, nkey in [(0, 5), (1, 1), (1000, 37), (5000, 3000)]:
        keys = rng.integers(0, nkey, size=n).astype(np.int32)
        start, order = orc.counting_sort(keys, nkey)
        ref = np.argsort(keys, kind="stable")
        assert np.array_equal(order, ref)
        cnt = np.bincount(keys, minlength=nkey)
        assert np.array_equal(start, np.concatenate([[0], np.cumsum(cnt)]))


def _pairs_from_lists(count, lst):
    a = np.repeat(np.arange(len(count)), count)
    return set(zip(a.tolist(), lst.tolist()))


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (3, 0), (3, 1), (3, 2)])
def test_cell_neighbours_equal_bruteforce(orc, dim, seed):
    rng = np.random.default_rng(seed)
    h = 0.013
    n = 700 if dim == 3 else 400
    xa = rng.uniform(0, 12 * h, size=(n, dim))
    xb = np.concatenate([rng.uniform(-2 * h, 10 * h, size=(n // 2, dim)), xa[:7]])  # coincident points
    count, lst = orc.neighbours(dim, h, xa, xb)
    got = _pairs_from_lists(count, lst)
    d2 = ((xa[:, None, :] - xb[None, :, :]) ** 2).sum(-1)
    ref = set(zip(*np.nonzero(d2 < 4 * h * h)))
    ref = {(int(a), int(b)) for a, b in ref}
    assert got == ref
    # same set against itself includes every point once
    c2, l2 = orc.neighbours(dim, h, xa, xa)
    assert all((i, i) in _pairs_from_lists(c2, l2) for i in range(n))


@pytest.mark.parametrize("dim,expected", [(2, 21), (3, 81)])
def test_full_lattice_neighbour_count(orc, dim, expected):
    # Interior lattice point: lattice vectors k with |k| dx < 2.6 dx.
    ref = sum(1 for k in itertools.product(range(-3, 4), repeat=dim) if sum(x * x for x in k) < 2.6 ** 2)
    assert ref == expected
    dx = 0.01
    n = 9
    pts = np.stack(np.meshgrid(*[np.arange(n) * dx] * dim, indexing="ij"), -1).reshape(-1, dim)
    count, _ = orc.neighbours(dim, 1.3 * dx, pts, pts)
    centre = np.all(np.abs(pts - 4 * dx) < 1e-12, axis=1)
    assert count[centre][0] == expected


@pytest.mark.parametrize("dim", [2, 3])
def test_pair_decision_in_cell_offset_form(orc, dim):
    # The cell+offset pair test agrees with the FP64 absolute-position test
    # except for pairs whose distance lies within a few ulps of the cutoff.
    rng = np.random.default_rng(7)
    h = np.float32(0.0052)
    L = np.float32(2 * h)
    rc2 = float(np.float32(4.0 * float(h) * float(h)))
    n = 600
    cells = rng.integers(0, 4, size=(n, dim)).astype(np.int32)
    off = rng.uniform(0, float(L), size=(n, dim)).astype(np.float32).astype(np.float64)
    for single in (True, False):
        hit = orc.pairs_bruteforce(dim, single, cells, off, cells, off, float(L), rc2)
        x = cells * float(L) + off
        d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
        ref = d2 < rc2
        diff = hit != ref
        assert np.all(np.abs(d2[diff] - rc2) < 1e-5 * rc2)
        assert diff.sum() <= 2
        assert np.all(np.diag(hit))
        assert np.array_equal(hit, hit.T)
