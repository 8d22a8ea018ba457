"""Pins of the oracle's random streams, Eq. 1 and TV proximal step."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import lsq_linear
from scipy.stats import chisquare

from oracle import rng
from oracle.bsgd import eq1, draw_subdetector
from oracle import tv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def test_splitmix64_published_sequence():
    # first outputs of SplitMix64 from state 0 (Steele, Lea, Flood 2014; reference C code output)
    assert rng.splitmix64_sequence(0, 4) == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_choose_is_a_sorted_subset():
    for k in range(50):
        for n, m in ((16, 1), (16, 5), (9, 9), (64, 64), (256, 64)):
            s = rng.choose(99, rng.STREAM_BLOCKS, k, n, m)
            assert s == sorted(set(s)) and len(s) == m and 0 <= s[0] and s[-1] < n


def test_choose_frequencies_are_uniform():
    n, m, trials = 12, 3, 4000
    counts = np.zeros(n)
    for k in range(trials):
        for i in rng.choose(5, rng.STREAM_ROWS, k, n, m):
            counts[i] += 1
    assert chisquare(counts).pvalue > 1e-3


def test_permutation():
    p = rng.permutation(3, rng.STREAM_PARTITION, 101)
    assert sorted(p) == list(range(101)) and p != list(range(101))


def test_streams_are_distinct():
    a = [rng.hash_keys(1, s, 0, 0) for s in (1, 2, 3, 4)]
    assert len(set(a)) == 4


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["eq1_examples"])
def test_eq1_worked_examples(case):
    alpha, gamma = eq1(case["P"], case["M"], case["N"])
    assert alpha == pytest.approx(case["alpha"]) and gamma == pytest.approx(case["gamma"])


def test_im_fraction_example():
    c = json.load(open(GOLDEN))["im_fraction_example"]
    assert c["angles"] * c["fraction"] == c["equivalent_full"]


def test_im_draw_frequencies_follow_table():
    q = np.array([1 << 19, 1 << 18, 0, (1 << 18)], dtype=np.uint32)
    counts = np.zeros(4)
    for k in range(6000):
        counts[draw_subdetector(17, k, 3, 5, q)] += 1
    assert counts[2] == 0
    expected = q / q.sum() * counts.sum()
    assert chisquare(counts[[0, 1, 3]], expected[[0, 1, 3]]).pvalue > 1e-3
    assert draw_subdetector(17, 0, 0, 0, np.zeros(4, dtype=np.uint32)) == -1


# ---------------------------------------------------------------- TV prox

def test_grad_adjoint():
    r = np.random.Generator(np.random.PCG64(1))
    for shape in ((7, 9), (4, 5, 6)):
        x = r.normal(size=shape)
        p = r.normal(size=(len(shape),) + shape)
        assert np.isclose(np.sum(tv.grad(x) * p), np.sum(x * tv.grad_adjoint(p)), rtol=1e-12)


def test_tv_of_known_images():
    x = np.zeros((4, 4))
    x[:, 2:] = 1.0  # a vertical edge of height 4: backward differences along columns
    assert tv.tv(x) == pytest.approx(4.0)
    x = np.arange(9.0).reshape(3, 3)
    # backward differences: rows step 3, columns step 1; zero at the low boundary
    expect = 0 + 1 + 1 + 3 + math.sqrt(10) * 2 + 3 + math.sqrt(10) * 2
    assert tv.tv(x) == pytest.approx(expect)


def test_prox_identity_and_constants():
    r = np.random.Generator(np.random.PCG64(2))
    b = r.normal(size=(6, 7))
    assert np.array_equal(tv.fgp_prox(b, 0.0, 20), b)
    c = np.full((5, 6, 4), 3.25)
    assert np.allclose(tv.fgp_prox(c, 0.7, 20), c, atol=1e-14)


def test_prox_two_level_step_closed_form():
    # 1/2||t-b||^2 + w|jump| on a two-level signal: the levels move towards each
    # other by w/n1 and w/n2 as long as they do not cross (optimality conditions).
    n1, n2, h, w = 7, 5, 2.0, 0.9
    b = np.concatenate([np.full(n1, h), np.zeros(n2)])[None, :]
    t = tv.fgp_prox(b, w, 4000)
    expect = np.concatenate([np.full(n1, h - w / n1), np.full(n2, w / n2)])[None, :]
    assert np.allclose(t, expect, atol=1e-6)


def test_prox_1d_matches_exact_qp():
    r = np.random.Generator(np.random.PCG64(4))
    n, w = 40, 0.35
    b = np.cumsum(r.normal(size=n)) * 0.3
    D = np.zeros((n - 1, n))  # backward differences x_c - x_{c-1}, c = 1..n-1
    for c in range(1, n):
        D[c - 1, c], D[c - 1, c - 1] = 1.0, -1.0
    sol = lsq_linear(D.T, b, bounds=(-w, w), tol=1e-14, lsmr_tol="auto", max_iter=10000)
    exact = b - D.T @ sol.x
    t = tv.fgp_prox(b[None, :], w, 6000)[0]
    assert np.allclose(t, exact, atol=1e-5)


def test_prox_duality_gap_shrinks():
    r = np.random.Generator(np.random.PCG64(5))
    for shape, w in (((12, 10), 0.4), ((6, 7, 5), 0.3)):
        b = r.normal(size=shape)
        gaps = []
        for K in (5, 50, 500):
            t, p = tv.fgp_prox(b, w, K, return_dual=True)
            g = tv.primal_objective(t, b, w) - tv.dual_objective(p, b, w)
            assert g >= -1e-10
            gaps.append(g)
        assert gaps[2] < gaps[1] < gaps[0]
        assert gaps[2] < 1e-3 * gaps[0]
