"""The paper's qualitative convergence claims on its 2D setups, checked on the oracle.

Sec. III-A: with alpha = gamma = 1 (M = 4, N = 2) BSGD converges linearly to the
least-squares solution. Sec. III-B: with 64 blocks cut as 2x32, 4x16 or 8x8 and one pair
per iteration it still approaches that solution, at a speed that depends on the cut
(the text pairs 2 row blocks with 31 column blocks, which does not make 64; read as 32).
Sec. III-C: at fixed M and N with four pairs per iteration, a smaller gamma converges
more slowly. Sec. III-E: on the 64x64 setup, BSGD-TV reaches a far higher image SNR
than gradient descent without TV at the same step length. The paper shows these as
figures only, so the checks are orderings and rates, not printed values; the step
lengths are multiples of 1/(2 ||A||^2), the paper's absolute mu being in other units.
"""
import numpy as np
import pytest

from bsgd_inputs.configs import study_geometry
from oracle.bsgd import run, snr_db

from helpers import oracle_ds_curve, oracle_problem, oracle_study

PRODUCTS = 8000
GAMMA_PAIRS = ((4, 1), (2, 2), (1, 4))


def _ds(M, bx, by, R, B, scale, n_products=PRODUCTS):
    p0, y, _, x_lsq, L = oracle_study("e1")
    p = oracle_problem(study_geometry("e1", M, bx, by))
    return oracle_ds_curve(p, y, x_lsq, R, B, scale / (2 * L), n_products)


def test_all_blocks_converge_linearly_to_least_squares():
    _, _, _, x_lsq, _ = oracle_study("e1")
    d = [v for _, v in _ds(4, 2, 1, 4, 2, 1.0)]
    ds0 = np.linalg.norm(x_lsq)
    assert d[-1] < 0.01 * ds0
    assert all(b < 0.8 * a for a, b in zip(d, d[1:]))


def test_one_pair_of_64_blocks_approaches_least_squares_at_a_cut_dependent_rate():
    _, _, _, x_lsq, _ = oracle_study("e1")
    ds0 = np.linalg.norm(x_lsq)
    ends = []
    for M, bx, by in ((2, 8, 4), (4, 4, 4), (8, 4, 2)):
        d = [v for _, v in _ds(M, bx, by, 1, 1, 2.0)]
        assert d[-1] < 0.04 * ds0, (M, d)
        assert all(b < a for a, b in zip(d[-4:], d[-3:])), (M, d)
        ends.append(d[-1])
    assert max(ends) > 2.0 * min(ends)


def test_smaller_gamma_converges_more_slowly():
    curves = [[v for _, v in _ds(4, 4, 4, R, B, 2.0)] for R, B in GAMMA_PAIRS]
    for k in range(4, 8):
        assert curves[0][k] > curves[1][k] > curves[2][k]
    assert curves[0][-1] > 3.0 * curves[2][-1]


def test_tv_beats_gradient_descent_on_the_64x64_setup():
    _, y, x_true, _, L = oracle_study("e6")
    p = oracle_problem(study_geometry("e6", 20, 2, 2, partition_seed=6))
    mu, epochs = 1.0 / (2 * L), 60
    tv = run(p, y, mu, 1, 2, epochs * 40, seed=1, tv_lambda=100.0)
    gd = run(p, y, mu, 20, 4, epochs, seed=1)
    assert snr_db(x_true, tv.x) > snr_db(x_true, gd.x) + 5.0
