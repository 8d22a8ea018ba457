"""Pins of the oracle's BSGD iteration (Algorithms 1, 2, 4) against closed forms and invariants."""
import math

import numpy as np
import pytest

from bsgd_inputs.configs import GeometrySpec
from bsgd_inputs.phantoms import ellipse_phantom_2d, add_gaussian_noise
from oracle import rng
from oracle import geometry as geo
from oracle.bsgd import (Problem, run, initial_state, iterate, lipschitz, ds, im_weights,
                         quantise, im_table, tv_period)
from oracle.tv import fgp_prox


def _e1_problem(M=4, bx=2, by=1, su=1, im="none"):
    # the paper's first 2D experiment: 16x16 image, OP = OD = 50, 30 bins, 10 degree steps
    g = GeometrySpec(kind="fan2d", nx=16, ny=16, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=36,
                     angle_span=2 * math.pi, nu=30, nv=1, du=1.0, dv=1.0, sod=50.0, sdd=100.0,
                     bx=bx, by=by, bz=1, n_row_blocks=M, partition_seed=3, su=su, im_mode=im)
    return Problem.build(g)


@pytest.fixture(scope="module")
def e1():
    p = _e1_problem()
    x_true = ellipse_phantom_2d(16, 16, 6, 5).ravel()
    y = add_gaussian_noise(p.A @ x_true, 0.05, 9)
    L = lipschitz(p.A)
    return p, y, L


def test_partitions_cover_everything(e1):
    p, _, _ = e1
    views = sorted(v for grp in p.groups for v in grp)
    assert views == list(range(p.g.n_views))
    vox = np.sort(np.concatenate(p.blocks))
    assert np.array_equal(vox, np.arange(p.A.shape[1]))


def test_full_sweep_gives_closed_form_gradient(e1):
    p, y, _ = e1
    x0 = np.random.Generator(np.random.PCG64(1)).uniform(size=p.A.shape[1])
    st = initial_state(p, y, x0)
    iterate(p, st, y, 0.0, p.M, p.N, seed=3)
    assert np.allclose(st.gsum, 2.0 * p.A.T @ (y - p.A @ x0), rtol=1e-12, atol=1e-12)
    assert np.array_equal(st.x, x0)


@pytest.mark.parametrize("M,bx", [(4, 2), (1, 1)])
def test_all_blocks_is_gradient_descent(M, bx):
    p = _e1_problem(M=M, bx=bx)
    r = np.random.Generator(np.random.PCG64(2))
    y = p.A @ r.uniform(size=p.A.shape[1]) + r.normal(size=p.A.shape[0])
    mu = 0.4 / (2 * lipschitz(p.A))
    st = run(p, y, mu, p.M, p.N, 25, seed=5)
    x = np.zeros(p.A.shape[1])
    for _ in range(25):
        x = x + 2 * mu * (p.A.T @ (y - p.A @ x))
    assert np.allclose(st.x, x, rtol=1e-11, atol=1e-12)


def test_gradient_descent_objective_is_monotone(e1):
    p, y, L = e1
    mu = 0.5 / (2 * L)
    f = []
    run(p, y, mu, p.M, p.N, 30, seed=1, callback=lambda st: f.append(np.sum((y - p.A @ st.x) ** 2)))
    assert all(b <= a * (1 + 1e-14) for a, b in zip(f, f[1:]))


def test_gamma_one_is_sag_over_row_blocks(e1):
    p, y, L = e1
    mu = 0.3 / (2 * L)
    seed, n_iter = 11, 60
    st = run(p, y, mu, 1, p.N, n_iter, seed=seed)
    # an independent SAG: one stored gradient per row block, refreshed at the current x
    rows = [geo.rays_of_group(p.g, grp) for grp in p.groups]
    mem = np.zeros((p.M, p.A.shape[1]))
    x = np.zeros(p.A.shape[1])
    for k in range(n_iter):
        (i,) = rng.choose(seed, rng.STREAM_ROWS, k, p.M, 1)
        Ai = p.A[rows[i]]
        mem[i] = 2 * Ai.T @ (y[rows[i]] - Ai @ x)
        x = x + mu * mem.sum(axis=0)
    assert np.allclose(st.x, x, rtol=1e-10, atol=1e-12)


def test_converges_to_least_squares(e1):
    p, y, L = e1
    x_lsq = np.linalg.lstsq(p.A.toarray(), y, rcond=None)[0]
    d = []
    run(p, y, 0.5 / (2 * L), 1, 1, 3000, seed=7,
        callback=lambda st: d.append(ds(st.x, x_lsq)) if st.k % 500 == 0 else None)
    assert d[-1] < 3e-3 * np.linalg.norm(x_lsq)
    assert d[-1] < 0.1 * d[0] and d[-1] < d[-2] < d[-3]


def test_invariants_after_importance_sampled_run():
    p = _e1_problem(M=3, bx=2, by=2, su=3, im="colnorm")
    r = np.random.Generator(np.random.PCG64(8))
    y = p.A @ r.uniform(size=p.A.shape[1])
    q = im_table(p, "colnorm")
    trace = []
    st = run(p, y, 0.3 / (2 * lipschitz(p.A)), 2, 2, 40, seed=4, q=q, trace=trace)
    assert np.allclose(st.r, y - st.z.sum(axis=0), atol=1e-12)
    assert np.allclose(st.gsum, st.ghat.sum(axis=0), atol=1e-12)
    # z entries outside the footprint of their block stay zero
    for j, J in enumerate(p.blocks):
        touched = np.asarray(abs(p.A[:, J]).sum(axis=1)).ravel() > 0
        assert not np.any(st.z[j][~touched])
    # every draw is a sub-detector with nonzero weight
    for t in trace:
        for (v, j), s in t["draws"].items():
            assert s >= 0 and q[v, s, j] > 0


def test_colnorm_weights_partition_frobenius_norm():
    p = _e1_problem(M=3, bx=2, by=2, su=3, im="colnorm")
    w = im_weights(p)
    A2 = p.A.multiply(p.A)
    assert np.isclose(w.sum(), A2.sum(), rtol=1e-12)
    per_view_block = w.sum(axis=1)
    for v in (0, 7, 35):
        rows = geo.rays_of_view(p.g, v)
        for j, J in enumerate(p.blocks):
            assert np.isclose(per_view_block[v, j], A2[rows][:, J].sum(), rtol=1e-12)
    q = quantise(w)
    tot = q.sum(axis=1).astype(np.int64)
    assert np.all(np.abs(tot - (1 << 20)) <= q.shape[1])
    assert np.all((q > 0) == (w > 0))


def test_tv_period_and_zero_lambda(e1):
    p, y, L = e1
    assert tv_period(20, 4, 1, 2) == 40 and tv_period(5, 8, 1, 2) == 20
    a = run(p, y, 0.3 / (2 * L), 1, 1, 20, seed=2)
    b = run(p, y, 0.3 / (2 * L), 1, 1, 20, seed=2, tv_lambda=0.0)
    assert np.array_equal(a.x, b.x)
    # with TV on, the prox fires exactly at multiples of T = M N / (alpha M gamma N)
    mu, lam = 0.3 / (2 * L), 0.5
    st = initial_state(p, y)
    T = tv_period(p.M, p.N, 1, 1)
    plain = initial_state(p, y)
    for k in range(T):
        iterate(p, plain, y, mu, 1, 1, 2)
        iterate(p, st, y, mu, 1, 1, 2, tv_lambda=lam)
        if k < T - 1:
            assert np.array_equal(st.x, plain.x)
    assert np.allclose(st.x, fgp_prox(plain.x.reshape(16, 16), mu * lam, 20).ravel(), atol=1e-14)


def test_auto_mu_shrinks_a_diverging_step_and_grows_a_small_one():
    from oracle.bsgd import AutoMu
    p = _e1_problem(M=4, bx=2)
    r = np.random.Generator(np.random.PCG64(12))
    y = p.A @ r.uniform(size=p.A.shape[1])
    L = lipschitz(p.A)
    big = AutoMu()
    st = run(p, y, 3.0 / (2 * L), 1, 1, 400, seed=3, auto_mu=big)
    assert len(big.mu_history) == 100
    assert min(big.mu_history) < 3.0 / (2 * L)          # criteria 1 + 2 cut the step
    assert np.isfinite(st.x).all()
    small = AutoMu()
    run(p, y, 0.02 / (2 * L), 1, 1, 400, seed=3, auto_mu=small)
    assert small.mu_history[-1] > 0.02 / (2 * L)         # steady decrease grows the step
    # no change before three residual norms and two thetas exist (k < 3M)
    assert small.mu_history[0] == small.mu_history[1] == 0.02 / (2 * L)


def test_unbiased_tail_removes_the_importance_sampling_bias():
    """Sec. II-A: importance sampling biases BSGD (g_hat holds gradients over the sampled
    rows only), so its iterates stall short of the least-squares solution; running the
    last iterations without sampling (im_until) restores convergence to it."""
    p = _e1_problem(M=4, bx=2, by=2, su=3, im="colnorm")
    r = np.random.Generator(np.random.PCG64(5))
    y = p.A @ r.uniform(size=p.A.shape[1]) + 0.01 * r.normal(size=p.A.shape[0])
    x_lsq = np.linalg.lstsq(p.A.toarray(), y, rcond=None)[0]
    q = im_table(p, "colnorm")
    mu = 0.5 / (2 * lipschitz(p.A))
    im_only, tail = [], []
    run(p, y, mu, 1, 2, 6000, seed=3, q=q,
        callback=lambda st: im_only.append(ds(st.x, x_lsq)) if st.k % 1500 == 0 else None)
    run(p, y, mu, 1, 2, 6000, seed=3, q=q, im_until=3000,
        callback=lambda st: tail.append(ds(st.x, x_lsq)) if st.k % 1500 == 0 else None)
    assert im_only[:2] == tail[:2]                   # identical until the switch
    assert im_only[3] > 0.5 * im_only[2]             # sampling alone has nearly stalled
    assert tail[3] < 0.25 * im_only[3]               # the plain tail keeps converging
    assert tail[3] < 0.5 * tail[2]


@pytest.mark.parametrize("su", [1, 3])
def test_subdetector_memory_without_sampling_is_algorithm_1(su):
    """The memories of a row block's (view, sub-detector) parts sum to its g_hat, so
    without sampling the per-part memory reproduces Algorithm 1."""
    p = _e1_problem(M=4, bx=2, by=2, su=su)
    r = np.random.Generator(np.random.PCG64(6))
    y = p.A @ r.uniform(size=p.A.shape[1]) + 0.05 * r.normal(size=p.A.shape[0])
    mu = 0.5 / (2 * lipschitz(p.A))
    a = run(p, y, mu, 2, 2, 150, seed=3)
    b = run(p, y, mu, 2, 2, 150, seed=3, subdet_memory=True)
    assert np.allclose(a.x, b.x, rtol=1e-12, atol=1e-13)
    assert np.allclose(a.gsum, b.gsum, rtol=1e-12, atol=1e-12)
    assert np.allclose(b.mem.sum(axis=(0, 1)), b.gsum, rtol=1e-12, atol=1e-12)
    # a full sweep at mu = 0 refreshes every memory at x0: g = 2 A^T (y - A x0)
    x0 = r.uniform(size=p.A.shape[1])
    st = initial_state(p, y, x0)
    iterate(p, st, y, 0.0, p.M, p.N, seed=3, subdet_memory=True)
    assert np.allclose(st.gsum, 2.0 * p.A.T @ (y - p.A @ x0), rtol=1e-12, atol=1e-12)


def test_subdetector_memory_removes_the_importance_sampling_bias():
    """Sec. II-A: with g_hat overwritten by the sampled rows' gradient, importance
    sampling stalls short of the least-squares solution; with one memory per
    (view, sub-detector, block) the sampled iteration itself converges to it."""
    p = _e1_problem(M=4, bx=2, by=2, su=3, im="colnorm")
    r = np.random.Generator(np.random.PCG64(5))
    y = p.A @ r.uniform(size=p.A.shape[1]) + 0.01 * r.normal(size=p.A.shape[0])
    x_lsq = np.linalg.lstsq(p.A.toarray(), y, rcond=None)[0]
    q = im_table(p, "colnorm")
    mu = 1.0 / (2 * lipschitz(p.A))
    lit, mem = [], []
    run(p, y, mu, 1, 2, 6000, seed=3, q=q,
        callback=lambda st: lit.append(ds(st.x, x_lsq)) if st.k % 1000 == 0 else None)
    run(p, y, mu, 1, 2, 6000, seed=3, q=q, subdet_memory=True,
        callback=lambda st: mem.append(ds(st.x, x_lsq)) if st.k % 1000 == 0 else None)
    assert lit[5] > 0.9 * lit[4]                     # the literal form has stalled
    assert mem[5] < 0.6 * mem[4] and mem[5] < 0.1 * lit[5]


# ---------------------------------------------------------------- Algorithm 3 by hand
#
# Gradient descent (every row and column block selected) on A = diag(1, 2), y = (1, 1),
# x0 = 0. With D = A A^T = diag(1, 4) the residual obeys r_{k+1} = (I - 2 mu D) r_k, so
# with a = 1 - 2 mu, b = 1 - 8 mu:  r_k = (a^k, b^k)  and  g_k = 2 A^T r_k = (2 a^k, 4 b^k).
# The check after iteration k (1-based count k a multiple of M) sees the residual of the
# last iteration, r_{k-1}, and the EUD = g_{k-M} + ... + g_{k-1}; theta is the cosine of
# two consecutive EUDs. These closed forms are derived here, not taken from the oracle.

def _diag_problem(M):
    """Two pixels, two rays (one per view when M = 2, both in one view when M = 1)."""
    import scipy.sparse as sparse
    if M == 2:
        g = GeometrySpec(kind="parallel2d", nx=2, ny=1, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=2,
                         angle_span=math.pi, nu=1, nv=1, du=1.0, dv=1.0, n_row_blocks=2, partition_seed=0)
    else:
        g = GeometrySpec(kind="parallel2d", nx=2, ny=1, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=1,
                         angle_span=math.pi, nu=2, nv=1, du=1.0, dv=1.0, n_row_blocks=1, partition_seed=0)
    return Problem.build(g, sparse.csr_matrix(np.diag([1.0, 2.0])))


def _cos(u, v):
    return float(np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v)))


def test_auto_mu_by_hand_growth_and_eud_reset():
    """M = 2, mu = 1/16 (a = 7/8, b = 1/2): residual norms fall at every check, so the
    third check (three norms, two cosines) grows mu by 1 + eps, and so does the
    fourth, whose EUD holds only the two iterations run with the grown step."""
    from oracle.bsgd import AutoMu
    p = _diag_problem(2)
    y = np.array([1.0, 1.0])
    mu = 1.0 / 16
    a, b = 7.0 / 8, 1.0 / 2
    am = AutoMu(eps=0.05)
    st = run(p, y, mu, 2, 1, 8, seed=1, auto_mu=am)
    # checks after 2, 4, 6 iterations: r_1, r_3, r_5 and EUDs g0+g1, g2+g3, g4+g5
    E = [np.array([2 * a ** (2 * j) * (1 + a), 4 * b ** (2 * j) * (1 + b)]) for j in range(3)]
    r = [math.hypot(a ** (2 * j + 1), b ** (2 * j + 1)) for j in range(3)]
    mu1 = mu * 1.05
    a1, b1 = 1 - 2 * mu1, 1 - 8 * mu1
    # iterations 6, 7 run with mu1 from r_6 = (a^6, b^6): r_7 = (a1 a^6, b1 b^6), EUD g6 + g7
    r7 = math.hypot(a1 * a ** 6, b1 * b ** 6)
    E4 = np.array([2 * a ** 6 * (1 + a1), 4 * b ** 6 * (1 + b1)])
    assert np.allclose(am.r_history, r + [r7], rtol=1e-13)
    assert np.allclose(am.theta_history, [_cos(E[1], E[0]), _cos(E[2], E[1]), _cos(E4, E[2])], rtol=1e-13)
    assert am.mu_history == [mu, mu, mu1, mu1 * 1.05]
    # and the iterate: x = A^{-1} (y - r_8), r_8 = (a1^2 a^6, b1^2 b^6) ... with mu2 unused yet
    r8 = np.array([a1 ** 2 * a ** 6, b1 ** 2 * b ** 6])
    assert np.allclose(st.x, (y - r8) / np.array([1.0, 2.0]), rtol=1e-13)


def test_auto_mu_by_hand_shrink_on_rising_norms():
    """M = 2, mu = 5/16 (a = 3/8, b = -3/2): norms rise, the EUD turns (|theta_3 -
    theta_2| > t1), so the third check cuts mu by 1 - delta; with the cut step the
    next norm falls and mu stays."""
    from oracle.bsgd import AutoMu
    p = _diag_problem(2)
    y = np.array([1.0, 1.0])
    mu = 5.0 / 16
    a, b = 3.0 / 8, -3.0 / 2
    am = AutoMu(delta=0.4, t1=0.1, t2=0.5)
    run(p, y, mu, 2, 1, 8, seed=1, auto_mu=am)
    E = [np.array([2 * a ** (2 * j) * (1 + a), 4 * b ** (2 * j) * (1 + b)]) for j in range(3)]
    th2, th3 = _cos(E[1], E[0]), _cos(E[2], E[1])
    assert abs(th3 - th2) > 0.1 and th3 > 0.5          # the first criterion decides
    mu1 = 0.6 * mu
    a1, b1 = 1 - 2 * mu1, 1 - 8 * mu1
    r = [math.hypot(a ** (2 * j + 1), b ** (2 * j + 1)) for j in range(3)] + \
        [math.hypot(a1 * a ** 6, b1 * b ** 6)]
    assert r[0] < r[1] < r[2] and r[3] < r[2]
    assert np.allclose(am.r_history, r, rtol=1e-13)
    assert np.allclose(am.theta_history[:2], [th2, th3], rtol=1e-13)
    assert am.mu_history == [mu, mu, mu1, mu1]


@pytest.mark.parametrize("t2,cut", [(0.5, True), (-1.0, False)])
def test_auto_mu_by_hand_alternating_direction(t2, cut):
    """M = 1 (a check after every iteration, EUD = the last g), mu = 5/16: g alternates
    its sign, theta stays near -1 (|theta_2 - theta_1| = 0.156 < t1 = 0.2), so only the
    second criterion theta < t2 can cut the step."""
    from oracle.bsgd import AutoMu
    p = _diag_problem(1)
    y = np.array([1.0, 1.0])
    mu = 5.0 / 16
    a, b = 3.0 / 8, -3.0 / 2
    am = AutoMu(delta=0.4, t1=0.2, t2=t2)
    run(p, y, mu, 1, 1, 3, seed=1, auto_mu=am)
    g = [np.array([2 * a ** k, 4 * b ** k]) for k in range(3)]
    th = [_cos(g[1], g[0]), _cos(g[2], g[1])]
    assert th[0] == pytest.approx(-22.5 / math.sqrt(20.0 * 36.5625), rel=1e-13)
    assert abs(th[1] - th[0]) < 0.2 and th[1] < 0.5
    assert np.allclose(am.r_history, [math.hypot(a ** k, b ** k) for k in range(3)], rtol=1e-13)
    assert np.allclose(am.theta_history, th, rtol=1e-13)
    assert am.mu_history == [mu, mu, 0.6 * mu if cut else mu]
