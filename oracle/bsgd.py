"""Block stochastic gradient descent, step by step, on an explicit sparse A.

TEST INFRASTRUCTURE (oracle), FP64. Follows Algorithms 1 (BSGD), 2 (BSGD-IM)
and 4 (BSGD-TV) in the paper's order and notation, in the precise form of the
state-update equations of the fixed-point analysis (Eqs. (Updaz), (Updag),
(Updax)):

  state: x, z^j (one r-vector per column block), g^i_hat (one c-vector per row
  block), g; initially z = 0, g_hat = 0, g = 0, r = y.

  iteration k:
    1. choose alpha M row blocks R and gamma N column blocks C at random
    2. rows(i, j) = all rays of the views of I_i; with importance sampling, for
       each view of I_i one sub-detector drawn with probability proportional to
       the quantised weight table q[v][s][j] (views with no weight are skipped)
    3. with x frozen, z^j[rows(i, j)] = A[rows(i, j), J_j] x[J_j]   for (i, j) in R x C
    4. r = y - sum_j z^j
    5. g_hat^i[J_j] = 2 A[rows(i, j), J_j]^T r[rows(i, j)]          for (i, j) in R x C
    6. g = sum_i g_hat^i
    7. x[J_j] += mu g[J_j]                                            for j in C
    8. k <- k + 1; with TV, when k is a multiple of T = round(1/(alpha gamma)):
       x <- argmin_t ||t - x||^2 + 2 mu lambda TV(t)

Readings of unstated details (each listed in the design notes):
* the factor 2 in the gradient is kept literally (g = 2 A^T r, x += mu g);
* blocks are drawn uniformly without replacement within an iteration and
  independently across iterations (counter-based stream, see ``rng``);
* importance weights are squared Frobenius norms of the sub-matrices A[sub-detector
  rows, J_j] ("block column norms"), quantised to integers q_s = round(2^20 w_s /
  sum w) with q_s >= 1 whenever w_s > 0; the drawn sub-detector is the first s
  whose running sum of q exceeds bounded(hash(seed, IM, k, v, j), sum q);
* the IM gradient memory is overwritten without reweighting (literal Algorithm 2).

Pinned by: closed-form gradient (mu = 0, all blocks), the gradient-descent special
case alpha = gamma = 1, the SAG special case gamma = 1, convergence to the least
squares solution (fixed-point analysis), monotone objective decrease in the GD
case, the invariants r = y - sum z and g = sum g_hat, and Eq. 1's worked examples.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from bsgd_inputs.configs import GeometrySpec
from . import geometry as geo
from . import rng
from .tv import fgp_prox

Q_BITS = 20


def eq1(node_count: int, M: int, N: int):
    """Eq. 1: gamma = min(1, P/N), alpha = P/(M N gamma). Returns (alpha, gamma)."""
    gamma = min(1.0, node_count / N)
    alpha = node_count / (M * N * gamma)
    return alpha, gamma


@dataclass
class Problem:
    g: GeometrySpec
    A: sp.csr_matrix
    groups: List[List[int]]
    blocks: List[np.ndarray]
    A_cols: list = field(default_factory=list)  # A[:, J_j] as CSR, one per block

    @staticmethod
    def build(g: GeometrySpec, A: Optional[sp.csr_matrix] = None) -> "Problem":
        if A is None:
            from .system import matrix
            A = matrix(g)
        A = sp.csr_matrix(A)
        blocks = geo.column_blocks(g)
        groups = geo.view_groups(g)
        cols = [sp.csr_matrix(A[:, J]) for J in blocks]
        return Problem(g=g, A=A, groups=groups, blocks=blocks, A_cols=cols)

    @property
    def M(self):
        return len(self.groups)

    @property
    def N(self):
        return len(self.blocks)


def im_weights(p: Problem) -> np.ndarray:
    """w[v][s][j] = || A[rows of sub-detector s of view v, J_j] ||_F^2 (float64)."""
    g = p.g
    S = g.su * g.sv
    w = np.zeros((g.n_views, S, p.N))
    A2 = [Aj.multiply(Aj).tocsr() for Aj in p.A_cols]
    for j, Aj2 in enumerate(A2):
        per_ray = np.asarray(Aj2.sum(axis=1)).reshape(-1)
        for v in range(g.n_views):
            for s in range(S):
                w[v, s, j] = per_ray[geo.subdetector_rays(g, v, s)].sum()
    return w


def quantise(w: np.ndarray) -> np.ndarray:
    """q = round(2^20 w / sum_s w) per (view, block), forced >= 1 where w > 0."""
    tot = w.sum(axis=1, keepdims=True)
    q = np.zeros(w.shape, dtype=np.int64)
    nz = tot > 0
    ratio = np.where(nz, w / np.where(nz, tot, 1.0), 0.0)
    q = np.floor(ratio * (1 << Q_BITS) + 0.5).astype(np.int64)
    q = np.where((w > 0) & (q == 0), 1, q)
    return q.astype(np.uint32)


def im_table(p: Problem, mode: str) -> Optional[np.ndarray]:
    g = p.g
    S = g.su * g.sv
    if mode == "none":
        return None
    if mode == "uniform":
        return np.ones((g.n_views, S, p.N), dtype=np.uint32)
    if mode == "colnorm":
        return quantise(im_weights(p))
    if mode == "area":
        from .area import area_weights
        return quantise(area_weights(g))
    raise ValueError(mode)


def draw_subdetector(seed: int, k: int, view: int, block: int, qcol) -> int:
    """Sub-detector for (iteration, view, block), or -1 when the view has no weight."""
    qcol = [int(v) for v in qcol]
    total = sum(qcol)
    if total == 0:
        return -1
    u = rng.bounded(rng.hash_keys(seed, rng.STREAM_IM, k, view, block), total)
    acc = 0
    for s, qs in enumerate(qcol):
        acc += qs
        if acc > u:
            return s
    raise AssertionError("unreachable")


@dataclass
class State:
    x: np.ndarray
    z: np.ndarray       # [N][r]
    ghat: np.ndarray    # [M][c]
    gsum: np.ndarray    # [c]
    r: np.ndarray       # [r]
    k: int = 0
    mem: Optional[np.ndarray] = None   # [views][S][c] per-sub-detector gradient memory


def initial_state(p: Problem, y: np.ndarray, x0: Optional[np.ndarray] = None) -> State:
    r_n, c_n = p.A.shape
    x = np.zeros(c_n) if x0 is None else np.array(x0, dtype=np.float64)
    return State(x=x, z=np.zeros((p.N, r_n)), ghat=np.zeros((p.M, c_n)), gsum=np.zeros(c_n),
                 r=np.array(y, dtype=np.float64))


def parts_for_pair(p: Problem, i: int, j: int, k: int, seed: int, q, draws_out=None):
    """The rays of row block i that pair (i, j) uses at iteration k, as ((view,
    sub-detector), rays) parts: every sub-detector of every view without sampling,
    one drawn sub-detector per view with it (Algorithm 2), none for a view whose
    weights are all zero."""
    g = p.g
    parts = []
    for v in p.groups[i]:
        if q is None:
            subs = range(g.su * g.sv)
        else:
            s = draw_subdetector(seed, k, v, j, q[v, :, j])
            if draws_out is not None:
                draws_out[(v, j)] = s
            subs = [s] if s >= 0 else []
        for s in subs:
            parts.append(((v, s), geo.subdetector_rays(g, v, s)))
    return parts


def rows_for_pair(p: Problem, i: int, j: int, k: int, seed: int, q, draws_out=None):
    if q is None:
        return geo.rays_of_group(p.g, p.groups[i])
    parts = [rows for _, rows in parts_for_pair(p, i, j, k, seed, q, draws_out)]
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)


def iterate(p: Problem, st: State, y: np.ndarray, mu: float, rows_per_iter: int,
            blocks_per_iter: int, seed: int, q=None, tv_lambda: float = 0.0,
            tv_iters: int = 20, trace: Optional[list] = None, im_until: Optional[int] = None,
            subdet_memory: bool = False):
    """One BSGD iteration in place on ``st``, as the state updates of Sec. IV define it.
    The stacked memories are z-bar (one r-vector z^j per column block) and g-bar (one
    c-vector g_hat^i per row block); random 0/1 diagonal selections R1, R2, R3 pick the
    slots of the chosen (row block, column block) pairs and the chosen blocks' voxels:

      Eq. (Updaz)  z-bar += R1 (A-bar x - z-bar): z^j on the chosen rows becomes A^{J_j} x_{J_j}
                   (x as it stood when the iteration began);
      Eq. (Updag)  g-bar += R2 (2 A^T-bar (y - I z-bar) - g-bar): g_hat^i on the chosen
                   blocks becomes the gradient of those rows at the refreshed residual
                   (the factor 2 of Eq. (SGDITE) kept literally);
      Eq. (Updax)  x += mu R3 I g-bar: the chosen blocks move along g = sum_i g_hat^i;

    then the TV prox every round(1/(alpha gamma)) iterations (Algorithm 4). Which pairs
    are chosen is Algorithm 1's selection; with importance sampling (Algorithm 2) a pair
    uses only its view's drawn sub-detector rows. With ``im_until``,
    iterations k >= im_until run without importance sampling (all rays of the selected
    row blocks): the unbiased tail that Sec. II-A recommends for the last iterations.

    With ``subdet_memory`` the gradient memory is kept per (view, sub-detector, column
    block) instead of per (row block, column block): a pair refreshes the memories of
    the (view, sub-detector) parts it used, 2 (A_part^J)^T r_part, and g is the sum of
    all memories. Without sampling this is Algorithm 1 (the memories of a row block's
    parts sum to its g_hat); with sampling, a drawn sub-detector no longer replaces the
    whole row block's gradient, so g at a fixed point is the full gradient (unbiased IM)."""
    k = st.k
    if im_until is not None and k >= im_until:
        q = None
    R = rng.choose(seed, rng.STREAM_ROWS, k, p.M, rows_per_iter)
    C = rng.choose(seed, rng.STREAM_BLOCKS, k, p.N, blocks_per_iter)
    draws = {} if trace is not None else None
    pairs = [(i, j, parts_for_pair(p, i, j, k, seed, q, draws)) for i in R for j in C]
    pairs = [(i, j, parts, geo.rays_of_group(p.g, p.groups[i]) if q is None else
              np.concatenate([r for _, r in parts]) if parts else np.zeros(0, dtype=np.int64))
             for i, j, parts in pairs]
    x_frozen = st.x.copy()
    # Eq. (Updaz): refresh the chosen z slots
    for i, j, _, rows in pairs:
        st.z[j][rows] = p.A_cols[j][rows] @ x_frozen[p.blocks[j]]
    # the residual y - I z-bar that Eq. (Updag) reads
    st.r = y - st.z.sum(axis=0)
    if subdet_memory:
        if st.mem is None:
            st.mem = np.zeros((p.g.n_views, p.g.su * p.g.sv, p.A.shape[1]))
        for i, j, parts, _ in pairs:
            for (v, s), rows in parts:
                st.mem[v, s, p.blocks[j]] = 2.0 * (p.A_cols[j][rows].T @ st.r[rows])
        st.gsum = st.mem.sum(axis=(0, 1))
    else:
        # Eq. (Updag): refresh the chosen g_hat slots; g = I g-bar
        for i, j, _, rows in pairs:
            st.ghat[i][p.blocks[j]] = 2.0 * (p.A_cols[j][rows].T @ st.r[rows])
        st.gsum = st.ghat.sum(axis=0)
    # Eq. (Updax): the chosen blocks' voxels move
    for j in C:
        st.x[p.blocks[j]] += mu * st.gsum[p.blocks[j]]
    st.k += 1
    if tv_lambda > 0.0:
        T = tv_period(p.M, p.N, rows_per_iter, blocks_per_iter)
        if st.k % T == 0:
            shape = image_shape(p.g)
            st.x = fgp_prox(st.x.reshape(shape), mu * tv_lambda, tv_iters).reshape(-1)
    if trace is not None:
        trace.append({"k": k, "rows": R, "blocks": C, "draws": draws})


def tv_period(M: int, N: int, rows_per_iter: int, blocks_per_iter: int) -> int:
    """Iterations per effective epoch, round(1/(alpha gamma))."""
    return max(1, int(round((M * N) / (rows_per_iter * blocks_per_iter))))


def image_shape(g: GeometrySpec):
    return (g.nz, g.ny, g.nx) if g.is_3d else (g.ny, g.nx)


@dataclass
class AutoMu:
    """Algorithm 3 (automatic step length). Every M iterations the g's of the last M
    iterations are summed into an effective update direction (EUD); theta is the
    cosine between consecutive EUDs; ||r|| is the norm of the maintained residual
    y - sum_j z^j. Once three residual norms and two thetas exist (k >= 3M, the
    reading used for the paper's "k > M" whose earlier terms are undefined):
      ||r||^k < ||r||^{k-M} < ||r||^{k-2M}                   -> mu *= 1 + eps
      ||r||^k > ||r||^{k-M} > ||r||^{k-2M} and
        (|theta^k - theta^{k-M}| > t1 or theta^k < t2)        -> mu *= 1 - delta
    The paper gives delta = 0.4 (Sec. III-C); eps, t1, t2 are not given (readings).
    The residual norms and cosines of every check are recorded beside the step lengths.

    Parity pin: gradient descent on a diagonal two-pixel system, where residuals,
    EUDs and cosines have closed forms (a hand derivation in the tests), fixes the
    norms, the cosines, each decision and the EUD reset after every check."""
    eps: float = 0.05
    delta: float = 0.4
    t1: float = 0.1
    t2: float = 0.5
    mu_history: list = field(default_factory=list)
    r_history: list = field(default_factory=list)
    theta_history: list = field(default_factory=list)


def run(p: Problem, y: np.ndarray, mu: float, rows_per_iter: int, blocks_per_iter: int,
        n_iters: int, seed: int, q=None, x0=None, tv_lambda: float = 0.0, tv_iters: int = 20,
        trace: Optional[list] = None, callback=None, auto_mu: Optional[AutoMu] = None,
        im_until: Optional[int] = None, subdet_memory: bool = False) -> State:
    st = initial_state(p, y, x0)
    eud = np.zeros(p.A.shape[1])
    prev_eud = None
    r_hist, theta_hist = [], []
    for _ in range(n_iters):
        iterate(p, st, y, mu, rows_per_iter, blocks_per_iter, seed, q, tv_lambda, tv_iters, trace, im_until,
                subdet_memory)
        if auto_mu is not None:
            eud += st.gsum
            if st.k % p.M == 0:
                r_hist.append(float(np.linalg.norm(st.r)))
                if prev_eud is not None:
                    theta_hist.append(float(eud @ prev_eud / (np.linalg.norm(eud) * np.linalg.norm(prev_eud))))
                if len(r_hist) >= 3 and len(theta_hist) >= 2:
                    r0, r1, r2 = r_hist[-1], r_hist[-2], r_hist[-3]
                    th, th_prev = theta_hist[-1], theta_hist[-2]
                    if r0 < r1 < r2:
                        mu = (1.0 + auto_mu.eps) * mu
                    if r0 > r1 > r2 and (abs(th - th_prev) > auto_mu.t1 or th < auto_mu.t2):
                        mu = (1.0 - auto_mu.delta) * mu
                auto_mu.mu_history.append(mu)
                auto_mu.r_history = list(r_hist)
                auto_mu.theta_history = list(theta_hist)
                prev_eud = eud
                eud = np.zeros(p.A.shape[1])
        if callback is not None:
            callback(st)
    return st


def lipschitz(A: sp.spmatrix, iters: int = 30, seed: int = 0) -> float:
    """sigma_max(A)^2 by power iteration on A^T A."""
    v = np.random.Generator(np.random.PCG64(seed)).uniform(size=A.shape[1])
    lam = 0.0
    for _ in range(iters):
        w = A.T @ (A @ v)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def ds(x_rec, x_lsq) -> float:
    """Distance to the least-squares solution (Sec. III-A)."""
    return float(np.linalg.norm(np.asarray(x_rec) - np.asarray(x_lsq)))


def gap(A, y, x) -> float:
    """GAP = ||y - A x|| (Sec. III-E)."""
    return float(np.linalg.norm(y - A @ x))


def snr_db(x_true, x) -> float:
    """SNR = 20 log10(||x_true|| / ||x_true - x||) (Sec. III-D)."""
    return 20.0 * math.log10(np.linalg.norm(x_true) / np.linalg.norm(np.asarray(x_true) - x))
