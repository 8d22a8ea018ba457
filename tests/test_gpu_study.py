"""The convergence-study helpers on the HIP path against the oracle, and the paper's
qualitative 2D claims (Sec. III-A to III-C, the TV comparison of Sec. III-E) on GPU runs.

Parity: the least-squares reference and ||A||^2 within 1e-5 relative; DS curves within
2e-4 DS0 + 1e-3 DS of the oracle's at every checkpoint (same seeds, so the same block
selections; FP32 iterates against FP64); image SNR within 0.05 dB.
"""
import numpy as np
import pytest

from bsgd_inputs.configs import study_geometry

from helpers import log, oracle_ds_curve, oracle_problem, oracle_study, rel_l2, require_gpu

pytestmark = pytest.mark.gpu
PRODUCTS = 8000


def _dev(a, dev):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)


def _close(gpu, ref, ds0):
    assert [p for p, _ in gpu] == [p for p, _ in ref]
    for (_, a), (_, b) in zip(gpu, ref):
        assert abs(a - b) <= 2e-4 * ds0 + 1e-3 * b, (gpu, ref)


def test_least_squares_reference_and_norm():
    import torch
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.study import least_squares, spectral_norm_sq
    dev = require_gpu()
    log("study: CGLS and power iteration on the 16x16 setup")
    _, y, _, x_lsq, L = oracle_study("e1")
    geom = Geometry(study_geometry("e1", 1, 1, 1))
    x = least_squares(geom, _dev(y, dev))
    assert x.dtype == torch.float64
    assert rel_l2(x.cpu().numpy(), x_lsq) <= 1e-5
    assert abs(spectral_norm_sq(geom, dev) - L) <= 1e-5 * L


@pytest.mark.parametrize("M,bx,by,R,B,scale", [(4, 2, 1, 4, 2, 1.0), (2, 8, 4, 1, 1, 2.0), (4, 4, 4, 1, 1, 2.0),
                                               (8, 4, 2, 1, 1, 2.0), (4, 4, 4, 4, 1, 2.0), (4, 4, 4, 2, 2, 2.0),
                                               (4, 4, 4, 1, 4, 2.0)])
def test_ds_curves_match_oracle(M, bx, by, R, B, scale):
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.study import ds_curve
    dev = require_gpu()
    log(f"study: DS curve {M}x{bx * by} pairs {R}x{B}")
    _, y, _, x_lsq, L = oracle_study("e1")
    mu = scale / (2 * L)
    g = study_geometry("e1", M, bx, by)
    gpu = ds_curve(Geometry(g), _dev(y, dev), _dev(x_lsq, dev), R, B, mu, PRODUCTS)
    ref = oracle_ds_curve(oracle_problem(g), y, x_lsq, R, B, mu, PRODUCTS)
    _close(gpu, ref, np.linalg.norm(x_lsq))


def test_paper_claims_on_gpu_runs():
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.study import ds_curve
    dev = require_gpu()
    log("study: claims of Sec. III-A to III-C")
    _, y, _, x_lsq, L = oracle_study("e1")
    yd, xd = _dev(y, dev), _dev(x_lsq, dev)
    ds0 = np.linalg.norm(x_lsq)

    def curve(M, bx, by, R, B, scale):
        return [v for _, v in ds_curve(Geometry(study_geometry("e1", M, bx, by)), yd, xd, R, B,
                                       scale / (2 * L), PRODUCTS)]

    d = curve(4, 2, 1, 4, 2, 1.0)
    assert d[-1] < 0.01 * ds0 and all(b < 0.8 * a for a, b in zip(d, d[1:]))
    ends = []
    for M, bx, by in ((2, 8, 4), (4, 4, 4), (8, 4, 2)):
        d = curve(M, bx, by, 1, 1, 2.0)
        assert d[-1] < 0.04 * ds0 and all(b < a for a, b in zip(d[-4:], d[-3:]))
        ends.append(d[-1])
    assert max(ends) > 2.0 * min(ends)
    c = [curve(4, 4, 4, R, B, 2.0) for R, B in ((4, 1), (2, 2), (1, 4))]
    assert all(c[0][k] > c[1][k] > c[2][k] for k in range(4, 8))
    assert c[0][-1] > 3.0 * c[2][-1]


def test_tv_comparison_matches_oracle():
    from oracle.bsgd import run, snr_db
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.study import snr_curve
    dev = require_gpu()
    log("study: TV comparison on the 64x64 setup")
    _, y, x_true, _, L = oracle_study("e6")
    g = study_geometry("e6", 20, 2, 2, partition_seed=6)
    p = oracle_problem(g)
    mu, epochs = 1.0 / (2 * L), 60
    geom = Geometry(g)
    yd, xt = _dev(y, dev), _dev(x_true, dev)
    tv = snr_curve(geom, yd, xt, 1, 2, mu, epochs, n_points=1, tv_lambda=100.0)[-1][1]
    gd = snr_curve(geom, yd, xt, 20, 4, mu, epochs, n_points=1)[-1][1]
    tv_ref = snr_db(x_true, run(p, y, mu, 1, 2, epochs * 40, seed=1, tv_lambda=100.0).x)
    gd_ref = snr_db(x_true, run(p, y, mu, 20, 4, epochs, seed=1).x)
    assert abs(tv - tv_ref) <= 0.05 and abs(gd - gd_ref) <= 0.05
    assert tv > gd + 5.0


def test_study_tables_run():
    from paper_1903_11874_amd.study import gamma_study, partition_study
    dev = require_gpu()
    log("study: table drivers")
    res = partition_study(dev, n_products=2000)
    assert len(res["rows"]) == 4
    for scale, curve in res["rows"].values():
        assert np.isfinite(curve[-1][1]) and curve[-1][1] < res["ds0"]
    res = gamma_study(dev, n_products=2000)
    assert len(res["rows"]) == 3
