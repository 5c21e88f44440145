"""Pins of the reference solvers (oracle/solvers.py) against facts outside
them: the largest singular value from a dense SVD, the least-squares and
Tikhonov solutions from direct dense solves, and the monotone decrease of the
CGLS data residual.  The system matrices are the oracle's on tiny scans."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import solvers as S
from paper_2511_12235_amd import workloads as wl


@pytest.fixture(scope="module")
def small2d():
    # 8 x 8 pixels, 30 views, 16 cells: 480 rays >> 64 unknowns
    g = wl.make_geometry(2, (8, 8), (1.0, 1.0), 30, 40.0, 40.0, (16,), (1.25,))
    W = O.matrix(g)
    return g, W, W.toarray()


@pytest.fixture(scope="module")
def small3d():
    g = wl.make_geometry(3, (5, 4, 4), (1.0, 1.0, 1.0), 24, 30.0, 30.0, (10, 9), (1.1, 1.2))
    W = O.matrix(g)
    return g, W, W.toarray()


def test_power_norm_matches_svd(small2d, small3d):
    for g, W, Wd in (small2d, small3d):
        sig = np.linalg.svd(Wd, compute_uv=False)[0]
        v0 = wl.uniform(g.vol_shape, 5)
        est = S.power_norm(W, v0, 400)
        assert est <= sig * (1 + 1e-12)
        assert abs(est - sig) / sig < 1e-9


def test_cgls_reaches_least_squares(small2d):
    g, W, Wd = small2d
    x_true = wl.ellipse_phantom(g, 3, seed=4).ravel()
    p = Wd @ x_true + 1e-3 * np.random.default_rng(1).standard_normal(Wd.shape[0])
    x_ls = np.linalg.lstsq(Wd, p, rcond=None)[0]
    x, hist = S.cgls(W, p, np.zeros(g.n_vox), 3 * g.n_vox)
    assert np.linalg.norm(x - x_ls) / np.linalg.norm(x_ls) < 1e-8
    assert hist[-1] < 1e-16 * hist[0]


def test_cgls_tikhonov_and_scale(small3d):
    g, W, Wd = small3d
    p = wl.uniform(g.sino_shape, 2).ravel()
    lam, s = 0.05, 0.3
    x_ref = np.linalg.solve(s * s * Wd.T @ Wd + lam * np.eye(g.n_vox), s * Wd.T @ p)
    x, _ = S.cgls(W, p, np.zeros(g.n_vox), 200, lam=lam, s=s)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-9


def test_cgls_residual_is_monotone(small3d):
    """CGLS minimises |p - W x| over growing Krylov spaces, so the data
    residual never increases."""
    g, W, Wd = small3d
    p = wl.uniform(g.sino_shape, 3).ravel()
    res = []
    for k in range(12):
        x, _ = S.cgls(W, p, np.zeros(g.n_vox), k)
        res.append(np.linalg.norm(p - Wd @ x))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))


def test_nag_converges_to_tikhonov_solution(small2d):
    g, W, Wd = small2d
    p = wl.uniform(g.sino_shape, 6).ravel()
    sig = np.linalg.svd(Wd, compute_uv=False)[0]
    lam, s = 0.02, 1.0 / sig
    x_ref = np.linalg.solve(s * s * Wd.T @ Wd + lam * np.eye(g.n_vox), s * Wd.T @ p)
    x, hist = S.nag(W, p, np.zeros(g.n_vox), 3000, sig, lam=lam, s=s)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8
    assert hist[-1] < 1e-12 * hist[0]
    # the objective at the limit is the minimum: no direction decreases it
    f0 = S.objective(W, p, x_ref, lam, s)
    for seed in range(3):
        d = wl.random_unit(g.n_vox, seed).ravel() * 1e-3
        assert S.objective(W, p, x_ref + d, lam, s) >= f0
