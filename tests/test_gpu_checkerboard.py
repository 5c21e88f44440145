"""The checkerboard reconstructions of Sec. IV on the GPU against the same
pipeline run with the FP64 oracle's W on the CPU (oracle power iteration,
data and NAG), at 16^2 and 16^3: the reconstructed images must agree to
1e-8 relative L2 in FP64.  The MSE against the true checkerboard is checked
only loosely (the paper's printed values are context, not a target)."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import solvers as S
from paper_2511_12235_amd import experiments as E

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dim", [2, 3])
def test_checkerboard_matches_oracle_pipeline(dim):
    print("[case] checkerboard", dim, flush=True)
    n, seed = 16, 0
    r = E.run(dim, n, "fov", "fp64", seed=seed)
    g = E.geometry(dim, n, "fov")
    W = O.matrix(g)
    u = E.checkerboard(g).ravel()
    norm = S.power_norm(W, E.start_vector(g, seed + 1).ravel(), E.POWER_ITERS)
    assert abs(r["norm"] - norm) <= 1e-12 * norm
    p = (W @ u) / norm + E.noise(g, seed + 2).ravel()
    x_ref, h_ref = S.nag(W, p, np.zeros(g.n_vox), E.ITERS[dim], norm, lam=E.LAM, s=1.0 / norm)
    assert _rel(r["x"].ravel(), x_ref) <= 1e-8
    assert r["mse"] == pytest.approx(float(np.mean((x_ref - u) ** 2)), rel=1e-6)
    assert r["mse"] < 0.1
