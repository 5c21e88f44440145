"""Stored-W mode (device CSR of W and W^T, sparse products) against the
host CSR of sm_weights_csr (bit-exact pattern and values), the FP64 oracle
and the matrix-free operators."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import oracle as O
from paper_2511_12235_amd import workloads as wl
from paper_2511_12235_amd.projector import StoredMatrix, SystemMatrix

from _errlog import errors, record

from test_gpu_parity import GEOMS, TOL, _t

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("name", ["fan_odd", "cone_small", "cone_many_rows"])
def test_stored_arrays_equal_host_csr(name):
    print("[case] stored arrays", name, flush=True)
    g = GEOMS[name]
    A = SystemMatrix(g, "fp64", device=DEV)
    ptr, col, val = A.weights_csr("fp64")
    S = StoredMatrix(A, "fp64")
    assert S.nnz == len(col)
    assert np.array_equal(S.W[0].cpu().numpy(), ptr)
    assert np.array_equal(S.W[1].cpu().numpy()[: S.nnz], col)
    assert np.array_equal(S.W[2].cpu().numpy()[: S.nnz], val)
    Wt = sp.csr_matrix((val, col, ptr), shape=(A.n_rays, A.n_vox)).T.tocsr()
    Wt.sort_indices()
    assert np.array_equal(S.Wt[0].cpu().numpy(), Wt.indptr)
    assert np.array_equal(S.Wt[1].cpu().numpy()[: S.nnz], Wt.indices)
    assert np.array_equal(S.Wt[2].cpu().numpy()[: S.nnz], Wt.data)


@pytest.mark.parametrize("name", ["c1_fan64", "cone_small", "cone_aniso_offset"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stored_products_match_oracle_and_matrix_free(name, prec):
    print("[case] stored products", name, prec, flush=True)
    g = GEOMS[name]
    W = O.matrix(g)
    A = SystemMatrix(g, prec, device=DEV)
    S = StoredMatrix(A)
    x = wl.ellipse_phantom(g, 5, seed=3)
    y = wl.uniform(g.sino_shape, 4)
    ys = S.forward(_t(x, prec)).cpu().numpy()
    xs = S.back(_t(y, prec)).cpu().numpy()
    assert record("stored W x, %s %s" % (name, prec), ys, W @ x.ravel(), TOL[prec])[0] <= TOL[prec]
    assert record("stored W^T y, %s %s" % (name, prec), xs, W.T @ y.ravel(), TOL[prec])[0] <= TOL[prec]
    assert errors(ys, A.forward(_t(x, prec)).cpu().numpy())[0] <= 2 * TOL[prec]
    assert errors(xs, A.back(_t(y, prec)).cpu().numpy())[0] <= 2 * TOL[prec]
    # deterministic, and batches are independent products
    assert np.array_equal(ys, S.forward(_t(x, prec)).cpu().numpy())
    xb = np.stack([x, 2.0 * x])
    yb = S.forward(_t(xb, prec)).cpu().numpy()
    assert np.array_equal(yb[0], ys)


def test_stored_medium_size_matches_matrix_free():
    print("[case] stored 64^3", flush=True)
    g = wl.scaled(wl.c2_cone128(), (64, 64, 64), (96, 64), 45)
    A = SystemMatrix(g, "fp32", device=DEV)
    S = StoredMatrix(A)
    x = torch.from_numpy(wl.ellipse_phantom(g, 10, seed=1)).to(DEV, torch.float32)
    y = torch.from_numpy(wl.uniform(g.sino_shape, 2)).to(DEV, torch.float32)
    assert errors(S.forward(x).cpu().numpy(), A.forward(x).cpu().numpy())[0] <= 2e-5
    assert errors(S.back(y).cpu().numpy(), A.back(y).cpu().numpy())[0] <= 2e-5
