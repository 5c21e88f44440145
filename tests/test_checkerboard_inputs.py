"""CPU checks of the checkerboard experiment's inputs (Sec. IV): block
layout, scan parameters of both pixel-size readings, noise level."""
import numpy as np
import pytest

from paper_2511_12235_amd import experiments as E


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 48), (3, 16), (3, 32)])
def test_checkerboard_blocks(dim, n):
    g = E.geometry(dim, n)
    u = E.checkerboard(g)
    assert u.shape == g.vol_shape
    assert set(np.unique(u)) == {0.0, 1.0}
    assert u.mean() == 0.5
    b = n // 4  # 4 blocks per axis, constant inside each block
    blocks = (u[0] if dim == 2 else u).reshape(*([4, b] * dim))
    axes = tuple(range(1, 2 * dim, 2))
    assert np.all(blocks.min(axis=axes) == blocks.max(axis=axes))
    # neighbouring blocks differ along every axis
    cells = blocks.min(axis=axes)
    for ax in range(dim):
        assert np.all(np.diff(cells, axis=ax) != 0)


def test_scan_parameters():
    for dim in (2, 3):
        for reading, pitch in (("fov", 16.0 / 32), ("unit", 1.0)):
            g = E.geometry(dim, 32, reading)
            assert g.n_p == 60 and g.det_ny == 60 and g.dy == 0.75
            assert g.s == 250.0 and g.d == 250.0 and g.a == pitch
            assert np.allclose(g.phi, 2 * np.pi * np.arange(60) / 60)
            if dim == 3:
                assert g.det_nz == 60 and g.dz == 0.75 and g.c == pitch
    # the "fov" reading keeps the image inside the beam: the 60 x 0.75 detector
    # at magnification 500 / 250 sees a field 22.5 units wide at the centre,
    # more than the 16-unit image (its corners, 11.3 from the axis, lie nearer
    # the source or the detector and are covered as well in every view)
    assert 0.5 * 60 * 0.75 * 250.0 / 500.0 > 8.0


def test_noise_level():
    g = E.geometry(2, 16)
    e = E.noise(g, 3)
    assert e.shape == g.sino_shape
    assert abs(e.std() - E.SIGMA) < 0.05 * E.SIGMA
    assert np.array_equal(e, E.noise(g, 3))
