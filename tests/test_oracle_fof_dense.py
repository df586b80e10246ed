"""Pins of the oracle's dense-particle FOF variant (Section 3.1, `fof_dense`):
brute-force components of the variant's links, the bounds the paper states
(at least the standard groups), and the off switch."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from tests.test_oracle_pins import brute_fof, clustered, particles


def brute_dense(pos, box, ll, t):
    """Friends within ll, plus every pair within 2 ll that has a particle
    with more than t friends within ll; components labelled by their
    smallest index."""
    n = pos.shape[0]
    d = pos[:, None, :] - pos[None, :, :]
    d = d - box * np.round(d / box)
    r2 = (d * d).sum(-1)
    np.fill_diagonal(r2, np.inf)
    near = r2 <= ll * ll
    dense = near.sum(1) > t
    adj = near | ((dense[:, None] | dense[None, :]) & (r2 <= 4 * ll * ll))
    ncomp, lab = connected_components(csr_matrix(adj), directed=False)
    mins = np.full(ncomp, n)
    np.minimum.at(mins, lab, np.arange(n))
    return mins[lab], dense


@pytest.mark.parametrize("seed,f64,n,box,b", [(1, True, 1500, 10.0, 0.28),
                                              (2, False, 2000, 10.0, 0.28),
                                              (3, True, 400, 2.0, 1.5)])
def test_dense_variant_matches_brute_force(orc, seed, f64, n, box, b):
    """Cell-grid path (a box of >= 3 cells of 2 ll) and, with b = 1.5 (2 ll
    over a third of the box), the all-pairs path."""
    pos, vel = clustered(n, box, seed, f64=f64)
    t = 16
    p = orc.make_params(box, 1.0, 0.01, b=b, fof_dense=t)
    lab = orc.fof3d(p, particles(orc, pos, vel))
    ll = b * box / n ** (1 / 3)
    want, dense = brute_dense(pos.astype(np.float64), box, ll, t)
    assert dense.sum() > 20
    np.testing.assert_array_equal(lab, want)


def test_dense_variant_is_a_coarsening(orc):
    """Every standard group lies inside one variant group (the paper's
    'links at minimum the same particles'), and the variant joins some."""
    pos, vel = clustered(3000, 12.0, 4, f64=True, spread=0.6)
    P = particles(orc, pos, vel)
    std = orc.fof3d(orc.make_params(12.0, 1.0, 0.01), P)
    var = orc.fof3d(orc.make_params(12.0, 1.0, 0.01, fof_dense=16), P)
    np.testing.assert_array_equal(std, brute_fof(pos, 12.0, 0.28 * 12.0 / 3000 ** (1 / 3)))
    for g in np.unique(std):
        assert np.unique(var[std == g]).shape[0] == 1
    assert np.unique(var).shape[0] < np.unique(std).shape[0]


def test_dense_threshold_above_every_count_is_standard(orc):
    pos, vel = clustered(1500, 10.0, 5, f64=True)
    P = particles(orc, pos, vel)
    a = orc.fof3d(orc.make_params(10.0, 1.0, 0.01), P)
    b = orc.fof3d(orc.make_params(10.0, 1.0, 0.01, fof_dense=10 ** 6), P)
    np.testing.assert_array_equal(a, b)
