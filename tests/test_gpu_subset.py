"""The subset form of the linking length (Section 3.2, `ell_subset`) on the
GPU against the oracle: the whole hierarchy, halo table and memberships bit
for bit, through the all-pairs and the tile-search paths, in both launch
forms."""
import numpy as np
import pytest

from tests.gpu_util import note, particles_from_arrays, to_np
from tests.test_gpu_edges import compare_all
from tests.test_oracle_pins import clustered, particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


@pytest.mark.parametrize("m", [1000, 3000])
def test_subset_c1(H, orc, c1, m):
    note(f"ell subset c1 m={m}")
    o = orc.run_all(orc.params_of(c1, ell_subset=m), orc.Particles.of(c1))
    big = int(np.sum((o["nodes"]["count"] > m) & (o["nodes"]["ell2"] >= 0)))
    assert big >= 3  # the subset form is exercised
    r = H.Halo(H.params_for_catalog(c1, ell_subset=m)).run_all(H.Particles.from_catalog(c1))
    compare_all(r, o)
    np.testing.assert_array_equal(to_np(r["bound"]), o["bound"])


@pytest.mark.parametrize("grid_min,mode", [(64, 1), (64, 0), (0, 0)])
def test_subset_clustered(H, orc, grid_min, mode):
    """Nodes above 300 particles take the subset; grid_min = 64 sends every
    node through the tile search (and its all-pairs fall-back)."""
    note(f"ell subset clustered grid_min={grid_min} mode={mode}")
    n, box = 9000, 15.0
    pos, vel = clustered(n, box, 32, nblob=5, spread=0.3, f64=False)
    p = orc.make_params(box, 1e11, 0.005, ell_subset=300)
    o = orc.run_all(p, particles(orc, pos, vel))
    r = H.Halo(H.Params(box=box, particle_mass=1e11, softening=0.005, ell_subset=300,
                        grid_min=grid_min, mode=mode)).run_all(particles_from_arrays(pos, vel))
    compare_all(r, o)


def test_subset_above_every_node_is_exact(H, c1):
    note("ell subset above every node == exact")
    P = H.Particles.from_catalog(c1)
    a = H.Halo(H.params_for_catalog(c1)).run_all(P)
    b = H.Halo(H.params_for_catalog(c1, ell_subset=10 ** 7)).run_all(P)
    for k in a["nodes"]:
        np.testing.assert_array_equal(to_np(a["nodes"][k]), to_np(b["nodes"][k]), err_msg=k)
    np.testing.assert_array_equal(to_np(a["halo_of"]), to_np(b["halo_of"]))
