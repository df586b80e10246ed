"""The dense-particle FOF variant (Section 3.1, `fof_dense`) on the GPU against
the oracle: labels bit for bit, the whole path on the 32^3 catalogue, the
off switch and the small-box error."""
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


@pytest.mark.parametrize("seed,f64,n,box", [(1, True, 1500, 10.0), (2, False, 2000, 10.0),
                                            (6, False, 20000, 25.0)])
def test_dense_labels(H, orc, seed, f64, n, box):
    note(f"fof dense seed={seed} f64={f64} n={n}")
    pos, vel = clustered(n, box, seed, f64=f64)
    o = orc.fof3d(orc.make_params(box, 1.0, 0.01, fof_dense=16), particles(orc, pos, vel))
    ctx = H.Halo(H.Params(box=box, particle_mass=1.0, softening=0.01, fof_dense=16))
    g = ctx.fof3d(particles_from_arrays(pos, vel))
    np.testing.assert_array_equal(to_np(g["label"]).astype(np.int64), o.astype(np.int64))


def test_dense_whole_path_c1(H, orc, c1):
    note("fof dense whole path c1")
    o = orc.run_all(orc.params_of(c1, fof_dense=16), orc.Particles.of(c1))
    r = H.Halo(H.params_for_catalog(c1, fof_dense=16)).run_all(H.Particles.from_catalog(c1))
    compare_all(r, o)


def test_dense_off(H, c1):
    note("fof dense off == standard")
    P = H.Particles.from_catalog(c1)
    a = H.Halo(H.params_for_catalog(c1)).fof3d(P)
    b = H.Halo(H.params_for_catalog(c1, fof_dense=10 ** 6)).fof3d(P)
    np.testing.assert_array_equal(to_np(a["label"]), to_np(b["label"]))


def test_dense_small_box_error(H):
    """b = 1.8 leaves 8 cells per side: enough for the ll stencil (2R+1 = 5),
    too few for the 2 ll one (2Q+1 = 9)."""
    note("fof dense small box error")
    pos, vel = clustered(400, 2.0, 3)
    ctx = H.Halo(H.Params(box=2.0, particle_mass=1.0, softening=0.01, b=1.8, fof_dense=16))
    with pytest.raises(H.HaloError) as e:
        ctx.fof3d(particles_from_arrays(pos, vel))
    assert e.value.code == -1
