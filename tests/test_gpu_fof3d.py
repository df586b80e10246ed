"""3D FOF on the GPU against the CPU oracle (Section 3.1): labels bit-exact."""
import numpy as np
import pytest

from tests.gpu_util import note, particles_from_arrays, to_np
from tests.test_oracle_pins import clustered, particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def _run(H, orc, pos, vel, box, **kw):
    p_orc = orc.make_params(box, 1e10, 0.01, **kw)
    want = orc.fof3d(p_orc, particles(orc, pos, vel))
    ctx = H.Halo(H.Params(box=box, particle_mass=1e10, softening=0.01, **kw))
    P = particles_from_arrays(pos, vel)
    got = ctx.fof3d(P)
    return want, got


def _check_groups(want, got, mm=10):
    lab = to_np(got["label"]).astype(np.int64)
    np.testing.assert_array_equal(lab, want.astype(np.int64))
    sizes = np.bincount(want, minlength=want.shape[0])
    members = np.nonzero(sizes[want] >= mm)[0]
    order = np.lexsort((members, want[members]))
    np.testing.assert_array_equal(to_np(got["perm"]).astype(np.int64), members[order])
    labels = np.unique(want[members])
    assert got["n_groups"] == labels.shape[0]
    np.testing.assert_array_equal(to_np(got["grp_count"]), sizes[labels])
    first = to_np(got["grp_first"]).astype(np.int64)
    np.testing.assert_array_equal(to_np(got["perm"])[first], labels)


@pytest.mark.parametrize("n,seed,f64", [(1500, 1, True), (5000, 2, False), (20011, 3, True),
                                        (777, 4, False)])
def test_fof3d_clustered(H, orc, n, seed, f64):
    note(f"fof3d clustered n={n} seed={seed} f64={f64}")
    box = 10.0 * (n / 1500) ** (1 / 3)
    pos, vel = clustered(n, box, seed, f64=f64)
    want, got = _run(H, orc, pos, vel, box)
    _check_groups(want, got)


def test_fof3d_c1(H, orc, c1):
    note("fof3d c1 32^3")
    pos = np.stack([c1.x, c1.y, c1.z], 1)
    vel = np.stack([c1.vx, c1.vy, c1.vz], 1)
    want, got = _run(H, orc, pos, vel, c1.box)
    _check_groups(want, got)


def test_fof3d_c2_full(H, c2, c2_fof_oracle):
    """128^3 in a 100 Mpc/h box (float32 positions), full comparison."""
    note("fof3d c2 128^3")
    ctx = H.Halo(H.params_for_catalog(c2))
    got = ctx.fof3d(H.Particles.from_catalog(c2))
    _check_groups(c2_fof_oracle, got)


def test_fof3d_lattice_edge(H, orc):
    """Lattice with spacing just below / above ll: one group / singletons."""
    m = 16
    g = np.arange(m, dtype=np.float64)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    vel = np.zeros_like(pos, dtype=np.float32)
    for b, one in ((1.01, True), (0.99, False)):
        note(f"fof3d lattice b={b}")
        want, got = _run(H, orc, pos, vel, float(m), b=b)
        _check_groups(want, got)
        assert (np.unique(want).shape[0] == 1) == one


def test_fof3d_rejects_out_of_box(H):
    note("fof3d rejects positions outside the box")
    pos = np.array([[1.0, 2.0, 3.0]] * 20 + [[10.0, 1.0, 1.0]])
    vel = np.zeros_like(pos, dtype=np.float32)
    ctx = H.Halo(H.Params(box=10.0, particle_mass=1.0, softening=0.01))
    with pytest.raises(H.HaloError) as e:
        ctx.fof3d(particles_from_arrays(pos, vel))
    assert e.value.code == -1


def test_fof3d_repeat_deterministic(H, c1):
    note("fof3d repeat x3")
    ctx = H.Halo(H.params_for_catalog(c1))
    P = H.Particles.from_catalog(c1)
    outs = [ctx.fof3d(P) for _ in range(3)]
    for o in outs[1:]:
        assert np.array_equal(to_np(o["label"]), to_np(outs[0]["label"]))
        assert np.array_equal(to_np(o["perm"]), to_np(outs[0]["perm"]))
