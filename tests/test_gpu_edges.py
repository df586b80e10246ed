"""Edge cases of the whole path on the GPU: no FOF group at all, a single
group of exactly min_members particles, the smallest inputs, and the two
errors the method raises (a group spanning half the box, an out-of-range
velocity).  Where there is output, it is compared with the oracle's."""
import numpy as np
import pytest
import torch

from tests.gpu_util import note, particles_from_arrays, to_np
from tests.test_gpu_assign import assert_halos_equal
from tests.test_gpu_refine6d import assert_nodes_equal, gpu_nodes
from tests.test_oracle_pins import particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def run_gpu(H, pos, vel, box, **kw):
    P = particles_from_arrays(pos, vel)
    ctx = H.Halo(H.Params(box=box, particle_mass=1e10, softening=0.01, **kw))
    r = ctx.run_all(P)
    torch.cuda.synchronize()
    return r


def compare_all(r, o):
    np.testing.assert_array_equal(to_np(r["fof"]["label"]).astype(np.int64),
                                  o["label"].astype(np.int64))
    assert_nodes_equal(gpu_nodes(r["nodes"]), o["nodes"])
    np.testing.assert_array_equal(to_np(r["deepest"]).astype(np.int64),
                                  o["deepest"].astype(np.int64))
    assert_halos_equal({k: to_np(v) for k, v in r["halos"].items()},
                       {k: np.asarray(v) for k, v in o["halos"].items()})
    np.testing.assert_array_equal(to_np(r["halo_of"]).astype(np.int64),
                                  o["halo_of"].astype(np.int64))


def test_no_group(H, orc):
    """Uniform points far sparser than the linking length: every FOF group is
    below min_members, so there are no nodes, no haloes and nothing bound."""
    note("edges: no FOF group")
    rng = np.random.default_rng(41)
    box = 100.0
    pos = rng.random((3000, 3)) * box
    vel = (100 * rng.standard_normal((3000, 3))).astype(np.float32)
    r = run_gpu(H, pos, vel, box)
    assert int(r["fof"]["n_groups"]) == 0
    assert r["nodes"]["parent"].shape[0] == 0
    assert r["halos"]["seed_node"].shape[0] == 0
    assert bool((to_np(r["halo_of"]) == -1).all())
    assert int(to_np(r["bound"]).sum()) == 0
    o = orc.run_all(orc.make_params(box, 1e10, 0.01), particles(orc, pos, vel))
    np.testing.assert_array_equal(to_np(r["fof"]["label"]).astype(np.int64),
                                  o["label"].astype(np.int64))
    assert o["nodes"]["parent"].shape[0] == 0


def test_single_group_of_min_members(H, orc):
    """Exactly min_members particles in one tight clump among isolated points:
    one node, one halo, the whole path as the oracle has it."""
    note("edges: one group of 10")
    rng = np.random.default_rng(42)
    box = 100.0
    far = rng.random((2000, 3)) * box
    far = far[np.linalg.norm(far - 50.0, axis=1) > 5.0]  # nothing within reach of the clump
    clump = 50.0 + 0.01 * rng.standard_normal((10, 3))
    pos = np.concatenate([far, clump])
    vel = (30 * rng.standard_normal((pos.shape[0], 3))).astype(np.float32)
    r = run_gpu(H, pos, vel, box)
    o = orc.run_all(orc.make_params(box, 1e10, 0.01), particles(orc, pos, vel))
    assert int(r["fof"]["n_groups"]) == 1
    compare_all(r, o)
    np.testing.assert_array_equal(to_np(r["bound"]), o["bound"])


@pytest.mark.parametrize("n", [1, 2])
def test_smallest_inputs(H, orc, n):
    note(f"edges: n = {n}")
    pos = np.array([[1.0, 1.0, 1.0], [1.0001, 1.0, 1.0]])[:n]
    vel = np.zeros((n, 3), np.float32)
    r = run_gpu(H, pos, vel, 10.0)
    o = orc.run_all(orc.make_params(10.0, 1e10, 0.01), particles(orc, pos, vel))
    np.testing.assert_array_equal(to_np(r["fof"]["label"]).astype(np.int64),
                                  o["label"].astype(np.int64))
    assert r["halos"]["seed_node"].shape[0] == 0


def test_group_spanning_half_the_box(H):
    """A chain of friends across more than half the periodic box cannot be
    unwrapped about its anchor: refinement reports a geometry error."""
    note("edges: group spanning L/2")
    box = 10.0
    n = 200
    ll = 0.28 * box / n ** (1.0 / 3.0)
    chain = np.stack([0.5 + 0.9 * ll * np.arange(14), np.full(14, 5.0), np.full(14, 5.0)], 1)
    assert chain[-1, 0] - chain[0, 0] > 0.5 * box
    rng = np.random.default_rng(44)
    rest = rng.random((n - 14, 3)) * box
    rest[:, 1] = np.where(np.abs(rest[:, 1] - 5.0) < 2.0, rest[:, 1] + 4.0, rest[:, 1]) % box
    pos = np.concatenate([chain, rest])
    vel = np.zeros((n, 3), np.float32)
    P = particles_from_arrays(pos, vel)
    ctx = H.Halo(H.Params(box=box, particle_mass=1e10, softening=0.01))
    fof = ctx.fof3d(P)
    assert int(fof["n_groups"]) >= 1
    with pytest.raises(H.HaloError) as e:
        ctx.refine6d(P, fof)
    assert e.value.code == -5


def test_velocity_out_of_range(H):
    """Velocities are summed in 2^-24 km/s fixed point; |v| >= 2^16 km/s is
    rejected rather than overflowing."""
    note("edges: velocity out of range")
    rng = np.random.default_rng(43)
    pos = 5.0 + 0.01 * rng.standard_normal((50, 3))
    vel = np.zeros((50, 3), np.float32)
    vel[7, 1] = 7.0e4
    P = particles_from_arrays(pos, vel)
    ctx = H.Halo(H.Params(box=10.0, particle_mass=1e10, softening=0.01))
    fof = ctx.fof3d(P)
    with pytest.raises(H.HaloError) as e:
        ctx.refine6d(P, fof)
    assert e.value.code == -1
