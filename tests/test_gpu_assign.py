"""Seeds, merging, assignment and host/sub on the GPU against the oracle
(Sections 3.3-3.4).  Integer outputs and the FP64 seed metrics must match bit
for bit (exact sums and maxima on both sides)."""
import numpy as np
import pytest

from tests.gpu_util import note, particles_from_arrays, to_np
from tests.test_gpu_refine6d import gpu_nodes, subset_nodes
from tests.test_oracle_pins import clustered, particles
from tests.test_oracle_readings import clump_lattice

pytestmark = pytest.mark.gpu

HFIELDS = ["seed_node", "merged_into", "host", "fof", "n_assigned", "xs", "ys", "zs", "vxs",
           "vys", "vzs", "sv2", "vmax2"]


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def assert_halos_equal(g, o):
    assert g["seed_node"].shape[0] == o["seed_node"].shape[0], "halo counts differ"
    for f in HFIELDS:
        a, b = np.asarray(g[f]), np.asarray(o[f])
        if a.dtype.kind == "f":
            ok = np.array_equal(a.view(np.uint64), b.astype(np.float64).view(np.uint64))
        else:
            ok = np.array_equal(a.astype(np.int64), b.astype(np.int64))
        if not ok:
            bad = np.nonzero(a.astype(np.float64) != b.astype(np.float64))[0][:5]
            raise AssertionError(f"halo field {f} differs at {bad}: gpu {a[bad]} oracle {b[bad]}")


def gpu_pipeline(H, P, params):
    ctx = H.Halo(params)
    fof = ctx.fof3d(P)
    nodes, deepest = ctx.refine6d(P, fof)
    halos, halo_of = ctx.assign(P, nodes, deepest)
    return fof, nodes, deepest, {k: to_np(v) for k, v in halos.items()}, to_np(halo_of)


@pytest.mark.parametrize("n,seed,f64,mode", [(4000, 21, True, 1), (9000, 22, False, 1),
                                             (4000, 21, True, 0)])
def test_assign_clustered(H, orc, n, seed, f64, mode):
    note(f"assign clustered n={n} seed={seed} f64={f64} mode={mode}")
    box = 10.0 * (n / 1500) ** (1 / 3)
    pos, vel = clustered(n, box, seed, nblob=5, spread=0.3, f64=f64)
    p = orc.make_params(box, 1e10, 0.01)
    P = particles(orc, pos, vel)
    o = orc.run_all(p, P)
    _, _, _, gh, gho = gpu_pipeline(H, particles_from_arrays(pos, vel),
                                    H.Params(box=box, particle_mass=1e10, softening=0.01,
                                             mode=mode))
    assert_halos_equal(gh, o["halos"])
    np.testing.assert_array_equal(gho, o["halo_of"])


def test_assign_c1(H, c1, c1_oracle):
    note("assign c1")
    _, _, _, gh, gho = gpu_pipeline(H, H.Particles.from_catalog(c1), H.params_for_catalog(c1))
    o = c1_oracle
    assert_halos_equal(gh, o["halos"])
    np.testing.assert_array_equal(gho, o["halo_of"])
    kept = gh["merged_into"] == np.arange(gh["merged_into"].shape[0])
    assert kept.sum() >= 10 and (~kept).sum() >= 1


def test_assign_c2_sampled(H, orc, c2, c2_fof_oracle):
    """128^3 catalogue; the oracle runs refine + assign on sampled FOF groups
    (its own FOF labels, every other group cut into singletons)."""
    note("assign c2 sampled")
    cat = c2
    fof, gn, gd, gh, gho = gpu_pipeline(H, H.Particles.from_catalog(cat),
                                        H.params_for_catalog(cat))
    lab = np.asarray(c2_fof_oracle).astype(np.int64)
    sizes = np.bincount(lab, minlength=lab.shape[0])
    groups = np.nonzero(sizes >= 10)[0]
    rng = np.random.default_rng(1)
    small = groups[sizes[groups] <= 1500]
    mid = groups[(sizes[groups] > 2000) & (sizes[groups] <= 8000)]
    keep = np.sort(np.concatenate([rng.choice(small, 150, replace=False),
                                   rng.choice(mid, min(3, mid.shape[0]), replace=False)]))
    lab_s = np.where(np.isin(lab, keep), lab, np.arange(lab.shape[0])).astype(np.uint32)
    p = orc.params_of(cat)
    Pc = orc.Particles.of(cat)
    on, od = orc.refine6d(p, Pc, lab_s)
    oh, oho = orc.assign(p, Pc, on, od)
    gn = gpu_nodes(gn)
    _, node_remap = subset_nodes(gn, keep)
    rows = np.nonzero(np.isin(gh["fof"].astype(np.int64), keep))[0]
    hre = np.full(gh["fof"].shape[0] + 1, -1, np.int64)
    hre[rows] = np.arange(rows.shape[0])
    sub = {k: v[rows].copy() for k, v in gh.items()}
    sub["seed_node"] = node_remap[sub["seed_node"]]
    for k in ("merged_into", "host"):
        v = sub[k].astype(np.int64)
        sub[k] = np.where(v >= 0, hre[v], -1)
    assert_halos_equal(sub, oh)
    inside = np.isin(lab, keep)
    g_in = gho[inside].astype(np.int64)
    np.testing.assert_array_equal(np.where(g_in >= 0, hre[g_in], -1), oho[inside])
    assert np.all((gho >= 0) == (sizes[lab] >= 10))


def test_assign_repeat(H, c1):
    note("assign repeat x2")
    a = gpu_pipeline(H, H.Particles.from_catalog(c1), H.params_for_catalog(c1))
    b = gpu_pipeline(H, H.Particles.from_catalog(c1), H.params_for_catalog(c1))
    assert_halos_equal(a[3], b[3])
    np.testing.assert_array_equal(a[4], b[4])


def test_assign_many_seeds_one_group(H, orc):
    """One FOF group with more than 512 seeds: merging runs in the block-per-
    group form, and the host/subhalo relation covers hundreds of halos in one
    group."""
    note("assign many seeds in one group")
    pos, vel, box = clump_lattice()
    p = orc.make_params(box, 1e10, 0.01)
    P = particles(orc, pos, vel)
    o = orc.run_all(p, P)
    fof = np.asarray(o["halos"]["fof"])
    assert np.unique(fof).shape[0] == 1 and fof.shape[0] > 512
    assert np.any(np.asarray(o["halos"]["merged_into"]) != np.arange(fof.shape[0]))
    _, _, _, gh, gho = gpu_pipeline(H, particles_from_arrays(pos, vel),
                                    H.Params(box=box, particle_mass=1e10, softening=0.01))
    assert_halos_equal(gh, o["halos"])
    np.testing.assert_array_equal(gho, o["halo_of"])
