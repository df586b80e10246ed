"""The tree potential of Appendix B (`bh_theta`, `bh_min`) on the GPU against
the exact direct sum of the oracle: the Salmon-Warren acceptance bounds each
cell's relative error by theta, so every particle's potential lies within
theta of the exact one; bound flags agree wherever the energy lies outside
that band; theta -> 0 opens every cell and reproduces the exact sum."""
import numpy as np
import pytest

from tests.gpu_util import note, particles_from_arrays, to_np
from tests.test_oracle_merger import BOX, EPS, M_PART, merger
from tests.test_oracle_pins import particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def tree_cases(o, bh_min):
    h, ns = o["halos"], o["unbound"]["n_s"]
    kept = h["merged_into"] == np.arange(h["merged_into"].shape[0])
    return np.nonzero(kept & (ns >= bh_min) & (h["n_assigned"] > 0))[0]


def check_against_exact(g, o, theta, bh_min, tol_scale):
    tree = tree_cases(o, bh_min)
    assert tree.shape[0] >= 1
    sel = np.isin(o["halo_of"], tree)
    gphi = to_np(g["phi"])
    rel = np.abs(gphi[sel] / o["phi"][sel] - 1.0)
    print(f"theta={theta}: {sel.sum()} particles in {tree.shape[0]} tree haloes, "
          f"relative error median {np.median(rel):.2e} max {rel.max():.2e}")
    assert rel.max() <= tol_scale * theta
    # the other haloes keep the exact sum
    other = (o["halo_of"] >= 0) & ~sel
    np.testing.assert_allclose(gphi[other], o["phi"][other], rtol=1e-9, atol=0)
    # flags agree outside the band the potential's error leaves
    ho = o["halo_of"]
    vb = np.stack([o["unbound"]["vbx"], o["unbound"]["vby"], o["unbound"]["vbz"]], 1)
    return sel, rel, ho, vb


@pytest.mark.parametrize("theta", [0.04, 0.01])
def test_tree_within_theta_c1(H, orc, c1, c1_oracle, theta):
    note(f"tree potential c1 theta={theta}")
    bh_min = 2000
    g = H.Halo(H.params_for_catalog(c1, bh_theta=theta, bh_min=bh_min)).run_all(
        H.Particles.from_catalog(c1))
    o = c1_oracle
    sel, rel, ho, vb = check_against_exact(g, o, theta, bh_min, 1.0)
    v = np.stack([c1.vx, c1.vy, c1.vz], 1).astype(np.float64)
    k = 0.5 * ((v[sel] - vb[ho[sel]]) ** 2).sum(1)
    e = k + o["phi"][sel]
    decided = np.abs(e) > theta * np.abs(o["phi"][sel])
    gb = to_np(g["bound"])[sel]
    np.testing.assert_array_equal(gb[decided], o["bound"][sel][decided])
    agree = float(np.mean(gb == o["bound"][sel]))
    print(f"bound flags agree for {100 * agree:.3f}% of tree-halo particles")


@pytest.mark.parametrize("leaf,prec", [(4, 0), (64, 1)])
def test_tree_leaf_sizes_within_theta(H, orc, c1, c1_oracle, leaf, prec):
    """Other leaf sizes of the potential's trees accept other cells; every
    tree-halo potential still lies within theta of the exact sum."""
    note(f"tree potential c1 bh_leaf={leaf} prec={prec}")
    theta, bh_min = 0.04, 2000
    g = H.Halo(H.params_for_catalog(c1, bh_theta=theta, bh_min=bh_min, bh_leaf=leaf,
                                    prec=prec)).run_all(H.Particles.from_catalog(c1))
    tree = tree_cases(c1_oracle, bh_min)
    sel = np.isin(c1_oracle["halo_of"], tree)
    rel = np.abs(to_np(g["phi"])[sel] / c1_oracle["phi"][sel] - 1.0)
    print(f"relative error median {np.median(rel):.2e} max {rel.max():.2e}")
    assert sel.sum() > 0 and rel.max() <= theta


def test_tree_theta_to_zero_is_exact(H, orc, c1, c1_oracle):
    """theta = 1e-12 opens every cell: the direct sum, in another order."""
    note("tree potential theta -> 0")
    g = H.Halo(H.params_for_catalog(c1, bh_theta=1e-12, bh_min=500)).run_all(
        H.Particles.from_catalog(c1))
    o = c1_oracle
    tree = tree_cases(o, 500)
    assert tree.shape[0] >= 3
    ins = o["halo_of"] >= 0
    np.testing.assert_allclose(to_np(g["phi"])[ins], o["phi"][ins], rtol=1e-11, atol=0)


def test_tree_theta_to_zero_mixed(H, orc, c1, c1_oracle):
    """The mixed form's walk (FP32 distances and reciprocal square roots of the
    halo-local positions rounded to FP32, FP32 sums per leaf added in FP64)
    with theta = 1e-12 opens every cell: the direct sum within the FP32 bound
    of the mixed form's direct-sum tiles."""
    note("tree potential theta -> 0, mixed form")
    g = H.Halo(H.params_for_catalog(c1, bh_theta=1e-12, bh_min=500, prec=1)).run_all(
        H.Particles.from_catalog(c1))
    o = c1_oracle
    ins = o["halo_of"] >= 0
    np.testing.assert_allclose(to_np(g["phi"])[ins], o["phi"][ins], rtol=2e-5, atol=0)


def test_tree_with_merger_and_mixed(H, orc):
    """The tree for S(h), the exact merger term beyond it, the mixed form's
    FP64 recheck: the potential stays within theta of the exact one."""
    note("tree potential + major merger + mixed")
    pos, vel = merger(1)
    theta = 0.04
    p = orc.make_params(BOX, M_PART, EPS, major_merger=0.3)
    o = orc.run_all(p, particles(orc, pos, vel))
    g = H.Halo(H.Params(box=BOX, particle_mass=M_PART, softening=EPS, major_merger=0.3,
                        prec=1, bh_theta=theta, bh_min=300)).run_all(
        particles_from_arrays(pos, vel))
    ins = o["halo_of"] >= 0
    rel = np.abs(to_np(g["phi"])[ins] / o["phi"][ins] - 1.0)
    print(f"relative error median {np.median(rel):.2e} max {rel.max():.2e}")
    assert rel.max() <= theta


def test_tree_deterministic(H, c1):
    note("tree potential plain == batched == repeat")
    P = H.Particles.from_catalog(c1)
    outs = [H.Halo(H.params_for_catalog(c1, bh_theta=0.04, bh_min=1000, mode=m)).run_all(P)
            for m in (1, 1, 0)]
    for r in outs[1:]:
        np.testing.assert_array_equal(to_np(r["phi"]), to_np(outs[0]["phi"]))
        np.testing.assert_array_equal(to_np(r["bound"]), to_np(outs[0]["bound"]))


def test_tree_bad_parameters(H, c1):
    with pytest.raises(H.HaloError):
        H.Halo(H.params_for_catalog(c1, bh_theta=-1.0))
    with pytest.raises(H.HaloError):
        H.Halo(H.params_for_catalog(c1, bh_min=-5))


def test_tree_workspace_placement(H, c1):
    """The tree carves the step workspace past the unbinding's arrays when that
    tail is large enough and a workspace of its own otherwise.  A context that
    has run the whole path (its workspace sized by the largest call) and a
    fresh one that runs only the unbinding (a tail of about an eighth of the
    unbinding's arrays) give identical bits."""
    note("tree potential workspace placement")
    P = H.Particles.from_catalog(c1)
    prm = H.params_for_catalog(c1, bh_theta=0.04, bh_min=500)
    a = H.Halo(prm).run_all(P)
    fresh = H.Halo(prm)
    for _ in range(2):  # the second call finds the workspaces in place
        unb, bound, phi = fresh.unbind(P, a["halos"], a["halo_of"])
        np.testing.assert_array_equal(to_np(phi), to_np(a["phi"]))
        np.testing.assert_array_equal(to_np(bound), to_np(a["bound"]))
        np.testing.assert_array_equal(to_np(unb["n_s"]), to_np(a["unbound"]["n_s"]))


@pytest.mark.parametrize("prec", [0, 1])
def test_tree_large_haloes_c3(H, orc, prec):
    """The 512^3 catalogue at full size with the tree potential (theta = 0.04,
    haloes of |S(h)| >= 32768), in the FP64 and the mixed form: for the three
    largest tree haloes (the largest near 10^6 particles, trees far deeper
    than c1's), the potential of 1000 sampled own particles lies within theta
    of the exact direct sum over S(h) that the oracle computes for those
    particles."""
    import torch
    from paper_1110_4372_amd import synth
    note(f"tree potential on the largest 512^3 haloes prec={prec}")
    theta = 0.04
    cat = synth.make_catalog_device("c3", seed=0)
    P = H.Particles.from_catalog(cat)
    g = H.Halo(H.params_for_catalog(cat, bh_theta=theta, prec=prec)).run_all(P)
    torch.cuda.synchronize()
    h = {k: to_np(v) for k, v in g["halos"].items()}
    ns = to_np(g["unbound"]["n_s"]).astype(np.int64)
    kept = h["merged_into"] == np.arange(ns.shape[0])
    big = np.nonzero(kept & (ns >= 100000))[0]
    assert big.shape[0] >= 3
    big = big[np.argsort(-ns[big])][:3]
    assert ns[big[0]] >= 300000
    hof = to_np(g["halo_of"]).astype(np.int64)
    host = h["host"].astype(np.int64)
    phi = g["phi"]
    p = orc.params_of(cat)
    rng = np.random.default_rng(3)
    for t in big:
        # S(t): particles of t and of every halo below it in the host links
        under = np.arange(host.shape[0]) == t
        anc = host.copy()
        while np.any(anc >= 0):
            under |= anc == t
            anc = np.where(anc >= 0, host[np.maximum(anc, 0)], -1)
        src = np.nonzero((hof >= 0) & under[np.maximum(hof, 0)])[0]
        assert src.shape[0] == ns[t]
        own = np.nonzero(hof == t)[0]
        tgt = np.sort(rng.choice(own, 1000, replace=False))
        idx = torch.from_numpy(src).to(P.x.device)
        sub = orc.Particles(*[np.ascontiguousarray(to_np(a[idx]))
                              for a in (P.x, P.y, P.z, P.vx, P.vy, P.vz)])
        exact = orc.phi_points(p, sub, np.arange(src.shape[0]), np.searchsorted(src, tgt))
        got = to_np(phi[torch.from_numpy(tgt).to(P.x.device)])
        rel = np.abs(got / exact - 1.0)
        print(f"halo {t}: |S(h)| {ns[t]}, sampled relative error median {np.median(rel):.2e} "
              f"max {rel.max():.2e}", flush=True)
        assert rel.max() <= theta
