"""Pins of the oracle's major-merger unbinding (Section 3.5.3, MP of Table 2):
the off switch, the monotonicity the reading implies, and a brute-force
evaluation of the definition on constructed mergers of two NFW clumps."""
import numpy as np
import pytest

from paper_1110_4372_amd import synth
from tests.test_oracle_pins import particles

M_PART = 2e9
EPS = 0.005
BOX = 20.0


def merger(seed, n1=1200, n2=700, sep=0.15, dv=600.0):
    """Two overlapping NFW clumps (the second offset by sep in each axis and by
    dv km/s in x) in a uniform background: the smaller becomes a subhalo of
    the larger with |S(sub)| / |S(host)| ~ 0.37."""
    p1, v1, _ = synth.nfw_halo(n1, 6.0, 2e12 * n1 / 1000, seed=seed, box=BOX)
    p2, v2, _ = synth.nfw_halo(n2, 6.0, 2e12 * n2 / 1000, seed=seed + 1, box=BOX,
                               center=np.full(3, 0.5 * BOX) + sep, bulk=(dv, 0.0, 0.0))
    rng = np.random.default_rng(seed)
    bg = rng.random((600, 3)) * BOX
    vbg = (100.0 * rng.standard_normal((600, 3))).astype(np.float32)
    return np.concatenate([p1, p2, bg]), np.concatenate([v1, v2, vbg]).astype(np.float32)


def run(orc, pos, vel, mp):
    p = orc.make_params(BOX, M_PART, EPS, major_merger=mp)
    return p, orc.run_all(p, particles(orc, pos, vel))


@pytest.mark.parametrize("seed", [1, 5])
def test_mp_off_leaves_everything_unchanged(orc, seed):
    """MP = 0 is the plain single-halo unbinding; MP > 1 can select no merger
    (S(host) contains S(h)), so it must give the same bits."""
    pos, vel = merger(seed)
    _, a = run(orc, pos, vel, 0.0)
    _, b = run(orc, pos, vel, 1.5)
    np.testing.assert_array_equal(a["bound"], b["bound"])
    np.testing.assert_array_equal(a["phi"], b["phi"])
    for k in a["unbound"]:
        np.testing.assert_array_equal(a["unbound"][k], b["unbound"][k])


@pytest.mark.parametrize("seed", [1, 3, 5, 7])
def test_mp_only_deepens_and_binds(orc, seed):
    """The merging system S(t) contains S(h): every potential is at least as
    deep and, with the kinetic term unchanged, no particle turns unbound; the
    subhalo keeps more of its particles; the host's own particles and every
    non-merging halo are untouched."""
    pos, vel = merger(seed)
    _, a = run(orc, pos, vel, 0.0)
    _, b = run(orc, pos, vel, 0.3)
    assert np.all(b["phi"] <= a["phi"] * (1 - 1e-12) + 1e-300)
    assert np.all(b["bound"] >= a["bound"])
    h = a["halos"]
    kept = np.nonzero(h["merged_into"] == np.arange(h["merged_into"].shape[0]))[0]
    ns = a["unbound"]["n_s"]
    major = [s for s in kept if h["host"][s] >= 0 and ns[s] >= 0.3 * ns[h["host"][s]]]
    assert len(major) == 1
    s = major[0]
    assert b["unbound"]["n_bound_own"][s] > a["unbound"]["n_bound_own"][s]
    untouched = ~np.isin(a["halo_of"], major)
    np.testing.assert_array_equal(a["phi"][untouched], b["phi"][untouched])
    np.testing.assert_array_equal(a["bound"][untouched], b["bound"][untouched])


@pytest.mark.parametrize("seed,mp", [(3, 0.3), (7, 0.3), (7, 0.36)])
def test_mp_brute_force(orc, seed, mp):
    """The definition evaluated directly in numpy from the oracle's halo table
    and membership: the target by following major-merger host links, phi over
    S(target) by a dense distance matrix, the kinetic term about the
    plain mean velocity of S(h) (the oracle's fixed-point mean differs by
    < 2^-24 km/s, so flags are compared outside a 1e-6 relative band)."""
    pos, vel = merger(seed)
    p, o = run(orc, pos, vel, mp)
    h, hof = o["halos"], o["halo_of"]
    nh = h["host"].shape[0]
    kept = h["merged_into"] == np.arange(nh)
    members = {s: [] for s in range(nh)}
    for i in np.nonzero(hof >= 0)[0]:
        a = hof[i]
        while a >= 0:
            members[a].append(i)
            a = h["host"][a]
    size = {s: len(v) for s, v in members.items()}
    G, m = p.G, p.particle_mass
    checked = 0
    for s in np.nonzero(kept)[0]:
        t = s
        while h["host"][t] >= 0 and size[t] >= mp * size[h["host"][t]]:
            t = h["host"][t]
        own = np.nonzero(hof == s)[0]
        src = np.array(sorted(members[t]))
        d = pos[own][:, None, :] - pos[src][None, :, :]
        d -= BOX * np.round(d / BOX)
        r2 = np.einsum("ijk,ijk->ij", d, d)
        inv = 1.0 / np.sqrt(r2 + EPS * EPS)
        inv[own[:, None] == src[None, :]] = 0.0
        phi = -G * m * inv.sum(1)
        np.testing.assert_allclose(o["phi"][own], phi, rtol=1e-10, atol=0)
        vb = vel[np.array(sorted(members[s]))].astype(np.float64).mean(0)
        k = 0.5 * ((vel[own].astype(np.float64) - vb) ** 2).sum(1)
        e = k + phi
        decided = np.abs(e) > 1e-6 * (k + np.abs(phi))
        np.testing.assert_array_equal(o["bound"][own][decided], (e < 0)[decided])
        checked += int(t != s)
    assert checked >= 1
