"""Brute-force pins of three oracle readings that no closed form fixes:
the seed-merge visit (Section 3.3, Eq. 2), the host/subhalo choice
(Section 3.4) and the halo-centre chain (Section 3.5.1).

Each pin recomputes the oracle's result in numpy from the definition, using
only quantities pinned elsewhere (node moments, memberships, seed means), and
then shows that the test data tell the reading from a plausible mistake: the
same numpy code with the mistake planted gives a different answer, so an
oracle carrying that mistake would fail the pin.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_pins import clustered, particles


def clump_lattice(seed=41, side=9, per=30, box=20.0):
    """side^3 tight clumps of `per` particles on a lattice finer than the
    linking length (one FOF group), each with its own bulk velocity, so each
    clump becomes a seed of that group."""
    rng = np.random.default_rng(seed)
    g = np.arange(side) * 0.2
    cx, cy, cz = np.meshgrid(g, g, g, indexing="ij")
    c = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1) + 8.0
    k = c.shape[0]
    pos = np.repeat(c, per, 0) + 0.01 * rng.standard_normal((k * per, 3))
    bulk = 300.0 * rng.standard_normal((k, 3))
    vel = (np.repeat(bulk, per, 0) + 5.0 * rng.standard_normal((k * per, 3))).astype(np.float32)
    return pos, vel, box


def _min_image(d, box):
    return d - box * np.round(d / box)


@pytest.fixture(scope="module")
def cases(orc, c1, c1_oracle):
    """(name, params, particle positions, velocities, oracle outputs)."""
    out = [("c1", orc.params_of(c1), np.stack([c1.x, c1.y, c1.z], 1).astype(np.float64),
            np.stack([c1.vx, c1.vy, c1.vz], 1), c1_oracle)]
    pos, vel, box = clump_lattice()
    p = orc.make_params(box, 1e10, 0.01)
    out.append(("lattice", p, pos, vel, orc.run_all(p, particles(orc, pos, vel))))
    pos, vel = clustered(6000, 14.0, 23, nblob=6, spread=0.35)
    p = orc.make_params(14.0, 1e10, 0.01)
    out.append(("clustered", p, pos, vel, orc.run_all(p, particles(orc, pos, vel))))
    return out


# ------------------------------------------------------------ seed merge --

def merge_visit(nodes, halos, box, q2, order="size", mu_from="visited"):
    """Eq. 2 from its definition: within a FOF group visit the seeds by
    decreasing leaf size (ties: lower id); a visited seed b merges into the
    kept seed a of least q = |dx|^2/mu_x^2 + |dv|^2/mu_v^2 (mu = sigma/sqrt(n)
    of b, the smaller seed; ties: lower id) when q < q2, else it is kept.
    `order` and `mu_from` plant the mistakes the pin must detect."""
    sn = halos["seed_node"].astype(np.int64)
    n = nodes["count"][sn].astype(np.float64)
    sx2, sv2 = nodes["sx2"][sn], nodes["sv2"][sn]
    x = np.stack([halos["xs"], halos["ys"], halos["zs"]], 1)
    v = np.stack([halos["vxs"], halos["vys"], halos["vzs"]], 1)
    fof = halos["fof"].astype(np.int64)
    merged = np.arange(sn.shape[0])
    for g in np.unique(fof):
        ids = np.nonzero(fof == g)[0]
        if order == "size":
            ids = ids[np.lexsort((ids, -n[ids]))]
        kept = []
        for b in ids:
            if kept and sx2[b] > 0 and sv2[b] > 0:
                a = np.array(kept)
                src = b if mu_from == "visited" else a
                dx2 = (_min_image(x[b] - x[a], box) ** 2).sum(1)
                dv2 = ((v[b] - v[a]) ** 2).sum(1)
                q = dx2 * (n[src] / sx2[src]) + dv2 * (n[src] / sv2[src])
                j = np.lexsort((a, q))[0]
                if q[j] < q2:
                    merged[b] = a[j]
                    continue
            kept.append(b)
    return merged


def test_merge_visit_brute_force(cases):
    """Section 3.3, Eq. 2: the oracle's merged_into equals the visit computed
    from the definition, on groups of many seeds; visiting by id, or taking mu
    from the kept seed, gives a different result on the same data."""
    differs_order = differs_mu = 0
    many = 0
    for name, p, pos, vel, o in cases:
        nodes, halos = o["nodes"], o["halos"]
        got = halos["merged_into"].astype(np.int64)
        want = merge_visit(nodes, halos, p.box, p.merge_q2)
        assert np.array_equal(got, want), f"{name}: merge visit differs"
        fof = halos["fof"]
        many += int(np.max(np.bincount(np.unique(fof, return_inverse=True)[1])) >= 3)
        differs_order += int(not np.array_equal(
            merge_visit(nodes, halos, p.box, p.merge_q2, order="id"), got))
        differs_mu += int(not np.array_equal(
            merge_visit(nodes, halos, p.box, p.merge_q2, mu_from="kept"), got))
    assert many >= 2, "no group of three or more seeds"
    assert differs_order >= 1, "the data cannot tell the size order from the id order"
    assert differs_mu >= 1, "the data cannot tell mu of the visited seed from the kept one"


# ------------------------------------------------------------- host / sub --

def halo_metrics(p, pos, vel, halos, halo_of):
    """Final sigma_v^2 and vmax^2 of each halo from its assigned particles
    (Sections 3.3-3.4): 3D velocity variance about their mean, and
    G m max_k k / max(r_k, eps) over the sorted distances from the seed."""
    ns = halos["seed_node"].shape[0]
    sv2 = np.zeros(ns)
    vm2 = np.zeros(ns)
    xs = np.stack([halos["xs"], halos["ys"], halos["zs"]], 1)
    for s in range(ns):
        mem = np.nonzero(halo_of == s)[0]
        if mem.shape[0] == 0:
            continue
        v = vel[mem].astype(np.float64)
        sv2[s] = ((v - v.mean(0)) ** 2).sum(1).mean()
        r = np.sort(np.sqrt((_min_image(pos[mem] - xs[s], p.box) ** 2).sum(1)))
        vm2[s] = p.G * p.particle_mass * np.max(np.arange(1, r.shape[0] + 1) /
                                                np.maximum(r, p.softening))
    return sv2, vm2


def host_choice(p, halos, n_assigned, sv2, vm2, metric="host", strict=True, pick="min"):
    """Section 3.4: each halo's host is the halo of its FOF group, among those
    with more assigned particles, closest by the Eq. 3 distance in that
    candidate's metric (|dx|^2 4/3 pi G rho_vir / vmax^2 + |dv|^2 / sigma_v^2;
    ties: lower id); -1 if there is none.  `metric`, `strict` and `pick`
    plant the mistakes the pin must detect."""
    kept = halos["merged_into"] == np.arange(halos["merged_into"].shape[0])
    cdyn = 4.0 / 3.0 * math.pi * p.G * p.rho_vir
    x = np.stack([halos["xs"], halos["ys"], halos["zs"]], 1)
    v = np.stack([halos["vxs"], halos["vys"], halos["vzs"]], 1)
    fof = halos["fof"]
    host = np.full(kept.shape[0], -1, np.int64)
    for s in np.nonzero(kept)[0]:
        if strict:
            cand = kept & (fof == fof[s]) & (n_assigned > n_assigned[s])
        else:
            cand = kept & (fof == fof[s]) & (n_assigned >= n_assigned[s])
            cand[s] = False
        H = np.nonzero(cand)[0]
        if H.shape[0] == 0:
            continue
        m = H if metric == "host" else np.full_like(H, s)
        d = ((_min_image(x[s] - x[H], p.box) ** 2).sum(1) * (cdyn / vm2[m]) +
             ((v[s] - v[H]) ** 2).sum(1) / np.maximum(sv2[m], 1e-300))
        j = np.lexsort((H, d))[0] if pick == "min" else np.lexsort((H, -d))[0]
        host[s] = H[j]
    return host


def test_host_sub_brute_force(cases):
    """Section 3.4: the oracle's hosts equal the brute-force choice over the
    strictly larger halos of the group in the candidate's metric, with the
    final sigma_v and vmax recomputed from the memberships.  The sub's own
    metric, the farthest candidate, or admitting equal-count halos each give a
    different result on the same data."""
    d_metric = d_pick = d_strict = 0
    for name, p, pos, vel, o in cases:
        halos, halo_of = o["halos"], o["halo_of"]
        kept = halos["merged_into"] == np.arange(halos["merged_into"].shape[0])
        n_assigned = np.bincount(halo_of[halo_of >= 0], minlength=kept.shape[0])
        assert np.array_equal(halos["n_assigned"].astype(np.int64), n_assigned)
        sv2, vm2 = halo_metrics(p, pos, vel, halos, halo_of)
        # the oracle sums velocities quantised to 2^-24 km/s (exact fixed-point
        # moments), so its sigma_v^2 differs from the plain FP64 one by ~1e-8
        np.testing.assert_allclose(halos["sv2"][kept], sv2[kept], rtol=1e-7)
        np.testing.assert_allclose(halos["vmax2"][kept], vm2[kept], rtol=1e-12)
        # the oracle's own final metrics (pinned just above) break exact ties alike
        sv2, vm2 = halos["sv2"], halos["vmax2"]
        got = halos["host"].astype(np.int64)
        want = host_choice(p, halos, n_assigned, sv2, vm2)
        assert np.array_equal(got[kept], want[kept]), f"{name}: hosts differ"
        d_metric += int(not np.array_equal(
            host_choice(p, halos, n_assigned, sv2, vm2, metric="sub")[kept], got[kept]))
        d_pick += int(not np.array_equal(
            host_choice(p, halos, n_assigned, sv2, vm2, pick="max")[kept], got[kept]))
        d_strict += int(not np.array_equal(
            host_choice(p, halos, n_assigned, sv2, vm2, strict=False)[kept], got[kept]))
    assert d_metric >= 1 and d_pick >= 1 and d_strict >= 1, (d_metric, d_pick, d_strict)


# ----------------------------------------------------------------- centre --

def seed_sets(nodes, halos):
    """Set of kept-halo ids of the leaves below each node."""
    nn = nodes["parent"].shape[0]
    sets = [set() for _ in range(nn)]
    for s, k in enumerate(halos["seed_node"]):
        h = int(halos["merged_into"][s])
        k = int(k)
        while k >= 0:
            sets[k].add(h)
            k = int(nodes["parent"][k])
    return sets


def centre_choice(nodes, halos, pick="min", tie="deeper", chain="own"):
    """Section 3.5.1: the centre is the mean position of the node, on the
    chain from the halo's seed leaf upwards while the node holds no other
    halo's seed, of least sigma_x^2 / n (ties: the deeper node).  `pick`,
    `tie` and `chain` plant the mistakes the pin must detect."""
    sets = seed_sets(nodes, halos)
    ns = halos["seed_node"].shape[0]
    out = np.zeros((ns, 3))
    for s in range(ns):
        if halos["merged_into"][s] != s:
            continue
        k = int(halos["seed_node"][s])
        best, bv = k, None
        while k >= 0 and (chain == "root" or sets[k] == {s}):
            v = nodes["sx2"][k] / float(nodes["count"][k])
            if pick == "max":
                v = -v
            if bv is None or v < bv or (tie == "shallower" and v == bv):
                best, bv = k, v
            k = int(nodes["parent"][k])
        out[s] = nodes["cx"][best], nodes["cy"][best], nodes["cz"][best]
    return out


def test_centre_chain_brute_force(cases):
    """Section 3.5.1: the oracle's halo centres equal the node chosen from the
    definition; the largest sigma_x^2/n, or a chain running past other seeds to
    the FOF group, gives a different centre on the same data."""
    d_pick = d_chain = 0
    long_chains = 0
    for name, p, pos, vel, o in cases:
        nodes, halos, pr = o["nodes"], o["halos"], o["props"]
        kept = halos["merged_into"] == np.arange(halos["merged_into"].shape[0])
        got = np.stack([pr["px"], pr["py"], pr["pz"]], 1)
        want = centre_choice(nodes, halos)
        assert np.array_equal(got[kept], want[kept]), f"{name}: centres differ"
        sets = seed_sets(nodes, halos)
        for s in np.nonzero(kept)[0]:
            k = int(halos["seed_node"][s])
            q = int(nodes["parent"][k])
            long_chains += int(q >= 0 and sets[q] == {s})
        d_pick += int(not np.array_equal(centre_choice(nodes, halos, pick="max")[kept],
                                         got[kept]))
        d_chain += int(not np.array_equal(centre_choice(nodes, halos, chain="root")[kept],
                                          got[kept]))
    assert long_chains >= 5, "too few halos whose chain has more than one node"
    assert d_pick >= 1 and d_chain >= 1, (d_pick, d_chain)
