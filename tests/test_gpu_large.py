"""The 512^3 catalogue at full size (134M particles, drawn on the GPU), checked
against the oracle on sampled FOF groups.

FOF membership is local: a group whose members all lie more than ll inside a
sub-cube of the box is the same group when FOF runs on the sub-cube's
particles alone.  The oracle runs the whole path on the particles of a few
random sub-cubes (the box and the linking length of the full catalogue), and
the GPU's output for the interior groups -- labels, node table, deepest node,
halo table, halo_of and bound flags -- must match it exactly, as at the
smaller sizes; the basic and additional halo properties within 1e-5."""

import numpy as np
import pytest
import torch

from tests.gpu_util import note, to_np
from tests.test_gpu_assign import assert_halos_equal
from tests.test_gpu_props_extra import compare_extra_rows
from tests.test_gpu_refine6d import assert_nodes_equal, gpu_nodes, subset_nodes
from tests.test_gpu_unbind_props import energy_band

pytestmark = pytest.mark.gpu

CUBE = 30.0  # Mpc/h; ~17k particles of the 512^3 catalogue on average
MAX_SUB = 60000
# virial, 200 and 500 times critical, and half the virial density
SO_THRESHOLDS = [360.0 * 0.27 * 2.77536627e11, 200.0 * 2.77536627e11, 500.0 * 2.77536627e11,
                 0.5 * 360.0 * 0.27 * 2.77536627e11]


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def _subset_halos(hal, keep_fof, node_remap):
    """Rows of the haloes of the FOF groups in keep_fof, re-indexed."""
    rows = np.nonzero(np.isin(hal["fof"].astype(np.int64), keep_fof))[0]
    remap = np.full(hal["fof"].shape[0] + 1, -1, np.int64)
    remap[rows] = np.arange(rows.shape[0])
    out = {k: np.asarray(v)[rows].copy() for k, v in hal.items()}
    out["seed_node"] = node_remap[out["seed_node"].astype(np.int64)]
    for k in ("merged_into", "host"):
        v = out[k].astype(np.int64)
        out[k] = np.where(v >= 0, remap[v], -1)
    return out, remap


def subcube_parity(H, orc, cat, P, prec, ncubes=6, seed=7, cube=CUBE, extras=True):
    """Runs the whole path on the GPU at full size, then the oracle on random
    sub-cubes, and compares the interior groups exactly (properties, and with
    `extras` the additional properties, to 1e-5 relative where the oracle's
    and the GPU's bound flags of the group agree).  Returns the numbers of
    groups, nodes and haloes checked."""
    ctx = H.Halo(H.params_for_catalog(cat, prec=prec))
    fof = ctx.fof3d(P)
    nodes, deep = ctx.refine6d(P, fof)
    torch.cuda.synchronize()
    print("fof3d and refine6d done", flush=True)
    halos, hof = ctx.assign(P, nodes, deep)
    unb, bound, _ = ctx.unbind(P, halos, hof, want_phi=False)
    if extras:
        props, extra = ctx.props_extra(P, nodes, halos, hof, bound, SO_THRESHOLDS)
    else:
        props, extra = ctx.props(P, nodes, halos, hof, bound), None
    torch.cuda.synchronize()
    print("assign, unbind and props done" + (" (with the additional ones)" if extras else ""),
          flush=True)
    label_d = fof["label"].long()
    gsize_d = torch.bincount(label_d, minlength=P.n)
    gn = gpu_nodes(nodes)
    gh = {k: to_np(v) for k, v in halos.items()}
    gp = {k: to_np(v) for k, v in props.items()}
    gx = {k: to_np(v) for k, v in extra.items()} if extras else None

    N, L = cat.n, cat.box
    ll = 0.28 * L / N ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    checked_groups = checked_nodes = checked_halos = checked_props = 0
    for corner in rng.random((ncubes, 3)) * (L - cube):
        lo, hi = corner, corner + cube
        inside = torch.ones(N, dtype=torch.bool, device=P.x.device)
        for a, t in enumerate((P.x, P.y, P.z)):
            inside &= (t >= float(lo[a])) & (t < float(hi[a]))
        idx_d = torch.nonzero(inside).flatten()
        idx = to_np(idx_d).astype(np.int64)
        n_sub = idx.shape[0]
        print(f"cube at {np.round(lo, 1)}: {n_sub} particles", flush=True)
        if n_sub > MAX_SUB:
            continue  # part of a very large halo: the serial oracle would take minutes
        pos = np.stack([to_np(t[idx_d]) for t in (P.x, P.y, P.z)], 1)
        vel = np.stack([to_np(t[idx_d]) for t in (P.vx, P.vy, P.vz)], 1)
        glab = to_np(label_d[idx_d]).astype(np.int64)
        gdeep = to_np(deep[idx_d]).astype(np.int64)
        ghof = to_np(hof[idx_d]).astype(np.int64)
        gbound = to_np(bound[idx_d])
        # the oracle derives ll = b L / n^(1/3) from the particles it is given
        p = orc.make_params(L, cat.particle_mass, cat.softening,
                            b=0.28 * (n_sub / N) ** (1.0 / 3.0))
        Po = orc.Particles(*(np.ascontiguousarray(pos[:, a]) for a in range(3)),
                           *(np.ascontiguousarray(vel[:, a]) for a in range(3)))
        o = orc.run_all(p, Po)
        olab = o["label"].astype(np.int64)
        sizes = np.bincount(olab, minlength=n_sub)
        p64 = pos.astype(np.float64)
        far = np.all((p64 >= lo + ll) & (p64 < hi - ll), axis=1)
        groups = np.nonzero(sizes >= 10)[0]
        interior = groups[np.array([far[olab == g].all() for g in groups], bool)] \
            if groups.shape[0] else groups
        if interior.shape[0] == 0:
            continue
        mem = np.isin(olab, interior)
        # FOF: same members, label = smallest input index
        np.testing.assert_array_equal(glab[mem], idx[olab[mem]])
        keep = idx[interior]
        np.testing.assert_array_equal(to_np(gsize_d[torch.from_numpy(keep).to(P.x.device)]),
                                      sizes[interior])
        # hierarchy of the interior groups
        gsub, gremap = subset_nodes(gn, keep)
        osub, oremap = subset_nodes(o["nodes"], interior)
        for f in ("canon", "fof"):
            osub[f] = idx[osub[f].astype(np.int64)]
        assert_nodes_equal(gsub, osub)
        np.testing.assert_array_equal(gremap[gdeep[mem]],
                                      oremap[o["deepest"].astype(np.int64)[mem]])
        # haloes and memberships
        ghs, ghre = _subset_halos(gh, keep, gremap)
        oh = {k: np.asarray(v) for k, v in o["halos"].items()}
        ohs, ohre = _subset_halos(oh, interior, oremap)
        ohs["fof"] = idx[ohs["fof"].astype(np.int64)]
        assert_halos_equal(ghs, ohs)
        gm = ghof[mem]
        om = o["halo_of"].astype(np.int64)[mem]
        np.testing.assert_array_equal(np.where(gm >= 0, ghre[gm], -1),
                                      np.where(om >= 0, ohre[om], -1))
        # bound flags wherever the energy lies outside the FP64 error band
        decided = energy_band(o, Po, 1e-9) & mem
        np.testing.assert_array_equal(gbound[decided], o["bound"][decided])
        # properties of the haloes whose group has the same flags on both sides
        agree = [g for g in interior if np.array_equal(gbound[olab == g], o["bound"][olab == g])]
        grows = np.nonzero(np.isin(gh["fof"].astype(np.int64), idx[agree]))[0]
        orows = np.nonzero(np.isin(oh["fof"].astype(np.int64), agree))[0]
        assert grows.shape[0] == orows.shape[0]
        for k in ("px", "py", "pz", "vcx", "vcy", "vcz", "vbx", "vby", "vbz", "mvir", "rvir",
                  "vmax", "voff"):
            np.testing.assert_allclose(gp[k][grows], np.asarray(o["props"][k])[orows],
                                       rtol=1e-5, atol=1e-9, err_msg=k)
        np.testing.assert_array_equal(gp["n_bound"][grows],
                                      np.asarray(o["props"]["n_bound"])[orows])
        if extras:
            oex = orc.props_extra(p, Po, o["halos"], o["halo_of"], o["bound"], o["props"],
                                  SO_THRESHOLDS)
            pick = {k: (v[:, grows] if k in ("m_so", "r_so") else v[grows]) for k, v in gx.items()}
            opick = {k: (v[:, orows] if k in ("m_so", "r_so") else v[orows])
                     for k, v in oex.items() if k != "k"}
            compare_extra_rows(pick, opick, np.asarray(o["props"]["mvir"])[orows],
                               np.asarray(o["props"]["rvir"])[orows])
        checked_groups += interior.shape[0]
        checked_nodes += osub["parent"].shape[0]
        checked_halos += ohs["seed_node"].shape[0]
        checked_props += grows.shape[0]
    print(f"checked {checked_groups} groups, {checked_nodes} nodes, {checked_halos} halos, "
          f"{checked_props} halo property rows", flush=True)
    return checked_groups, checked_nodes, checked_halos, checked_props


def test_c3_full_size_subcubes(H, orc):
    from paper_1110_4372_amd import synth
    note("c3 full size, oracle on sub-cubes")
    cat = synth.make_catalog_device("c3", seed=0)
    P = H.Particles.from_catalog(cat)
    g, _, h, pr = subcube_parity(H, orc, cat, P, H.PREC_FP64)
    assert g >= 20 and h >= 20 and pr >= 20


def test_c4_full_size_subcubes(H, orc):
    """256^3 plus the 5e6-particle cluster at full size, mixed precision, against
    the oracle on sub-cubes of 20 Mpc/h (the catalogue is twice as dense as the
    512^3 one; cubes cutting the cluster exceed the oracle's size limit)."""
    from paper_1110_4372_amd import synth
    note("c4 full size (mixed), oracle on sub-cubes")
    cat = synth.make_catalog("c4", seed=0)
    P = H.Particles.from_catalog(cat)
    g, _, h, pr = subcube_parity(H, orc, cat, P, H.PREC_MIXED, ncubes=6, seed=5, cube=20.0)
    assert g >= 20 and h >= 20 and pr >= 20


def test_c5_full_size_subcubes(H, orc):
    """The 1024^3 catalogue (1.07e9 particles) at full size on one GPU, mixed
    precision, against the oracle on sub-cubes."""
    from paper_1110_4372_amd import synth
    note("c5 full size (mixed), oracle on sub-cubes")
    cat = synth.make_catalog_device("c5", seed=0)
    P = H.Particles.from_catalog(cat)
    # the additional properties' pair sum over V(h) would add minutes at this size
    g, _, h, pr = subcube_parity(H, orc, cat, P, H.PREC_MIXED, ncubes=8, seed=11, extras=False)
    assert g >= 20 and h >= 20 and pr >= 20


def test_c3_plain_equals_batched(H):
    """The 512^3 catalogue at full size in the plain form (one launch sequence
    per node and per halo) and the batched form (every node of a level and
    every halo per launch, persistent grids, work queues): every output of the
    whole path -- labels, node table, deepest node, halo table, halo_of, bound
    flags, phi and the properties -- is the same bit for bit (the sums are
    exact fixed-point, so the schedule cannot change them)."""
    from paper_1110_4372_amd import synth
    note("c3 full size, plain == batched")
    cat = synth.make_catalog_device("c3", seed=0)
    P = H.Particles.from_catalog(cat)
    out = {}
    for mode in (H.BATCHED, H.PLAIN):
        r = H.Halo(H.params_for_catalog(cat, mode=mode)).run_all(P)
        torch.cuda.synchronize()
        out[mode] = {"label": to_np(r["fof"]["label"]), "deepest": to_np(r["deepest"]),
                     "halo_of": to_np(r["halo_of"]), "bound": to_np(r["bound"]),
                     "phi": to_np(r["phi"]),
                     **{"node_" + k: to_np(v) for k, v in r["nodes"].items()},
                     **{"halo_" + k: to_np(v) for k, v in r["halos"].items()},
                     **{"prop_" + k: to_np(v) for k, v in r["props"].items()}}
        del r
    a, b = out[H.BATCHED], out[H.PLAIN]
    assert a.keys() == b.keys()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    print(f"{a['node_count'].shape[0]} nodes, {a['halo_seed_node'].shape[0]} halo rows identical")


def test_c4_mixed_matches_fp64(H):
    """256^3 plus a 5e6-particle cluster at full size: the mixed-precision form
    (FP32 potential tiles, FP64 recheck of energies within 1e-4 of zero) against
    the FP64 form.  Stages before unbinding do not depend on the precision and
    must match bit for bit; a bound flag may differ only where the FP64 energy
    lies within the FP64 error band of zero; phi agrees to 2e-5 and, where no
    flag differs, the properties are identical."""
    from paper_1110_4372_amd import synth
    note("c4 full size, mixed vs fp64")
    cat = synth.make_catalog("c4", seed=0)
    P = H.Particles.from_catalog(cat)
    out = {}
    for prec in (H.PREC_FP64, H.PREC_MIXED):
        ctx = H.Halo(H.params_for_catalog(cat, prec=prec))
        r = ctx.run_all(P)
        torch.cuda.synchronize()
        out[prec] = r
    a, b = out[H.PREC_FP64], out[H.PREC_MIXED]
    for k in ("label",):
        np.testing.assert_array_equal(to_np(a["fof"][k]), to_np(b["fof"][k]))
    for k in a["halos"]:
        np.testing.assert_array_equal(to_np(a["halos"][k]), to_np(b["halos"][k]))
    np.testing.assert_array_equal(to_np(a["halo_of"]), to_np(b["halo_of"]))
    hof = to_np(a["halo_of"]).astype(np.int64)
    inside = hof >= 0
    pa, pb = to_np(a["phi"]), to_np(b["phi"])
    np.testing.assert_allclose(pb[inside], pa[inside], rtol=2e-5, atol=0)
    ua = {k: to_np(v) for k, v in a["unbound"].items()}
    vb = np.stack([ua["vbx"], ua["vby"], ua["vbz"]], 1)
    v = np.stack([to_np(P.vx), to_np(P.vy), to_np(P.vz)], 1).astype(np.float64)
    kin = np.zeros(hof.shape[0])
    kin[inside] = 0.5 * ((v[inside] - vb[hof[inside]]) ** 2).sum(1)
    e = kin + pa
    ba, bb = to_np(a["bound"]), to_np(b["bound"])
    changed = np.nonzero(ba != bb)[0]
    print(f"assigned {int(inside.sum())}, changed flags {changed.shape[0]}, "
          f"max phi rel err {np.max(np.abs(pb[inside] - pa[inside]) / np.abs(pa[inside])):.2e}")
    assert np.all(np.abs(e[changed]) <= 1e-9 * (kin[changed] + np.abs(pa[changed])))
    if changed.shape[0] == 0:
        for k in a["props"]:
            np.testing.assert_array_equal(to_np(a["props"][k]), to_np(b["props"][k]))


def test_c3_single_large_group(H, orc):
    """A FOF group of the 512^3 catalogue of 131072-200000 particles, above the
    tree threshold (the nodes above it take the tree search of Section 3.2's
    nearest neighbours and 6D FOF), refined alone on the GPU at its real size; the oracle computes the
    same group's level-0 node (moments, normalised coordinates, every
    nearest-neighbour distance, ell^2) and its 6D FOF components in full, its
    O(n^2) loops split over the host's cores.  The level-0 row, the children
    and every particle's level-1 subgroup must match exactly."""
    from paper_1110_4372_amd import synth
    note("c3 single large group through the tree search")
    cat = synth.make_catalog_device("c3", seed=0)
    P = H.Particles.from_catalog(cat)
    ctx = H.Halo(H.params_for_catalog(cat))
    fof = ctx.fof3d(P)
    cnt = to_np(fof["grp_count"]).astype(np.int64)
    first = to_np(fof["grp_first"]).astype(np.int64)
    big = np.nonzero((cnt > 131072) & (cnt <= 200000))[0]
    assert big.shape[0] >= 1
    g = int(big[np.argmin(cnt[big])])
    n = int(cnt[g])
    members = fof["perm"][int(first[g]):int(first[g]) + n].clone()
    one = dict(perm=members, grp_first=torch.zeros(1, dtype=torch.int32, device=P.x.device),
               grp_count=torch.full((1,), n, dtype=torch.int32, device=P.x.device),
               n_groups=1, n_members=n)
    nodes, deep = ctx.refine6d(P, one)
    gn = gpu_nodes(nodes)
    mem = to_np(members).astype(np.int64)
    assert np.all(np.diff(mem) > 0)
    sub = [to_np(a[members.long()]) for a in (P.x, P.y, P.z, P.vx, P.vy, P.vz)]
    Ps = orc.Particles(*[np.ascontiguousarray(a) for a in sub])
    p = orc.params_of(cat)
    xi, mom = orc.node_normalise(p, Ps, np.arange(n))
    # level-0 row: moments and the linking length from every particle's
    # nearest neighbour
    row0 = [gn[f][0] for f in ("cx", "cy", "cz", "vx", "vy", "vz", "sx2", "sv2")]
    np.testing.assert_array_equal(np.array(row0), mom)
    assert gn["count"][0] == n and gn["canon"][0] == mem[0] and gn["level"][0] == 0
    D = orc.nn6d_threads(xi, threads=16)
    l2 = float(orc.ell2(D, p.f))
    assert np.float32(gn["ell2"][0]).view(np.uint32) == np.float32(l2).view(np.uint32)
    comp = orc.fof6d_threads(xi, l2, threads=16)
    size = np.bincount(comp, minlength=n)
    kids = np.nonzero(size >= p.min_members)[0]
    # children of row 0, in canonical order, and each particle's level-1 node
    rows = np.nonzero(gn["parent"] == 0)[0]
    assert np.array_equal(gn["canon"][rows].astype(np.int64), mem[kids])
    assert np.array_equal(gn["count"][rows].astype(np.int64), size[kids])
    cur = to_np(deep)[mem].astype(np.int64)
    assert np.all(cur >= 0)
    lev = gn["level"][cur]
    while np.any(lev > 1):
        cur = np.where(lev > 1, gn["parent"][cur], cur)
        lev = gn["level"][cur]
    lvl1 = np.where(lev == 1, cur, -1)
    want = np.where(size[comp] >= p.min_members, mem[comp], -1)
    got = np.where(lvl1 >= 0, gn["canon"][np.maximum(lvl1, 0)].astype(np.int64), -1)
    np.testing.assert_array_equal(got, want)
    print(f"group of {n} particles: ell^2 {l2:.6g}, {rows.shape[0]} children, "
          f"{int(np.sum(D <= l2))} linkable", flush=True)
