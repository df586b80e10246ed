"""Pins of the oracle's additional halo properties (Sections 3.5.2 and 3.5.4)
against closed forms and independent routes: the NFW circular-velocity
maximum, rigid rotation, a regular tetrahedron, a brute-force pair sum by
another library, a rotated axis-aligned point set, and unit invariance of
the dimensionless spins."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.distance import pdist

from oracle import oracle as O


def test_klypin_radius_constant():
    """Eq. 5: the maximum of f(b)/b, f(b) = ln(1+b) - b/(1+b), lies at the
    printed 2.1626 (Eq. 6), to its four decimals."""
    root = minimize_scalar(lambda b: -O.nfw_f(b) / b, bounds=(0.5, 10.0), method="bounded",
                           options={"xatol": 1e-12}).x
    assert abs(root - O.KLYPIN_X) < 5e-5


@pytest.mark.parametrize("c0", [2.5, 4.0, 9.0, 17.0, 60.0, 400.0])
def test_klypin_recovers_nfw_concentration(c0):
    """For an NFW halo of concentration c0, v_max^2 is the maximum over r of
    G M(<r) / r, M(<r) = M_vir f(r/R_s) / f(c0): Eq. 7 must give c0 back."""
    G, M, R = 4.30091e-9, 3.7e12, 0.31
    Rs = R / c0
    res = minimize_scalar(lambda r: -G * M * O.nfw_f(r / Rs) / O.nfw_f(c0) / r,
                          bounds=(1e-6 * R, R), method="bounded", options={"xatol": 1e-14 * R})
    vmax = np.sqrt(-res.fun)
    c = O.klypin_concentration(vmax, M, R, G)
    assert c == pytest.approx(c0, rel=1e-6)


def test_klypin_clamps():
    G, M, R = 1.0, 1.0, 1.0
    # v_max below the circular velocity at R_vir: R_max would lie outside
    assert O.klypin_concentration(0.9, M, R, G) == O.KLYPIN_X
    assert O.klypin_concentration(1e4, M, R, G) == O.KLYPIN_CMAX
    assert O.klypin_concentration(1.0, 0.0, R, G) == 0.0


def symmetric_set(rng, n=40):
    pts = rng.standard_normal((n, 3)) * np.array([0.3, 0.2, 0.1])
    return np.concatenate([pts, -pts])


def test_sums_rigid_rotation():
    """v = v0 + w x r on a point-symmetric set: the bulk velocity is v0, the
    angular momentum per unit mass is sum (w r^2 - r (r . w)) and the
    rotational kinetic energy is w . J / 2."""
    rng = np.random.default_rng(3)
    r = symmetric_set(rng)
    w = np.array([0.4, -1.3, 2.2]) * 100.0
    v0 = np.array([150.0, -40.0, 7.0])
    v = v0 + np.cross(w, r)
    s = O.halo_sums(r[:, 0], r[:, 1], r[:, 2], v[:, 0], v[:, 1], v[:, 2],
                    np.ones(len(r)), v0, 1e-4)
    J = (w[None, :] * (r * r).sum(1)[:, None] - r * (r @ w)[:, None]).sum(0)
    np.testing.assert_allclose(s[3:6], J, rtol=1e-12)
    assert s[6] == pytest.approx(float(w @ J), rel=1e-12)
    np.testing.assert_allclose(s[0:3], 0.0, atol=1e-13)
    # rotation the other way: J flips, T stays
    v2 = v0 - np.cross(w, r)
    s2 = O.halo_sums(r[:, 0], r[:, 1], r[:, 2], v2[:, 0], v2[:, 1], v2[:, 2],
                     np.ones(len(r)), v0, 1e-4)
    np.testing.assert_allclose(s2[3:6], -J, rtol=1e-12)
    assert s2[6] == pytest.approx(s[6], rel=1e-12)


def test_pair_energy_tetrahedron_and_brute_force():
    a, eps = 0.37, 0.05
    tet = a / np.sqrt(8.0) * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    z = np.zeros(4)
    s = O.halo_sums(tet[:, 0], tet[:, 1], tet[:, 2], z, z, z, np.ones(4), np.zeros(3), eps * eps)
    assert s[7] == pytest.approx(6.0 / np.sqrt(a * a + eps * eps), rel=1e-14)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((300, 3))
    z = np.zeros(300)
    s = O.halo_sums(r[:, 0], r[:, 1], r[:, 2], z, z, z, np.ones(300), np.zeros(3), eps * eps)
    d = pdist(r)
    assert s[7] == pytest.approx(float(np.sum(1.0 / np.sqrt(d * d + eps * eps))), rel=1e-12)


def test_shape_of_rotated_axes():
    """Points at +-a e1, +-b e2, +-c e3, rotated: Eq. 11 gives the axis
    ratios b/a and c/a and the major axis along R e1; particles that are not
    the halo's own (substructure) leave it unchanged."""
    a, b, c = 2.0, 1.3, 0.4
    base = np.array([[a, 0, 0], [-a, 0, 0], [0, b, 0], [0, -b, 0], [0, 0, c], [0, 0, -c]])
    Q, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((3, 3)))
    r = base @ Q.T
    sub = np.array([[5.0, 5.0, 5.0], [4.0, -3.0, 1.0]])
    pts = np.concatenate([r, sub])
    own = np.array([1] * 6 + [0, 0])
    z = np.zeros(len(pts))
    s = O.halo_sums(pts[:, 0], pts[:, 1], pts[:, 2], z, z, z, own, np.zeros(3), 1e-4)
    assert s[14] == 6
    ba, ca, A = O.shape_from_tensor(*s[8:14], int(s[14]))
    assert ba == pytest.approx(b / a, rel=1e-12)
    assert ca == pytest.approx(c / a, rel=1e-12)
    e1 = Q[:, 0]
    assert np.linalg.norm(A) == pytest.approx(a / np.sqrt(3.0), rel=1e-12)
    assert abs(float(A @ e1)) == pytest.approx(np.linalg.norm(A), rel=1e-12)
    assert A[int(np.argmax(np.abs(A)))] > 0


def test_centre_of_mass_offset():
    rng = np.random.default_rng(11)
    d = np.array([0.013, -0.002, 0.007])
    r = symmetric_set(rng) + d
    z = np.zeros(len(r))
    s = O.halo_sums(r[:, 0], r[:, 1], r[:, 2], z, z, z, np.ones(len(r)), np.zeros(3), 1e-4)
    np.testing.assert_allclose(s[0:3] / len(r), d, rtol=1e-10)


def test_so_count_constructed():
    """Radii placed just inside (then just outside) the threshold density at a
    known index give exactly that count; a first particle outside gives 0."""
    C_thr = 2.5e-4
    K = 37
    j = np.arange(1, 80)
    r = np.cbrt(j * C_thr) * np.where(j <= K, 0.999, 1.001)
    assert O.so_count(r * r, C_thr) == K
    r[0] = np.cbrt(C_thr) * 1.01
    assert O.so_count(r * r, C_thr) == 0


def test_spins_are_dimensionless():
    """Scaling lengths by al, velocities by be and masses by mu, with G scaled
    to keep G M / R ~ v^2, leaves both spin parameters unchanged; a wrong
    power of M, R or E would not."""
    J, T, U, M, R, G = 3.1e15, 2.2e17, -5.9e17, 1.4e13, 0.35, 4.30091e-9
    lam, lamb = O.spin_parameters(J, T, U, M, R, G)
    al, be, mu = 3.7, 0.61, 19.0
    lam2, lamb2 = O.spin_parameters(J * mu * al * be, T * mu * be * be, U * mu * be * be,
                                    M * mu, R * al, G * be * be * al / mu)
    assert float(lam2) == pytest.approx(float(lam), rel=1e-12)
    assert float(lamb2) == pytest.approx(float(lamb), rel=1e-12)
    # the two forms of Eq. 10 agree: J / (sqrt(2) M V_vir R_vir), V_vir^2 = G M / R
    assert float(lamb) == pytest.approx(J / (np.sqrt(2.0) * M * np.sqrt(G * M / R) * R),
                                        rel=1e-12)


def virial_sets(orc, cat, r):
    """V(h) of each kept halo assembled in numpy from the oracle's outputs:
    the bound particles of the halo and of every halo below it on the host
    tree, by distance from the centre (ties by index), cut at k*."""
    p = orc.params_of(cat)
    halos, pr, halo_of, bound = r["halos"], r["props"], r["halo_of"], r["bound"]
    nh = halos["seed_node"].shape[0]
    pos = np.stack([cat.x, cat.y, cat.z], 1).astype(np.float64)
    host = halos["host"]
    chains = [[h] for h in range(nh)]
    for h in range(nh):
        a = host[h]
        while a >= 0:
            chains[h].append(a)
            a = host[a]
    members = [[] for _ in range(nh)]
    for i in np.nonzero((halo_of >= 0) & (bound != 0))[0]:
        for a in chains[halo_of[i]]:
            members[a].append(i)
    C_vir = 3.0 * p.particle_mass / (4.0 * np.pi * p.rho_vir)
    out = {}
    for h in range(nh):
        if halos["merged_into"][h] != h or not members[h]:
            continue
        idx = np.array(sorted(members[h]))
        c = np.array([pr["px"][h], pr["py"][h], pr["pz"][h]])
        d = pos[idx] - c
        d -= p.box * np.round(d / p.box)
        r2 = np.einsum("ij,ij->i", d, d)
        o = np.lexsort((idx, r2))
        idx, d, r2 = idx[o], d[o], r2[o]
        j = np.arange(1, len(idx) + 1)
        ok = r2 ** 3 <= (j * C_vir) ** 2
        k = len(idx) if ok.all() else int(np.argmin(ok))
        out[h] = (idx[:k], d[:k])
    return out


def test_props_extra_sets_match_numpy(orc):
    """End to end on a small catalogue: orc_props_extra's sums equal plain
    numpy sums over V(h) assembled independently, and the virial threshold
    among the extra thresholds reproduces M_vir."""
    from paper_1110_4372_amd import synth
    cat = synth.make_catalog("c1", seed=2)
    p = orc.params_of(cat)
    P = orc.Particles.of(cat)
    r = orc.run_all(p, P)
    so = [p.rho_vir, 200.0 * 2.77536627e11, 0.5 * p.rho_vir]
    s = orc.props_extra_sums(p, P, r["halos"], r["halo_of"], r["bound"], r["props"], so)
    sets = virial_sets(orc, cat, r)
    assert len(sets) >= 5
    vel = np.stack([cat.vx, cat.vy, cat.vz], 1).astype(np.float64)
    for h, (idx, d) in sets.items():
        k = len(idx)
        assert s["k"][h] == k
        assert s["k_so"][0, h] == k
        assert r["props"]["mvir"][h] == k * p.particle_mass
        assert s["k_so"][1, h] <= k <= s["k_so"][2, h]  # 200 rho_c is above rho_vir
        if k == 0:
            continue
        vb = np.array([r["props"]["vbx"][h], r["props"]["vby"][h], r["props"]["vbz"][h]])
        u = vel[idx] - vb
        np.testing.assert_allclose([s["sx"][h], s["sy"][h], s["sz"][h]], d.sum(0),
                                   rtol=1e-9, atol=1e-9 * k)
        np.testing.assert_allclose([s["jx"][h], s["jy"][h], s["jz"][h]],
                                   np.cross(d, u).sum(0), rtol=1e-9, atol=1e-8 * k)
        assert s["t2"][h] == pytest.approx(float((u * u).sum()), rel=1e-10)
        if k > 1:
            dd = pdist(d)
            eps2 = p.softening ** 2
            assert s["uinv"][h] == pytest.approx(float(np.sum(1.0 / np.sqrt(dd * dd + eps2))),
                                                 rel=1e-10)
        own = r["halo_of"][idx] == h
        assert s["n_own"][h] == int(own.sum())
        do = d[own]
        np.testing.assert_allclose(
            [s["mxx"][h], s["myy"][h], s["mzz"][h], s["mxy"][h], s["mxz"][h], s["myz"][h]],
            [do[:, 0] @ do[:, 0], do[:, 1] @ do[:, 1], do[:, 2] @ do[:, 2],
             do[:, 0] @ do[:, 1], do[:, 0] @ do[:, 2], do[:, 1] @ do[:, 2]],
            rtol=1e-9, atol=1e-12)
    ex = orc.props_extra(p, P, r["halos"], r["halo_of"], r["bound"], r["props"], so)
    kept = [h for h in sets if len(sets[h][0]) > 1]
    assert all(ex["spin"][h] > 0 and ex["spin_bullock"][h] > 0 for h in kept)
    assert all(ex["c_klypin"][h] >= O.KLYPIN_X for h in kept)
    assert all(0.0 < ex["t_u"][h] for h in kept)
    np.testing.assert_array_equal(ex["m_so"][0], r["props"]["mvir"])
