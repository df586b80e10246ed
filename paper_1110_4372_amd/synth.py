"""Seeded synthetic particle catalogues for the halo-finding path.

This module is the only code shared by the GPU path's tests/benchmark and the
CPU oracle's tests: it draws inputs and holds none of the halo finder's
arithmetic.  The paper evaluates on N-body snapshots (Bolshoi, LasDamas,
Consuelo; Section 4, Table 1) that are not available here, so these seeded
catalogues stand in for them: NFW host haloes (the profile the paper uses for
its scale-radius discussion, Section 3.5.4) with NFW subhaloes, plus a uniform
background, in a periodic box.

Units: positions in comoving Mpc/h, velocities in km/s, masses in Msun/h.
Every configuration uses one numpy PCG64 stream seeded with ``seed``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Physical constants of the synthetic universe (inputs, not method arithmetic).
G_NEWTON = 4.30091e-9          # (Mpc/h) (km/s)^2 / (Msun/h)
RHO_CRIT = 2.77536627e11       # h^2 Msun / Mpc^3, i.e. (Msun/h) / (Mpc/h)^3
OMEGA_M = 0.27                 # Bolshoi cosmology (Table 1)
RHO_M = OMEGA_M * RHO_CRIT
DELTA_VIR = 360.0              # virial overdensity vs background at z=0 (Section 3.3)
RHO_VIR = DELTA_VIR * RHO_M


@dataclasses.dataclass(frozen=True)
class CatalogSpec:
    name: str
    n_side: int                 # N = n_side**3
    box: float                  # Mpc/h
    pos_f64: bool               # store positions as float64 (else float32)
    kind: str                   # "dirichlet8" | "powerlaw"
    bg_frac: float = 0.4        # fraction of particles in the uniform background
    n_min: float = 20.0         # power-law host size range (particles)
    n_max: float = 2.0e5
    slope: float = 1.9          # dN/dn ~ n^-slope
    sub_min_host: int = 200     # hosts with at least this many particles get a subhalo
    sub_frac: float = 0.1       # subhalo size as a fraction of its host
    cluster_n: int = 0          # optional single massive cluster (precision workload)
    cluster_core_frac: float = 0.05
    cluster_core_kick: float = 350.0
    cluster_n_subs: int = 20

    @property
    def n(self) -> int:
        return self.n_side ** 3


SPECS = {
    # 32^3 in a 25 Mpc/h box: 8 NFW hosts of 1000-8000 particles with 0-3
    # subhaloes each, ~30% uniform background, float64 positions.
    "c1": CatalogSpec("c1", 32, 25.0, True, "dirichlet8", bg_frac=0.3),
    # 128^3 in 100 Mpc/h: power-law host sizes on [20, 2e5], 40% background.
    "c2": CatalogSpec("c2", 128, 100.0, False, "powerlaw", 0.4, 20.0, 2.0e5),
    # 512^3 in 500 Mpc/h: power-law hosts on [10, 1e6].
    "c3": CatalogSpec("c3", 512, 500.0, False, "powerlaw", 0.4, 10.0, 1.0e6),
    # 256^3 in 200 Mpc/h plus one 5e6-particle cluster with a kicked core.
    "c4": CatalogSpec("c4", 256, 200.0, False, "powerlaw", 0.4, 20.0, 2.0e5,
                      cluster_n=5_000_000),
    # 1024^3 in 1 Gpc/h: power-law hosts on [20, 1e7].
    "c5": CatalogSpec("c5", 1024, 1000.0, False, "powerlaw", 0.4, 20.0, 1.0e7),
}


def particle_mass(n: int, box: float) -> float:
    """Mass per particle so that the box holds the mean matter density."""
    return RHO_M * (box / n ** (1.0 / 3.0)) ** 3


def default_softening(n: int, box: float) -> float:
    """Plummer softening, 2% of the mean interparticle spacing."""
    return 0.02 * box / n ** (1.0 / 3.0)


def virial_radius(mass: np.ndarray) -> np.ndarray:
    return np.cbrt(3.0 * mass / (4.0 * math.pi * RHO_VIR))


def _nfw_f(x):
    return np.log1p(x) - x / (1.0 + x)


def _nfw_radii(rng, conc: np.ndarray, rvir: np.ndarray, lo: float = 0.0,
               hi: float = 1.0) -> np.ndarray:
    """Radii drawn from a truncated NFW mass profile between lo*R and hi*R.

    Inverse CDF of f(r/r_s)/f(c), solved with the Lambert W function:
    f(x) = p  <=>  x = -1/W0(-exp(-1-p)) - 1.
    """
    from scipy.special import lambertw

    fc_lo = _nfw_f(conc * lo)
    fc_hi = _nfw_f(conc * hi)
    p = fc_lo + rng.random(conc.shape[0]) * (fc_hi - fc_lo)
    w = lambertw(-np.exp(-1.0 - p), 0).real
    x = -1.0 / w - 1.0
    return x * (rvir / conc)


def _iso_dirs(rng, n: int) -> np.ndarray:
    mu = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * math.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)


@dataclasses.dataclass
class Catalog:
    spec_name: str
    box: float
    n: int
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    particle_mass: float
    softening: float
    truth: np.ndarray           # generating halo per particle (-1 = background)
    halos: dict                 # generating halo table (centres, sizes, ...)

    @property
    def pos_f64(self) -> bool:
        return self.x.dtype == np.float64


def _draw_host_sizes(rng, spec: CatalogSpec) -> np.ndarray:
    n_total = spec.n
    if spec.kind == "dirichlet8":
        budget = int(round((1.0 - spec.bg_frac) * n_total)) - 8 * 1000
        while True:
            w = rng.dirichlet(np.ones(8))
            sizes = 1000 + np.floor(budget * w).astype(np.int64)
            if sizes.max() <= 8000:
                return sizes
    target = int((1.0 - spec.bg_frac) * n_total) - spec.cluster_n
    a = 1.0 - spec.slope
    lo, hi = spec.n_min ** a, spec.n_max ** a
    chunks, total = [], 0
    while total < target:
        u = rng.random(65536)
        s = np.floor((lo + u * (hi - lo)) ** (1.0 / a)).astype(np.int64)
        chunks.append(s)
        total += int(s.sum())
    sizes = np.concatenate(chunks)
    cum = np.cumsum(sizes)
    k = int(np.searchsorted(cum, target))
    sizes = sizes[: k + 1].copy()
    sizes[-1] -= int(cum[k] - target)
    if sizes[-1] < spec.n_min:
        sizes = sizes[:-1]
    return sizes


def _sample_halo_particles(rng, sizes, centres, bulk, conc, rvir, sigma):
    """Particles of a batch of NFW haloes: positions and velocities."""
    hid = np.repeat(np.arange(sizes.shape[0]), sizes)
    r = _nfw_radii(rng, conc[hid], rvir[hid])
    pos = centres[hid] + r[:, None] * _iso_dirs(rng, hid.shape[0])
    vel = bulk[hid] + sigma[hid, None] * rng.standard_normal((hid.shape[0], 3))
    return pos, vel, hid


def make_catalog(name: str = "c1", seed: int = 0, spec: CatalogSpec | None = None
                 ) -> Catalog:
    """Draw the seeded synthetic catalogue ``name`` (see SPECS)."""
    spec = spec or SPECS[name]
    rng = np.random.default_rng(seed)
    n_total, box = spec.n, spec.box
    mp = particle_mass(n_total, box)

    sizes = _draw_host_sizes(rng, spec)
    n_host = sizes.shape[0]
    # Subhalo table: per host a list of subhalo sizes carved out of its budget.
    if spec.kind == "dirichlet8":
        n_sub_per = rng.integers(0, 4, size=n_host)
        sub_host = np.repeat(np.arange(n_host), n_sub_per)
        frac = 0.02 + 0.08 * rng.random(sub_host.shape[0])
        sub_sizes = np.floor(frac * sizes[sub_host]).astype(np.int64)
    else:
        sub_host = np.nonzero(sizes >= spec.sub_min_host)[0]
        sub_sizes = np.floor(spec.sub_frac * sizes[sub_host]).astype(np.int64)

    host_mass = sizes * mp
    host_rvir = virial_radius(host_mass)
    host_c = 5.0 + 5.0 * rng.random(n_host)
    host_sig = np.sqrt(G_NEWTON * host_mass / (2.0 * host_rvir))
    host_ctr = rng.random((n_host, 3)) * box
    host_bulk = 300.0 * rng.standard_normal((n_host, 3))

    # Host particle budgets after carving out their subhaloes.
    own = sizes.copy()
    np.subtract.at(own, sub_host, sub_sizes)

    sub_mass = sub_sizes * mp
    sub_rvir = virial_radius(np.maximum(sub_mass, mp))
    sub_c = 5.0 + 5.0 * rng.random(sub_host.shape[0])
    sub_sig = np.sqrt(G_NEWTON * np.maximum(sub_mass, mp) / (2.0 * sub_rvir))
    sub_r = _nfw_radii(rng, host_c[sub_host], host_rvir[sub_host], 0.1, 1.0)
    sub_ctr = host_ctr[sub_host] + sub_r[:, None] * _iso_dirs(rng, sub_host.shape[0])
    sub_bulk = host_bulk[sub_host] + host_sig[sub_host, None] * rng.standard_normal(
        (sub_host.shape[0], 3))

    cl = None
    if spec.cluster_n:
        cl_n = spec.cluster_n
        cl_mass = cl_n * mp
        cl_rvir = float(virial_radius(np.array([cl_mass]))[0])
        cl_sig = math.sqrt(G_NEWTON * cl_mass / (2.0 * cl_rvir))
        cl = dict(n=cl_n, rvir=cl_rvir, sig=cl_sig, c=5.0,
                  ctr=rng.random(3) * box, bulk=np.zeros(3),
                  kick_dir=_iso_dirs(rng, 1)[0])

    all_sizes = np.concatenate([own, sub_sizes])
    all_ctr = np.concatenate([host_ctr, sub_ctr])
    all_bulk = np.concatenate([host_bulk, sub_bulk])
    all_c = np.concatenate([host_c, sub_c])
    all_rvir = np.concatenate([host_rvir, sub_rvir])
    all_sig = np.concatenate([host_sig, sub_sig])
    pos, vel, hid = _sample_halo_particles(rng, all_sizes, all_ctr, all_bulk, all_c,
                                           all_rvir, all_sig)
    parts_pos, parts_vel, parts_tid = [pos], [vel], [hid]
    next_id = all_sizes.shape[0]

    if cl is not None:
        n_sub = spec.cluster_n_subs
        core_r = None
        # Cluster body.
        r = _nfw_radii(rng, np.full(cl["n"], cl["c"]), np.full(cl["n"], cl["rvir"]))
        cpos = cl["ctr"] + r[:, None] * _iso_dirs(rng, cl["n"])
        cvel = cl["bulk"] + cl["sig"] * rng.standard_normal((cl["n"], 3))
        order = np.argsort(r, kind="stable")
        n_core = int(spec.cluster_core_frac * cl["n"])
        core_r = r[order[n_core - 1]]
        kick = spec.cluster_core_kick * cl["kick_dir"]
        cvel[order[:n_core]] += kick
        parts_pos.append(cpos)
        parts_vel.append(cvel)
        parts_tid.append(np.full(cl["n"], next_id))
        next_id += 1
        # Subhaloes inside the kicked core, moving with it.
        ssz = rng.integers(500, 5001, size=n_sub)
        smass = ssz * mp
        srv = virial_radius(smass)
        ssig = np.sqrt(G_NEWTON * smass / (2.0 * srv))
        sctr = cl["ctr"] + (core_r * rng.random(n_sub) ** (1.0 / 3.0))[:, None] * \
            _iso_dirs(rng, n_sub)
        sbulk = cl["bulk"] + kick + cl["sig"] * 0.3 * rng.standard_normal((n_sub, 3))
        spos, svel, shid = _sample_halo_particles(
            rng, ssz, sctr, sbulk, 5.0 + 5.0 * rng.random(n_sub), srv, ssig)
        parts_pos.append(spos)
        parts_vel.append(svel)
        parts_tid.append(shid + next_id)
        next_id += n_sub

    n_halo_parts = sum(p.shape[0] for p in parts_pos)
    n_bg = n_total - n_halo_parts
    if n_bg < 0:
        raise ValueError("halo particles exceed the particle budget")
    parts_pos.append(rng.random((n_bg, 3)) * box)
    parts_vel.append(100.0 * rng.standard_normal((n_bg, 3)))
    parts_tid.append(np.full(n_bg, -1))

    pos = np.concatenate(parts_pos)
    vel = np.concatenate(parts_vel)
    tid = np.concatenate(parts_tid)
    perm = rng.permutation(n_total)
    pos, vel, tid = pos[perm], vel[perm], tid[perm]
    pos = np.mod(pos, box)

    pdt = np.float64 if spec.pos_f64 else np.float32
    cols = []
    for a in range(3):
        c = np.ascontiguousarray(pos[:, a]).astype(pdt)
        # Rounding can push a coordinate just below L onto L: wrap it to 0.
        c[c >= pdt(box)] = pdt(0.0)
        cols.append(c)
    vcols = [np.ascontiguousarray(vel[:, a]).astype(np.float32) for a in range(3)]
    halos = dict(host_sizes=sizes, host_centres=host_ctr, host_bulk=host_bulk,
                 host_rvir=host_rvir, host_c=host_c, sub_host=sub_host,
                 sub_sizes=sub_sizes, cluster=cl)
    return Catalog(spec.name, box, n_total, cols[0], cols[1], cols[2],
                   vcols[0], vcols[1], vcols[2], mp, default_softening(n_total, box),
                   tid.astype(np.int64), halos)


def nfw_halo(n: int, conc: float, mass: float, seed: int = 0,
             box: float = 100.0, bulk=(0.0, 0.0, 0.0), sigma: float | None = None,
             center=None):
    """One isolated NFW halo of ``n`` particles (for analytic pins).

    Returns (pos float64 (n,3), vel float32 (n,3), rvir).
    """
    rng = np.random.default_rng(seed)
    rvir = float(virial_radius(np.array([mass]))[0])
    r = _nfw_radii(rng, np.full(n, conc), np.full(n, rvir))
    ctr = np.full(3, 0.5 * box) if center is None else np.asarray(center, float)
    pos = ctr + r[:, None] * _iso_dirs(rng, n)
    if sigma is None:
        sigma = math.sqrt(G_NEWTON * mass / (2.0 * rvir))
    vel = np.asarray(bulk, float) + sigma * rng.standard_normal((n, 3))
    return np.mod(pos, box), vel.astype(np.float32), rvir


@dataclasses.dataclass
class DeviceCatalog:
    """A catalogue whose particle arrays live on the GPU (torch tensors)."""
    spec_name: str
    box: float
    n: int
    x: "object"
    y: "object"
    z: "object"
    vx: "object"
    vy: "object"
    vz: "object"
    particle_mass: float
    softening: float
    halos: dict


def make_catalog_device(name: str, seed: int = 0, device: str = "cuda",
                        chunk: int = 1 << 25) -> DeviceCatalog:
    """The power-law catalogues (c2, c3, c5) drawn with the same recipe as
    ``make_catalog``, with the particles sampled on the GPU in chunks of haloes.

    The halo and subhalo tables come from numpy's generator seeded by ``seed``
    exactly as in ``make_catalog``; particle positions, velocities, the
    background and the final shuffle come from torch's generator on ``device``
    seeded by ``seed``, so the realisation differs from ``make_catalog``'s while
    every distribution is the same.  NFW radii solve f(x) = p by bisection in
    FP64 instead of through the Lambert W function.
    """
    import torch

    spec = SPECS[name]
    if spec.kind != "powerlaw" or spec.cluster_n:
        raise NotImplementedError("device generator covers the power-law catalogues")
    rng = np.random.default_rng(seed)
    n_total, box = spec.n, spec.box
    mp = particle_mass(n_total, box)

    sizes = _draw_host_sizes(rng, spec)
    n_host = sizes.shape[0]
    sub_host = np.nonzero(sizes >= spec.sub_min_host)[0]
    sub_sizes = np.floor(spec.sub_frac * sizes[sub_host]).astype(np.int64)
    host_mass = sizes * mp
    host_rvir = virial_radius(host_mass)
    host_c = 5.0 + 5.0 * rng.random(n_host)
    host_sig = np.sqrt(G_NEWTON * host_mass / (2.0 * host_rvir))
    host_ctr = rng.random((n_host, 3)) * box
    host_bulk = 300.0 * rng.standard_normal((n_host, 3))
    own = sizes.copy()
    np.subtract.at(own, sub_host, sub_sizes)
    sub_mass = sub_sizes * mp
    sub_rvir = virial_radius(np.maximum(sub_mass, mp))
    sub_c = 5.0 + 5.0 * rng.random(sub_host.shape[0])
    sub_sig = np.sqrt(G_NEWTON * np.maximum(sub_mass, mp) / (2.0 * sub_rvir))
    sub_r = _nfw_radii(rng, host_c[sub_host], host_rvir[sub_host], 0.1, 1.0)
    sub_ctr = host_ctr[sub_host] + sub_r[:, None] * _iso_dirs(rng, sub_host.shape[0])
    sub_bulk = host_bulk[sub_host] + host_sig[sub_host, None] * rng.standard_normal(
        (sub_host.shape[0], 3))

    all_sizes = np.concatenate([own, sub_sizes])
    tables = [np.concatenate([host_ctr, sub_ctr]), np.concatenate([host_bulk, sub_bulk]),
              np.concatenate([host_c, sub_c]), np.concatenate([host_rvir, sub_rvir]),
              np.concatenate([host_sig, sub_sig])]
    dev = torch.device(device)
    ctr_t, bulk_t, c_t, rv_t, sig_t = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                                       for a in tables)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    f64 = torch.float64
    P = torch.empty((3, n_total), dtype=torch.float32, device=dev)
    V = torch.empty((3, n_total), dtype=torch.float32, device=dev)

    def uni(k):
        return torch.rand(k, generator=gen, device=dev, dtype=f64)

    def nfw_f(x):
        return torch.log1p(x) - x / (1.0 + x)

    cum = np.concatenate([[0], np.cumsum(all_sizes)])
    off, h0, nh = 0, 0, all_sizes.shape[0]
    while h0 < nh:
        h1 = int(np.searchsorted(cum, cum[h0] + chunk, side="right")) - 1
        h1 = max(h1, h0 + 1)
        h1 = min(h1, nh)
        cnt = torch.from_numpy(all_sizes[h0:h1]).to(dev)
        hid = torch.repeat_interleave(torch.arange(h0, h1, device=dev), cnt)
        k = int(hid.shape[0])
        c = c_t[hid]
        p = uni(k) * nfw_f(c)
        lo = torch.zeros(k, dtype=f64, device=dev)
        hi = c.clone()
        for _ in range(60):  # f(x) = p on [0, c]; f increases monotonically
            mid = 0.5 * (lo + hi)
            below = nfw_f(mid) < p
            lo = torch.where(below, mid, lo)
            hi = torch.where(below, hi, mid)
        r = 0.5 * (lo + hi) * (rv_t[hid] / c)
        del lo, hi, p, c
        mu = 2.0 * uni(k) - 1.0
        phi = (2.0 * math.pi) * uni(k)
        s = torch.sqrt(torch.clamp(1.0 - mu * mu, min=0.0))
        d = (s * torch.cos(phi), s * torch.sin(phi), mu)
        for a in range(3):
            P[a, off:off + k] = (ctr_t[hid, a] + r * d[a]).float()
            V[a, off:off + k] = (bulk_t[hid, a] + sig_t[hid] * torch.randn(
                k, generator=gen, device=dev, dtype=f64)).float()
        off += k
        h0 = h1
        del hid, r, mu, phi, s, d
    n_bg = n_total - off
    if n_bg < 0:
        raise ValueError("halo particles exceed the particle budget")
    for a in range(3):
        P[a, off:] = (uni(n_bg) * box).float()
        V[a, off:] = (100.0 * torch.randn(n_bg, generator=gen, device=dev, dtype=f64)).float()
    perm = torch.randperm(n_total, generator=gen, device=dev)
    cols = []
    for a in range(3):
        col = torch.remainder(P[a][perm].double(), box).float()
        col[col >= box] = 0.0
        cols.append(col.contiguous())
    del P
    vcols = [V[a][perm].contiguous() for a in range(3)]
    del V, perm
    halos = dict(host_sizes=sizes, host_centres=host_ctr, host_bulk=host_bulk,
                 host_rvir=host_rvir, host_c=host_c, sub_host=sub_host, sub_sizes=sub_sizes)
    return DeviceCatalog(spec.name, box, n_total, cols[0], cols[1], cols[2], vcols[0],
                         vcols[1], vcols[2], mp, default_softening(n_total, box), halos)
