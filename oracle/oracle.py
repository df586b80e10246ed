"""ctypes front end of the plain serial FP64 CPU oracle (halo_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library and imports nothing from the product package; the two
meet only in the seeded catalogues that the tests pass to both.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "halo_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

# ---- units and constants (Section 3.3 and Table 1; positions in Mpc/h,
# velocities in km/s, masses in Msun/h) -- the oracle's own definitions.
# G in (Mpc/h) (km/s)^2 / (Msun/h): G M_sun / (1 Mpc (1 km/s)^2); the h factors
# cancel.  Pinned against the SI values in tests/test_oracle_pins.py.
G_NEWTON = 4.30091e-9
# critical density 3 H0^2 / (8 pi G) with H0 = 100 h km/s/Mpc, in
# (Msun/h) / (Mpc/h)^3
RHO_CRIT = 2.77536627e11
# matter density of the Bolshoi cosmology (Table 1)
OMEGA_M = 0.27
RHO_M = OMEGA_M * RHO_CRIT
# virial overdensity against the background density at z = 0 (Section 3.3)
DELTA_VIR = 360.0
RHO_VIR = DELTA_VIR * RHO_M


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, FP64, no fused contractions)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("box", C.c_double), ("b", C.c_double), ("f", C.c_double),
                ("min_members", C.c_int32), ("max_levels", C.c_int32),
                ("merge_q2", C.c_double), ("particle_mass", C.c_double),
                ("G", C.c_double), ("rho_vir", C.c_double), ("softening", C.c_double),
                ("core_frac", C.c_double), ("unbound_threshold", C.c_double),
                ("ell_subset", C.c_int32), ("major_merger", C.c_double),
                ("fof_dense", C.c_int32)]


_P = C.c_void_p

NODE_FIELDS = [("parent", np.int32), ("level", np.int32), ("first_child", np.int32),
               ("n_children", np.int32), ("count", np.uint32), ("canon", np.uint32),
               ("fof", np.uint32), ("flags", np.uint32), ("cx", np.float64),
               ("cy", np.float64), ("cz", np.float64), ("vx", np.float64),
               ("vy", np.float64), ("vz", np.float64), ("sx2", np.float64),
               ("sv2", np.float64), ("ell2", np.float32)]
HALO_FIELDS = [("seed_node", np.int32), ("merged_into", np.int32), ("host", np.int32),
               ("fof", np.uint32), ("n_assigned", np.uint32), ("xs", np.float64),
               ("ys", np.float64), ("zs", np.float64), ("vxs", np.float64),
               ("vys", np.float64), ("vzs", np.float64), ("sv2", np.float64),
               ("vmax2", np.float64)]
UNB_FIELDS = [("n_bound_own", np.uint32), ("n_s", np.uint32), ("n_bound_s", np.uint32),
              ("valid", np.uint8), ("vbx", np.float64), ("vby", np.float64),
              ("vbz", np.float64)]
PROP_FIELDS = [("px", np.float64), ("py", np.float64), ("pz", np.float64),
               ("vcx", np.float64), ("vcy", np.float64), ("vcz", np.float64),
               ("vbx", np.float64), ("vby", np.float64), ("vbz", np.float64),
               ("mvir", np.float64), ("rvir", np.float64), ("vmax", np.float64),
               ("voff", np.float64), ("n_bound", np.uint32)]


EXTRA_FIELDS = [("sx", np.float64), ("sy", np.float64), ("sz", np.float64),
                ("jx", np.float64), ("jy", np.float64), ("jz", np.float64),
                ("t2", np.float64), ("uinv", np.float64), ("mxx", np.float64),
                ("myy", np.float64), ("mzz", np.float64), ("mxy", np.float64),
                ("mxz", np.float64), ("myz", np.float64), ("k", np.uint32),
                ("n_own", np.uint32), ("k_so", np.uint32)]


def _struct(fields):
    return type("S", (C.Structure,), {"_fields_": [(n, _P) for n, _ in fields]})


NodesS, HalosS, UnbS, PropsS, ExtraS = (_struct(NODE_FIELDS), _struct(HALO_FIELDS),
                                       _struct(UNB_FIELDS), _struct(PROP_FIELDS),
                                       _struct(EXTRA_FIELDS))


def _alloc(fields, cap):
    arrs = {n: np.zeros(max(cap, 1), dtype=t) for n, t in fields}
    return arrs


def _fill(S, fields, arrs):
    s = S()
    for n, _ in fields:
        setattr(s, n, arrs[n].ctypes.data)
    return s


def _trim(arrs, k):
    return {n: a[:k].copy() for n, a in arrs.items()}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        i64, i32 = C.c_int64, C.c_int
        L.orc_fof3d.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P]
        L.orc_refine6d.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P, _P, _P, _P,
                                   i64, C.POINTER(NodesS), _P, C.POINTER(C.c_int64)]
        L.orc_assign.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P, _P, _P,
                                 C.POINTER(NodesS), i64, _P, i64, C.POINTER(HalosS), _P,
                                 C.POINTER(C.c_int64)]
        L.orc_unbind.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P, _P, _P,
                                 C.POINTER(HalosS), i64, _P, _P, _P, _P, C.POINTER(UnbS)]
        L.orc_props.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P, _P, _P,
                                C.POINTER(NodesS), i64, C.POINTER(HalosS), i64, _P, _P,
                                C.POINTER(PropsS)]
        L.orc_props_extra.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P, _P, _P,
                                      C.POINTER(HalosS), i64, _P, _P, C.POINTER(PropsS), i32,
                                      _P, C.POINTER(ExtraS)]
        L.orc_halo_sums.argtypes = [i64, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double, _P]
        L.orc_halo_sums.restype = None
        L.orc_so_count.argtypes = [i64, _P, C.c_double]
        L.orc_so_count.restype = C.c_int64
        L.orc_node_normalise.argtypes = [C.POINTER(Params), i64, i32, _P, _P, _P, _P, _P,
                                         _P, _P, _P, _P]
        L.orc_nn6d.argtypes = [i64, _P, _P]
        L.orc_nn6d.restype = None
        L.orc_ell2.argtypes = [i64, _P, C.c_double]
        L.orc_ell2.restype = C.c_float
        L.orc_fof6d.argtypes = [i64, _P, C.c_float, _P]
        L.orc_fof6d.restype = None
        L.orc_nn6d_range.argtypes = [i64, _P, i64, i64, _P]
        L.orc_nn6d_range.restype = None
        L.orc_friends6d_range.argtypes = [i64, _P, C.c_float, i64, i64, i64, _P]
        L.orc_friends6d_range.restype = C.c_int64
        L.orc_phi_points.argtypes = [C.POINTER(Params), i32, _P, _P, _P, _P, i64, _P, i64, _P]
        L.orc_phi_points.restype = None
        L.orc_in_subset.argtypes = [C.c_uint64, C.c_int64, C.c_int64]
        L.orc_in_subset.restype = C.c_int
        L.orc_position_shift.argtypes = [C.c_double]
        L.orc_position_shift.restype = C.c_int32
        _lib = L
    return _lib


@dataclasses.dataclass
class Particles:
    """Particle arrays in input order (positions float64 or float32)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray

    @classmethod
    def of(cls, cat):
        return cls(cat.x, cat.y, cat.z, cat.vx, cat.vy, cat.vz)

    @property
    def n(self):
        return int(self.x.shape[0])

    @property
    def f64(self):
        return int(self.x.dtype == np.float64)

    def ptrs(self, vel=True):
        for a in (self.x, self.y, self.z) + ((self.vx, self.vy, self.vz) if vel else ()):
            assert a.flags.c_contiguous
        for a in (self.x, self.y, self.z):
            assert a.dtype == self.x.dtype
        if vel:
            for a in (self.vx, self.vy, self.vz):
                assert a.dtype == np.float32
        arrs = (self.x, self.y, self.z) + ((self.vx, self.vy, self.vz) if vel else ())
        return [a.ctypes.data for a in arrs]


def make_params(box, particle_mass, softening, *, b=0.28, f=0.7, min_members=10,
                max_levels=200, merge_q2=200.0, G=None, rho_vir=None, core_frac=0.1,
                unbound_threshold=0.5, major_merger=0.0, ell_subset=0,
                fof_dense=0) -> Params:
    return Params(box, b, f, min_members, max_levels, merge_q2, particle_mass,
                  G_NEWTON if G is None else G,
                  RHO_VIR if rho_vir is None else rho_vir, softening, core_frac,
                  unbound_threshold, ell_subset, major_merger, fof_dense)


def params_of(cat, **kw) -> Params:
    return make_params(cat.box, cat.particle_mass, cat.softening, **kw)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def fof3d(p: Params, P: Particles) -> np.ndarray:
    lab = np.zeros(P.n, dtype=np.uint32)
    _check(lib().orc_fof3d(C.byref(p), P.n, P.f64, *P.ptrs(False), lab.ctypes.data), "fof3d")
    return lab


def refine6d(p: Params, P: Particles, label: np.ndarray):
    label = np.ascontiguousarray(label, dtype=np.uint32)
    cap = max(16, P.n // 4)
    while True:
        arrs = _alloc(NODE_FIELDS, cap)
        S = _fill(NodesS, NODE_FIELDS, arrs)
        deepest = np.zeros(P.n, dtype=np.int32)
        nn = C.c_int64(0)
        rc = lib().orc_refine6d(C.byref(p), P.n, P.f64, *P.ptrs(), label.ctypes.data, cap,
                                C.byref(S), deepest.ctypes.data, C.byref(nn))
        if rc == -4:
            cap = nn.value
            continue
        _check(rc, "refine6d")
        return _trim(arrs, nn.value), deepest


def assign(p: Params, P: Particles, nodes: dict, deepest: np.ndarray):
    nn = int(nodes["parent"].shape[0])
    nodes = {k: np.ascontiguousarray(v) for k, v in nodes.items()}
    NS = _fill(NodesS, NODE_FIELDS, nodes)
    cap = max(1, int(np.sum(nodes["n_children"] == 0)))
    arrs = _alloc(HALO_FIELDS, cap)
    HS = _fill(HalosS, HALO_FIELDS, arrs)
    halo_of = np.zeros(P.n, dtype=np.int32)
    nh = C.c_int64(0)
    deepest = np.ascontiguousarray(deepest, dtype=np.int32)
    _check(lib().orc_assign(C.byref(p), P.n, P.f64, *P.ptrs(), C.byref(NS), nn,
                            deepest.ctypes.data, cap, C.byref(HS), halo_of.ctypes.data,
                            C.byref(nh)), "assign")
    return _trim(arrs, nh.value), halo_of


def unbind(p: Params, P: Particles, halos: dict, halo_of: np.ndarray):
    nh = int(halos["seed_node"].shape[0])
    halos = {k: np.ascontiguousarray(v) for k, v in halos.items()}
    HS = _fill(HalosS, HALO_FIELDS, halos)
    out = _alloc(UNB_FIELDS, nh)
    US = _fill(UnbS, UNB_FIELDS, out)
    bound = np.zeros(P.n, dtype=np.uint8)
    phi = np.zeros(P.n, dtype=np.float64)
    phia = np.zeros(P.n, dtype=np.float64)
    halo_of = np.ascontiguousarray(halo_of, dtype=np.int32)
    _check(lib().orc_unbind(C.byref(p), P.n, P.f64, *P.ptrs(), C.byref(HS), nh,
                            halo_of.ctypes.data, bound.ctypes.data, phi.ctypes.data,
                            phia.ctypes.data, C.byref(US)), "unbind")
    return _trim(out, nh), bound, phi, phia


def props(p: Params, P: Particles, nodes: dict, halos: dict, halo_of, bound):
    nn = int(nodes["parent"].shape[0])
    nh = int(halos["seed_node"].shape[0])
    nodes = {k: np.ascontiguousarray(v) for k, v in nodes.items()}
    halos = {k: np.ascontiguousarray(v) for k, v in halos.items()}
    NS = _fill(NodesS, NODE_FIELDS, nodes)
    HS = _fill(HalosS, HALO_FIELDS, halos)
    out = _alloc(PROP_FIELDS, nh)
    PS = _fill(PropsS, PROP_FIELDS, out)
    halo_of = np.ascontiguousarray(halo_of, dtype=np.int32)
    bound = np.ascontiguousarray(bound, dtype=np.uint8)
    _check(lib().orc_props(C.byref(p), P.n, P.f64, *P.ptrs(), C.byref(NS), nn, C.byref(HS), nh,
                           halo_of.ctypes.data, bound.ctypes.data, C.byref(PS)), "props")
    return _trim(out, nh)


def props_extra_sums(p: Params, P: Particles, halos: dict, halo_of, bound, pr: dict,
                     so_rho=()):
    """orc_props_extra: the per-halo sums behind the additional properties."""
    nh = int(halos["seed_node"].shape[0])
    halos = {k: np.ascontiguousarray(v) for k, v in halos.items()}
    HS = _fill(HalosS, HALO_FIELDS, halos)
    prc = {k: np.ascontiguousarray(v) for k, v in pr.items()}
    PS = _fill(PropsS, PROP_FIELDS, prc)
    so = np.ascontiguousarray(np.asarray(so_rho, dtype=np.float64).reshape(-1))
    n_so = int(so.shape[0])
    out = {n: np.zeros(max(nh, 1), dtype=t) for n, t in EXTRA_FIELDS if n != "k_so"}
    out["k_so"] = np.zeros(max(nh * n_so, 1), dtype=np.uint32)
    ES = _fill(ExtraS, EXTRA_FIELDS, out)
    halo_of = np.ascontiguousarray(halo_of, dtype=np.int32)
    bound = np.ascontiguousarray(bound, dtype=np.uint8)
    _check(lib().orc_props_extra(C.byref(p), P.n, P.f64, *P.ptrs(), C.byref(HS), nh,
                                 halo_of.ctypes.data, bound.ctypes.data, C.byref(PS), n_so,
                                 so.ctypes.data if n_so else None, C.byref(ES)), "props_extra")
    res = {k: v[:nh].copy() for k, v in out.items() if k != "k_so"}
    res["k_so"] = out["k_so"][:nh * n_so].reshape(n_so, nh).copy()
    return res


def halo_sums(dx, dy, dz, vx, vy, vz, own, vbulk, eps2):
    """orc_halo_sums on one explicit set (15 sums; see halo_oracle.c)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (dx, dy, dz, vx, vy, vz)]
    own = np.ascontiguousarray(own, dtype=np.uint8)
    vb = np.ascontiguousarray(vbulk, dtype=np.float64)
    out = np.zeros(15, dtype=np.float64)
    lib().orc_halo_sums(arrs[0].shape[0], *[a.ctypes.data for a in arrs], own.ctypes.data,
                        vb.ctypes.data, float(eps2), out.ctypes.data)
    return out


def so_count(r2_sorted, C_thr: float) -> int:
    r2 = np.ascontiguousarray(r2_sorted, dtype=np.float64)
    return int(lib().orc_so_count(r2.shape[0], r2.ctypes.data, float(C_thr)))


# Section 3.5.4, Eq. 5-6: radius of the NFW circular-velocity maximum in units
# of R_s, rounded as the paper prints it.  The concentration is sought on the
# branch c >= KLYPIN_X (R_max inside R_vir) and clamped to [KLYPIN_X,
# KLYPIN_CMAX] (reading: the paper gives no range).
KLYPIN_X = 2.1626
KLYPIN_CMAX = 1.0e4


def nfw_f(x):
    """f(x) = ln(1 + x) - x / (1 + x) (Eq. 8)."""
    return np.log1p(x) - x / (1.0 + x)


def klypin_concentration(vmax: float, mvir: float, rvir: float, G: float) -> float:
    """Eq. 7: c / f(c) = vmax^2 R_vir / (G M_vir) * X / f(X), X = KLYPIN_X,
    inverted numerically (Brent's method); 0 for a halo without mass."""
    from scipy.optimize import brentq
    if not (mvir > 0.0 and rvir > 0.0 and vmax > 0.0):
        return 0.0
    rhs = vmax * vmax * rvir / (G * mvir) * KLYPIN_X / nfw_f(KLYPIN_X)

    def g(c):
        return c / nfw_f(c) - rhs

    if g(KLYPIN_X) >= 0.0:
        return KLYPIN_X
    if g(KLYPIN_CMAX) <= 0.0:
        return KLYPIN_CMAX
    return float(brentq(g, KLYPIN_X, KLYPIN_CMAX, xtol=1e-14, rtol=1e-15, maxiter=1000))


def spin_parameters(Jmag, T, U, M, R, G):
    """Eq. 9 (Peebles): lambda = J sqrt(|E|) / (G M^2.5), E = T + U; Eq. 10
    (Bullock): lambda_B = J / sqrt(2 G M^3 R).  Zero for M = 0."""
    Jmag, T, U, M, R = (np.asarray(a, dtype=np.float64) for a in (Jmag, T, U, M, R))
    ok = M > 0.0
    Ms = np.where(ok, M, 1.0)
    Rs = np.where(R > 0.0, R, 1.0)
    lam = np.where(ok, Jmag * np.sqrt(np.abs(T + U)) / (G * Ms ** 2.5), 0.0)
    lamb = np.where(ok & (R > 0.0), Jmag / np.sqrt(2.0 * G * Ms ** 3 * Rs), 0.0)
    return lam, lamb


def shape_from_tensor(mxx, myy, mzz, mxy, mxz, myz, n):
    """Eq. 11: M_ab = (1/N) sum x_a x_b; its eigenvalues sorted a^2 >= b^2 >=
    c^2 give b/a, c/a and the major axis vector A = a e_1, signed so that its
    largest-magnitude component is positive.  Zeros when N = 0 or a = 0."""
    if n <= 0:
        return 0.0, 0.0, np.zeros(3)
    M = np.array([[mxx, mxy, mxz], [mxy, myy, myz], [mxz, myz, mzz]], dtype=np.float64) / n
    w, V = np.linalg.eigh(M)
    w = np.maximum(w[::-1], 0.0)
    V = V[:, ::-1]
    if w[0] <= 0.0:
        return 0.0, 0.0, np.zeros(3)
    e = V[:, 0]
    if e[int(np.argmax(np.abs(e)))] < 0.0:
        e = -e
    return float(np.sqrt(w[1] / w[0])), float(np.sqrt(w[2] / w[0])), np.sqrt(w[0]) * e


def props_extra(p: Params, P: Particles, halos: dict, halo_of, bound, pr: dict, so_rho=()):
    """The additional halo properties of Sections 3.5.2 and 3.5.4 from the
    oracle's own centre, bulk velocity, M_vir, R_vir and v_max:
      xoff        |centre of mass of V(h) - centre|
      jx, jy, jz  angular momentum m sum (x - c) x (v - v_bulk) over V(h)
      kin, pot    T = m/2 sum |v - v_bulk|^2 and U = -G m^2 sum_pairs
                  1/sqrt(r^2 + eps^2) over V(h); t_u = T / |U| (0 if U = 0)
      spin, spin_bullock  Eq. 9 and Eq. 10
      c_klypin, rs_klypin Eq. 7-8, R_s = R_vir / c
      b_to_a, c_to_a, ax, ay, az, n_shape  Eq. 11 over the own particles
      m_so, r_so  [n_so, n_halos] SO mass and radius at each threshold
    V(h) is the set that defines M_vir (the k* innermost bound particles of
    S(h))."""
    s = props_extra_sums(p, P, halos, halo_of, bound, pr, so_rho)
    m, G = p.particle_mass, p.G
    nh = int(halos["seed_node"].shape[0])
    k = s["k"].astype(np.float64)
    kk = np.maximum(k, 1.0)
    com = np.stack([s["sx"], s["sy"], s["sz"]], 1) / kk[:, None]
    out = {"xoff": np.where(k > 0, np.linalg.norm(com, axis=1), 0.0)}
    J = m * np.stack([s["jx"], s["jy"], s["jz"]], 1)
    out["jx"], out["jy"], out["jz"] = J[:, 0], J[:, 1], J[:, 2]
    T = 0.5 * m * s["t2"]
    U = -G * m * m * s["uinv"]
    out["kin"], out["pot"] = T, U
    out["t_u"] = np.where(U != 0.0, T / np.where(U != 0.0, np.abs(U), 1.0), 0.0)
    out["spin"], out["spin_bullock"] = spin_parameters(np.linalg.norm(J, axis=1), T, U,
                                                       pr["mvir"], pr["rvir"], G)
    c = np.array([klypin_concentration(float(pr["vmax"][h]), float(pr["mvir"][h]),
                                       float(pr["rvir"][h]), G) for h in range(nh)])
    out["c_klypin"] = c
    out["rs_klypin"] = np.where(c > 0, pr["rvir"] / np.where(c > 0, c, 1.0), 0.0)
    ba, ca, A = np.zeros(nh), np.zeros(nh), np.zeros((nh, 3))
    for h in range(nh):
        ba[h], ca[h], A[h] = shape_from_tensor(s["mxx"][h], s["myy"][h], s["mzz"][h],
                                               s["mxy"][h], s["mxz"][h], s["myz"][h],
                                               int(s["n_own"][h]))
    out["b_to_a"], out["c_to_a"] = ba, ca
    out["ax"], out["ay"], out["az"] = A[:, 0], A[:, 1], A[:, 2]
    out["n_shape"] = s["n_own"].copy()
    so = np.asarray(so_rho, dtype=np.float64).reshape(-1)
    ks = s["k_so"].astype(np.float64)
    out["m_so"] = ks * m
    out["r_so"] = np.cbrt(ks * (3.0 * m) / (4.0 * np.pi * so[:, None])) if so.size else ks
    out["k"] = s["k"]
    return out


def node_normalise(p: Params, P: Particles, members: np.ndarray):
    members = np.ascontiguousarray(members, dtype=np.int64)
    nm = int(members.shape[0])
    xi = np.zeros((nm, 6), dtype=np.float32)
    mom = np.zeros(8, dtype=np.float64)
    _check(lib().orc_node_normalise(C.byref(p), nm, P.f64, *P.ptrs(), members.ctypes.data,
                                    xi.ctypes.data, mom.ctypes.data), "normalise")
    return xi, mom


def nn6d(xi: np.ndarray) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    d = np.zeros(xi.shape[0], dtype=np.float32)
    lib().orc_nn6d(xi.shape[0], xi.ctypes.data, d.ctypes.data)
    return d


def ell2(dmin: np.ndarray, f: float = 0.7) -> float:
    dmin = np.ascontiguousarray(dmin, dtype=np.float32)
    return float(lib().orc_ell2(dmin.shape[0], dmin.ctypes.data, f))


def fof6d(xi: np.ndarray, l2: float) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    comp = np.zeros(xi.shape[0], dtype=np.int64)
    lib().orc_fof6d(xi.shape[0], xi.ctypes.data, C.c_float(l2), comp.ctypes.data)
    return comp


def _chunks(n, threads):
    """Contiguous ranges of the particles, more of them than threads, the
    early ones (longer rows in the pair loop) shorter."""
    k = 4 * threads
    edges = [int(round(n * (1.0 - math.sqrt(1.0 - t / k)))) for t in range(k + 1)]
    return [(a, b) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def nn6d_threads(xi: np.ndarray, threads: int = 8) -> np.ndarray:
    """nn6d with the particles split over threads (each range by the oracle's
    plain loop; ctypes releases the GIL during the calls)."""
    from concurrent.futures import ThreadPoolExecutor
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    n = xi.shape[0]
    d = np.zeros(n, dtype=np.float32)
    even = [(n * t // (4 * threads), n * (t + 1) // (4 * threads)) for t in range(4 * threads)]

    def run(r):
        a, b = r
        if b > a:
            lib().orc_nn6d_range(n, xi.ctypes.data, a, b, d[a:].ctypes.data)
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, even))
    return d


def fof6d_threads(xi: np.ndarray, l2: float, threads: int = 8) -> np.ndarray:
    """fof6d from the friend pairs (d^2 <= l2) found by the oracle's plain loop
    over ranges of particles in threads; components by scipy.  Returns the
    smallest member index of each particle's component."""
    from concurrent.futures import ThreadPoolExecutor
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    n = xi.shape[0]

    def run(r):
        a, b = r
        cap = 1 << 20
        while True:
            buf = np.zeros(2 * cap, dtype=np.int64)
            k = lib().orc_friends6d_range(n, xi.ctypes.data, C.c_float(l2), a, b, cap,
                                          buf.ctypes.data)
            if k <= cap:
                return buf[:2 * k].reshape(-1, 2)
            cap = int(k)
    with ThreadPoolExecutor(threads) as ex:
        pairs = np.concatenate(list(ex.map(run, _chunks(n, threads))) + [np.zeros((0, 2), np.int64)])
    g = coo_matrix((np.ones(pairs.shape[0], np.int8), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    mins = np.full(lab.max() + 1, n, dtype=np.int64)
    np.minimum.at(mins, lab, np.arange(n))
    return mins[lab]


def phi_points(p: Params, P: Particles, src: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    src = np.ascontiguousarray(src, dtype=np.int64)
    tgt = np.ascontiguousarray(tgt, dtype=np.int64)
    out = np.zeros(tgt.shape[0], dtype=np.float64)
    lib().orc_phi_points(C.byref(p), P.f64, *P.ptrs(False), src.ctypes.data, src.shape[0],
                         tgt.ctypes.data, tgt.shape[0], out.ctypes.data)
    return out


def position_shift(box: float) -> int:
    return int(lib().orc_position_shift(box))


def run_all(p: Params, P: Particles):
    """The whole path on the CPU: fof3d -> refine6d -> assign -> unbind -> props."""
    lab = fof3d(p, P)
    nodes, deepest = refine6d(p, P, lab)
    halos, halo_of = assign(p, P, nodes, deepest)
    unb, bound, phi, phia = unbind(p, P, halos, halo_of)
    pr = props(p, P, nodes, halos, halo_of, bound)
    return dict(label=lab, nodes=nodes, deepest=deepest, halos=halos, halo_of=halo_of,
                unbound=unb, bound=bound, phi=phi, phi_abs=phia, props=pr)
