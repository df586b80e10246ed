"""Thin Python binding of libhalo (ctypes).  Argument marshalling only: every
step of the path runs in the HIP kernels of libhalo.so.  PyTorch provides the
device memory (caller-owned outputs) and the stream.

The library must be built (``paper_1110_4372_amd.build.build()``); loading
fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhalo.so")

F32, F64 = 0, 1
PLAIN, BATCHED = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ECAPACITY", -5: "EGEOMETRY"}


class HaloError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhalo {STATUS.get(code, code)}: {msg}")
        self.code = code


class CParams(C.Structure):
    _fields_ = [("box", C.c_double), ("b", C.c_double), ("f", C.c_double),
                ("min_members", C.c_int32), ("max_levels", C.c_int32),
                ("merge_q2", C.c_double), ("particle_mass", C.c_double), ("G", C.c_double),
                ("rho_vir", C.c_double), ("softening", C.c_double), ("core_frac", C.c_double),
                ("unbound_threshold", C.c_double), ("e_recheck", C.c_double),
                ("mode", C.c_int32), ("prec", C.c_int32), ("grid_min", C.c_int32),
                ("ell_subset", C.c_int32), ("major_merger", C.c_double),
                ("fof_dense", C.c_int32), ("bh_min", C.c_int32), ("bh_theta", C.c_double),
                ("nn_chunk", C.c_int32), ("fof_chunk", C.c_int32), ("pot_chunk", C.c_int32),
                ("kd_leaf", C.c_int32), ("bh_leaf", C.c_int32), ("nn_bracket", C.c_double)]


@dataclasses.dataclass
class Params:
    box: float
    particle_mass: float
    softening: float
    # (Mpc/h)(km/s)^2/(Msun/h); 360 x the background density of Omega_m = 0.27
    # (Table 1, Section 3.3) with rho_crit = 2.77536627e11 (Msun/h)/(Mpc/h)^3
    G: float = 4.30091e-9
    rho_vir: float = 360.0 * 0.27 * 2.77536627e11
    b: float = 0.28
    f: float = 0.7
    min_members: int = 10
    max_levels: int = 200
    merge_q2: float = 200.0
    core_frac: float = 0.1
    unbound_threshold: float = 0.5
    e_recheck: float = 1e-4
    mode: int = BATCHED
    prec: int = PREC_FP64
    grid_min: int = 0
    major_merger: float = 0.0
    ell_subset: int = 0
    fof_dense: int = 0
    bh_min: int = 0
    bh_theta: float = 0.0
    # work-unit sizes of the batched kernels (0 = library default; speed only)
    nn_chunk: int = 0
    fof_chunk: int = 0
    pot_chunk: int = 0
    # leaf sizes of the 6D search trees and of the tree potential (0 = 16)
    kd_leaf: int = 0
    bh_leaf: int = 0
    # nearest-neighbour bracket of ell^2 in sample standard deviations (0 = 4;
    # < 0: every walk exact; speed only)
    nn_bracket: float = 0.0

    def c(self) -> CParams:
        return CParams(self.box, self.b, self.f, self.min_members, self.max_levels,
                       self.merge_q2, self.particle_mass, self.G, self.rho_vir,
                       self.softening, self.core_frac, self.unbound_threshold,
                       self.e_recheck, self.mode, self.prec, self.grid_min,
                       self.ell_subset, self.major_merger, self.fof_dense, self.bh_min,
                       self.bh_theta, self.nn_chunk, self.fof_chunk, self.pot_chunk,
                       self.kd_leaf, self.bh_leaf, self.nn_bracket)


NODE_FIELDS = [("parent", torch.int32), ("level", torch.int32), ("first_child", torch.int32),
               ("n_children", torch.int32), ("count", torch.int32), ("canon", torch.int32),
               ("fof", torch.int32), ("flags", torch.int32), ("cx", torch.float64),
               ("cy", torch.float64), ("cz", torch.float64), ("vx", torch.float64),
               ("vy", torch.float64), ("vz", torch.float64), ("sx2", torch.float64),
               ("sv2", torch.float64), ("ell2", torch.float32)]
HALO_FIELDS = [("seed_node", torch.int32), ("merged_into", torch.int32), ("host", torch.int32),
               ("fof", torch.int32), ("n_assigned", torch.int32), ("xs", torch.float64),
               ("ys", torch.float64), ("zs", torch.float64), ("vxs", torch.float64),
               ("vys", torch.float64), ("vzs", torch.float64), ("sv2", torch.float64),
               ("vmax2", torch.float64)]
UNB_FIELDS = [("n_bound_own", torch.int32), ("n_s", torch.int32), ("n_bound_s", torch.int32),
              ("valid", torch.uint8), ("vbx", torch.float64), ("vby", torch.float64),
              ("vbz", torch.float64)]
PROP_FIELDS = [("px", torch.float64), ("py", torch.float64), ("pz", torch.float64),
               ("vcx", torch.float64), ("vcy", torch.float64), ("vcz", torch.float64),
               ("vbx", torch.float64), ("vby", torch.float64), ("vbz", torch.float64),
               ("mvir", torch.float64), ("rvir", torch.float64), ("vmax", torch.float64),
               ("voff", torch.float64), ("n_bound", torch.int32)]

EXTRA_FIELDS = [("xoff", torch.float64), ("jx", torch.float64), ("jy", torch.float64),
                ("jz", torch.float64), ("kin", torch.float64), ("pot", torch.float64),
                ("t_u", torch.float64), ("spin", torch.float64), ("spin_bullock", torch.float64),
                ("c_klypin", torch.float64), ("rs_klypin", torch.float64),
                ("b_to_a", torch.float64), ("c_to_a", torch.float64), ("ax", torch.float64),
                ("ay", torch.float64), ("az", torch.float64), ("n_shape", torch.int32),
                ("m_so", torch.float64), ("r_so", torch.float64)]
MAX_SO = 8

_P = C.c_void_p


def _struct(fields, with_cap):
    f = [(n, _P) for n, _ in fields]
    if with_cap:
        f.append(("cap", C.c_int64))
    return type("S", (C.Structure,), {"_fields_": f})


NodesS = _struct(NODE_FIELDS, True)
HalosS = _struct(HALO_FIELDS, True)
UnbS = _struct(UNB_FIELDS, False)
PropsS = _struct(PROP_FIELDS, False)
ExtraS = _struct(EXTRA_FIELDS, True)

# Exported symbols (the C ABI of include/libhalo.h).
SYMBOLS = ["libhalo_ctx_create", "libhalo_ctx_destroy", "libhalo_last_error",
           "libhalo_set_params", "libhalo_version", "libhalo_profile", "libhalo_profile_reset",
           "libhalo_profile_read", "libhalo_profile_work", "libhalo_fof3d",
           "libhalo_fof3d_noalloc", "libhalo_refine6d",
           "libhalo_assign", "libhalo_unbind", "libhalo_props", "libhalo_props_extra"]

# Workspace allocator callbacks of libhalo_ctx_create.
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def torch_allocator(device: int):
    """(alloc, free) callables serving the library's workspace from torch's
    caching allocator on `device`, on the stream the library names."""
    def alloc(nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except RuntimeError:  # out of memory: the library reports ENOMEM
            return None

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhalo.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_1110_4372_amd.build.build()")
    L = C.CDLL(path)
    i64, i32 = C.c_int64, C.c_int
    pi64 = C.POINTER(C.c_int64)
    L.libhalo_ctx_create.argtypes = [C.POINTER(CParams), i32, ALLOC_FN, FREE_FN, _P,
                                     C.POINTER(_P)]
    L.libhalo_ctx_destroy.argtypes = [_P]
    L.libhalo_last_error.argtypes = [_P]
    L.libhalo_last_error.restype = C.c_char_p
    L.libhalo_set_params.argtypes = [_P, C.POINTER(CParams)]
    L.libhalo_version.restype = C.c_char_p
    L.libhalo_profile.argtypes = [_P, i32]
    L.libhalo_profile_reset.argtypes = [_P]
    L.libhalo_profile_read.argtypes = [_P, C.c_char_p, C.POINTER(C.c_double), pi64]
    L.libhalo_profile_work.argtypes = [_P, C.c_char_p, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
    L.libhalo_fof3d.argtypes = [_P, i64, i32, _P, _P, _P, _P, _P, _P, _P, i64, pi64, pi64, _P]
    L.libhalo_fof3d_noalloc.argtypes = L.libhalo_fof3d.argtypes
    L.libhalo_refine6d.argtypes = [_P, i64, i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, i64,
                                   C.POINTER(NodesS), _P, pi64, _P]
    L.libhalo_assign.argtypes = [_P, i64, i32, _P, _P, _P, _P, _P, _P, C.POINTER(NodesS), i64,
                                 _P, C.POINTER(HalosS), _P, pi64, _P]
    L.libhalo_unbind.argtypes = [_P, i64, i32, _P, _P, _P, _P, _P, _P, C.POINTER(HalosS), i64,
                                 _P, _P, _P, C.POINTER(UnbS), _P]
    L.libhalo_props.argtypes = [_P, i64, i32, _P, _P, _P, _P, _P, _P, C.POINTER(NodesS), i64,
                                C.POINTER(HalosS), i64, _P, _P, C.POINTER(PropsS), _P]
    L.libhalo_props_extra.argtypes = [_P, i64, i32, _P, _P, _P, _P, _P, _P, C.POINTER(NodesS),
                                      i64, C.POINTER(HalosS), i64, _P, _P, C.POINTER(PropsS),
                                      i32, _P, C.POINTER(ExtraS), _P]
    _lib = L
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _table(fields, cap, device):
    return {n: torch.empty(max(cap, 1), dtype=t, device=device) for n, t in fields}


def _cstruct(S, fields, tab, cap=None):
    s = S()
    for n, _ in fields:
        setattr(s, n, tab[n].data_ptr())
    if cap is not None:
        s.cap = cap
    return s


class Particles:
    """Device particle arrays (input order): positions float32/float64, velocities float32."""

    def __init__(self, x, y, z, vx, vy, vz):
        self.x, self.y, self.z, self.vx, self.vy, self.vz = x, y, z, vx, vy, vz
        assert x.dtype in (torch.float32, torch.float64)
        for t in (x, y, z, vx, vy, vz):
            assert t.is_cuda and t.is_contiguous() and t.shape == x.shape
        for t in (y, z):
            assert t.dtype == x.dtype
        for t in (vx, vy, vz):
            assert t.dtype == torch.float32

    @classmethod
    def from_catalog(cls, cat, device="cuda"):
        def t(a):
            return a if isinstance(a, torch.Tensor) else torch.from_numpy(a).to(device)
        return cls(t(cat.x), t(cat.y), t(cat.z), t(cat.vx), t(cat.vy), t(cat.vz))

    @property
    def n(self):
        return int(self.x.shape[0])

    @property
    def dtype_code(self):
        return F64 if self.x.dtype == torch.float64 else F32

    def args(self, vel=True):
        a = [_ptr(self.x), _ptr(self.y), _ptr(self.z)]
        if vel:
            a += [_ptr(self.vx), _ptr(self.vy), _ptr(self.vz)]
        return a


class Halo:
    """A libhalo context on one device with its parameters.  The workspace
    comes from torch's caching allocator unless `allocator` gives other
    (alloc(nbytes, stream) -> int or None, free(ptr, stream)) callables."""

    def __init__(self, params: Params, device: int = 0, allocator=None):
        self.L = load_library()
        self.params = params
        self.device = torch.device("cuda", device)
        self._cp = params.c()
        alloc, free = allocator if allocator is not None else torch_allocator(device)
        # the ctypes thunks must outlive the context
        self._alloc = ALLOC_FN(lambda nbytes, user, stream: alloc(nbytes, stream))
        self._free = FREE_FN(lambda ptr, user, stream: free(ptr, stream))
        h = C.c_void_p()
        rc = self.L.libhalo_ctx_create(C.byref(self._cp), device, self._alloc, self._free,
                                       None, C.byref(h))
        if rc != 0:
            raise HaloError(rc, "context creation failed")
        self.h = h

    def close(self):
        if self.h:
            self.L.libhalo_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        self._cp = params.c()
        self._check(self.L.libhalo_set_params(self.h, C.byref(self._cp)))
        self.params = params

    def _check(self, rc):
        if rc != 0:
            msg = self.L.libhalo_last_error(self.h).decode()
            raise HaloError(rc, msg)

    # ------------------------------------------------------------ timing --
    def profile(self, enable: bool = True, count: bool = False):
        """Bracket the library's hot kernel launches with HIP events (enable),
        and run the tree walks in their work-counting form (count)."""
        self._check(self.L.libhalo_profile(self.h, (1 if enable else 0) | (2 if count else 0)))

    def profile_reset(self):
        self._check(self.L.libhalo_profile_reset(self.h))

    def profile_read(self, kernel: str):
        """(total device ms, launches) of `kernel` since the last reset."""
        t, k = C.c_double(0.0), C.c_int64(0)
        self._check(self.L.libhalo_profile_read(self.h, kernel.encode(), C.byref(t), C.byref(k)))
        return t.value, k.value

    def profile_work(self, kernel: str):
        """(box tests, distances) counted by a tree walk since the last reset:
        "k_kd_walk_nn" or "k_kd_walk_fof"; for "k_bh_walk" (cells tested,
        terms added), summed over target particles."""
        t, e = C.c_double(0.0), C.c_double(0.0)
        self._check(self.L.libhalo_profile_work(self.h, kernel.encode(), C.byref(t), C.byref(e)))
        return t.value, e.value

    # ------------------------------------------------------------ stages --
    def fof3d(self, P: Particles, grp_cap: int | None = None):
        dev = self.device
        n = P.n
        label = torch.empty(n, dtype=torch.int32, device=dev)
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        cap = grp_cap if grp_cap is not None else max(1, n // self.params.min_members)
        first = torch.empty(cap, dtype=torch.int32, device=dev)
        count = torch.empty(cap, dtype=torch.int32, device=dev)
        ng, nm = C.c_int64(0), C.c_int64(0)
        self._check(self.L.libhalo_fof3d(self.h, n, P.dtype_code, *P.args(False), _ptr(label),
                                         _ptr(perm), _ptr(first), _ptr(count), cap,
                                         C.byref(ng), C.byref(nm), _stream()))
        g = ng.value
        return dict(label=label, perm=perm[: nm.value], grp_first=first[:g],
                    grp_count=count[:g], n_groups=g, n_members=nm.value)

    def fof3d_noalloc(self, P: Particles, label, perm, grp_first, grp_count):
        """libhalo_fof3d_noalloc into caller-allocated int32 tensors (label and
        perm of P.n entries, grp_first and grp_count of the table's capacity):
        the call allocates nothing.  Returns (n_groups, n_members)."""
        assert grp_first.shape[0] == grp_count.shape[0]
        assert label.shape[0] >= P.n and perm.shape[0] >= P.n
        ng, nm = C.c_int64(0), C.c_int64(0)
        self._check(self.L.libhalo_fof3d_noalloc(
            self.h, P.n, P.dtype_code, *P.args(False), _ptr(label), _ptr(perm),
            _ptr(grp_first), _ptr(grp_count), grp_first.shape[0], C.byref(ng), C.byref(nm),
            _stream()))
        return ng.value, nm.value

    def refine6d(self, P: Particles, fof: dict, node_cap: int | None = None):
        dev = self.device
        cap = node_cap if node_cap is not None else max(16, fof["n_members"] // 4)
        while True:
            tab = _table(NODE_FIELDS, cap, dev)
            S = _cstruct(NodesS, NODE_FIELDS, tab, cap)
            deepest = torch.empty(P.n, dtype=torch.int32, device=dev)
            nn = C.c_int64(0)
            rc = self.L.libhalo_refine6d(self.h, P.n, P.dtype_code, *P.args(), _ptr(fof["perm"]),
                                         _ptr(fof["grp_first"]), _ptr(fof["grp_count"]),
                                         fof["n_groups"], C.byref(S), _ptr(deepest),
                                         C.byref(nn), _stream())
            if rc == -4 and node_cap is None:
                cap = nn.value
                continue
            self._check(rc)
            k = nn.value
            return {n: t[:k] for n, t in tab.items()}, deepest

    def assign(self, P: Particles, nodes: dict, deepest, halo_cap: int | None = None):
        dev = self.device
        nn = int(nodes["parent"].shape[0])
        NS = _cstruct(NodesS, NODE_FIELDS, nodes, nn)
        cap = halo_cap if halo_cap is not None else max(1, nn)
        tab = _table(HALO_FIELDS, cap, dev)
        HS = _cstruct(HalosS, HALO_FIELDS, tab, cap)
        halo_of = torch.empty(P.n, dtype=torch.int32, device=dev)
        nh = C.c_int64(0)
        self._check(self.L.libhalo_assign(self.h, P.n, P.dtype_code, *P.args(), C.byref(NS), nn,
                                          _ptr(deepest), C.byref(HS), _ptr(halo_of),
                                          C.byref(nh), _stream()))
        k = nh.value
        return {n: t[:k] for n, t in tab.items()}, halo_of

    def unbind(self, P: Particles, halos: dict, halo_of, want_phi: bool = True):
        dev = self.device
        nh = int(halos["seed_node"].shape[0])
        HS = _cstruct(HalosS, HALO_FIELDS, halos, nh)
        out = _table(UNB_FIELDS, nh, dev)
        US = _cstruct(UnbS, UNB_FIELDS, out)
        bound = torch.empty(P.n, dtype=torch.uint8, device=dev)
        phi = torch.empty(P.n, dtype=torch.float64, device=dev) if want_phi else None
        self._check(self.L.libhalo_unbind(self.h, P.n, P.dtype_code, *P.args(), C.byref(HS), nh,
                                          _ptr(halo_of), _ptr(bound), _ptr(phi), C.byref(US),
                                          _stream()))
        return {n: t[:nh] for n, t in out.items()}, bound, phi

    def props(self, P: Particles, nodes: dict, halos: dict, halo_of, bound):
        dev = self.device
        nn = int(nodes["parent"].shape[0])
        nh = int(halos["seed_node"].shape[0])
        NS = _cstruct(NodesS, NODE_FIELDS, nodes, nn)
        HS = _cstruct(HalosS, HALO_FIELDS, halos, nh)
        out = _table(PROP_FIELDS, nh, dev)
        PS = _cstruct(PropsS, PROP_FIELDS, out)
        self._check(self.L.libhalo_props(self.h, P.n, P.dtype_code, *P.args(), C.byref(NS), nn,
                                         C.byref(HS), nh, _ptr(halo_of), _ptr(bound),
                                         C.byref(PS), _stream()))
        return {n: t[:nh] for n, t in out.items()}

    def props_extra(self, P: Particles, nodes: dict, halos: dict, halo_of, bound, so_rho=()):
        """libhalo_props_extra: (basic properties, additional properties); m_so
        and r_so have shape [len(so_rho), n_halos]."""
        dev = self.device
        nn = int(nodes["parent"].shape[0])
        nh = int(halos["seed_node"].shape[0])
        so = [float(r) for r in so_rho]
        if len(so) > MAX_SO:
            raise ValueError(f"at most {MAX_SO} SO thresholds")
        NS = _cstruct(NodesS, NODE_FIELDS, nodes, nn)
        HS = _cstruct(HalosS, HALO_FIELDS, halos, nh)
        out = _table(PROP_FIELDS, nh, dev)
        PS = _cstruct(PropsS, PROP_FIELDS, out)
        cap = max(nh, 1)
        ext = {n: torch.zeros(cap * max(len(so), 1) if n in ("m_so", "r_so") else cap,
                              dtype=t, device=dev) for n, t in EXTRA_FIELDS}
        ES = _cstruct(ExtraS, EXTRA_FIELDS, ext, cap)
        rho_arr = (C.c_double * max(len(so), 1))(*so)
        rho = C.cast(rho_arr, C.c_void_p) if so else None
        self._check(self.L.libhalo_props_extra(
            self.h, P.n, P.dtype_code, *P.args(), C.byref(NS), nn, C.byref(HS), nh,
            _ptr(halo_of), _ptr(bound), C.byref(PS), len(so), rho, C.byref(ES), _stream()))
        res = {n: t[:nh] for n, t in ext.items() if n not in ("m_so", "r_so")}
        for n in ("m_so", "r_so"):
            res[n] = ext[n][:cap * len(so)].view(len(so), cap)[:, :nh]
        return {n: t[:nh] for n, t in out.items()}, res

    def run_all(self, P: Particles):
        """One pass of the whole path: fof3d -> refine6d -> assign -> unbind -> props."""
        fof = self.fof3d(P)
        nodes, deepest = self.refine6d(P, fof)
        halos, halo_of = self.assign(P, nodes, deepest)
        unb, bound, phi = self.unbind(P, halos, halo_of)
        pr = self.props(P, nodes, halos, halo_of, bound)
        return dict(fof=fof, nodes=nodes, deepest=deepest, halos=halos, halo_of=halo_of,
                    unbound=unb, bound=bound, phi=phi, props=pr)


def params_for_catalog(cat, **kw) -> Params:
    """Parameters of a catalogue (box, particle mass, softening); G and the
    virial density keep the defaults of Params."""
    return Params(box=cat.box, particle_mass=cat.particle_mass, softening=cat.softening, **kw)
