"""The workspace allocator of the boundary: every byte of device workspace comes
from the caller's callback (torch's caching allocator by default), a refused
request is reported as LIBHALO_ENOMEM with the outputs left untouched, and the
context returns every block when it ends."""
import numpy as np
import pytest
import torch

from tests.gpu_util import note, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


class Counting:
    """torch's caching allocator with a ledger of the live blocks."""

    def __init__(self, H, device=0, limit=None):
        self.inner_alloc, self.inner_free = H.torch_allocator(device)
        self.live = {}
        self.calls = 0
        self.frees = 0
        self.limit = limit

    def alloc(self, nbytes, stream):
        self.calls += 1
        if self.limit is not None and nbytes > self.limit:
            return None
        p = self.inner_alloc(nbytes, stream)
        if p:
            self.live[p] = nbytes
        return p

    def free(self, ptr, stream):
        assert ptr in self.live, "the library freed a block it was not given"
        del self.live[ptr]
        self.frees += 1
        self.inner_free(ptr, stream)


def test_counting_allocator_sees_every_block(H, c1):
    note("allocator: counting allocator over the whole path")
    P = H.Particles.from_catalog(c1)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    cnt = Counting(H)
    ctx = H.Halo(H.params_for_catalog(c1), allocator=(cnt.alloc, cnt.free))
    ref = H.Halo(H.params_for_catalog(c1)).run_all(P)
    torch.cuda.synchronize()
    mid = torch.cuda.memory_allocated()
    out = ctx.run_all(P)
    torch.cuda.synchronize()
    # identical results whatever serves the workspace
    np.testing.assert_array_equal(to_np(out["halo_of"]), to_np(ref["halo_of"]))
    np.testing.assert_array_equal(to_np(out["phi"]), to_np(ref["phi"]))
    live = sum(cnt.live.values())
    assert cnt.calls >= 2 and live >= 256 + 1024 * 1024
    # the blocks are torch's: its allocator accounts for them
    assert torch.cuda.memory_allocated() - mid >= live
    ctx.close()
    torch.cuda.synchronize()
    assert cnt.live == {} and cnt.frees == cnt.calls
    del out, ref
    assert base >= 0


@pytest.mark.parametrize("stage", ["fof3d", "refine6d", "assign", "unbind", "props"])
def test_refused_workspace_is_enomem(H, c1, stage):
    """An allocator that refuses every block above 4 KiB (the 4 KiB error block
    of the context passes): the stage fails with ENOMEM and its outputs keep the
    values they had."""
    note(f"allocator: refused workspace in {stage}")
    P = H.Particles.from_catalog(c1)
    good = H.Halo(H.params_for_catalog(c1))
    fof = good.fof3d(P)
    nodes, deepest = good.refine6d(P, fof)
    halos, halo_of = good.assign(P, nodes, deepest)
    unb, bound, phi = good.unbind(P, halos, halo_of)
    torch.cuda.synchronize()
    cnt = Counting(H, limit=4096)
    bad = H.Halo(H.params_for_catalog(c1), allocator=(cnt.alloc, cnt.free))
    L, dev, n = bad.L, bad.device, P.n
    sentinel = torch.full((n,), 12345, dtype=torch.int32, device=dev)
    cs = H._cstruct
    if stage == "fof3d":
        lab, perm = sentinel.clone(), sentinel.clone()
        first = torch.full((8,), 7, dtype=torch.int32, device=dev)
        count = first.clone()
        ng, nm = H.C.c_int64(0), H.C.c_int64(0)
        outs = [lab, perm, first, count]

        def call():
            return L.libhalo_fof3d(bad.h, n, P.dtype_code, *P.args(False), H._ptr(lab),
                                   H._ptr(perm), H._ptr(first), H._ptr(count), 8,
                                   H.C.byref(ng), H.C.byref(nm), H._stream())
    elif stage == "refine6d":
        cap = max(16, fof["n_members"] // 4)
        tab = {k: torch.full((cap,), 7, dtype=t, device=dev) for k, t in H.NODE_FIELDS}
        S = cs(H.NodesS, H.NODE_FIELDS, tab, cap)
        dp = sentinel.clone()
        nn = H.C.c_int64(0)
        outs = [dp] + list(tab.values())

        def call():
            return L.libhalo_refine6d(bad.h, n, P.dtype_code, *P.args(), H._ptr(fof["perm"]),
                                      H._ptr(fof["grp_first"]), H._ptr(fof["grp_count"]),
                                      fof["n_groups"], H.C.byref(S), H._ptr(dp), H.C.byref(nn),
                                      H._stream())
    elif stage == "assign":
        nn = int(nodes["parent"].shape[0])
        NS = cs(H.NodesS, H.NODE_FIELDS, nodes, nn)
        tab = {k: torch.full((nn,), 7, dtype=t, device=dev) for k, t in H.HALO_FIELDS}
        HS = cs(H.HalosS, H.HALO_FIELDS, tab, nn)
        ho = sentinel.clone()
        nh = H.C.c_int64(0)
        outs = [ho] + list(tab.values())

        def call():
            return L.libhalo_assign(bad.h, n, P.dtype_code, *P.args(), H.C.byref(NS), nn,
                                    H._ptr(deepest), H.C.byref(HS), H._ptr(ho), H.C.byref(nh),
                                    H._stream())
    elif stage == "unbind":
        nh = int(halos["seed_node"].shape[0])
        HS = cs(H.HalosS, H.HALO_FIELDS, halos, nh)
        out = {k: torch.full((nh,), 7, dtype=t, device=dev) for k, t in H.UNB_FIELDS}
        US = cs(H.UnbS, H.UNB_FIELDS, out)
        bd = torch.full((n,), 9, dtype=torch.uint8, device=dev)
        ph = torch.full((n,), 3.5, dtype=torch.float64, device=dev)
        outs = [bd, ph] + list(out.values())

        def call():
            return L.libhalo_unbind(bad.h, n, P.dtype_code, *P.args(), H.C.byref(HS), nh,
                                    H._ptr(halo_of), H._ptr(bd), H._ptr(ph), H.C.byref(US),
                                    H._stream())
    else:
        nn = int(nodes["parent"].shape[0])
        nh = int(halos["seed_node"].shape[0])
        NS = cs(H.NodesS, H.NODE_FIELDS, nodes, nn)
        HS = cs(H.HalosS, H.HALO_FIELDS, halos, nh)
        out = {k: torch.full((nh,), 7, dtype=t, device=dev) for k, t in H.PROP_FIELDS}
        PS = cs(H.PropsS, H.PROP_FIELDS, out)
        outs = list(out.values())

        def call():
            return L.libhalo_props(bad.h, n, P.dtype_code, *P.args(), H.C.byref(NS), nn,
                                   H.C.byref(HS), nh, H._ptr(halo_of), H._ptr(bound),
                                   H.C.byref(PS), H._stream())
    before = [o.clone() for o in outs]
    torch.cuda.synchronize()
    rc = call()
    torch.cuda.synchronize()
    assert rc == -2, (rc, L.libhalo_last_error(bad.h))
    assert b"allocator" in L.libhalo_last_error(bad.h)
    for a, b in zip(outs, before):
        assert torch.equal(a, b), "an output was written before the workspace was refused"
    bad.close()
    assert cnt.live == {}


def test_ctx_create_enomem(H, c1):
    """A context whose allocator refuses even the error word is not created."""
    note("allocator: refused error word")
    with pytest.raises(H.HaloError) as e:
        H.Halo(H.params_for_catalog(c1), allocator=(lambda nb, st: None, lambda p, st: None))
    assert e.value.code == -2
