"""The no-alloc form of the 3D FOF entry point: libhalo_fof3d_noalloc takes its
workspace from the library's fixed device scratch array instead of the
context's allocator.  Two calls in a row on one context (the second with fewer
particles, so stale scratch from the first must not leak into it) give the
labels, permutation and group table of libhalo_fof3d bit for bit, the
context's allocator is never called, and particles that need more scratch
than the array holds are refused with ENOMEM before any output is touched."""
import numpy as np
import pytest
import torch

from tests.gpu_util import note, to_np
from tests.test_gpu_alloc import Counting

pytestmark = pytest.mark.gpu

SENTINEL = -7


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def outputs(n, cap, dev="cuda"):
    return [torch.full((k,), SENTINEL, dtype=torch.int32, device=dev)
            for k in (n, n, cap, cap)]


def small_catalog():
    """8000 particles in a 15 Mpc/h box, power-law hosts of 20-2000, FP32."""
    from paper_1110_4372_amd import synth
    spec = synth.CatalogSpec("noalloc_small", 20, 15.0, False, "powerlaw", 0.4, 20.0, 2000.0)
    return synth.make_catalog(spec=spec, seed=3)


def test_noalloc_matches_fof3d(H, c1):
    small = small_catalog()
    assert small.n < c1.n and small.x.dtype == np.float32 and c1.x.dtype == np.float64
    cats = [c1, small]
    Ps = [H.Particles.from_catalog(c) for c in cats]
    # the outputs of both calls exist before the first one
    bufs = [outputs(c.n, max(1, c.n // 10)) for c in cats]
    cnt = Counting(H)
    ctx = H.Halo(H.params_for_catalog(c1), allocator=(cnt.alloc, cnt.free))
    torch.cuda.synchronize()
    calls0 = cnt.calls
    got = []
    for c, P, (label, perm, first, count) in zip(cats, Ps, bufs):
        note(f"fof3d_noalloc n={c.n} dtype={c.x.dtype}")
        ctx.set_params(H.params_for_catalog(c))
        ng, nm = ctx.fof3d_noalloc(P, label, perm, first, count)
        torch.cuda.synchronize()
        got.append((ng, nm))
    assert cnt.calls == calls0, "the no-alloc call used the context's allocator"
    for c, P, (label, perm, first, count), (ng, nm) in zip(cats, Ps, bufs, got):
        ref = H.Halo(H.params_for_catalog(c)).fof3d(P)
        torch.cuda.synchronize()
        assert (ng, nm) == (ref["n_groups"], ref["n_members"])
        assert ng >= 5
        np.testing.assert_array_equal(to_np(label), to_np(ref["label"]))
        np.testing.assert_array_equal(to_np(perm)[:nm], to_np(ref["perm"]))
        np.testing.assert_array_equal(to_np(first)[:ng], to_np(ref["grp_first"]))
        np.testing.assert_array_equal(to_np(count)[:ng], to_np(ref["grp_count"]))
        # entries past the group table are left alone
        assert np.all(to_np(first)[ng:] == SENTINEL)
    ctx.close()
    assert cnt.live == {}


def test_noalloc_refuses_beyond_scratch(H):
    """4M uniform particles need more than the 256 MiB array: ENOMEM with a
    message naming the scratch size, and the outputs keep their contents."""
    n, box = 4 << 20, 100.0
    note(f"fof3d_noalloc beyond the scratch array n={n}")
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    xyz = [torch.rand(n, generator=g, device="cuda", dtype=torch.float32) * box
           for _ in range(3)]
    zero = torch.zeros(n, dtype=torch.float32, device="cuda")
    P = H.Particles(*xyz, zero, zero, zero)
    label, perm, first, count = outputs(n, 16)
    ctx = H.Halo(H.Params(box=box, particle_mass=1e10, softening=0.01))
    with pytest.raises(H.HaloError) as e:
        ctx.fof3d_noalloc(P, label, perm, first, count)
    assert e.value.code == -2 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    for t in (label, perm, first, count):
        assert bool((t == SENTINEL).all())
    # the context still works afterwards
    small = small_catalog()
    Ps = H.Particles.from_catalog(small)
    ctx.set_params(H.params_for_catalog(small))
    bl = outputs(small.n, 1000)
    ng, nm = ctx.fof3d_noalloc(Ps, *bl)
    ref = ctx.fof3d(Ps)
    torch.cuda.synchronize()
    assert (ng, nm) == (ref["n_groups"], ref["n_members"])
    np.testing.assert_array_equal(to_np(bl[0]), to_np(ref["label"]))
