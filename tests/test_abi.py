"""The C ABI library loads and exports every entry point of include/libhalo.h."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "libhalo.h")).read()
    return sorted(set(re.findall(r"\b(libhalo_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1110_4372_amd import build, halo
    if not os.path.exists(halo.LIB_PATH):
        build.build()
    return ctypes.CDLL(halo.LIB_PATH)


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"


def test_binding_lists_every_symbol():
    from paper_1110_4372_amd import halo
    assert sorted(halo.SYMBOLS) == declared_symbols()


def test_version_and_bad_args_without_gpu(lib):
    lib.libhalo_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.libhalo_version()
    # null arguments are rejected before any device call
    assert lib.libhalo_ctx_create(None, 0, None, None, None, None) == -1
    assert lib.libhalo_ctx_destroy(None) == -1
    assert lib.libhalo_fof3d(None, 10, 0, None, None, None, None, None, None, None, 0,
                             None, None, None) == -1


def test_params_struct_matches_header():
    """ctypes mirror of libhalo_params has the header's field order."""
    from paper_1110_4372_amd import halo
    src = open(os.path.join(ROOT, "include", "libhalo.h")).read()
    body = src[src.index("typedef struct {\n  double box;"):src.index("} libhalo_params;")]
    fields = re.findall(r"^\s*(?:double|int32_t)\s+([A-Za-z_0-9]+);", body, re.M)
    assert fields == [f for f, _ in halo.CParams._fields_]


def test_product_path_does_not_import_oracle():
    """The binding and build modules never touch the oracle."""
    for f in ("halo.py", "build.py", "synth.py", "__init__.py"):
        src = open(os.path.join(ROOT, "paper_1110_4372_amd", f)).read()
        assert not re.search(r"^\s*(from|import)\s+oracle", src, re.M), f


def test_library_allocates_no_device_memory():
    """The workspace comes only from the caller's allocator callback: no HIP
    source of the library calls the runtime's device allocators."""
    import glob
    pat = re.compile(r"\bhip(Malloc|MallocManaged|MallocAsync|ExtMallocWithFlags|Free|FreeAsync)"
                     r"\s*\(")
    srcs = glob.glob(os.path.join(ROOT, "paper_1110_4372_amd", "csrc", "*"))
    assert srcs
    for f in srcs:
        code = re.sub(r"//[^\n]*|/\*.*?\*/", "", open(f).read(), flags=re.S)
        assert not pat.search(code), f"{f} allocates device memory itself"


def test_ctx_create_requires_allocator(lib):
    """A null alloc or free callback is rejected before any device call."""
    from paper_1110_4372_amd import halo
    p = halo.Params(box=10.0, particle_mass=1.0, softening=0.01).c()
    h = ctypes.c_void_p()
    lib.libhalo_ctx_create.argtypes = [ctypes.POINTER(halo.CParams), ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]
    assert lib.libhalo_ctx_create(ctypes.byref(p), 0, None, None, None, ctypes.byref(h)) == -1
    assert not h.value


@pytest.mark.parametrize("field,value", [
    ("nn_chunk", 100), ("nn_chunk", 8192), ("fof_chunk", 300), ("fof_chunk", 32768),
    ("pot_chunk", 3000), ("kd_leaf", 2), ("kd_leaf", 65), ("bh_leaf", 3), ("bh_leaf", 100),
    ("grid_min", 32), ("bh_theta", -1.0), ("f", 1.5), ("nn_bracket", float("nan")),
    ("nn_bracket", float("inf"))])
def test_ctx_create_rejects_bad_parameters(lib, field, value):
    """Out-of-range parameters are EINVAL before any device call (a counting
    allocator sees no request)."""
    import dataclasses
    from paper_1110_4372_amd import halo
    calls = []
    alloc = halo.ALLOC_FN(lambda n, user, stream: calls.append(n) or None)
    free = halo.FREE_FN(lambda ptr, user, stream: None)
    p = dataclasses.replace(halo.Params(box=10.0, particle_mass=1.0, softening=0.01),
                            **{field: value}).c()
    h = ctypes.c_void_p()
    lib.libhalo_ctx_create.argtypes = [ctypes.POINTER(halo.CParams), ctypes.c_int,
                                       halo.ALLOC_FN, halo.FREE_FN, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]
    assert lib.libhalo_ctx_create(ctypes.byref(p), 0, alloc, free, None, ctypes.byref(h)) == -1
    assert not h.value and calls == []
