"""Major-merger unbinding on the GPU (Section 3.5.3, MP of Table 2) against
the oracle: constructed two-clump mergers and the 32^3 catalogue, FP64 and
mixed potentials, with the same bar as the single-halo pass (flags outside
the rounding band, phi, properties)."""
import numpy as np
import pytest

from tests.gpu_util import note, particles_from_arrays, to_np
from tests.test_gpu_unbind_props import compare_props_agreeing, compare_unbind
from tests.test_oracle_merger import BOX, EPS, M_PART, merger
from tests.test_oracle_pins import particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1110_4372_amd import halo
    halo.load_library()
    return halo


def n_major(o, mp):
    h, ns = o["halos"], o["unbound"]["n_s"]
    kept = np.nonzero(h["merged_into"] == np.arange(h["merged_into"].shape[0]))[0]
    return sum(1 for s in kept if h["host"][s] >= 0 and ns[s] >= mp * ns[h["host"][s]])


@pytest.mark.parametrize("seed,prec,f64", [(1, 0, True), (3, 0, False), (5, 1, True),
                                           (7, 1, False)])
def test_merger_matches_oracle(H, orc, seed, prec, f64):
    note(f"major merger seed={seed} prec={prec} f64={f64}")
    pos, vel = merger(seed)
    if not f64:
        pos = pos.astype(np.float32)
        pos[pos >= np.float32(BOX)] = 0
    mp = 0.3
    p = orc.make_params(BOX, M_PART, EPS, major_merger=mp)
    P = particles(orc, pos, vel)
    o = orc.run_all(p, P)
    assert n_major(o, mp) == 1
    ctx = H.Halo(H.Params(box=BOX, particle_mass=M_PART, softening=EPS, prec=prec,
                          major_merger=mp))
    g = ctx.run_all(particles_from_arrays(pos, vel))
    tol, rtol = (1e-9, 1e-9) if prec == 0 else (1e-4, 2e-5)
    amb, changed = compare_unbind(g["unbound"], g["bound"], g["phi"], o, P, tol, rtol)
    rows = compare_props_agreeing(g, o)
    print(f"ambiguous={amb} changed={changed} property rows={rows}")


def test_merger_off_is_the_single_halo_pass(H, c1):
    """major_merger = 0 and a ratio above 1 (no host can qualify) give the
    single-halo pass bit for bit."""
    note("major merger off == single-halo pass (c1)")
    P = H.Particles.from_catalog(c1)
    outs = [H.Halo(H.params_for_catalog(c1, major_merger=mp)).run_all(P) for mp in (0.0, 1.5)]
    np.testing.assert_array_equal(to_np(outs[0]["bound"]), to_np(outs[1]["bound"]))
    np.testing.assert_array_equal(to_np(outs[0]["phi"]), to_np(outs[1]["phi"]))


@pytest.mark.parametrize("prec", [0, 1])
def test_merger_c1(H, orc, c1, prec):
    """The 32^3 catalogue with MP = 0.3 (Table 2's default) and, to reach more
    pairs, MP = 0.05."""
    for mp in (0.3, 0.05):
        note(f"major merger c1 prec={prec} mp={mp}")
        p = orc.params_of(c1, major_merger=mp)
        o = orc.run_all(p, orc.Particles.of(c1))
        g = H.Halo(H.params_for_catalog(c1, prec=prec, major_merger=mp)).run_all(
            H.Particles.from_catalog(c1))
        tol, rtol = (1e-9, 1e-9) if prec == 0 else (1e-4, 2e-5)
        amb, changed = compare_unbind(g["unbound"], g["bound"], g["phi"], o, c1, tol, rtol)
        rows = compare_props_agreeing(g, o)
        print(f"mp={mp} majors={n_major(o, mp)} ambiguous={amb} changed={changed} "
              f"property rows={rows}")


def test_merger_bad_parameter(H, c1):
    with pytest.raises(H.HaloError):
        H.Halo(H.params_for_catalog(c1, major_merger=-0.1))


def test_merger_plain_equals_batched(H):
    """The merger term's fixed-point sums do not depend on the launch form."""
    note("major merger plain == batched")
    pos, vel = merger(5)
    P = particles_from_arrays(pos, vel)
    outs = [H.Halo(H.Params(box=BOX, particle_mass=M_PART, softening=EPS, mode=mode,
                            major_merger=0.3)).run_all(P) for mode in (1, 0)]
    np.testing.assert_array_equal(to_np(outs[0]["phi"]), to_np(outs[1]["phi"]))
    np.testing.assert_array_equal(to_np(outs[0]["bound"]), to_np(outs[1]["bound"]))
