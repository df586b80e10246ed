"""The autotuner: its choice rule on the CPU; on the GPU, that every
candidate threshold and pair-unit chunk gives the same hierarchy, the
potential chunk the same potential to rounding (so each choice is a speed
choice), and that the tuner picks among its candidates."""
import numpy as np
import pytest

from paper_1110_4372_amd.autotune import choose


def test_choose_fastest_and_ties():
    assert choose({65536: 3.0, 131072: 2.0, 262144: 2.5}) == 131072
    # equal times: the larger threshold (all-pairs, no sample or sort)
    assert choose({65536: 2.0, 131072: 2.0}) == 131072
    with pytest.raises(ValueError):
        choose({})


@pytest.mark.gpu
def test_tune_grid_min_same_hierarchy():
    import torch
    from paper_1110_4372_amd import halo as H
    from tests.gpu_util import note, particles_from_arrays, to_np
    from tests.test_oracle_pins import clustered
    H.load_library()
    note("autotune grid_min on a clustered set")
    pos, vel = clustered(20000, 20.0, seed=11)
    P = particles_from_arrays(pos, vel)
    params = H.Params(box=20.0, particle_mass=1e10, softening=0.01)
    best, t = H_tune(H, params, P)
    assert best in t and set(t) == {64, 1 << 30}
    tabs = []
    for g in (64, 1 << 30):
        from dataclasses import replace
        ctx = H.Halo(replace(params, grid_min=g))
        fof = ctx.fof3d(P)
        nodes, deep = ctx.refine6d(P, fof)
        torch.cuda.synchronize()
        tabs.append(({k: to_np(v) for k, v in nodes.items()}, to_np(deep)))
    for k in tabs[0][0]:
        np.testing.assert_array_equal(tabs[0][0][k], tabs[1][0][k])
    np.testing.assert_array_equal(tabs[0][1], tabs[1][1])


def H_tune(H, params, P):
    from paper_1110_4372_amd.autotune import tune_grid_min
    return tune_grid_min(H, params, P, candidates=(64, 1 << 30), repeats=1)


@pytest.mark.gpu
def test_unit_chunks_same_results():
    """The pair-unit chunks change no bit of the hierarchy and the potential
    chunk changes phi only at the rounding level (128^3 catalogue: its first
    levels hold more than the 262144 particles above which the chunks apply)."""
    import torch
    from dataclasses import replace
    from paper_1110_4372_amd import halo as H
    from paper_1110_4372_amd import synth
    from tests.gpu_util import note, to_np
    H.load_library()
    note("work-unit chunks on the 128^3 catalogue")
    cat = synth.make_catalog("c2", seed=0)
    P = H.Particles.from_catalog(cat)
    base = H.params_for_catalog(cat)
    ref = H.Halo(base).run_all(P)
    torch.cuda.synchronize()
    for kw in ({"nn_chunk": 256, "fof_chunk": 16384}, {"nn_chunk": 4096, "fof_chunk": 256},
               {"pot_chunk": 1024}, {"pot_chunk": 4096},
               {"grid_min": 2048, "kd_leaf": 4}, {"grid_min": 2048, "kd_leaf": 64}):
        out = H.Halo(replace(base, **kw)).run_all(P)
        torch.cuda.synchronize()
        for k in ref["nodes"]:
            np.testing.assert_array_equal(to_np(out["nodes"][k]), to_np(ref["nodes"][k]))
        np.testing.assert_array_equal(to_np(out["halo_of"]), to_np(ref["halo_of"]))
        pa, pb = to_np(ref["phi"]), to_np(out["phi"])
        ins = to_np(ref["halo_of"]) >= 0
        if "pot_chunk" in kw:
            np.testing.assert_allclose(pb[ins], pa[ins], rtol=1e-12, atol=0)
        else:
            np.testing.assert_array_equal(pb, pa)
        assert int((to_np(out["bound"]) != to_np(ref["bound"])).sum()) <= 2


@pytest.mark.gpu
def test_tune_picks_candidates():
    import torch
    from paper_1110_4372_amd import halo as H
    from paper_1110_4372_amd import autotune
    from tests.gpu_util import note, particles_from_arrays
    from tests.test_oracle_pins import clustered
    H.load_library()
    note("autotune every knob on a clustered set")
    pos, vel = clustered(20000, 20.0, seed=12)
    P = particles_from_arrays(pos, vel)
    params = H.Params(box=20.0, particle_mass=1e10, softening=0.01)
    p, rep = autotune.tune(H, params, P, repeats=1, grid=(64, 1 << 30), nn=(512, 1024),
                           fof_c=(1024, 2048), pot=(1024, 2048), kd_leaf=(8, 16))
    torch.cuda.synchronize()
    assert p.grid_min in (64, 1 << 30) and p.nn_chunk in (512, 1024)
    assert p.fof_chunk in (1024, 2048) and p.pot_chunk in (1024, 2048)
    assert p.kd_leaf in (8, 16)
    assert set(rep) == {"grid_min", "nn_chunk", "fof_chunk", "kd_leaf", "pot_chunk"}
