"""The size-bin autotuner: its choice rule on the CPU, and on the GPU that
every candidate threshold gives the same hierarchy (so the choice is a pure
speed choice)."""
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
