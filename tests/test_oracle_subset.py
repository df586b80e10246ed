"""Pins of the oracle's subset linking length (Section 3.2: the nearest
neighbours of large groups are found for a random subset only): the hashed
draw against an independent SplitMix64, the off switch, and the linking
length of a large node against its definition."""
import numpy as np
import pytest

from tests.test_oracle_pins import clustered, particles

MASK = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 (Steele, Lea & Flood 2014), from its published definition."""
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def in_subset(i, n, m):
    return m <= 0 or n <= m or splitmix64(i) * n < (m << 64)


def test_subset_draw_matches_splitmix(orc):
    L = orc.lib()
    rng = np.random.default_rng(1)
    for i, n, m in zip(rng.integers(0, 2 ** 40, 3000), rng.integers(1, 10 ** 7, 3000),
                       rng.integers(1, 20000, 3000)):
        assert bool(L.orc_in_subset(int(i), int(n), int(m))) == in_subset(int(i), int(n), int(m))
    # known values of the generator (seed 0 and 1 of the reference stream)
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    assert splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_subset_rate():
    """The draw keeps each particle with probability m / n: over 2e5 indices
    the count lies within 5 sigma of the binomial mean."""
    n, m = 200000, 10000
    k = sum(in_subset(i, n, m) for i in range(n))
    assert abs(k - m) < 5 * np.sqrt(m * (1 - m / n))


def test_subset_off_and_large_bound(orc):
    """ell_subset = 0, or larger than every node, is the exact linking length."""
    pos, vel = clustered(6000, 18.0, 21, nblob=3, spread=0.5)
    P = particles(orc, pos, vel)
    lab = orc.fof3d(orc.make_params(18.0, 1e11, 0.005), P)
    a, _ = orc.refine6d(orc.make_params(18.0, 1e11, 0.005), P, lab)
    b, _ = orc.refine6d(orc.make_params(18.0, 1e11, 0.005, ell_subset=10 ** 6), P, lab)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_subset_ell_of_a_large_node(orc):
    """A level-0 node of more than m particles: ell^2 is the k-th smallest,
    k = ceil(f n_sub), of the subset's nearest-neighbour distances taken
    against every particle of the node (not only the subset)."""
    pos, vel = clustered(6000, 18.0, 21, nblob=3, spread=0.5)
    P = particles(orc, pos, vel)
    m = 300
    p = orc.make_params(18.0, 1e11, 0.005, ell_subset=m)
    lab = orc.fof3d(p, P)
    nodes, _ = orc.refine6d(p, P, lab)
    big = [k for k in range(nodes["parent"].shape[0])
           if nodes["level"][k] == 0 and nodes["count"][k] > m]
    assert big
    for k in big[:2]:
        members = np.nonzero(lab == nodes["canon"][k])[0]
        xi, _ = orc.node_normalise(p, P, members)
        dmin = orc.nn6d(xi)  # every particle against every other
        n = members.shape[0]
        pick = np.array([in_subset(int(i), n, m) for i in members])
        sub = np.sort(dmin[pick])
        kk = int(np.ceil(0.7 * sub.shape[0]))
        assert nodes["ell2"][k] == sub[kk - 1]
        # a subset-only neighbour search would give larger distances
        assert np.all(dmin[pick] <= orc.nn6d(xi[pick]))
