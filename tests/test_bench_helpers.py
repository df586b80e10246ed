"""Host-side helpers of the benchmark (CPU only)."""
import numpy as np

import bench


def test_changed_membership():
    # identical up to relabelling: nothing changed
    a = np.array([0, 0, 0, 1, 1, -1, 2, 2])
    b = np.array([5, 5, 5, 9, 9, -1, 7, 7])
    assert bench.changed_membership(a, b) == (7, 0)
    # one particle moves, one is dropped, one is newly assigned
    b2 = np.array([5, 5, 9, 9, 9, 3, 7, -1])
    assigned, changed = bench.changed_membership(a, b2)
    assert assigned == 8
    # halo 0 -> best match 5 (2 of 3): 1 changed; halo 1 -> 9 (2): 0; halo 2 -> 7 (1 of 1
    # assigned in both); particle 5 (new) and particle 7 (dropped) changed
    assert changed == 3
    assert bench.changed_membership(np.full(4, -1), np.full(4, -1)) == (0, 0)
