"""Helpers of the GPU tests: device catalogues and a shared libhalo context."""
import numpy as np
import torch

from paper_1110_4372_amd import halo as H


def to_np(t):
    return t.detach().cpu().numpy()


def particles_from_arrays(pos, vel):
    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return H.Particles(t(pos[:, 0]), t(pos[:, 1]), t(pos[:, 2]), t(vel[:, 0]), t(vel[:, 1]),
                       t(vel[:, 2]))


def note(msg):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
