"""Autotuner for the size bin of the 6D neighbour search.

Nodes above `grid_min` particles take the exact tile search; the others the
symmetric all-pairs pass.  Both give the same node table, so the threshold is
purely a speed choice, and the best one depends on the catalogue (the share of
particles in giant nodes).  `tune_grid_min` times the refinement call on the
caller's particles at each candidate threshold (HIP events on the library's
stream) and returns the fastest.

    python -m paper_1110_4372_amd.autotune --config c3 --gen device
"""
from __future__ import annotations

import argparse
import json
import sys

CANDIDATES = (32768, 65536, 131072, 262144, 524288)


def choose(timings: dict) -> int:
    """The candidate with the least time; ties go to the larger threshold (the
    all-pairs pass, which needs no sample or sort)."""
    if not timings:
        raise ValueError("no timings")
    return min(timings, key=lambda g: (timings[g], -g))


def tune_grid_min(H, params, P, candidates=CANDIDATES, repeats: int = 2):
    """Times libhalo_refine6d at each candidate threshold (after one warm-up
    call per context) and returns (best threshold, {threshold: ms})."""
    import torch
    from dataclasses import replace
    ctx0 = H.Halo(params)
    fof = ctx0.fof3d(P)
    timings = {}
    for g in candidates:
        ctx = H.Halo(replace(params, grid_min=int(g)))
        ctx.refine6d(P, fof)  # warm-up: workspace and code objects
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(repeats):
            ctx.refine6d(P, fof)
        ev1.record()
        torch.cuda.synchronize()
        timings[int(g)] = ev0.elapsed_time(ev1) / repeats
    return choose(timings), timings


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", default="c2")
    ap.add_argument("--gen", default="host", choices=["host", "device"])
    ap.add_argument("--repeats", type=int, default=2)
    args = ap.parse_args()
    from paper_1110_4372_amd import halo as H
    from paper_1110_4372_amd import synth
    cat = (synth.make_catalog_device(args.config, seed=0) if args.gen == "device"
           else synth.make_catalog(args.config, seed=0))
    P = H.Particles.from_catalog(cat)
    best, t = tune_grid_min(H, H.params_for_catalog(cat), P, repeats=args.repeats)
    print(json.dumps({"config": args.config, "grid_min": best,
                      "refine_ms": {str(k): v for k, v in t.items()}}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
