"""Autotuner of the batched form's size bin and work-unit sizes.

Every knob here is a speed choice:
  grid_min   nodes above it take the exact tree search of the 6D neighbours,
             the others the symmetric all-pairs pass (same node table);
  nn_chunk   smallest j-chunk of an all-pairs nearest-neighbour unit on large
             levels (same distances);
  fof_chunk  j particles of an all-pairs 6D FOF unit on large levels (same
             components);
  pot_chunk  j particles of a direct-sum potential unit, one of the compiled
             instantiations (the partial sums are grouped differently: phi
             agrees to rounding);
  kd_leaf    most points of a leaf of the 6D search trees (same node table);
  bh_leaf    most particles of a leaf of the tree potential (with bh_theta > 0;
             other cells are accepted, phi stays within the theta bound).
The best values depend on the catalogue (the share of particles in giant
nodes and haloes).  `tune` times the refinement call (HIP events on the
library's stream) at each candidate of the refinement knobs in turn, keeping
the best of each, then the unbinding call at each potential knob, and returns
the picks with every timing.

    python -m paper_1110_4372_amd.autotune --config c3
"""
from __future__ import annotations

import argparse
import json
import sys

CANDIDATES = (8192, 16384, 32768, 65536, 131072)
NN_CHUNKS = (512, 1024, 2048)
FOF_CHUNKS = (1024, 2048, 4096)
POT_CHUNKS = (1024, 2048, 4096)
KD_LEAVES = (8, 16, 32)
BH_LEAVES = (8, 16, 32)


def choose(timings: dict) -> int:
    """The candidate with the least time; ties go to the larger value (the
    all-pairs pass, which needs no tree build; the fewer, larger units)."""
    if not timings:
        raise ValueError("no timings")
    return min(timings, key=lambda g: (timings[g], -g))


def _time(call, repeats):
    import torch
    call()  # warm-up: workspace and code objects
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(repeats):
        call()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / repeats


def tune_knob(H, params, P, knob, candidates, stage_inputs, repeats: int = 2):
    """Times one stage at each candidate value of `knob` (a Params field) and
    returns (best value, {value: ms}).  stage_inputs(ctx) -> the stage call."""
    from dataclasses import replace
    timings = {}
    for g in candidates:
        ctx = H.Halo(replace(params, **{knob: int(g)}))
        try:
            timings[int(g)] = _time(stage_inputs(ctx), repeats)
        finally:
            ctx.close()  # one workspace at a time: at 1024^3 two do not fit
        print(f"autotune {knob}={int(g)}: {timings[int(g)]:.1f} ms", file=sys.stderr, flush=True)
    return choose(timings), timings


def tune_grid_min(H, params, P, candidates=CANDIDATES, repeats: int = 2):
    """Times libhalo_refine6d at each candidate threshold (after one warm-up
    call per context) and returns (best threshold, {threshold: ms})."""
    fof = H.Halo(params).fof3d(P)
    return tune_knob(H, params, P, "grid_min", candidates,
                     lambda ctx: (lambda: ctx.refine6d(P, fof)), repeats)


def tune(H, params, P, repeats: int = 2, grid=CANDIDATES, nn=NN_CHUNKS, fof_c=FOF_CHUNKS,
         pot=POT_CHUNKS, kd_leaf=KD_LEAVES, bh_leaf=BH_LEAVES):
    """Coordinate search over grid_min, nn_chunk, fof_chunk, kd_leaf
    (refinement time), pot_chunk and, with the tree potential on, bh_leaf
    (unbinding time).  Returns (tuned Params, report)."""
    from dataclasses import replace
    ctx0 = H.Halo(params)
    fof = ctx0.fof3d(P)
    ctx0.close()  # the outputs are the caller's; its workspace is not needed
    refine = lambda ctx: (lambda: ctx.refine6d(P, fof))  # noqa: E731
    report = {}
    p = params
    for knob, cands in (("grid_min", grid), ("nn_chunk", nn), ("fof_chunk", fof_c),
                        ("kd_leaf", kd_leaf)):
        best, t = tune_knob(H, p, P, knob, cands, refine, repeats)
        p = replace(p, **{knob: best})
        report[knob] = {"pick": best, "refine_ms": {str(k): v for k, v in t.items()}}
    ctx1 = H.Halo(p)
    nodes, deep = ctx1.refine6d(P, fof)
    halos, hof = ctx1.assign(P, nodes, deep)
    ctx1.close()
    unbind = lambda ctx: (lambda: ctx.unbind(P, halos, hof, want_phi=False))  # noqa: E731
    knobs = [("pot_chunk", pot)] + ([("bh_leaf", bh_leaf)] if p.bh_theta > 0 else [])
    for knob, cands in knobs:
        best, t = tune_knob(H, p, P, knob, cands, unbind, repeats)
        p = replace(p, **{knob: best})
        report[knob] = {"pick": best, "unbind_ms": {str(k): v for k, v in t.items()}}
    return p, report


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", default="c2")
    ap.add_argument("--gen", default="auto", choices=["auto", "host", "device"])
    ap.add_argument("--prec", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--repeats", type=int, default=2)
    args = ap.parse_args()
    from paper_1110_4372_amd import halo as H
    from paper_1110_4372_amd import synth
    gen = args.gen if args.gen != "auto" else ("device" if args.config in ("c3", "c5")
                                               else "host")
    cat = (synth.make_catalog_device(args.config, seed=0) if gen == "device"
           else synth.make_catalog(args.config, seed=0))
    P = H.Particles.from_catalog(cat)
    prec = H.PREC_FP64 if args.prec == "fp64" else H.PREC_MIXED
    _, rep = tune(H, H.params_for_catalog(cat, prec=prec), P, repeats=args.repeats)
    print(json.dumps({"config": args.config, **rep}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
