"""Benchmark of the MI355X halo-finding path: particles/s through
FOF -> 6D refine -> assign -> unbind (-> properties), batched vs plain, 1 GPU.

A step is one pass of the whole path (libhalo_fof3d, libhalo_refine6d,
libhalo_assign, libhalo_unbind, libhalo_props) over a seeded synthetic
catalogue held in HBM.  The default workload is the 1024^3 catalogue (1 Gpc/h
box, power-law NFW hosts of 20-1e7 particles with subhaloes, 40% uniform
background, float32 positions, drawn on the GPU) in the batched form with the
mixed-precision potential and the tree potential of Appendix B (theta = 0.04)
for haloes of >= 32768 particles.  The plain form (one launch sequence per node
and halo) is timed beside the batched one on the 128^3 catalogue, where it fits
the run time.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/s through FOF→6D refine→assign→unbind; batched vs plain at 1 GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

# Fabric bytes per dispatch of the hot kernels on the 1024^3 workload, from the
# committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs (profiles/c5_hbm_traffic.md,
# scaled by a plain copy of known size: fetch x2, write x1).  Reported only for
# that workload and while the source files that set the kernel's work (its
# own, and for the 6D walks the refinement that drives them) are the ones that
# were measured.
TRAFFIC_WORKLOAD = "c5"
_GRID = ("paper_1110_4372_amd/csrc/grid6d.hip", "728bf98344d9e996b72ed78dec7ba90b521a0add")
_REFINE = ("paper_1110_4372_amd/csrc/refine6d.hip", "c8c946562558e02e125eed24496a815dbf149760")
MEASURED_TRAFFIC = {
    "k_bh_walk": {"bytes": 75.13e9,
                  "srcs": [("paper_1110_4372_amd/csrc/bh.hip",
                            "e96751a07b9187a8bc6c9148c4179cbd1b725b9a")]},
    "k_kd_walk_nn": {"bytes": 243.56e9, "srcs": [_GRID, _REFINE]},
    "k_kd_walk_fof": {"bytes": 641.79e9, "srcs": [_GRID, _REFINE]},
    "k_nn": {"bytes": 8.55e9, "srcs": [_REFINE]},
    "k_potential_f32": {"bytes": 45.63e9,
                        "srcs": [("paper_1110_4372_amd/csrc/unbind.hip",
                                  "3a13952c28ac85b7e9fa4a58347e7c9c62140c4b")]},
}


def measured_traffic(kernel, workload):
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None or workload != TRAFFIC_WORKLOAD:
        return None
    for src, sha in rec["srcs"]:
        path = os.path.join(ROOT, src)
        if not os.path.exists(path):
            return None
        if hashlib.sha1(open(path, "rb").read()).hexdigest() != sha:
            return None
    return rec["bytes"]


STAGES = ("fof3d", "refine6d", "assign", "unbind", "props")


def one_step(ctx, P, ev=None):
    """The five calls; ev (6 HIP events on the launch stream) brackets them."""
    def rec(i):
        if ev:
            ev[i].record()
        if PROGRESS and i > 0:
            import torch
            torch.cuda.synchronize()
            progress(f"  {STAGES[i - 1]} done")
    rec(0)
    fof = ctx.fof3d(P)
    rec(1)
    nodes, deepest = ctx.refine6d(P, fof)
    rec(2)
    halos, halo_of = ctx.assign(P, nodes, deepest)
    rec(3)
    unb, bound, phi = ctx.unbind(P, halos, halo_of, want_phi=False)
    rec(4)
    ctx.props(P, nodes, halos, halo_of, bound)
    rec(5)
    return fof, nodes, halos, halo_of, unb, bound


PROGRESS = False


_T0 = time.perf_counter()


def progress(msg):
    """A line on stderr after each long step (--progress): large catalogues take
    minutes per step.  Prefixed with the seconds since the start."""
    if PROGRESS:
        print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


HOT = ("k_kd_walk_nn", "k_kd_walk_fof", "k_kd_group_fof", "k_bh_walk", "k_nn", "k_fof6",
       "k_potential_f64", "k_potential_f32", "k_link", "k_mom_accum", "k_select_small",
       "k_assign_level")
WALKS = ("k_kd_walk_nn", "k_kd_walk_fof", "k_bh_walk")


def timed(ctx, P, steps, warmup, prof=False):
    """Mean wall time per step over `steps` after `warmup`, the mean device
    time of each call (HIP events on the launch stream, read after the timed
    region), and with `prof` the library's own HIP-event timing of its hot
    kernels over the same timed steps (total ms and launches per kernel) and
    the tree walks' work counts per step (from one more, untimed step in the
    walks' counting form).  With --progress each step is synchronised to
    report it."""
    import torch
    for k in range(warmup):
        one_step(ctx, P)
        if PROGRESS:
            torch.cuda.synchronize()
            progress(f"warm-up step {k + 1}/{warmup} done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    torch.cuda.synchronize()
    if prof:
        ctx.profile(True)
        ctx.profile_reset()
    t0 = time.perf_counter()
    for k in range(steps):
        out = one_step(ctx, P, evs[k])
        if PROGRESS:
            torch.cuda.synchronize()
            progress(f"timed step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    stage = {STAGES[i]: sum(e[i].elapsed_time(e[i + 1]) for e in evs) / steps
             for i in range(5)}
    kp = None
    if prof:
        kp = {"kern": {k: ctx.profile_read(k) for k in HOT}}
        # the walks' work counts come from one more step in their counting form
        # (slower, so it is not one of the timed steps); counts are per step
        ctx.profile(False, count=True)
        ctx.profile_reset()
        one_step(ctx, P)
        torch.cuda.synchronize()
        kp["work"] = {k: ctx.profile_work(k) for k in WALKS}
        ctx.profile(False)
        progress("work-counting step done")
    return sec, out, stage, kp


# the library's tree threshold when grid_min = 0: 16384 on levels of at least
# 2^23 particles, 131072 on smaller ones
GRID_MIN_LARGE, GRID_MIN_SMALL, GRID_LEVEL = 16384, 131072, 1 << 23
BH_MIN_DEFAULT = 32768     # the library's smallest tree halo when bh_min = 0
# FLOP of one evaluation, as counted for the ALU roofline:
NN_PAIR_FLOP = 17.0   # 6D distance: 6 sub, 1 mul, 5 fma
BOX_TEST_FLOP = 23.0  # point-to-box gap: per axis 2 sub + fma, 6 axes, minus the first fma's add
CELL_TEST_FLOP = 9.0  # tree-potential cell test: 3 sub, squared distance (1 mul, 2 fma), compare
TERM_FLOP = 12.0      # a term 1/sqrt(r^2 + eps^2), as counted for the direct sum


def pair_work(out, grid_min, bh_theta, bh_min):
    """Algorithmic FLOPs of one step of the all-pairs kernels.

    Nearest neighbour (k_nn): each distinct pair of a node handled by the
    all-pairs pass (not degenerate, at most grid_min particles; larger nodes
    take the tree search) once, 17 FLOP.  Potential (k_potential_*): a term
    1/sqrt(r^2 + eps^2) is 12 FLOP (3 sub, r^2 as 1 mul + 2 fma, + eps^2,
    rsqrt counted as sqrt + div, accumulate); a pair of two own particles of a
    halo is one term added to both particles' sums (13 FLOP), a pair of an own
    particle and a subhalo particle of S(h) one term added to the own
    particle's sum (12 FLOP), over the halos the direct sum handles (with the
    tree on, those with |S(h)| < bh_min)."""
    import numpy as np
    fof, nodes, halos, halo_of, unb = out[:5]
    cnt = nodes["count"].cpu().numpy().astype(np.float64)
    flags = nodes["flags"].cpu().numpy()
    if grid_min > 0:
        gmin = grid_min
    else:  # per node, from its level's particle count
        lev = nodes["level"].cpu().numpy().astype(np.int64)
        tot = np.bincount(lev, weights=cnt)
        gmin = np.where(tot[lev] >= GRID_LEVEL, GRID_MIN_LARGE, GRID_MIN_SMALL)
    on = ((flags & 2) == 0) & (cnt <= gmin)
    nn_flops = NN_PAIR_FLOP * float(np.sum(cnt[on] * (cnt[on] - 1.0) / 2.0))
    h = {k: v.cpu().numpy() for k, v in halos.items()}
    ns = unb["n_s"].cpu().numpy().astype(np.float64)
    kept = h["merged_into"] == np.arange(h["merged_into"].shape[0])
    if bh_theta > 0:
        kept &= ns < (bh_min if bh_min > 0 else BH_MIN_DEFAULT)
    nown = h["n_assigned"][kept].astype(np.float64)
    nsk = ns[kept]
    pot_flops = float(np.sum(13.0 * nown * (nown - 1.0) / 2.0 + 12.0 * nown * (nsk - nown)))
    return nn_flops, pot_flops


def roofline_report(kp, out, steps, prec_fp64, grid_min, bh_theta, bh_min, workload):
    """The roofline object of the dominant kernel of the timed steps (the hot
    kernel with the largest device time).  All-pairs kernels: algorithmic
    FLOP (pair_work) per launch over the average launch time, against the
    VALU peak of their arithmetic.  Tree searches of large nodes: the work
    the exact pruned search performs, from its device counters (box tests x 23
    + distances x 17 FLOP), against the FP32 VALU peak."""
    kern, work = kp["kern"], kp["work"]
    nn_flops, pot_flops = pair_work(out, grid_min, bh_theta, bh_min)
    pot = "k_potential_f64" if prec_fp64 else "k_potential_f32"
    figures = {
        "k_nn": (nn_flops * steps, FP32_PEAK_TFLOPS,
                 "distinct pairs of the all-pairs nodes x 17 FLOP"),
        pot: (pot_flops * steps, FP64_PEAK_TFLOPS if prec_fp64 else FP32_PEAK_TFLOPS,
              "direct-sum pairs x 12-13 FLOP"),
    }
    # work counts are per step; the kernel times cover `steps` steps
    for w in WALKS[:2]:
        tests, evals = work[w]
        figures[w] = (steps * (BOX_TEST_FLOP * tests + NN_PAIR_FLOP * evals), FP32_PEAK_TFLOPS,
                      f"counted work of the exact tree search per step: {tests:.4g} box "
                      f"tests x 23 + {evals:.4g} distances x 17 FLOP")
    cells, terms = work["k_bh_walk"]
    figures["k_bh_walk"] = (steps * (CELL_TEST_FLOP * cells + TERM_FLOP * terms),
                            FP64_PEAK_TFLOPS if prec_fp64 else FP32_PEAK_TFLOPS,
                            f"counted work of the tree potential per step, summed over "
                            f"targets: {cells:.4g} cell tests x 9 + {terms:.4g} terms x 12 "
                            f"FLOP")
    dom = max(kern, key=lambda k: kern[k][0])
    t_ms, launches = kern[dom]
    rec = {"kernel": dom, "launches": launches, "avg_launch_ms": t_ms / max(launches, 1),
           "per_step_ms": {k: v[0] / steps for k, v in kern.items()}}
    if dom in figures and t_ms > 0:
        flops, peak, what = figures[dom]
        achieved = flops / (t_ms * 1e-3) / 1e12
        rec.update({"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": measured_traffic(dom, workload),
                    "work": what})
    else:
        rec.update({"bound": "alu", "achieved": None, "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": None, "traffic": None,
                    "work": "no algorithmic count for this kernel"})
    # every candidate with a figure, for the record
    rec["others"] = {k: {"ms_per_step": kern[k][0] / steps,
                         "frac": (v[0] / (kern[k][0] * 1e-3) / 1e12 / v[1])
                         if kern[k][0] > 0 else None}
                     for k, v in figures.items() if k in kern}
    return rec


RHO_CRIT = 2.77536627e11


def extras_report(ctx, P, out, particle_mass, rho_vir):
    """libhalo_props_extra on the step's output, outside the timed step: the
    call's device time (it recomputes the basic properties too), and its pair
    kernel, the potential energy of V(h) (the k* innermost bound particles of
    S(h)), against the FP64 VALU peak: each pair of V(h) is one term
    1/sqrt(r^2 + eps^2) added once, 13 FLOP as the potential's own pairs."""
    import numpy as np
    import torch
    fof, nodes, halos, halo_of, unb, bound = out
    so = [rho_vir, 200.0 * RHO_CRIT, 500.0 * RHO_CRIT]
    ctx.props_extra(P, nodes, halos, halo_of, bound, so)  # workspace and code objects
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    pr, ex = ctx.props_extra(P, nodes, halos, halo_of, bound, so)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ctx.profile(True)
    ctx.profile_reset()
    ctx.props_extra(P, nodes, halos, halo_of, bound, so)
    torch.cuda.synchronize()
    t_pe, l_pe = ctx.profile_read("k_pair_energy")
    ctx.profile(False)
    h = {k: v.cpu().numpy() for k, v in halos.items()}
    kept = h["merged_into"] == np.arange(h["merged_into"].shape[0])
    k = np.rint(pr["mvir"].cpu().numpy()[kept] / particle_mass)
    pairs = float(np.sum(k * (k - 1.0) / 2.0))
    ach = 13.0 * pairs / (t_pe * 1e-3) / 1e12 if t_pe > 0 else 0.0
    return {"call_ms": ms, "pair_kernel": "k_pair_energy", "pair_ms": t_pe,
            "pair_launches": l_pe, "pairs": pairs, "achieved_tflops": ach,
            "peak_tflops": FP64_PEAK_TFLOPS, "frac": ach / FP64_PEAK_TFLOPS,
            "so_thresholds": so,
            "largest_halo_k": float(k.max()) if k.size else 0.0}


# Algorithmic HBM bytes of each pass (what the pass must move, not what it
# re-reads), from the per-particle figures of the method's data flow:
#   fof3d   cell keys 24 + ~5 sort passes x 24 + gather 24 + union-find and
#           labels 32 + label sort 4 x 16 + group gather 64  -> 340 B/particle
#   refine6d per particle visit of a node: moments 24 + normalised 6D write 24
#           + pair-pass reads 24 + child compaction 52        -> 124 B/visit
#   assign  per visit: read 24 + write 4; per assigned particle a radial sort
#           and scan of 64 B
#   unbind  per assigned particle: gather pos/vel 24 + halo_of 4, layout write
#           44, key sort 64, energy pass 24                   -> 160 B
#   props   per assigned particle: radial sort and scans       -> 64 B
PASS_BOUND = {"fof3d": "hbm", "refine6d": "alu (6D pair kernels)", "assign": "hbm",
              "unbind": "alu (potential)", "props": "hbm"}


def pass_report(n, out, stage):
    import numpy as np
    visits = float(out[1]["count"].double().sum().item())
    nas = float((out[3] >= 0).sum().item())
    nbytes = {"fof3d": 340.0 * n, "refine6d": 124.0 * visits,
              "assign": 28.0 * visits + 64.0 * nas, "unbind": 160.0 * nas, "props": 64.0 * nas}
    rep = {}
    for k in STAGES:
        ms = stage[k]
        gbs = nbytes[k] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        rep[k] = {"ms": ms, "bytes": nbytes[k], "GB/s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                  "bound": PASS_BOUND[k]}
    return rep


def precision_report(H, cat, P, grid_min):
    """The mixed form against the FP64 form, both on the GPU: the count of
    changed bound flags and halo validity, and the largest relative error of
    phi and of each property."""
    import numpy as np
    res = {}
    for prec in (H.PREC_FP64, H.PREC_MIXED):
        ctx = H.Halo(H.params_for_catalog(cat, mode=H.BATCHED, prec=prec, grid_min=grid_min))
        res[prec] = ctx.run_all(P)
    a, b = res[H.PREC_FP64], res[H.PREC_MIXED]
    hof = a["halo_of"].cpu().numpy()
    ins = hof >= 0
    pa, pb = a["phi"].cpu().numpy()[ins], b["phi"].cpu().numpy()[ins]
    rep = {"assigned": int(ins.sum()),
           "changed_bound": int((a["bound"] != b["bound"]).sum().item()),
           "changed_valid": int((a["unbound"]["valid"] != b["unbound"]["valid"]).sum().item()),
           "phi_max_rel_err": float(np.max(np.abs(pb - pa) / np.abs(pa))) if pa.size else 0.0}
    va = a["unbound"]["valid"].cpu().numpy().astype(bool)
    vb = b["unbound"]["valid"].cpu().numpy().astype(bool)
    both = va & vb
    errs = {}
    for k in ("px", "py", "pz", "vcx", "vcy", "vcz", "vbx", "vby", "vbz", "mvir", "rvir",
              "vmax", "voff"):
        xa = a["props"][k].cpu().numpy()[both]
        xb = b["props"][k].cpu().numpy()[both]
        den = np.maximum(np.abs(xa), 1e-300)
        errs[k] = float(np.max(np.abs(xb - xa) / den)) if xa.size else 0.0
    rep["props_max_rel_err"] = errs
    return rep


def merger_report(H, cat, P, grid_min, prec, mp=0.3):
    """The major-merger form (major_merger = MP of Table 2) against the
    single-halo pass, outside the timed steps: the unbind call's device time
    in both, the merger term's kernel, the number of merging subhaloes and
    the bound flags gained (the merger form can only add flags)."""
    import numpy as np
    import torch
    out = {}
    for m in (0.0, mp):
        ctx = H.Halo(H.params_for_catalog(cat, mode=H.BATCHED, prec=prec, grid_min=grid_min,
                                          major_merger=m))
        fof = ctx.fof3d(P)
        nodes, deep = ctx.refine6d(P, fof)
        halos, hof = ctx.assign(P, nodes, deep)
        ctx.unbind(P, halos, hof, want_phi=False)  # warm-up
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        unb, bound, _ = ctx.unbind(P, halos, hof, want_phi=False)
        e1.record()
        torch.cuda.synchronize()
        ext = ctx.profile_read("k_potential_ext_f64")
        ctx.profile(False)
        h = {k: v.cpu().numpy() for k, v in halos.items()}
        ns = unb["n_s"].cpu().numpy()
        kept = np.nonzero(h["merged_into"] == np.arange(h["merged_into"].shape[0]))[0]
        major = [s for s in kept if h["host"][s] >= 0 and m > 0 and ns[s] >= m * ns[h["host"][s]]]
        out[m] = dict(ms=e0.elapsed_time(e1), ext_ms=ext[0], bound=bound.clone(),
                      majors=len(major),
                      major_particles=int(sum(int(h["n_assigned"][s]) for s in major)))
    a, b = out[0.0], out[mp]
    return {"major_merger": mp, "merging_subhaloes": b["majors"],
            "their_particles": b["major_particles"],
            "unbind_ms_single": a["ms"], "unbind_ms_merger": b["ms"],
            "merger_kernel": "k_potential_ext_f64", "merger_kernel_ms": b["ext_ms"],
            "flags_gained": int((b["bound"].int() - a["bound"].int()).clamp(min=0).sum().item()),
            "flags_lost": int((a["bound"].int() - b["bound"].int()).clamp(min=0).sum().item())}


def changed_membership(wa, wb):
    """Particles whose halo differs between two catalogues of the same
    particles (halo labels wa, wb; -1 = none): each halo of wa is matched to
    the halo of wb holding most of its particles, and a particle changed when
    it is not in its halo's match or is assigned in one catalogue only.
    Returns (particles assigned in either, changed)."""
    import numpy as np
    wa, wb = np.asarray(wa), np.asarray(wb)
    both = (wa >= 0) & (wb >= 0)
    kept = 0
    if both.any():
        pairs, cnt = np.unique(np.stack([wa[both], wb[both]], 1), axis=0, return_counts=True)
        best = np.zeros(int(pairs[:, 0].max()) + 1, dtype=np.int64)
        np.maximum.at(best, pairs[:, 0], cnt)
        kept = int(best.sum())
    assigned = int(((wa >= 0) | (wb >= 0)).sum())
    return assigned, assigned - kept


def subset_report(H, cat, P, grid_min, prec, m=10000, steps=3):
    """The paper's subset linking length (ell_subset = 10^4, Section 3.2)
    against the exact one: step time and stage times of each (same steps
    and warm-up), node and halo counts, and the particles whose halo changed,
    halos identified by their seed leaf's smallest particle index."""
    import numpy as np
    res = {}
    for mm in (0, m):
        ctx = H.Halo(H.params_for_catalog(cat, mode=H.BATCHED, prec=prec, grid_min=grid_min,
                                          ell_subset=mm))
        sec, out, stage, _ = timed(ctx, P, steps, 1)
        fof, nodes, halos, halo_of = out[:4]
        canon = nodes["canon"].cpu().numpy().astype(np.int64)
        seed = halos["seed_node"].cpu().numpy().astype(np.int64)
        merged = halos["merged_into"].cpu().numpy().astype(np.int64)
        key = canon[seed[merged]] if seed.size else seed
        hof = halo_of.cpu().numpy().astype(np.int64)
        res[mm] = dict(ms=sec * 1e3, stage=stage, nodes=int(canon.shape[0]),
                       halos=int((merged == np.arange(merged.shape[0])).sum()),
                       who=np.where(hof >= 0, key[np.maximum(hof, 0)] if key.size else -1, -1))
    a, b = res[0], res[m]
    assigned, changed = changed_membership(a["who"], b["who"])
    return {"ell_subset": m, "ms_per_step_exact": a["ms"], "ms_per_step_subset": b["ms"],
            "refine_ms_exact": a["stage"]["refine6d"], "refine_ms_subset": b["stage"]["refine6d"],
            "nodes_exact": a["nodes"], "nodes_subset": b["nodes"],
            "halos_exact": a["halos"], "halos_subset": b["halos"],
            "assigned": assigned, "changed_membership": changed,
            "changed_fraction": changed / max(assigned, 1)}


def dense_report(H, cat, P, grid_min, prec, t=16, steps=3):
    """The paper's dense-particle FOF variant (fof_dense = 16, Section 3.1)
    against standard FOF: step and fof3d times of each (same steps and
    warm-up), FOF group counts, and the particles whose group grew (the
    variant only merges standard groups)."""
    import numpy as np
    res = {}
    for tt in (0, t):
        ctx = H.Halo(H.params_for_catalog(cat, mode=H.BATCHED, prec=prec, grid_min=grid_min,
                                          fof_dense=tt))
        sec, out, stage, _ = timed(ctx, P, steps, 1)
        lab = out[0]["label"].cpu().numpy().astype(np.int64)
        size = np.bincount(lab, minlength=lab.shape[0])[lab]
        res[tt] = dict(ms=sec * 1e3, fof_ms=stage["fof3d"], groups=int(out[0]["n_groups"]),
                       halos=int(out[2]["seed_node"].shape[0]), size=size)
    a, b = res[0], res[t]
    return {"fof_dense": t, "ms_per_step_standard": a["ms"], "ms_per_step_dense": b["ms"],
            "fof3d_ms_standard": a["fof_ms"], "fof3d_ms_dense": b["fof_ms"],
            "groups_standard": a["groups"], "groups_dense": b["groups"],
            "halo_rows_standard": a["halos"], "halo_rows_dense": b["halos"],
            "particles_in_grown_groups": int((b["size"] != a["size"]).sum())}


def tree_report(ctx, P, out, theta=0.04, bh_min=BH_MIN_DEFAULT):
    """The tree potential of Appendix B (bh_theta = 0.04, haloes with |S(h)| >=
    bh_min) against the exact direct sum, outside the timed steps, on the
    step's own halo table and context (no second workspace): unbind device
    time of each, the relative error of the tree haloes' potentials, and their
    bound flags that differ."""
    import dataclasses
    import numpy as np
    import torch
    fof, nodes, halos, hof = out[:4]
    base = ctx.params
    res = {}
    for th in (0.0, theta):
        ctx.set_params(dataclasses.replace(base, bh_theta=th, bh_min=bh_min))
        if th > 0.0:  # the exact form is warm from the timed steps
            # the library allocates outside torch's cache: return torch's idle blocks first
            torch.cuda.empty_cache()
            ctx.unbind(P, halos, hof, want_phi=False)  # warm-up: the tree's workspace
            torch.cuda.synchronize()
            progress("tree form warmed up")
        ctx.profile(True)
        ctx.profile_reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        unb, bound, phi = ctx.unbind(P, halos, hof)
        e1.record()
        torch.cuda.synchronize()
        walk = ctx.profile_read("k_bh_walk")
        ctx.profile(False)
        progress(f"unbind timed with bh_theta = {th}")
        hofn = hof.cpu().numpy()
        res[th] = dict(ms=e0.elapsed_time(e1), walk_ms=walk[0],
                       ns=unb["n_s"].cpu().numpy(), bound=bound.cpu().numpy(),
                       phi=phi.cpu().numpy())
        del unb, bound, phi
    ctx.set_params(base)
    a, b = res[0.0], res[theta]
    h = {k: v.cpu().numpy() for k, v in halos.items()}
    kept = h["merged_into"] == np.arange(h["merged_into"].shape[0])
    tree = np.nonzero(kept & (a["ns"] >= bh_min) & (h["n_assigned"] > 0))[0]
    sel = np.isin(hofn, tree)
    pa, pb = a["phi"][sel], b["phi"][sel]
    rel = np.abs(pb / pa - 1.0) if pa.size else np.zeros(1)
    ba, bb = a["bound"][sel], b["bound"][sel]
    return {"bh_theta": theta, "bh_min": bh_min, "tree_haloes": int(tree.shape[0]),
            "tree_particles": int(sel.sum()), "unbind_ms_exact": a["ms"],
            "unbind_ms_tree": b["ms"], "walk_ms": b["walk_ms"],
            "rel_err_median": float(np.median(rel)), "rel_err_max": float(rel.max()),
            "flags_differ": int((ba != bb).sum()),
            "flags_agree_fraction": float(np.mean(ba == bb)) if ba.size else 1.0}


def _oracle_job(job):
    """One serial oracle run (a worker process of cpu_baseline): the whole path
    over the particles of one sub-cube, treated as a periodic box of its own
    side with the full catalogue's linking length.  Returns (particles,
    seconds)."""
    import numpy as np
    from oracle import oracle as O
    side, ll, mass, soft, cols = job
    n = int(cols[0].shape[0])
    p = O.make_params(side, mass, soft, b=ll * n ** (1.0 / 3.0) / side)
    t0 = time.perf_counter()
    O.run_all(p, O.Particles(*[np.ascontiguousarray(c) for c in cols]))
    return n, time.perf_counter() - t0


def cpu_model():
    """The host CPU's model name (lscpu's "Model name")."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cat, workers: int = 16, target: int = 65536):
    """The CPU oracle (serial FP64 C, as it stands) on the host's cores: one
    worker process per core (at most `workers`), each running the whole path
    over one sub-cube of the catalogue of side L/k (k so that a cube holds
    about `target` particles on average) with the full catalogue's linking
    length; the cubes sit on a coarse lattice through the box and one holding
    more than twice the average is passed over (a cube through the core of one
    of the largest haloes would need hours of direct-sum unbinding).  Reports
    the particles of all cubes over the wall time of the pool."""
    import multiprocessing as mp
    import numpy as np
    from oracle import oracle as O
    O.build(force=False)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nw = max(1, min(workers, ncpu or 1))
    k = max(4, int(round((cat.n / float(target)) ** (1.0 / 3.0))))
    side = cat.box / k
    ll = 0.28 * cat.box / round(cat.n ** (1.0 / 3.0))
    mean = cat.n / float(k ** 3)
    cols_all = (cat.x, cat.y, cat.z, cat.vx, cat.vy, cat.vz)
    jobs = []
    step = max(1, k // 5)
    for ix in range(0, k, step):
        for iy in range(0, k, step):
            if len(jobs) == nw:
                break
            o = (ix * side, iy * side, 0.0)
            sel = ((cat.x >= o[0]) & (cat.x < o[0] + side) & (cat.y >= o[1])
                   & (cat.y < o[1] + side) & (cat.z < side))
            cnt = int(sel.sum())
            if cnt < 100 or cnt > 2 * mean:
                continue
            cols = []
            for a, off in zip(cols_all, (o[0], o[1], 0.0, None, None, None)):
                v = a[sel]
                v = v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)
                if off is not None:
                    v = (v - v.dtype.type(off)).astype(v.dtype)
                    v = np.clip(v, 0, np.nextafter(v.dtype.type(side), v.dtype.type(0)))
                cols.append(np.ascontiguousarray(v))
            jobs.append((side, ll, cat.particle_mass, cat.softening, cols))
    if not jobs:
        return None
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(jobs)) as pool:
        res = pool.map(_oracle_job, jobs)
    wall = time.perf_counter() - t0
    nsum = sum(r[0] for r in res)
    return dict(value=nsum / wall, unit="particles/s", cores=len(jobs), kind="oracle",
                cpu=cpu_model(), host_cpus=ncpu,
                sample=f"{len(jobs)} sub-cubes of side L/{k} ({nsum} particles, "
                       f"{min(r[0] for r in res)}-{max(r[0] for r in res)} per cube) of "
                       f"the same catalogue on a lattice through the box, full path "
                       f"fof3d..props, one serial oracle process per cube, "
                       f"{wall:.1f} s wall (per-cube {min(r[1] for r in res):.1f}-"
                       f"{max(r[1] for r in res):.1f} s)")


def make_cat(name, gen):
    from paper_1110_4372_amd import synth
    if gen == "auto":
        gen = "device" if name in ("c3", "c5") else "host"
    if gen == "device":
        return synth.make_catalog_device(name, seed=0), gen
    return synth.make_catalog(name, seed=0), gen


def workload_name(name, cat, gen):
    return (f"{name}: {cat.n} particles, box {cat.box} Mpc/h, "
            + ("8 NFW hosts + subhaloes + 30% uniform" if name == "c1" else
               "power-law NFW hosts + 5e6-particle cluster + 40% uniform" if name == "c4" else
               "power-law NFW hosts + subhaloes + 40% uniform")
            + ", seed 0" + (" (GPU-drawn)" if gen == "device" else ""))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5",
                    help="workload of the timed steps (default c5, the 1024^3 catalogue)")
    ap.add_argument("--side-config", default="c2",
                    help="workload of the plain form and of the comparisons outside the "
                         "timed steps (default c2, where the plain form fits the run time)")
    ap.add_argument("--side-steps", type=int, default=3,
                    help="timed steps of each form on the side workload")
    ap.add_argument("--no-side", action="store_true",
                    help="skip everything on the side workload")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--progress", action="store_true",
                    help="report each step and stage on stderr (synchronises after each)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other precision form and the mixed-vs-FP64 comparison")
    ap.add_argument("--prec", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-tree", action="store_true",
                    help="skip the tree-potential comparison (not part of the step)")
    ap.add_argument("--bh-theta", type=float, default=0.04,
                    help="tree potential (Appendix B) in the timed steps, for haloes of at "
                         "least --bh-min particles; 0 keeps the exact direct sum")
    ap.add_argument("--bh-min", type=int, default=BH_MIN_DEFAULT,
                    help="smallest |S(h)| that takes the tree")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense-particle FOF variant comparison (not part of the step)")
    ap.add_argument("--no-subset", action="store_true",
                    help="skip the subset-linking-length comparison (not part of the step)")
    ap.add_argument("--no-merger", action="store_true",
                    help="skip timing the major-merger unbinding (not part of the step)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip timing libhalo_props_extra (not part of the step)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration)")
    ap.add_argument("--grid-min", type=int, default=0,
                    help="nodes above this many particles use the 6D tree search "
                         "(0: the library default, or the autotuner's pick with --autotune)")
    ap.add_argument("--autotune", action="store_true",
                    help="before the timed steps, pick grid_min (unless given), the pair-unit "
                         "chunks and the potential unit by timing (paper_1110_4372_amd.autotune)")
    ap.add_argument("--gen", default="auto", choices=["auto", "host", "device"],
                    help="catalogue generator: numpy (host) or torch on the GPU (device); "
                         "auto draws the 512^3 and 1024^3 catalogues on the GPU")
    args = ap.parse_args()
    global PROGRESS
    PROGRESS = args.progress
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1110_4372_amd import halo as H

    cat, gen = make_cat(args.config, args.gen)
    P = H.Particles.from_catalog(cat)
    progress(f"catalogue {args.config}: {cat.n} particles")
    prec = H.PREC_FP64 if args.prec == "fp64" else H.PREC_MIXED
    tuned = None
    base = H.params_for_catalog(cat, mode=H.BATCHED, prec=prec, grid_min=args.grid_min,
                                bh_theta=args.bh_theta, bh_min=args.bh_min)
    if args.autotune:
        # the framework's own tuning step, before (and outside) the timed steps:
        # grid_min, the pair-unit chunks and the potential unit, each timed in turn
        from paper_1110_4372_amd import autotune
        grid = (args.grid_min,) if args.grid_min > 0 else autotune.CANDIDATES
        base, tuned = autotune.tune(H, base, P, repeats=2, grid=grid)
        args.grid_min = base.grid_min
        progress(f"autotuned: {json.dumps({k: v['pick'] for k, v in tuned.items()})}")
    ctx = H.Halo(base)
    sec, out, stage, kp = timed(ctx, P, args.steps, args.warmup, prof=True)
    roofline = roofline_report(kp, out, args.steps, prec == H.PREC_FP64, args.grid_min,
                               args.bh_theta, args.bh_min, args.config)
    passes = pass_report(cat.n, out, stage)
    counts = {"n_groups": int(out[0]["n_groups"]), "n_nodes": int(out[1]["parent"].shape[0]),
              "n_halos": int(out[2]["seed_node"].shape[0])}
    del out
    progress("timed steps done")

    names = {H.PREC_FP64: "fp64", H.PREC_MIXED: "mixed"}
    forms = {f"batched_{names[prec]}": {"workload": args.config, "value": cat.n / sec,
                                          "ms_per_step": sec * 1e3, "stage_ms": stage}}
    plain = precision = extras = merger = subset = dense = tree = None
    side = None
    if not args.no_side:
        # the forms and comparisons outside the timed steps, on the side workload
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        scat, sgen = make_cat(args.side_config, "auto")
        SP = H.Particles.from_catalog(scat)
        side = workload_name(args.side_config, scat, sgen)
        ss = max(1, args.side_steps)
        sctx = None
        for pr in (prec, H.PREC_MIXED if prec == H.PREC_FP64 else H.PREC_FP64):
            if args.no_forms and pr != prec:
                continue
            c2 = H.Halo(H.params_for_catalog(scat, mode=H.BATCHED, prec=pr,
                                             grid_min=args.grid_min, bh_theta=args.bh_theta,
                                             bh_min=args.bh_min))
            s2, o2, st2, _ = timed(c2, SP, ss, 1)
            forms[f"side_batched_{names[pr]}"] = {"workload": args.side_config,
                                                  "value": scat.n / s2,
                                                  "ms_per_step": s2 * 1e3, "stage_ms": st2}
            if pr == prec:
                sctx, sout = c2, o2
            else:
                del c2, o2
        progress("side workload: batched forms timed")
        if not args.no_plain:
            for pr in ((prec,) if args.no_forms else (prec, H.PREC_MIXED if prec == H.PREC_FP64
                                                      else H.PREC_FP64)):
                ctxp = H.Halo(H.params_for_catalog(scat, mode=H.PLAIN, prec=pr,
                                                   grid_min=args.grid_min,
                                                   bh_theta=args.bh_theta, bh_min=args.bh_min))
                sp, _, stp, _ = timed(ctxp, SP, 1, 1)
                forms[f"side_plain_{names[pr]}"] = {"workload": args.side_config,
                                                    "value": scat.n / sp,
                                                    "ms_per_step": sp * 1e3, "stage_ms": stp}
                if pr == prec:
                    bt = forms[f"side_batched_{names[pr]}"]["ms_per_step"]
                    plain = {"workload": args.side_config, "value": scat.n / sp,
                             "ms_per_step": sp * 1e3, "batched_ms_per_step": bt,
                             "batched_over_plain": sp * 1e3 / bt}
                del ctxp
            progress("side workload: plain forms timed")
        if not args.no_forms:
            precision = precision_report(H, scat, SP, args.grid_min)
        if not args.no_extras:
            extras = extras_report(sctx, SP, sout, scat.particle_mass,
                                   H.params_for_catalog(scat).rho_vir)
            progress("additional properties timed")
        if not args.no_merger:
            merger = merger_report(H, scat, SP, args.grid_min, prec)
            progress("major-merger form timed")
        if not args.no_subset:
            subset = subset_report(H, scat, SP, args.grid_min, prec)
            progress("subset linking length timed")
        if not args.no_dense:
            dense = dense_report(H, scat, SP, args.grid_min, prec)
            progress("dense-particle FOF variant timed")
        if not args.no_tree:
            tree = tree_report(sctx, SP, sout, theta=args.bh_theta or 0.04,
                               bh_min=args.bh_min)
            progress("tree potential timed")
        del sctx, sout, SP, scat

    if args.copy_probe:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    cpu = None if args.no_cpu else cpu_baseline(cat)
    if cpu is not None:
        progress("CPU oracle baseline done")
    rec = {
        "metric": METRIC, "value": cat.n / sec, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if prec == H.PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload_name(args.config, cat, gen),
                   "form": "batched", "potential": args.prec,
                   "bh_theta": args.bh_theta,
                   "bh_min": args.bh_min if args.bh_theta > 0 else None,
                   "grid_min": args.grid_min, "autotune": tuned, **counts,
                   "side_workload": side},
        "stage_ms": stage,
        "passes": passes,
        "plain": plain,
        "forms": forms,
        "precision": precision,
        "extras": extras,
        "merger": merger,
        "subset": subset,
        "fof_dense": dense,
        "tree": tree,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
