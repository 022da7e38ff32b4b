#!/usr/bin/env python3
"""Headline benchmark: one-GPU Barnes-Hut leapfrog on a 2^20-body rubble pile.

Workload: N = 1,048,576 rubble-pile aggregation cloud (uniform ball of radius
1, lognormal radii with median 1e-3 and log-sigma 0.3, mass ~ r^3 summing to 1,
isotropic velocities at 0.1x virial plus solid-body spin 0.2 about z), G = 1,
per-body softening = radius, theta = 0.5, FP32 pair terms with FP64 state,
kick-drift-kick steps of dt = 5e-4. The leaf size (bodies per bucket) is left
open by the workload; the default, 4, is the fastest step of a measured sweep
over 1..64 (the paper's own leaves hold one body), and the same step at leaf
16 is reported beside it. A step is one whole hot path: tree
rebuild (box, keys, sort, gather, build, moments), walk, and both kicks.

Prints one JSON line: steps/s (value), Ginteractions/s, the direct N^2 and
plain-FP64 comparisons on the same GPU, the force error against the FP64
direct sum, the walk kernel's roofline fraction (HIP events on the launch
stream), and the FP64 CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "steps/s & Ginteractions/s at N=1M, theta=0.5 vs direct N^2; force rel. err vs FP64"
FLOPS_PER_INTERACTION = 20  # conventional count for one softened monopole/pair term
PEAK_FP32_TFLOPS = 157.3    # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6     # MI355X published FP64 vector peak
NODE_BYTES = 56             # NodeInfo 16 + NodeMom 32 + node eps^2 8
PEAK_HBM_TBS = 8.0           # MI355X published HBM3E bandwidth
# Algorithmic HBM bytes per body of each phase of a step of a multi-step call
# (reads and writes the phase cannot avoid, once each), plus the node tables
# (NODE_BYTES per node) written once by the build and read once by the walk.
BYTES_PER_BODY = {
    # first kick, drift and box over the sorted state (body 32, v 24, a 24,
    # eps^2 8, caller index 4 read; body, v, eps^2, index written: 160) + keys
    # (positions read, key and index written) 36 + sort (one read and one
    # write of key and index) 24 + gather (index, body, v, eps^2, caller index
    # read; body, v, eps^2, caller index written) 140 + octree (keys searched)
    # 8 + moments (bodies and eps^2 read) 40
    "build": 408,
    # target body and eps^2 40, index 4, acceleration written 24
    "walk": 68,
    # second kick (v, a read; v written)
    "integrate": 72,
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def walk_traffic(leaf):
    """HBM bytes per walk launch from the committed rocprofv3 counter runs, or
    None when the walk kernel's source has changed since they were taken or
    they were taken at another leaf size."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "profiles", "walk_counters.json")) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, "paper_1912_04197_amd", "csrc", "walk.hip"), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    ok = rec.get("walk_source_sha256_16") == h and rec.get("leaf") == leaf
    return rec["hbm_bytes_per_launch"] if ok else None


def _sync_time(fn):
    import torch

    torch.cuda.synchronize()
    t = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3


def bench_batched(args, n_scenes=256, steps=10, theta=0.5, dt=1e-3, soft=1e-3):
    """Many independent scenes at once: 256 uniform balls with N log-uniform in
    [1024, 65536], FP32C, KDK steps of every scene captured into one graph per
    call, with the bucket and walk-group sizes picked by the autotuner; against
    the same steps run scene by scene and against FP64."""
    import numpy as np
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context, autotune

    scenes = ics.batched_scenes(n_scenes, seed=44)
    ns = np.array([sc.n for sc in scenes])
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    n = int(off[-1])
    log(f"batched: {n_scenes} scenes, {n} bodies")
    pos0 = torch.from_numpy(np.vstack([sc.pos for sc in scenes])).cuda()
    vel0 = torch.from_numpy(np.vstack([sc.vel for sc in scenes])).cuda()
    mass = torch.from_numpy(np.concatenate([sc.mass for sc in scenes])).cuda()
    t = time.perf_counter()
    leaf, group, tune_ms = autotune(off, pos0, vel0, mass, theta=theta, dt=dt, softening=soft,
                                    steps=3)
    tune_s = time.perf_counter() - t
    log(f"autotune: leaf {leaf}, group {group} ({tune_ms:.2f} ms/step, {tune_s:.1f} s)")

    def graph_steps(lf, gr, prec):
        ctx = Context(n, leaf_size=lf, precision=prec, walk_group=gr, max_scenes=n_scenes,
                      graph=True)
        p, v = pos0.clone(), vel0.clone()
        a = ctx.batched_accel(off, p, mass, theta, softening=soft)
        ctx.batched_step(off, p, v, mass, a, dt, steps, theta=theta, softening=soft)
        ms = _sync_time(lambda: ctx.batched_step(off, p, v, mass, a, dt, steps, theta=theta,
                                                 softening=soft, sync=False)) / steps
        ctx.close()
        return ms

    ms_tuned = graph_steps(leaf, group, "fp32c")
    ms_default = graph_steps(16, 64, "fp32c")
    ms_fp64 = graph_steps(leaf, group, "fp64")
    cctx = Context(n, leaf_size=leaf, precision="fp32c", counts=True, max_scenes=n_scenes,
                   walk_group=group)
    cctx.batched_accel(off, pos0, mass, theta, softening=soft)
    st = cctx.stats()
    inter = st["nodes_accepted"] + st["leaf_pairs"]
    cctx.close()

    # the same steps issued scene by scene from one context (no graph)
    one = Context(int(ns.max()), leaf_size=leaf, precision="fp32c", walk_group=group)
    p, v = pos0.clone(), vel0.clone()
    a = torch.empty_like(p)
    views = [(p[off[k]:off[k + 1]], v[off[k]:off[k + 1]], mass[off[k]:off[k + 1]],
              a[off[k]:off[k + 1]]) for k in range(n_scenes)]
    for pk, vk, mk, ak in views:
        one.compute_accel(pk, mk, theta, softening=soft, out=ak, sync=False)

    def loop():
        for pk, vk, mk, ak in views:
            one.step_leapfrog(pk, vk, mk, ak, dt, 1, theta=theta, softening=soft, sync=False)

    loop()
    ms_loop = _sync_time(loop)
    one.close()
    log(f"batched: graph {ms_tuned:.2f} ms/step (default 16/64 {ms_default:.2f}, fp64 "
        f"{ms_fp64:.2f}), scene-by-scene {ms_loop:.2f} ms/step")
    return {
        "workload": f"{n_scenes} uniform balls, N log-uniform in [1024, 65536], {n} bodies, "
                    f"theta={theta} eps={soft} dt={dt}, FP32C, {steps} KDK steps per graph call",
        "bodies": n,
        "autotune": {"leaf": leaf, "walk_group": group, "ms_per_step": round(tune_ms, 4),
                     "seconds": round(tune_s, 2)},
        "ms_per_step": round(ms_tuned, 4),
        "body_steps_per_s": round(n / (ms_tuned * 1e-3), 1),
        "ginteractions_per_s": round(inter / (ms_tuned * 1e-3) / 1e9, 3),
        "interactions_per_body": round(inter / n, 1),
        "ms_per_step_leaf16_group64": round(ms_default, 4),
        "ms_per_step_fp64": round(ms_fp64, 4),
        "ms_per_step_scene_by_scene": round(ms_loop, 4),
        "speedup_vs_scene_by_scene": round(ms_loop / ms_tuned, 2),
    }


def bench_adjoint(n=65536, nsteps=200, every=20, theta=0.5, dt=1e-3, soft=1e-3, leaf=2):
    """Differentiable rollout: forward KDK steps with checkpoints, then the
    hand-written adjoint back to (x0, v0, m), against the forward alone (each
    the median of 3 runs after a warm-up); the tree gradient against the FP64
    direct-sum gradient, and FP32C (FP32C forward and FP32C tree VJPs)
    against FP64. The `_keep` entries keep every step's positions (24 B per
    body and step) so that the backward pass recomputes nothing. Leaf 2: the
    fastest forward+backward of leaves 1-16 on this workload (the VJP's terms
    are dearer than the forward's, so fewer interactions pay more)."""
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context
    from paper_1912_04197_amd.autograd import rollout

    s = ics.uniform_ball(n, seed=55)
    xt = torch.from_numpy(ics.perturbed_target(s.pos, seed=56)).cuda()
    out = {"workload": f"uniform ball N={n} theta={theta} eps={soft} dt={dt}, leaf {leaf}, "
                       f"{nsteps} KDK steps, checkpoint every {every}, loss sum |x_T - x*|^2"}
    grads = {}
    for label, prec, th, keep in (("fp32c", "fp32c", theta, False), ("fp64", "fp64", theta, False),
                                  ("direct_fp64", "fp64", -1.0, False),
                                  ("fp32c_keep", "fp32c", theta, True),
                                  ("fp64_keep", "fp64", theta, True)):
        ctx = Context(n, leaf_size=leaf, precision=prec, adjoint=True)
        x0 = torch.from_numpy(s.pos).cuda().requires_grad_(True)
        v0 = torch.from_numpy(s.vel).cuda().requires_grad_(True)
        m = torch.from_numpy(s.mass).cuda().requires_grad_(True)

        def fwd():
            with torch.no_grad():
                rollout(x0, v0, m, ctx, dt, nsteps, theta=th, softening=soft,
                        checkpoint_every=every, keep_positions=keep)

        def fwd_bwd():
            for t in (x0, v0, m):
                t.grad = None
            x, _ = rollout(x0, v0, m, ctx, dt, nsteps, theta=th, softening=soft,
                           checkpoint_every=every, keep_positions=keep)
            ((x - xt) ** 2).sum().backward()

        fwd_bwd()  # warm-up: first-touch of the workspaces and kernels
        torch.cuda.reset_peak_memory_stats()
        t_fb = sorted(_sync_time(fwd_bwd) for _ in range(3))[1]  # median of 3
        t_f = sorted(_sync_time(fwd) for _ in range(3))[1]
        peak = torch.cuda.max_memory_allocated()
        grads[label] = [t.grad.detach().clone() for t in (x0, v0, m)]
        ctx.close()
        out[label] = {"forward_ms": round(t_f, 2), "forward_backward_ms": round(t_fb, 2),
                      "backward_over_forward": round((t_fb - t_f) / t_f, 2),
                      "torch_peak_mib": round(peak / 2**20, 1)}
        log(f"adjoint {label}: forward {t_f:.1f} ms, forward+backward {t_fb:.1f} ms")

    def gap(a, b):
        return [round(float(torch.linalg.norm(x - y) / torch.linalg.norm(y)), 8)
                for x, y in zip(a, b)]

    out["rel_l2_gap_x0_v0_m"] = {
        "tree_fp64_vs_direct_fp64": gap(grads["fp64"], grads["direct_fp64"]),
        "tree_fp32c_vs_tree_fp64": gap(grads["fp32c"], grads["fp64"]),
        "fp32c_keep_vs_fp32c": gap(grads["fp32c_keep"], grads["fp32c"]),
        "fp64_keep_vs_fp64": gap(grads["fp64_keep"], grads["fp64"]),
    }
    return out


def bench_plummer(n=131072, nsteps=500, every=100, dt=1e-3, soft=1e-3, thetas=(0.3, 0.5, 0.7)):
    """Plummer sphere, leaf 16, FP32C forces: steps/s per theta, the force error
    against the FP64 direct sum every 100 steps, the FP32C-vs-FP64 tree gap and
    the relative energy drift over the run."""
    import numpy as np
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    sc = ics.plummer(n, seed=22)
    mass = torch.from_numpy(sc.mass).cuda()
    c32 = Context(n, leaf_size=16, precision="fp32c", graph=True)
    c64 = Context(n, leaf_size=16, precision="fp64")
    out = {"workload": f"Plummer N={n} a=1 M=1, leaf 16, eps={soft}, {nsteps} KDK steps of "
                       f"dt={dt}, FP32C forces, FP64 state"}

    def err(a, ref):
        e = (torch.linalg.norm(a - ref, dim=1) / torch.linalg.norm(ref, dim=1)).cpu().numpy()
        return {"rms": float(np.sqrt(np.mean(e ** 2))), "p99": float(np.quantile(e, 0.99))}

    def energy(p, v):
        d = c64.diagnostics(p, v, mass, softening=soft)
        return d[0] + d[1]

    for th in thetas:
        p = torch.from_numpy(sc.pos).cuda()
        v = torch.from_numpy(sc.vel).cuda()
        a = c32.compute_accel(p, mass, th, softening=soft)
        e0 = energy(p, v)
        errs, ms = [], 0.0
        for k in range(0, nsteps + 1, every):
            ref = c64.compute_accel_direct(p, mass, softening=soft)
            t32 = c32.compute_accel(p, mass, th, softening=soft)
            t64 = c64.compute_accel(p, mass, th, softening=soft)
            errs.append({"step": k, "tree_fp32c": err(t32, ref),
                         "fp32c_vs_fp64_tree": err(t32, t64)})
            if k < nsteps:
                ms += _sync_time(lambda: c32.step_leapfrog(p, v, mass, a, dt, every, theta=th,
                                                           softening=soft, sync=False))
        e1 = energy(p, v)
        out[f"theta_{th}"] = {"steps_per_s": round(nsteps / (ms * 1e-3), 1),
                              "ms_per_step": round(ms / nsteps, 4),
                              "energy_rel_drift": float((e1 - e0) / abs(e0)),
                              "force_error": errs}
        log(f"plummer theta {th}: {ms / nsteps:.3f} ms/step, dE/E {(e1 - e0) / abs(e0):.2e}")
    c32.close()
    c64.close()
    return out


def bench_cold_collapse(n=1000, thetas=(0.1, 0.25, 0.5, 0.75), soft=2.0, dt=5e-3, every=10,
                        t_max=16.0):
    """The paper's accuracy experiment: N bodies at rest, uniform in a cube of
    side 2, pulse through one contraction and re-expansion; every body's
    position under the tree is compared with the direct sum's through
    e_i(t) = |r_BH - r_N2| / |r_N2| in percent. The softening (2, the cube's
    side) makes the collapse a nearly reversible pulsation, as the paper
    describes it: the end of the contraction is the direct run's minimum of the
    half-mass radius (about its COM), and the pulsation ends at the next
    maximum, where the bodies are nearly at rest again. Reported per theta:
    the largest e_i over bodies at the end of the contraction, its maximum over
    the pulsation and when, measured from the barycentre (frame-free) and in a
    frame whose origin is a corner of the cube (domain [0, 2]^3, positions as a
    simulation of a cubic domain would hold them). Semi-implicit Euler with
    gravity every substep, FP64, one-body leaves."""
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    sc = ics.uniform_cube(n, seed=12)
    nsamp = int(round(t_max / dt / every))
    m = torch.from_numpy(sc.mass).cuda()

    def run(theta, diag=False):
        ctx = Context(n, leaf_size=1, precision="fp64")
        p = torch.from_numpy(sc.pos).cuda()
        v = torch.zeros_like(p)
        a = (ctx.compute_accel(p, m, theta, softening=soft) if theta >= 0
             else ctx.compute_accel_direct(p, m, softening=soft))
        e0 = ctx.diagnostics(p, v, m, softening=soft) if diag else None
        snaps, ekin, energy = [], [], []
        for _ in range(nsamp):
            ctx.step_euler(p, v, m, a, dt, every, theta=theta, softening=soft, sync=False)
            snaps.append(p.clone())
            if diag:
                d = ctx.diagnostics(p, v, m, softening=soft)
                ekin.append(d[0])
                energy.append(d[0] + d[1])
        ctx.sync()
        ctx.close()
        return snaps, e0, ekin, energy

    t0 = time.perf_counter()
    ref, e0, ekin, energy = run(-1.0, diag=True)
    com = torch.from_numpy((sc.mass[:, None] * sc.pos).sum(0) / sc.mass.sum()).cuda()
    rhalf = [float(torch.linalg.norm(x - com, dim=1).median()) for x in ref]
    r0 = float(torch.linalg.norm(torch.from_numpy(sc.pos).cuda() - com, dim=1).median())
    kmin = min(range(len(rhalf)), key=rhalf.__getitem__)
    kend = max(range(kmin, len(rhalf)), key=rhalf.__getitem__)
    E0 = e0[0] + e0[1]
    out = {"workload": f"uniform cube N={n} side 2 at rest, eps={soft}, semi-implicit Euler "
                       f"dt={dt} (gravity every substep), leaf 1, FP64; positions sampled every "
                       f"{every} substeps",
           "direct_run": {
               "t_end_of_contraction": round((kmin + 1) * every * dt, 3),
               "t_end_of_pulsation": round((kend + 1) * every * dt, 3),
               "half_mass_radius_initial": round(r0, 4),
               "half_mass_radius_min": round(rhalf[kmin], 4),
               "half_mass_radius_end": round(rhalf[kend], 4),
               "ekin_end_over_max": round(ekin[kend] / max(ekin[: kend + 1]), 5),
               "energy_rel_error_max": float(max(abs(e - E0) for e in energy[: kend + 1]) / abs(E0)),
               "half_mass_radius_curve": [round(rhalf[k], 4) for k in
                                          range(0, kend + 1, max(1, (kend + 1) // 12))],
           }}
    corner = torch.ones(3, dtype=torch.float64, device="cuda")  # cube [-1, 1]^3 -> [0, 2]^3
    for th in thetas:
        snaps = run(th)[0][: kend + 1]
        e_com = torch.stack([torch.linalg.norm(a - b, dim=1) / torch.linalg.norm(b - com, dim=1)
                             for a, b in zip(snaps, ref)]) * 100
        e_box = torch.stack([torch.linalg.norm(a - b, dim=1) / torch.linalg.norm(b + corner, dim=1)
                             for a, b in zip(snaps, ref)]) * 100
        rec = {}
        for name, e in (("barycentric", e_com), ("corner_frame", e_box)):
            mx = e.max(dim=1).values
            k = int(mx.argmax())
            rec[name] = {"max_pct_end_of_contraction": round(float(mx[kmin]), 6),
                         "max_pct_over_pulsation": round(float(mx[k]), 6),
                         "at_fraction_of_pulsation": round((k + 1) / len(mx), 3)}
        out[f"theta_{th}"] = rec
    for name in ("barycentric", "corner_frame"):
        ends = [out[f"theta_{th}"][name]["max_pct_end_of_contraction"] for th in thetas]
        out[f"ratio_theta_{thetas[-1]}_over_{thetas[0]}_{name}"] = round(ends[-1] / ends[0], 1)
        out[f"error_increases_with_theta_{name}"] = all(x < y for x, y in zip(ends, ends[1:]))
    out["paper_context"] = ("paper (N=1000, GeForce 940M): max error about 0.3 % at theta 0.75 at the "
                            "end of contraction, about two orders of magnitude between theta 0.1 "
                            "and 0.75; ICs, units and softening not stated")
    log(f"cold collapse: end of contraction t={out['direct_run']['t_end_of_contraction']}, "
        f"max error {[out[f'theta_{th}']['corner_frame']['max_pct_end_of_contraction'] for th in thetas]} % "
        f"(corner frame) ({time.perf_counter() - t0:.1f} s)")
    return out


def bench_quadrupole(n=131072, thetas=(0.3, 0.5, 0.7, 0.9), soft=1e-3):
    """Error against cost of quadrupole nodes: Plummer sphere, leaf 16, FP32C;
    per theta the time of one force evaluation (tree rebuilt) and the RMS / p99
    relative force error against the FP64 direct sum, monopole vs quadrupole."""
    import numpy as np
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    sc = ics.plummer(n, seed=22)
    p = torch.from_numpy(sc.pos).cuda()
    m = torch.from_numpy(sc.mass).cuda()
    c64 = Context(n, precision="fp64")
    ref = c64.compute_accel_direct(p, m, softening=soft)
    c64.close()
    rn = torch.linalg.norm(ref, dim=1)
    out = {"workload": f"Plummer N={n}, leaf 16, eps={soft}, FP32C, one force evaluation"}
    for quad in (False, True):
        ctx = Context(n, leaf_size=16, precision="fp32c", quad=quad)
        for th in thetas:
            a = ctx.compute_accel(p, m, th, softening=soft)
            reps = 10
            ms = _sync_time(lambda: [ctx.compute_accel(p, m, th, softening=soft, sync=False)
                                     for _ in range(reps)]) / reps
            e = (torch.linalg.norm(a - ref, dim=1) / rn).cpu().numpy()
            out[f"{'quad' if quad else 'mono'}_theta_{th}"] = {
                "ms": round(ms, 4), "rms": float(np.sqrt(np.mean(e ** 2))),
                "p99": float(np.quantile(e, 0.99))}
        ctx.close()
    log("quadrupole: " + ", ".join(f"{k} {v['ms']:.2f} ms rms {v['rms']:.2e}"
                                   for k, v in out.items() if k != "workload"))
    return out


def bench_contacts(n=1 << 20, scale=4.0, n_small=20000):
    """Aggregate identification: contact graph of the rubble pile's spheres
    (radii scaled so that contacts exist) and its connected components; the
    O(N^2) oracle is timed beside it on a smaller pile."""
    import numpy as np
    import torch

    import oracle
    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    out = {}
    for label, size in (("large", n), ("small", n_small)):
        sc = ics.rubble_pile(size, seed=33)
        r = scale * sc.eps
        ctx = Context(size)
        P, M, R = (torch.from_numpy(a).cuda() for a in (sc.pos, sc.mass, r))
        lab, nc, na = ctx.contact_components(P, M, R)
        reps = 5
        ms = _sync_time(lambda: [ctx.contact_components(P, M, R) for _ in range(reps)]) / reps
        ctx.close()
        sizes = np.bincount(lab.cpu().numpy())
        row = {"n": size, "ms": round(ms, 3), "contacts": nc, "aggregates": na,
               "largest_aggregate": int(sizes.max())}
        if label == "small":
            t0 = time.perf_counter()
            lab_ref, nc_ref, na_ref = oracle.contact_components(sc.pos, r)
            row["oracle_s"] = round(time.perf_counter() - t0, 3)
            row["matches_oracle"] = bool(nc_ref == nc and na_ref == na and
                                         np.array_equal(lab_ref, lab.cpu().numpy()))
        out[label] = row
    out["workload"] = (f"rubble pile (seed 33) spheres of radius {scale} x eps, contact iff "
                       "|x_i - x_j| <= r_i + r_j; tree build + contact search + union-find")
    log(f"contacts: {out['large']}")
    return out


def bench_crossover(ns=(1000, 2048, 4000, 16000, 64000), thetas=(0.25, 0.5, 0.75), soft=1e-3):
    """The paper's timing experiment on this GPU: one FP64 force evaluation
    (tree rebuilt) against the FP64 direct sum on uniform random cubes."""
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    rows = []
    for n in ns:
        sc = ics.uniform_cube(n, seed=12)
        p = torch.from_numpy(sc.pos).cuda()
        m = torch.from_numpy(sc.mass).cuda()
        ctx = Context(n, leaf_size=1, precision="fp64")
        ctx.compute_accel_direct(p, m, softening=soft)
        reps = 5
        t_dir = _sync_time(lambda: [ctx.compute_accel_direct(p, m, softening=soft, sync=False)
                                    for _ in range(reps)]) / reps
        row = {"n": n, "direct_ms": round(t_dir, 4)}
        for th in thetas:
            ctx.compute_accel(p, m, th, softening=soft)
            t = _sync_time(lambda: [ctx.compute_accel(p, m, th, softening=soft, sync=False)
                                    for _ in range(reps)]) / reps
            row[f"tree_ms_theta_{th}"] = round(t, 4)
            row[f"speedup_theta_{th}"] = round(t_dir / t, 2)
        ctx.close()
        rows.append(row)
        log(f"crossover n={n}: {row}")
    return {"workload": "uniform random cube, leaf 1 (the paper's one-body leaves), eps "
                        f"{soft}, FP64, one force evaluation with the tree rebuilt",
            "rows": rows}


def ceilings(walk_tflops):
    """Achievable ceilings measured on this GPU beside the datasheet ones: HBM
    by a device-to-device copy of 1 GiB (bytes read + written, best of 5),
    vector FP32 (non-packed) and FP64 by the library's FMA probe."""
    import torch

    from paper_1912_04197_amd.api import probe_fma

    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    copy_tbs = 2 * n * 8 / (best * 1e-3) / 1e12
    del src, dst
    fp32 = probe_fma("fp32")
    fp64 = probe_fma("fp64")
    log(f"ceilings: copy {copy_tbs:.2f} TB/s, FMA fp32 {fp32:.1f} fp64 {fp64:.1f} TFLOP/s")
    return {
        "hbm_copy_tb_s": round(copy_tbs, 3),
        "hbm_datasheet_tb_s": PEAK_HBM_TBS,
        "fp32_fma_tflops": round(fp32, 2),
        "fp32_datasheet_tflops": PEAK_FP32_TFLOPS,
        "fp32_datasheet_nonpacked_tflops": round(PEAK_FP32_TFLOPS / 2, 2),
        "fp64_fma_tflops": round(fp64, 2),
        "fp64_datasheet_tflops": 78.6,
        "walk_frac_of_measured_fp32": round(walk_tflops / fp32, 4) if fp32 > 0 else None,
        "how": "copy: torch device-to-device copy of 1 GiB, best of 5; FMA: 8 independent "
               "chains per lane, 8 wavefronts per SIMD on every CU (bh_probe_fma)",
    }


def step_phases(n, nnodes, interactions, ms_step, build_ms, walk_ms):
    """Per-phase roofline of one step: each phase's floor is its algorithmic
    HBM bytes at the HBM peak or, for the walk, its flops at the FP32 vector
    peak if that is longer; the step fraction is the sum of the floors over
    the measured step time. Build and walk are HIP-event times (the build
    includes the first kick and the drift, fused into its bounding-box pass);
    `integrate` is the rest of the step (the second kick, the gaps between
    launches, and the call's packing and unpacking of the state spread over
    its steps)."""
    out = {}
    floor_total = 0.0
    measured = {"build": build_ms, "walk": walk_ms,
                "integrate": max(ms_step - build_ms - walk_ms, 1e-6)}
    for ph, ms in measured.items():
        nbytes = BYTES_PER_BODY[ph] * n + (NODE_BYTES * nnodes if ph != "integrate" else 0)
        floor_ms = nbytes / (PEAK_HBM_TBS * 1e12) * 1e3
        bound = "hbm"
        if ph == "walk":
            alu_ms = FLOPS_PER_INTERACTION * interactions / (PEAK_FP32_TFLOPS * 1e12) * 1e3
            if alu_ms > floor_ms:
                floor_ms, bound = alu_ms, "alu"
        floor_total += floor_ms
        out[ph] = {"ms": round(ms, 4), "bound": bound, "floor_ms": round(floor_ms, 4),
                   "frac": round(floor_ms / ms, 4),
                   "algorithmic_bytes": nbytes,
                   "achieved_gb_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    out["step_floor_ms"] = round(floor_total, 4)
    out["step_roofline_frac"] = round(floor_total / ms_step, 4)
    return out


def bench_leaf(args, leaf, pos0, vel0, mass, eps):
    """The headline FP32C step at another leaf size: step and walk times, the
    interactions it does and its walk's roofline fraction."""
    import torch

    from paper_1912_04197_amd.api import Context

    n, theta, dt = args.n, args.theta, args.dt
    ctx = Context(n, leaf_size=leaf, precision="fp32c", timing=True, walk_group=args.walk_group)
    pos, vel = pos0.clone(), vel0.clone()
    acc = ctx.compute_accel(pos, mass, theta, eps=eps)
    steps = max(5, min(20, args.steps))
    ctx.step_leapfrog(pos, vel, mass, acc, dt, 2, theta=theta, eps=eps, sync=False)
    ctx.sync()
    ctx.timing_reset()
    ms = _sync_time(lambda: ctx.step_leapfrog(pos, vel, mass, acc, dt, steps, theta=theta, eps=eps,
                                              sync=False)) / steps
    ctx.sync()
    st = ctx.stats()
    walk_ms = st["walk_ms"] / max(st["timed_evals"], 1)
    ctx.close()
    cctx = Context(n, leaf_size=leaf, precision="fp32c", counts=True)
    cctx.compute_accel(pos0, mass, theta, eps=eps)
    s2 = cctx.stats()
    inter = s2["nodes_accepted"] + s2["leaf_pairs"]
    cctx.close()
    ach = FLOPS_PER_INTERACTION * inter / (walk_ms * 1e-3) / 1e12
    log(f"leaf {leaf}: {ms:.3f} ms/step, walk {walk_ms:.3f} ms, {inter / n:.1f} interactions/body")
    return {"ms_per_step": round(ms, 4), "steps_per_s": round(1e3 / ms, 2),
            "walk_ms": round(walk_ms, 4), "interactions_per_body": round(inter / n, 1),
            "ginteractions_per_s_walk": round(inter / (walk_ms * 1e-3) / 1e9, 2),
            "walk_roofline_frac": round(ach / PEAK_FP32_TFLOPS, 4)}


def cpu_oracle_beside(args, scene, result):
    """The FP64 CPU oracle timed beside the GPU on the other workloads, each on a
    bounded sample (what was timed is stated per entry): a one-thread figure
    for the headline walk, the Plummer sphere per theta, sampled batched
    scenes and the rollout gradient at 256 and 4096 bodies."""
    import numpy as np

    import oracle
    from paper_1912_04197_amd import ics

    out = {"threads": oracle.num_threads()}
    n, theta, leaf = args.n, args.theta, args.leaf
    rng = np.random.default_rng(7)

    def timed(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t

    # headline walk on 65536 sampled targets, all threads and one thread
    targets = np.sort(rng.choice(n, min(n, 65536), replace=False))
    tree = oracle.Tree(scene.pos, scene.mass, scene.eps, leaf=leaf)
    t_all = timed(lambda: tree.accel(theta, targets=targets))
    nthr = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t_one = timed(lambda: tree.accel(theta, targets=targets))
    finally:
        oracle.set_num_threads(nthr)
    scale = n / len(targets)
    out["headline_walk"] = {
        "sample": f"tree walk of {len(targets)} sampled bodies of the 2^20 rubble pile (leaf {leaf}), "
                  "built tree excluded; full-walk seconds extrapolated x N / sample",
        "seconds_all_threads": round(t_all, 3), "seconds_one_thread": round(t_one, 3),
        "full_walk_s_extrapolated_all_threads": round(t_all * scale, 2),
        "full_walk_s_extrapolated_one_thread": round(t_one * scale, 2),
        "gpu_walk_ms": result.get("walk_ms"),
    }
    # Plummer sphere (131072, leaf 16): the step-0 tree force per theta, full N;
    # the direct sum on 1024 sampled targets
    pl = ics.plummer(131072, seed=22)
    pl_out = {"sample": "oracle tree force at step 0 on all 131072 bodies per theta (leaf 16, "
                        "eps 1e-3); direct sum on 1024 sampled targets, extrapolated x N / 1024"}
    gpu_pl = result.get("plummer", {})
    for th in (0.3, 0.5, 0.7):
        t = timed(lambda: oracle.bh(pl.pos, pl.mass, th, softening=1e-3, leaf=16))
        g = gpu_pl.get(f"theta_{th}", {}).get("ms_per_step")
        pl_out[f"theta_{th}"] = {"oracle_s": round(t, 3), "gpu_step_ms": g,
                                 "gpu_speedup": round(t * 1e3 / g, 1) if g else None}
    tg = np.sort(rng.choice(131072, 1024, replace=False))
    t = timed(lambda: oracle.direct(pl.pos, pl.mass, softening=1e-3, targets=tg))
    pl_out["direct_s_extrapolated"] = round(t * 131072 / 1024, 2)
    out["plummer_131072"] = pl_out
    # batched: 8 of the 256 scenes, the tree force at the tuned leaf
    scenes = ics.batched_scenes(256, seed=44)
    pick = rng.choice(256, 8, replace=False)
    tuned = result.get("batched", {}).get("autotune", {}).get("leaf", 4)
    t = sum(timed(lambda sc=scenes[k]: oracle.bh(sc.pos, sc.mass, 0.5, softening=1e-3, leaf=tuned))
            for k in pick)
    nb = sum(scenes[k].n for k in pick)
    out["batched_8_scenes"] = {"sample": f"oracle tree force of 8 sampled scenes ({nb} bodies, "
                                         f"leaf {tuned})", "oracle_s": round(t, 3),
                               "oracle_us_per_body": round(t * 1e6 / nb, 3)}
    # rollout gradient (tree theta 0.5, leaf 16) at 256 and 4096 bodies, 20 steps
    ro = {"sample": "oracle rollout gradient (forward KDK steps, then one tree VJP per step), "
                    "20 steps of dt 1e-3, eps 1e-3, theta 0.5, leaf 16"}
    for nn in (256, 4096):
        b = ics.uniform_ball(nn, seed=55)
        xb = ics.perturbed_target(b.pos, seed=56) - b.pos
        t = timed(lambda: oracle.rollout_grad(b.pos, b.vel, b.mass, 1e-3, 20, xb, np.zeros_like(xb),
                                              softening=1e-3, theta=0.5, leaf=16))
        ro[f"n_{nn}_ms_per_step"] = round(t * 1e3 / 20, 3)
    out["rollout_gradient"] = ro
    log(f"cpu oracle beside: one-thread walk {t_one:.2f} s on {len(targets)} bodies")
    return out


def direct_only(args):
    """One FP32C and one FP64 direct N^2 evaluation on the headline bodies, for
    profiler runs of the direct kernel."""
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    n = args.n
    scene = ics.rubble_pile(n, seed=33)
    pos = torch.from_numpy(scene.pos).cuda()
    mass = torch.from_numpy(scene.mass).cuda()
    eps = torch.from_numpy(scene.eps).cuda()
    out = {"workload": f"rubble_pile N={n} eps=radius, direct N^2", "n": n}
    for prec in ("fp32c", "fp64"):
        ctx = Context(n, precision=prec)
        ms = _sync_time(lambda: ctx.compute_accel_direct(pos, mass, eps=eps))
        out[f"{prec}_ms"] = round(ms, 3)
        out[f"{prec}_ginteractions_per_s"] = round(n * (n - 1) / (ms * 1e-3) / 1e9, 2)
        ctx.close()
        log(f"direct {prec}: {ms:.1f} ms")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 20, help="bodies (default 2^20)")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--leaf", type=int, default=4,
                    help="bodies per leaf bucket (4: the fastest step of a measured sweep)")
    ap.add_argument("--dt", type=float, default=5e-4)
    ap.add_argument("--walk-group", type=int, default=0,
                    help="target bodies per wavefront in the walk (16/32/64; 0 = library default)")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="full KDK steps the CPU oracle runs for its baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps (for profiler runs)")
    ap.add_argument("--markers", action="store_true",
                    help="roctx ranges around the headline context's phases (for marker traces)")
    ap.add_argument("--direct-only", action="store_true",
                    help="only one FP32C and one FP64 direct evaluation (for profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (to scale HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE={world}) is not "
              "supported: the library runs the whole step on a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1912_04197_amd import ics
    from paper_1912_04197_amd.api import Context

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}))
        return
    if args.direct_only:
        direct_only(args)
        return
    n, theta, leaf, dt = args.n, args.theta, args.leaf, args.dt
    log(f"generating rubble pile n={n}")
    scene = ics.rubble_pile(n, seed=33)
    pos0 = torch.from_numpy(scene.pos).cuda()
    vel0 = torch.from_numpy(scene.vel).cuda()
    mass = torch.from_numpy(scene.mass).cuda()
    eps = torch.from_numpy(scene.eps).cuda()

    def run_steps(ctx, k, pos, vel, acc):
        # one call of k steps: the library keeps the state in Morton order
        # between them (tree rebuilt every step)
        if k > 0:
            ctx.step_leapfrog(pos, vel, mass, acc, dt, k, theta=theta, eps=eps, sync=False)

    # ---- headline: FP32C tree leapfrog
    ctx = Context(n, leaf_size=leaf, precision="fp32c", timing=True, walk_group=args.walk_group,
                  markers=args.markers)
    pos, vel = pos0.clone(), vel0.clone()
    acc = ctx.compute_accel(pos, mass, theta, eps=eps)
    log(f"warmup {args.warmup} steps")
    run_steps(ctx, args.warmup, pos, vel, acc)
    ctx.sync()
    ctx.timing_reset()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    run_steps(ctx, args.steps, pos, vel, acc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    st = ctx.stats()
    ms_step = (t1 - t0) * 1e3 / args.steps
    walk_ms = st["walk_ms"] / max(st["timed_evals"], 1)
    build_ms = st["build_ms"] / max(st["timed_evals"], 1)
    log(f"{ms_step:.3f} ms/step (walk {walk_ms:.3f} ms, build {build_ms:.3f} ms, "
        f"{st['timed_evals']} timed evaluations)")
    # the same steps as one-step calls: the state is read from and written to
    # the caller's arrays (caller order) around every step
    p1, v1, a1 = pos.clone(), vel.clone(), acc.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.step_leapfrog(p1, v1, mass, a1, dt, 1, theta=theta, eps=eps, sync=False)
    torch.cuda.synchronize()
    ms_one = (time.perf_counter() - t0) * 1e3 / args.steps
    del p1, v1, a1
    log(f"one-step calls: {ms_one:.3f} ms/step")

    # interactions per step: counted at the first and the last timed state
    cctx = Context(n, leaf_size=leaf, precision="fp32c", counts=True)
    inter = []
    for p in (pos0, pos):
        cctx.compute_accel(p, mass, theta, eps=eps)
        s2 = cctx.stats()
        inter.append(s2["nodes_accepted"] + s2["leaf_pairs"])
    interactions = 0.5 * (inter[0] + inter[1])
    nnodes = cctx.stats()["nnodes"]
    cctx.close()
    gint_step = interactions / (ms_step * 1e-3) / 1e9
    gint_walk = interactions / (walk_ms * 1e-3) / 1e9
    achieved = FLOPS_PER_INTERACTION * interactions / (walk_ms * 1e-3) / 1e12

    result = {
        "metric": METRIC,
        "value": round(1e3 / ms_step, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair terms, f64 state",
        "data": "synthetic",
        "config": {
            "workload": f"rubble_pile N={n} theta={theta} leaf={leaf} eps=radius dt={dt} "
                        "kick-drift-kick, tree rebuilt every step",
            "n": n, "theta": theta, "leaf": leaf, "dt": dt, "precision": "fp32c",
            "walk_group": args.walk_group or "default",
        },
        "ginteractions_per_s": round(gint_step, 3),
        "ginteractions_per_s_walk": round(gint_walk, 3),
        "interactions_per_step": int(interactions),
        "interactions_per_body": round(interactions / n, 1),
        "nodes": nnodes,
        "walk_ms": round(walk_ms, 4),
        "build_ms": round(build_ms, 4),
        "ms_per_step_one_step_calls": round(ms_one, 4),
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": walk_traffic(leaf),
            "kernel": "k_walk<fp32c, per-body eps>",
            "flops_per_interaction": FLOPS_PER_INTERACTION,
        },
        "phases": step_phases(n, nnodes, interactions, ms_step, build_ms, walk_ms),
        "ceilings": ceilings(achieved),
    }

    if not args.no_extras:
        if leaf != 16:
            result["leaf16"] = bench_leaf(args, 16, pos0, vel0, mass, eps)
        # plain FP64 form of the same step
        c64 = Context(n, leaf_size=leaf, precision="fp64", timing=True, walk_group=args.walk_group)
        p64, v64 = pos0.clone(), vel0.clone()
        a64 = c64.compute_accel(p64, mass, theta, eps=eps)
        k64 = max(3, min(10, args.steps))
        run_steps(c64, 1, p64, v64, a64)
        c64.sync()
        c64.timing_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(c64, k64, p64, v64, a64)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / k64
        c64.sync()
        st64 = c64.stats()
        walk64 = st64["walk_ms"] / max(st64["timed_evals"], 1)
        ach64 = FLOPS_PER_INTERACTION * interactions / (walk64 * 1e-3) / 1e12
        result["roofline_fp64"] = {
            "bound": "alu", "achieved": round(ach64, 3), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach64 / PEAK_FP64_TFLOPS, 4), "traffic": None,
            "kernel": "k_walk<fp64, per-body eps>", "walk_ms": round(walk64, 4),
            "flops_per_interaction": FLOPS_PER_INTERACTION,
        }
        log(f"fp64 tree step {ms64:.3f} ms (walk {walk64:.3f} ms)")

        # direct N^2 on the same GPU, and the force error against FP64 direct
        def timed(fn):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            return out, (time.perf_counter() - t) * 1e3

        a_dir64, ms_dir64 = timed(lambda: c64.compute_accel_direct(pos0, mass, eps=eps))
        a_dir32, ms_dir32 = timed(lambda: ctx.compute_accel_direct(pos0, mass, eps=eps))
        a_tree32 = ctx.compute_accel(pos0, mass, theta, eps=eps)
        a_tree64 = c64.compute_accel(pos0, mass, theta, eps=eps)
        log(f"direct fp32c {ms_dir32:.1f} ms, fp64 {ms_dir64:.1f} ms")

        def err_stats(a, ref):
            e = (torch.linalg.norm(a - ref, dim=1) / torch.linalg.norm(ref, dim=1)).cpu().numpy()
            return {"rms": float(np.sqrt(np.mean(e ** 2))), "p99": float(np.quantile(e, 0.99)),
                    "max": float(e.max())}

        result["comparisons"] = {
            "fp64_tree_ms_per_step": round(ms64, 4),
            "speedup_vs_fp64_tree": round(ms64 / ms_step, 3),
            "direct_fp32c_ms": round(ms_dir32, 3),
            "direct_fp64_ms": round(ms_dir64, 3),
            "direct_fp32c_ginteractions_per_s": round(n * (n - 1) / (ms_dir32 * 1e-3) / 1e9, 2),
            "speedup_tree_step_vs_direct_fp32c_force": round(ms_dir32 / ms_step, 2),
            "force_rel_err_vs_fp64_direct": {
                "tree_fp32c": err_stats(a_tree32, a_dir64),
                "tree_fp64": err_stats(a_tree64, a_dir64),
                "direct_fp32c": err_stats(a_dir32, a_dir64),
            },
            "force_rel_err_fp32c_vs_fp64_tree": err_stats(a_tree32, a_tree64),
        }
        c64.close()

        # the same FP32C step captured once in a HIP graph and replayed
        cg = Context(n, leaf_size=leaf, precision="fp32c", walk_group=args.walk_group, graph=True)
        pg, vg = pos0.clone(), vel0.clone()
        ag = cg.compute_accel(pg, mass, theta, eps=eps)
        run_steps(cg, 2, pg, vg, ag)
        cg.sync()
        kg = max(5, min(50, args.steps))
        ms_graph = _sync_time(lambda: run_steps(cg, kg, pg, vg, ag)) / kg
        cg.sync()
        cg.close()
        result["comparisons"]["graph_ms_per_step"] = round(ms_graph, 4)
        log(f"graph-captured step {ms_graph:.3f} ms")

        # the paper's preferred stepper, semi-implicit Euler, with gravity every
        # substep and (two-rate scheme) every 10th substep
        ce = Context(n, leaf_size=leaf, precision="fp32c", walk_group=args.walk_group)
        pe, ve = pos0.clone(), vel0.clone()
        ae = ce.compute_accel(pe, mass, theta, eps=eps)
        ce.step_euler(pe, ve, mass, ae, dt, 2, every=1, theta=theta, eps=eps)
        ke = max(5, min(50, args.steps))
        ms_e1 = _sync_time(lambda: ce.step_euler(pe, ve, mass, ae, dt, ke, every=1, theta=theta,
                                                 eps=eps, sync=False)) / ke
        ms_e10 = _sync_time(lambda: ce.step_euler(pe, ve, mass, ae, dt, 10 * ke, every=10,
                                                  theta=theta, eps=eps, sync=False)) / (10 * ke)
        ce.close()
        result["euler"] = {
            "workload": f"rubble_pile N={n} theta={theta} leaf={leaf} eps=radius, semi-implicit "
                        f"Euler substeps of dt={dt}, FP32C forces",
            "ms_per_substep_gravity_every_substep": round(ms_e1, 4),
            "ms_per_substep_gravity_every_10": round(ms_e10, 4),
            "substeps_per_s_gravity_every_10": round(1e3 / ms_e10, 1),
        }
        log(f"euler: {ms_e1:.3f} ms/substep (gravity each), {ms_e10:.3f} (gravity every 10th)")
        result["batched"] = bench_batched(args)
        result["adjoint"] = bench_adjoint()
        result["plummer"] = bench_plummer()
        result["crossover"] = bench_crossover()
        result["cold_collapse"] = bench_cold_collapse()
        result["quadrupole"] = bench_quadrupole()
        result["contacts"] = bench_contacts()

    if not args.no_cpu:
        import oracle

        k = max(1, args.cpu_steps)
        log(f"cpu oracle: initial force, then {k} timed KDK steps of all {n} bodies")
        acc0 = oracle.bh(scene.pos, scene.mass, theta, eps=scene.eps, leaf=leaf)[0]
        t0 = time.perf_counter()
        oracle.leapfrog(scene.pos, scene.vel, scene.mass, dt, k, eps=scene.eps, theta=theta,
                        leaf=leaf, acc=acc0)
        step_s = (time.perf_counter() - t0) / k
        result["cpu_baseline"] = {
            "value": round(1.0 / step_s, 6),
            "unit": "steps/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"FP64 oracle: {k} full kick-drift-kick steps of the 2^20-body rubble pile "
                       f"(tree rebuilt and every body walked each step; {step_s:.2f} s a step), "
                       "timed after one untimed force evaluation"),
            "cpu_model": cpu_model(),
            "gpu_speedup": round(step_s * 1e3 / ms_step, 1),
        }
        log(f"cpu oracle {step_s:.2f} s per step on {oracle.num_threads()} threads")
        result["cpu_oracle_beside"] = cpu_oracle_beside(args, scene, result)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
