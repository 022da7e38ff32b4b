"""A workload that runs every kernel family once, for the checked-build test:
`run(api)` returns its outputs; run as a script (with BHX_LIBRARY=checked) it
saves them to the .npz named by its argument."""
import sys

import numpy as np
import torch

from paper_1912_04197_amd import ics


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run(api):
    out = {}
    # tree and walk, FP64 and FP32C, counts; one-block build and per-level build
    for prec in ("fp64", "fp32c"):
        for n in (3000, 30000):
            s = ics.plummer(n, seed=81)
            ctx = api.Context(n, leaf_size=8, precision=prec, counts=True)
            a = ctx.compute_accel(_dev(s.pos), _dev(s.mass), 0.5, softening=1e-3)
            out[f"acc_{prec}_{n}"] = a.cpu().numpy()
            out[f"cnt_{prec}_{n}"] = ctx.walk_counts(n).cpu().numpy()
    # multi-step steps: sorted state, bucket sort from the second build
    s = ics.rubble_pile(300000, seed=82)
    ctx = api.Context(s.n, leaf_size=4, precision="fp32c")
    p, v, m, e = _dev(s.pos), _dev(s.vel), _dev(s.mass), _dev(s.eps)
    a = ctx.compute_accel(p, m, 0.5, eps=e)
    ctx.step_leapfrog(p, v, m, a, 5e-4, 4, theta=0.5, eps=e)
    out["steps_pos"], out["steps_acc"] = p.cpu().numpy(), a.cpu().numpy()
    out["bucket"] = np.array([ctx.stats()["bucket_sort"]])
    # 2^20 bodies: the 1024-thread bucket sort on the second build
    s = ics.rubble_pile(1 << 20, seed=83)
    ctx = api.Context(s.n, leaf_size=4, precision="fp32c")
    for _ in range(2):
        ctx.build_tree(_dev(s.pos), _dev(s.mass), _dev(s.eps))
    out["order_2p20"] = ctx.tree().order.cpu().numpy()
    # batched scenes, graph-captured steps
    scenes = [ics.uniform_ball(int(k), seed=840 + i) for i, k in enumerate((700, 5000, 12000))]
    off = np.array([0, 700, 5700, 17700], dtype=np.int64)
    ctx = api.Context(17700, leaf_size=8, precision="fp32c", max_scenes=3, graph=True)
    p = _dev(np.vstack([sc.pos for sc in scenes]))
    m = _dev(np.concatenate([sc.mass for sc in scenes]))
    v = torch.zeros_like(p)
    a = ctx.batched_accel(off, p, m, 0.5, softening=1e-3)
    ctx.batched_step(off, p, v, m, a, 1e-3, 3, theta=0.5, softening=1e-3)
    out["batched_pos"] = p.cpu().numpy()
    # force VJP and a segment VJP with kept trees
    s = ics.uniform_ball(8000, seed=85)
    ctx = api.Context(s.n, leaf_size=16, precision="fp64", adjoint=True)
    x, v, m = _dev(s.pos), _dev(s.vel), _dev(s.mass)
    gp, gm = ctx.accel_vjp(x, m, torch.ones_like(x), theta=0.5, softening=1e-3)
    out["vjp_gp"], out["vjp_gm"] = gp.cpu().numpy(), gm.cpu().numpy()
    a = ctx.compute_accel(x, m, 0.5, softening=1e-3)
    traj = torch.empty((4, s.n, 3), dtype=torch.float64, device="cuda")
    xb, vb, ab, g = torch.ones_like(x), torch.zeros_like(x), torch.zeros_like(x), torch.zeros_like(m)
    ctx.leapfrog_vjp(x, v, a, m, 1e-3, 4, traj, xb, vb, ab, g, theta=0.5, softening=1e-3)
    out["seg_xbar"], out["seg_gm"] = xb.cpu().numpy(), g.cpu().numpy()
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    from paper_1912_04197_amd import api as A

    np.savez(sys.argv[1], **run(A))
    print("checked workload done", flush=True)
