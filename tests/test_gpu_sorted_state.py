"""Multi-step calls keep the state in Morton order between their steps.

Bars: a call of k steps equals k one-step calls (caller-order state around
every step) bit for bit - positions, velocities, accelerations, per-body walk
counts and the exported tree's order and node set - when no two bodies share
a cell of the finest grid; with coincident bodies (whose order inside a leaf
may differ) the steps stay within the FP64 leapfrog bar of the oracle's
rollout; bad input is latched as on the caller-order path.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04197_amd import ics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_1912_04197_amd import api as A

    return A


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision,per_body_eps", [("fp64", False), ("fp32c", True),
                                                    ("fp32c", False)])
def test_multi_step_call_equals_one_step_calls(api, precision, per_body_eps):
    s = ics.uniform_ball(30000, seed=51)
    rng = np.random.default_rng(51)
    vel = 0.3 * rng.standard_normal(s.pos.shape)
    eps = _dev(rng.uniform(1e-3, 3e-3, s.n)) if per_body_eps else None
    out = []
    for k_per_call in (5, 1):
        ctx = api.Context(s.n, leaf_size=4, precision=precision, counts=True)
        p, v, m = _dev(s.pos), _dev(vel), _dev(s.mass)
        a = ctx.compute_accel(p, m, 0.5, softening=1e-3, eps=eps)
        for _ in range(5 // k_per_call):
            ctx.step_leapfrog(p, v, m, a, 2e-3, k_per_call, theta=0.5, softening=1e-3, eps=eps)
        torch.cuda.synchronize()
        out.append((p, v, a, ctx.walk_counts(s.n), *_node_set(ctx.tree())))
    for name, x, y in zip(("pos", "vel", "acc", "counts", "order", "nodes", "moments"), *out):
        assert torch.equal(x, y), name


def _node_set(t):
    """The exported tree as the set of its nodes: rows (first, count, level and
    child count) with their moments, sorted; node numbers within a level
    depend on the order in which blocks reserved them."""
    info = t.info.cpu().numpy()
    mom = t.mom.cpu().numpy()
    key = info[:, [0, 1, 3]]
    o = np.lexsort(key.T[::-1])
    return t.order, torch.from_numpy(key[o]), torch.from_numpy(mom[o])


def test_batched_multi_step_equals_one_step_calls(api):
    rng = np.random.default_rng(52)
    ns = rng.integers(300, 9000, 7)
    scenes = [ics.uniform_ball(int(n), seed=520 + i) for i, n in enumerate(ns)]
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    pos = np.vstack([sc.pos for sc in scenes])
    mass = np.concatenate([sc.mass for sc in scenes])
    vel = 0.2 * rng.standard_normal(pos.shape)
    out = []
    for k_per_call in (4, 1):
        ctx = api.Context(int(off[-1]), leaf_size=8, precision="fp32c", max_scenes=7)
        p, v, m = _dev(pos), _dev(vel), _dev(mass)
        a = ctx.batched_accel(off, p, m, 0.5, softening=1e-3)
        for _ in range(4 // k_per_call):
            ctx.batched_step(off, p, v, m, a, 1e-3, k_per_call, theta=0.5, softening=1e-3)
        torch.cuda.synchronize()
        out.append((p, v, a))
    for x, y in zip(*out):
        assert torch.equal(x, y)


def test_coincident_bodies_multi_step(api):
    """Every body has an exact twin (1200 coincident pairs among 6000 bodies):
    a 6-step call stays within the FP64 leapfrog bars of the oracle."""
    s = ics.uniform_ball(6000, seed=53)
    pos, vel, mass = s.pos.copy(), s.vel.copy(), s.mass.copy()
    pos[1::5] = pos[0::5]
    vel[1::5] = vel[0::5]
    xr, vr, _ = oracle.leapfrog(pos, vel, mass, 1e-3, 6, softening=1e-3, theta=0.5, leaf=8)
    ctx = api.Context(s.n, leaf_size=8, precision="fp64")
    p, v, m = _dev(pos), _dev(vel), _dev(mass)
    a = ctx.compute_accel(p, m, 0.5, softening=1e-3)
    ctx.step_leapfrog(p, v, m, a, 1e-3, 6, theta=0.5, softening=1e-3)
    assert np.abs(p.cpu().numpy() - xr).max() < 1e-13
    assert np.abs(v.cpu().numpy() - vr).max() < 1e-11


def test_multi_step_bad_input_latched(api):
    s = ics.uniform_ball(8000, seed=54)
    ctx = api.Context(s.n, leaf_size=8, precision="fp32c")
    p, v, m = _dev(s.pos), _dev(s.vel), _dev(s.mass)
    a = ctx.compute_accel(p, m, 0.5, softening=1e-3)
    bad_m = m.clone()
    bad_m[17] = float("nan")
    with pytest.raises(api.BHError, match="BH_E_NONFINITE"):
        ctx.step_leapfrog(p.clone(), v.clone(), bad_m, a.clone(), 1e-3, 3, theta=0.5,
                          softening=1e-3)
    bad_v = v.clone()
    bad_v[100, 2] = float("inf")  # the first drift makes the position infinite
    with pytest.raises(api.BHError, match="BH_E_NONFINITE"):
        ctx.step_leapfrog(p.clone(), bad_v, m, a.clone(), 1e-3, 3, theta=0.5, softening=1e-3)
    ctx.step_leapfrog(p, v, m, a, 1e-3, 3, theta=0.5, softening=1e-3)  # the latch was cleared
    assert torch.isfinite(p).all()


@pytest.mark.parametrize("n,leaf,clump", [(50, 2, 0), (5000, 16, 4000)])
def test_level_launches_small_and_clumped_multi_step(api, n, leaf, clump):
    """Multi-step calls build through the per-level launches at any size (the
    top levels read off the sorted keys): a 50-body scene, and 5000 bodies of
    which 4000 sit on one point, against the oracle's FP64 leapfrog."""
    s = ics.uniform_ball(n, seed=54)
    pos, vel, mass = s.pos.copy(), s.vel.copy(), s.mass.copy()
    pos[:clump] = [0.1, -0.2, 0.3]
    xr, vr, _ = oracle.leapfrog(pos, vel, mass, 1e-3, 6, softening=1e-3, theta=0.5, leaf=leaf)
    ctx = api.Context(n, leaf_size=leaf, precision="fp64")
    p, v, m = _dev(pos), _dev(vel), _dev(mass)
    a = ctx.compute_accel(p, m, 0.5, softening=1e-3)
    ctx.step_leapfrog(p, v, m, a, 1e-3, 6, theta=0.5, softening=1e-3)
    assert np.abs(p.cpu().numpy() - xr).max() < 1e-13
    assert np.abs(v.cpu().numpy() - vr).max() < 1e-11
