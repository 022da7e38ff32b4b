"""Many independent scenes per call, and graph-captured steps.

Bars: per scene, the same bars as the single-scene parity tests (counts exact;
FP64 1e-12 A_i; FP32C 64u A_i). A batched call gives every scene the same
tree, groups and interaction order as a call on that scene alone, so the two
must agree bit for bit; a replayed step graph must agree bit for bit with the
same steps run eagerly.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04197_amd import ics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
FP32C_TOL = 64 * 2.0 ** -24


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_1912_04197_amd import api as A

    return A


def _scenes(k, lo, hi, seed):
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), k))).astype(int)
    sc = [ics.uniform_ball(int(n), seed=seed * 100 + i) for i, n in enumerate(ns)]
    offsets = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    pos = np.vstack([s.pos for s in sc])
    mass = np.concatenate([s.mass for s in sc])
    return sc, offsets, pos, mass


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_batched_accel_parity(api, precision):
    sc, off, pos, mass = _scenes(12, 60, 5000, 7)
    ctx = api.Context(len(mass), leaf_size=8, precision=precision, counts=True, max_scenes=16)
    acc = ctx.batched_accel(off, _dev(pos), _dev(mass), 0.5, softening=1e-3).cpu().numpy()
    cnt = ctx.walk_counts(len(mass)).cpu().numpy()
    tol = FP64_TOL if precision == "fp64" else FP32C_TOL
    for k, s in enumerate(sc):
        a, b = off[k], off[k + 1]
        ref, _, aabs, rc = oracle.bh(s.pos, s.mass, 0.5, softening=1e-3, leaf=8)
        assert np.array_equal(cnt[a:b], rc), k
        err = np.linalg.norm(acc[a:b] - ref, axis=1)
        assert np.all(err <= tol * aabs), (k, (err / aabs).max())


@pytest.mark.parametrize("group", [64, 16])
def test_batched_equals_single_scene_calls(api, group):
    """Each scene of a batch equals its own single-scene call bit for bit, on
    the first batched build (sorted by passes) and on the second (sorted by
    buckets of the top key bits per scene, chosen from the first build's
    hint)."""
    sc, off, pos, mass = _scenes(9, 30, 3000, 8)
    assert off[-1] > 4096  # the bucket sort needs more than one block's bodies
    ctx = api.Context(len(mass), leaf_size=16, precision="fp32c", max_scenes=9, walk_group=group)
    single = api.Context(len(mass), leaf_size=16, precision="fp32c", walk_group=group)
    for call in range(2):
        acc = ctx.batched_accel(off, _dev(pos), _dev(mass), 0.6, softening=1e-3).cpu().numpy()
        assert ctx.stats()["bucket_sort"] == (call == 1)
        for k, s in enumerate(sc):
            a1 = single.compute_accel(_dev(s.pos), _dev(s.mass), 0.6, softening=1e-3).cpu().numpy()
            assert np.array_equal(acc[off[k]:off[k + 1]], a1), (call, k)


def test_batched_step_graph_replays(api):
    """Graph-captured batched steps, replayed in several calls with other GPU
    work and synchronisations in between, equal the eager steps bit for bit."""
    sc, off, pos, mass = _scenes(8, 100, 4000, 9)
    rng = np.random.default_rng(9)
    vel = 0.1 * rng.standard_normal(pos.shape)
    n = len(mass)
    eager = api.Context(n, leaf_size=8, precision="fp32c", max_scenes=8)
    graph = api.Context(n, leaf_size=8, precision="fp32c", max_scenes=8, graph=True)
    other = api.Context(4096, leaf_size=16)
    s_other = ics.plummer(4096, seed=3)
    state = []
    for ctx in (eager, graph):
        p, v, m = _dev(pos), _dev(vel), _dev(mass)
        a = ctx.batched_accel(off, p, m, 0.5, softening=1e-3)
        state.append((ctx, p, v, m, a))
    for rep in range(4):
        for ctx, p, v, m, a in state:
            ctx.batched_step(off, p, v, m, a, 1e-3, 3, theta=0.5, softening=1e-3)
        other.compute_accel(_dev(s_other.pos), _dev(s_other.mass), 0.5, softening=1e-3)
        torch.cuda.synchronize()
        (_, p0, v0, _, a0), (_, p1, v1, _, a1) = state
        assert torch.equal(p0, p1) and torch.equal(v0, v1) and torch.equal(a0, a1), rep


def test_batched_step_graph_follows_layout_changes(api):
    """A graph captured for one scene layout is not replayed for another with
    the same body count, scene count and arrays but different walk groups:
    graph-captured steps equal eager ones bit for bit across layout changes."""
    s = ics.uniform_ball(4000, seed=19)
    rng = np.random.default_rng(19)
    vel = 0.05 * rng.standard_normal(s.pos.shape)
    layouts = [np.array([0, 1000, 4000]), np.array([0, 2000, 4000]), np.array([0, 1000, 4000])]
    eager = api.Context(s.n, leaf_size=8, precision="fp64", max_scenes=2, walk_group=64)
    graph = api.Context(s.n, leaf_size=8, precision="fp64", max_scenes=2, walk_group=64,
                        graph=True)
    st = []
    for ctx in (eager, graph):
        p, v, m = _dev(s.pos), _dev(vel), _dev(s.mass)
        st.append((ctx, p, v, m, ctx.batched_accel(layouts[0], p, m, 0.5, softening=1e-3)))
    for k, off in enumerate(layouts):
        for ctx, p, v, m, a in st:
            ctx.batched_accel(off, p, m, 0.5, softening=1e-3, out=a)
            ctx.batched_step(off, p, v, m, a, 1e-3, 3, theta=0.5, softening=1e-3)
        torch.cuda.synchronize()
        (_, p0, v0, _, a0), (_, p1, v1, _, a1) = st
        assert torch.equal(p0, p1) and torch.equal(v0, v1) and torch.equal(a0, a1), k


def test_step_leapfrog_graph_replays(api):
    s = ics.plummer(30000, seed=10)
    eager = api.Context(s.n, precision="fp32c")
    graph = api.Context(s.n, precision="fp32c", graph=True)
    st = []
    for ctx in (eager, graph):
        p, v, m = _dev(s.pos), _dev(s.vel), _dev(s.mass)
        st.append((ctx, p, v, m, ctx.compute_accel(p, m, 0.5, softening=1e-3)))
    for rep in range(3):
        for ctx, p, v, m, a in st:
            ctx.step_leapfrog(p, v, m, a, 1e-3, 4, theta=0.5, softening=1e-3)
        torch.cuda.synchronize()
        assert torch.equal(st[0][1], st[1][1]) and torch.equal(st[0][2], st[1][2]), rep


def test_step_graph_follows_tree_depth(api):
    """A step graph is captured with the tree depth of its first build; the
    bodies are then moved in place (same pointers) into a much deeper tree:
    the replayed steps build it through the deep-level block, the next call
    captures again, and every step equals the eager one bit for bit."""
    n = 20000
    s = ics.uniform_ball(n, seed=31)
    deep = s.pos.copy()
    deep[: n // 2] = 1e-6 * deep[: n // 2] + 0.3  # half the bodies in a tiny cluster
    eager = api.Context(n, leaf_size=4, precision="fp32c")
    graph = api.Context(n, leaf_size=4, precision="fp32c", graph=True)
    st = []
    for ctx in (eager, graph):
        p, v, m = _dev(s.pos), _dev(s.vel), _dev(s.mass)
        st.append((ctx, p, v, m, ctx.compute_accel(p, m, 0.5, softening=1e-3)))
    for rep in range(4):
        if rep == 2:
            for ctx, p, v, m, a in st:
                p.copy_(_dev(deep))
                a.copy_(ctx.compute_accel(p, m, 0.5, softening=1e-3))
        for ctx, p, v, m, a in st:
            ctx.step_leapfrog(p, v, m, a, 1e-4, 3, theta=0.5, softening=1e-3)
        torch.cuda.synchronize()
        assert torch.equal(st[0][1], st[1][1]) and torch.equal(st[0][4], st[1][4]), rep
    assert eager.tree().depth >= 15


@pytest.mark.parametrize("leaf,group", [(16, 0), (4, 64)])
def test_batched_256_scene_workload(api, leaf, group):
    """The batched workload at full size: 256 uniform balls, N log-uniform in
    [1024, 65536] (about 4 million bodies), theta 0.5, FP32C, at leaf 16 with
    the default walk group and at the bucket and group sizes the autotuner
    picks for this workload on an MI355X (leaf 4, 64-body groups); eight
    scenes are checked against the oracle on 256 sampled targets each."""
    scenes = ics.batched_scenes(256, seed=44)
    ns = np.array([s.n for s in scenes])
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    n = int(off[-1])
    ctx = api.Context(n, leaf_size=leaf, precision="fp32c", counts=True, max_scenes=256,
                      walk_group=group)
    pos = _dev(np.vstack([s.pos for s in scenes]))
    mass = _dev(np.concatenate([s.mass for s in scenes]))
    acc = ctx.batched_accel(off, pos, mass, 0.5, softening=1e-3).cpu().numpy()
    cnt = ctx.walk_counts(n).cpu().numpy()
    # a second build sorts each scene by buckets (the first build's hint): the
    # same order, so the same accelerations bit for bit
    acc2 = ctx.batched_accel(off, pos, mass, 0.5, softening=1e-3).cpu().numpy()
    assert ctx.stats()["bucket_sort"]
    assert np.array_equal(acc2, acc)
    rng = np.random.default_rng(4)
    for k in rng.choice(256, 8, replace=False):
        s = scenes[k]
        t = np.sort(rng.choice(s.n, min(256, s.n), replace=False))
        ref, _, aabs, rc = oracle.Tree(s.pos, s.mass, leaf=leaf).accel(0.5, softening=1e-3,
                                                                       targets=t)
        a = acc[off[k]:off[k + 1]][t]
        assert np.array_equal(cnt[off[k]:off[k + 1]][t], rc), k
        assert np.all(np.linalg.norm(a - ref, axis=1) <= FP32C_TOL * aabs), k


def test_batched_layout_errors(api):
    ctx = api.Context(100, max_scenes=4)
    p = torch.zeros((100, 3), dtype=torch.float64, device="cuda")
    m = torch.ones(100, dtype=torch.float64, device="cuda")
    for bad in ([0, 50, 50, 100], [1, 50, 100], [0, 20, 40, 60, 80, 100]):
        with pytest.raises((api.BHError, ValueError)):
            ctx.batched_accel(np.array(bad), p, m, 0.5)


def test_autotune_picks_a_candidate_and_caches(api, tmp_path, monkeypatch):
    sc, off, pos, mass = _scenes(6, 200, 3000, 11)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("BHX_AUTOTUNE_CACHE", str(cache))
    P, V, M = _dev(pos), _dev(np.zeros_like(pos)), _dev(mass)
    before = P.clone()
    leaf, group, ms = api.autotune(off, P, V, M, theta=0.5, dt=1e-3, softening=1e-3, steps=2)
    assert leaf in (4, 8, 16, 32) and group in (16, 32, 64) and ms > 0
    assert torch.equal(P, before)
    assert cache.read_text().count("\"leaf\"") == 1
    again = api.autotune(off, P, V, M, theta=0.5, dt=1e-3, softening=1e-3, steps=2)
    assert again == (leaf, group, ms)
    assert cache.read_text().count("\"leaf\"") == 1
    # quadrupole nodes time other kernels: a separate entry, not the monopole one
    api.autotune(off, P, V, M, theta=0.5, dt=1e-3, softening=1e-3, steps=2, quad=True)
    assert cache.read_text().count("\"leaf\"") == 2
