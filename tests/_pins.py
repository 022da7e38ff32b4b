"""Pins for the FP64 oracle: checks against closed forms, invariants and an
independent set-based statement of the Barnes-Hut walk.

Each pin is a plain function that raises AssertionError when the oracle is
wrong. ``test_oracle_pins.py`` runs them as tests; ``test_oracle_mutants.py``
re-runs them against copies of the oracle with planted mistakes and checks
that every planted mistake makes at least one pin fail.
"""
from __future__ import annotations

import math
import os

import numpy as np

import oracle
from paper_1912_04197_amd import ics

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


# ------------------------------------------------------------------ direct sum

def pin_two_body_softened():
    """Hand-derived softened pair with unequal per-body softening."""
    g = _golden("two_body_soft.txt")
    acc, phi, _ = oracle.direct(g[:, 0:3], g[:, 3], eps=g[:, 4])
    np.testing.assert_allclose(acc, g[:, 5:8], rtol=1e-15, atol=0)
    np.testing.assert_allclose(phi, g[:, 8], rtol=1e-15, atol=0)


def pin_three_collinear():
    g = _golden("three_collinear.txt")
    acc, phi, _ = oracle.direct(g[:, 0:3], g[:, 3])
    np.testing.assert_allclose(acc[:, 0], g[:, 4], rtol=1e-15, atol=1e-15)
    assert np.all(acc[:, 1:] == 0.0)
    np.testing.assert_allclose(phi, g[:, 5], rtol=1e-15)


def pin_two_body_uniform_softening_formula():
    """Random pairs against a_1 = G m_2 d / (|d|^2 + eps^2)^(3/2)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        x = rng.standard_normal((2, 3))
        m = rng.random(2) + 0.1
        e = float(rng.random())
        G = float(rng.random() + 0.5)
        acc, phi, _ = oracle.direct(x, m, softening=e, G=G)
        d = x[1] - x[0]
        r2 = float(d @ d) + e * e
        np.testing.assert_allclose(acc[0], G * m[1] * d / r2 ** 1.5, rtol=1e-14)
        np.testing.assert_allclose(acc[1], -G * m[0] * d / r2 ** 1.5, rtol=1e-14)
        np.testing.assert_allclose(phi, [-G * m[1] / math.sqrt(r2), -G * m[0] / math.sqrt(r2)],
                                   rtol=1e-14)


def pin_newton_third_law():
    """sum_i m_i a_i = 0 for the direct sum (symmetric pair softening)."""
    rng = np.random.default_rng(7)
    n = 400
    x = rng.standard_normal((n, 3))
    m = rng.random(n)
    eps = 0.05 * rng.random(n)
    acc, _, aabs = oracle.direct(x, m, eps=eps)
    net = (m[:, None] * acc).sum(0)
    scale = float((m * aabs).sum())
    assert np.abs(net).max() <= 1e-14 * scale, (net, scale)


def _polyhedra():
    phi = (1 + 5 ** 0.5) / 2
    octa = [(s * (i == 0), s * (i == 1), s * (i == 2)) for i in range(3) for s in (1.0, -1.0)]
    cube = [(a, b, c) for a in (1.0, -1.0) for b in (1.0, -1.0) for c in (1.0, -1.0)]
    ico = []
    for a in (1.0, -1.0):
        for b in (phi, -phi):
            ico += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    return {"octahedron": octa, "cube": cube, "icosahedron": ico}


def pin_symmetric_shells():
    """A body at the centre of a regular polyhedron of equal masses feels no
    force, and every vertex body is pulled exactly towards the centre."""
    for name, verts in _polyhedra().items():
        v = np.array(verts, dtype=np.float64)
        x = np.vstack([np.zeros((1, 3)), 2.5 * v])
        m = np.full(len(x), 0.3)
        acc, _, aabs = oracle.direct(x, m, softening=0.1)
        assert np.abs(acc[0]).max() <= 1e-15 * aabs[0], name
        for k in range(1, len(x)):
            radial = -x[k] / np.linalg.norm(x[k])
            perp = acc[k] - (acc[k] @ radial) * radial
            assert np.linalg.norm(perp) <= 1e-14 * aabs[k], name
            assert acc[k] @ radial > 0, name


def pin_shell_theorem():
    """Uniform ball of mass M, radius R: a(r) = -G M r / R^3 inside and
    -G M / r^2 outside; phi(r) = -G M (3R^2 - r^2) / (2 R^3) inside, -G M / r
    outside. Massless probes in many directions per radius, small softening,
    Monte-Carlo tolerance."""
    n = 200_000
    s = ics.uniform_ball(n, seed=3)
    radii = [0.25, 0.5, 0.75, 1.5, 3.0]
    rng = np.random.default_rng(31)
    dirs = rng.standard_normal((48, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    probes = np.vstack([r * dirs for r in radii])
    x = np.vstack([s.pos, probes])
    m = np.concatenate([s.mass, np.zeros(len(probes))])
    targets = np.arange(n, n + len(probes))
    acc, phi, _ = oracle.direct(x, m, softening=0.02, targets=targets)
    for k, r in enumerate(radii):
        sl = slice(48 * k, 48 * (k + 1))
        a_rad = -(acc[sl] * dirs).sum(1).mean()
        a_exp = r if r < 1 else 1.0 / r ** 2
        p_exp = -(3 - r * r) / 2 if r < 1 else -1.0 / r
        assert abs(a_rad - a_exp) <= 0.015 * a_exp, (r, a_rad, a_exp)
        assert abs(phi[sl].mean() - p_exp) <= 0.005 * abs(p_exp), (r, phi[sl].mean(), p_exp)


def pin_torch_bruteforce_direct():
    """Direct sum against an all-pairs broadcast in numpy (N = 300)."""
    rng = np.random.default_rng(9)
    n = 300
    x = rng.standard_normal((n, 3))
    m = rng.random(n)
    eps = 0.1 * rng.random(n)
    acc, phi, _ = oracle.direct(x, m, eps=eps, G=2.0)
    d = x[None, :, :] - x[:, None, :]
    r2 = (d * d).sum(-1) + 0.5 * (eps[:, None] ** 2 + eps[None, :] ** 2)
    np.fill_diagonal(r2, np.inf)
    a_ref = 2.0 * (m[None, :, None] * d / r2[..., None] ** 1.5).sum(1)
    p_ref = -2.0 * (m[None, :] / np.sqrt(r2)).sum(1)
    np.testing.assert_allclose(acc, a_ref, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(phi, p_ref, rtol=1e-12)


# -------------------------------------------------------------------- octree

def _quantise(x):
    """Integer cell coordinates of the root cube on a 2^21 grid (the reading
    of the cell definition; the tree pins below check its geometry)."""
    lo, hi = x.min(0), x.max(0)
    L = float((hi - lo).max())
    if L == 0.0:
        L = 1.0
    x0 = (lo + hi) * 0.5 - L * 0.5
    S = 2097152.0 / L
    q = np.clip(np.floor((x - x0) * S), 0, 2097151).astype(np.int64)
    return q, x0, L


def set_based_bh(x, m, theta, leaf, softening=0.0, eps=None):
    """Barnes-Hut as a set definition, with no recursion and no bottom-up pass.

    Cells exist at level l when their parent cell (level l-1) holds more than
    ``leaf`` bodies; a cell is a leaf when it holds at most ``leaf`` bodies or
    l = 21. For body B the accepted nodes are the internal cells that pass
    s^2 < theta^2 D^2 while every proper ancestor fails it; the leaf pairs are
    the members j != B of leaves whose proper ancestors all fail it. Centres of
    mass are mass-weighted means over each cell's members.
    Returns (acc, counts) with counts[:, 0] nodes and counts[:, 1] pairs.
    """
    n = len(x)
    q, x0, L = _quantise(x)
    cells = {}  # (level, cx, cy, cz) -> member indices
    for lvl in range(22):
        key = q >> (21 - lvl)
        groups = {}
        for i in range(n):
            groups.setdefault((lvl, *key[i]), []).append(i)
        for k, mem in groups.items():
            if lvl == 0:
                cells[k] = np.array(mem)
            else:
                parent = (lvl - 1, *(np.array(k[1:]) >> 1))
                if parent in cells and len(cells[parent]) > leaf:
                    cells[k] = np.array(mem)
    info = {}
    for k, mem in cells.items():
        mm = m[mem].sum()
        com = (m[mem, None] * x[mem]).sum(0) / mm
        e2 = (m[mem] * eps[mem] ** 2).sum() / mm if eps is not None else 0.0
        is_leaf = len(mem) <= leaf or k[0] == 21
        # passes[b]: does cell k pass the opening test for body b?
        D2 = ((com[None, :] - x) ** 2).sum(1)
        s = L / 2 ** k[0]
        info[k] = (mem, mm, com, e2, is_leaf, s * s < theta * theta * D2)
    acc = np.zeros((n, 3))
    counts = np.zeros((n, 2), np.int64)
    eb2 = eps ** 2 if eps is not None else None
    for k, (mem, mm, com, e2, is_leaf, passes) in info.items():
        lvl = k[0]
        reach = np.ones(n, bool)  # every proper ancestor fails the test
        for a in range(lvl):
            anc = (a, *(np.array(k[1:]) >> (lvl - a)))
            reach &= ~info[anc][5]
        if is_leaf:
            for j in mem:
                sel = reach.copy()
                sel[j] = False
                d = x[j][None, :] - x[sel]
                e = 0.5 * (eb2[sel] + eps[j] ** 2) if eps is not None else softening ** 2
                acc[sel] += m[j] * d / ((d * d).sum(1) + e)[:, None] ** 1.5
                counts[sel, 1] += 1
        else:
            sel = reach & passes
            d = com[None, :] - x[sel]
            e = 0.5 * (eb2[sel] + e2) if eps is not None else softening ** 2
            acc[sel] += mm * d / ((d * d).sum(1) + e)[:, None] ** 1.5
            counts[sel, 0] += 1
    return acc, counts


def pin_set_based_walk():
    """Recursive walk == set-based definition: identical per-body node and pair
    counts, accelerations to 1e-12 of the absolute-term sum."""
    cases = [
        (ics.uniform_ball(300, seed=1).pos, 0.5, 4, None),
        (ics.plummer(256, seed=2).pos, 0.7, 1, None),
        (ics.uniform_cube(200, seed=3).pos, 0.3, 8, None),
    ]
    rng = np.random.default_rng(4)
    for x, theta, leaf, _ in cases:
        n = len(x)
        m = rng.random(n) + 0.2
        eps = 0.02 * rng.random(n)
        acc_s, cnt_s = set_based_bh(x, m, theta, leaf, eps=eps)
        acc, _, aabs, cnt = oracle.bh(x, m, theta, eps=eps, leaf=leaf)
        assert np.array_equal(cnt, cnt_s), (theta, leaf, np.abs(cnt - cnt_s).max())
        err = np.linalg.norm(acc - acc_s, axis=1)
        assert np.all(err <= 1e-12 * aabs), (theta, leaf, (err / aabs).max())


def pin_tree_structure():
    """Node table invariants: children partition the parent's segment in octant
    order, leaves obey the bucket rule, every body lies in its leaf's cube,
    and the root holds the total mass at the global centre of mass."""
    for s, leaf in ((ics.uniform_ball(5000, seed=8), 8), (ics.plummer(3000, seed=9), 1),
                    (ics.uniform_cube(2000, seed=10), 16)):
        x, m = s.pos, s.mass * (1 + np.arange(s.n) % 3)
        T = oracle.Tree(x, m, leaf=leaf)
        t = T.export()
        box = T.box()
        L, x0 = box["L"], box["x0"]
        assert sorted(t["order"].tolist()) == list(range(s.n))
        assert t["level"][0] == 0 and t["first"][0] == 0 and t["count"][0] == s.n
        ms = m.sum()
        assert abs(t["mass"][0] - ms) <= 1e-15 * ms
        com = (m[:, None] * x).sum(0) / ms
        assert np.abs(t["com"][0] - com).max() <= 1e-14 * L
        for k in range(T.nnodes):
            lvl, f, c, c0, nc = (int(t[a][k]) for a in ("level", "first", "count", "child0", "nchild"))
            mem = t["order"][f:f + c]
            if nc == 0:
                assert c <= leaf or lvl == 21
                side = L / 2 ** lvl
                cell = t["q"][mem[0]] >> (21 - lvl)
                lo_c = x0 + cell * side
                assert np.all(x[mem] >= lo_c - 1e-12 * L) and np.all(x[mem] <= lo_c + side + 1e-12 * L)
                assert np.all((t["q"][mem] >> (21 - lvl)) == cell)
            else:
                assert c > leaf and lvl < 21 and 1 <= nc <= 8
                ch = range(c0, c0 + nc)
                assert t["first"][c0] == f
                assert sum(int(t["count"][j]) for j in ch) == c
                for j in ch:
                    assert t["level"][j] == lvl + 1
                    assert t["count"][j] > 0
                octs = [int(((t["q"][t["order"][t["first"][j]]] >> (20 - lvl)) & 1) @ [4, 2, 1])
                        for j in ch]
                assert octs == sorted(set(octs))
                for a, b in zip(ch, list(ch)[1:]):
                    assert t["first"][b] == t["first"][a] + t["count"][a]
            mm = m[mem].sum()
            assert abs(t["mass"][k] - mm) <= 1e-14 * mm
            assert np.abs(t["com"][k] - (m[mem, None] * x[mem]).sum(0) / mm).max() <= 1e-14 * L


def pin_theta_zero_is_direct():
    """theta = 0 opens every node: the same pair set as the direct sum."""
    s = ics.uniform_ball(1500, seed=12)
    eps = 0.01 * (1 + np.arange(s.n) % 5)
    for e in (None, eps):
        acc_d, phi_d, aabs = oracle.direct(s.pos, s.mass, softening=1e-3, eps=e)
        acc_t, phi_t, _, cnt = oracle.bh(s.pos, s.mass, 0.0, softening=1e-3, eps=e, leaf=4)
        assert np.all(cnt[:, 0] == 0) and np.all(cnt[:, 1] == s.n - 1)
        assert np.all(np.linalg.norm(acc_t - acc_d, axis=1) <= 1e-13 * aabs)
        np.testing.assert_allclose(phi_t, phi_d, rtol=1e-13)


def pin_leaf_ge_n_is_direct():
    s = ics.plummer(700, seed=13)
    acc_d, _, aabs = oracle.direct(s.pos, s.mass, softening=1e-2)
    acc_t, _, _, cnt = oracle.bh(s.pos, s.mass, 0.9, softening=1e-2, leaf=700)
    assert np.all(cnt[:, 1] == s.n - 1)
    assert np.all(np.linalg.norm(acc_t - acc_d, axis=1) <= 1e-13 * aabs)


def pin_error_monotone_in_theta():
    """RMS force error against the direct sum grows with theta, roughly as
    theta^2 for a monopole about the centre of mass."""
    s = ics.uniform_ball(6000, seed=14)
    acc_d, _, _ = oracle.direct(s.pos, s.mass, softening=1e-3)
    norm = np.linalg.norm(acc_d, axis=1)
    errs = []
    for th in (0.2, 0.4, 0.6, 0.8):
        acc_t, _, _, _ = oracle.bh(s.pos, s.mass, th, softening=1e-3, leaf=8)
        errs.append(math.sqrt(np.mean((np.linalg.norm(acc_t - acc_d, axis=1) / norm) ** 2)))
    assert all(a < b for a, b in zip(errs, errs[1:])), errs
    assert errs[0] < 1e-3 and errs[-1] < 0.1, errs
    assert errs[-1] / errs[0] > 4.0, errs


def pin_coincident_and_tiny():
    """n = 1 gives zero; bodies that share one point end in one level-21 leaf
    and, softened, pull each other with zero force."""
    acc, phi, _, cnt = oracle.bh(np.array([[0.3, -0.2, 0.1]]), np.array([2.0]), 0.5,
                                 softening=0.1, leaf=1)
    assert np.all(acc == 0) and np.all(cnt == 0) and phi[0] == 0
    x = np.vstack([np.tile([[0.1, 0.2, 0.3]], (40, 1)), [[1.0, 1.0, 1.0]]])
    m = np.ones(41)
    T = oracle.Tree(x, m, leaf=16)
    t = T.export()
    leaves = t["nchild"] == 0
    assert t["count"][leaves].max() == 40 and t["level"][leaves].max() == 21
    acc, phi, _, cnt = T.accel(0.5, softening=0.01)
    d = np.array([0.9, 0.8, 0.7])
    a_far = d / (d @ d + 1e-4) ** 1.5
    np.testing.assert_allclose(acc[0], a_far, rtol=1e-6)


# ------------------------------------------------------------------ leapfrog

def pin_leapfrog_circular_orbit():
    """Circular two-body orbit returns to its start after one period
    2 pi sqrt(a^3 / (G M)); the phase error is O(dt^2)."""
    s = ics.two_body_circular(0.7, 0.3, 1.0)
    period = 2 * math.pi * math.sqrt(1.0 / 1.0)
    errs = []
    for nsteps in (400, 800):
        dt = period / nsteps
        x, v, a = oracle.leapfrog(s.pos, s.vel, s.mass, dt, nsteps)
        errs.append(np.linalg.norm(x - s.pos))
    assert errs[0] < 2e-3, errs
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def pin_leapfrog_reversible():
    """n steps forward, reverse the velocities, n steps back: the start again."""
    s = ics.plummer(64, seed=15)
    x, v, a = oracle.leapfrog(s.pos, s.vel, s.mass, 1e-3, 200, softening=0.05)
    x2, v2, _ = oracle.leapfrog(x, -v, s.mass, 1e-3, 200, softening=0.05, acc=a)
    assert np.abs(x2 - s.pos).max() < 1e-12
    assert np.abs(v2 + s.vel).max() < 1e-11


def pin_leapfrog_conservation():
    """Direct-sum leapfrog: momentum and angular momentum to round-off, energy
    error bounded and oscillating with no secular drift."""
    s = ics.plummer(48, seed=16)
    e0 = oracle.diagnostics(s.pos, s.vel, s.mass, softening=0.05)
    x, v, a = s.pos, s.vel, None
    devs = []
    for _ in range(8):
        x, v, a = oracle.leapfrog(x, v, s.mass, 2e-3, 250, softening=0.05, acc=a)
        d = oracle.diagnostics(x, v, s.mass, softening=0.05)
        devs.append(abs((d[0] + d[1]) - (e0[0] + e0[1])) / abs(e0[0] + e0[1]))
        assert np.abs(d[2:5] - e0[2:5]).max() < 1e-14
        assert np.abs(d[5:8] - e0[5:8]).max() < 1e-13
    assert max(devs) < 1e-3, devs
    assert max(devs[4:]) < 3 * max(devs[:4]) + 1e-12, devs


def pin_leapfrog_tree_theta0():
    s = ics.uniform_ball(300, seed=17)
    xd, vd, _ = oracle.leapfrog(s.pos, s.vel, s.mass, 1e-3, 5, softening=1e-2)
    xt, vt, _ = oracle.leapfrog(s.pos, s.vel, s.mass, 1e-3, 5, softening=1e-2, theta=0.0, leaf=4)
    assert np.abs(xt - xd).max() < 1e-13 and np.abs(vt - vd).max() < 1e-11


# --------------------------------------------------------------- quadrupole

def pin_quad_dumbbell_closed_form():
    """Two masses m at +-h on z: Q_zz = 4 m h^2, Q_xx = Q_yy = -2 m h^2 about
    their centre; on the axis at distance R the quadrupole correction is
    -6 G m h^2 / R^4 (the 1/R^4 term of the exact 1/(R-h)^2 + 1/(R+h)^2)."""
    m, h, R = 0.7, 0.05, 2.0
    pos = np.array([[0, 0, h], [0, 0, -h], [0, 0, R]], float)
    T = oracle.Tree(pos, np.array([m, m, 1e-30]), leaf=1)
    q = T.quadrupoles()
    ex = T.export()
    k = [i for i in range(len(q)) if ex["count"][i] == 2 and ex["nchild"][i] > 0]
    np.testing.assert_allclose(q[k[0]], [-2 * m * h * h, -2 * m * h * h, 4 * m * h * h, 0, 0, 0],
                               rtol=1e-12, atol=1e-18)
    a_mono = T.accel(0.9)[0][2, 2]
    a_quad = T.accel(0.9, quad=True)[0][2, 2]
    np.testing.assert_allclose(a_quad - a_mono, -6 * m * h * h / R ** 4, rtol=1e-12)


def pin_quad_far_field_order():
    """A compact cluster seen from distance R: the monopole's error falls as
    R^-4 and with the quadrupole term as R^-5 (the dipole vanishes about the
    centre of mass), each checked as the ratio between R and 2R."""
    rng = np.random.default_rng(41)
    cl = 0.05 * rng.standard_normal((30, 3))
    m = rng.uniform(0.5, 1.5, 30)
    direc = np.array([0.6, -0.48, 0.64])
    errs = {False: [], True: []}
    for R in (1.0, 2.0):
        pos = np.vstack([cl, R * direc])
        mass = np.append(m, 1e-30)
        exact = oracle.direct(pos, mass)[0][30]
        T = oracle.Tree(pos, mass, leaf=1)
        for q in (False, True):
            a, _, _, cnt = T.accel(0.9, quad=q)
            assert cnt[30, 1] == 0  # the probe sees the cluster through nodes only
            errs[q].append(np.linalg.norm(a[30] - exact))
    r_mono = errs[False][0] / errs[False][1]
    r_quad = errs[True][0] / errs[True][1]
    assert 12 < r_mono < 20 and 26 < r_quad < 40, (r_mono, r_quad)
    assert errs[True][0] < 0.2 * errs[False][0]


def pin_quad_cubic_symmetry_vanishes():
    """Equal masses on the six octahedron vertices have no quadrupole (cubic
    symmetry), so the quadrupole walk equals the monopole walk."""
    h = 0.05
    v = h * np.vstack([np.eye(3), -np.eye(3)])
    pos = np.vstack([v, [[1.3, 0.7, -0.9]]])
    mass = np.append(np.ones(6), 1e-30)
    T = oracle.Tree(pos, mass, leaf=1)
    a0 = T.accel(0.9)[0][6]
    a1 = T.accel(0.9, quad=True)[0][6]
    assert np.abs(a1 - a0).max() < 1e-15 * np.abs(a0).max()


def pin_quad_improves_accuracy():
    """Plummer sphere, theta 0.5: adding the quadrupole term cuts the RMS force
    error against the direct sum; theta 0 still equals the direct sum."""
    s = ics.plummer(3000, seed=42)
    ref = oracle.direct(s.pos, s.mass, softening=1e-3)[0]
    T = oracle.Tree(s.pos, s.mass, leaf=8)

    def rms(a):
        return np.sqrt(np.mean(np.sum((a - ref) ** 2, 1) / np.sum(ref ** 2, 1)))

    e_m = rms(T.accel(0.5, softening=1e-3)[0])
    e_q = rms(T.accel(0.5, softening=1e-3, quad=True)[0])
    assert e_q < 0.5 * e_m, (e_m, e_q)
    a0 = T.accel(0.0, softening=1e-3, quad=True)[0]
    assert np.abs(a0 - ref).max() <= 1e-13 * np.abs(ref).max()


# --------------------------------------------------------------- aggregates

def pin_contacts_hand_built():
    """A chain of touching spheres (centre distance exactly r_i + r_j counts as
    contact), a pair a hair too far apart, and two single bodies: components
    and contact counts by hand; the skin closes the gap."""
    r = np.array([0.5, 0.25, 0.25, 0.5, 1.0, 1.0, 0.1, 0.1])
    pos = np.array([[0, 0, 0], [0.75, 0, 0], [1.25, 0, 0], [2.0, 0, 0],   # chain 0-1-2-3
                    [10, 0, 0], [12.0 + 1e-9, 0, 0],                      # gap 1e-9
                    [20, 0, 0], [30, 0, 0]], float)                       # singles
    label, nc, na = oracle.contact_components(pos, r)
    assert label.tolist() == [0, 0, 0, 0, 4, 5, 6, 7] and nc == 3 and na == 1
    label, nc, na = oracle.contact_components(pos, r, skin=1e-6)
    assert label.tolist() == [0, 0, 0, 0, 4, 4, 6, 7] and nc == 4 and na == 2


def pin_contacts_scipy_components():
    """Random spheres: the partition into components equals scipy's connected
    components of the contact graph, labels are each component's smallest
    index, and aggregates are the components with more than one body."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(61)
    n = 500
    pos = rng.random((n, 3))
    r = 0.02 * rng.random(n) + 0.01
    label, nc, na = oracle.contact_components(pos, r)
    d2 = ((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1)
    R = r[:, None] + r[None, :]
    i, j = np.nonzero(np.triu(d2 <= R * R, 1))
    assert nc == len(i) > 0
    k, comp = connected_components(coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n)),
                                   directed=False)
    for c in range(k):
        members = np.nonzero(comp == c)[0]
        assert np.all(label[members] == members.min())
    sizes = np.bincount(comp)
    assert na == int((sizes > 1).sum()) and len(np.unique(label)) == k


# ------------------------------------------------------------- semi-implicit Euler

def pin_euler_held_gravity_closed_form():
    """With gravity held over the whole call (every > nsteps) the substeps are
    v_s = v0 + s dt a0 and x_s = x0 + s dt v0 + dt^2 a0 s (s + 1) / 2: the kick
    comes first and the drift uses the new velocity."""
    s = ics.plummer(40, seed=31)
    rng = np.random.default_rng(31)
    a0 = rng.standard_normal((40, 3))
    for nsteps in (1, 2, 7):
        dt = 1e-2
        x, v, a = oracle.euler(s.pos, s.vel, s.mass, dt, nsteps, every=nsteps + 1, acc=a0)
        k = nsteps
        np.testing.assert_allclose(v, s.vel + k * dt * a0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(x, s.pos + k * dt * s.vel + dt * dt * a0 * k * (k + 1) / 2,
                                   rtol=0, atol=1e-14)
        assert np.array_equal(a, a0)


def pin_euler_circular_orbit():
    """Circular two-body orbit after one period. Semi-implicit Euler is the
    leapfrog map with velocities taken half a step early (it is conjugate to
    it), so over a closed orbit its position error falls as dt^2; its energy
    error stays bounded (a symplectic map) instead of drifting, where an
    explicit Euler step would spiral outwards."""
    s = ics.two_body_circular(0.7, 0.3, 1.0)
    period = 2 * math.pi
    errs = []
    for nsteps in (2000, 4000):
        dt = period / nsteps
        x, v, a = oracle.euler(s.pos, s.vel, s.mass, dt, nsteps)
        errs.append(np.linalg.norm(x - s.pos))
    assert errs[0] < 1e-4 and 3.5 < errs[0] / errs[1] < 4.5, errs
    e0 = oracle.diagnostics(s.pos, s.vel, s.mass)
    x, v, a = s.pos, s.vel, None
    devs = []
    for _ in range(10):
        x, v, a = oracle.euler(x, v, s.mass, period / 500, 500, acc=a)
        d = oracle.diagnostics(x, v, s.mass)
        devs.append(abs((d[0] + d[1]) - (e0[0] + e0[1])) / abs(e0[0] + e0[1]))
    # an explicit Euler step of this size changes the energy by ~40 % in ten orbits
    assert max(devs) < 1e-6, devs


def pin_euler_two_rate_momentum():
    """Direct forces: total momentum is conserved to round-off whatever the
    gravity rate (every term of sum m a cancels pairwise)."""
    s = ics.plummer(48, seed=32)
    e0 = oracle.diagnostics(s.pos, s.vel, s.mass, softening=0.05)
    x, v, a = oracle.euler(s.pos, s.vel, s.mass, 2e-3, 300, every=4, softening=0.05)
    d = oracle.diagnostics(x, v, s.mass, softening=0.05)
    assert np.abs(d[2:5] - e0[2:5]).max() < 1e-14


def pin_gravity_dt_bound():
    """eq. (dt_g): 1 / (2 sqrt(G rho)) for one body of each density the paper
    quotes for asteroid material (golden, SI units; of the order of thousands
    of seconds), the densest body decides for a mixed set, massless bodies are
    skipped, and a massive point (radius 0) allows no step."""
    rows = _golden("dt_g.txt")
    for G, rho, r, bound in rows:
        m = rho * (4.0 / 3.0) * math.pi * r ** 3
        got = oracle.gravity_dt_bound([m], [r], G=G)
        assert abs(got - bound) <= 1e-13 * bound, (rho, got, bound)
        assert 500.0 < got < 5000.0
    # mixed set: the 4 g/cm^3 body decides whatever the order and sizes
    G = rows[0][0]
    m = [1000 * (4 / 3) * math.pi * 7.0 ** 3, 4000 * (4 / 3) * math.pi * 2.0 ** 3, 0.0]
    r = [7.0, 2.0, 0.5]
    for perm in ([0, 1, 2], [2, 1, 0], [1, 2, 0]):
        got = oracle.gravity_dt_bound([m[i] for i in perm], [r[i] for i in perm], G=G)
        assert abs(got - rows[1][3]) <= 1e-13 * rows[1][3]
    assert oracle.gravity_dt_bound([0.0, 0.0], [1.0, 2.0]) == math.inf
    assert oracle.gravity_dt_bound([1.0, 1e-3], [1.0, 0.0]) == 0.0


def pin_coincident_below_double_range():
    """Two unsoftened bodies 1e-100 apart attract as G m / d^2 (1e200 here, in
    range); 1e-160 apart their squared distance is below the smallest normal
    double, 1 / r^3 is not representable, and (like r^2 = 0) the pair adds
    nothing: direct sum, tree walk and VJP alike."""
    for d, want in ((1e-100, 1e200), (1e-160, 0.0)):
        x = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
        m = np.array([1.0, 1.0])
        a, _, _ = oracle.direct(x, m)
        assert abs(a[0, 0] - want) <= 1e-15 * want and a[0, 1] == a[0, 2] == 0.0, (d, a)
        assert a[1, 0] == -a[0, 0]
        at = oracle.bh(x, m, 0.5, leaf=2)[0]
        assert np.array_equal(at, a), d
        if want == 0.0:
            gx, gm = oracle.direct_vjp(x, m, np.ones((2, 3)))
            assert np.all(gx == 0.0) and np.all(gm == 0.0)


def pin_diagnostics_two_body():
    s = ics.two_body_circular(0.7, 0.3, 1.0)
    d = oracle.diagnostics(s.pos, s.vel, s.mass)
    mu = 0.7 * 0.3 / 1.0
    np.testing.assert_allclose(d[1], -0.7 * 0.3, rtol=1e-15)
    np.testing.assert_allclose(d[0], 0.5 * 0.7 * 0.3 / 1.0, rtol=1e-14)
    np.testing.assert_allclose(d[7], mu * math.sqrt(1.0 * 1.0), rtol=1e-14)
    assert np.abs(d[2:5]).max() < 1e-16


# ------------------------------------------------------------------- adjoint

def _fd_case(seed=21, n=160):
    s = ics.uniform_ball(n, seed=seed)
    rng = np.random.default_rng(seed)
    m = s.mass * (1.0 + rng.random(n))
    eps = 0.02 + 0.02 * rng.random(n)
    lam = rng.standard_normal((n, 3))
    return s.pos, m, eps, lam, rng


def _frozen(x1, x2, m1, m2, eps, theta, leaf):
    """True when the tree and every opening decision agree for two inputs."""
    t1, t2 = oracle.Tree(x1, m1, eps, leaf), oracle.Tree(x2, m2, eps, leaf)
    e1, e2 = t1.export(), t2.export()
    if t1.nnodes != t2.nnodes:
        return False
    for k in ("level", "first", "count", "nchild"):
        if not np.array_equal(e1[k], e2[k]):
            return False
    return np.array_equal(t1.accel(theta)[3], t2.accel(theta)[3])


def _check_fd(f, grad_x, grad_m, x, m, coords, mcoords, tol, freeze=None):
    checked = 0
    for (i, a) in coords:
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        if freeze is not None and not (freeze(xp, x, m, m) and freeze(xm, x, m, m)):
            continue
        fd = (f(xp, m) - f(xm, m)) / (2 * h)
        assert abs(grad_x[i, a] - fd) <= tol * max(abs(fd), 1e-3), (i, a, grad_x[i, a], fd)
        checked += 1
    for i in mcoords:
        h = 1e-5 * m[i]
        mp, mm = m.copy(), m.copy()
        mp[i] += h
        mm[i] -= h
        if freeze is not None and not (freeze(x, x, mp, m) and freeze(x, x, mm, m)):
            continue
        fd = (f(x, mp) - f(x, mm)) / (2 * h)
        assert abs(grad_m[i] - fd) <= tol * max(abs(fd), 1e-3), (i, grad_m[i], fd)
        checked += 1
    assert checked >= 12, checked


def pin_vjp_direct_finite_differences():
    """Direct-sum VJP against central differences of lambda . a(x, m)."""
    x, m, eps, lam, rng = _fd_case()
    f = lambda xx, mm: float((lam * oracle.direct(xx, mm, eps=eps, G=1.3)[0]).sum())
    gx, gm = oracle.direct_vjp(x, m, lam, eps=eps, G=1.3)
    coords = [(int(rng.integers(len(x))), int(rng.integers(3))) for _ in range(12)]
    _check_fd(f, gx, gm, x, m, coords, rng.integers(len(x), size=6), 1e-6)


def pin_vjp_tree_finite_differences():
    """Tree VJP (decisions fixed) against central differences of the tree
    force map; a coordinate whose +-h moves a cell boundary or flips an
    opening decision is skipped."""
    x, m, eps, lam, rng = _fd_case(seed=22)
    theta, leaf = 0.65, 4
    f = lambda xx, mm: float((lam * oracle.bh(xx, mm, theta, eps=eps, leaf=leaf)[0]).sum())
    gx, gm = oracle.tree_vjp(x, m, lam, theta, eps=eps, leaf=leaf)
    freeze = lambda x1, x2, m1, m2: _frozen(x1, x2, m1, m2, eps, theta, leaf)
    coords = [(int(rng.integers(len(x))), int(rng.integers(3))) for _ in range(14)]
    _check_fd(f, gx, gm, x, m, coords, rng.integers(len(x), size=6), 1e-6, freeze)


def pin_vjp_invariants():
    """Translation invariance (sum_i g_x_i = 0) and degree-1 homogeneity in the
    masses (sum_j m_j g_m_j = lambda . a), for the direct sum and the tree."""
    x, m, eps, lam, _ = _fd_case(seed=23, n=400)
    for theta in (None, 0.4, 0.8):
        if theta is None:
            gx, gm = oracle.direct_vjp(x, m, lam, eps=eps)
            a = oracle.direct(x, m, eps=eps)[0]
        else:
            gx, gm = oracle.tree_vjp(x, m, lam, theta, eps=eps, leaf=8)
            a = oracle.bh(x, m, theta, eps=eps, leaf=8)[0]
        scale = float(np.abs(gx).sum())
        assert np.abs(gx.sum(0)).max() <= 1e-13 * scale, theta
        la = float((lam * a).sum())
        assert abs(float((m * gm).sum()) - la) <= 1e-12 * float(np.abs(lam * a).sum()), theta


def pin_vjp_abs_two_body_closed_form():
    """The error scale of the VJP for two bodies in one leaf, written out:
    body 0 is the target of body 1's term and the source of body 0's term in
    body 1's row; with d = x_1 - x_0, r^2 = |d|^2 + eps^2 and
    L_i = sum_a |lam_i,a| |d_a|: g_x0,a = G m_1 (|lam_0,a| / r^3 + 3 |d_a| L_0 / r^5)
    + G m_0 (|lam_1,a| / r^3 + 3 |d_a| L_1 / r^5), g_m0 = G L_1 / r^3."""
    x = np.array([[0.1, -0.2, 0.3], [0.7, 0.4, -0.5]])
    m = np.array([0.3, 1.7])
    lam = np.array([[1.0, -2.0, 0.5], [-0.25, 0.75, 3.0]])
    G, soft = 1.3, 0.2
    gx, gm = oracle.tree_vjp_abs(x, m, lam, 0.5, softening=soft, leaf=16, G=G)
    d = np.abs(x[1] - x[0])
    r2 = float((d * d).sum()) + soft * soft
    inv3, inv5 = r2 ** -1.5, r2 ** -2.5
    L0, L1 = float((np.abs(lam[0]) * d).sum()), float((np.abs(lam[1]) * d).sum())
    for b, (mo, Lb, Lo) in enumerate(((m[1], L0, L1), (m[0], L1, L0))):
        o = 1 - b
        want = (G * mo * (np.abs(lam[b]) * inv3 + 3 * d * Lb * inv5)
                + G * m[b] * (np.abs(lam[o]) * inv3 + 3 * d * Lo * inv5))
        np.testing.assert_allclose(gx[b], want, rtol=1e-14)
        np.testing.assert_allclose(gm[b], G * Lo * inv3, rtol=1e-14)


def set_based_vjp_abs(x, m, lam, theta, leaf, softening=0.0, eps=None, G=1.0):
    """The VJP's error scale from the set definition of the walk (as in
    set_based_bh): each term's part magnitudes G m_s (|l_a| / r^3 +
    3 |d_a| L / r^5), G L / r^3 and 3/2 G m_s L / r^5 with L = sum |l_a||d_a|
    go to the target (position part) and the source (all parts); an accepted
    cell hands its sums to its members with |x_j - X| and |eps_j^2 - <eps^2>|."""
    n = len(x)
    q, x0, L = _quantise(x)
    cells = {}
    for lvl in range(22):
        key = q >> (21 - lvl)
        groups = {}
        for i in range(n):
            groups.setdefault((lvl, *key[i]), []).append(i)
        for k, mem in groups.items():
            if lvl == 0:
                cells[k] = np.array(mem)
            else:
                parent = (lvl - 1, *(np.array(k[1:]) >> 1))
                if parent in cells and len(cells[parent]) > leaf:
                    cells[k] = np.array(mem)
    eb2 = eps ** 2 if eps is not None else np.zeros(n)
    gx = np.zeros((n, 3))
    gm = np.zeros(n)

    def parts(d, e2, ms, l):
        r2 = (d * d).sum(1) + e2
        inv3, inv5 = r2 ** -1.5, r2 ** -2.5
        Ld = (np.abs(l) * np.abs(d)).sum(1)
        gd = G * ms[:, None] * (np.abs(l) * inv3[:, None] + 3 * np.abs(d) * (Ld * inv5)[:, None])
        return gd, G * Ld * inv3, 1.5 * G * ms * Ld * inv5

    info = {}
    for k, mem in cells.items():
        mm = m[mem].sum()
        com = (m[mem, None] * x[mem]).sum(0) / mm
        e2 = (m[mem] * eb2[mem]).sum() / mm
        is_leaf = len(mem) <= leaf or k[0] == 21
        D2 = ((com[None, :] - x) ** 2).sum(1)
        s2 = (L / 2 ** k[0]) ** 2
        info[k] = (mem, mm, com, e2, is_leaf, s2 < theta * theta * D2)
    for k, (mem, mm, com, e2, is_leaf, passes) in info.items():
        lvl = k[0]
        reach = np.ones(n, bool)
        for a in range(lvl):
            reach &= ~info[(a, *(np.array(k[1:]) >> (lvl - a)))][5]
        if is_leaf:
            for j in mem:
                sel = reach.copy()
                sel[j] = False
                if not sel.any():
                    continue
                d = x[j][None, :] - x[sel]
                e = 0.5 * (eb2[sel] + eb2[j]) if eps is not None else np.full(sel.sum(), softening ** 2)
                gd, gmm, _ = parts(d, e, np.full(sel.sum(), m[j]), lam[sel])
                gx[sel] += gd
                gx[j] += gd.sum(0)
                gm[j] += gmm.sum()
        else:
            sel = reach & passes
            if not sel.any():
                continue
            d = com[None, :] - x[sel]
            e = 0.5 * (eb2[sel] + e2) if eps is not None else np.full(sel.sum(), softening ** 2)
            gd, gmm, ge2 = parts(d, e, np.full(sel.sum(), mm), lam[sel])
            gx[sel] += gd
            nX, nm, ne2 = gd.sum(0), gmm.sum(), 0.5 * ge2.sum()
            for j in mem:
                gx[j] += m[j] / mm * nX
                gm[j] += nm + (np.abs(x[j] - com) * nX).sum() / mm
                if eps is not None:
                    gm[j] += ne2 * abs(eb2[j] - e2) / mm
    return gx, gm


def pin_vjp_abs_set_based():
    """The oracle's VJP error scale equals the one built from the set
    definition (nodes accepted, leaf pairs, hand-down to members)."""
    rng = np.random.default_rng(26)
    for x, theta, leaf, per_body in ((ics.uniform_ball(150, seed=5).pos, 0.7, 2, True),
                                     (ics.plummer(120, seed=6).pos, 0.5, 1, False)):
        n = len(x)
        m = rng.random(n) + 0.2
        eps = 0.02 + 0.02 * rng.random(n) if per_body else None
        lam = rng.standard_normal((n, 3))
        ax, am = oracle.tree_vjp_abs(x, m, lam, theta, softening=0.01, eps=eps, leaf=leaf, G=1.1)
        sx, sm = set_based_vjp_abs(x, m, lam, theta, leaf, softening=0.01, eps=eps, G=1.1)
        np.testing.assert_allclose(ax, sx, rtol=1e-12)
        np.testing.assert_allclose(am, sm, rtol=1e-12)


def pin_vjp_abs_bounds_vjp():
    """Every output of the VJP's error scale bounds the VJP's absolute value
    (tree with nodes, per-body softening), the scale does not depend on the
    sign of lambda and is linear in its size."""
    s = ics.rubble_pile(600, seed=25)
    rng = np.random.default_rng(25)
    lam = rng.standard_normal((600, 3))
    gx, gm = oracle.tree_vjp(s.pos, s.mass, lam, 0.6, eps=s.eps, leaf=4)
    ax, am = oracle.tree_vjp_abs(s.pos, s.mass, lam, 0.6, eps=s.eps, leaf=4)
    assert np.all(np.abs(gx) <= ax) and np.all(np.abs(gm) <= am)
    assert np.median(np.abs(gx) / ax) < 0.5  # terms of both signs: a real bound, not |g| itself
    bx, bm = oracle.tree_vjp_abs(s.pos, s.mass, -2.0 * lam, 0.6, eps=s.eps, leaf=4)
    np.testing.assert_allclose(bx, 2.0 * ax, rtol=1e-14)
    np.testing.assert_allclose(bm, 2.0 * am, rtol=1e-14)


def pin_vjp_theta_zero_is_direct():
    x, m, eps, lam, _ = _fd_case(seed=24, n=300)
    for e in (None, eps):
        gd = oracle.direct_vjp(x, m, lam, softening=0.01, eps=e)
        gt = oracle.tree_vjp(x, m, lam, 0.0, softening=0.01, eps=e, leaf=3)
        np.testing.assert_allclose(gt[0], gd[0], rtol=1e-11, atol=1e-11 * np.abs(gd[0]).max())
        np.testing.assert_allclose(gt[1], gd[1], rtol=1e-11, atol=1e-11 * np.abs(gd[1]).max())


def pin_vjp_direct_torch_autograd():
    """Direct VJP against torch autograd of an all-pairs FP64 force (CPU)."""
    import torch

    x, m, eps, lam, _ = _fd_case(seed=25, n=120)
    xt = torch.tensor(x, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    e = torch.tensor(eps)
    d = xt[None, :, :] - xt[:, None, :]
    r2 = (d * d).sum(-1) + 0.5 * (e[:, None] ** 2 + e[None, :] ** 2)
    eye = torch.eye(len(x), dtype=torch.bool)
    inv3 = torch.where(eye, torch.zeros_like(r2), r2.clamp_min(1e-300) ** -1.5)
    acc = (mt[None, :, None] * d * inv3[..., None]).sum(1)
    (acc * torch.tensor(lam)).sum().backward()
    gx, gm = oracle.direct_vjp(x, m, lam, eps=eps)
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(gx).max())
    np.testing.assert_allclose(gm, mt.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(gm).max())


def _rollout_case():
    s = ics.plummer(40, seed=26)
    rng = np.random.default_rng(26)
    m = s.mass * (1.0 + rng.random(40))
    xt = s.pos + 0.01 * rng.standard_normal(s.pos.shape)
    return s, m, xt, rng


def pin_rollout_grad_finite_differences():
    """Reverse-mode rollout gradient against central differences of
    L = sum |x_T - x*|^2 + 0.3 sum |v_T|^2 through 10 KDK steps."""
    s, m, xt, rng = _rollout_case()
    dt, T, soft = 2e-3, 10, 0.05
    for theta in (-1.0, 0.6):
        def loss(x0, v0, mm):
            x, v, _ = oracle.leapfrog(x0, v0, mm, dt, T, softening=soft, theta=theta, leaf=4)
            return float(((x - xt) ** 2).sum() + 0.3 * (v ** 2).sum())
        x, v, _ = oracle.leapfrog(s.pos, s.vel, m, dt, T, softening=soft, theta=theta, leaf=4)
        gx, gv, gm = oracle.rollout_grad(s.pos, s.vel, m, dt, T, 2 * (x - xt), 0.6 * v,
                                         softening=soft, theta=theta, leaf=4)
        for (i, a) in [(3, 0), (21, 1), (39, 2)]:
            for arr, g in ((s.pos, gx), (s.vel, gv)):
                h = 1e-6
                p, q = arr.copy(), arr.copy()
                p[i, a] += h
                q[i, a] -= h
                if arr is s.pos:
                    fd = (loss(p, s.vel, m) - loss(q, s.vel, m)) / (2 * h)
                else:
                    fd = (loss(s.pos, p, m) - loss(s.pos, q, m)) / (2 * h)
                assert abs(g[i, a] - fd) <= 1e-5 * max(abs(fd), 1e-4), (theta, i, a, g[i, a], fd)
        for i in (2, 30):
            h = 1e-4 * m[i]
            p, q = m.copy(), m.copy()
            p[i] += h
            q[i] -= h
            fd = (loss(s.pos, s.vel, p) - loss(s.pos, s.vel, q)) / (2 * h)
            assert abs(gm[i] - fd) <= 1e-4 * max(abs(fd), 1e-4), (theta, i, gm[i], fd)


def pin_rollout_grad_torch_autograd():
    """Direct-sum rollout gradient against torch autograd of the same KDK
    steps written with torch FP64 CPU ops."""
    import torch

    s, m, xt, _ = _rollout_case()
    dt, T, soft = 2e-3, 8, 0.05
    x0 = torch.tensor(s.pos, requires_grad=True)
    v0 = torch.tensor(s.vel, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)

    def accel(x):
        d = x[None, :, :] - x[:, None, :]
        inv3 = ((d * d).sum(-1) + soft * soft) ** -1.5
        inv3 = inv3 * (1 - torch.eye(len(m), dtype=x.dtype))
        return (mt[None, :, None] * d * inv3[..., None]).sum(1)

    x, v, a = x0, v0, accel(x0)
    for _ in range(T):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = accel(x)
        v = v + 0.5 * dt * a
    loss = ((x - torch.tensor(xt)) ** 2).sum() + 0.3 * (v ** 2).sum()
    loss.backward()
    xf, vf, _ = oracle.leapfrog(s.pos, s.vel, m, dt, T, softening=soft)
    gx, gv, gm = oracle.rollout_grad(s.pos, s.vel, m, dt, T, 2 * (xf - xt), 0.6 * vf,
                                     softening=soft)
    np.testing.assert_allclose(gx, x0.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gv, v0.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gm, mt.grad.numpy(), rtol=1e-9, atol=1e-12)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
