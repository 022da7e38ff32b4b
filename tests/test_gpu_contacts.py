"""Aggregate identification on the GPU against the oracle: the contact graph
of spheres and its connected components. Integer results, so the bar is
exact: every label (the smallest index of the body's component), the number
of contact pairs and the number of aggregates."""
import numpy as np
import pytest

import oracle
from paper_1912_04197_amd import ics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_1912_04197_amd import api as A

    return A


def _random_spheres(n, seed, rmax):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)), rmax * (0.3 + 0.7 * rng.random(n))


def _chain(n):
    # touching spheres along a helix: one long component, unions deep chains
    t = np.arange(n) * 0.05
    pos = np.stack([np.cos(t), np.sin(t), 0.01 * t], 1)
    step = np.linalg.norm(pos[1] - pos[0])
    return pos, np.full(n, 0.5 * step)


CASES = [
    ("random3000_sparse", lambda: _random_spheres(3000, 71, 0.01), 0.0),
    ("random6000_dense", lambda: _random_spheres(6000, 72, 0.03), 0.0),
    ("random5000_skin", lambda: _random_spheres(5000, 73, 0.01), 0.01),
    ("chain2000", lambda: _chain(2000), 0.0),
    ("rubble20000_x3", lambda: (ics.rubble_pile(20000, seed=74).pos,
                                3.0 * ics.rubble_pile(20000, seed=74).eps), 0.0),
    ("coincident", lambda: (np.repeat(np.random.default_rng(75).random((50, 3)), 20, 0),
                            np.full(1000, 1e-4)), 0.0),
    ("single", lambda: (np.zeros((1, 3)), np.ones(1)), 0.0),
]


@pytest.mark.parametrize("name,make,skin", CASES, ids=[c[0] for c in CASES])
def test_contact_components_parity(api, name, make, skin):
    pos, r = make()
    n = len(r)
    label_ref, nc_ref, na_ref = oracle.contact_components(pos, r, skin)
    ctx = api.Context(n)
    label, nc, na = ctx.contact_components(_dev(pos), _dev(np.ones(n) / n), _dev(r), skin)
    assert nc == nc_ref and na == na_ref, (nc, nc_ref, na, na_ref)
    assert np.array_equal(label.cpu().numpy(), label_ref)


def test_contact_components_large_properties(api):
    """2^20-body rubble pile with radii x4: every contact pair of 512 sampled
    bodies (brute force over all bodies) has equal labels, labels are roots
    (label[label[i]] == label[i] <= i), and repeated calls agree exactly."""
    s = ics.rubble_pile(1 << 20, seed=33)
    r = 4.0 * s.eps
    ctx = api.Context(s.n)
    P, M, R = _dev(s.pos), _dev(s.mass), _dev(r)
    label, nc, na = ctx.contact_components(P, M, R)
    lab = label.cpu().numpy()
    assert nc > 0 and na > 0
    idx = np.arange(s.n)
    assert np.all(lab <= idx) and np.array_equal(lab[lab], lab)
    rng = np.random.default_rng(76)
    for i in rng.choice(s.n, 512, replace=False):
        d2 = ((s.pos - s.pos[i]) ** 2).sum(1)
        rr = r + r[i]
        j = np.nonzero(d2 <= rr * rr)[0]
        assert np.all(lab[j] == lab[i]), i
    label2, nc2, na2 = ctx.contact_components(P, M, R)
    assert nc2 == nc and na2 == na and torch.equal(label, label2)
