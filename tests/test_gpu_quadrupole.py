"""Quadrupole nodes (an optional refinement beyond the paper's monopoles)
against the oracle's quadrupole walk.

Bars: node quadrupoles to 1e-12 of m_N s_N^2 (the GPU shifts the children's
moments to the parent, the oracle sums each node's bodies); accelerations as
for the monopole walk (FP64 1e-12 A_i, FP32C 64u A_i), counts exact (the
opening decisions do not change).
"""
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


@pytest.mark.parametrize("n,leaf", [(3000, 4), (40000, 16)])
def test_node_quadrupoles(api, n, leaf):
    s = ics.plummer(n, seed=51)
    m = s.mass * (1.0 + (np.arange(n) % 3))
    T = oracle.Tree(s.pos, m, leaf=leaf)
    ref, q_ref, L = T.export(), T.quadrupoles(), T.box()["L"]
    ctx = api.Context(n, leaf_size=leaf, precision="fp64", quad=True)
    ctx.build_tree(_dev(s.pos), _dev(m))
    v = ctx.tree()
    info = v.info.cpu().numpy()
    q = v.quad.cpu().numpy()
    gpu = {(int(l), int(f), int(c)): k for k, (l, f, c) in
           enumerate(zip(info[:, 3] & 0xFF, info[:, 0], info[:, 1]))}
    for ko, key in enumerate(zip(ref["level"], ref["first"], ref["count"])):
        kg = gpu[tuple(int(x) for x in key)]
        scale = ref["mass"][ko] * (L / 2.0 ** key[0]) ** 2
        assert np.abs(q[kg] - q_ref[ko]).max() <= 1e-12 * scale + 1e-300, key


CASES = [
    ("ball4096_t0.7_l8", lambda: ics.uniform_ball(4096, seed=52), 0.7, 8, 1e-3, False),
    ("plummer20000_t0.5_l16", lambda: ics.plummer(20000, seed=53), 0.5, 16, 1e-3, False),
    ("rubble30000_t0.5_l16_eps", lambda: ics.rubble_pile(30000, seed=54), 0.5, 16, 0.0, True),
]


@pytest.mark.parametrize("group", [16, 64])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("name,make,theta,leaf,soft,per_body", CASES, ids=[c[0] for c in CASES])
def test_quadrupole_walk_parity(api, name, make, theta, leaf, soft, per_body, precision, group):
    s = make()
    eps = s.eps if per_body else None
    ref, ref_phi, aabs, ref_cnt = oracle.bh(s.pos, s.mass, theta, softening=soft, eps=eps,
                                            leaf=leaf, quad=True)
    ctx = api.Context(s.n, leaf_size=leaf, precision=precision, counts=True, walk_group=group,
                      quad=True)
    acc, phi = ctx.compute_accel(_dev(s.pos), _dev(s.mass), theta, softening=soft,
                                 eps=None if eps is None else _dev(eps), potential=True)
    assert np.array_equal(ctx.walk_counts(s.n).cpu().numpy(), ref_cnt)
    tol = 1e-12 if precision == "fp64" else 64 * 2.0 ** -24
    err = np.linalg.norm(acc.cpu().numpy() - ref, axis=1)
    assert np.all(err <= tol * aabs), (err / aabs).max()
    perr = np.abs(phi.cpu().numpy() - ref_phi)
    assert np.all(perr <= tol * np.abs(ref_phi) * 4), (perr / np.abs(ref_phi)).max()


def test_quadrupole_vjp_rejected(api):
    ctx = api.Context(100, quad=True, adjoint=True)
    z = torch.zeros((100, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(api.BHError, match="BH_E_STATE"):
        ctx.accel_vjp(z, torch.ones(100, dtype=torch.float64, device="cuda"), z, theta=0.5)
