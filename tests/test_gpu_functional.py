"""The package-level functional forms (compute_accel, compute_accel_direct,
step_leapfrog): the same library calls as a Context, so bit-identical to it,
and within the parity bars of the oracle (FP32C 64u A_i)."""
import numpy as np
import pytest

import oracle
from paper_1912_04197_amd import ics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP32C_TOL = 64 * 2.0 ** -24


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1912_04197_amd as P

    return P


def test_functional_accel_matches_context_and_oracle(P):
    s = ics.uniform_ball(5000, seed=61)
    p, m = _dev(s.pos), _dev(s.mass)
    a = P.compute_accel(p, m, 1e-3, 0.5).cpu().numpy()
    ctx = P.Context(5000, leaf_size=16, precision="fp32c")
    a_ctx = ctx.compute_accel(p, m, 0.5, softening=1e-3).cpu().numpy()
    assert np.array_equal(a, a_ctx)
    ref, _, aabs, _ = oracle.bh(s.pos, s.mass, 0.5, softening=1e-3, leaf=16)
    assert np.all(np.linalg.norm(a - ref, axis=1) <= FP32C_TOL * aabs)
    # a larger call grows the cached context; a smaller one reuses it
    s2 = ics.uniform_ball(3000, seed=62)
    b = P.compute_accel(_dev(s2.pos), _dev(s2.mass), 1e-3, 0.5).cpu().numpy()
    ref2, _, aabs2, _ = oracle.bh(s2.pos, s2.mass, 0.5, softening=1e-3, leaf=16)
    assert np.all(np.linalg.norm(b - ref2, axis=1) <= FP32C_TOL * aabs2)


def test_functional_direct_and_leapfrog(P):
    s = ics.plummer(2048, seed=63)
    p, v, m = _dev(s.pos), _dev(s.vel), _dev(s.mass)
    d = P.compute_accel_direct(p, m, 1e-3, precision="fp64").cpu().numpy()
    ref, _, aabs = oracle.direct(s.pos, s.mass, softening=1e-3)
    assert np.all(np.linalg.norm(d - ref, axis=1) <= 1e-12 * aabs)
    ctx = P.Context(2048, leaf_size=16, precision="fp32c")
    p1, v1 = p.clone(), v.clone()
    a0 = P.compute_accel(p, m, 1e-3, 0.5)
    a1 = ctx.compute_accel(p1, m, 0.5, softening=1e-3)
    P.step_leapfrog(p, v, m, a0, 1e-3, 5, theta=0.5, softening=1e-3)
    ctx.step_leapfrog(p1, v1, m, a1, 1e-3, 5, theta=0.5, softening=1e-3)
    assert torch.equal(p, p1) and torch.equal(v, v1) and torch.equal(a0, a1)


def test_probe_fma_rates(P):
    """The measured FMA rates are positive and within the datasheet peaks
    (FP32 non-packed issues at the FP64 rate: half the packed 157.3)."""
    fp32 = P.probe_fma("fp32", iters=4096)
    fp64 = P.probe_fma("fp64", iters=4096)
    assert 5.0 < fp32 <= 1.05 * 157.3 / 2
    assert 5.0 < fp64 <= 1.05 * 78.6
