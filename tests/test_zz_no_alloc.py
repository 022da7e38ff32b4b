"""The entry point that allocates nothing (bh_compute_accel_direct_noalloc)
against bh_compute_accel_direct on the same inputs, through the C ABI: two
calls in a row, the second on fewer bodies, so the second reuses the
library's per-device partial-sum array after the first filled it."""
import numpy as np
import pytest

from paper_1912_04197_amd import ics

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(n, seed, per_body_eps):
    s = ics.rubble_pile(n, seed=seed) if per_body_eps else ics.uniform_ball(n, seed=seed)
    dev = torch.device("cuda", 0)
    p = torch.from_numpy(s.pos).to(dev)
    m = torch.from_numpy(s.mass).to(dev)
    e = torch.from_numpy(np.ascontiguousarray(s.eps, dtype=np.float64)).to(dev) if per_body_eps else None
    return p, m, e


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("per_body_eps", [False, True])
def test_noalloc_matches_direct(precision, per_body_eps):
    from paper_1912_04197_amd.api import Context, compute_accel_direct_noalloc

    ctx = Context(6000, precision=precision)
    for n, seed in ((5003, 91), (1777, 92)):  # several block rows of partial sums each
        p, m, e = _case(n, seed, per_body_eps)
        soft = 0.0 if per_body_eps else 1e-3
        ref, ref_phi = ctx.compute_accel_direct(p, m, softening=soft, eps=e, potential=True)
        out = torch.full((n, 3), float("nan"), dtype=torch.float64, device=p.device)
        phi = torch.full((n,), float("nan"), dtype=torch.float64, device=p.device)
        compute_accel_direct_noalloc(p, m, softening=soft, eps=e, precision=precision, out=out,
                                     phi=phi)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical results
        assert torch.equal(out, ref), f"n={n}: accelerations differ"
        assert torch.equal(phi, ref_phi), f"n={n}: potentials differ"


def test_noalloc_rejects_bad_arguments():
    from paper_1912_04197_amd import _lib as L

    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    dev = torch.device("cuda", 0)
    p = torch.zeros((4, 3), dtype=torch.float64, device=dev)
    m = torch.ones(4, dtype=torch.float64, device=dev)
    a = torch.zeros((4, 3), dtype=torch.float64, device=dev)
    import ctypes as C
    P = lambda t: C.c_void_p(t.data_ptr())
    assert lib.bh_compute_accel_direct_noalloc(C.c_void_p(stream), L.BH_FP64, 1.0, P(p), P(m), 0.0,
                                               None, P(a), None, (1 << 30) + 1) == L.BH_E_CAPACITY
    assert lib.bh_compute_accel_direct_noalloc(C.c_void_p(stream), 7, 1.0, P(p), P(m), 0.0,
                                               None, P(a), None, 4) == L.BH_E_INVALID
    assert lib.bh_compute_accel_direct_noalloc(C.c_void_p(stream), L.BH_FP64, 1.0, P(p), P(m), -1.0,
                                               None, P(a), None, 4) == L.BH_E_INVALID
    assert lib.bh_compute_accel_direct_noalloc(C.c_void_p(stream), L.BH_FP64, 1.0, None, P(m), 0.0,
                                               None, P(a), None, 4) == L.BH_E_INVALID
    assert lib.bh_compute_accel_direct_noalloc(C.c_void_p(stream), L.BH_FP64, 1.0, None, None, 0.0,
                                               None, None, None, 0) == L.BH_OK
