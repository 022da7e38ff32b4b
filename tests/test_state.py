"""Checkpoint files: save_state/load_state round-trip FP64 state bit for bit
and refuse what they did not write. Host-side IO only (CPU tensors)."""
import numpy as np
import pytest
import torch

from paper_1912_04197_amd import api, ics


def _state(n=257, seed=3):
    s = ics.plummer(n, seed=seed)
    rng = np.random.default_rng(seed)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    return (t(s.pos), t(s.vel), t(s.mass), t(rng.standard_normal((n, 3))),
            t(rng.uniform(1e-3, 1e-2, n)))


def test_round_trip_bit_exact(tmp_path):
    pos, vel, mass, acc, eps = _state()
    pos[0, 0] = np.nextafter(1.0, 2.0)  # one ulp above 1 survives
    vel[1, 2] = 5e-324                   # a subnormal survives
    path = api.save_state(tmp_path / "ck", pos, vel, mass, acc=acc, eps=eps, t=0.125, step=17,
                          theta=0.5)
    assert path.endswith(".npz")
    arrays, meta = api.load_state(path, device="cpu")
    assert meta == {"t": 0.125, "step": 17, "theta": 0.5}
    for k, want in (("pos", pos), ("vel", vel), ("mass", mass), ("acc", acc), ("eps", eps)):
        got = arrays[k]
        assert got.dtype == torch.float64
        assert np.array_equal(got.numpy().view(np.uint64), want.numpy().view(np.uint64)), k
    assert [p.name for p in tmp_path.iterdir()] == ["ck.npz"]  # no temporary left behind


def test_optional_arrays_absent(tmp_path):
    pos, vel, mass, _, _ = _state(31)
    arrays, meta = api.load_state(api.save_state(tmp_path / "a.npz", pos, vel, mass),
                                  device="cpu")
    assert sorted(arrays) == ["mass", "pos", "vel"] and meta == {}


def test_save_overwrites_previous(tmp_path):
    pos, vel, mass, _, _ = _state(40)
    p = api.save_state(tmp_path / "c.npz", pos, vel, mass, step=1)
    api.save_state(p, pos + 1.0, vel, mass, step=2)
    arrays, meta = api.load_state(p, device="cpu")
    assert meta["step"] == 2 and torch.equal(arrays["pos"], pos + 1.0)


@pytest.mark.parametrize("bad", ["dtype", "shape"])
def test_save_rejects_bad_arrays(tmp_path, bad):
    pos, vel, mass, _, _ = _state(20)
    if bad == "dtype":
        pos = pos.float()
    else:
        vel = vel[:10]
    with pytest.raises(ValueError):
        api.save_state(tmp_path / "x.npz", pos, vel, mass)


def test_load_refuses_foreign_files(tmp_path):
    f = tmp_path / "other.npz"
    np.savez(f, pos=np.zeros((3, 3)), vel=np.zeros((3, 3)), mass=np.ones(3))
    with pytest.raises(ValueError):
        api.load_state(f, device="cpu")
    g = tmp_path / "obj.npz"
    np.savez(g, format=np.array("bhx-state-1"), meta=np.array("{}"),
             pos=np.array([object()], dtype=object))
    with pytest.raises(ValueError):  # object arrays would need unpickling: refused
        api.load_state(g, device="cpu")
