"""The checked library (libbhx_checked.so: the same kernels with device-side
invariant checks that latch a status bit instead of stopping) runs a workload
touching every kernel family without a failed check, and computes what the
release library computes: bit for bit wherever the release results are
deterministic, and the force VJPs (FP64 atomics in any order) to 1e-10."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_checked_build_matches_release(tmp_path):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    out = tmp_path / "checked.npz"
    env = dict(os.environ, BHX_LIBRARY="checked", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, os.path.join(HERE, "_checked_workload.py"), str(out)],
                       env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    sys.path.insert(0, HERE)
    import _checked_workload as W
    from paper_1912_04197_amd import api

    ref = W.run(api)
    got = np.load(out)
    assert bool(got["bucket"][0])
    for k, v in ref.items():
        if k.startswith("vjp_") or k.startswith("seg_"):
            assert np.abs(got[k] - v).max() <= 1e-10 * np.abs(v).max(), k
        else:
            assert np.array_equal(got[k], v), k
