"""Python entry points over libbhx: torch tensors in, torch tensors out.

torch supplies device memory and the current HIP stream; every step of the
computation runs in the library's HIP kernels. There is no CPU fallback: a
missing library or a non-GPU tensor raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


_hip = None


def _hip_copy_d2d(dst: int, src: int, nbytes: int):
    """Synchronous device-to-device copy through the HIP runtime."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


class BHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = L.STATUS_NAMES[status] if 0 <= status < len(L.STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_f64(name, t, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64 (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class TreeView:
    n: int
    nnodes: int
    depth: int
    info: torch.Tensor   # (nnodes, 4) int32: first, count, child0, level | nchild << 8
    mom: torch.Tensor    # (nnodes, 4) float64: com x, y, z, mass
    eps2: torch.Tensor | None
    order: torch.Tensor  # (n,) int64 caller index of each sorted body
    keys: torch.Tensor   # (n,) int64 Morton keys
    box: list
    quad: torch.Tensor | None = None  # (nnodes, 6) xx, yy, zz, xy, xz, yz with quad=True


class Context:
    """One library context: workspace for up to ``n_max`` bodies on the current device.

    precision: "fp64" (all FP64) or "fp32c" (FP32 pair terms with FP32 partial
    sums flushed to FP64, FP64 state and opening test).
    """

    def __init__(self, n_max: int, leaf_size: int = 16, precision: str = "fp32c", G: float = 1.0,
                 counts: bool = False, timing: bool = False, walk_group: int = 0,
                 adjoint: bool = False, max_scenes: int = 1, graph: bool = False,
                 quad: bool = False, markers: bool = False):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libbhx runs on the GPU only")
        prec = {"fp64": L.BH_FP64, "fp32c": L.BH_FP32C}[precision]
        flags = ((L.BH_FLAG_COUNTS if counts else 0) | (L.BH_FLAG_TIMING if timing else 0)
                 | (L.BH_FLAG_ADJOINT if adjoint else 0) | (L.BH_FLAG_GRAPH if graph else 0)
                 | (L.BH_FLAG_QUAD if quad else 0) | (L.BH_FLAG_MARKERS if markers else 0))
        cfg = L.bh_config(int(n_max), int(leaf_size), prec, float(G), flags, int(walk_group),
                          int(max_scenes))
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.n_max, self.leaf_size, self.precision, self.G = int(n_max), int(leaf_size), precision, float(G)
        h = C.c_void_p()
        rc = self._lib.bh_create(C.byref(cfg), C.c_void_p(self._stream()), C.byref(h))
        if rc != 0:
            raise BHError(rc, "bh_create failed")
        self._h = h

    # -- plumbing
    def _stream(self) -> int:
        return torch.cuda.current_stream().cuda_stream

    def _bind(self):
        self._lib.bh_set_stream(self._h, C.c_void_p(self._stream()))

    def _rc(self, rc):
        if rc != 0:
            raise BHError(rc, self._lib.bh_last_error(self._h).decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.bh_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        """Waits for queued work and raises on a latched device error."""
        self._rc(self._lib.bh_sync(self._h))

    def _bodies(self, pos, mass, eps):
        n = int(pos.shape[0]) if pos.dim() == 2 else -1
        _check_f64("pos", pos, (n, 3), self.device)
        _check_f64("mass", mass, (n,), self.device)
        if eps is not None:
            _check_f64("eps", eps, (n,), self.device)
        return n

    # -- entry points
    def build_tree(self, pos, mass, eps=None, sync=True):
        n = self._bodies(pos, mass, eps)
        self._bind()
        self._rc(self._lib.bh_build_tree(self._h, _ptr(pos), _ptr(mass), _ptr(eps), n))
        if sync:
            self.sync()

    def compute_accel(self, pos, mass, theta, softening=0.0, eps=None, out=None, potential=False,
                      sync=True):
        """Barnes-Hut accelerations (n, 3); with potential=True returns (acc, phi)."""
        n = self._bodies(pos, mass, eps)
        acc = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device=self.device)
        _check_f64("out", acc, (n, 3), self.device)
        phi = torch.empty(n, dtype=torch.float64, device=self.device) if potential else None
        self._bind()
        self._rc(self._lib.bh_compute_accel(self._h, _ptr(pos), _ptr(mass), float(softening),
                                            _ptr(eps), float(theta), _ptr(acc), _ptr(phi), n))
        if sync:
            self.sync()
        return (acc, phi) if potential else acc

    def compute_accel_direct(self, pos, mass, softening=0.0, eps=None, out=None, potential=False,
                             sync=True):
        """Direct N^2 accelerations (n, 3); with potential=True returns (acc, phi)."""
        n = self._bodies(pos, mass, eps)
        acc = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device=self.device)
        _check_f64("out", acc, (n, 3), self.device)
        phi = torch.empty(n, dtype=torch.float64, device=self.device) if potential else None
        self._bind()
        self._rc(self._lib.bh_compute_accel_direct(self._h, _ptr(pos), _ptr(mass), float(softening),
                                                   _ptr(eps), _ptr(acc), _ptr(phi), n))
        if sync:
            self.sync()
        return (acc, phi) if potential else acc

    def step_leapfrog(self, pos, vel, mass, acc, dt, nsteps, theta=0.5, softening=0.0, eps=None,
                      sync=True):
        """nsteps KDK steps in place on pos, vel and acc (theta < 0: direct sum)."""
        n = self._bodies(pos, mass, eps)
        _check_f64("vel", vel, (n, 3), self.device)
        _check_f64("acc", acc, (n, 3), self.device)
        self._bind()
        self._rc(self._lib.bh_step_leapfrog(self._h, _ptr(pos), _ptr(vel), _ptr(mass),
                                            float(softening), _ptr(eps), float(theta), float(dt),
                                            int(nsteps), _ptr(acc), n))
        if sync:
            self.sync()

    def step_euler(self, pos, vel, mass, acc, dt, nsteps, every=1, theta=0.5, softening=0.0,
                   eps=None, sync=True):
        """nsteps semi-implicit Euler substeps in place, gravity re-evaluated
        after every `every`-th one (see bh_step_euler; theta < 0: direct sum)."""
        n = self._bodies(pos, mass, eps)
        _check_f64("vel", vel, (n, 3), self.device)
        _check_f64("acc", acc, (n, 3), self.device)
        self._bind()
        self._rc(self._lib.bh_step_euler(self._h, _ptr(pos), _ptr(vel), _ptr(mass),
                                         float(softening), _ptr(eps), float(theta), float(dt),
                                         int(nsteps), int(every), _ptr(acc), n))
        if sync:
            self.sync()

    def contact_components(self, pos, mass, radius, skin=0.0):
        """(label (n,) int32 tensor, n_contacts, n_aggregates); see
        bh_contact_components."""
        n = self._bodies(pos, mass, radius)
        label = torch.empty(n, dtype=torch.int32, device=self.device)
        nc, na = C.c_int64(0), C.c_int64(0)
        self._bind()
        self._rc(self._lib.bh_contact_components(self._h, _ptr(pos), _ptr(mass), _ptr(radius),
                                                 float(skin), _ptr(label), C.byref(nc),
                                                 C.byref(na), n))
        return label, int(nc.value), int(na.value)

    @staticmethod
    def _offsets(offsets):
        o = np.ascontiguousarray(offsets, dtype=np.int64)
        return o, int(o.shape[0]) - 1

    def batched_accel(self, offsets, pos, mass, theta, softening=0.0, eps=None, out=None,
                      potential=False, sync=True):
        """Per-scene Barnes-Hut accelerations of scenes stored back to back;
        offsets (host, n_scenes + 1) delimit the scenes."""
        o, ns = self._offsets(offsets)
        n = self._bodies(pos, mass, eps)
        if int(o[-1]) != n:
            raise ValueError("offsets[-1] must equal the number of bodies")
        acc = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device=self.device)
        _check_f64("out", acc, (n, 3), self.device)
        phi = torch.empty(n, dtype=torch.float64, device=self.device) if potential else None
        self._bind()
        self._rc(self._lib.bh_batched_accel(self._h, ns, o.ctypes.data_as(C.c_void_p), _ptr(pos),
                                            _ptr(mass), float(softening), _ptr(eps), float(theta),
                                            _ptr(acc), _ptr(phi)))
        if sync:
            self.sync()
        return (acc, phi) if potential else acc

    def batched_step(self, offsets, pos, vel, mass, acc, dt, nsteps, theta=0.5, softening=0.0,
                     eps=None, sync=True):
        """nsteps KDK steps of every scene, in place (see bh_batched_step)."""
        o, ns = self._offsets(offsets)
        n = self._bodies(pos, mass, eps)
        if int(o[-1]) != n:
            raise ValueError("offsets[-1] must equal the number of bodies")
        _check_f64("vel", vel, (n, 3), self.device)
        _check_f64("acc", acc, (n, 3), self.device)
        self._bind()
        self._rc(self._lib.bh_batched_step(self._h, ns, o.ctypes.data_as(C.c_void_p), _ptr(pos),
                                           _ptr(vel), _ptr(mass), float(softening), _ptr(eps),
                                           float(theta), float(dt), int(nsteps), _ptr(acc)))
        if sync:
            self.sync()

    def accel_vjp(self, pos, mass, lam, theta=0.5, softening=0.0, eps=None, g_pos=None,
                  g_mass=None, sync=True):
        """Adds the gradient of sum lam_i . a_i into (g_pos, g_mass) and returns them
        (new zero tensors when not given). theta < 0: direct sum."""
        n = self._bodies(pos, mass, eps)
        _check_f64("lam", lam, (n, 3), self.device)
        g_pos = torch.zeros((n, 3), dtype=torch.float64, device=self.device) if g_pos is None else g_pos
        g_mass = torch.zeros(n, dtype=torch.float64, device=self.device) if g_mass is None else g_mass
        _check_f64("g_pos", g_pos, (n, 3), self.device)
        _check_f64("g_mass", g_mass, (n,), self.device)
        self._bind()
        self._rc(self._lib.bh_accel_vjp(self._h, _ptr(pos), _ptr(mass), float(softening), _ptr(eps),
                                        float(theta), _ptr(lam), _ptr(g_pos), _ptr(g_mass), n))
        if sync:
            self.sync()
        return g_pos, g_mass

    def leapfrog_vjp(self, pos, vel, acc, mass, dt, nsteps, traj, xbar, vbar, abar, g_mass,
                     theta=0.5, softening=0.0, eps=None, sync=True):
        """Backward over one checkpoint segment (see bh_leapfrog_vjp); updates
        xbar, vbar, abar in place and adds into g_mass."""
        n = self._bodies(pos, mass, eps)
        for name, t in (("vel", vel), ("acc", acc), ("xbar", xbar), ("vbar", vbar), ("abar", abar)):
            _check_f64(name, t, (n, 3), self.device)
        _check_f64("g_mass", g_mass, (n,), self.device)
        if nsteps > 0:
            if traj.dtype != torch.float64 or not traj.is_contiguous() or traj.numel() < nsteps * n * 3:
                raise ValueError("traj must be a contiguous float64 GPU buffer of nsteps x n x 3")
        self._bind()
        self._rc(self._lib.bh_leapfrog_vjp(self._h, _ptr(pos), _ptr(vel), _ptr(acc), _ptr(mass),
                                           float(softening), _ptr(eps), float(theta), float(dt),
                                           int(nsteps), _ptr(traj), _ptr(xbar), _ptr(vbar),
                                           _ptr(abar), _ptr(g_mass), n))
        if sync:
            self.sync()

    def leapfrog_vjp_stored(self, traj, mass, dt, nsteps, xbar, vbar, abar, g_mass, theta=0.5,
                            softening=0.0, eps=None, sync=True):
        """Backward over nsteps steps whose end positions traj[0..nsteps) the
        caller kept (see bh_leapfrog_vjp_stored); no recomputation."""
        n = int(mass.shape[0])
        _check_f64("mass", mass, (n,), self.device)
        if eps is not None:
            _check_f64("eps", eps, (n,), self.device)
        for name, t in (("xbar", xbar), ("vbar", vbar), ("abar", abar)):
            _check_f64(name, t, (n, 3), self.device)
        _check_f64("g_mass", g_mass, (n,), self.device)
        if (traj.dtype != torch.float64 or not traj.is_contiguous() or traj.device != self.device
                or traj.numel() < max(nsteps, 1) * n * 3):
            raise ValueError("traj must be a contiguous float64 GPU tensor of nsteps x n x 3")
        self._bind()
        self._rc(self._lib.bh_leapfrog_vjp_stored(self._h, _ptr(traj), _ptr(mass),
                                                  float(softening), _ptr(eps), float(theta),
                                                  float(dt), int(nsteps), _ptr(xbar), _ptr(vbar),
                                                  _ptr(abar), _ptr(g_mass), n))
        if sync:
            self.sync()

    def walk_counts(self, n):
        """(n, 2) int32 per-body counts of the last tree walk: accepted nodes, leaf pairs."""
        out = torch.empty((n, 2), dtype=torch.int32, device=self.device)
        self._bind()
        self._rc(self._lib.bh_walk_counts(self._h, _ptr(out), int(n)))
        self.sync()
        return out

    def tree(self) -> TreeView:
        """Copies of the last built tree (synchronises)."""
        self._bind()
        v = L.bh_tree_view()
        self._rc(self._lib.bh_tree_export(self._h, C.byref(v)))
        nn, n = int(v.nnodes), int(v.n)

        def dev(ptr, count, dtype):
            out = torch.empty(count, dtype=dtype, device=self.device)
            if count:
                torch.cuda.synchronize()
                _hip_copy_d2d(out.data_ptr(), ptr, count * out.element_size())
            return out

        info = dev(v.info, 4 * nn, torch.int32).view(nn, 4)
        mom = dev(v.mom, 4 * nn, torch.float64).view(nn, 4)
        eps2 = dev(v.eps2, nn, torch.float64) if v.eps2 else None
        order = dev(v.order, n, torch.int32).to(torch.int64) & 0xFFFFFFFF
        keys = dev(v.keys, n, torch.int64)
        quad = dev(v.quad, 6 * nn, torch.float64).view(nn, 6) if v.quad else None
        return TreeView(n, nn, int(v.depth), info, mom, eps2, order, keys, list(v.box), quad)

    def stats(self) -> dict:
        s = L.bh_stats_t()
        self._bind()
        self._rc(self._lib.bh_stats(self._h, C.byref(s)))
        return {"nnodes": int(s.nnodes), "depth": int(s.depth),
                "bucket_sort": bool(s.bucket_sort),
                "nodes_accepted": int(s.total_nodes_accepted), "leaf_pairs": int(s.total_leaf_pairs),
                "timed_evals": int(s.timed_evals), "build_ms": float(s.build_ms),
                "walk_ms": float(s.walk_ms)}

    def timing_reset(self):
        self._bind()
        self._rc(self._lib.bh_timing_reset(self._h))

    def gravity_dt_bound(self, mass, radius):
        """Largest gravity time step of eq. (dt_g) for bodies of these masses
        and radii (float64 GPU tensors): 1 / (2 sqrt(G rho)), rho the largest
        body density (see bh_gravity_dt_bound)."""
        n = int(mass.shape[0]) if mass.dim() == 1 else -1
        _check_f64("mass", mass, (n,), self.device)
        _check_f64("radius", radius, (n,), self.device)
        out = C.c_double(0.0)
        self._bind()
        self._rc(self._lib.bh_gravity_dt_bound(self._h, _ptr(mass), _ptr(radius), n,
                                               C.byref(out)))
        return float(out.value)

    def diagnostics(self, pos, vel, mass, softening=0.0, eps=None):
        """[E_kin, E_pot, Px, Py, Pz, Lx, Ly, Lz] (host floats)."""
        n = self._bodies(pos, mass, eps)
        _check_f64("vel", vel, (n, 3), self.device)
        out = (C.c_double * 8)()
        self._bind()
        self._rc(self._lib.bh_diagnostics(self._h, _ptr(pos), _ptr(vel), _ptr(mass),
                                          float(softening), _ptr(eps), out, n))
        return [float(x) for x in out]


def autotune(offsets, pos, vel, mass, theta=0.5, dt=1e-3, softening=0.0, eps=None,
             precision="fp32c", G=1.0, steps=3, quad=False):
    """Fastest (leaf_size, walk_group, ms_per_step) for bh_batched_step on these
    scenes (see bh_autotune); the state tensors are not modified."""
    lib = L.load()
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    ns = int(o.shape[0]) - 1
    n = int(o[-1])
    dev = pos.device
    for name, t, shape in (("pos", pos, (n, 3)), ("vel", vel, (n, 3)), ("mass", mass, (n,))):
        _check_f64(name, t, shape, dev)
    if eps is not None:
        _check_f64("eps", eps, (n,), dev)
    prec = {"fp64": L.BH_FP64, "fp32c": L.BH_FP32C}[precision]
    cfg = L.bh_config(n, 16, prec, float(G), L.BH_FLAG_QUAD if quad else 0, 0, ns)
    out = L.bh_tune_result()
    rc = lib.bh_autotune(C.byref(cfg), C.c_void_p(torch.cuda.current_stream().cuda_stream), ns,
                         o.ctypes.data_as(C.c_void_p), _ptr(pos), _ptr(vel), _ptr(mass),
                         float(softening), _ptr(eps), float(theta), float(dt), int(steps),
                         C.byref(out))
    if rc != 0:
        raise BHError(rc, "bh_autotune failed")
    return int(out.leaf_size), int(out.walk_group), float(out.ms_per_step)


def probe_fma(precision="fp32", iters=65536):
    """Measured vector FMA rate of the current GPU in TFLOP/s (2 flops per
    FMA): 8 independent FMA chains per lane on 8 wavefronts per SIMD, in FP32
    (non-packed) or FP64; the achievable ceiling of VALU-bound kernels."""
    lib = L.load()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libbhx runs on the GPU only")
    prec = {"fp64": L.BH_FP64, "fp32": L.BH_FP32C}[precision]
    out = C.c_double(0.0)
    rc = lib.bh_probe_fma(C.c_void_p(torch.cuda.current_stream().cuda_stream), prec, int(iters),
                          C.byref(out))
    if rc != 0:
        raise BHError(rc, "bh_probe_fma failed")
    return float(out.value)


# -- functional forms: one cached context per (device, leaf, precision, G),
# re-created with a larger workspace when a call needs more bodies
_CONTEXTS: dict = {}


def _context_for(n, leaf, precision, G):
    dev = torch.cuda.current_device()
    key = (dev, int(leaf), precision, float(G))
    ctx = _CONTEXTS.get(key)
    if ctx is None or ctx.n_max < n:
        if ctx is not None:
            ctx.close()
        cap = 1 << max(10, (max(int(n), 1) - 1).bit_length())  # next power of two, >= 1024
        ctx = Context(cap, leaf_size=leaf, precision=precision, G=G)
        _CONTEXTS[key] = ctx
    return ctx


def compute_accel(pos, mass, softening=0.0, theta=0.5, *, eps=None, leaf=16, precision="fp32c",
                  G=1.0, potential=False):
    """Barnes-Hut accelerations of the bodies (pos (n, 3), mass (n,), float64
    on the GPU) with a context cached per device, leaf size, precision and G."""
    ctx = _context_for(pos.shape[0], leaf, precision, G)
    return ctx.compute_accel(pos, mass, theta, softening=softening, eps=eps, potential=potential)


def compute_accel_direct(pos, mass, softening=0.0, *, eps=None, precision="fp32c", G=1.0,
                         potential=False):
    """Direct N^2 accelerations, as compute_accel."""
    ctx = _context_for(pos.shape[0], 16, precision, G)
    return ctx.compute_accel_direct(pos, mass, softening=softening, eps=eps, potential=potential)


def compute_accel_direct_noalloc(pos, mass, softening=0.0, *, eps=None, precision="fp32c",
                                 G=1.0, out=None, phi=None):
    """Direct N^2 accelerations through the entry point that allocates nothing
    on the device (bh_compute_accel_direct_noalloc): no context; the caller
    passes the outputs (out (n, 3) and optionally phi (n,), float64 on the
    GPU) and the library's own per-device array holds the partial sums.
    Queued on the current stream without synchronising. Returns out."""
    lib = L.load()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libbhx runs on the GPU only")
    n = int(pos.shape[0]) if pos.dim() == 2 else -1
    dev = pos.device
    _check_f64("pos", pos, (n, 3), dev)
    _check_f64("mass", mass, (n,), dev)
    if eps is not None:
        _check_f64("eps", eps, (n,), dev)
    if out is None:
        raise ValueError("out is required: this entry point allocates nothing")
    _check_f64("out", out, (n, 3), dev)
    if phi is not None:
        _check_f64("phi", phi, (n,), dev)
    prec = {"fp64": L.BH_FP64, "fp32c": L.BH_FP32C}[precision]
    rc = lib.bh_compute_accel_direct_noalloc(C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                             prec, float(G), _ptr(pos), _ptr(mass),
                                             float(softening), _ptr(eps), _ptr(out), _ptr(phi), n)
    if rc != 0:
        raise BHError(rc, "bh_compute_accel_direct_noalloc failed")
    return out


def gravity_dt_bound(mass, radius, G=1.0):
    """Largest gravity time step of eq. (dt_g) for bodies of these masses and
    radii, with a context cached per device and G (see Context.gravity_dt_bound)."""
    ctx = _context_for(1, 16, "fp64", G)
    return ctx.gravity_dt_bound(mass, radius)


def step_leapfrog(pos, vel, mass, acc, dt, nsteps, theta=0.5, softening=0.0, *, eps=None, leaf=16,
                  precision="fp32c", G=1.0):
    """nsteps kick-drift-kick steps in place on pos, vel and acc (acc must hold
    the accelerations at pos on entry; theta < 0: direct sum)."""
    ctx = _context_for(pos.shape[0], leaf, precision, G)
    ctx.step_leapfrog(pos, vel, mass, acc, dt, nsteps, theta=theta, softening=softening, eps=eps)


_STATE_FORMAT = "bhx-state-1"
_STATE_ARRAYS = ("pos", "vel", "acc", "mass", "eps")


def save_state(path, pos, vel, mass, acc=None, eps=None, **meta):
    """Writes a checkpoint of a simulation to ``path`` (a .npz file).

    pos, vel (n, 3) and mass (n,) FP64, and optionally acc (n, 3), the
    accelerations at pos that a kick-drift-kick step takes on entry, and eps
    (n,) per-body softening lengths, are stored bit for bit; ``meta`` holds any
    JSON-serialisable scalars (time, step count, theta, dt ...). With acc
    stored, steps resumed from the checkpoint equal the uninterrupted steps bit
    for bit. The file is written to a temporary name and renamed, so an
    interrupted save leaves the previous checkpoint intact.
    """
    arrays = {"pos": pos, "vel": vel, "mass": mass, "acc": acc, "eps": eps}
    n = int(mass.shape[0])
    shapes = {"pos": (n, 3), "vel": (n, 3), "acc": (n, 3), "mass": (n,), "eps": (n,)}
    out = {}
    for k, t in arrays.items():
        if t is None:
            continue
        if t.dtype != torch.float64 or tuple(t.shape) != shapes[k]:
            raise ValueError(f"{k} must be float64 of shape {shapes[k]}")
        out[k] = t.detach().cpu().numpy()
    out["format"] = np.array(_STATE_FORMAT)
    out["meta"] = np.array(json.dumps(meta, sort_keys=True))
    path = os.fspath(path)
    if not path.endswith(".npz"):
        path += ".npz"
    tmp = path + ".tmp.npz"
    np.savez(tmp, **out)
    os.replace(tmp, path)
    return path


def load_state(path, device=None):
    """Reads a checkpoint written by save_state.

    Returns (arrays, meta): arrays maps "pos", "vel", "mass" and, when stored,
    "acc" and "eps" to FP64 tensors on ``device`` (default: the current GPU),
    and meta is the dict of scalars given at save time. Nothing in the file is
    unpickled.
    """
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    with np.load(path, allow_pickle=False) as z:
        if "format" not in z.files or str(z["format"]) != _STATE_FORMAT:
            raise ValueError(f"{path}: not a {_STATE_FORMAT} checkpoint")
        meta = json.loads(str(z["meta"]))
        arrays = {k: torch.from_numpy(np.ascontiguousarray(z[k])).to(device)
                  for k in _STATE_ARRAYS if k in z.files}
    n = arrays["mass"].shape[0]
    for k, t in arrays.items():
        want = (n, 3) if k in ("pos", "vel", "acc") else (n,)
        if t.dtype != torch.float64 or tuple(t.shape) != want:
            raise ValueError(f"{path}: {k} has dtype {t.dtype} and shape {tuple(t.shape)}")
    return arrays, meta
