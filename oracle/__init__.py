"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU implementation of the gravity hot path of
Ferrari, Lavagna & Blazquez (MNRAS 2020), Section "Gravitational dynamics":
the direct sum (eq. Newton with softening, eq. Force_rComp), the octree with
bottom-up moments (eq. COMinternal), the per-body theta walk (eqs. accuracy,
Force_leaf, Force_thetaTrue) and a kick-drift-kick leapfrog.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU library; the C source is
``bh_oracle.c`` (built by :func:`build`) and this module only marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bh_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {1: "invalid argument", 2: "non-finite input", 3: "negative mass", 4: "out of memory"}


class OracleError(RuntimeError):
    pass


def compile_source(src: str, out: str) -> str:
    """Compile one oracle C source to a shared library at ``out``."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-I", _HERE, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


def use_library(path: str | None = None) -> None:
    """Switch to another build of the oracle (the mutation tests load copies
    with planted mistakes); ``None`` returns to ``liboracle.so``."""
    global _lib
    _lib = None
    _load(path)


def _load(path: str | None = None):
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = _LIB_PATH
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
    lib = C.CDLL(path)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.orc_direct.argtypes = [I64, P, P, P, D, D, P, I64, P, P, P]
    lib.orc_direct.restype = C.c_int
    lib.orc_tree_build.argtypes = [I64, P, P, P, I32, C.POINTER(C.c_int)]
    lib.orc_tree_build.restype = P
    lib.orc_tree_free.argtypes = [P]
    lib.orc_tree_free.restype = None
    lib.orc_tree_nnodes.argtypes = [P]
    lib.orc_tree_nnodes.restype = I64
    lib.orc_tree_box.argtypes = [P, P]
    lib.orc_tree_box.restype = None
    lib.orc_tree_export.argtypes = [P] * 11
    lib.orc_tree_export.restype = None
    lib.orc_tree_accel.argtypes = [P, P, P, P, D, D, D, P, I64, P, P, P, P]
    lib.orc_tree_accel.restype = C.c_int
    lib.orc_tree_accel_q.argtypes = [P, P, P, P, D, D, D, P, I64, P, P, P, P, C.c_int]
    lib.orc_tree_accel_q.restype = C.c_int
    lib.orc_tree_quadrupoles.argtypes = [P, P, P]
    lib.orc_tree_quadrupoles.restype = C.c_int
    lib.orc_tree_quad_export.argtypes = [P, P]
    lib.orc_tree_quad_export.restype = C.c_int
    lib.orc_leapfrog.argtypes = [I64, P, P, P, P, D, D, D, I32, D, I32, P]
    lib.orc_leapfrog.restype = C.c_int
    lib.orc_euler.argtypes = [I64, P, P, P, P, D, D, D, I32, D, I32, I32, P]
    lib.orc_euler.restype = C.c_int
    lib.orc_contact_components.argtypes = [I64, P, P, D, P, P, P]
    lib.orc_contact_components.restype = C.c_int
    lib.orc_diagnostics.argtypes = [I64, P, P, P, P, D, D, P]
    lib.orc_diagnostics.restype = C.c_int
    lib.orc_direct_vjp.argtypes = [I64, P, P, P, D, D, P, P, P]
    lib.orc_direct_vjp.restype = C.c_int
    lib.orc_tree_vjp.argtypes = [P, P, P, P, D, D, D, P, P, P]
    lib.orc_tree_vjp.restype = C.c_int
    lib.orc_tree_vjp_abs.argtypes = [P, P, P, P, D, D, D, P, P, P]
    lib.orc_tree_vjp_abs.restype = C.c_int
    lib.orc_rollout_grad.argtypes = [I64, P, P, P, P, D, D, D, I32, D, I32, P, P, P, P, P]
    lib.orc_rollout_grad.restype = C.c_int
    lib.orc_gravity_dt_bound.argtypes = [I64, P, P, D, P]
    lib.orc_gravity_dt_bound.restype = C.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc):
    if rc:
        raise OracleError(ERRORS.get(rc, f"error {rc}"))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Threads for the oracle's later calls (timing a one-thread baseline)."""
    lib = _load()
    lib.orc_set_num_threads.argtypes = [C.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads(int(k))


def _targets(n, targets):
    if targets is None:
        return None, n
    t = np.ascontiguousarray(targets, dtype=np.int64)
    return t, int(t.shape[0])


def direct(pos, mass, softening=0.0, eps=None, G=1.0, targets=None):
    """Direct N^2 sum. Returns (acc (nt,3), phi (nt,), absacc (nt,))."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    eps = None if eps is None else _f64(eps, (n,))
    t, nt = _targets(n, targets)
    acc = np.zeros((nt, 3))
    phi = np.zeros(nt)
    aabs = np.zeros(nt)
    _check(lib.orc_direct(n, _ptr(pos), _ptr(mass), _ptr(eps), float(softening), float(G),
                          _ptr(t), nt, _ptr(acc), _ptr(phi), _ptr(aabs)))
    return acc, phi, aabs


class Tree:
    """Oracle octree over all bodies (bucket leaves of at most ``leaf``)."""

    def __init__(self, pos, mass, eps=None, leaf=16):
        lib = _load()
        self.pos = _f64(pos)
        self.n = self.pos.shape[0]
        self.mass = _f64(mass, (self.n,))
        self.eps = None if eps is None else _f64(eps, (self.n,))
        self.leaf = int(leaf)
        err = C.c_int(0)
        h = lib.orc_tree_build(self.n, _ptr(self.pos), _ptr(self.mass), _ptr(self.eps),
                               self.leaf, C.byref(err))
        if not h:
            _check(err.value or 4)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    @property
    def nnodes(self) -> int:
        return int(_load().orc_tree_nnodes(self._h))

    def box(self) -> dict:
        b = np.zeros(8)
        _load().orc_tree_box(self._h, _ptr(b))
        return {"lo": b[0:3].copy(), "x0": b[3:6].copy(), "L": float(b[6]), "S": float(b[7])}

    def export(self) -> dict:
        nn, n = self.nnodes, self.n
        out = {
            "level": np.zeros(nn, np.int32), "first": np.zeros(nn, np.int64),
            "count": np.zeros(nn, np.int64), "child0": np.zeros(nn, np.int64),
            "nchild": np.zeros(nn, np.int32), "mass": np.zeros(nn),
            "com": np.zeros((nn, 3)), "eps2": np.zeros(nn),
            "order": np.zeros(n, np.int64), "q": np.zeros((n, 3), np.uint32),
        }
        _load().orc_tree_export(self._h, *[_ptr(out[k]) for k in
                                           ("level", "first", "count", "child0", "nchild",
                                            "mass", "com", "eps2", "order", "q")])
        return out

    def quadrupoles(self) -> np.ndarray:
        """(nnodes, 6) traceless quadrupoles (xx, yy, zz, xy, xz, yz) about each
        node's centre of mass, in the node order of export()."""
        lib = _load()
        if not getattr(self, "_has_quad", False):
            _check(lib.orc_tree_quadrupoles(self._h, _ptr(self.pos), _ptr(self.mass)))
            self._has_quad = True
        out = np.zeros((self.nnodes, 6))
        _check(lib.orc_tree_quad_export(self._h, _ptr(out)))
        return out

    def accel(self, theta, softening=0.0, G=1.0, targets=None, quad=False):
        """Barnes-Hut walk. Returns (acc, phi, absacc, counts (nt,2): accepted nodes, pairs).
        quad=True adds each accepted node's quadrupole term."""
        t, nt = _targets(self.n, targets)
        acc = np.zeros((nt, 3))
        phi = np.zeros(nt)
        aabs = np.zeros(nt)
        cnt = np.zeros((nt, 2), np.int64)
        lib = _load()
        if quad and not getattr(self, "_has_quad", False):
            _check(lib.orc_tree_quadrupoles(self._h, _ptr(self.pos), _ptr(self.mass)))
            self._has_quad = True
        _check(lib.orc_tree_accel_q(self._h, _ptr(self.pos), _ptr(self.mass), _ptr(self.eps),
                                    float(softening), float(G), float(theta), _ptr(t), nt,
                                    _ptr(acc), _ptr(phi), _ptr(aabs), _ptr(cnt), int(bool(quad))))
        return acc, phi, aabs, cnt


def direct_vjp(pos, mass, lam, softening=0.0, eps=None, G=1.0):
    """(g_pos, g_mass): gradient of sum_i lam_i . a_i for the direct sum."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass, (n,))
    lam = _f64(lam, (n, 3))
    eps = None if eps is None else _f64(eps, (n,))
    gx = np.zeros((n, 3))
    gm = np.zeros(n)
    _check(lib.orc_direct_vjp(n, _ptr(pos), _ptr(mass), _ptr(eps), float(softening), float(G),
                              _ptr(lam), _ptr(gx), _ptr(gm)))
    return gx, gm


def tree_vjp(pos, mass, lam, theta, softening=0.0, eps=None, leaf=16, G=1.0):
    """(g_pos, g_mass) for the Barnes-Hut force map with its decisions held fixed."""
    T = Tree(pos, mass, eps, leaf)
    lam = _f64(lam, (T.n, 3))
    gx = np.zeros((T.n, 3))
    gm = np.zeros(T.n)
    _check(_load().orc_tree_vjp(T._h, _ptr(T.pos), _ptr(T.mass), _ptr(T.eps), float(softening),
                                float(G), float(theta), _ptr(lam), _ptr(gx), _ptr(gm)))
    return gx, gm


def tree_vjp_abs(pos, mass, lam, theta, softening=0.0, eps=None, leaf=16, G=1.0):
    """(g_pos, g_mass) error scales of tree_vjp: the same walk with the
    magnitudes of every contribution's parts added (each bounds |tree_vjp|)."""
    T = Tree(pos, mass, eps, leaf)
    lam = _f64(lam, (T.n, 3))
    gx = np.zeros((T.n, 3))
    gm = np.zeros(T.n)
    _check(_load().orc_tree_vjp_abs(T._h, _ptr(T.pos), _ptr(T.mass), _ptr(T.eps),
                                    float(softening), float(G), float(theta), _ptr(lam), _ptr(gx),
                                    _ptr(gm)))
    return gx, gm


def rollout_grad(pos0, vel0, mass, dt, nsteps, xbar, vbar, softening=0.0, eps=None,
                 theta=-1.0, leaf=16, G=1.0):
    """(gx0, gv0, gm) of a loss with dL/dx_T = xbar, dL/dv_T = vbar through
    nsteps KDK steps from (pos0, vel0), a0 = A(pos0); theta < 0: direct sum."""
    lib = _load()
    pos0 = _f64(pos0)
    n = pos0.shape[0]
    vel0 = _f64(vel0, (n, 3))
    mass = _f64(mass, (n,))
    xbar = _f64(xbar, (n, 3))
    vbar = _f64(vbar, (n, 3))
    eps = None if eps is None else _f64(eps, (n,))
    gx, gv, gm = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
    _check(lib.orc_rollout_grad(n, _ptr(pos0), _ptr(vel0), _ptr(mass), _ptr(eps),
                                float(softening), float(G), float(theta), int(leaf), float(dt),
                                int(nsteps), _ptr(xbar), _ptr(vbar), _ptr(gx), _ptr(gv),
                                _ptr(gm)))
    return gx, gv, gm


def bh(pos, mass, theta, softening=0.0, eps=None, leaf=16, G=1.0, targets=None, quad=False):
    """Build the tree and walk it: (acc, phi, absacc, counts)."""
    return Tree(pos, mass, eps, leaf).accel(theta, softening, G, targets, quad=quad)


def leapfrog(pos, vel, mass, dt, nsteps, softening=0.0, eps=None, theta=-1.0, leaf=16,
             G=1.0, acc=None):
    """KDK leapfrog; theta < 0 uses the direct sum. Returns (pos, vel, acc) copies."""
    lib = _load()
    pos = _f64(pos).copy()
    n = pos.shape[0]
    vel = _f64(vel, (n, 3)).copy()
    mass = _f64(mass, (n,))
    eps = None if eps is None else _f64(eps, (n,))
    if acc is None:
        if theta < 0:
            acc = direct(pos, mass, softening, eps, G)[0]
        else:
            acc = bh(pos, mass, theta, softening, eps, leaf, G)[0]
    acc = _f64(acc, (n, 3)).copy()
    _check(lib.orc_leapfrog(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(eps), float(softening),
                            float(G), float(theta), int(leaf), float(dt), int(nsteps), _ptr(acc)))
    return pos, vel, acc


def euler(pos, vel, mass, dt, nsteps, every=1, softening=0.0, eps=None, theta=-1.0, leaf=16,
          G=1.0, acc=None):
    """Semi-implicit Euler with gravity evaluated after every `every`-th substep;
    theta < 0 uses the direct sum. Returns (pos, vel, acc) copies."""
    lib = _load()
    pos = _f64(pos).copy()
    n = pos.shape[0]
    vel = _f64(vel, (n, 3)).copy()
    mass = _f64(mass, (n,))
    eps = None if eps is None else _f64(eps, (n,))
    if acc is None:
        if theta < 0:
            acc = direct(pos, mass, softening, eps, G)[0]
        else:
            acc = bh(pos, mass, theta, softening, eps, leaf, G)[0]
    acc = _f64(acc, (n, 3)).copy()
    _check(lib.orc_euler(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(eps), float(softening),
                         float(G), float(theta), int(leaf), float(dt), int(nsteps), int(every),
                         _ptr(acc)))
    return pos, vel, acc


def contact_components(pos, radius, skin=0.0):
    """(label, n_contacts, n_aggregates): label[i] = smallest index of body i's
    contact component (all pairs tested; O(N^2))."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    radius = _f64(radius, (n,))
    label = np.zeros(n, np.int32)
    nc = C.c_int64(0)
    na = C.c_int64(0)
    _check(lib.orc_contact_components(n, _ptr(pos), _ptr(radius), float(skin), _ptr(label),
                                      C.byref(nc), C.byref(na)))
    return label, int(nc.value), int(na.value)


def gravity_dt_bound(mass, radius, G=1.0) -> float:
    """Largest gravity time step of eq. (dt_g) for bodies of these masses and
    radii: 1 / (2 sqrt(G rho)) with rho the largest body density."""
    mass = _f64(mass)
    n = mass.shape[0]
    radius = _f64(radius, (n,))
    out = np.zeros(1)
    _check(_load().orc_gravity_dt_bound(n, _ptr(mass), _ptr(radius), float(G), _ptr(out)))
    return float(out[0])


def diagnostics(pos, vel, mass, softening=0.0, eps=None, G=1.0) -> np.ndarray:
    """[E_kin, E_pot, Px, Py, Pz, Lx, Ly, Lz] by plain FP64 sums (direct potential)."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    vel = _f64(vel, (n, 3))
    mass = _f64(mass, (n,))
    eps = None if eps is None else _f64(eps, (n,))
    out = np.zeros(8)
    _check(lib.orc_diagnostics(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(eps), float(softening),
                               float(G), _ptr(out)))
    return out
