"""Python face of the FP64 CPU oracle (``liboracle_sph.so``).

TEST INFRASTRUCTURE: imported only by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports, links or calls
anything here, and nothing here imports the GPU package.

Each function takes and returns float64 numpy arrays in the caller's particle
order.  ``tree=True`` selects the k-d tree neighbour finder, ``tree=False``
the O(N^2) brute force (both FP64).  Box-by-box evaluation of multi-box sets
is done by :func:`split_domains` + the single-box functions.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_sph.c")
_LIB = os.path.join(_HERE, "liboracle_sph.so")

GAMMA_K = math.sqrt(10.0 / 3.0)
ETA = 1.2348


def build(force=False):
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("gamma", C.c_double), ("eta", C.c_double),
                ("kernel_gamma", C.c_double), ("h_tol", C.c_double), ("max_iter", C.c_int),
                ("pad", C.c_int), ("h_limit", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.POINTER(Params)
        L.oracle_W.restype = C.c_double
        L.oracle_W.argtypes = [C.c_double, C.c_double]
        L.oracle_dWdr.restype = C.c_double
        L.oracle_dWdr.argtypes = [C.c_double, C.c_double]
        L.oracle_dWdH.restype = C.c_double
        L.oracle_dWdH.argtypes = [C.c_double, C.c_double]
        L.oracle_tree_new.restype = C.c_void_p
        L.oracle_tree_new.argtypes = [C.c_int64, _D, _D, _D, _D, C.c_int]
        L.oracle_tree_free.argtypes = [C.c_void_p]
        L.oracle_density.argtypes = [P, C.c_void_p, C.c_int64, _D, _D, _D, _D, _D, C.c_int64,
                                     _I64, _D, _D, _I64]
        L.oracle_solve_h.argtypes = [P, C.c_void_p, C.c_int64, _D, _D, _D, _D, _D, C.c_int64,
                                     _I64, _D, _D, _I64, _I32, _I64]
        L.oracle_ghost.argtypes = [P, C.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]
        L.oracle_force.argtypes = [P, C.c_void_p, C.c_int64, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                   C.c_int64, _I64, _D, _D, _D, _D, _I64, _D, _D]
        L.oracle_step.argtypes = [P, C.c_int, C.c_int64] + [_D] * 9 + [_D] * 4 + [_D] * 5 + \
                                 [_I64, _I64, C.c_double]
        L.oracle_conserved.argtypes = [C.c_int64, _D, _D, _D, _D, _D, _D]
        L.oracle_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(box, gamma=5.0 / 3.0, eta=ETA, kernel_gamma=GAMMA_K, h_tol=1e-10, max_iter=50,
           h_limit=0.0):
    p = Params()
    for k in range(3):
        p.box[k] = float(box[k])
    p.gamma, p.eta, p.kernel_gamma = gamma, eta, kernel_gamma
    p.h_tol, p.max_iter, p.pad, p.h_limit = h_tol, max_iter, 0, h_limit
    return p


class Tree:
    """k-d tree over positions (median split, leaf size 16)."""

    def __init__(self, x, y, z, box, leaf=16):
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        b = _f64(box)
        self.h = lib().oracle_tree_new(self.x.size, _d(self.x), _d(self.y), _d(self.z), _d(b), leaf)
        if not self.h:
            raise MemoryError("oracle tree")

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_tree_free(self.h)
            self.h = None


def W(r, H):
    return lib().oracle_W(float(r), float(H))


def dWdr(r, H):
    return lib().oracle_dWdr(float(r), float(H))


def dWdH(r, H):
    return lib().oracle_dWdH(float(r), float(H))


def _idx(idx):
    if idx is None:
        return 0, None, None
    a = np.ascontiguousarray(idx, dtype=np.int64)
    return a.size, a, a.ctypes.data_as(_I64)


def density(x, y, z, m, H, box, tree=True, idx=None, **kw):
    """rho, d rho/dH and the neighbour count (r < H_i, self included) at the
    given H (eq. (rho))."""
    x, y, z, m, H = map(_f64, (x, y, z, m, H))
    n = x.size
    p = params(box, **kw)
    t = Tree(x, y, z, box) if tree is True else (tree or None)
    rho, drho = np.zeros(n), np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    ni, ia, ip = _idx(idx)
    st = lib().oracle_density(C.byref(p), t.h if t else None, n, _d(x), _d(y), _d(z), _d(m),
                              _d(H), ni, ip, _d(rho), _d(drho), cnt.ctypes.data_as(_I64))
    if st != 0:
        raise RuntimeError("oracle_density status %d" % st)
    return rho, drho, cnt


def solve_h(x, y, z, m, H0, box, tree=True, idx=None, check=True, **kw):
    """Converged H with rho, d rho/dH, neighbour count and iteration count at
    that H (bracketed Newton on rho H^3 = (kernel_gamma eta)^3 m)."""
    x, y, z, m = map(_f64, (x, y, z, m))
    H = _f64(H0).copy()
    n = x.size
    p = params(box, **kw)
    t = Tree(x, y, z, box) if tree is True else (tree or None)
    rho, drho = np.zeros(n), np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    iters = np.zeros(n, dtype=np.int32)
    nfail = C.c_int64(0)
    ni, ia, ip = _idx(idx)
    st = lib().oracle_solve_h(C.byref(p), t.h if t else None, n, _d(x), _d(y), _d(z), _d(m),
                              _d(H), ni, ip, _d(rho), _d(drho), cnt.ctypes.data_as(_I64),
                              iters.ctypes.data_as(_I32), C.byref(nfail))
    if check and st != 0:
        raise RuntimeError("oracle_solve_h status %d (%d unconverged)" % (st, nfail.value))
    return dict(H=H, rho=rho, drho=drho, cnt=cnt, iters=iters, status=st, n_fail=nfail.value)


def ghost(rho, drho, H, u, gamma=5.0 / 3.0):
    """Omega, P, A = P/(Omega rho^2) and the sound speed."""
    rho, drho, H, u = map(_f64, (rho, drho, H, u))
    n = rho.size
    p = params((1, 1, 1), gamma=gamma)
    om, P, A, cs = (np.zeros(n) for _ in range(4))
    lib().oracle_ghost(C.byref(p), n, _d(rho), _d(drho), _d(H), _d(u), _d(om), _d(P), _d(A),
                       _d(cs))
    return dict(omega=om, P=P, A=A, cs=cs)


def force(x, y, z, vx, vy, vz, m, H, A, box, tree=True, idx=None):
    """a (3 arrays), du/dt and the per-particle count of j with
    r_ij < max(H_i, H_j) (eqs. (dvdt), (dudt)), plus the magnitude scales
    sa = sum_j m_j |A_i dW_i + A_j dW_j| and su = sum_j |A_i m_j dW_i v_ij.r_ij/r|."""
    x, y, z, vx, vy, vz, m, H, A = map(_f64, (x, y, z, vx, vy, vz, m, H, A))
    n = x.size
    p = params(box)
    t = Tree(x, y, z, box) if tree is True else (tree or None)
    ax, ay, az, du, sa, su = (np.zeros(n) for _ in range(6))
    fc = np.zeros(n, dtype=np.int64)
    ni, ia, ip = _idx(idx)
    st = lib().oracle_force(C.byref(p), t.h if t else None, n, _d(x), _d(y), _d(z), _d(vx),
                            _d(vy), _d(vz), _d(m), _d(H), _d(A), ni, ip, _d(ax), _d(ay), _d(az),
                            _d(du), fc.ctypes.data_as(_I64), _d(sa), _d(su))
    if st != 0:
        raise RuntimeError("oracle_force status %d" % st)
    return dict(ax=ax, ay=ay, az=az, dudt=du, fcnt=fc, sa=sa, su=su)


def full(d, tree=True, h_tol=1e-10, max_iter=50, gamma=5.0 / 3.0, idx=None, eta=ETA):
    """Density solve, ghost and force for a one-box particle set ``d`` (the
    dict layout of the input generators).  With ``idx``, H is solved for all
    particles but the force only for idx."""
    box = d["box"]
    t = Tree(d["x"], d["y"], d["z"], box) if tree else None
    s = solve_h(d["x"], d["y"], d["z"], d["m"], d["H"], box, tree=t if tree else False,
                h_tol=h_tol, max_iter=max_iter, eta=eta)
    g = ghost(s["rho"], s["drho"], s["H"], d["u"], gamma=gamma)
    f = force(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], s["H"], g["A"], box,
              tree=t if tree else False, idx=idx)
    out = dict(s)
    out.update(g)
    out.update(f)
    out["n_dens"] = int(s["cnt"].sum())
    if idx is None:
        out["n_force"] = int(f["fcnt"].sum()) // 2
    return out


def step(state, dt, tree=True, h_tol=1e-10, max_iter=50, gamma=5.0 / 3.0):
    """One kick-drift-kick step on a state dict (positions, velocities, u, m,
    H and the forces of the current positions ax, ay, az, dudt), in place."""
    s = state
    n = s["x"].size
    for k in ("rho", "drho", "omega", "P", "A"):
        s.setdefault(k, np.zeros(n))
    s.setdefault("cnt", np.zeros(n, dtype=np.int64))
    s.setdefault("fcnt", np.zeros(n, dtype=np.int64))
    p = params(s["box"], gamma=gamma, h_tol=h_tol, max_iter=max_iter)
    names = ["x", "y", "z", "vx", "vy", "vz", "u", "m", "H", "ax", "ay", "az", "dudt", "rho",
             "drho", "omega", "P", "A"]
    for k in names:
        assert s[k].dtype == np.float64 and s[k].flags.c_contiguous, k
    args = [_d(s[k]) for k in names]
    st = lib().oracle_step(C.byref(p), 1 if tree else 0, n, *args,
                           s["cnt"].ctypes.data_as(_I64), s["fcnt"].ctypes.data_as(_I64), dt)
    if st != 0:
        raise RuntimeError("oracle_step status %d" % st)
    return s


def conserved(m, vx, vy, vz, u):
    """FP64 totals: mass, momentum x/y/z, kinetic + thermal energy."""
    m, vx, vy, vz, u = map(_f64, (m, vx, vy, vz, u))
    out = np.zeros(5)
    lib().oracle_conserved(m.size, _d(m), _d(vx), _d(vy), _d(vz), _d(u), _d(out))
    return out


def num_threads():
    return lib().oracle_num_threads()


def split_domains(d):
    """Per-box sub-dicts of a multi-box set (keeps the original indices)."""
    out = []
    for b in range(d["boxes"].shape[0]):
        idx = np.nonzero(d["domain"] == b)[0]
        s = {k: np.ascontiguousarray(d[k][idx]) for k in
             ("x", "y", "z", "vx", "vy", "vz", "u", "m", "H", "id")}
        s["box"] = d["boxes"][b]
        s["index"] = idx
        out.append(s)
    return out
