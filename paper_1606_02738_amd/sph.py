"""ctypes binding of libsph_hip (the C-ABI in include/sph.h).

Argument marshalling only: every stage runs in the library's HIP kernels.
Particle arrays are torch tensors on the GPU (float64 unless stated), and so
is the workspace the library carves its device buffers from (a uint8 tensor
sized by sph_workspace_size); torch provides device memory and the stream,
nothing else.  If the library is not built this module raises at import of
:func:`lib` -- there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph_hip.so")

SPH_FP64, SPH_FP32C, SPH_FP32 = 0, 1, 2
SPH_EXEC_GRID, SPH_EXEC_PERSISTENT = 0, 1
PRECISIONS = {"fp64": SPH_FP64, "fp32c": SPH_FP32C, "fp32": SPH_FP32}
EXEC_MODES = {"grid": SPH_EXEC_GRID, "persistent": SPH_EXEC_PERSISTENT}
SPH_PRUNE_BOX, SPH_PRUNE_SORTED = 0, 1
PRUNE_MODES = {"box": SPH_PRUNE_BOX, "sorted": SPH_PRUNE_SORTED}
SPH_FORCE_PAIRS, SPH_FORCE_GATHER = 0, 1
FORCE_MODES = {"pairs": SPH_FORCE_PAIRS, "gather": SPH_FORCE_GATHER}
SPH_LISTS_CELL, SPH_LISTS_PARTICLE = 0, 1
LIST_MODES = {"cell": SPH_LISTS_CELL, "particle": SPH_LISTS_PARTICLE}

STATUS = {0: "SPH_OK", -1: "SPH_ERR_INVALID", -2: "SPH_ERR_HIP", -3: "SPH_ERR_NOT_CONVERGED",
          -4: "SPH_ERR_H_EXCEEDS_CELL", -5: "SPH_ERR_BOX_TOO_SMALL", -6: "SPH_ERR_WORKSPACE",
          -7: "SPH_ERR_STATE"}
WORKSPACE_MIN = 1 << 20

FLOAT_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "m", "H", "rho", "drho_dH", "omega", "P",
                "ax", "ay", "az", "dudt")


class SPHError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, STATUS.get(status, "?"), status))


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("eta", C.c_double), ("kernel_gamma", C.c_double),
                ("h_tol", C.c_double), ("max_h_iter", C.c_int), ("n_split", C.c_int),
                ("precision", C.c_int), ("exec_mode", C.c_int), ("n_domains", C.c_int),
                ("persistent_wgs", C.c_int), ("use_graph", C.c_int), ("prune", C.c_int),
                ("rebuild_steps", C.c_int), ("h_drift", C.c_int), ("force_mode", C.c_int),
                ("lists", C.c_int), ("tile", C.c_int), ("waves_density", C.c_int), ("waves_force", C.c_int),
                ("batch", C.c_int), ("boxes", C.POINTER(C.c_double))]


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.c_void_p) for f in FLOAT_FIELDS] + \
               [("id", C.c_void_p), ("domain", C.c_void_p), ("nngb", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_leaves", C.c_int64), ("n_nodes", C.c_int64),
                ("n_list", C.c_int64), ("n_pair_tasks", C.c_int64), ("n_dens", C.c_int64),
                ("n_force", C.c_int64), ("sweeps", C.c_int32), ("n_unconverged", C.c_int32),
                ("relists", C.c_int32), ("rebuilds", C.c_int32), ("depth", C.c_int32),
                ("key_bits", C.c_int32), ("conserved", C.c_double * 5),
                ("t_density_ms", C.c_double), ("t_ghost_ms", C.c_double),
                ("t_force_ms", C.c_double), ("t_build_ms", C.c_double),
                ("t_density_kernels_ms", C.c_double), ("t_force_kernel_ms", C.c_double),
                ("n_dens_evals", C.c_int64), ("n_density_launches", C.c_int32),
                ("graph_captures", C.c_int32), ("graph_fallbacks", C.c_int32), ("precision_rebuilds", C.c_int32),
                ("unconv_after", C.c_int32 * 8), ("t_predict_ms", C.c_double),
                ("steps_since_build", C.c_int64), ("n_builds", C.c_int64), ("list_margin", C.c_double),
                ("n_chunks", C.c_int64), ("n_plist", C.c_int64), ("n_union", C.c_int64),
                ("stale_moved", C.c_int64), ("stale_grown", C.c_int64),
                ("workspace_bytes", C.c_int64), ("workspace_in_use", C.c_int64),
                ("workspace_high", C.c_int64), ("workspace_needed", C.c_int64),
                ("n_force_total", C.c_int64), ("n_dens_total", C.c_int64), ("force_calls", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["conserved"] = list(self.conserved)
        d["unconv_after"] = list(self.unconv_after)
        return d


_lib = None
EXPORTS = ("sph_workspace_size", "sph_mlp_workspace_size", "sph_create", "sph_destroy", "sph_build_cells", "sph_sort_cells", "sph_density",
           "sph_ghost", "sph_force", "sph_density_ghost_force", "sph_step", "sph_get_stats", "sph_domain_sums",
           "sph_status_str", "sph_version", "sph_mlp_forward", "sph_mlp_loss_grad", "sph_mlp_loss_grad_noalloc", "sph_mlp_adam",
           "sph_h_features", "sph_h_record", "sph_h_train", "sph_h_set_params", "sph_h_get_params",
           "sph_h_predict", "sph_interpolate")

MLP_NF, MLP_XSTRIDE, MLP_NIN, MLP_NH, MLP_NT, MLP_NP = 7, 8, 16, 64, 9473, 9507


def lib():
    """Load libsph_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsph_hip.so is not built (run paper_1606_02738_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.sph_workspace_size.argtypes = [C.POINTER(Params), C.c_int64, C.POINTER(C.c_size_t)]
        L.sph_mlp_workspace_size.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
        L.sph_create.argtypes = [C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.sph_destroy.argtypes = [vp]
        L.sph_build_cells.argtypes = [vp, C.POINTER(Particles)]
        for f in ("sph_sort_cells", "sph_density", "sph_ghost", "sph_force", "sph_density_ghost_force"):
            getattr(L, f).argtypes = [vp]
        L.sph_step.argtypes = [vp, C.c_double]
        L.sph_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.sph_domain_sums.argtypes = [vp, C.POINTER(C.c_double)]
        L.sph_status_str.restype = C.c_char_p
        L.sph_status_str.argtypes = [C.c_int]
        L.sph_version.restype = C.c_char_p
        L.sph_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_size_t, vp]
        L.sph_mlp_loss_grad.argtypes = [vp, vp, vp, C.c_int64, vp, C.POINTER(C.c_double), vp, C.c_size_t, vp]
        L.sph_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, C.c_int64, vp, C.POINTER(C.c_double), vp]
        L.sph_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.sph_h_features.argtypes = [vp, C.c_double, vp]
        L.sph_h_record.argtypes = [vp, vp, vp, C.c_int64, C.c_double, C.c_uint64, C.POINTER(C.c_int64)]
        L.sph_h_train.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_uint64, C.c_int, C.POINTER(C.c_double)]
        L.sph_h_set_params.argtypes = [vp, C.POINTER(C.c_float)]
        L.sph_h_get_params.argtypes = [vp, C.POINTER(C.c_float)]
        L.sph_h_predict.argtypes = [vp, C.c_int]
        L.sph_interpolate.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, vp]
        for f in EXPORTS:
            if f not in ("sph_status_str", "sph_version"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(st, where):
    if st != 0:
        raise SPHError(st, where)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _mlp_workspace(n, device):
    import torch
    b = C.c_size_t()
    _check(lib().sph_mlp_workspace_size(int(n), C.byref(b)), "sph_mlp_workspace_size")
    return torch.empty(b.value, dtype=torch.uint8, device=device)


def mlp_forward(params, X, stream=None):
    """Network output y (predicted log(H_new/H_prev)) for feature rows X
    (n x 8 float32 device tensor); params: float32 device tensor of MLP_NP."""
    import torch
    assert params.dtype == torch.float32 and params.numel() == MLP_NP and params.is_cuda
    assert X.dtype == torch.float32 and X.is_contiguous() and X.shape[-1] == MLP_XSTRIDE
    n = X.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    ws = _mlp_workspace(n, X.device)
    _check(lib().sph_mlp_forward(params.data_ptr(), X.data_ptr(), n, y.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream_ptr(stream)), "sph_mlp_forward")
    return y


def mlp_loss_grad(params, X, y, stream=None):
    """(mean loss, gradient tensor of MLP_NT floats) over the rows."""
    import torch
    assert X.dtype == torch.float32 and X.is_contiguous() and X.shape[-1] == MLP_XSTRIDE
    assert y.dtype == torch.float32 and y.numel() == X.shape[0]
    g = torch.empty(MLP_NT, dtype=torch.float32, device=X.device)
    L = C.c_double()
    ws = _mlp_workspace(X.shape[0], X.device)
    _check(lib().sph_mlp_loss_grad(params.data_ptr(), X.data_ptr(), y.data_ptr(), X.shape[0], g.data_ptr(),
                                   C.byref(L), ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
           "sph_mlp_loss_grad")
    return L.value, g


def mlp_loss_grad_noalloc(params, X, y, grad=None, stream=None):
    """mlp_loss_grad through the entry point that allocates nothing (its
    partials live in the library's own device array); grad: an optional
    preallocated float32 tensor of MLP_NT."""
    import torch
    assert X.dtype == torch.float32 and X.is_contiguous() and X.shape[-1] == MLP_XSTRIDE
    assert y.dtype == torch.float32 and y.numel() == X.shape[0]
    g = grad if grad is not None else torch.empty(MLP_NT, dtype=torch.float32, device=X.device)
    assert g.dtype == torch.float32 and g.numel() == MLP_NT and g.is_contiguous()
    L = C.c_double()
    _check(lib().sph_mlp_loss_grad_noalloc(params.data_ptr(), X.data_ptr(), y.data_ptr(), X.shape[0], g.data_ptr(),
                                           C.byref(L), _stream_ptr(stream)), "sph_mlp_loss_grad_noalloc")
    return L.value, g


def mlp_adam(params, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step in place on params, m, v (float32 device tensors)."""
    _check(lib().sph_mlp_adam(params.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(), int(t), float(lr),
                              float(beta1), float(beta2), float(eps), _stream_ptr(stream)), "sph_mlp_adam")


def to_device(d, device="cuda"):
    """Copy a generator dict (numpy) to GPU tensors with every field the
    library binds (outputs zero-initialised)."""
    import torch
    n = d["x"].size
    t = {}
    for k in FLOAT_FIELDS:
        if k in d:
            t[k] = torch.from_numpy(np.ascontiguousarray(d[k], dtype=np.float64)).to(device)
        else:
            t[k] = torch.zeros(n, dtype=torch.float64, device=device)
    t["id"] = torch.from_numpy(np.ascontiguousarray(d.get("id", np.arange(n)), dtype=np.int64)).to(device)
    dom = d.get("domain")
    t["domain"] = torch.from_numpy(np.ascontiguousarray(
        dom if dom is not None else np.zeros(n), dtype=np.int32)).to(device)
    t["nngb"] = torch.zeros(n, dtype=torch.int32, device=device)
    return t


def to_host(t, order_by_id=True):
    """Tensors -> numpy, optionally back in the original particle order."""
    out = {k: v.detach().cpu().numpy() for k, v in t.items()}
    if order_by_id:
        inv = np.argsort(out["id"], kind="stable")
        out = {k: v[inv] for k, v in out.items()}
    return out


class SPH:
    """One context of the library bound to one particle set."""

    def __init__(self, boxes, precision="fp32c", exec_mode="grid", gamma=5.0 / 3.0, eta=1.2348,
                 kernel_gamma=math.sqrt(10.0 / 3.0), h_tol=None, max_h_iter=40, n_split=64,
                 persistent_wgs=0, prune="box", use_graph=False, rebuild_steps=0, h_drift=True, force=None,
                 lists="cell", tile=0, waves_density=0, waves_force=0, batch=0, workspace_bytes=None,
                 stream=None):
        import torch
        self._torch = torch
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 3))
        self.n_domains = b.shape[0]
        self._boxes = b
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if h_tol is None:
            h_tol = 1e-10 if prec == SPH_FP64 else 2e-6
        p = Params()
        p.gamma, p.eta, p.kernel_gamma, p.h_tol = gamma, eta, kernel_gamma, h_tol
        p.max_h_iter, p.n_split, p.precision = max_h_iter, n_split, prec
        p.exec_mode = EXEC_MODES[exec_mode] if isinstance(exec_mode, str) else int(exec_mode)
        p.n_domains, p.persistent_wgs, p.use_graph = self.n_domains, persistent_wgs, int(bool(use_graph))
        p.prune = PRUNE_MODES[prune] if isinstance(prune, str) else int(prune)
        p.rebuild_steps = int(rebuild_steps)
        p.h_drift = int(bool(h_drift))
        if force is None:  # the gather form where it is available (box pruning)
            force = "gather" if p.prune == SPH_PRUNE_BOX else "pairs"
        p.force_mode = FORCE_MODES[force] if isinstance(force, str) else int(force)
        p.lists = LIST_MODES[lists] if isinstance(lists, str) else int(lists)
        p.tile = int(tile)
        p.waves_density, p.waves_force, p.batch = int(waves_density), int(waves_force), int(batch)
        p.boxes = b.ctypes.data_as(C.POINTER(C.c_double))
        self.params = p
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        self._ws_bytes = workspace_bytes
        self.ws = None
        self.h = C.c_void_p()
        self._predict = False
        self.t = None
        # the context checks the parameters now; it is created again with a
        # workspace sized for the particle set at bind()
        self._create(4 * WORKSPACE_MIN)

    def workspace_size(self, n):
        """sph_workspace_size for n particles with this context's parameters."""
        b = C.c_size_t()
        _check(lib().sph_workspace_size(C.byref(self.params), int(n), C.byref(b)), "sph_workspace_size")
        return b.value

    def _create(self, nbytes):
        torch = self._torch
        ws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _check(lib().sph_create(C.byref(self.params), C.c_void_p(ws.data_ptr()), ws.numel(),
                                C.c_void_p(self.stream.cuda_stream), C.byref(h)), "sph_create")
        self.h = h
        self.ws = ws

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            if _lib is None:  # interpreter shutdown: the module state is gone
                return
            _lib.sph_destroy(self.h)
            self.h = C.c_void_p()
        self.ws = None

    __del__ = close

    def bind(self, t):
        """Attach device tensors (dict from :func:`to_device`).  The context is
        (re)created with a workspace for this many particles when its
        workspace is smaller (the predictor's parameters are carried over)."""
        for k in FLOAT_FIELDS:
            v = t[k]
            assert v.is_cuda and v.dtype == self._torch.float64 and v.is_contiguous(), k
        n = t["x"].numel()
        # (an empty set keeps the workspace: the library rejects it at the build)
        need = int(self._ws_bytes) if self._ws_bytes else (self.workspace_size(n) if n > 0 else 0)
        if self.ws is None or self.ws.numel() < need:
            keep = None
            try:
                keep = self.h_get_params()
            except SPHError:
                pass
            self.close()
            self._create(need)
            if keep is not None:
                self.h_set_params(keep)
                if self._predict:
                    self.h_predict(True)
        self.t = t
        P = Particles()
        P.n = t["x"].numel()
        for k in FLOAT_FIELDS:
            setattr(P, k, t[k].data_ptr())
        P.id = t["id"].data_ptr() if "id" in t else None
        P.domain = t["domain"].data_ptr() if self.n_domains > 1 else None
        P.nngb = t["nngb"].data_ptr() if "nngb" in t else None
        self._P = P
        return self

    def build_cells(self):
        _check(lib().sph_build_cells(self.h, C.byref(self._P)), "sph_build_cells")

    def sort_cells(self):
        _check(lib().sph_sort_cells(self.h), "sph_sort_cells")

    def density(self):
        _check(lib().sph_density(self.h), "sph_density")

    def ghost(self):
        _check(lib().sph_ghost(self.h), "sph_ghost")

    def force(self):
        _check(lib().sph_force(self.h), "sph_force")

    def density_ghost_force(self):
        _check(lib().sph_density_ghost_force(self.h), "sph_density_ghost_force")

    def step(self, dt):
        _check(lib().sph_step(self.h, float(dt)), "sph_step")

    def interpolate(self, Q, px, py, pz, pdom=None):
        """Eq. (interp) at the given points (device float64 tensors; Q in the
        bound arrays' current order); returns a float64 tensor."""
        T = self._torch
        m_pts = px.numel()
        for t in (Q, px, py, pz):
            assert t.dtype == T.float64 and t.is_contiguous() and t.is_cuda
        assert py.numel() == m_pts and pz.numel() == m_pts and Q.numel() == self.t["x"].numel()
        if pdom is not None:
            assert pdom.dtype == T.int32 and pdom.numel() == m_pts and pdom.is_contiguous()
        out = T.empty(m_pts, dtype=T.float64, device=px.device)
        _check(lib().sph_interpolate(self.h, Q.data_ptr(), px.data_ptr(), py.data_ptr(), pz.data_ptr(),
                                     None if pdom is None else pdom.data_ptr(), m_pts, out.data_ptr()),
               "sph_interpolate")
        return out

    def h_features(self, dt):
        """Predictor features of the bound particles (n x 8 float32 tensor)."""
        X = self._torch.empty((self.t["x"].numel(), MLP_XSTRIDE), dtype=self._torch.float32,
                              device=self.t["x"].device)
        _check(lib().sph_h_features(self.h, float(dt), X.data_ptr()), "sph_h_features")
        return X

    def h_record(self, capacity, rate=1.0, seed=1):
        """Start (capacity > 0) or stop (0) recording training samples in
        sph_step into device tensors this object keeps; returns the number
        held."""
        torch = self._torch
        held = C.c_int64()
        if capacity > 0:
            rec = getattr(self, "_rec", None)
            if rec is None or rec[1].numel() != capacity:
                rec = (torch.empty((capacity, MLP_XSTRIDE), dtype=torch.float32, device="cuda"),
                       torch.empty(capacity, dtype=torch.float32, device="cuda"))
                self._rec = rec
            _check(lib().sph_h_record(self.h, rec[0].data_ptr(), rec[1].data_ptr(), int(capacity), float(rate),
                                      int(seed), C.byref(held)), "sph_h_record")
        else:
            _check(lib().sph_h_record(self.h, None, None, 0, float(rate), int(seed), C.byref(held)), "sph_h_record")
            self._rec = None
        return held.value

    def h_train(self, epochs, batch=16384, lr=1e-3, seed=1, init=True):
        """Train the predictor on the recorded samples; returns the mean
        minibatch loss of the last epoch."""
        L = C.c_double()
        _check(lib().sph_h_train(self.h, int(epochs), int(batch), float(lr), int(seed), int(bool(init)),
                                 C.byref(L)), "sph_h_train")
        return L.value

    def h_set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == MLP_NP
        _check(lib().sph_h_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))), "sph_h_set_params")

    def h_get_params(self):
        a = np.zeros(MLP_NP, dtype=np.float32)
        _check(lib().sph_h_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))), "sph_h_get_params")
        return a

    def h_predict(self, on=True):
        _check(lib().sph_h_predict(self.h, int(bool(on))), "sph_h_predict")
        self._predict = bool(on)

    def stats(self):
        s = Stats()
        _check(lib().sph_get_stats(self.h, C.byref(s)), "sph_get_stats")
        return s.as_dict()

    def domain_sums(self):
        out = np.zeros(5 * self.n_domains)
        _check(lib().sph_domain_sums(self.h, out.ctypes.data_as(C.POINTER(C.c_double))),
               "sph_domain_sums")
        return out.reshape(self.n_domains, 5)

    def run(self):
        """build_cells -> sort_cells -> density -> ghost -> force."""
        self.build_cells()
        self.sort_cells()
        self.density()
        self.ghost()
        self.force()
        return self
