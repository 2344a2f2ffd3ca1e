"""Host-side checks of the C-ABI library: it loads, exports every function
that include/sph.h declares, and rejects bad arguments before touching the
GPU.  No compute calls (no GPU needed)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1606_02738_amd import sph as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sph.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"(?:sph_status|const char\s*\*)\s+(sph_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(S.LIB_PATH):
        from paper_1606_02738_amd import build
        build.build()
    return S.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 12, names
    for f in names:
        assert hasattr(L, f), f
    assert set(S.EXPORTS) <= set(names)


def test_status_strings_and_version(L):
    assert L.sph_status_str(0) == b"ok"
    for code in (-1, -2, -3, -4, -5, -6, -7):
        assert L.sph_status_str(code) != b"unknown status"
    assert b"gfx950" in L.sph_version()


def _params(**kw):
    p = S.Params()
    box = np.ones(3)
    p.gamma, p.eta, p.kernel_gamma, p.h_tol = 5 / 3, 1.2348, math.sqrt(10 / 3), 1e-6
    p.max_h_iter, p.n_split, p.precision, p.exec_mode = 20, 64, 1, 0
    p.n_domains, p.persistent_wgs, p.use_graph, p.prune = 1, 0, 0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    p.boxes = box.ctypes.data_as(C.POINTER(C.c_double))
    return p, box


@pytest.mark.parametrize("bad", [dict(gamma=1.0), dict(eta=0.0), dict(h_tol=0.0), dict(max_h_iter=0),
                                 dict(n_split=0), dict(n_split=65), dict(precision=7),
                                 dict(exec_mode=3), dict(n_domains=0), dict(prune=2), dict(use_graph=2), dict(rebuild_steps=-1),
                                 dict(h_drift=2), dict(force_mode=2), dict(force_mode=1, prune=1),
                                 dict(lists=2), dict(lists=1, force_mode=0), dict(tile=100),
                                 dict(waves_density=3), dict(waves_force=7), dict(batch=8)])
def test_create_rejects_bad_params(L, bad):
    p, box = _params(**bad)
    h = C.c_void_p()
    # the parameters are checked before the workspace is touched
    assert L.sph_create(C.byref(p), C.c_void_p(4096), S.WORKSPACE_MIN, None, C.byref(h)) == -1
    assert not h.value


def test_create_requires_a_workspace(L):
    p, box = _params()
    h = C.c_void_p()
    assert L.sph_create(C.byref(p), None, 1 << 30, None, C.byref(h)) == -1
    assert L.sph_create(C.byref(p), C.c_void_p(4096), S.WORKSPACE_MIN - 1, None, C.byref(h)) == -1
    assert not h.value


def test_workspace_size_queries(L):
    p, box = _params()
    b = C.c_size_t()
    assert L.sph_workspace_size(C.byref(p), 1000, C.byref(b)) == 0
    small = b.value
    assert small >= S.WORKSPACE_MIN
    assert L.sph_workspace_size(C.byref(p), 1 << 24, C.byref(b)) == 0
    assert b.value > small + (1 << 24) * 64
    assert L.sph_workspace_size(C.byref(p), 0, C.byref(b)) == -1
    assert L.sph_workspace_size(None, 10, C.byref(b)) == -1
    p2, _ = _params(lists=1, force_mode=1)
    assert L.sph_workspace_size(C.byref(p2), 1 << 24, C.byref(b)) == 0
    # the gradient kernel runs at most 256 workgroups of 32-row tiles: the
    # workspace grows with n up to 256 workgroups' partials, then stays
    assert L.sph_mlp_workspace_size(1024, C.byref(b)) == 0
    assert b.value >= 1024 // 32 * S.MLP_NT * 4
    assert L.sph_mlp_workspace_size(16384, C.byref(b)) == 0
    cap = b.value
    assert cap >= 256 * S.MLP_NT * 4
    assert L.sph_mlp_workspace_size(1 << 26, C.byref(b)) == 0
    assert b.value == cap
    assert L.sph_mlp_workspace_size(-1, C.byref(b)) == -1


def test_library_allocates_no_device_memory():
    """The library carves every buffer from the caller's workspace: its
    dynamic symbol table imports no HIP allocation routine."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None or not os.path.exists(S.LIB_PATH):
        pytest.skip("nm or the library not available")
    out = subprocess.run([nm, "-D", "--undefined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    imported = {l.split()[-1].split("@")[0] for l in out.splitlines() if l.strip()}
    assert "hipLaunchKernel" in imported
    for f in ("hipMalloc", "hipFree", "hipMallocManaged", "hipExtMallocWithFlags", "hipMallocAsync",
              "hipFreeAsync", "hipHostMalloc"):
        assert f not in imported, f


def test_null_arguments(L):
    assert L.sph_create(None, None, 0, None, None) == -1
    assert L.sph_destroy(None) == 0
    for f in ("sph_sort_cells", "sph_density", "sph_ghost", "sph_force", "sph_density_ghost_force"):
        assert getattr(L, f)(None) == -1
    assert L.sph_step(None, 0.1) == -1
    assert L.sph_build_cells(None, None) == -1
    assert L.sph_interpolate(None, None, None, None, None, None, 0, None) == -1


def test_predictor_calls_reject_bad_arguments(L):
    """The predictor entry points check their arguments before any GPU work."""
    vp = C.c_void_p
    assert L.sph_mlp_forward(None, None, 0, None, None, 0, None) == 0        # nothing to do
    assert L.sph_mlp_forward(None, None, 5, None, None, 0, None) == -1
    assert L.sph_mlp_forward(vp(1), vp(1), -1, vp(1), None, 0, None) == -1
    assert L.sph_mlp_forward(vp(1), vp(1), 5, vp(1), None, 1 << 20, None) == -1   # no workspace
    assert L.sph_mlp_loss_grad(None, None, None, 0, None, None, None, 0, None) == -1
    assert L.sph_mlp_loss_grad(vp(1), vp(1), vp(1), 5, vp(1), None, None, 1 << 20, None) == -1
    assert L.sph_mlp_adam(None, None, None, None, 1, C.c_float(1e-3), C.c_float(0.9), C.c_float(0.999),
                          C.c_float(1e-8), None) == -1
    assert L.sph_mlp_adam(vp(1), vp(1), vp(1), vp(1), 0, C.c_float(1e-3), C.c_float(0.9), C.c_float(0.999),
                          C.c_float(1e-8), None) == -1
    assert L.sph_h_features(None, 0.1, None) == -1
    held = C.c_int64()
    assert L.sph_h_record(None, None, None, 10, 0.5, 1, C.byref(held)) == -1
    assert L.sph_h_train(None, 1, 16, 1e-3, 1, 1, None) == -1
    assert L.sph_h_set_params(None, None) == -1
    assert L.sph_h_get_params(None, None) == -1
    assert L.sph_h_predict(None, 1) == -1


def test_predictor_layout_constants_match_the_oracle():
    from oracle import mlp as M
    txt = open(os.path.join(ROOT, "include", "sph.h")).read()
    consts = dict(re.findall(r"#define (SPH_MLP_\w+) (\d+)", txt))
    assert int(consts["SPH_MLP_NT"]) == M.NT == S.MLP_NT
    assert int(consts["SPH_MLP_NP"]) == M.NP == S.MLP_NP
    assert int(consts["SPH_MLP_NIN"]) == M.NIN and int(consts["SPH_MLP_NH"]) == M.NH
    assert int(consts["SPH_MLP_NF"]) == M.NF
