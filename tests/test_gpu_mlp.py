"""Learned H predictor on the GPU against its FP64 oracle (oracle/mlp.py):
network inference (MFMA, split-bfloat16 activations), loss gradient and Adam
(float32), the feature kernel, and the end-to-end effect in KDK steps: the
converged state does not depend on the predictor, and the trained network
leaves fewer particles for the second sweep than the plain warm start."""
import numpy as np
import pytest
import torch  # noqa: F401

import gen
import oracle
from gpu_helpers import log
from oracle import mlp as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()
    from paper_1606_02738_amd import sph as S
    S.lib()
    oracle.build()


def _params(seed=3):
    rng = np.random.default_rng(seed)
    p = M.init_params(seed, xmu=rng.normal(size=M.NIN) * 0.3, xsd=0.5 + rng.uniform(size=M.NIN),
                      ymu=0.002, ysd=0.01)
    for k in ("b1", "b2", "b3", "b4"):
        o, s = M.OFF[k]
        p[o:o + s] = rng.normal(size=s) * 0.3
    return p.astype(np.float32)


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 8), dtype=np.float32)
    X[:, :7] = rng.normal(size=(n, 7)) * np.array([1.0, 1.5, 0.5, 0.3, 0.2, 0.01, 0.05])
    y = (0.002 + 0.01 * rng.normal(size=n)).astype(np.float32)
    return X, y


def _pad(X):
    out = np.zeros((X.shape[0], M.NIN))
    out[:, :X.shape[1]] = X
    return out


@pytest.mark.parametrize("n", [1, 16, 1037])
def test_forward_matches_oracle(n):
    import torch
    from paper_1606_02738_amd import sph as S
    log("case mlp forward n=%d" % n)
    p = _params()
    X, _ = _rows(n, 7)
    yg = S.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    w = M.unpack(p.astype(np.float64))
    lay = M._layers(w, _pad(X.astype(np.float64)))
    o = lay[-1]
    yo = w["ymu"] + w["ysd"] * o
    # float32 accumulation with activations carried as two bfloat16 terms
    # (relative error 2^-17 each): bound by the magnitude of the output sum
    scale = np.abs(lay[-2]) @ np.abs(w["w4"]) + abs(w["b4"])
    err = np.abs(yg - yo) / (w["ysd"] * scale)
    log("max normalised error %.3g" % err.max())
    assert err.max() < 2e-5


@pytest.mark.parametrize("n", [1000, 20011])
def test_loss_grad_matches_oracle(n):
    """1000 rows: one tile of 32 rows per workgroup; 20011: 626 tiles over
    the 256 workgroups, the last one ragged."""
    import torch
    from paper_1606_02738_amd import sph as S
    log("case mlp loss/grad n=%d" % n)
    p = _params(5)
    X, y = _rows(n, 9)
    L, g = S.mlp_loss_grad(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    Lo, go = M.loss_grad(p.astype(np.float64), _pad(X.astype(np.float64)), y.astype(np.float64))
    log("loss gpu %.8g oracle %.8g" % (L, Lo))
    assert abs(L - Lo) <= 1e-5 * Lo
    for k in ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4"):
        o, s = M.OFF[k]
        ref = go[o:o + s]
        e = np.max(np.abs(g[o:o + s] - ref)) / (np.max(np.abs(ref)) + 1e-30)
        log("grad %s rel err %.3g" % (k, e))
        assert e < 1e-4, k


def test_adam_matches_oracle():
    import torch
    from paper_1606_02738_amd import sph as S
    log("case mlp adam")
    rng = np.random.default_rng(4)
    p = _params(2)
    pt = torch.from_numpy(p.copy()).cuda()
    m = torch.zeros(M.NT, dtype=torch.float32, device="cuda")
    v = torch.zeros(M.NT, dtype=torch.float32, device="cuda")
    po, mo, vo = p.astype(np.float64), np.zeros(M.NT), np.zeros(M.NT)
    for t in range(1, 4):
        g = (rng.normal(size=M.NT) * 10.0 ** rng.uniform(-4, 0, size=M.NT)).astype(np.float32)
        S.mlp_adam(pt, m, v, torch.from_numpy(g).cuda(), t, 1e-3)
        po, mo, vo = M.adam(po, mo, vo, g.astype(np.float64), t, 1e-3)
    pg = pt.cpu().numpy().astype(np.float64)
    # float32 rounding of p and of the update
    assert np.max(np.abs(pg[:M.NT] - po[:M.NT]) / (np.abs(po[:M.NT]) * 2e-7 + 1e-3 * 1e-4)) < 3.0
    assert np.array_equal(pg[M.NT:], p[M.NT:].astype(np.float64))


@pytest.mark.parametrize("case", ["clustered", "ensemble"])
def test_features_match_oracle(case):
    """Feature kernel vs the oracle's features on the oracle's converged
    state (H, rho, P, du/dt handed to the GPU as inputs)."""
    import torch
    from paper_1606_02738_amd import sph as S
    log("case features %s" % case)
    if case == "clustered":
        d = gen.clustered(24, n_halos=10, seed=2741)
        parts = [d]
    else:
        d = gen.ensemble(4, side_range=(10, 14), seed=5)
        parts = oracle.split_domains(d)
    n = d["x"].size
    for k in ("H", "rho", "P", "dudt"):
        d[k] = np.zeros(n)
    dt = 1e-3
    Fo = np.zeros((n, M.NIN))
    for b in parts:
        o = oracle.full(b, tree=True)
        idx = b["index"] if "index" in b else np.arange(n)
        for k in ("H", "rho", "P", "dudt"):
            d[k][idx] = o[k]
        F, _ = M.features(b["x"], b["y"], b["z"], b["vx"], b["vy"], b["vz"], o["H"], o["rho"], o["P"], o["dudt"],
                          b["box"], dt)
        Fo[idx] = F
    boxes = d["boxes"] if d["boxes"].shape[0] > 1 else d["box"]
    sim = S.SPH(boxes, precision="fp32c")
    t = S.to_device(d)
    sim.bind(t)
    sim.build_cells()
    X = sim.h_features(dt)
    torch.cuda.synchronize()
    ids = t["id"].cpu().numpy()
    Xg = np.zeros((n, 8))
    Xg[ids] = X.cpu().numpy()
    sim.close()
    # integer counts behind columns 1 and 2 are exact
    assert np.array_equal(np.rint(np.exp(Xg[:, 1])), np.rint(np.exp(Fo[:, 1])))
    # FP64 on both sides, then one rounding to float32 (a rounding boundary
    # can put the two one float32 ulp apart)
    for k in range(7):
        e = np.max(np.abs(Xg[:, k] - Fo[:, k]) / (np.abs(Fo[:, k]) + 1e-300))
        log("feature %d max rel err %.3g" % (k, e))
        assert np.all(np.abs(Xg[:, k] - Fo[:, k]) <= 2.5e-7 * np.abs(Fo[:, k])), k
    assert np.all(Xg[:, 7] == 0)


def _clone(t):
    return {k: v.clone() for k, v in t.items()}


def test_predictor_in_steps():
    """Record samples over plain steps, train with the library's kernels,
    then run the same steps from one state with and without the predictor:
    identical converged state within the convergence tolerance, fewer
    particles left for a second sweep with the predictor than with the
    previous H as the start of the iteration (the method the predictor
    replaces).  The start carried along the flow (h_drift) is run from the
    same state as well and its fraction printed beside them."""
    import math
    import torch
    from paper_1606_02738_amd import sph as S
    log("case predictor clustered 40^3 fp32c")
    d = gen.clustered(40, n_halos=30, seed=2741)
    sim = S.SPH(d["box"], precision="fp32c", h_drift=False)
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    H = t["H"]
    cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(t["u"].max()))
    dt = 0.25 * float(H.min()) / math.sqrt(10.0 / 3.0) / cs
    sim.h_record(2_000_000, rate=0.5, seed=9)
    for _ in range(16):
        sim.step(dt)
    held = sim.h_record(2_000_000, rate=0.5, seed=9)
    log("samples held %d" % held)
    assert held > 100_000
    loss = sim.h_train(epochs=6, batch=4096, lr=2e-3, seed=3)
    log("training loss (standardised) %.4g" % loss)
    assert loss < 0.5
    sim.h_record(0)
    n = t["x"].numel()
    state = _clone(t)
    res = {}
    for mode in ("plain", "mlp", "drift"):
        for k in t:
            t[k].copy_(state[k])
        ss = S.SPH(d["box"], precision="fp32c", h_drift=True) if mode == "drift" else sim
        ss.bind(t)
        ss.build_cells()
        ss.sort_cells()
        ss.density()
        ss.ghost()
        ss.force()
        if ss is sim:
            sim.h_predict(mode == "mlp")
        fb, sw = [], []
        for _ in range(4):
            ss.step(dt)
            st = ss.stats()
            fb.append(st["unconv_after"][0] / n)
            sw.append(st["sweeps"])
        torch.cuda.synchronize()
        res[mode] = (S.to_host(t), np.mean(fb), np.mean(sw))
        log("%s: second-sweep fraction %.4g, mean sweeps %.2f" % (mode, res[mode][1], res[mode][2]))
        if ss is not sim:
            ss.close()
    sim.close()
    a = res["plain"][0]
    for other in ("mlp", "drift"):
        b = res[other][0]
        # same physical state: H and rho agree to the FP32 convergence tolerance
        assert np.max(np.abs(a["H"] - b["H"]) / a["H"]) < 1e-4
        assert np.max(np.abs(a["rho"] - b["rho"]) / a["rho"]) < 3e-4
    assert res["mlp"][1] < res["plain"][1]
