"""Eq. (interp) on the GPU (sph_interpolate through the C-ABI) against the
oracle's brute-force sum, on points that are random, on particles, on the
box faces and outside the box, after the density stage and after lazy steps
whose particles have moved since the cells were built.  The error of each
point is normalised by the same sum taken with |Q| (the scale of the terms)."""
import numpy as np
import pytest
import torch  # noqa: F401

import gen
import oracle
from oracle import interp as OI
from gpu_helpers import log, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()
    from paper_1606_02738_amd import sph as S
    S.lib()
    oracle.build()


def _points(d, box, n_rand, seed, n_mesh=0):
    """Random points, particle positions, points on the faces and outside,
    and the cell centres of an n_mesh^3 mesh (dense enough that the 64
    points of a wave after the sort share one top cell: the wave-cooperative
    walk)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64)
    P = [rng.random((n_rand, 3)) * L]
    if n_mesh:
        g = (np.arange(n_mesh) + 0.5) / n_mesh
        X, Y, Z = np.meshgrid(g * L[0], g * L[1], g * L[2], indexing="ij")
        P.append(np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1))
    idx = rng.choice(d["x"].size, size=min(200, d["x"].size), replace=False)
    P.append(np.stack([d["x"][idx], d["y"][idx], d["z"][idx]], 1))
    f = rng.random((64, 3)) * L
    f[:16, 0] = 0.0
    f[16:32, 1] = np.nextafter(L[1], 0.0)
    f[32:48, 2] = L[2]
    f[48:, :] += L * rng.integers(-2, 3, (16, 3))
    P.append(f)
    P = np.concatenate(P)
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy()


def _gpu_interp(sim, t, Q, px, py, pz, pdom=None):
    import torch
    dev = t["x"].device
    Qc = torch.from_numpy(Q).to(dev)[t["id"]].contiguous()  # current particle order
    args = [torch.from_numpy(a).to(dev) for a in (px, py, pz)]
    pd = None if pdom is None else torch.from_numpy(pdom.astype(np.int32)).to(dev)
    out = sim.interpolate(Qc, *args, pdom=pd)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(g, o, s_abs, tol, what):
    err = np.abs(g - o) / np.maximum(s_abs, 1e-300)
    log("%s: %d points, max normalised error %.3g (mean |Q| sum %.3g)" % (what, g.size, float(np.max(err)),
                                                                         float(np.mean(s_abs))))
    assert np.all(np.isfinite(g))
    assert np.max(err) <= tol, what


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-7), ("fp32c", 1e-4)])
def test_interp_after_density(prec, tol):
    from paper_1606_02738_amd import sph as S
    log("case interp lattice16 jitter %s" % prec)
    d = gen.lattice(16, vsigma=0.1, seed=4401)
    rng = np.random.default_rng(4402)
    Q = rng.normal(size=d["x"].size)
    sim = S.SPH(d["box"], precision=prec)
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    px, py, pz = _points(d, d["box"], 3000, 4403, n_mesh=24)
    g = _gpu_interp(sim, t, Q, px, py, pz)
    # the unit field through the same call: the normalisation sum
    g1 = _gpu_interp(sim, t, np.ones_like(Q), px, py, pz)
    sim.close()
    o = oracle_run(d)
    args = (d["x"], d["y"], d["z"], d["m"], o["rho"], o["H"])
    ov = OI.interpolate(px, py, pz, *args, Q, d["box"])
    sa = OI.interpolate(px, py, pz, *args, np.abs(Q), d["box"])
    _check(g, ov, sa, tol, "random Q")
    o1 = OI.interpolate(px, py, pz, *args, np.ones_like(Q), d["box"])
    _check(g1, o1, o1, tol, "unit Q")


def test_interp_clustered_deep_tree():
    """Clustered particles: H over several decades, a deep octree to prune."""
    from paper_1606_02738_amd import sph as S
    log("case interp clustered 32^3 fp64")
    d = gen.clustered(32, n_halos=20, seed=4411)
    rng = np.random.default_rng(4412)
    Q = 1.0 + 0.5 * rng.normal(size=d["x"].size)
    sim = S.SPH(d["box"], precision="fp64")
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    # half of the points at particles (dense regions), half random
    px, py, pz = _points(d, d["box"], 1000, 4413, n_mesh=16)
    idx = rng.choice(d["x"].size, 1000, replace=False)
    px = np.concatenate([px, d["x"][idx]])
    py = np.concatenate([py, d["y"][idx]])
    pz = np.concatenate([pz, d["z"][idx]])
    g = _gpu_interp(sim, t, Q, px, py, pz)
    st = sim.stats()
    sim.close()
    log("depth %d leaves %d" % (st["depth"], st["n_leaves"]))
    o = oracle_run(d)
    args = (d["x"], d["y"], d["z"], d["m"], o["rho"], o["H"])
    ov = OI.interpolate(px, py, pz, *args, Q, d["box"])
    sa = OI.interpolate(px, py, pz, *args, np.abs(Q), d["box"])
    _check(g, ov, sa, 1e-7, "clustered")


def test_interp_after_lazy_steps():
    """Cells kept across steps (rebuild every 8): particles have moved since
    the build, so the walk relies on the motion margin."""
    from paper_1606_02738_amd import sph as S
    log("case interp lattice16 fp64 three lazy steps")
    d = gen.lattice(16, vsigma=0.3, seed=4421)
    dt = 0.01
    rng = np.random.default_rng(4422)
    Q = rng.normal(size=d["x"].size)
    sim = S.SPH(d["box"], precision="fp64", rebuild_steps=8)
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    for _ in range(3):
        sim.step(dt)
    st = sim.stats()
    assert st["steps_since_build"] > 0 and st["list_margin"] > 0.0
    h = S.to_host(t)
    px, py, pz = _points(h, d["box"], 3000, 4423, n_mesh=24)
    g = _gpu_interp(sim, t, Q, px, py, pz)
    sim.close()
    o = oracle.full(d, tree=True)
    s = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d.items()}
    s["H"] = o["H"].copy()
    for k in ("ax", "ay", "az", "dudt"):
        s[k] = o[k].copy()
    for _ in range(3):
        oracle.step(s, dt, tree=True)
    args = (s["x"], s["y"], s["z"], s["m"], s["rho"], s["H"])
    ov = OI.interpolate(px, py, pz, *args, Q, d["box"])
    sa = OI.interpolate(px, py, pz, *args, np.abs(Q), d["box"])
    _check(g, ov, sa, 1e-7, "after lazy steps")


def test_interp_ensemble_with_box_index():
    """Several boxes: each point names its box; a bad box index or a NaN
    coordinate gives NaN for that point only."""
    from paper_1606_02738_amd import sph as S
    log("case interp ensemble 4 boxes fp32c")
    d = gen.ensemble(4, (12, 16), seed=4431)
    rng = np.random.default_rng(4432)
    Q = rng.normal(size=d["x"].size)
    sim = S.SPH(d["boxes"], precision="fp32c")
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    o = oracle_run(d)
    PX, PY, PZ, PD, OV, SA = [], [], [], [], [], []
    for b, sub in enumerate(oracle.split_domains(d)):
        px, py, pz = _points(sub, sub["box"], 500, 4433 + b, n_mesh=12)
        ix = sub["index"]
        args = (sub["x"], sub["y"], sub["z"], sub["m"], o["rho"][ix], o["H"][ix])
        OV.append(OI.interpolate(px, py, pz, *args, Q[ix], sub["box"]))
        SA.append(OI.interpolate(px, py, pz, *args, np.abs(Q[ix]), sub["box"]))
        PX.append(px), PY.append(py), PZ.append(pz), PD.append(np.full(px.size, b))
    px, py, pz, pd = (np.concatenate(a) for a in (PX, PY, PZ, PD))
    # two bad points at the end
    px = np.concatenate([px, [0.5, np.nan]])
    py = np.concatenate([py, [0.5, 0.5]])
    pz = np.concatenate([pz, [0.5, 0.5]])
    pd = np.concatenate([pd, [7, 0]])
    g = _gpu_interp(sim, t, Q, px, py, pz, pdom=pd)
    sim.close()
    assert np.isnan(g[-1]) and np.isnan(g[-2])
    _check(g[:-2], np.concatenate(OV), np.concatenate(SA), 1e-4, "ensemble")


def test_interp_errors():
    from paper_1606_02738_amd import sph as S
    import torch
    d = gen.lattice(16, seed=4441)
    sim = S.SPH(d["box"], precision="fp64")
    t = S.to_device(d)
    sim.bind(t)
    sim.build_cells()
    sim.sort_cells()
    p = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SPHError):
        sim.interpolate(t["u"], p, p, p)  # before the density stage
    sim.density()
    out = sim.interpolate(t["u"], p[:0], p[:0], p[:0])
    assert out.numel() == 0
    sim.close()
