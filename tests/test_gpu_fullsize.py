"""Parity at the benchmark's full size: the clustered 256^3 workload in the
configuration bench.py times (FP32 compensated, box pruning, grid launch),
checked on a sample of particles that the oracle evaluates one by one (its
smoothing lengths are solved for every particle, its forces only for the
sample)."""
import numpy as np
import pytest
import torch  # noqa: F401

import gen
import oracle
from gpu_helpers import TOL_FP32, log

pytestmark = pytest.mark.gpu


def test_clustered_256_sampled():
    from paper_1606_02738_amd import sph as S
    log("case clustered 256^3 fp32c sampled parity: generating")
    d = gen.clustered(256, seed=2741)
    n = d["x"].size
    sim = S.SPH(d["box"], precision="fp32c", exec_mode="grid", prune="box")
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    torch.cuda.synchronize()
    st = sim.stats()
    g = S.to_host(t)
    sim.close()
    del t
    log("gpu done: sweeps=%d leaves=%d; oracle solve on all %d particles" % (st["sweeps"], st["n_leaves"], n))
    assert st["n_unconverged"] == 0
    tree = oracle.Tree(d["x"], d["y"], d["z"], d["box"])
    s = oracle.solve_h(d["x"], d["y"], d["z"], d["m"], d["H"], d["box"], tree=tree)
    gh = oracle.ghost(s["rho"], s["drho"], s["H"], d["u"])
    rng = np.random.default_rng(7)
    order = np.argsort(s["H"])
    idx = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), order[:200], order[-200:]]))
    log("oracle force on %d sampled particles" % idx.size)
    f = oracle.force(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], s["H"], gh["A"], d["box"],
                     tree=tree, idx=idx)
    e_rho = np.max(np.abs(g["rho"][idx] - s["rho"][idx]) / s["rho"][idx])
    e_H = np.max(np.abs(g["H"][idx] - s["H"][idx]) / s["H"][idx])
    e_om = np.max(np.abs(g["omega"][idx] - gh["omega"][idx]) / np.abs(gh["omega"][idx]))
    da = np.sqrt((g["ax"][idx] - f["ax"][idx]) ** 2 + (g["ay"][idx] - f["ay"][idx]) ** 2 +
                 (g["az"][idx] - f["az"][idx]) ** 2)
    e_a = np.max(da / f["sa"][idx])
    e_u = np.max(np.abs(g["dudt"][idx] - f["dudt"][idx]) / f["su"][idx])
    mism = int(np.sum(g["nngb"][idx] != s["cnt"][idx]))
    log("errors on sample: rho=%.3g H=%.3g omega=%.3g a=%.3g du=%.3g count mismatches=%d" %
        (e_rho, e_H, e_om, e_a, e_u, mism))
    assert e_rho <= TOL_FP32["rho"] and e_H <= TOL_FP32["H"] and e_om <= TOL_FP32["omega"]
    assert e_a <= TOL_FP32["a"] and e_u <= TOL_FP32["du"]
    assert mism <= max(2, 1e-3 * idx.size)
    # totals are properties that hold at any size: momentum sum and the
    # dv/dt - du/dt pairing, relative to the sums of magnitudes
    m = g["m"]
    S_a = np.sum(m * np.sqrt(g["ax"] ** 2 + g["ay"] ** 2 + g["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert abs(np.sum(m * g[k])) < 1e-6 * S_a
    pw = m * (g["vx"] * g["ax"] + g["vy"] * g["ay"] + g["vz"] * g["az"])
    assert abs(np.sum(pw) + np.sum(m * g["dudt"])) < 1e-4 * np.sum(np.abs(pw))


def test_clustered_256_lazy_steps_properties():
    """The benchmark's stepping configuration at full size (cells and lists
    kept up to 64 steps, H started along the flow, gather force): three
    steps agree with the same steps rebuilding every step (to the FP32
    convergence tolerance), and the step's outputs keep the properties that
    hold at any size (zero momentum sum of the forces)."""
    import math
    from paper_1606_02738_amd import sph as S
    log("case clustered 256^3 fp32c three lazy steps: generating")
    d = gen.clustered(256, seed=2742)
    res = {}
    for rs in (64, 0):
        sim = S.SPH(d["box"], precision="fp32c", exec_mode="grid", prune="box", rebuild_steps=rs)
        t = S.to_device(d)
        sim.bind(t)
        sim.run()
        cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(t["u"].max()))
        dt = 0.25 * float(t["H"].min()) / math.sqrt(10.0 / 3.0) / cs
        for _ in range(3):
            sim.step(dt)
        torch.cuda.synchronize()
        st = sim.stats()
        res[rs] = (S.to_host(t), st)
        sim.close()
        del t
        log("rebuild_steps=%d: builds %d, sweeps %d, n_force %d" % (rs, st["n_builds"], st["sweeps"], st["n_force"]))
    a, b = res[64][0], res[0][0]
    assert res[64][1]["n_builds"] < res[0][1]["n_builds"]
    L = d["box"][0]
    for k in ("x", "y", "z"):
        dx = a[k] - b[k]
        dx -= L * np.round(dx / L)
        assert np.max(np.abs(dx)) < 1e-6 * L, k
    for k in ("rho", "H"):
        assert np.max(np.abs(a[k] - b[k]) / b[k]) < 1e-4, k
    m = a["m"]
    S_a = np.sum(m * np.sqrt(a["ax"] ** 2 + a["ay"] ** 2 + a["az"] ** 2))
    for k in ("ax", "ay", "az"):
        assert abs(np.sum(m * a[k])) < 1e-6 * S_a, k
        assert np.max(np.abs(a[k] - b[k])) <= 1e-3 * np.max(np.abs(b[k])), k
