"""The 3D shock tube at full size (100^3 + 50^3 = 1,125,000 particles, box
2x1x1, P_L = 1, P_R = 0.1): 20 kick-drift-kick steps of dt = 2^-11 on the
GPU in FP32 cell-relative arithmetic against the FP64 oracle stepping the
same state, with the per-quantity errors and the conservation of mass,
momentum and energy of both printed."""
import math

import numpy as np
import pytest
import torch  # noqa: F401

import gen
import oracle
from gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_sod_full_twenty_steps():
    from paper_1606_02738_amd import sph as S
    oracle.build()
    log("case sod 100/50 (1.125M) twenty steps fp32c vs oracle")
    d = gen.sod(100)
    dt = 2.0 ** -11
    n_steps = 20
    sim = S.SPH(d["box"], precision="fp32c")
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    cons_g = []
    for _ in range(n_steps):
        sim.step(dt)
        cons_g.append(sim.stats()["conserved"])
    torch.cuda.synchronize()
    g = S.to_host(t)
    sim.close()
    o = oracle.full(d, tree=True)
    s = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d.items()}
    s["H"] = o["H"].copy()
    for k in ("ax", "ay", "az", "dudt"):
        s[k] = o[k].copy()
    e0 = oracle.conserved(s["m"], s["vx"], s["vy"], s["vz"], s["u"])
    cons_o = []
    for _ in range(n_steps):
        oracle.step(s, dt, tree=True)
        cons_o.append(oracle.conserved(s["m"], s["vx"], s["vy"], s["vz"], s["u"]))
    spacing = 0.01
    vs = np.max(np.sqrt(s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2))
    err = {
        "x": max(np.max(np.abs(g[k] - s[k])) for k in ("x", "y", "z")) / spacing,
        "v": max(np.max(np.abs(g[k] - s[k])) for k in ("vx", "vy", "vz")) / vs,
        "u": float(np.max(np.abs(g["u"] - s["u"]) / s["u"])),
        "rho": float(np.max(np.abs(g["rho"] - s["rho"]) / s["rho"])),
        "H": float(np.max(np.abs(g["H"] - s["H"]) / s["H"])),
    }
    log("after %d steps, errors vs oracle: %s" % (n_steps, ", ".join("%s=%.3g" % kv for kv in err.items())))
    cg, co = np.array(cons_g), np.array(cons_o)
    log("energy drift: gpu %.3g, oracle %.3g (relative to the initial total)" % (
        abs(cg[-1, 4] - e0[4]) / e0[4], abs(co[-1, 4] - e0[4]) / e0[4]))
    log("momentum (x): gpu %.3g, oracle %.3g (mass-weighted |v| scale %.3g)" % (
        cg[-1, 1], co[-1, 1], float(np.sum(s["m"]) * vs)))
    # measured after 20 steps: all five below 1e-6
    for k in ("x", "v", "u", "rho", "H"):
        assert err[k] < 1e-5, k
    mass = math.fsum(d["m"])  # exactly rounded total
    assert abs(cg[-1, 0] - mass) <= 1e-12 * mass
    assert np.all(np.abs(cg[:, 4] - co[:, 4]) <= 1e-5 * e0[4])
    assert np.all(np.abs(cg[:, 1:4]) <= 1e-6 * float(np.sum(s["m"]) * vs) + np.abs(co[:, 1:4]) + 1e-12)
