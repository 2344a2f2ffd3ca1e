"""The configuration the benchmark times, against the oracle.

The benchmark steps with cells and neighbour lists kept across steps (a skin
of rebuild_steps step displacements), the force loop drained from the
persistent per-XCD queues, and each step's H iteration started from the
previous H carried along the flow.  These tests put exactly that path next
to the FP64 oracle:

- small boxes: the oracle steps the same initial state itself (its own
  kick-drift-kick, Sec. 3.1 integrator) and the trajectories are compared
  per particle; then the GPU evaluates density, ghost and force on its final
  state with the kept lists and the oracle evaluates that same state;
- the full 256^3 clustered box: after the benchmark's warm-up steps the
  GPU evaluates density, ghost and force on the stepped state with the lists
  built steps earlier, and the oracle evaluates the same state from scratch
  (H solved for every particle, forces on a sample that includes both tails
  of the H distribution).  The state after the steps is the common input;
  the converged H, rho, Omega, a and du/dt are what is compared.
"""
import math

import numpy as np
import pytest
import torch  # noqa: F401

import gen
import oracle
from gpu_helpers import TOL_FP32, log

pytestmark = pytest.mark.gpu


def _cfl_dt(t):
    """The benchmark's step: CFL 0.25 on the smallest H (in the Dehnen-Aly
    convention) with the largest sound speed (u is uniform at the start)."""
    cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(t["u"].max()))
    return 0.25 * float(t["H"].min()) / math.sqrt(10.0 / 3.0) / cs


def _sample_errors(g, s, gh, f, idx):
    e = {}
    e["rho"] = float(np.max(np.abs(g["rho"][idx] - s["rho"][idx]) / s["rho"][idx]))
    e["H"] = float(np.max(np.abs(g["H"][idx] - s["H"][idx]) / s["H"][idx]))
    e["omega"] = float(np.max(np.abs(g["omega"][idx] - gh["omega"][idx]) / np.abs(gh["omega"][idx])))
    da = np.sqrt((g["ax"][idx] - f["ax"][idx]) ** 2 + (g["ay"][idx] - f["ay"][idx]) ** 2 +
                 (g["az"][idx] - f["az"][idx]) ** 2)
    e["a"] = float(np.max(da / f["sa"][idx]))
    e["du"] = float(np.max(np.abs(g["dudt"][idx] - f["dudt"][idx]) / np.maximum(f["su"][idx], 1e-300)))
    e["count_mismatch"] = int(np.sum(g["nngb"][idx] != s["cnt"][idx]))
    return e


CASES = [("clustered32", "fp64", 8), ("clustered32", "fp64", 64), ("clustered32", "fp32c", 8),
         ("clustered32", "fp32c", 64), ("sod", "fp64", 64), ("sod", "fp32c", 64)]


@pytest.mark.parametrize("case,prec,rs", CASES)
def test_kept_lists_steps_vs_oracle(case, prec, rs):
    """Six steps with kept lists, persistent force queues and the flow-carried
    H start, against six oracle steps from the same converged state; then
    the GPU's density + ghost + force on its final state with the lists kept
    from its last build, against the oracle's evaluation of that state."""
    from paper_1606_02738_amd import sph as S
    log("case kept lists %s %s rebuild_steps=%d persistent h_drift" % (case, prec, rs))
    if case == "sod":
        d = gen.sod(16)
    else:
        d = gen.clustered(32, n_halos=20, seed=2761)
    n_steps = 6
    sim = S.SPH(d["box"], precision=prec, exec_mode="persistent", rebuild_steps=rs, h_drift=True,
                force="gather")
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    torch.cuda.synchronize()
    dt = 2.0 ** -11 if case == "sod" else _cfl_dt(t)
    kept = 0
    for _ in range(n_steps):
        sim.step(dt)
        kept += sim.stats()["steps_since_build"] > 0
    traj = S.to_host(t)
    sim.density_ghost_force()
    torch.cuda.synchronize()
    st = sim.stats()
    g = S.to_host(t)
    sim.close()
    log("steps with kept lists %d of %d; final evaluation %d steps after its build" % (
        kept, n_steps, st["steps_since_build"]))
    if case != "sod" and rs == 64:
        assert kept >= n_steps - 1 and st["steps_since_build"] > 0

    # the oracle: the same initial state, its own converged start and steps
    o = oracle.full(d, tree=True)
    s = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d.items()}
    s["H"] = o["H"].copy()
    for k in ("ax", "ay", "az", "dudt"):
        s[k] = o[k].copy()
    for _ in range(n_steps):
        oracle.step(s, dt, tree=True)
    tol = 1e-9 if prec == "fp64" else 2e-5
    L = np.asarray(d["box"], dtype=np.float64)
    for a, k in enumerate(("x", "y", "z")):
        dx = traj[k] - s[k]
        dx -= L[a] * np.round(dx / L[a])
        assert np.max(np.abs(dx)) < tol * 0.1 * L[a], k
    vs = max(np.max(np.abs(s[k])) for k in ("vx", "vy", "vz")) + 1e-30
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(traj[k] - s[k])) < tol * vs, k
    assert np.max(np.abs(traj["u"] - s["u"]) / s["u"]) < tol

    # final evaluation: the GPU's density, ghost and force with its kept lists
    # on its own final state, against the oracle's evaluation of that state
    # (its H solve starts from the oracle trajectory's H)
    fin = {k: traj[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m")}
    fin["H"] = s["H"].copy()
    fin["box"] = d["box"]
    of = oracle.full(fin, tree=True)
    e = {}
    e["rho"] = float(np.max(np.abs(g["rho"] - of["rho"]) / of["rho"]))
    e["H"] = float(np.max(np.abs(g["H"] - of["H"]) / of["H"]))
    e["omega"] = float(np.max(np.abs(g["omega"] - of["omega"]) / np.abs(of["omega"])))
    da = np.sqrt((g["ax"] - of["ax"]) ** 2 + (g["ay"] - of["ay"]) ** 2 + (g["az"] - of["az"]) ** 2)
    e["a"] = float(np.max(da / of["sa"]))
    e["du"] = float(np.max(np.abs(g["dudt"] - of["dudt"]) / np.maximum(of["su"], 1e-300)))
    mism = int(np.sum(g["nngb"] != of["cnt"]))
    log("final evaluation errors: " + ", ".join("%s=%.3g" % kv for kv in e.items()) +
        ", count mismatches %d" % mism)
    if prec == "fp64":
        for k in ("rho", "H", "omega", "a", "du"):
            assert e[k] <= 1e-8, (k, e[k])
        assert mism == 0
        assert st["n_dens"] == of["n_dens"] and st["n_force"] == of["n_force"]
    else:
        for k in ("rho", "H", "omega", "a", "du"):
            assert e[k] <= TOL_FP32[k], (k, e[k])
        assert mism <= max(2, 1e-3 * g["nngb"].size)


def test_clustered_256_timed_config_vs_oracle():
    """The benchmark's workload and configuration at full size: cold start,
    five kept-list steps of the benchmark's dt (persistent force queues,
    rebuild_steps = 64, gather force, flow-carried H start), then density,
    ghost and force on the stepped state with the lists built before the
    steps.  The oracle solves H for every particle of that state and
    evaluates the force on 3000 random particles plus the 200 of smallest
    and the 200 of largest H.  Targets: rho and H <= 1e-5 relative, Omega
    <= 1e-4, a <= 1e-4 of S_a = sum_j m_j |A_i dW_i + A_j dW_j| and du/dt
    <= 1e-4 of its own magnitude sum, per particle."""
    from paper_1606_02738_amd import sph as S
    log("case clustered 256^3 fp32c timed configuration: generating")
    d = gen.clustered(256, seed=2741)
    n = d["x"].size
    sim = S.SPH(d["box"], precision="fp32c", exec_mode="persistent", prune="box", rebuild_steps=64,
                h_drift=True, force="gather")
    t = S.to_device(d)
    del d
    sim.bind(t)
    sim.run()
    dt = _cfl_dt(t)
    for _ in range(5):
        sim.step(dt)
    sim.density_ghost_force()
    torch.cuda.synchronize()
    st = sim.stats()
    g = S.to_host(t, order_by_id=False)
    sim.close()
    del t
    log("gpu: %d steps since the build, sweeps %d, unconverged %d" % (
        st["steps_since_build"], st["sweeps"], st["n_unconverged"]))
    assert st["steps_since_build"] >= 4 and st["n_unconverged"] == 0
    box = np.array([1.0, 1.0, 1.0])
    tree = oracle.Tree(g["x"], g["y"], g["z"], box)
    # the oracle's own starting guess (cell counts of the stepped positions)
    H0 = gen._initial_H_from_counts(g["x"], g["y"], g["z"], g["m"], box)
    s = oracle.solve_h(g["x"], g["y"], g["z"], g["m"], H0, box, tree=tree)
    gh = oracle.ghost(s["rho"], s["drho"], s["H"], g["u"])
    rng = np.random.default_rng(7)
    order = np.argsort(s["H"])
    idx = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), order[:200], order[-200:]]))
    f = oracle.force(g["x"], g["y"], g["z"], g["vx"], g["vy"], g["vz"], g["m"], s["H"], gh["A"], box,
                     tree=tree, idx=idx)
    e = _sample_errors(g, s, gh, f, idx)
    log("errors on %d sampled particles: %s" % (idx.size, e))
    e_all_rho = float(np.max(np.abs(g["rho"] - s["rho"]) / s["rho"]))
    e_all_H = float(np.max(np.abs(g["H"] - s["H"]) / s["H"]))
    log("all particles: rho %.3g H %.3g" % (e_all_rho, e_all_H))
    assert e_all_rho <= TOL_FP32["rho"] and e_all_H <= TOL_FP32["H"]
    assert e["omega"] <= TOL_FP32["omega"] and e["a"] <= TOL_FP32["a"] and e["du"] <= TOL_FP32["du"]
    assert e["count_mismatch"] <= max(2, 1e-3 * idx.size)
