#!/usr/bin/env python3
"""Benchmark of the SPH neighbour-interaction hot path on one MI355X.

Workload: the clustered cosmology-like periodic unit box, 256^3 = 16,777,216
equal-mass particles (lognormal density field with sigma_ln = 1.5 plus 500
NFW halos, concentrations 5-15, log-uniform masses over 3 decades),
synthetic and seeded.  One step = one kick-drift-kick step through the
C-ABI: cell rebuild (Morton keys, radix sort, octree, neighbour-cell lists),
per-direction sort, density sweeps with the FP64 smoothing-length test
(warm-started), ghost, symmetric force, kicks and FP64 conservation sums.

Metric: SPH neighbour interactions per second, counting N_dens = sum_i
#{j : r_ij < H_i} (self included) plus 2 N_force with N_force the unordered
pairs within max(H_i, H_j), divided by the wall time of whole steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32/FP64 operations per evaluated interaction (an FMA counts
# as 2): density pair (distance, kernel value and H-derivative, two
# accumulations; the FP32 modes add the second H-derivative sum used to
# accept a final small Newton update) and symmetric force pair (distance, both kernel gradients,
# both sides' acceleration and du/dt).  Compensated sums add 4 per
# accumulation.  Only pairs inside the range are counted.
FLOPS_DENS = {"fp32c": 39, "fp32": 31, "fp64": 23}
FLOPS_FORCE = {"fp32c": 64, "fp32": 52, "fp64": 52}
# gather-form force: per ordered pair (each unordered pair is evaluated from
# both sides), distance, both kernel gradients, the particle's own
# acceleration and du/dt only
FLOPS_FORCE_GATHER = {"fp32c": 59, "fp32": 47, "fp64": 47}
# MI355X published peaks: FP32 vector 157.3 TFLOP/s (the packed-FP32 rate),
# FP64 vector 78.6 TFLOP/s.  256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x
# 2.4 GHz = 78.6 TFLOP/s is also the FP32 rate without packed instructions,
# which this build does not generate; it is reported beside the published peak.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def measured_traffic(kernel, workload, cfg):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none, it was taken with another launch
    configuration, or the interaction-kernel sources have changed since."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "%s_%s_hbm.md" % (kernel, workload))
    if not os.path.exists(f):
        return None
    kv = {}
    for line in open(f):
        if ":" in line and not line.startswith((" ", "#", "|")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in ("paper_1606_02738_amd/csrc/sph_interact.hip", "paper_1606_02738_amd/csrc/sph_device.h",
                "paper_1606_02738_amd/csrc/sph_internal.h"):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if kv.get("sources_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in kv:
        return None
    want = "n_split=%d exec=%s persistent_wgs=%d prune=%s" % (cfg["n_split"], cfg["exec_mode"],
                                                            cfg["persistent_wgs"], cfg["prune"])
    if kv.get("config") != want:
        return None
    return float(kv["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_interp(d, o, seed, n_pts=16):
    """The interpolation oracle (brute force over all particles, numpy on
    the host) on the oracle's own converged state of the baseline sample."""
    import numpy as np
    from oracle import interp as OI
    rng = np.random.default_rng(seed + 99)
    P = rng.random((n_pts, 3)) * d["box"]
    t0 = time.perf_counter()
    OI.interpolate(P[:, 0], P[:, 1], P[:, 2], d["x"], d["y"], d["z"], d["m"], o["rho"], o["H"], d["u"],
                   d["box"], chunk=4)
    dt = time.perf_counter() - t0
    return {"value": n_pts / dt, "unit": "points/s", "kind": "oracle",
            "sample": "%d random points over the %d particles of the baseline sample (all particles "
                      "visited per point), %.1f s" % (n_pts, d["x"].size, dt)}


def interp_eval(sim, t, box, n_grid=128, reps=5):
    """Eq. (interp) of u onto the cell centres of an n_grid^3 mesh from the
    current state (after the timed steps), timed with events on the
    library's stream."""
    import torch
    dev = t["x"].device
    L = [float(b) for b in box]
    axes = [(torch.arange(n_grid, device=dev, dtype=torch.float64) + 0.5) * (L[a] / n_grid) for a in range(3)]
    X, Y, Z = torch.meshgrid(*axes, indexing="ij")
    px, py, pz = X.contiguous().view(-1), Y.contiguous().view(-1), Z.contiguous().view(-1)
    del X, Y, Z
    out = sim.interpolate(t["u"], px, py, pz)  # warm-up
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(reps):
        out = sim.interpolate(t["u"], px, py, pz)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    m_pts = px.numel()
    # the mesh mean of the interpolant estimates its exact box average
    # sum_i (m_i/rho_i) u_i / V (each kernel integrates to one): equal up to
    # the mesh sampling (a consistency figure of the field, not a parity check)
    exact = float((t["m"] / t["rho"] * t["u"]).sum()) / (L[0] * L[1] * L[2])
    log("interpolation: %d points in %.3f ms" % (m_pts, ms))
    return {"points": m_pts, "ms_per_call": ms, "points_per_s": m_pts / (ms / 1e3), "field": "u",
            "mesh_mean": float(out.mean()), "box_average": exact}


def cpu_baseline(n_side, seed):
    """The FP64 oracle (k-d tree, OpenMP over the host's threads) on the same
    clustered recipe at n_side^3 particles: density solve from the same kind
    of initial guess, ghost and force."""
    import gen
    import oracle
    oracle.build()
    d = gen.clustered(n_side, seed=seed, n_halos=max(1, int(round(500 * (n_side / 256) ** 3))))
    t0 = time.perf_counter()
    o = oracle.full(d, tree=True)
    dt = time.perf_counter() - t0
    inter = o["n_dens"] + 2 * o["n_force"]
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    interp = cpu_interp(d, o, seed)
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle", "interpolation": interp,
            "sample": "clustered recipe at %d^3 = %d particles (%.3g of the workload), full density "
                      "solve + ghost + force, %.1f s; %s, %d cores in the affinity mask" % (
                          n_side, n_side ** 3, (n_side / 256) ** 3, dt, model, len(os.sched_getaffinity(0)))}


def parity_eval(sim, t, box, n_sample=3000, tails=200, seed=7):
    """Per-quantity errors of the timed configuration against the FP64
    oracle, after the timed region: density, ghost and force on the stepped
    state with the cells and lists kept from their last build, against the
    oracle's H solved for every particle of that state (from its own
    count-based starting guess) and its force on a sample of particles (random
    plus both tails of the H distribution).  a and du/dt are normalised per
    particle by the sums of their term magnitudes."""
    import numpy as np
    import torch
    import gen
    import oracle
    from paper_1606_02738_amd import sph as S
    sim.density_ghost_force()
    torch.cuda.synchronize()
    st = sim.stats()
    g = S.to_host(t, order_by_id=False)
    n = g["x"].size
    t0 = time.perf_counter()
    b = np.asarray(box, dtype=np.float64)
    tree = oracle.Tree(g["x"], g["y"], g["z"], b)
    H0 = gen._initial_H_from_counts(g["x"], g["y"], g["z"], g["m"], b)
    s = oracle.solve_h(g["x"], g["y"], g["z"], g["m"], H0, b, tree=tree)
    gh = oracle.ghost(s["rho"], s["drho"], s["H"], g["u"])
    rng = np.random.default_rng(seed)
    order = np.argsort(s["H"])
    idx = np.unique(np.concatenate([rng.choice(n, n_sample, replace=False), order[:tails], order[-tails:]]))
    f = oracle.force(g["x"], g["y"], g["z"], g["vx"], g["vy"], g["vz"], g["m"], s["H"], gh["A"], b,
                     tree=tree, idx=idx)
    oracle_s = time.perf_counter() - t0
    da = np.sqrt((g["ax"][idx] - f["ax"][idx]) ** 2 + (g["ay"][idx] - f["ay"][idx]) ** 2 +
                 (g["az"][idx] - f["az"][idx]) ** 2)
    out = {"state": "after the timed steps; density, ghost and force with lists kept %d steps since their "
                    "build" % st["steps_since_build"],
           "rho_max_rel": float(np.max(np.abs(g["rho"] - s["rho"]) / s["rho"])),
           "H_max_rel": float(np.max(np.abs(g["H"] - s["H"]) / s["H"])),
           "omega_max_rel_sample": float(np.max(np.abs(g["omega"][idx] - gh["omega"][idx]) /
                                                np.abs(gh["omega"][idx]))),
           "a_max_over_Sa_sample": float(np.max(da / f["sa"][idx])),
           "a_l2_rel_sample": float(np.sqrt(np.sum(da ** 2) / np.sum(f["ax"][idx] ** 2 + f["ay"][idx] ** 2 +
                                                                     f["az"][idx] ** 2))),
           "dudt_max_over_Su_sample": float(np.max(np.abs(g["dudt"][idx] - f["dudt"][idx]) /
                                                   np.maximum(f["su"][idx], 1e-300))),
           "count_mismatch_sample": int(np.sum(g["nngb"][idx] != s["cnt"][idx])),
           "rho_H_particles": int(n), "force_sample": int(idx.size),
           "targets": {"rho": 1e-5, "H": 1e-5, "a": 1e-4},
           "oracle_s": oracle_s, "oracle_threads": oracle.num_threads()}
    out["within_targets"] = bool(out["rho_max_rel"] <= 1e-5 and out["H_max_rel"] <= 1e-5 and
                                 out["a_max_over_Sa_sample"] <= 1e-4)
    log("parity vs oracle: rho %.3g H %.3g a %.3g du %.3g (oracle %.1f s)" % (
        out["rho_max_rel"], out["H_max_rel"], out["a_max_over_Sa_sample"], out["dudt_max_over_Su_sample"],
        oracle_s))
    return out


def wide_h_eval(S, prec, cfg, n_side=128, steps=10, warmup=2, seed=77):
    """Smoothing lengths over three decades (Sec. 2: h follows the local
    density over orders of magnitude): log-density sigma 3, half of the
    particles in concentrated halos over four decades of mass, at n_side^3,
    stepped in the timed configuration; step time and interactions per
    second, then the sampled oracle parity of the stepped state."""
    import numpy as np
    import torch
    import gen
    n_halos = max(1, int(round(40 * (n_side / 40) ** 3)))
    log("wide H range: generating %d^3 ..." % n_side)
    d = gen.clustered(n_side, seed=seed, n_halos=n_halos, sigma_ln=3.0, halo_frac=0.5, c_range=(15.0, 40.0),
                      decades=4.0)
    box = d["box"]
    t = S.to_device(d)
    del d
    sim = S.SPH(box, precision=prec, **cfg)
    sim.bind(t)
    t0 = time.perf_counter()
    sim.run()
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
    stc = sim.stats()
    H = t["H"]
    Hs = H.float()
    q = torch.quantile(Hs[::max(1, Hs.numel() // 2_000_000)], torch.tensor([0.001, 0.999], device=Hs.device))
    q = q.cpu().numpy()
    span = float(H.max() / H.min())
    cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(t["u"].max()))
    dt = 0.25 * float(H.min()) / math.sqrt(10.0 / 3.0) / cs
    for _ in range(warmup):
        sim.step(dt)
    torch.cuda.synchronize()
    st0 = sim.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step(dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st1 = sim.stats()
    inter = (st1["n_dens_total"] - st0["n_dens_total"]) + 2 * (st1["n_force_total"] - st0["n_force_total"])
    out = {"n_particles": int(H.numel()), "n_halos": n_halos, "H_span_min_max": span,
           "H_span_0.1_99.9": float(q[1] / q[0]), "cold_start_s": cold, "cold_start_sweeps": stc["sweeps"],
           "depth": stc["depth"], "leaves": stc["n_leaves"], "dt": dt, "steps": steps,
           "ms_per_step": wall / steps * 1e3, "interactions_per_s": inter / wall,
           "builds": st1["n_builds"] - st0["n_builds"]}
    log("wide H range %d^3: H span %.0f, %.2f ms/step, %.3g interactions/s" % (
        n_side, span, out["ms_per_step"], out["interactions_per_s"]))
    out["parity"] = parity_eval(sim, t, box)
    sim.close()
    return out


def mlp_eval(S, sim, t, dt, steps, make_sim, rec_steps=50, seed=17):
    """Learned H predictor on the same workload: record samples over
    `rec_steps` plain steps, train with the library's kernels, then time
    `steps` steps from one saved state with the plain start of the H
    iteration (previous H carried along the flow; and the previous H as
    is, in a context made by `make_sim(h_drift=False)`) and with the
    predictor."""
    import torch
    n = t["x"].numel()
    rate = min(1.0, 6.0e6 / (rec_steps * n))
    cap = int(rate * n * rec_steps * 1.2) + 1024
    sim.h_record(cap, rate=rate, seed=seed)
    t0 = time.perf_counter()
    for _ in range(rec_steps):
        sim.step(dt)
    torch.cuda.synchronize()
    rec_s = time.perf_counter() - t0
    held = sim.h_record(cap, rate=rate, seed=seed)
    log("predictor: %d samples from %d plain steps (%.1f s)" % (held, rec_steps, rec_s))
    t0 = time.perf_counter()
    loss = sim.h_train(epochs=4, batch=16384, lr=2e-3, seed=seed)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log("predictor: trained in %.2f s, loss %.4g" % (train_s, loss))
    sim.h_record(0)
    state = {k: v.clone() for k, v in t.items()}
    res = {}
    for mode in ("plain", "plain_previous_h", "mlp"):
        for k in t:
            t[k].copy_(state[k])
        ss = make_sim(h_drift=False) if mode == "plain_previous_h" else sim
        ss.bind(t)
        ss.run()
        if ss is sim:
            sim.h_predict(mode == "mlp")
        ss.step(dt)
        torch.cuda.synchronize()
        per = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ss.step(dt)
            per.append(ss.stats())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if ss is not sim:
            ss.close()
        res[mode] = {"ms_per_step": wall / steps * 1e3,
                     "mean_sweeps": sum(q["sweeps"] for q in per) / steps,
                     "second_sweep_fraction": sum(q["unconv_after"][0] for q in per) / (steps * n),
                     "density_ms_per_step": sum(q["t_density_ms"] for q in per) / steps,
                     "density_evals_per_neighbour": sum(q["n_dens_evals"] for q in per)
                     / max(1, sum(q["n_dens"] for q in per)),
                     "predict_ms_per_step": (sum(q["t_predict_ms"] for q in per) / steps) if mode == "mlp" else 0.0,
                     "H": t["H"].clone()}
        log("predictor %s: %.2f ms/step, sweeps %.2f, second-sweep fraction %.4g" % (
            mode, res[mode]["ms_per_step"], res[mode]["mean_sweeps"], res[mode]["second_sweep_fraction"]))
    sim.h_predict(False)
    dH = float(((res["mlp"]["H"] - res["plain"]["H"]).abs() / res["plain"]["H"]).max())
    for m in res.values():
        del m["H"]
    return {"samples": held, "record_steps": rec_steps, "train_s": train_s, "train_loss": loss,
            "epochs": 4, "batch": 16384, "plain": res["plain"], "plain_previous_h": res["plain_previous_h"],
            "mlp": res["mlp"],
            "max_rel_H_difference": dH,
            "step_time_ratio_mlp_over_plain": res["mlp"]["ms_per_step"] / res["plain"]["ms_per_step"]}


def precision_eval(S, box, t, dt, cfg, steps=5):
    """Form (1) against the plain precisions: the same state stepped with
    each arithmetic (FP64, FP32 plain sums, FP32 cell-relative compensated),
    same launch configuration; ms per step and interactions per second."""
    import torch
    state = {k: v.clone() for k, v in t.items()}
    res = {}
    for prec in ("fp64", "fp32", "fp32c"):
        for k in t:
            t[k].copy_(state[k])
        sim = S.SPH(box, precision=prec, **cfg)
        sim.bind(t)
        sim.run()
        sim.step(dt)
        torch.cuda.synchronize()
        per = []
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step(dt)
            per.append(sim.stats())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        res[prec] = {"ms_per_step": wall / steps * 1e3,
                     "interactions_per_s": sum(q["n_dens"] + 2 * q["n_force"] for q in per) / wall,
                     "force_kernel_ms": sum(q["t_force_kernel_ms"] for q in per) / steps,
                     "density_kernels_ms": sum(q["t_density_kernels_ms"] for q in per) / steps}
        log("precision %s: %.2f ms/step" % (prec, res[prec]["ms_per_step"]))
    for k in t:
        t[k].copy_(state[k])
    return res


def rebuild_every_step_eval(S, box, t, dt, cfg, prec, steps=10):
    """The same state and launch configuration with the cells and lists
    rebuilt at every step (rebuild_steps = 0): the step time without the
    amortisation of keeping them."""
    import torch
    state = {k: v.clone() for k, v in t.items()}
    sim = S.SPH(box, precision=prec, **dict(cfg, rebuild_steps=0))
    sim.bind(t)
    sim.run()
    sim.step(dt)
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step(dt)
        per.append(sim.stats())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    for k in t:
        t[k].copy_(state[k])
    inter = sum(q["n_dens"] + 2 * q["n_force"] for q in per)
    out = {"ms_per_step": wall / steps * 1e3, "interactions_per_s": inter / wall, "steps": steps,
           "build_ms_per_step": sum(q["t_build_ms"] for q in per) / steps}
    log("rebuild every step: %.2f ms/step" % out["ms_per_step"])
    return out


def ensemble_eval(S, prec, steps=3, seed=2743, rebuild_steps=0):
    """64 independent periodic boxes (n_side ~ U{16..96}): every stage of a
    step as one launch over all boxes, against 64 contexts stepped one after
    the other (the plain solves).  Same dt for both; per-box FP64 totals."""
    import numpy as np
    import torch
    import gen
    t0 = time.perf_counter()
    d = gen.ensemble(64, seed=seed)
    log("ensemble: %d particles in 64 boxes (%.1f s)" % (d["x"].size, time.perf_counter() - t0))
    boxes = d["boxes"]
    out = {"n_particles": int(d["x"].size), "boxes": 64,
           "box_sizes": [int(v) for v in np.bincount(d["domain"], minlength=64)]}
    # sequential plain solves: one context per box
    parts = []
    for b in range(64):
        idx = np.nonzero(d["domain"] == b)[0]
        sub = {k: np.ascontiguousarray(d[k][idx]) for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m", "H", "id")}
        parts.append((boxes[b], sub))
    t_all = S.to_device(d)
    union = {}
    dt = None
    for mode in ("persistent", "grid"):
        tt = {k: v.clone() for k, v in t_all.items()}
        sim = S.SPH(boxes, precision=prec, exec_mode=mode, rebuild_steps=rebuild_steps)
        sim.bind(tt)
        sim.run()
        if dt is None:
            cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(tt["u"].max()))
            dt = 0.25 * float(tt["H"].min()) / math.sqrt(10.0 / 3.0) / cs
        sim.step(dt)
        torch.cuda.synchronize()
        sums0 = sim.domain_sums()
        per = []
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step(dt)
            per.append(sim.stats())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sums1 = sim.domain_sums()
        inter = sum(q["n_dens"] + 2 * q["n_force"] for q in per)
        union[mode] = {"ms_per_step": wall / steps * 1e3, "interactions_per_s": inter / wall,
                       "mean_sweeps": sum(q["sweeps"] for q in per) / steps,
                       "phase_ms_per_step": {k: sum(q["t_%s_ms" % k] for q in per) / steps
                                             for k in ("density", "ghost", "force")},
                       "builds": per[-1]["n_builds"] - per[0]["n_builds"] + (per[0]["steps_since_build"] == 0),
                       "max_rel_mass_change": float(np.max(np.abs(sums1[:, 0] - sums0[:, 0]) / sums0[:, 0])),
                       "max_rel_energy_change": float(np.max(np.abs(sums1[:, 4] - sums0[:, 4]) / sums0[:, 4]))}
        sim.close()
        del tt
        log("ensemble union (%s): %.2f ms/step" % (mode, union[mode]["ms_per_step"]))
    del t_all
    sims = []
    for box, sub in parts:
        tb = S.to_device(sub)
        sb = S.SPH(box, precision=prec, rebuild_steps=rebuild_steps)
        sb.bind(tb)
        sb.run()
        sb.step(dt)
        sims.append((sb, tb))
    torch.cuda.synchronize()
    inter = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        for sb, tb in sims:
            sb.step(dt)
            q = sb.stats()
            inter += q["n_dens"] + 2 * q["n_force"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for sb, tb in sims:
        sb.close()
    seq = {"ms_per_step": wall / steps * 1e3, "interactions_per_s": inter / wall}
    log("ensemble sequential: %.2f ms/step" % seq["ms_per_step"])
    best = min(union.values(), key=lambda r: r["ms_per_step"])
    out.update({"precision": prec, "rebuild_steps": rebuild_steps, "dt": dt, "steps": steps, "union": union,
                "sequential": seq,
                "speedup_union_over_sequential": seq["ms_per_step"] / best["ms_per_step"]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-side", type=int, default=256)
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp64"])
    ap.add_argument("--exec", dest="exec_mode", default="grid", choices=["grid", "persistent"])
    ap.add_argument("--n-split", type=int, default=64)
    ap.add_argument("--prune", default="box", choices=["box", "sorted"])
    ap.add_argument("--graph", action="store_true", help="density, ghost and force from one captured hipGraph")
    ap.add_argument("--persistent-wgs", type=int, default=0)
    ap.add_argument("--rebuild-steps", type=int, default=0,
                    help="keep cells and lists across steps with a skin for this many steps (0: rebuild every step)")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="run the configuration given by the flags instead of the autotuner's choice")
    ap.add_argument("--cpu-n-side", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--force", choices=("pairs", "gather"), default=None,
                    help="force form (default: the autotuner's choice, else gather with box pruning)")
    ap.add_argument("--lists", choices=("cell", "particle"), default="cell",
                    help="neighbour lists of the density and force kernels (default: the autotuner's choice)")
    ap.add_argument("--tile", type=int, default=0, help="LDS segment of the particle-list kernels")
    ap.add_argument("--waves-density", type=int, default=0, help="occupancy target of the density kernel (0: 6)")
    ap.add_argument("--waves-force", type=int, default=0, help="occupancy target of the force kernel (0: 5)")
    ap.add_argument("--batch", type=int, default=0, help="neighbour-cell entries staged per batch (0: 32)")
    ap.add_argument("--no-h-drift", action="store_true",
                    help="start the H iteration of a step from the previous H as is")
    ap.add_argument("--seed", type=int, default=2741)
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned H predictor comparison")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-box ensemble comparison")
    ap.add_argument("--no-wide-h", action="store_true", help="skip the three-decade smoothing-length workload")
    ap.add_argument("--wide-h-n-side", type=int, default=128)
    ap.add_argument("--no-forms", action="store_true", help="skip the FP64 / FP32 / FP32C step comparison")
    ap.add_argument("--mlp-steps", type=int, default=5)
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the oracle comparison of the stepped state after the timed region")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 512 MiB device copy first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    from paper_1606_02738_amd import sph as S

    assert torch.cuda.is_available(), "needs a GPU"
    S.lib()
    if args.calib_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log("generating clustered %d^3 ..." % args.n_side)
    t0 = time.perf_counter()
    d = gen.clustered(args.n_side, seed=args.seed,
                      n_halos=max(1, int(round(500 * (args.n_side / 256) ** 3))))
    log("generated in %.1f s" % (time.perf_counter() - t0))
    n = d["x"].size
    box = d["box"]
    cfg = dict(n_split=args.n_split, exec_mode=args.exec_mode, persistent_wgs=args.persistent_wgs,
               prune=args.prune, use_graph=args.graph, rebuild_steps=args.rebuild_steps,
               h_drift=not args.no_h_drift, force=args.force or ("gather" if args.prune == "box" else "pairs"),
               lists=args.lists, tile=args.tile, waves_density=args.waves_density, waves_force=args.waves_force,
               batch=args.batch)
    sim = S.SPH(box, precision=args.precision, **cfg)
    t = S.to_device(d)
    del d
    sim.bind(t)
    log("initial convergence (cold start) ...")
    t0 = time.perf_counter()
    sim.run()
    torch.cuda.synchronize()
    st0 = sim.stats()
    log("cold start: %.2f s, sweeps=%d leaves=%d depth=%d list=%d" % (
        time.perf_counter() - t0, st0["sweeps"], st0["n_leaves"], st0["depth"], st0["n_list"]))
    H = t["H"]
    Hs = H[::max(1, n // 2_000_000)].float()
    q = torch.quantile(Hs, torch.tensor([0.001, 0.999], device=Hs.device)).cpu().numpy()
    h_span = float(q[1] / q[0])
    cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(t["u"].max()))
    dt = 0.25 * float(H.min()) / math.sqrt(10.0 / 3.0) / cs
    tune_table = None
    if args.tune:
        from paper_1606_02738_amd import autotune as AT
        sim.close()
        t0 = time.perf_counter()
        cfg, tune_table = AT.autotune(box, t, args.precision, dt, cache=None, log=log)
        cfg = dict(cfg, h_drift=not args.no_h_drift)
        if args.force:
            cfg["force"] = args.force
        log("autotune: %s (%.1f s)" % (cfg, time.perf_counter() - t0))
        sim = S.SPH(box, precision=args.precision, **cfg)
        sim.bind(t)
        sim.run()

    for k in range(args.warmup):
        sim.step(dt)
        log("warmup step %d done" % k)
    torch.cuda.synchronize()
    # the timed region: steps only (a step reads the device twice on its own;
    # the interaction counts are running totals on the device, read after)
    st0 = sim.stats()
    tstep = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sim.step(dt)
        tstep.append(time.perf_counter())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st1 = sim.stats()
    dts = np.diff([t0] + tstep) * 1e3
    builds = st1["n_builds"] - st0["n_builds"]
    assert st1["force_calls"] - st0["force_calls"] == args.steps
    inter = (st1["n_dens_total"] - st0["n_dens_total"]) + 2 * (st1["n_force_total"] - st0["n_force_total"])
    force_pairs = st1["n_force_total"] - st0["n_force_total"]
    dens_total = st1["n_dens_total"] - st0["n_dens_total"]
    log("timed %d steps in %.3f s (%d cell builds)" % (args.steps, wall, builds))
    # phase breakdown and kernel durations: further steps, each followed by a
    # stats read, after the timed region
    per = []
    for k in range(min(args.steps, 10)):
        sim.step(dt)
        per.append(sim.stats())
    kper = per
    if cfg["use_graph"]:
        # kernels inside the graph are not timed one by one: time the same
        # kernels, launched the same way without the graph, after the timed region
        ksim = S.SPH(box, precision=args.precision, **dict(cfg, use_graph=False))
        ksim.bind(t)
        ksim.run()
        kper = []
        for _ in range(min(args.steps, 3)):
            ksim.step(dt)
            kper.append(ksim.stats())
        ksim.close()
        sim.bind(t)
        sim.run()

    t_dgf = sum(s["t_density_ms"] + s["t_ghost_ms"] + s["t_force_ms"] for s in per) / 1e3
    inter_phase = sum(s["n_dens"] + 2 * s["n_force"] for s in per)
    # per-kernel durations and the work of those launches
    dens_ms = sum(s["t_density_kernels_ms"] for s in kper)
    dens_launch = sum(s["n_density_launches"] for s in kper)
    force_ms = sum(s["t_force_kernel_ms"] for s in kper)
    prec = args.precision
    # the method's own work: density interactions evaluated (all sweeps) and
    # unordered force pairs, each counted once (Sec. 3.1 pair symmetry), with
    # the algorithmic flops of one evaluation; the gather form's issued work
    # (every pair from both sides) is reported beside it
    dens_flops = sum(s["n_dens_evals"] for s in kper) * FLOPS_DENS[prec]
    force_flops = sum(s["n_force"] for s in kper) * FLOPS_FORCE[prec]
    force_issued = (sum(2 * s["n_force"] for s in kper) * FLOPS_FORCE_GATHER[prec] if cfg["force"] == "gather"
                    else force_flops)
    fname = "k_force_gather" if cfg["force"] == "gather" else "k_force"
    if dens_ms >= force_ms:
        kname, kflops, kms, klaunch, kissued = "k_density", dens_flops, dens_ms, dens_launch, dens_flops
    else:
        kname, kflops, kms, klaunch, kissued = fname, force_flops, force_ms, len(kper), force_issued
    peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
    achieved = kflops / (kms / 1e3) / 1e12
    traffic = measured_traffic(kname, "clustered%d_%s" % (args.n_side, prec), cfg)
    roof = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "peak_source": "published MI355X %s vector peak" % ("FP64" if prec == "fp64" else "FP32"),
            "peak_nonpacked": PEAK_NONPACKED_TFLOPS,
            "frac_of_nonpacked": achieved / PEAK_NONPACKED_TFLOPS,
            "launches": klaunch, "avg_launch_ms": kms / max(1, klaunch),
            "flop_per_launch": kflops / max(1, klaunch),
            "flop_basis": ("unordered pairs x %d flops (each pair once)" % FLOPS_FORCE[prec]) if kname != "k_density"
            else ("density interactions evaluated x %d flops" % FLOPS_DENS[prec]),
            "issued_flop_per_launch": kissued / max(1, klaunch)}
    other = {"k_density": {"ms_total": dens_ms, "launches": dens_launch,
                           "tflops": dens_flops / max(dens_ms, 1e-9) / 1e9,
                           "frac_of_peak": dens_flops / max(dens_ms, 1e-9) / 1e9 / peak},
             fname: {"ms_total": force_ms, "launches": len(kper),
                     "tflops": force_flops / max(force_ms, 1e-9) / 1e9,
                     "frac_of_peak": force_flops / max(force_ms, 1e-9) / 1e9 / peak,
                     "issued_tflops": force_issued / max(force_ms, 1e-9) / 1e9},
             "timed_without_graph": bool(cfg["use_graph"])}

    out = {
        "metric": "SPH neighbour interactions/s (density+force) + step time, 256^3 clustered, vs oracle",
        "value": inter / wall,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "ms_per_step_median": float(np.median(dts)),
        "ms_per_step_mean_without_first_last": float(np.mean(dts[1:-1])) if len(dts) > 2 else float(np.mean(dts)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "clustered %d^3 periodic unit box: lognormal sigma_ln=1.5 + NFW halos, "
                               "h span %.0fx (0.1-99.9%%)" % (args.n_side, h_span),
                   "n_particles": n, "precision": prec, "exec": cfg["exec_mode"], "n_split": cfg["n_split"],
                   "persistent_wgs": cfg["persistent_wgs"], "prune": cfg["prune"], "graph": bool(cfg["use_graph"]),
                   "rebuild_steps": cfg["rebuild_steps"], "h_drift": bool(cfg["h_drift"]),
                   "force": cfg["force"], "lists": cfg.get("lists", "cell"), "tile": cfg.get("tile", 0),
                   "waves_density": cfg.get("waves_density", 0), "waves_force": cfg.get("waves_force", 0),
                   "batch": cfg.get("batch", 0),
                   "autotuned": bool(args.tune), "dt": dt},
        "builds": builds,
        "interactions_per_step": inter / args.steps,
        "n_dens_per_step": dens_total / args.steps,
        "n_force_per_step": force_pairs / args.steps,
        "phase_steps": len(per),
        "build_ms_per_step": sum(s["t_build_ms"] for s in per) / len(per),
        "interactions_per_s_density_ghost_force": inter_phase / t_dgf,
        "mean_sweeps": sum(s["sweeps"] for s in per) / len(per),
        "unconverged_after_sweep": [s["unconv_after"][:s["sweeps"]] for s in per],
        "density_evals_per_neighbour": sum(s["n_dens_evals"] for s in per) / max(1, sum(s["n_dens"] for s in per)),
        "phase_ms_per_step": {"density": sum(s["t_density_ms"] for s in per) / len(per),
                              "ghost": sum(s["t_ghost_ms"] for s in per) / len(per),
                              "force": sum(s["t_force_ms"] for s in per) / len(per)},
        "kernels": other,
        "roofline": roof,
    }
    if tune_table is not None:
        out["autotune"] = [dict(c, ms_per_step=ms) for c, ms in tune_table]
    if not args.no_parity:
        out["parity"] = parity_eval(sim, t, box)
    if not args.no_forms:
        sim.close()
        out["rebuild_every_step"] = rebuild_every_step_eval(S, box, t, dt, cfg, prec)
        out["precision_forms"] = precision_eval(S, box, t, dt, cfg)
        sim = S.SPH(box, precision=args.precision, **cfg)
        sim.bind(t)
        sim.run()
    out["interpolation"] = interp_eval(sim, t, box)
    if not args.no_mlp:
        out["h_predictor"] = mlp_eval(S, sim, t, dt, args.mlp_steps,
                                      lambda **kw: S.SPH(box, precision=args.precision, **dict(cfg, **kw)))
    sim.close()
    del t
    torch.cuda.empty_cache()
    if not args.no_wide_h:
        out["wide_h_range"] = wide_h_eval(S, args.precision, cfg, n_side=args.wide_h_n_side)
        torch.cuda.empty_cache()
    if not args.no_ensemble:
        out["ensemble"] = ensemble_eval(S, args.precision, rebuild_steps=cfg["rebuild_steps"])
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n_side, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
