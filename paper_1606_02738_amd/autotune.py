"""Launch-configuration autotuner of the SPH step.

Times whole kick-drift-kick steps through the C-ABI for a set of candidate
configurations on the caller's particle set and returns the fastest.  The
tunables are the leaf size (n_split: the tile of particles one wave holds),
the execution form of the force loop (one wave per leaf over a plain grid,
or persistent workgroups draining per-XCD leaf queues, with the number of
resident workgroups), the pair-pruning mode, the force form (each pair once with
atomic j-side sums, or every particle gathering its own pairs), hipGraph
capture of the density, ghost and force stages, and how many steps the
cells and lists are kept (the list skin).  A second stage sweeps, around
the fastest of those, the kernel axes: the occupancy target (waves per SIMD)
the density and the force kernels are compiled for, and the neighbour-cell
entries they stage per batch.  Every candidate starts from the same saved state, so each is timed
on identical work; the particle tensors are restored afterwards.  Steps are
averaged (not the median) so that the occasional rebuild of a candidate
that keeps its lists is paid for.

Results are cached in a JSON file keyed by a description of the workload
(particle count, box count, precision, smoothing-length span, device name).
"""
from __future__ import annotations

import json
import math
import os
import time

from . import sph as S

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sph_hip_autotune.json")


def _key(t, n_domains, precision):
    import torch
    H = t["H"]
    n = H.numel()
    Hs = H[:: max(1, n // 1_000_000)].float()
    q = torch.quantile(Hs, torch.tensor([0.001, 0.999], device=Hs.device)).cpu().numpy()
    span = float(q[1] / q[0])
    dev = torch.cuda.get_device_name(H.device)
    return "n=%d|boxes=%d|%s|hspan=%d|%s" % (n, n_domains, precision, int(round(math.log2(max(span, 1.0)))), dev)


def candidates(full=False):
    """Candidate configurations.  The default set is a coordinate sweep
    around the plain configuration; full=True is the whole product."""
    base = dict(n_split=64, exec_mode="grid", persistent_wgs=0, prune="box", use_graph=False, rebuild_steps=0,
                force="gather")
    if full:
        out = []
        for ns in (32, 48, 64):
            for ex, wgs in (("grid", 0), ("persistent", 1024), ("persistent", 2048), ("persistent", 4096)):
                for pr, fo in (("box", "gather"), ("box", "pairs"), ("sorted", "pairs")):
                    for g in (False, True):
                        for rs in (0, 8, 32):
                            out.append(dict(n_split=ns, exec_mode=ex, persistent_wgs=wgs, prune=pr, use_graph=g,
                                            rebuild_steps=rs, force=fo))
        return out
    out = [dict(base)]
    for ns in (32, 40, 48, 56):
        out.append(dict(base, n_split=ns))
    for wgs in (1024, 2048, 4096):
        out.append(dict(base, exec_mode="persistent", persistent_wgs=wgs))
    out.append(dict(base, force="pairs"))
    out.append(dict(base, prune="sorted", force="pairs"))
    out.append(dict(base, use_graph=True))
    for rs in (4, 8, 16, 32, 64):
        out.append(dict(base, rebuild_steps=rs))
        out.append(dict(base, rebuild_steps=rs, use_graph=True))
        out.append(dict(base, rebuild_steps=rs, exec_mode="persistent", persistent_wgs=2048))
    out.append(dict(base, rebuild_steps=32, force="pairs"))
    return out


KERNEL_WAVES = (4, 5, 6, 8)
KERNEL_BATCH = (16, 32)


def kernel_candidates(best):
    """Second-stage candidates: the kernel axes swept one at a time around
    `best` (the other two at their defaults, 0)."""
    base = dict(best, waves_density=0, waves_force=0, batch=0)
    out = []
    for w in KERNEL_WAVES:
        out.append(dict(base, waves_density=w))
        out.append(dict(base, waves_force=w))
    for b in KERNEL_BATCH:
        out.append(dict(base, batch=b))
    return out


def _time_config(boxes, t, state, cfg, precision, dt, steps, warmup):
    """Mean ms per step.  A candidate that keeps its cells and lists for
    many steps may rebuild rarely or never inside the few timed steps, so
    its builds are amortised: the timed steps without their builds, plus the
    mean build time over the interval between builds (seen in the timed
    steps when there are two or more, else half the candidate's
    rebuild_steps: the displacement margin, twice the displacement since
    the build, uses up the skin of rebuild_steps displacements by then)."""
    import torch
    for k in t:
        t[k].copy_(state[k])
    sim = S.SPH(boxes, precision=precision, **cfg)
    try:
        sim.bind(t)
        sim.run()
        cold_build_ms = sim.stats()["t_build_ms"]
        for _ in range(warmup):
            sim.step(dt)
        torch.cuda.synchronize()
        nb = sim.stats()["n_builds"]
        per = []
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step(dt)
            per.append(sim.stats())
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        return amortised_ms(wall_ms, per, nb, cold_build_ms, cfg.get("rebuild_steps", 0))
    finally:
        sim.close()


def amortised_ms(wall_ms, per, n_builds0, cold_build_ms, rebuild_steps):
    """Mean ms per step of `len(per)` timed steps (per: each step's stats,
    n_builds0: the build count before them) with the builds amortised over
    their interval (see _time_config)."""
    steps = len(per)
    if rebuild_steps == 0:
        return wall_ms / steps
    built = []
    nb = n_builds0
    for k, st in enumerate(per):
        if st["n_builds"] > nb:
            built.append(k)
        nb = st["n_builds"]
    build_ms = [per[k]["t_build_ms"] for k in built]
    rest = (wall_ms - sum(build_ms)) / steps
    mean_build = sum(build_ms) / len(build_ms) if build_ms else cold_build_ms
    interval = (built[-1] - built[0]) / (len(built) - 1) if len(built) >= 2 else max(1.0, rebuild_steps / 2.0)
    return rest + mean_build / interval


def autotune(boxes, t, precision, dt, steps=8, warmup=1, cands=None, cache=DEFAULT_CACHE, log=None, refresh=False,
             kernel_axes=True):
    """Return (best configuration dict, table of (configuration, ms/step)).
    t: the particle tensors (restored on return); dt: the step to time.
    kernel_axes: run the second stage over the kernel axes (FP32 modes)."""
    import numpy as np
    import torch
    n_domains = int(np.asarray(boxes).reshape(-1, 3).shape[0])
    key = _key(t, n_domains, precision)
    db = {}
    if cache and os.path.exists(cache):
        try:
            db = json.load(open(cache))
        except (OSError, ValueError):
            db = {}
    if not refresh and key in db:
        return db[key]["best"], db[key]["table"]
    state = {k: v.clone() for k, v in t.items()}
    table = []

    def run(cfgs):
        for cfg in cfgs:
            ms = _time_config(boxes, t, state, cfg, precision, dt, steps, warmup)
            table.append((cfg, ms))
            if log:
                log("autotune %s: %.2f ms/step" % (cfg, ms))

    try:
        run(cands or candidates())
        if kernel_axes and precision != "fp64":
            stage1 = min(table, key=lambda r: r[1])[0]
            run(kernel_candidates(stage1))
            # the best value of each kernel axis together
            best_of = {}
            for cfg, ms in table[-len(kernel_candidates(stage1)):]:
                for ax in ("waves_density", "waves_force", "batch"):
                    if cfg[ax] and (ax not in best_of or ms < best_of[ax][1]):
                        best_of[ax] = (cfg[ax], ms)
            combo = dict(stage1, **{ax: v for ax, (v, _) in best_of.items()})
            run([combo])
    finally:
        for k in t:
            t[k].copy_(state[k])
        del state
        torch.cuda.empty_cache()
    best = min(table, key=lambda r: r[1])[0]
    if cache:
        db[key] = {"best": best, "table": table}
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache + ".tmp", "w") as f:
                json.dump(db, f, indent=1)
            os.replace(cache + ".tmp", cache)
        except OSError:
            pass
    return best, table
