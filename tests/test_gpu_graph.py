"""Graph mode: density sweeps, ghost and force replayed from one captured
hipGraph.  Results must match the host-driven path (bit for bit where the
arithmetic is order-independent: density and H are gathers) and the oracle;
the host must finish what the graph cannot (more sweeps than captured,
list rebuilds); the graph must be reused across steps."""
import numpy as np
import pytest
import torch  # noqa: F401

import gen
import oracle
from gpu_helpers import TOL_FP32, TOL_FP64, assert_close, errors, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

DGF = ("density_ghost_force",)


@pytest.fixture(scope="module", autouse=True)
def _dev():
    import torch
    assert torch.cuda.is_available()
    from paper_1606_02738_amd import sph as S
    S.lib()
    oracle.build()


@pytest.mark.parametrize("prec,mode", [("fp64", "grid"), ("fp32c", "grid"), ("fp32c", "persistent"),
                                       ("fp64", "persistent")])
def test_graph_matches_host_path(prec, mode):
    log("case graph clustered 32^3 %s %s" % (prec, mode))
    d = gen.clustered(32, n_halos=20, seed=2741)
    g, st = gpu_run(d, precision=prec, exec_mode=mode, stages=DGF, use_graph=True)
    h, sh = gpu_run(d, precision=prec, exec_mode=mode)
    log("graph: sweeps=%d captures=%d fallbacks=%d; host: sweeps=%d" % (
        st["sweeps"], st["graph_captures"], st["graph_fallbacks"], sh["sweeps"]))
    assert st["graph_captures"] == 1
    assert st["sweeps"] == sh["sweeps"]
    assert np.array_equal(g["H"], h["H"]) and np.array_equal(g["rho"], h["rho"])
    assert np.array_equal(g["nngb"], h["nngb"])
    assert st["n_force"] == sh["n_force"] and st["n_dens"] == sh["n_dens"]
    # force: j-side sums are flushed with atomics, so only the order differs
    e = errors(g, dict(h, sa=np.abs(h["ax"]) + np.abs(h["ay"]) + np.abs(h["az"]) + 1e-300,
                       su=np.abs(h["dudt"]) + 1e-300))
    assert e["a"] < 1e-9 and e["du"] < 1e-9, e
    o = oracle_run(d)
    assert_close(g, o, TOL_FP64 if prec == "fp64" else TOL_FP32, counts_exact=prec == "fp64",
                 stats=st if prec == "fp64" else None)


def test_graph_host_takes_over():
    """Initial H a third of the converged value: more sweeps than the graph
    holds and smoothing lengths that outgrow the neighbour lists."""
    log("case graph fallback lattice 16^3 fp64")
    d = gen.lattice(16, vsigma=0.1, seed=11)
    d = dict(d)
    d["H"] = d["H"] / 3.0
    g, st = gpu_run(d, precision="fp64", stages=DGF, use_graph=True)
    log("graph: sweeps=%d relists=%d rebuilds=%d fallbacks=%d" % (st["sweeps"], st["relists"], st["rebuilds"],
                                                                 st["graph_fallbacks"]))
    assert st["graph_fallbacks"] == 1
    o = oracle_run(d)
    assert_close(g, o, TOL_FP64, stats=st)


def test_graph_steps_reuse():
    """Three KDK steps on the small shock tube with and without the graph:
    same trajectory, and the graph is captured far fewer times than run."""
    import torch
    from paper_1606_02738_amd import sph as S
    log("case graph steps sod small fp64")
    d = gen.sod(16)
    dt = 2.0 ** -11
    res = {}
    for use_graph in (False, True):
        sim = S.SPH(d["box"], precision="fp64", use_graph=use_graph)
        t = S.to_device(d)
        sim.bind(t)
        sim.run()
        caps = []
        for k in range(4):
            sim.step(dt)
            caps.append(sim.stats()["graph_captures"])
        torch.cuda.synchronize()
        res[use_graph] = (S.to_host(t), sim.stats(), caps)
        sim.close()
    a, b = res[False][0], res[True][0]
    caps = res[True][2]
    log("graph captures after each step: %s; fallbacks %d" % (caps, res[True][1]["graph_fallbacks"]))
    assert caps[-1] <= 2, caps
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "H", "rho"):
        scale = np.max(np.abs(a[k])) + 1e-300
        assert np.max(np.abs(a[k] - b[k])) / scale < 1e-9, k
    ca, cb = res[False][1]["conserved"], res[True][1]["conserved"]
    assert np.allclose(ca, cb, rtol=1e-9, atol=1e-12)


def test_autotune_picks_a_timed_candidate_and_restores_state():
    import torch
    from paper_1606_02738_amd import autotune as AT
    from paper_1606_02738_amd import sph as S
    log("case autotune clustered 24^3")
    d = gen.clustered(24, n_halos=8, seed=2741)
    t = S.to_device(d)
    sim = S.SPH(d["box"], precision="fp32c")
    sim.bind(t)
    sim.run()
    sim.close()
    before = {k: v.clone() for k, v in t.items()}
    cands = [dict(n_split=64, exec_mode="grid", persistent_wgs=0, prune="box", use_graph=False, rebuild_steps=0),
             dict(n_split=32, exec_mode="persistent", persistent_wgs=512, prune="box", use_graph=True,
                  rebuild_steps=4)]
    # the first stage only (the kernel-axis stage is covered in test_gpu_kernel_variants)
    best, table = AT.autotune(d["box"], t, "fp32c", 1e-5, steps=2, cands=cands, cache=None, kernel_axes=False)
    torch.cuda.synchronize()
    log("table: %s" % [(c["n_split"], c["exec_mode"], round(ms, 3)) for c, ms in table])
    assert best in cands and len(table) == 2 and all(ms > 0 for _, ms in table)
    for k in t:
        assert torch.equal(t[k], before[k]), k
