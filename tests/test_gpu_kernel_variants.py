"""The autotuner's tile and wave axes (form (2) of the batched method: the
occupancy target of the packed density and gather force kernels and the
neighbour-cell entries they stage per batch).  Every instantiation gives the
converged state of the default kernels bit for bit, so each one inherits
the default's oracle parity; the autotuner's own choice on a small clustered
box is then compared with the FP64 oracle directly."""
import math

import numpy as np
import pytest
import torch  # noqa: F401

import gen
from gpu_helpers import TOL_FP32, assert_close, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

VARIANTS = ([dict(waves_density=w) for w in (4, 5, 6, 8)] + [dict(waves_force=w) for w in (4, 5, 6, 8)] +
            [dict(batch=b) for b in (16, 32)] + [dict(waves_density=8, waves_force=4, batch=16)])
KEYS = ("rho", "H", "omega", "P", "ax", "ay", "az", "dudt", "nngb")


@pytest.fixture(scope="module")
def clustered():
    return gen.clustered(32, n_halos=20, seed=2761)


@pytest.fixture(scope="module")
def reference(clustered):
    out = {}
    for prec in ("fp32c", "fp32"):
        out[prec] = gpu_run(clustered, precision=prec, exec_mode="persistent", force="gather")[0]
    return out


@pytest.mark.parametrize("prec", ["fp32c", "fp32"])
@pytest.mark.parametrize("var", VARIANTS, ids=lambda v: "-".join("%s%d" % kv for kv in v.items()))
def test_variant_bit_identical_to_default(clustered, reference, prec, var):
    log("case kernel variant %s %s" % (prec, var))
    g, st = gpu_run(clustered, precision=prec, exec_mode="persistent", force="gather", **var)
    ref = reference[prec]
    for k in KEYS:
        assert np.array_equal(g[k], ref[k]), k


def test_autotuned_choice_vs_oracle(clustered):
    """The autotuner on the 32^3 clustered box (a reduced first stage, the
    full kernel-axis stage), then the density, ghost and force of its choice
    against the oracle."""
    from paper_1606_02738_amd import autotune as AT
    from paper_1606_02738_amd import sph as S
    log("case autotuned choice vs oracle, clustered 32^3 fp32c")
    d = clustered
    t = S.to_device(d)
    sim = S.SPH(d["box"], precision="fp32c")
    sim.bind(t)
    sim.run()
    sim.close()
    torch.cuda.synchronize()
    cs = math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * float(t["u"].max()))
    dt = 0.25 * float(t["H"].min()) / math.sqrt(10.0 / 3.0) / cs
    base = dict(n_split=64, exec_mode="persistent", persistent_wgs=256, prune="box", use_graph=False,
                rebuild_steps=8, force="gather")
    best, table = AT.autotune(d["box"], t, "fp32c", dt, steps=4, warmup=1, cache=None,
                              cands=[base, dict(base, exec_mode="grid", persistent_wgs=0)], log=log)
    log("choice %s" % best)
    assert len(table) == 2 + len(AT.kernel_candidates(base)) + 1
    assert all(k in best for k in ("waves_density", "waves_force", "batch"))
    kern = {k: best[k] for k in ("waves_density", "waves_force", "batch")}
    g, st = gpu_run(d, precision="fp32c", exec_mode=best["exec_mode"], n_split=best["n_split"],
                    force=best["force"], prune=best["prune"], **kern)
    o = oracle_run(d)
    assert_close(g, o, TOL_FP32, counts_exact=False)
