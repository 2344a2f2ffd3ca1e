"""The caller-owned workspace (C-ABI: sph_workspace_size, sph_create with a
workspace): the library carves every device buffer from the torch tensor the
caller passes, reports its use, and fails a call cleanly (SPH_ERR_WORKSPACE,
with the bytes it needed) when the workspace is too small."""
import numpy as np
import pytest
import torch  # noqa: F401

import gen
from gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_estimate_suffices_and_use_is_reported():
    from paper_1606_02738_amd import sph as S
    log("case workspace: estimate for a clustered 32^3 box, both list kinds")
    d = gen.clustered(32, n_halos=20, seed=2741)
    for lists in ("cell", "particle"):
        sim = S.SPH(d["box"], precision="fp32c", force="gather", lists=lists, rebuild_steps=8)
        t = S.to_device(d)
        sim.bind(t)
        sim.run()
        for _ in range(3):
            sim.step(1e-5)
        st = sim.stats()
        log("%s: workspace %d bytes, high %d, in use %d" % (lists, st["workspace_bytes"], st["workspace_high"],
                                                            st["workspace_in_use"]))
        assert sim.ws.numel() == sim.workspace_size(d["x"].size)
        assert 0 < st["workspace_high"] <= st["workspace_bytes"] <= sim.ws.numel()
        assert st["workspace_needed"] == 0
        sim.close()


def test_too_small_workspace_fails_cleanly_and_reports_need():
    from paper_1606_02738_amd import sph as S
    log("case workspace: too small")
    d = gen.lattice(32, vsigma=0.1, seed=3)
    small = S.WORKSPACE_MIN
    sim = S.SPH(d["box"], precision="fp32c", workspace_bytes=small)
    t = S.to_device(d)
    sim.bind(t)
    with pytest.raises(S.SPHError) as e:
        sim.build_cells()
    assert e.value.status == -6
    st = sim.stats()
    log("needed %d of %d" % (st["workspace_needed"], st["workspace_bytes"]))
    assert st["workspace_needed"] > st["workspace_bytes"]
    sim.close()
    # a workspace of the reported size carries the same calls
    sim = S.SPH(d["box"], precision="fp32c", workspace_bytes=2 * st["workspace_needed"] + S.WORKSPACE_MIN)
    t = S.to_device(d)
    sim.bind(t)
    sim.run()
    torch.cuda.synchronize()
    g = S.to_host(t)
    assert np.all(np.isfinite(g["rho"])) and np.all(g["rho"] > 0)
    sim.close()
