"""The loss-gradient entry point that allocates nothing
(sph_mlp_loss_grad_noalloc, partials in the library's own device array)
against sph_mlp_loss_grad with a caller workspace: two calls in a row on the
same GPU, the second on fewer rows, each compared with the workspace form on
the same inputs.  Both run the same kernels with the same launch shape and
no atomics, so the gradient and the loss agree bit for bit."""
import numpy as np
import pytest
import torch  # noqa: F401

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _params(seed):
    rng = np.random.default_rng(seed)
    from paper_1606_02738_amd import sph as S
    p = np.zeros(S.MLP_NP, dtype=np.float32)
    p[:S.MLP_NT] = rng.normal(size=S.MLP_NT) * 0.15
    # input and output standardisation: xmu[16] xsd[16] ymu ysd
    p[S.MLP_NT:S.MLP_NT + 16] = rng.normal(size=16) * 0.3
    p[S.MLP_NT + 16:S.MLP_NT + 32] = 0.5 + rng.uniform(size=16)
    p[S.MLP_NT + 32] = 0.002
    p[S.MLP_NT + 33] = 0.01
    return p


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 8), dtype=np.float32)
    X[:, :7] = rng.normal(size=(n, 7)) * np.array([1.0, 1.5, 0.5, 0.3, 0.2, 0.01, 0.05])
    y = (0.002 + 0.01 * rng.normal(size=n)).astype(np.float32)
    return X, y


def test_noalloc_matches_workspace_form_twice():
    import torch
    from paper_1606_02738_amd import sph as S
    p = torch.from_numpy(_params(11)).cuda()
    grad = torch.empty(S.MLP_NT, dtype=torch.float32, device="cuda")
    for n, seed in ((20011, 3), (777, 4)):
        log("case no-alloc loss/grad n=%d seed=%d" % (n, seed))
        X, y = _rows(n, seed)
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        grad.fill_(float("nan"))
        L0, g0 = S.mlp_loss_grad_noalloc(p, Xd, yd, grad=grad)
        L1, g1 = S.mlp_loss_grad(p, Xd, yd)
        torch.cuda.synchronize()
        a, b = g0.cpu().numpy(), g1.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
        assert L0 == L1 and np.isfinite(L0) and L0 > 0


def test_noalloc_rejects_bad_sizes():
    import ctypes as C
    import torch
    from paper_1606_02738_amd import sph as S
    p = torch.from_numpy(_params(1)).cuda()
    X = torch.zeros(4, 8, dtype=torch.float32, device="cuda")
    y = torch.zeros(4, dtype=torch.float32, device="cuda")
    g = torch.empty(S.MLP_NT, dtype=torch.float32, device="cuda")
    L = C.c_double()
    f = S.lib().sph_mlp_loss_grad_noalloc
    for n in (0, -1, (1 << 31)):
        assert f(p.data_ptr(), X.data_ptr(), y.data_ptr(), n, g.data_ptr(), C.byref(L), None) == -1
