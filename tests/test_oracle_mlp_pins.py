"""Pins of the FP64 predictor oracle (oracle/mlp.py) against facts fixed by
mathematics and by independent library routines: bfloat16 rounding against
torch's conversion, backpropagation against finite differences, closed forms
of the network on sparse weights, Adam on its degenerate settings, feature
counts against brute force, and the compression feature against the change
of the converged H along the flow."""
import math

import numpy as np

import gen
from oracle import mlp as M


def test_bf16_rounding_matches_torch_and_ties_to_even():
    import torch
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, size=4000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-38]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(v), ref)
    # halfway cases: 1 + 2^-8 lies between 1 (even) and 1 + 2^-7 (odd)
    assert M.bf16(np.float32(1.0 + 2.0 ** -8))[()] == 1.0
    assert M.bf16(np.float32(1.0 + 3 * 2.0 ** -8))[()] == 1.0 + 2.0 ** -6
    assert M.bf16(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20))[()] == 1.0 + 2.0 ** -7
    assert M.bf16(np.float32(-(1.0 + 3 * 2.0 ** -8)))[()] == -(1.0 + 2.0 ** -6)


def test_silu_identities():
    z = np.linspace(-8, 8, 101)
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert np.allclose(M.silu(z) - M.silu(-z), z, atol=1e-14)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(M.dsilu(z), fd, atol=1e-8)
    assert abs(M.dsilu(np.array([0.0]))[0] - 0.5) < 1e-15


def _random_params(seed=3):
    rng = np.random.default_rng(seed)
    p = M.init_params(seed, xmu=rng.normal(size=M.NIN) * 0.1, xsd=1.0 + rng.uniform(size=M.NIN),
                      ymu=0.01, ysd=0.02)
    o, s = M.OFF["b1"][0], M.NH
    for k in ("b1", "b2", "b3", "b4"):
        o, s = M.OFF[k]
        p[o:o + s] = rng.normal(size=s) * 0.3
    return p


def test_backprop_matches_finite_differences():
    """dL/dp of the oracle against central differences of L (unrounded
    weights, where L is smooth in p)."""
    rng = np.random.default_rng(11)
    p = _random_params()
    X = rng.normal(size=(37, M.NIN))
    y = 0.01 + 0.02 * rng.normal(size=37)
    L, g = M.loss_grad(p, X, y, rounded=False)
    idx = np.concatenate([rng.choice(M.NT, 300, replace=False), [M.OFF["b4"][0]],
                          M.OFF["W1"][0] + np.arange(0, 1024, 97)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss_grad(pp, X, y, rounded=False)[0] - M.loss_grad(pm, X, y, rounded=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (abs(fd) + 1e-3), (i, fd, g[i])


def test_forward_sparse_path_closed_form():
    """Only the path input 2 -> hidden 5 -> hidden 9 -> hidden 33 -> output
    is non-zero: o = d silu(c silu(b silu(a x2))) + b4 (silu(0) = 0 keeps
    the other units silent).  A transposed or shifted operand breaks the
    path."""
    p = np.zeros(M.NP)
    a, b, c, d, b4 = 0.75, -1.25, 2.0, 0.5, 0.125   # bfloat16-exact
    p[M.OFF["W1"][0] + 2 * M.NH + 5] = a
    p[M.OFF["W2"][0] + 5 * M.NH + 9] = b
    p[M.OFF["W3"][0] + 9 * M.NH + 33] = c
    p[M.OFF["w4"][0] + 33] = d
    p[M.OFF["b4"][0]] = b4
    p[M.OFF["xsd"][0]:M.OFF["xsd"][0] + M.NIN] = 1.0
    p[M.OFF["ymu"][0]] = 0.25
    p[M.OFF["ysd"][0]] = 2.0
    X = np.zeros((5, M.NIN))
    X[:, 2] = [-3.0, -0.5, 0.0, 0.7, 4.0]
    o, yv = M.forward(p, X)

    def s(t):
        return t / (1.0 + math.exp(-t))
    for k in range(5):
        ref = d * s(c * s(b * s(a * X[k, 2]))) + b4
        assert abs(o[k] - ref) < 1e-15
        assert abs(yv[k] - (0.25 + 2.0 * ref)) < 1e-14


def test_forward_uses_rounded_weights():
    """A weight of 1 + 2^-8 enters the network as 1.0 (bfloat16, ties to
    even); biases are not rounded."""
    def net(a, b1):
        p = np.zeros(M.NP)
        p[M.OFF["xsd"][0]:M.OFF["xsd"][0] + M.NIN] = 1.0
        p[M.OFF["ysd"][0]] = 1.0
        p[M.OFF["W1"][0] + 3 * M.NH + 7] = a
        p[M.OFF["b1"][0] + 7] = b1
        p[M.OFF["W2"][0] + 7 * M.NH + 1] = 1.0
        p[M.OFF["W3"][0] + 1 * M.NH + 60] = 1.0
        p[M.OFF["w4"][0] + 60] = 1.0
        return p
    X = np.zeros((1, M.NIN))
    X[0, 3] = 10.0

    def s(t):
        return t / (1.0 + math.exp(-t))
    b1 = 1.0 + 2.0 ** -12        # not bfloat16-exact, used as is
    o, _ = M.forward(net(1.0 + 2.0 ** -8, b1), X)
    assert abs(o[0] - s(s(s(10.0 + b1)))) < 1e-15
    o_exact, _ = M.forward(net(1.0 + 2.0 ** -8, b1), X, rounded=False)
    assert abs(o_exact[0] - s(s(s(10.0 * (1.0 + 2.0 ** -8) + b1)))) < 1e-15


def test_adam_degenerate_settings():
    rng = np.random.default_rng(2)
    p = _random_params()
    g = rng.normal(size=M.NT)
    # beta1 = beta2 = 0: the update is -lr g / (|g| + eps) exactly
    q, m, v = M.adam(p, np.zeros(M.NT), np.zeros(M.NT), g, 1, 1e-3, b1=0.0, b2=0.0, eps=1e-8)
    assert np.allclose(q[:M.NT] - p[:M.NT], -1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # first step with the usual betas: bias correction gives -lr sign(g)
    q, m, v = M.adam(p, np.zeros(M.NT), np.zeros(M.NT), g, 1, 1e-3)
    big = np.abs(g) > 1e-3
    assert np.allclose((q[:M.NT] - p[:M.NT])[big], -1e-3 * np.sign(g[big]), rtol=1e-4)
    assert np.array_equal(q[M.NT:], p[M.NT:])   # standardisation constants untouched


def test_feature_counts_brute_force():
    rng = np.random.default_rng(8)
    n = 300
    box = np.array([1.0, 0.7, 1.3])
    x, y, z = (rng.uniform(0, b, n) for b in box)
    H = rng.uniform(0.05, 0.1, n)
    zeros = np.zeros(n)
    F, counts = M.features(x, y, z, zeros, zeros, zeros, H, zeros + 1, zeros + 1, zeros, box, 0.0)
    G = M.feature_grid(box, n)
    assert counts.shape == tuple(G) and counts.sum() == n
    cell = [tuple(int(math.floor(c * g / b)) for c, g, b in zip(p, G, box)) for p in zip(x, y, z)]
    for i in range(0, n, 7):
        own = sum(1 for j in range(n) if cell[j] == cell[i])
        s27 = 0
        for j in range(n):
            dd = [(cell[j][a] - cell[i][a]) % G[a] for a in range(3)]
            # count each of the 27 offsets that maps onto j's cell (a small
            # grid wraps several offsets onto one cell)
            mult = 1
            for a in range(3):
                mult *= sum(1 for o in (-1, 0, 1) if o % G[a] == dd[a])
            s27 += mult
        assert math.isclose(F[i, 1], math.log(own), rel_tol=0, abs_tol=1e-14)
        nbar = n / np.prod(G)
        assert math.isclose(F[i, 2], math.log(s27 / (27 * nbar)), rel_tol=0, abs_tol=1e-13)
    assert np.all(F[:, 5] == 0) and np.all(F[:, 6] == 0)
    assert np.all(F[:, 7:] == 0)


def test_features_uniform_lattice():
    """Aligned exact lattice: every cell holds the same count, so the
    gradient estimate vanishes and the neighbourhood overdensity is zero."""
    d = gen.lattice(16, jitter=0.0)
    n = d["x"].size
    F, counts = M.features(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["H"], np.ones(n), np.ones(n),
                           np.zeros(n), d["box"], 0.0)
    assert counts.min() == counts.max()
    assert np.allclose(F[:, 2], 0.0, atol=1e-14)
    assert np.allclose(F[:, 3], 0.0, atol=1e-14) and np.allclose(F[:, 4], 0.0, atol=1e-14)
    assert np.allclose(F[:, 0], np.log(d["H"] / (1.0 / 16)), atol=1e-14)


def test_feature_gradient_points_up_the_density():
    """Two slabs, the left one 8x denser: at the interface cells the x
    component of g points to the dense side."""
    rng = np.random.default_rng(4)
    xl = rng.uniform(0.0, 0.5, 8000)
    xr = rng.uniform(0.5, 1.0, 1000)
    x = np.concatenate([xl, xr])
    n = x.size
    y, z = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    zeros = np.zeros(n)
    F, counts = M.features(x, y, z, zeros, zeros, zeros, zeros + 0.05, zeros + 1, zeros + 1, zeros,
                           np.ones(3), 0.0)
    G = M.feature_grid(np.ones(3), n)
    c = np.floor(x * G[0]).astype(int)
    # just right of the interface the dense side is at -x: S+ < S-
    sel = c == G[0] // 2
    assert np.all(F[sel, 3] > 0.1)
    fx = x * G[0] - c
    # F4 ~ g_x (f_x - 1/2) with g_x < 0: negative on the cell's right half
    assert np.mean(F[sel & (fx > 0.6), 4]) < -0.02
    assert np.mean(F[sel & (fx < 0.4), 4]) > 0.02


def test_compression_feature_predicts_h_change(oracle_mod):
    """Feature 5 is the first-order change of log H over a step: compare with
    the converged H re-solved at the drifted positions (smooth periodic
    velocity field, small dt)."""
    o = oracle_mod
    d = gen.lattice(12, vsigma=0.0, seed=3)
    L = d["box"][0]
    k = 2 * math.pi / L
    d["vx"] = 0.3 * np.sin(k * d["x"])
    d["vy"] = 0.2 * np.cos(k * d["y"])
    d["vz"] = 0.1 * np.sin(k * d["z"] + 0.4)
    base = o.full(d, tree=True, h_tol=1e-13, max_iter=100)
    dt = 2e-4
    e = dict(d)
    for c, v in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        e[c] = np.mod(d[c] + dt * d[v], L)
    s = o.solve_h(e["x"], e["y"], e["z"], e["m"], base["H"], e["box"], tree=True, h_tol=1e-13, max_iter=100)
    dlogH = np.log(s["H"] / base["H"])
    F, _ = M.features(e["x"], e["y"], e["z"], d["vx"], d["vy"], d["vz"], base["H"], base["rho"], base["P"],
                      base["dudt"], d["box"], dt)
    scale = np.max(np.abs(dlogH))
    assert scale > 1e-5
    assert np.max(np.abs(F[:, 5] - dlogH)) < 0.02 * scale
    assert np.allclose(F[:, 6], dt * np.sqrt(d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2) / base["H"])
