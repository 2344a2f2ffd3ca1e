"""FP64 oracle of the learned smoothing-length predictor.

TEST INFRASTRUCTURE: imported only by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  Nothing here imports the GPU package and the
GPU library never calls anything here.

The predictor replaces the warm start of the smoothing-length iteration of
the density loop (paper, section 2, the constraint between density and
smoothing length solved per particle by Newton-Raphson): after the drift of
a step it guesses the converged H of every particle; the plain iteration then
runs from that guess and alone decides convergence.

Contents, all plain numpy in float64:

* :func:`bf16` -- round-to-nearest-even of float32 values to bfloat16 (the
  storage type of the network's weights), from the bit-level definition.
* :func:`features` -- the per-particle inputs (previous H, the particle's
  grid-cell count, the 27-cell neighbourhood count, a density-gradient
  estimate from the neighbourhood counts, the compression rate implied by the
  previous step's energy equation, the displacement of the step).
* :func:`forward`, :func:`loss_grad` -- the network (16 inputs, three hidden
  layers of 64 SiLU units, one output) and its backpropagated gradient.
* :func:`adam` -- one Adam update.

Parameter vector layout (float32 on the device; the same offsets here):
W1[16][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4,
then the non-trained standardisation constants xmu[16], xsd[16], ymu, ysd.
Weight matrices and w4 enter the network rounded to bfloat16; biases are used
as they are.
"""
from __future__ import annotations

import math

import numpy as np

NF = 7        # features in use
NIN = 16      # network inputs (features padded with zeros)
NH = 64       # hidden width
OFF = {}
_o = 0
for _name, _size in (("W1", NIN * NH), ("b1", NH), ("W2", NH * NH), ("b2", NH), ("W3", NH * NH), ("b3", NH),
                     ("w4", NH), ("b4", 1)):
    OFF[_name] = (_o, _size)
    _o += _size
NT = _o       # trained parameters
for _name, _size in (("xmu", NIN), ("xsd", NIN), ("ymu", 1), ("ysd", 1)):
    OFF[_name] = (_o, _size)
    _o += _size
NP = _o       # whole vector
ROUNDED = ("W1", "W2", "W3", "w4")


def bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float64.  bfloat16 keeps the top 16 bits of the float32 pattern; the
    dropped 16 bits decide the rounding."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p, rounded=True):
    """Dictionary of named float64 arrays from a parameter vector; weights
    rounded to bfloat16 unless rounded=False."""
    p = np.asarray(p)
    out = {}
    for k, (o, s) in OFF.items():
        v = p[o:o + s]
        if rounded and k in ROUNDED:
            v = bf16(v.astype(np.float32))
        else:
            v = v.astype(np.float64)
        out[k] = v
    out["W1"] = out["W1"].reshape(NIN, NH)
    out["W2"] = out["W2"].reshape(NH, NH)
    out["W3"] = out["W3"].reshape(NH, NH)
    out["b4"] = float(out["b4"][0])
    out["ymu"] = float(out["ymu"][0])
    out["ysd"] = float(out["ysd"][0])
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _layers(w, X):
    xh = (np.asarray(X, dtype=np.float64) - w["xmu"]) / w["xsd"]
    z1 = xh @ w["W1"] + w["b1"]
    h1 = silu(z1)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = silu(z2)
    z3 = h2 @ w["W3"] + w["b3"]
    h3 = silu(z3)
    o = h3 @ w["w4"] + w["b4"]
    return xh, z1, h1, z2, h2, z3, h3, o


def forward(p, X, rounded=True):
    """Network output o (standardised) and the predicted log(H_new/H_prev)
    y = ymu + ysd * o for the rows of X (n x 16)."""
    w = unpack(p, rounded)
    o = _layers(w, X)[-1]
    return o, w["ymu"] + w["ysd"] * o


def loss_grad(p, X, y, rounded=True):
    """Mean loss L = (1/2n) sum (o - t)^2 with t = (y - ymu)/ysd, and dL/dp
    for the NT trained parameters (the gradient with respect to the rounded
    weights, applied to the stored ones)."""
    w = unpack(p, rounded)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    xh, z1, h1, z2, h2, z3, h3, o = _layers(w, X)
    t = (np.asarray(y, dtype=np.float64) - w["ymu"]) / w["ysd"]
    r = o - t
    L = 0.5 * float(np.sum(r * r)) / n
    do = r / n
    g = np.zeros(NT)

    def put(name, v):
        o_, s_ = OFF[name]
        g[o_:o_ + s_] = np.ravel(v)

    put("w4", h3.T @ do)
    put("b4", np.array([do.sum()]))
    dz3 = np.outer(do, w["w4"]) * dsilu(z3)
    put("W3", h2.T @ dz3)
    put("b3", dz3.sum(0))
    dz2 = (dz3 @ w["W3"].T) * dsilu(z2)
    put("W2", h1.T @ dz2)
    put("b2", dz2.sum(0))
    dz1 = (dz2 @ w["W2"].T) * dsilu(z1)
    put("W1", xh.T @ dz1)
    put("b1", dz1.sum(0))
    return L, g


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the NT trained parameters (step number t >= 1);
    returns new (p, m, v)."""
    p = np.array(p, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p[:NT] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def init_params(seed=1, xmu=None, xsd=None, ymu=0.0, ysd=1.0):
    """Scaled uniform initial weights (variance 1/fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NP)

    def put(name, v):
        o_, s_ = OFF[name]
        p[o_:o_ + s_] = np.ravel(v)

    for name, fan_in, shape in (("W1", NIN, (NIN, NH)), ("W2", NH, (NH, NH)), ("W3", NH, (NH, NH)),
                                ("w4", NH, (NH,))):
        a = math.sqrt(3.0 / fan_in)
        put(name, rng.uniform(-a, a, size=shape))
    put("xmu", np.zeros(NIN) if xmu is None else xmu)
    put("xsd", np.ones(NIN) if xsd is None else xsd)
    put("ymu", np.array([ymu]))
    put("ysd", np.array([ysd]))
    return p.astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------

def feature_grid(L, n):
    """Cells per axis of the feature grid of a box with edges L holding n
    particles: cell edge close to twice the mean interparticle spacing
    (about 8 particles per cell on average), rounded to the nearest count,
    between 1 and 256 cells per axis."""
    L = np.asarray(L, dtype=np.float64)
    s = 2.0 * math.pow(float(L[0] * L[1] * L[2]) / max(n, 1), 1.0 / 3.0)
    return np.array([int(min(256, max(1, math.floor(La / s + 0.5)))) for La in L])


def features(x, y, z, vx, vy, vz, H, rho, P, dudt, box, dt):
    """Feature matrix (n x 16, float64; columns 7..15 zero) of one periodic
    box.  Positions are after the drift; H, rho, P and du/dt are those of the
    previous evaluation; dt is the step.

    0  log(H / s), s = (V/n)^(1/3) the mean spacing of the box
    1  log(count of the particle's feature-grid cell)
    2  log(27-cell neighbourhood count / (27 * mean cell count))
    3  |g|, g_a = (S+_a - S-_a) / S27 with S+-_a the counts of the 9 cells at
       offset +-1 along axis a and S27 the neighbourhood count
    4  sum_a g_a (f_a - 1/2), f_a the particle's fractional position in its cell
    5  -dt rho du/dt / (3 P): first-order change of log H over the step, from
       the continuity equation with the velocity divergence the energy
       equation implies (0 where P <= 0)
    6  dt |v| / H
    """
    box = np.asarray(box, dtype=np.float64)
    pos = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64), np.asarray(z, np.float64)], 1)
    n = pos.shape[0]
    G = feature_grid(box, n)
    scale = G / box
    u = pos * scale
    idx = np.minimum(np.floor(u).astype(np.int64), G - 1)
    idx = np.maximum(idx, 0)
    frac = u - idx
    counts = np.zeros(tuple(G), dtype=np.int64)
    np.add.at(counts, (idx[:, 0], idx[:, 1], idx[:, 2]), 1)
    s27 = np.zeros(n, dtype=np.int64)
    sp = np.zeros((n, 3), dtype=np.int64)
    sm = np.zeros((n, 3), dtype=np.int64)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                c = counts[(idx[:, 0] + dx) % G[0], (idx[:, 1] + dy) % G[1], (idx[:, 2] + dz) % G[2]]
                s27 += c
                for a, d in enumerate((dx, dy, dz)):
                    if d == 1:
                        sp[:, a] += c
                    elif d == -1:
                        sm[:, a] += c
    own = counts[idx[:, 0], idx[:, 1], idx[:, 2]]
    nbar = n / float(np.prod(G))
    sbox = (float(np.prod(box)) / n) ** (1.0 / 3.0)
    g = (sp - sm) / s27[:, None].astype(np.float64)
    F = np.zeros((n, NIN))
    H = np.asarray(H, np.float64)
    F[:, 0] = np.log(H / sbox)
    F[:, 1] = np.log(own.astype(np.float64))
    F[:, 2] = np.log(s27 / (27.0 * nbar))
    F[:, 3] = np.sqrt(np.sum(g * g, 1))
    F[:, 4] = np.sum(g * (frac - 0.5), 1)
    P = np.asarray(P, np.float64)
    comp = np.zeros(n)
    ok = P > 0
    comp[ok] = -dt * np.asarray(rho, np.float64)[ok] * np.asarray(dudt, np.float64)[ok] / (3.0 * P[ok])
    F[:, 5] = comp
    v = np.sqrt(np.asarray(vx, np.float64) ** 2 + np.asarray(vy, np.float64) ** 2 + np.asarray(vz, np.float64) ** 2)
    F[:, 6] = dt * v / H
    return F, counts
