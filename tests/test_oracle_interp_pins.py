"""Pins of the interpolation oracle (oracle/interp.py): on an exact cubic
lattice with the converged uniform H, the interpolant of Q = 1 is 1 at every
particle (it is the density sum divided by the density), a field cos(2 pi x/L)
comes back scaled by one factor common to all particles (the lattice is the
same around every particle), and the result is the kernel sum written out
particle by particle."""
import math

import numpy as np

import gen
from oracle import interp as IP


def _exact_lattice(oracle_mod):
    d = gen.lattice(8, jitter=0.0)
    o = oracle_mod.full(d, tree=False, h_tol=1e-14, max_iter=200)
    return d, o


def test_unit_field_is_one_at_particles(oracle_mod):
    d, o = _exact_lattice(oracle_mod)
    q = IP.interpolate(d["x"], d["y"], d["z"], d["x"], d["y"], d["z"], d["m"], o["rho"], o["H"],
                       np.ones_like(d["x"]), d["box"])
    assert np.max(np.abs(q - 1.0)) < 1e-12


def test_cosine_field_scaled_uniformly(oracle_mod):
    d, o = _exact_lattice(oracle_mod)
    L = d["box"][0]
    Qf = np.cos(2 * math.pi * d["x"] / L)
    q = IP.interpolate(d["x"], d["y"], d["z"], d["x"], d["y"], d["z"], d["m"], o["rho"], o["H"], Qf, d["box"])
    # the sum is a symmetric average of cos over the neighbour shells: it
    # equals cos(x_i) times a factor that is the same for every particle
    ratio = q / Qf
    sel = np.abs(Qf) > 0.5
    assert np.ptp(ratio[sel]) < 1e-12
    assert 0.5 < ratio[sel][0] < 1.0


def test_matches_explicit_sum(oracle_mod):
    rng = np.random.default_rng(3)
    n = 200
    x, y, z = rng.uniform(0, 1, (3, n))
    m = rng.uniform(0.5, 1.5, n) / n
    rho = rng.uniform(0.5, 2.0, n)
    H = rng.uniform(0.1, 0.3, n)
    Q = rng.normal(size=n)
    p = rng.uniform(0, 1, (3, 7))
    q = IP.interpolate(p[0], p[1], p[2], x, y, z, m, rho, H, Q, np.ones(3))
    for k in range(7):
        s = 0.0
        for i in range(n):
            dd = [(p[a][k] - c[i]) - round(p[a][k] - c[i]) for a, c in enumerate((x, y, z))]
            r = math.sqrt(sum(v * v for v in dd))
            s += m[i] * Q[i] / rho[i] * oracle_mod.W(r, H[i])
        assert abs(q[k] - s) <= 1e-12 * (abs(s) + 1.0)
