"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of the expected values comes from the
GPU library; the ones that are not invariants come from independent
computations written here (textbook M4 spline form, lattice-shell counts,
scipy quadrature and root finding, finite differences of an energy).
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import gen

GK = math.sqrt(10.0 / 3.0)
ETA = 1.2348


# --- textbook M4 cubic spline (support 2h, sigma = 1/pi), independent form ---
def w_m4(r, h):
    s = r / h
    if s < 1.0:
        v = 1.0 - 1.5 * s * s + 0.75 * s ** 3
    elif s < 2.0:
        v = 0.25 * (2.0 - s) ** 3
    else:
        v = 0.0
    return v / (math.pi * h ** 3)


# number of integer vectors n with |n|^2 = k (sums of three squares)
R3 = {0: 1, 1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24, 7: 0, 8: 12, 9: 30, 10: 24}


def lattice_rho(H):
    """Unit cubic lattice (spacing 1, mass 1): sum over shells |n| < H."""
    return sum(c * w_m4(math.sqrt(k), H / 2.0) for k, c in R3.items() if math.sqrt(k) < H)


# ---------------------------------------------------------------- P1 / P2
def test_kernel_normalisation_and_shape(oracle_mod):
    """Sec. 2 kernel: unit integral over its support for any H, W(0) =
    8/(pi H^3), C^1 continuity at q = 1/2 and compact support."""
    o = oracle_mod
    for H in (0.01, 0.37, 1.0, 5.0):
        val, err = integrate.quad(lambda r: 4 * math.pi * r * r * o.W(r, H), 0.0, H,
                                  points=[0.5 * H], epsabs=1e-14, epsrel=1e-13)
        assert abs(val - 1.0) < 1e-12
        assert o.W(0.0, H) == pytest.approx(8.0 / (math.pi * H ** 3), rel=1e-15)
        assert o.W(H, H) == 0.0 and o.W(1.5 * H, H) == 0.0 and o.dWdr(H, H) == 0.0
        e = 1e-9 * H
        assert o.W(0.5 * H - e, H) == pytest.approx(o.W(0.5 * H + e, H), rel=1e-7)
        assert o.dWdr(0.5 * H - e, H) == pytest.approx(o.dWdr(0.5 * H + e, H), rel=1e-7)


def test_kernel_matches_textbook_m4():
    """The oracle's W(r, H) equals the classic M4 spline written with h = H/2."""
    import oracle as o
    rng = np.random.default_rng(1)
    for H in (0.03, 1.0, 2.7):
        for r in rng.uniform(0, 1.2 * H, 50):
            assert o.W(r, H) == pytest.approx(w_m4(r, H / 2.0), rel=1e-13, abs=1e-300)


def test_kernel_derivatives_fd(oracle_mod):
    """dW/dr and dW/dH agree with central differences of W."""
    o = oracle_mod
    for H in (0.2, 1.0):
        for q in (0.05, 0.3, 0.49, 0.51, 0.7, 0.95):
            r = q * H
            e = 1e-6 * H
            fd_r = (o.W(r + e, H) - o.W(r - e, H)) / (2 * e)
            fd_h = (o.W(r, H + e) - o.W(r, H - e)) / (2 * e)
            scale = 8 / (math.pi * H ** 4)
            assert abs(o.dWdr(r, H) - fd_r) < 1e-7 * scale
            assert abs(o.dWdH(r, H) - fd_h) < 1e-7 * scale


def test_kernel_second_moment_gives_kernel_gamma(oracle_mod):
    """H / (2 sigma) = sqrt(10/3) for the cubic spline (Dehnen & Aly 2012),
    with sigma^2 the per-dimension variance of W; so eta = 1.2348 means
    (4 pi / 3) (GK eta)^3 = 47.995 neighbours."""
    o = oracle_mod
    H = 1.0
    m2, _ = integrate.quad(lambda r: 4 * math.pi * r ** 4 * o.W(r, H), 0, H, points=[0.5],
                           epsabs=1e-15, epsrel=1e-13)
    sigma = math.sqrt(m2 / 3.0)
    assert H / (2 * sigma) == pytest.approx(GK, rel=1e-12)
    assert 4 * math.pi / 3 * (GK * ETA) ** 3 == pytest.approx(47.995, abs=1e-3)


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("tree", [True, False])
def test_exact_lattice(oracle_mod, tree):
    """Exact cubic lattice (density 1): rho at the initial H, the converged H,
    rho and Omega there, the 57-neighbour count and zero force, against a
    lattice-shell sum of the textbook M4 kernel and a scipy root."""
    o = oracle_mod
    ns = 16
    d = gen.lattice(ns, jitter=0.0)
    dx = 1.0 / ns
    H0 = GK * ETA
    r0, _, c0 = o.density(d["x"], d["y"], d["z"], d["m"], d["H"], d["box"], tree=tree)
    assert np.allclose(r0, lattice_rho(H0), rtol=1e-13, atol=0)
    assert r0[0] == pytest.approx(1.0039808, abs=2e-7)
    C = (GK * ETA) ** 3
    Hs = optimize.brentq(lambda h: lattice_rho(h) * h ** 3 - C, 2.0, 2.3, xtol=1e-15, rtol=1e-15)
    s = o.solve_h(d["x"], d["y"], d["z"], d["m"], d["H"], d["box"], tree=tree)
    assert np.allclose(s["H"], Hs * dx, rtol=1e-10, atol=0)
    assert np.allclose(s["rho"], lattice_rho(Hs), rtol=1e-9, atol=0)
    assert np.all(s["cnt"] == 57)
    # Omega from a Richardson-extrapolated difference of the shell sum
    def dr(e):
        return (lattice_rho(Hs + e) - lattice_rho(Hs - e)) / (2 * e)
    e = 1e-4
    drho = (4 * dr(e / 2) - dr(e)) / 3
    om_ref = 1 + Hs / (3 * lattice_rho(Hs)) * drho
    g = o.ghost(s["rho"], s["drho"], s["H"], d["u"])
    assert np.allclose(g["omega"], om_ref, rtol=1e-9, atol=0)
    assert om_ref == pytest.approx(0.990098, abs=2e-6)
    f = o.force(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["m"], s["H"], g["A"],
                d["box"], tree=tree)
    scale = np.max(np.abs(g["A"])) * d["m"][0] * 8 / math.pi / s["H"][0] ** 4 * 57
    assert np.max(np.abs(f["ax"])) < 1e-12 * scale
    assert np.max(np.abs(f["dudt"])) == 0.0  # v = 0


def test_lattice_density_tends_to_continuum(oracle_mod):
    """On a uniform lattice the density estimate approaches the mean density
    as the number of neighbours grows."""
    o = oracle_mod
    d = gen.lattice(24, jitter=0.0)
    errs = []
    for f in (1.0, 1.5, 2.5):
        H = d["H"] * f
        rho, _, _ = o.density(d["x"], d["y"], d["z"], d["m"], H, d["box"])
        errs.append(abs(rho[0] - 1.0))
    assert errs[-1] < 1e-3 and errs[0] > errs[-1]


# ---------------------------------------------------------------- P4 / P5
def test_drho_dH_matches_finite_difference(oracle_mod):
    o = oracle_mod
    d = gen.lattice(12, jitter=0.3, seed=5)
    idx = np.arange(0, d["x"].size, 37)
    H = d["H"].copy()
    rho, drho, _ = o.density(d["x"], d["y"], d["z"], d["m"], H, d["box"], idx=idx)
    e = 1e-6 * H
    rp, _, _ = o.density(d["x"], d["y"], d["z"], d["m"], H + e, d["box"], idx=idx)
    rm, _, _ = o.density(d["x"], d["y"], d["z"], d["m"], H - e, d["box"], idx=idx)
    fd = (rp - rm) / (2 * e)
    scale = rho / H
    assert np.max(np.abs(fd[idx] - drho[idx]) / scale[idx]) < 1e-7


def test_newton_root_equals_bisection(oracle_mod):
    """rho H^3 - C is monotone in H, so an independent bisection (using the
    oracle's rho(H) only as a black box) finds the same unique root."""
    o = oracle_mod
    d = gen.lattice(10, jitter=0.4, seed=7)
    rng = np.random.default_rng(3)
    d["m"] = d["m"] * rng.uniform(0.5, 1.5, d["m"].size)
    idx = np.arange(0, d["x"].size, 97)
    s = o.solve_h(d["x"], d["y"], d["z"], d["m"], d["H"], d["box"], idx=idx, h_tol=1e-13)
    t = o.Tree(d["x"], d["y"], d["z"], d["box"])
    for i in idx:
        C = (GK * ETA) ** 3 * d["m"][i]

        def f(h):
            H = d["H"].copy()
            H[i] = h
            rho, _, _ = o.density(d["x"], d["y"], d["z"], d["m"], H, d["box"], tree=t, idx=[i])
            return rho[i] * h ** 3 - C

        lo, hi = 1e-3, 0.3
        assert f(lo) < 0 < f(hi)
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        assert s["H"][i] == pytest.approx(0.5 * (lo + hi), rel=1e-11)


# ---------------------------------------------------------------- P6
def test_bruteforce_equals_tree_16cubed(oracle_mod):
    """Cell/tree neighbour finding is complete: identical integer pair counts
    and values to round-off against O(N^2) brute force."""
    o = oracle_mod
    d = gen.lattice(16, jitter=0.1, vsigma=0.1, seed=11)
    a = o.full(d, tree=True)
    b = o.full(d, tree=False)
    assert np.array_equal(a["cnt"], b["cnt"]) and np.array_equal(a["fcnt"], b["fcnt"])
    assert a["n_force"] == b["n_force"]
    for k in ("H", "rho", "omega"):
        assert np.allclose(a[k], b[k], rtol=1e-13, atol=0), k
    sa = np.abs(a["ax"]).max()
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(a[k] - b[k])) < 1e-12 * sa
    assert np.max(np.abs(a["dudt"] - b["dudt"])) < 1e-12 * np.abs(a["dudt"]).max()


def test_bruteforce_equals_tree_subset_of_32cubed(oracle_mod):
    """The first 4096 particles of the 32^3 jittered box, brute-forced
    against all 32768."""
    o = oracle_mod
    d = gen.lattice(32, seed=2739)
    idx = np.arange(4096)
    a = o.solve_h(d["x"], d["y"], d["z"], d["m"], d["H"], d["box"], tree=True, idx=idx)
    b = o.solve_h(d["x"], d["y"], d["z"], d["m"], d["H"], d["box"], tree=False, idx=idx)
    assert np.array_equal(a["cnt"][idx], b["cnt"][idx])
    assert np.allclose(a["H"][idx], b["H"][idx], rtol=1e-13, atol=0)
    assert np.allclose(a["rho"][idx], b["rho"][idx], rtol=1e-13, atol=0)


# ---------------------------------------------------------------- P7 / P8 / P10
def _irregular(n_side=8, seed=21, vs=0.2):
    d = gen.lattice(n_side, jitter=0.3, vsigma=vs, seed=seed)
    rng = np.random.default_rng(seed)
    d["m"] = d["m"] * rng.uniform(0.6, 1.4, d["m"].size)
    d["u"] = rng.uniform(0.5, 2.0, d["m"].size)
    return d


def test_momentum_and_energy_identities(oracle_mod):
    """Sum_i m_i a_i = 0 (pairwise antisymmetry of eq. (dvdt)) and
    Sum_i m_i (v_i.a_i + du_i/dt) = 0 (eq. (dudt) paired with eq. (dvdt))."""
    o = oracle_mod
    d = _irregular(10)
    r = o.full(d, tree=True, h_tol=1e-12)
    m = d["m"]
    S = np.sum(m * (np.abs(r["ax"]) + np.abs(r["ay"]) + np.abs(r["az"])))
    for k in ("ax", "ay", "az"):
        assert abs(np.sum(m * r[k])) < 1e-14 * S
    pw = m * (d["vx"] * r["ax"] + d["vy"] * r["ay"] + d["vz"] * r["az"])
    E = np.sum(m * r["dudt"]) + np.sum(pw)
    assert abs(E) < 1e-13 * np.sum(np.abs(pw))
    assert np.all(r["omega"] > 0)


def _energy(d, H0, K, gamma=5.0 / 3.0):
    import oracle as o
    s = o.solve_h(d["x"], d["y"], d["z"], d["m"], H0, d["box"], tree=False, h_tol=1e-15,
                  max_iter=200)
    u = K * s["rho"] ** (gamma - 1) / (gamma - 1)
    return np.sum(d["m"] * u), s


def test_acceleration_is_energy_gradient(oracle_mod):
    """With H tied to rho by the constraint, eq. (dvdt) is the exact gradient
    of the thermal energy at fixed entropy: m_k a_k = -dU/dx_k, where U is
    re-evaluated (H re-solved) at displaced positions."""
    o = oracle_mod
    g = 5.0 / 3.0
    d = _irregular(8)
    base = o.full(d, tree=False, h_tol=1e-15, max_iter=200)
    K = (g - 1) * d["u"] / base["rho"] ** (g - 1)
    scale = np.max(d["m"] * np.abs(base["ax"]))
    delta = 1e-5
    for k in (0, 77, 301):
        for ax, key in ((0, "x"), (1, "y"), (2, "z")):
            vals = []
            for sgn in (1, -1):
                e = dict(d)
                e[key] = d[key].copy()
                e[key][k] += sgn * delta
                U, _ = _energy(e, base["H"], K)
                vals.append(U)
            grad = (vals[0] - vals[1]) / (2 * delta)
            acc = base["a" + key]
            assert abs(d["m"][k] * acc[k] + grad) < 2e-7 * scale


def test_dudt_is_adiabatic_compression(oracle_mod):
    """du_i/dt of eq. (dudt) equals (P_i/rho_i^2) drho_i/dt along the flow
    x + v t, with H re-solved (finite difference in t)."""
    o = oracle_mod
    d = _irregular(8, seed=4)
    base = o.full(d, tree=False, h_tol=1e-15, max_iter=200)
    dt = 1e-6
    rr = []
    for sgn in (1, -1):
        e = dict(d)
        for c, v in (("x", "vx"), ("y", "vy"), ("z", "vz")):
            e[c] = np.mod(d[c] + sgn * dt * d[v], 1.0)
        s = o.solve_h(e["x"], e["y"], e["z"], e["m"], base["H"], e["box"], tree=False,
                      h_tol=1e-15, max_iter=200)
        rr.append(s["rho"])
    drho_dt = (rr[0] - rr[1]) / (2 * dt)
    ref = base["P"] / base["rho"] ** 2 * drho_dt
    scale = np.max(np.abs(base["dudt"]))
    assert np.max(np.abs(base["dudt"] - ref)) < 1e-6 * scale


def test_kdk_energy_error_is_second_order(oracle_mod):
    """Total energy drift of the kick-drift-kick step over a fixed time falls
    by ~4x when dt halves; mass and momentum stay at round-off."""
    o = oracle_mod
    d0 = _irregular(8, seed=9, vs=0.1)
    drifts = []
    for nsteps, dt in ((32, 0.0015), (64, 0.00075)):
        d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in d0.items()}
        r = o.full(d, tree=False, h_tol=1e-13)
        st = dict(d)
        st["H"] = r["H"].copy()
        for k in ("ax", "ay", "az", "dudt"):
            st[k] = r[k].copy()
        e0 = o.conserved(st["m"], st["vx"], st["vy"], st["vz"], st["u"])
        for _ in range(nsteps):
            o.step(st, dt, tree=False, h_tol=1e-13)
        e1 = o.conserved(st["m"], st["vx"], st["vy"], st["vz"], st["u"])
        drifts.append(abs(e1[4] - e0[4]) / e0[4])
        pscale = np.sum(st["m"] * np.abs(st["vx"]))
        assert abs(e1[1] - e0[1]) < 1e-13 * pscale
    ratio = drifts[0] / drifts[1]
    assert 3.5 < ratio < 4.5, (drifts, ratio)


# ---------------------------------------------------------------- P9
def test_invariances(oracle_mod):
    """Periodic translation, Galilean boost and the scaling x,H -> lx,lH,
    m -> l^3 m leave rho, a and du/dt unchanged."""
    o = oracle_mod
    d = _irregular(9, seed=13)
    a = o.full(d, tree=True, h_tol=1e-12)
    t = dict(d)
    for c, s in (("x", 0.31), ("y", 0.77), ("z", 0.05)):
        t[c] = np.mod(d[c] + s, 1.0)
    for c, s in (("vx", 3.0), ("vy", -1.0), ("vz", 0.5)):
        t[c] = d[c] + s
    b = o.full(t, tree=True, h_tol=1e-12)
    assert np.allclose(a["rho"], b["rho"], rtol=1e-10, atol=0)
    sa = np.abs(a["ax"]).max()
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(a[k] - b[k])) < 1e-9 * sa
    assert np.max(np.abs(a["dudt"] - b["dudt"])) < 1e-9 * np.abs(a["dudt"]).max()
    lam = 3.0
    s = dict(d)
    for c in ("x", "y", "z"):
        s[c] = d[c] * lam
    s["box"] = d["box"] * lam
    s["H"] = d["H"] * lam
    s["m"] = d["m"] * lam ** 3
    c = o.full(s, tree=True, h_tol=1e-12)
    assert np.allclose(c["rho"], a["rho"], rtol=1e-10, atol=0)
    assert np.allclose(c["H"], a["H"] * lam, rtol=1e-10, atol=0)
