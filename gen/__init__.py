"""Seeded synthetic particle sets shaped like the paper's SPH workloads.

Input generation only: positions, velocities, internal energies, masses and a
first guess of each particle's smoothing length.  Nothing here evaluates the
SPH sums, the smoothing-length iteration or the forces; both the FP64 oracle
and the GPU library consume these arrays.

Conventions (Section 2 of the paper):
  * ``H`` is the paper's smoothing length h: the radius of the sphere inside
    which neighbours contribute (the kernel's compact support).
  * The target neighbour number is fixed through ``eta`` in the
    Dehnen--Aly convention, h_DA = H / GAMMA_K with GAMMA_K = sqrt(10/3) for
    the cubic spline, so that a particle at uniform spacing ``dx`` starts from
    H = GAMMA_K * eta * dx.

All generators use numpy's PCG64 with an explicit seed.  Every array is
float64 except ``domain`` (int32) and ``id`` (int64).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA_K = math.sqrt(10.0 / 3.0)
ETA = 1.2348
GAMMA_GAS = 5.0 / 3.0
SEED_BASE = 2738


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _finish(d, n):
    d.setdefault("vx", np.zeros(n))
    d.setdefault("vy", np.zeros(n))
    d.setdefault("vz", np.zeros(n))
    d["id"] = np.arange(n, dtype=np.int64)
    if "domain" not in d:
        d["domain"] = np.zeros(n, dtype=np.int32)
        d["boxes"] = np.asarray(d["box"], dtype=np.float64).reshape(1, 3)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m", "H"):
        d[k] = np.ascontiguousarray(d[k], dtype=np.float64)
    return d


def lattice(n_side=32, jitter=0.1, vsigma=0.0, seed=SEED_BASE + 1, u0=1.0):
    """Periodic unit box, n_side^3 equal-mass particles at (i+1/2)*dx plus
    uniform jitter of +-``jitter``*dx per coordinate; rho = 1 in the mean."""
    rng = _rng(seed)
    n = n_side ** 3
    dx = 1.0 / n_side
    g = (np.arange(n_side) + 0.5) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = [a.ravel().copy() for a in (X, Y, Z)]
    if jitter > 0:
        for a in pos:
            a += rng.uniform(-jitter * dx, jitter * dx, size=n)
            np.mod(a, 1.0, out=a)
    d = dict(x=pos[0], y=pos[1], z=pos[2], box=np.array([1.0, 1.0, 1.0]))
    if vsigma > 0:
        d["vx"] = rng.normal(0.0, vsigma, n)
        d["vy"] = rng.normal(0.0, vsigma, n)
        d["vz"] = rng.normal(0.0, vsigma, n)
    d["u"] = np.full(n, u0)
    d["m"] = np.full(n, 1.0 / n)
    d["H"] = np.full(n, GAMMA_K * ETA * dx)
    return _finish(d, n)


def sod(n_left=100, seed=SEED_BASE + 2):
    """Sod-like tube in a periodic 2x1x1 box: a lattice of n_left^3 particles
    in [0,1)^3 and one of (n_left/2)^3 in [1,2)x[0,1)^2, equal masses, so the
    right half has 1/8 of the density; P_L = 1, P_R = 0.1 for gamma = 5/3."""
    assert n_left % 2 == 0
    n_right = n_left // 2
    dl, dr = 1.0 / n_left, 1.0 / n_right

    def lat(ns, dx, x0):
        g = (np.arange(ns) + 0.5) * dx
        X, Y, Z = np.meshgrid(g + x0, g, g, indexing="ij")
        return X.ravel(), Y.ravel(), Z.ravel()

    xl, yl, zl = lat(n_left, dl, 0.0)
    xr, yr, zr = lat(n_right, dr, 1.0)
    nl, nr = xl.size, xr.size
    n = nl + nr
    m = 1.0 / nl  # rho_L = 1
    d = dict(x=np.concatenate([xl, xr]), y=np.concatenate([yl, yr]),
             z=np.concatenate([zl, zr]), box=np.array([2.0, 1.0, 1.0]))
    d["m"] = np.full(n, m)
    # P = (gamma-1) rho u  ->  u_L = 1.5 (P=1, rho=1), u_R = 1.2 (P=0.1, rho=1/8)
    d["u"] = np.concatenate([np.full(nl, 1.5), np.full(nr, 1.2)])
    d["H"] = np.concatenate([np.full(nl, GAMMA_K * ETA * dl), np.full(nr, GAMMA_K * ETA * dr)])
    return _finish(d, n)


def _gaussian_field(n_grid, rng, slope, smooth):
    """Zero-mean unit-variance Gaussian random field on an n_grid^3 periodic
    grid (unit box) with power P(k) ~ k^slope times a Gaussian window of
    width ``smooth``."""
    white = rng.standard_normal((n_grid, n_grid, n_grid))
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n_grid) * n_grid * 2 * np.pi
    kz = np.fft.rfftfreq(n_grid) * n_grid * 2 * np.pi
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    amp = k2 ** (slope / 4.0) * np.exp(-0.5 * k2 * smooth * smooth)
    amp[0, 0, 0] = 0.0
    fk *= amp
    del k2, amp
    f = np.fft.irfftn(fk, s=(n_grid, n_grid, n_grid), axes=(0, 1, 2))
    f -= f.mean()
    f /= f.std()
    return f


def _initial_H_from_counts(x, y, z, m, box, n_min=32):
    """First guess of H from particle counts on successively coarser grids:
    the finest grid cell holding at least ``n_min`` particles gives the
    local number density."""
    n = x.size
    Lx, Ly, Lz = box
    rho_est = np.full(n, np.nan)
    g = 1
    while g * 2 <= max(2, round(n ** (1 / 3))):
        g *= 2
    while g >= 1:
        ix = np.minimum((x / Lx * g).astype(np.int64), g - 1)
        iy = np.minimum((y / Ly * g).astype(np.int64), g - 1)
        iz = np.minimum((z / Lz * g).astype(np.int64), g - 1)
        cell = (ix * g + iy) * g + iz
        cnt = np.bincount(cell, minlength=g ** 3)[cell]
        vol = Lx * Ly * Lz / g ** 3
        ok = np.isnan(rho_est) & (cnt >= n_min)
        rho_est[ok] = cnt[ok] * m[ok] / vol
        if not np.isnan(rho_est).any():
            break
        g //= 2
    rho_est[np.isnan(rho_est)] = m[np.isnan(rho_est)] * n / (Lx * Ly * Lz)
    H = GAMMA_K * ETA * (m / rho_est) ** (1.0 / 3.0)
    return np.minimum(H, 0.2 * min(box))


def clustered(n_side=256, seed=SEED_BASE + 3, n_halos=500, sigma_ln=1.5,
              halo_frac=0.3, vsigma=0.1, c_range=(5.0, 15.0), decades=3.0):
    """Clustered cosmology-like periodic unit box of n_side^3 equal-mass
    particles: a lognormal density field (Gaussian field with P(k) ~ k^-2,
    smoothed at L/64, sigma_ln of log-density) plus NFW halos with
    concentrations uniform in ``c_range`` and particle counts log-uniform
    over ``decades`` decades, centred on draws from the lognormal density."""
    rng = _rng(seed)
    n = n_side ** 3
    m = 1.0 / n
    ng = n_side
    delta = _gaussian_field(ng, rng, -2.0, 1.0 / 64.0)
    rho = np.exp(sigma_ln * delta - 0.5 * sigma_ln ** 2).ravel()
    del delta
    p = rho / rho.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0

    # halo particle counts: log-uniform over `decades`, rescaled to halo_frac*n
    n_halo_tot = int(round(halo_frac * n)) if n_halos > 0 else 0
    if n_halos > 0:
        raw = 10.0 ** rng.uniform(0.0, decades, n_halos)
        counts = np.floor(raw / raw.sum() * n_halo_tot).astype(np.int64)
        short = n_halo_tot - counts.sum()
        counts[np.argsort(-raw)[:short]] += 1
    n_ln = n - n_halo_tot

    def draw_cells(k):
        c = np.searchsorted(cdf, rng.random(k), side="right")
        c = np.minimum(c, ng ** 3 - 1)
        iz = c % ng
        iy = (c // ng) % ng
        ix = c // (ng * ng)
        return ((ix + rng.random(k)) / ng, (iy + rng.random(k)) / ng,
                (iz + rng.random(k)) / ng)

    xs, ys, zs = draw_cells(n_ln)
    parts_x, parts_y, parts_z = [xs], [ys], [zs]
    if n_halos > 0:
        cx, cy, cz = draw_cells(n_halos)
        conc = rng.uniform(c_range[0], c_range[1], n_halos)
        # inverse of the NFW enclosed-mass profile mu(x) = ln(1+x) - x/(1+x)
        xt = np.concatenate([[0.0], np.geomspace(1e-6, c_range[1], 4000)])
        mut = np.log1p(xt) - xt / (1.0 + xt)
        for h in range(n_halos):
            k = int(counts[h])
            if k == 0:
                continue
            r200 = (3.0 * k * m / (4.0 * math.pi * 200.0)) ** (1.0 / 3.0)
            c = conc[h]
            muc = math.log1p(c) - c / (1.0 + c)
            s = np.interp(rng.random(k) * muc, mut, xt)
            r = s * r200 / c
            cth = rng.uniform(-1.0, 1.0, k)
            phi = rng.uniform(0.0, 2 * math.pi, k)
            sth = np.sqrt(1.0 - cth * cth)
            parts_x.append(cx[h] + r * sth * np.cos(phi))
            parts_y.append(cy[h] + r * sth * np.sin(phi))
            parts_z.append(cz[h] + r * cth)
    x = np.mod(np.concatenate(parts_x), 1.0)
    y = np.mod(np.concatenate(parts_y), 1.0)
    z = np.mod(np.concatenate(parts_z), 1.0)
    # 1.0 can appear from rounding of mod on tiny negatives
    for a in (x, y, z):
        a[a >= 1.0] = 0.0
    perm = rng.permutation(n)
    x, y, z = x[perm], y[perm], z[perm]
    d = dict(x=x, y=y, z=z, box=np.array([1.0, 1.0, 1.0]))
    d["m"] = np.full(n, m)
    d["u"] = np.ones(n)
    if vsigma > 0:
        d["vx"] = rng.normal(0.0, vsigma, n)
        d["vy"] = rng.normal(0.0, vsigma, n)
        d["vz"] = rng.normal(0.0, vsigma, n)
    d["H"] = _initial_H_from_counts(x, y, z, d["m"], (1.0, 1.0, 1.0))
    return _finish(d, n)


def perturbed_lattice(n_side, rng, amp=0.3, smooth=0.1, jitter=0.1):
    """Jittered lattice in a unit box displaced along the gradient of a
    Gaussian random field (linear Zel'dovich step) so that the linear density
    contrast has r.m.s. ``amp``."""
    n = n_side ** 3
    dx = 1.0 / n_side
    delta = _gaussian_field(n_side, rng, 0.0, smooth) * amp
    fk = np.fft.rfftn(delta)
    kx = np.fft.fftfreq(n_side) * n_side * 2 * np.pi
    kz = np.fft.rfftfreq(n_side) * n_side * 2 * np.pi
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2[0, 0, 0] = 1.0
    # displacement psi with div(psi) = -delta
    psi = [np.fft.irfftn(1j * K * fk / k2, s=delta.shape, axes=(0, 1, 2)).ravel() for K in (KX, KY, KZ)]
    g = (np.arange(n_side) + 0.5) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = []
    for a, p in zip((X, Y, Z), psi):
        b = a.ravel() + p + rng.uniform(-jitter * dx, jitter * dx, n)
        b = np.mod(b, 1.0)
        b[b >= 1.0] = 0.0
        pos.append(b)
    return pos


def ensemble(n_boxes=64, side_range=(16, 96), seed=SEED_BASE + 5, amp=0.3):
    """``n_boxes`` independent periodic unit boxes, n_side ~ U{side_range},
    each a jittered lattice with a Gaussian density perturbation of r.m.s.
    ``amp``; particle masses 1/N_b per box, u = 1, v = 0.  Particles carry
    their box index in ``domain``."""
    rng = _rng(seed)
    sides = rng.integers(side_range[0], side_range[1] + 1, n_boxes)
    xs, ys, zs, ms, Hs, doms = [], [], [], [], [], []
    for b, ns in enumerate(sides):
        x, y, z = perturbed_lattice(int(ns), rng, amp=amp)
        nb = int(ns) ** 3
        m = np.full(nb, 1.0 / nb)
        xs.append(x), ys.append(y), zs.append(z), ms.append(m)
        Hs.append(_initial_H_from_counts(x, y, z, m, (1.0, 1.0, 1.0), n_min=16))
        doms.append(np.full(nb, b, dtype=np.int32))
    n = sum(a.size for a in xs)
    d = dict(x=np.concatenate(xs), y=np.concatenate(ys), z=np.concatenate(zs),
             m=np.concatenate(ms), H=np.concatenate(Hs), u=np.ones(n),
             domain=np.concatenate(doms), boxes=np.ones((n_boxes, 3)),
             box=np.array([1.0, 1.0, 1.0]), sides=sides)
    return _finish(d, n)


def make_config(k, seed=None, small=False):
    """The five workloads, by index 1..5 (``small`` gives a reduced size of
    the same shape for tests)."""
    s = SEED_BASE + k if seed is None else seed
    if k == 1:
        return lattice(16 if small else 32, seed=s)
    if k == 2:
        return sod(20 if small else 100, seed=s)
    if k in (3, 4):
        return clustered(32 if small else 256, seed=s, n_halos=20 if small else 500)
    if k == 5:
        return ensemble(4 if small else 64, (12, 16) if small else (16, 96), seed=s)
    raise ValueError(k)


def subset(d, idx):
    """Particle subset (same box) of a generated set."""
    out = dict(d)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "m", "H", "id", "domain"):
        out[k] = np.ascontiguousarray(d[k][idx])
    return out
