"""Pins of the reconstruction-side oracle of the iterative scatter correction
(section II-E: line integrals, FBP, Otsu segmentation, volume to density,
eq. (8)).

* FDK on the exact line integrals of a uniform ball (analytic chords): the
  interior reconstructs to mu within 0.5 % (0.2 % near the mid-plane, where
  FDK is exact up to discretisation), at the right place.
* The Ram-Lak kernel's frequency response: 0 at DC and 1/(2t) at Nyquist
  (|f|), from the kernel's series.
* Otsu on a two-mode histogram: the threshold lies between the modes, and
  equals the minimiser of the within-class variance (the other form of the
  criterion).
* Eq. (8) turns the measured line integral of primary + scatter into the
  primary's when Ip and Is are the true ones.
"""
import numpy as np
import pytest

from oracle import recon

GEO = dict(sod_mm=300.0, sdd_mm=600.0, nu=96, nv=64, pu_mm=2.0, pv_mm=2.0)


def ball_projections(geo, n_ang, r, mu0, c):
    R, D = geo["sod_mm"], geo["sdd_mm"]
    u = -geo["nu"] * geo["pu_mm"] / 2 + (np.arange(geo["nu"]) + 0.5) * geo["pu_mm"]
    v = -geo["nv"] * geo["pv_mm"] / 2 + (np.arange(geo["nv"]) + 0.5) * geo["pv_mm"]
    U, V = np.meshgrid(u, v, indexing="xy")
    proj = np.zeros((n_ang, geo["nv"], geo["nu"]))
    for i in range(n_ang):
        b = 2 * np.pi * i / n_ang
        S = np.array([R * np.cos(b), R * np.sin(b), 0.0])
        ax = -np.array([np.cos(b), np.sin(b), 0.0])
        eu, ev = np.array([-np.sin(b), np.cos(b), 0.0]), np.array([0.0, 0.0, 1.0])
        Q = S + D * ax + U[..., None] * eu + V[..., None] * ev
        w = Q - S
        w /= np.linalg.norm(w, axis=-1)[..., None]
        oc = S - c
        bq = w @ oc
        disc = bq * bq - (oc @ oc - r * r)
        proj[i] = np.where(disc > 0, 2 * np.sqrt(np.maximum(disc, 0.0)), 0.0) * mu0
    return proj


def test_fdk_uniform_ball():
    r, mu0, c = 30.0, 0.02, np.array([5.0, -3.0, 4.0])
    f = recon.fdk(ball_projections(GEO, 180, r, mu0, c), GEO, (40, 48, 48), 2.0)
    zs = (np.arange(40) + 0.5) * 2 - 40
    ys = (np.arange(48) + 0.5) * 2 - 48
    Z, Y, X = np.meshgrid(zs, ys, ys, indexing="ij")
    d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    inner = d < r - 5
    assert abs(f[inner].mean() / mu0 - 1) < 5e-3
    assert f[inner].std() / mu0 < 1e-2
    mid = inner & (np.abs(Z - c[2]) < 2)
    assert abs(f[mid].mean() / mu0 - 1) < 2e-3
    assert np.abs(f[d > r + 8]).mean() / mu0 < 2e-2
    # the object is where it is: centroid of the reconstruction
    w = np.clip(f, 0, None)
    cen = np.array([(w * X).sum(), (w * Y).sum(), (w * Z).sum()]) / w.sum()
    assert np.max(np.abs(cen - c)) < 0.5


def test_ramp_kernel_frequency_response():
    t = 0.7
    n = 200_001
    h = recon.ramp_kernel(n, t)
    k = np.arange(-(n - 1), n)
    H0 = t * h.sum()
    Hn = t * np.sum(h * np.cos(np.pi * k))
    assert abs(H0) < 2e-6 / t
    assert abs(Hn - 1.0 / (2 * t)) < 2e-6 / t


def test_otsu_two_modes():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0.2, 0.05, 30_000), rng.normal(0.8, 0.08, 10_000)])
    counts = recon.histogram(x, 0.0, 1.0, 256)
    t = recon.otsu_bin(counts)
    assert 0.3 < t / 256 < 0.7
    # the same split minimises the within-class variance
    c = counts.astype(np.float64)
    idx = np.arange(256.0)
    best = None
    for s in range(1, 256):
        w0, w1 = c[:s].sum(), c[s:].sum()
        if w0 == 0 or w1 == 0:
            continue
        v0 = ((idx[:s] - (c[:s] * idx[:s]).sum() / w0) ** 2 * c[:s]).sum()
        v1 = ((idx[s:] - (c[s:] * idx[s:]).sum() / w1) ** 2 * c[s:]).sum()
        if best is None or v0 + v1 < best[0] - 1e-9:
            best = (v0 + v1, s)
    assert best[1] == t


def test_histogram_bins():
    x = np.array([0.0, 0.1, 0.25, 0.999, 1.0, -0.1])
    assert list(recon.histogram(x, 0.0, 1.0, 4)) == [2, 1, 0, 1]


def test_eq8_recovers_primary():
    rng = np.random.default_rng(2)
    I0 = rng.uniform(5, 10, 1000)
    ip = I0 * np.exp(-rng.uniform(0, 4, 1000))
    is_ = rng.uniform(0.01, 2, 1000)
    a = recon.line_integrals(ip + is_, I0)
    c = recon.scatter_correct(a, ip, is_)
    assert np.max(np.abs(c - (-np.log(ip / I0)))) < 1e-12
    assert np.all(c > a)


def test_to_density_round_trip():
    rho = np.array([0.0, 0.5, 1.0, 1.37, 2.7])
    mu = rho * 0.1 * 0.2                     # mu/rho 0.2 cm^2/g
    ids, r = recon.to_density(mu, 0.012, 0.2, 1)
    assert list(ids) == [0, 0, 1, 1, 1]
    assert np.allclose(r[2:], [1.0, 1.37, 2.7], atol=0.0025)
    assert r[0] == np.float32(0.001205)
