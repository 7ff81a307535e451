"""Pins of the oracle's deterministic primary (eq. (7)) and of the angular
interpolation of scatter maps (section II-C-3).

* Empty object: the expected primary per emitted photon is the mean eta over
  the spectrum's draw probabilities times Omega_pixel / Omega_cone, the
  closed-form rectangle solid angle (no fit).
* Homogeneous box: Beer-Lambert exp(-mu L(ray)) with L the exact chord of the
  box (fp64 slab method), integrated over each pixel by a finer independent
  quadrature.
* A random polychromatic phantom: the analog primary counts of the Monte
  Carlo (eta = 1) are Poisson around N times the expectation, pixel by pixel.
* Interpolation: between samples of A + B cos(beta) + C sin(beta) taken every
  other angle, the mean of the two neighbours is exactly
  A + (B cos(beta) + C sin(beta)) cos(d_beta).
"""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs
from test_oracle_samplers import chi2_z
from test_oracle_transport import omega_cone, omega_pixels

GEO = dict(sod_mm=300.0, sdd_mm=600.0, nu=24, nv=20, pu_mm=6.0, pv_mm=6.0, step_mm=0.8)


def _setup(ids, rho, h, spec, eta=None):
    o = oracle.Oracle()
    o.load_phantom(ids, rho, h)
    o.set_geometry(**GEO)
    o.set_spectrum(*spec)
    if eta is not None:
        o.set_detector_response(eta)
    return o


def _mean_eta(spec, o):
    e, w = spec
    _, _, _, eta = o.tables(5)
    # the sampler's draw probabilities: differences of floor(W_k / W 2^32)
    cw = np.cumsum(w.astype(np.float64))
    thr = np.floor(cw / cw[-1] * 2.0 ** 32)
    thr[-1] = 2.0 ** 32
    p = np.diff(np.concatenate([[0.0], thr])) / 2.0 ** 32
    x = e.astype(np.float64) - 1
    j = np.clip(np.floor(x).astype(int), 0, len(eta) - 2)
    f = (e - 1).astype(np.float32) - j.astype(np.float32)
    et = eta[j] + f * (eta[j + 1] - eta[j])
    return float(np.sum(p * et.astype(np.float64)))


def test_primary_vacuum_solid_angles(oracle_lib):
    spec = inputs.kramers_spectrum(90, 1.0)
    ids, rho = inputs.box_phantom(12, 12, 12, 1, 0.0)
    o = _setup(ids, rho, 2.0, spec)
    det = o.primary_expected(0.4, sub=8)
    exp = _mean_eta(spec, o) * omega_pixels(GEO) / omega_cone(GEO)
    assert np.max(np.abs(det / exp - 1)) < 2e-5, np.max(np.abs(det / exp - 1))


def _chord(S, w, half):
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-half - S) / w
        t2 = (half - S) / w
    tin = np.nanmax(np.minimum(t1, t2), axis=-1)
    tout = np.nanmin(np.maximum(t1, t2), axis=-1)
    return np.clip(tout - tin, 0.0, None)


def test_primary_beer_lambert_box(oracle_lib):
    e0 = 70.0
    n, h, rho0 = 16, 3.0, 1.3
    ids, rho = inputs.box_phantom(n, n, n, 2, rho0)
    o = _setup(ids, rho, h, inputs.mono_spectrum(e0))
    pe, coh, inc, _ = o.tables(5)
    jj = int(e0 - 1)
    mu = np.float64(np.float32(rho0)) * np.float64(
        np.float32((np.float32(pe[2, jj]) + np.float32(coh[2, jj])) + np.float32(inc[2, jj])) *
        np.float32(0.1))
    beta = 0.25
    # the same 24 x 24 midpoint rule (the vacuum pin checks the rule itself); the
    # chords here are exact (fp64 slab method) instead of marched
    det = o.primary_expected(beta, sub=24)
    S = np.array([GEO["sod_mm"] * np.cos(beta), GEO["sod_mm"] * np.sin(beta), 0.0])
    ax = -np.array([np.cos(beta), np.sin(beta), 0.0])
    eu, ev = np.array([-np.sin(beta), np.cos(beta), 0.0]), np.array([0.0, 0.0, 1.0])
    D = S + GEO["sdd_mm"] * ax
    m = 24
    hu, hv = GEO["nu"] * GEO["pu_mm"] / 2, GEO["nv"] * GEO["pv_mm"] / 2
    us = -hu + (np.arange(GEO["nu"] * m) + 0.5) * GEO["pu_mm"] / m
    vs = -hv + (np.arange(GEO["nv"] * m) + 0.5) * GEO["pv_mm"] / m
    U, V = np.meshgrid(us, vs, indexing="xy")
    Q = D + U[..., None] * eu + V[..., None] * ev
    W = Q - S
    R = np.linalg.norm(W, axis=-1)
    w = W / R[..., None]
    L = _chord(S, w, n * h / 2)
    dA = GEO["pu_mm"] * GEO["pv_mm"] / m ** 2
    f = np.exp(-mu * L) * (w @ ax) * dA / R ** 2 * e0
    exp = f.reshape(GEO["nv"], m, GEO["nu"], m).sum(axis=(1, 3)) / omega_cone(GEO)
    rel = np.abs(det / exp - 1)
    assert np.max(rel) < 1e-5, np.max(rel)
    assert det.min() < 0.5 * det.max()              # the box does attenuate


def test_primary_matches_monte_carlo(oracle_lib):
    spec = inputs.kramers_spectrum(110, 2.0)
    ids, rho = inputs.ellipsoid_phantom(30, 2.0, seed=21)
    o = _setup(ids, rho, 2.0, spec, eta=np.ones(200, np.float32))
    det = o.primary_expected(1.3, sub=4)
    n = 3_000_000
    p, _ = o.project(1.3, n, 17, threads=8)
    counts = p.astype(np.float64) / 2 ** 20
    exp = n * det
    assert exp.min() > 20
    z = (counts - exp) / np.sqrt(exp)
    assert np.abs(z).max() < 5, np.abs(z).max()
    assert abs(chi2_z(np.append(counts.ravel(), n - counts.sum()),
                      np.append(exp.ravel(), n - exp.sum()) / n)) < 5


def test_interp_angles_closed_form(oracle_lib):
    n_sim, npx = 90, 37
    rng = np.random.default_rng(3)
    A, B, Cc = rng.uniform(1, 2, npx), rng.uniform(-0.3, 0.3, npx), rng.uniform(-0.3, 0.3, npx)
    beta = 2 * np.pi * np.arange(2 * n_sim) / (2 * n_sim)
    field = lambda b: A + B * np.cos(b)[:, None] + Cc * np.sin(b)[:, None]
    sim = field(beta[::2]).astype(np.float32)
    full = oracle.interp_angles(sim)
    assert np.array_equal(full[::2], sim)
    db = beta[1] - beta[0]
    exact = A + (B * np.cos(beta[1::2])[:, None] + Cc * np.sin(beta[1::2])[:, None]) * np.cos(db)
    assert np.max(np.abs(full[1::2] - exact)) < 2e-6
    # and against the field itself: second-order error in the angular step
    assert np.max(np.abs(full[1::2] - field(beta[1::2]))) < 0.31 * db ** 2
