"""Pins of the oracle's transport and tally against closed forms.

* Source: with an empty (vacuum) object, pixel counts are multinomial with
  p = Omega_pixel / Omega_cone (closed-form rectangle solid angles).
* Flight (Beer-Lambert): a homogeneous slab with every interaction absorbing
  transmits exp(-mu T / cos(gamma)) per ray; per-pixel expectation integrates
  this over the pixel's solid angle.
* Interaction fractions: first-interaction types in a thick block are
  multinomial with sigma_i / sigma_tot.
* Detector mapping: rays aimed at pixel centres land in that pixel at any
  projection angle (u along (-sin b, cos b, 0), v along z).
* Brute force on a tiny random phantom: the primary image against the
  deterministic expectation from an independent fp64 fixed-step line integral
  through the same voxels.
* Tally: fixed point keV * 2^20; photon ranges add up bitwise; the threaded
  driver equals the sequential one; overflow and argument errors are refused.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs
from test_oracle_samplers import chi2_z

ONE = 2 ** 20


def rect_solid_angle(u1, u2, v1, v2, d):
    F = lambda u, v: np.arctan(u * v / (d * np.sqrt(d * d + u * u + v * v)))
    return F(u2, v2) - F(u1, v2) - F(u2, v1) + F(u1, v1)


def make(ids, rho, h, spectrum=(60.0,), **geo):
    o = oracle.Oracle()
    o.load_phantom(ids, rho, h)
    g = dict(sod_mm=500.0, sdd_mm=1000.0, nu=64, nv=64, pu_mm=2.0, pv_mm=2.0, step_mm=0.5)
    g.update(geo)
    o.set_geometry(**g)
    o.set_spectrum(*inputs.mono_spectrum(spectrum[0]))
    return o


def pixel_grid(g, sub=1):
    """Sub-pixel edges (u, v) on the panel, in mm from the panel centre."""
    u = -g["nu"] * g["pu_mm"] / 2 + np.arange(g["nu"] * sub + 1) * g["pu_mm"] / sub
    v = -g["nv"] * g["pv_mm"] / 2 + np.arange(g["nv"] * sub + 1) * g["pv_mm"] / sub
    return u, v


def omega_pixels(g, sub=1):
    u, v = pixel_grid(g, sub)
    U1, V1 = np.meshgrid(u[:-1], v[:-1])
    U2, V2 = np.meshgrid(u[1:], v[1:])
    return rect_solid_angle(U1, U2, V1, V2, g["sdd_mm"])      # [v][u]


def omega_cone(g):
    hu, hv = g["nu"] * g["pu_mm"] / 2, g["nv"] * g["pv_mm"] / 2
    return 2 * np.pi * (1 - g["sdd_mm"] / np.sqrt(g["sdd_mm"] ** 2 + hu * hu + hv * hv))


def counting(o):
    o.set_detector_response(np.ones(1100, np.float32))      # eta = 1: counts


def test_source_multinomial_vacuum(oracle_lib):
    ids, rho = inputs.box_phantom(8, 8, 8, 0, 0.0)
    o = make(ids, rho, 1.0)
    counting(o)
    n = 1_000_000
    p, s = o.project(0.3, n, seed=11)
    assert s.sum() == 0
    assert np.all(p % ONE == 0)
    cnt = p // ONE
    probs = omega_pixels(o.geometry) / omega_cone(o.geometry)
    tot_p = probs.sum()
    assert abs(cnt.sum() - n * tot_p) < 5 * np.sqrt(n * tot_p * (1 - tot_p))
    z = chi2_z(np.append(cnt.ravel(), n - cnt.sum()), np.append(probs.ravel(), 1 - tot_p))
    assert abs(z) < 5, z


def test_beer_lambert_slab(oracle_lib):
    # water slab 10 mm thick (x), lateral +-64 mm: every ray in the cone enters
    # the front face and leaves the back face
    T = 10.0
    ids, rho = inputs.box_phantom(10, 128, 128, 1, 1.0)
    # 20.7 keV lies between grid points: mu is the linear interpolation of the
    # tabulated values at 20 and 21 keV
    o = make(ids, rho, 1.0, spectrum=(20.7,), flags=oracle.NO_SCATTER, nu=64, nv=64,
             pu_mm=2.0, pv_mm=2.0, step_mm=0.7)
    counting(o)
    pe, coh, inc, _ = o.tables(5)
    tot = pe[1].astype(np.float64) + coh[1] + inc[1]
    f = float(np.float32(20.7)) - 20.0
    mu = 1.0 * 0.1 * (tot[19] + f * (tot[20] - tot[19]))               # 1/mm
    n = 2_000_000
    p, s = o.project(0.0, n, seed=21)
    assert s.sum() == 0
    cnt = p // ONE
    sub = 8
    g = o.geometry
    om = omega_pixels(g, sub)
    u, v = pixel_grid(g, sub)
    uc, vc = 0.5 * (u[1:] + u[:-1]), 0.5 * (v[1:] + v[:-1])
    UC, VC = np.meshgrid(uc, vc)
    cosg = g["sdd_mm"] / np.sqrt(g["sdd_mm"] ** 2 + UC ** 2 + VC ** 2)
    trans = np.exp(-mu * T / cosg)
    exp_sub = n * om / omega_cone(g) * trans
    exp = exp_sub.reshape(g["nv"], sub, g["nu"], sub).sum(axis=(1, 3))
    assert abs(cnt.sum() - exp.sum()) < 5 * np.sqrt(exp.sum())
    z = chi2_z(np.append(cnt.ravel(), n - cnt.sum()),
               np.append(exp.ravel(), n - exp.sum()) / n)
    assert abs(z) < 5, z
    # and the absorbed fraction is what the slab removes
    st = o.stats()
    assert st["photo"] + st["primary_hits"] <= n


def test_interaction_fractions(oracle_lib):
    ids, rho = inputs.box_phantom(40, 40, 40, 2, 2.699)
    o = make(ids, rho, 2.0, spectrum=(60.0,), nu=16, nv=16, pu_mm=1.0, pv_mm=1.0)
    pe, coh, inc, _ = o.tables(5)
    n_int, steps, end, first = o.debug_histories(0.0, 0, 300_000, seed=5)
    f = first[first != oracle.FIRST_NONE]
    counts = np.bincount(f, minlength=4)[1:]
    sig = np.array([pe[2, 59], coh[2, 59], inc[2, 59]], np.float64)
    assert abs(chi2_z(counts, sig / sig.sum())) < 5
    assert len(f) > 250_000


def test_detector_pencil_rays(oracle_lib):
    ids, rho = inputs.box_phantom(8, 8, 8, 0, 0.0)
    o = make(ids, rho, 1.0, nu=48, nv=40, pu_mm=1.3, pv_mm=0.9)
    g = o.geometry
    rng = np.random.default_rng(0)
    for beta in [0.0, 0.7, np.pi / 2, 2.5, np.pi, 4.0, 5.9]:
        b = float(np.float32(beta))
        S = g["sod_mm"] * np.array([np.cos(b), np.sin(b), 0.0])
        a = -np.array([np.cos(b), np.sin(b), 0.0])
        eu = np.array([-np.sin(b), np.cos(b), 0.0])
        ev = np.array([0.0, 0.0, 1.0])
        D = S + g["sdd_mm"] * a
        for _ in range(40):
            iu, iv = int(rng.integers(g["nu"])), int(rng.integers(g["nv"]))
            # a point well inside the pixel, near its centre
            du = (iu + 0.5 + rng.uniform(-0.3, 0.3)) * g["pu_mm"] - g["nu"] * g["pu_mm"] / 2
            dv = (iv + 0.5 + rng.uniform(-0.3, 0.3)) * g["pv_mm"] - g["nv"] * g["pv_mm"] / 2
            q = D + du * eu + dv * ev
            d = (q - S) / np.linalg.norm(q - S)
            assert o.detector_pixel(b, S, d) == (iu, iv), (beta, iu, iv)
    # moving away from the panel never scores
    assert o.detector_pixel(0.0, [0, 0, 0], [1.0, 0, 0]) == (-1, -1)


def fixed_step_tau(ids, rho, h, mm, p, d, step):
    """Independent fp64 fixed-step optical depth along each ray (p, d are
    [n,3]): entry/exit of the box, steps of `step` with the last one clipped,
    material looked up at each step's nominal centre (k + 1/2) * step,
    clamped to the object."""
    n = np.array(ids.shape[::-1], np.float64)            # nx, ny, nz
    lo, hi = -n * h / 2, n * h / 2
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = (lo - p) / d, (hi - p) / d
    tin = np.maximum(np.nanmax(np.minimum(t1, t2), axis=1), 0)
    tout = np.nanmin(np.maximum(t1, t2), axis=1)
    L = np.maximum(tout - tin, 0)
    kmax = int(np.ceil(L.max() / step)) + 1
    tau = np.zeros(len(p))
    for k in range(kmax):
        a = k * step
        live = a < L
        b = np.minimum(a + step, L)
        s = tin + a + 0.5 * step
        m = p + d * s[:, None]
        idx = np.clip(np.floor((m - lo) / h).astype(np.int64), 0, n.astype(np.int64) - 1)
        mu = rho[idx[:, 2], idx[:, 1], idx[:, 0]] * mm[ids[idx[:, 2], idx[:, 1], idx[:, 0]]]
        tau += np.where(live, mu * (b - a), 0.0)
    return tau


def test_tiny_phantom_primary_brute_force(oracle_lib):
    rng = np.random.default_rng(3)
    ids = rng.integers(0, 5, size=(4, 4, 4)).astype(np.uint8)
    rho = rng.uniform(0.0, 3.0, size=(4, 4, 4)).astype(np.float32)
    h, step = 6.0, 1.0
    o = make(ids, rho, h, nu=8, nv=8, pu_mm=6.0, pv_mm=6.0, step_mm=step)
    counting(o)
    pe, coh, inc, _ = o.tables(5)
    mm = 0.1 * (pe[:, 59].astype(np.float64) + coh[:, 59] + inc[:, 59])
    n = 2_000_000
    p, _ = o.project(0.4, n, seed=8)
    cnt = (p // ONE).astype(np.float64)
    g = o.geometry
    b = float(np.float32(0.4))
    S = g["sod_mm"] * np.array([np.cos(b), np.sin(b), 0.0])
    a = -np.array([np.cos(b), np.sin(b), 0.0])
    eu = np.array([-np.sin(b), np.cos(b), 0.0])
    sub = 24
    u, v = pixel_grid(g, sub)
    uc, vc = 0.5 * (u[1:] + u[:-1]), 0.5 * (v[1:] + v[:-1])
    UC, VC = np.meshgrid(uc, vc)
    q = S + g["sdd_mm"] * a + UC.ravel()[:, None] * eu + VC.ravel()[:, None] * np.array([0, 0, 1.0])
    d = q - S
    d /= np.linalg.norm(d, axis=1)[:, None]
    tau = fixed_step_tau(ids, rho.astype(np.float64), h, mm, np.tile(S, (len(d), 1)), d, step)
    om = omega_pixels(g, sub).ravel()
    exp = (n * om / omega_cone(g) * np.exp(-tau)).reshape(g["nv"], sub, g["nu"], sub).sum(axis=(1, 3))
    zz = (cnt - exp) / np.sqrt(exp)
    assert np.abs(zz).max() < 5, np.abs(zz).max()
    assert abs(chi2_z(np.append(cnt.ravel(), n - cnt.sum()),
                      np.append(exp.ravel(), n - exp.sum()) / n)) < 5


def test_fixed_point_ranges_threads(oracle_lib):
    w = inputs.workload("cylinder64")
    o = oracle.Oracle()
    o.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    o.set_geometry(**w["geometry"])
    o.set_spectrum(*w["spectrum"])
    n = 60_000
    p, s = o.project(0.0, n, seed=0)
    assert np.all(p % (60 * ONE) == 0)                 # eta(60 keV) = 60 exactly
    assert s.sum() > 0
    # ranges add up bitwise
    p2, s2 = o.project_range(0.0, 0, 25_000, seed=0)
    o.project_range(0.0, 25_000, n - 25_000, seed=0, primary=p2, scatter=s2)
    assert np.array_equal(p, p2) and np.array_equal(s, s2)
    # threaded driver: per-thread images summed in a different order
    p3, s3 = o.project(0.0, n, seed=0, threads=7)
    assert np.array_equal(p, p3) and np.array_equal(s, s3)
    # another seed differs
    p4, _ = o.project(0.0, n, seed=1)
    assert not np.array_equal(p, p4)
    # n = 0: empty images
    p5, s5 = o.project(0.0, 0, seed=0)
    assert p5.sum() == 0 and s5.sum() == 0
    # debug records agree with the image
    n_int, steps, end, first = o.debug_histories(0.0, 0, n, seed=0)
    assert (end == oracle.END_PRIMARY).sum() == p.sum() // (60 * ONE)
    assert np.all(n_int[end == oracle.END_PRIMARY] == 0)
    assert np.all(n_int[end == oracle.END_SCATTER] >= 1)
    assert (end == oracle.END_SCATTER).sum() * 60 * ONE >= s.sum() > 0
    assert (end == oracle.END_CAP).sum() == 0


def test_errors(oracle_lib):
    o = oracle.Oracle()
    with pytest.raises(oracle.OracleError) as e:
        o.project(0.0, 10, 0) if o.geometry else o._check(
            o._L.mco_project(o._h, 0.0, 10, 0, None, None))
    ids, rho = inputs.box_phantom(4, 4, 4, 1, 1.0)
    bad = rho.copy(); bad[0, 0, 0] = np.nan
    with pytest.raises(oracle.OracleError):
        o.load_phantom(ids, bad, 1.0)
    with pytest.raises(oracle.OracleError):
        o.set_spectrum([0.5], [1.0])
    with pytest.raises(oracle.OracleError):
        o.set_spectrum([60.0], [0.0])
    with pytest.raises(oracle.OracleError):
        o.set_geometry(sod_mm=500.0, sdd_mm=1000.0, nu=10, nv=10, pu_mm=1, pv_mm=1, snu=3,
                       snv=10, step_mm=0.5)
    o.load_phantom(ids, rho, 1.0)
    o.set_geometry(sod_mm=500.0, sdd_mm=1000.0, nu=10, nv=10, pu_mm=1, pv_mm=1, step_mm=0.5)
    o.set_spectrum([60.0], [1.0])
    with pytest.raises(oracle.OracleError) as e:
        o.project(0.0, 2 ** 63 // (61 * ONE) + 10, 0)
    assert e.value.code == -4
    bad_ids = ids.copy(); bad_ids[1, 1, 1] = 9
    o.load_phantom(bad_ids, rho, 1.0)
    with pytest.raises(oracle.OracleError):
        o.project(0.0, 10, 0)


def test_scatter_binning(oracle_lib):
    """The scatter grid is the detector grid binned in nu/snu x nv/snv blocks."""
    w = inputs.workload("cylinder64")
    res = []
    for snu, snv in [(128, 128), (32, 16)]:
        o = oracle.Oracle()
        o.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
        g = dict(w["geometry"], snu=snu, snv=snv)
        o.set_geometry(**g)
        o.set_spectrum(*w["spectrum"])
        res.append(o.project(0.2, 40_000, seed=4))
    (p1, s1), (p2, s2) = res
    assert np.array_equal(p1, p2)
    assert s1.sum() > 0
    assert np.array_equal(s1.reshape(16, 8, 32, 4).sum(axis=(1, 3)), s2)
