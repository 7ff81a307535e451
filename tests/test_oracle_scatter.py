"""Pins of the oracle's scatter side: the direction update, the free path to
an interaction, and the single-scatter image.

* Rotation after a scattering (section II-A: the polar angle from eq. (1) or
  (2), the azimuth uniform): the new direction is a unit vector at the
  sampled polar angle to the old one, and the azimuth about the old direction
  is the drawn azimuth up to a constant offset (a rotation of the circle), so
  a uniform draw stays uniform -- in the general branch and in the one for
  directions within 0.26 degrees of the z axis.
* Free path: in a homogeneous block the distance from the entry point to the
  first interaction follows the exponential law, truncated at the chord:
  F(s) = (1 - exp(-mu s)) / (1 - exp(-mu L)).  The probability-integral
  transform of every sampled distance is uniform (Kolmogorov-Smirnov), with
  a march step comparable to the mean free path, so a point placed anywhere
  but its exact place inside the step fails.
* Single scatter: on a thin homogeneous block close to a large panel, the
  image of photons that scattered exactly once and then crossed the panel is
  compared with an fp64 integral over the block and the panel written from
  first principles: the source's photons per steradian, attenuation
  exp(-mu s) to the interaction point, the interaction fractions of the
  tables, the angular laws of eq. (1) (Klein-Nishina, S = 1) and eq. (2)
  (with the screened form factor) normalised by quadrature, the Compton
  energy relation, attenuation at the scattered energy to the block's exit,
  and the pixel's solid angle cos(gamma) dA / R^2.  Counts and energy are
  both checked (per-pixel z, chi-square, totals).
"""
import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from paper_2201_13191_amd import inputs
from test_oracle_samplers import chi2_z
from test_oracle_xs import MEC2, kn_dsigma_dcos, rayleigh_dsigma_dcos


def _frame(d):
    """An orthonormal pair (e1, e2) perpendicular to the unit vector d."""
    t = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(d, t)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(d, e1)


def _azimuth(d, dn):
    e1, e2 = _frame(d)
    return np.arctan2(dn @ e2, dn @ e1)


def _random_unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def _near_pole(rng, n):
    """Unit vectors with |d_z| >= 0.99999 (the pole branch of the update)."""
    out = []
    for _ in range(n):
        dz = rng.uniform(0.99999, 1.0) * rng.choice([-1.0, 1.0])
        ang = rng.uniform(0, 2 * np.pi)
        s = np.sqrt(1 - dz * dz)
        out.append([s * np.cos(ang), s * np.sin(ang), dz])
    out.append([0.0, 0.0, 1.0])
    out.append([0.0, 0.0, -1.0])
    return np.array(out)


@pytest.mark.parametrize("branch", ["general", "pole"])
def test_rotation_invariants(oracle_lib, branch):
    rng = np.random.default_rng(17 if branch == "general" else 18)
    dirs = _random_unit(rng, 300) if branch == "general" else _near_pole(rng, 300)
    if branch == "general":
        dirs = dirs[np.abs(dirs[:, 2]) < 0.999]
    # fp32 rounding divided by sqrt(1 - d_z^2) in the general branch; the pole
    # branch takes (0, 0, +-1) as the old direction: the angle to the
    # true one is at most asin(sqrt(1 - 0.99999^2)) = 4.5e-3
    tol = 2e-5 if branch == "general" else 5e-3
    phis = np.linspace(0.0, 2 * np.pi, 13)[:-1] + 0.1
    for d in dirs:
        d32 = d.astype(np.float32)
        dd = d32.astype(np.float64)
        dd /= np.linalg.norm(dd)
        for ct in rng.uniform(-1, 1, 3).tolist() + [0.0, 0.999]:
            ct = float(np.float32(ct))
            outs = np.array([oracle.rotate(d32, ct, phi).astype(np.float64) for phi in phis])
            assert np.all(np.abs(np.linalg.norm(outs, axis=1) - 1) < 1e-6)
            assert np.all(np.abs(outs @ dd - ct) < tol), (d, ct, outs @ dd)
            if abs(ct) > 0.99:
                continue
            # azimuth = +-phi + const: consecutive differences are all +step or all -step
            psi = np.array([_azimuth(dd, o) for o in outs])
            step = phis[1] - phis[0]
            dpsi = np.angle(np.exp(1j * np.diff(psi)))
            atol = 1e-4 if branch == "general" else 2e-2
            ok_plus = np.allclose(dpsi, step, atol=atol)
            ok_minus = np.allclose(dpsi, -step, atol=atol)
            assert ok_plus or ok_minus, (d, ct, dpsi)


def test_rotation_azimuth_uniform(oracle_lib):
    """Uniform azimuth draws give azimuths uniform about the old direction
    (chi-square in 36 bins), for a direction in each branch."""
    rng = np.random.default_rng(5)
    for d in (np.array([0.3, -0.5, 0.81]), np.array([0.0, 0.0, -1.0])):
        d = d / np.linalg.norm(d)
        d32 = d.astype(np.float32)
        psi = np.array([_azimuth(d, oracle.rotate(d32, 0.2, phi).astype(np.float64))
                        for phi in rng.uniform(0, 2 * np.pi, 20_000)])
        counts = np.histogram(psi, np.linspace(-np.pi, np.pi, 37))[0]
        assert abs(chi2_z(counts, np.full(36, 1 / 36))) < 5


def _box_t(p, d, lo, hi):
    """Slab-method entry and exit parameters of rays p + t d (fp64)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - p) / d
        t2 = (hi - p) / d
    return (np.nanmax(np.minimum(t1, t2), axis=-1), np.nanmin(np.maximum(t1, t2), axis=-1))


def test_free_path_exponential(oracle_lib):
    # aluminium block 40 mm on a side at 2.699 g/cm^3, 60 keV: mean free path
    # ~13 mm, march step 1.5 mm
    n_vox, h, step = 20, 2.0, 1.5
    ids, rho = inputs.box_phantom(n_vox, n_vox, n_vox, 2, 2.699)
    o = oracle.Oracle()
    o.load_phantom(ids, rho, h)
    g = dict(sod_mm=300.0, sdd_mm=600.0, nu=32, nv=32, pu_mm=2.0, pv_mm=2.0, step_mm=step)
    o.set_geometry(**g)
    o.set_spectrum(*inputs.mono_spectrum(60.0))
    pe, coh, inc, _ = o.tables(5)
    mu = 2.699 * 0.1 * (float(pe[2, 59]) + float(coh[2, 59]) + float(inc[2, 59]))
    x1, _, _ = o.debug_paths(0.0, 0, 200_000, seed=12)
    x1 = x1[~np.isnan(x1[:, 0])].astype(np.float64)
    assert len(x1) > 50_000
    S = np.array([g["sod_mm"], 0.0, 0.0])
    r = x1 - S
    dist = np.linalg.norm(r, axis=1)
    w = r / dist[:, None]
    half = n_vox * h / 2
    tin, tout = _box_t(np.broadcast_to(S, w.shape), w, -half, half)
    s = dist - tin
    L = tout - tin
    assert np.all(s >= -1e-3) and np.all(s <= L + 1e-3)
    u = -np.expm1(-mu * s) / -np.expm1(-mu * L)
    ks = stats.kstest(u, "uniform")
    assert ks.pvalue > 1e-4, ks
    # and the mean of the (truncated) free path
    mean_th = 1 / mu - L * np.exp(-mu * L) / -np.expm1(-mu * L)
    var_th = 2 / mu ** 2 - (L * L + 2 * L / mu) * np.exp(-mu * L) / -np.expm1(-mu * L) - mean_th ** 2
    assert abs(s.mean() - mean_th.mean()) < 5 * np.sqrt(var_th.mean() / len(s))


def _gauss(a, b, n, m):
    """Composite Gauss-Legendre nodes and weights: m panels of n nodes on [a, b]."""
    x, w = np.polynomial.legendre.leggauss(n)
    edges = np.linspace(a, b, m + 1)
    xs = [(x + 1) * (r - l) / 2 + l for l, r in zip(edges[:-1], edges[1:])]
    ws = [w * (r - l) / 2 for l, r in zip(edges[:-1], edges[1:])]
    return np.concatenate(xs), np.concatenate(ws)


# water block 16 mm on a side, 20 mm from the source, 20 mm in front of an
# 80 mm panel of 16 x 16 pixels: the panel subtends ~3.7 sr from the block
SS_GEO = dict(sod_mm=20.0, sdd_mm=40.0, nu=16, nv=16, pu_mm=5.0, pv_mm=5.0, step_mm=0.5)
SS_RHO, SS_E, SS_Z = 1.0, 60.0, 7.42


def single_scatter_expectation(pe, coh, inc, n_box=6, n_pix=3, panels=2):
    """Expected single-scatter counts and energy per photon emitted into the
    cone, per pixel [v][u], by fp64 quadrature over the block and the panel."""
    g = SS_GEO
    tot = pe[1].astype(np.float64) + coh[1] + inc[1]

    def lerp(t, e):
        e = np.asarray(e, np.float64)
        j = np.floor(e - 1).astype(int)
        f = (e - 1) - j
        return t[j] + f * (t[j + 1] - t[j])

    def mu_of(e):
        return SS_RHO * 0.1 * lerp(tot, e)

    mu0 = float(mu_of(SS_E))
    f_comp = SS_RHO * 0.1 * float(lerp(inc[1].astype(np.float64), SS_E)) / mu0
    f_rayl = SS_RHO * 0.1 * float(lerp(coh[1].astype(np.float64), SS_E)) / mu0
    sig_c = integrate.quad(kn_dsigma_dcos, -1, 1, args=(SS_E,), epsrel=1e-12)[0]
    sig_r = integrate.quad(rayleigh_dsigma_dcos, -1, 1, args=(SS_E, SS_Z), epsrel=1e-12,
                           limit=200)[0]
    S = np.array([g["sod_mm"], 0.0, 0.0])
    a = np.array([-1.0, 0.0, 0.0])
    eu, ev = np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])
    D = S + g["sdd_mm"] * a
    half = 8.0
    bx, bw = _gauss(-half, half, n_box, panels)
    X, Y, Z = np.meshgrid(bx, bx, bx, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    wx = np.einsum("i,j,k->ijk", bw, bw, bw).ravel()
    r = x - S
    rn = np.linalg.norm(r, axis=1)
    w0 = r / rn[:, None]
    tin, _ = _box_t(np.broadcast_to(S, x.shape), w0, -half, half)
    hu, hv = g["nu"] * g["pu_mm"] / 2, g["nv"] * g["pv_mm"] / 2
    om_cone = 2 * np.pi * (1 - g["sdd_mm"] / np.sqrt(g["sdd_mm"] ** 2 + hu * hu + hv * hv))
    # first interactions per unit volume per emitted photon
    fx = wx * mu0 * np.exp(-mu0 * (rn - tin)) / rn ** 2 / om_cone
    px, pw = np.polynomial.legendre.leggauss(n_pix)
    ww = np.outer(pw, pw).ravel() * (g["pu_mm"] / 2) * (g["pv_mm"] / 2)
    cnt = np.zeros((g["nv"], g["nu"]))
    en = np.zeros_like(cnt)
    for iv in range(g["nv"]):
        for iu in range(g["nu"]):
            u = -hu + iu * g["pu_mm"] + (px + 1) * g["pu_mm"] / 2
            v = -hv + iv * g["pv_mm"] + (px + 1) * g["pv_mm"] / 2
            U, V = np.meshgrid(u, v, indexing="xy")
            y = D + U.ravel()[:, None] * eu + V.ravel()[:, None] * ev
            R = y[None, :, :] - x[:, None, :]
            Rn = np.linalg.norm(R, axis=2)
            om = R / Rn[..., None]
            d_omega = (om @ a) * ww[None, :] / Rn ** 2
            ct = np.einsum("ia,ija->ij", w0, om)
            e_c = SS_E / (1 + SS_E / MEC2 * (1 - ct))
            _, tout = _box_t(np.broadcast_to(x[:, None, :], R.shape), om, -half, half)
            p_c = kn_dsigma_dcos(ct, SS_E) / (2 * np.pi) / sig_c
            p_r = rayleigh_dsigma_dcos(ct, SS_E, SS_Z) / (2 * np.pi) / sig_r
            comp = f_comp * p_c * np.exp(-mu_of(e_c) * tout)
            rayl = f_rayl * p_r * np.exp(-mu0 * tout)
            cnt[iv, iu] = np.sum(fx[:, None] * (comp + rayl) * d_omega)
            en[iv, iu] = np.sum(fx[:, None] * (comp * e_c + rayl * SS_E) * d_omega)
    return cnt, en


def test_single_scatter_brute_force(oracle_lib):
    ids, rho = inputs.box_phantom(8, 8, 8, 1, SS_RHO)
    o = oracle.Oracle()
    o.load_phantom(ids, rho, 2.0)
    o.set_geometry(**SS_GEO)
    o.set_spectrum(*inputs.mono_spectrum(SS_E))
    pe, coh, inc, _ = o.tables(5)
    cnt, en = single_scatter_expectation(pe, coh, inc)
    n = 4_000_000
    n_int, _, end, _ = o.debug_histories(0.0, 0, n, seed=3)
    _, pix, e_end = o.debug_paths(0.0, 0, n, seed=3)
    once = (n_int == 1) & (end == oracle.END_SCATTER)
    assert np.all(pix[once] >= 0)
    img = np.bincount(pix[once], minlength=256).reshape(16, 16).astype(np.float64)
    eimg = np.bincount(pix[once], weights=e_end[once].astype(np.float64),
                       minlength=256).reshape(16, 16)
    exp = n * cnt
    assert exp.sum() > 50_000
    assert abs(img.sum() - exp.sum()) < 4 * np.sqrt(exp.sum()), (img.sum(), exp.sum())
    z = (img - exp) / np.sqrt(exp)
    assert np.abs(z).max() < 5, np.abs(z).max()
    assert abs(chi2_z(np.append(img.ravel(), n - img.sum()),
                      np.append(exp.ravel(), n - exp.sum()) / n)) < 5
    # energy image: the sum of scattered energies per pixel; its spread is the
    # count's Poisson spread times the expected mean energy there
    e_exp = n * en
    ze = (eimg - e_exp) / (np.sqrt(exp) * (en / cnt))
    assert np.abs(ze).max() < 5, np.abs(ze).max()
    assert abs(eimg.sum() / e_exp.sum() - 1) < 4 / np.sqrt(exp.sum())
