"""Pins of the oracle's samplers against the distributions they must follow.

* Compton (Kahn's method): chi-square of cos(theta) in 100 bins against the
  bin integrals of eq. (1) with S = 1, at several energies including the
  paper's aluminium 100 keV check (Fig. of sampled PDFs, section II-A); mean
  cosine against quadrature; each sample obeys E' = E / (1 + (E/mc^2)(1-cos)).
* Rayleigh: chi-square against (1 + cos^2) F(x,Z)^2 (eq. (2)) bin integrals.
* Spectrum: bin frequencies against the weights (multinomial chi-square).
* Source direction: cos(theta) uniform on [cos(theta_max), 1] (uniform in
  solid angle inside the cone).
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2201_13191_amd import inputs
from test_oracle_xs import kn_dsigma_dcos, rayleigh_dsigma_dcos, MEC2

N = 400_000


def chi2_z(counts, probs):
    n = counts.sum()
    exp = n * probs
    keep = exp > 5
    other_o = counts[~keep].sum()
    other_e = exp[~keep].sum()
    chi2 = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    dof = keep.sum() - 1
    if other_e > 5:
        chi2 += (other_o - other_e) ** 2 / other_e
        dof += 1
    return (chi2 - dof) / np.sqrt(2 * dof)


@pytest.fixture(scope="module")
def orc(oracle_lib):
    o = oracle.Oracle()
    o.set_spectrum(*inputs.mono_spectrum(1000.0))
    return o


@pytest.mark.parametrize("e", [10.0, 60.0, 100.0, 150.0, 500.0, 1000.0])
def test_compton_angles_chi2(orc, e):
    cos, e2 = orc.test_sample(oracle.PROC_COMPTON, 2, e, N, seed=1000 + int(e))
    assert np.all(cos >= -1) and np.all(cos <= 1)
    edges = np.linspace(-1, 1, 101)
    tot = integrate.quad(kn_dsigma_dcos, -1, 1, args=(e,), epsrel=1e-12)[0]
    probs = np.array([integrate.quad(kn_dsigma_dcos, a, b, args=(e,), epsrel=1e-12)[0]
                      for a, b in zip(edges[:-1], edges[1:])]) / tot
    counts = np.histogram(cos.astype(np.float64), edges)[0]
    z = chi2_z(counts, probs)
    assert abs(z) < 5, z
    mean_q = integrate.quad(lambda c: c * kn_dsigma_dcos(c, e), -1, 1, epsrel=1e-12)[0] / tot
    var_q = integrate.quad(lambda c: c * c * kn_dsigma_dcos(c, e), -1, 1)[0] / tot - mean_q ** 2
    assert abs(cos.mean() - mean_q) < 5 * np.sqrt(var_q / N)


@pytest.mark.parametrize("e", [10.0, 100.0, 1000.0])
def test_compton_kinematics(orc, e):
    cos, e2 = orc.test_sample(oracle.PROC_COMPTON, 1, e, 100_000, seed=7)
    ref = e / (1.0 + (e / MEC2) * (1.0 - cos.astype(np.float64)))
    # both outputs are single roundings of one fp64 sample
    rel = np.abs(e2.astype(np.float64) - ref) / ref
    assert rel.max() < 3e-7
    assert np.all(e2 <= np.float32(e)) and np.all(e2 >= e / (1 + 2 * e / MEC2) * (1 - 1e-6))


@pytest.mark.parametrize("mat,e", [(2, 100.0), (1, 30.0), (1, 60.0), (4, 150.0), (0, 5.0),
                                   (3, 1.5)])
def test_rayleigh_angles_chi2(orc, mat, e):
    z = float(np.float32(inputs.DEFAULT_MATERIALS[mat]["z_eff"]))
    cos, e2 = orc.test_sample(oracle.PROC_RAYLEIGH, mat, e, N, seed=99 + mat)
    assert np.all(e2 == np.float32(e))
    # the distribution is peaked forward: bins uniform in (1 - cos)^(1/4)
    t = np.linspace(0, 2 ** 0.25, 101)
    edges = np.unique(1.0 - t ** 4)
    tot = integrate.quad(rayleigh_dsigma_dcos, -1, 1, args=(e, z), epsrel=1e-12,
                         points=[0.99, 0.999, 0.9999], limit=400)[0]
    probs = np.array([integrate.quad(rayleigh_dsigma_dcos, a, b, args=(e, z),
                                     epsrel=1e-12, limit=200)[0]
                      for a, b in zip(edges[:-1], edges[1:])]) / tot
    counts = np.histogram(cos.astype(np.float64), edges)[0]
    z_ = chi2_z(counts, probs)
    assert abs(z_) < 5, z_


def test_spectrum_multinomial(oracle_lib):
    o = oracle.Oracle()
    e, w = inputs.kramers_spectrum(150, 2.0)
    o.set_spectrum(e, w)
    _, es = o.test_sample(oracle.PROC_SOURCE_ENERGY, 0, 0.0, N, seed=3)
    idx = np.searchsorted(e, es)
    assert np.all(e[idx] == es)
    counts = np.bincount(idx, minlength=len(e))
    probs = w.astype(np.float64) / w.astype(np.float64).sum()
    assert counts[probs == 0].sum() == 0
    assert abs(chi2_z(counts, probs)) < 5


def test_source_cone_uniform(oracle_lib):
    o = oracle.Oracle()
    o.set_spectrum(*inputs.mono_spectrum(60.0))
    ids, rho = inputs.cylinder_phantom(8, 1.0)
    o.load_phantom(ids, rho, 1.0)
    o.set_geometry(sod_mm=500.0, sdd_mm=1000.0, nu=128, nv=96, pu_mm=1.0, pv_mm=1.0,
                   step_mm=0.5)
    cos, _ = o.test_sample(oracle.PROC_SOURCE_DIR, 0, 0.0, N, seed=5)
    ctm = 1000.0 / np.sqrt(1000.0 ** 2 + 64.0 ** 2 + 48.0 ** 2)
    c = cos.astype(np.float64)
    assert c.min() >= np.float32(ctm) - 1e-7 and c.max() <= 1.0
    counts = np.histogram((1 - c) / (1 - ctm), np.linspace(0, 1, 51))[0]
    assert abs(chi2_z(counts, np.full(50, 1 / 50))) < 5
