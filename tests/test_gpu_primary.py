"""GPU parity of the deterministic primary of eq. (7) and of the angular
interpolation (section II-C-3) against the oracle.

The primary kernel follows the oracle's sums in the same order (fp64 path
lengths and spectrum sum, the transport's fp32 step centres) and rounds once
to fp32: the bar is 1e-6 relative per pixel.  The interpolation is bitwise.
The GPU's Monte Carlo primary must also scatter around n times the
deterministic image within Poisson noise.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    mcx.load()
    return torch


def _det(torch, g, geo, angle, sub):
    out = torch.full((geo["nv"], geo["nu"]), -1.0, dtype=torch.float32, device="cuda:0")
    mcx.mc_primary_expected_async(g.ctx, angle, sub, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("case", ["cylinder64", "random_generic", "ellipsoids256_poly"])
def test_primary_matches_oracle(gpu, case):
    torch = gpu
    if case == "cylinder64":
        w = inputs.workload("cylinder64")
        ids, rho, h, geo, spec, sub, angle = (w["ids"], w["rho"], w["voxel_mm"], w["geometry"],
                                              inputs.kramers_spectrum(100, 1.0), 3, 0.6)
    elif case == "random_generic":
        rng = np.random.default_rng(7)
        ids = rng.integers(0, 5, size=(20, 22, 18)).astype(np.uint8)
        rho = rng.uniform(0.0, 3.0, size=ids.shape).astype(np.float32)
        h, sub, angle = 2.5, 2, 2.2
        geo = dict(sod_mm=250.0, sdd_mm=500.0, nu=40, nv=36, pu_mm=3.0, pv_mm=3.0, step_mm=1.1,
                   flags=0)
        spec = inputs.kramers_spectrum(130, 2.0)
    else:
        w = inputs.workload("ellipsoids256_poly")
        ids, rho, h, geo, spec, sub, angle = (w["ids"], w["rho"], w["voxel_mm"], w["geometry"],
                                              w["spectrum"], 1, 0.0)
    o, g = pair(ids, rho, h, geo, spec)
    say("eq. (7) primary", case, "sub", sub)
    d = _det(torch, g, geo, angle, sub)
    ref = o.primary_expected(angle, sub)
    rel = np.abs(d / ref - 1)
    say(case, f"max relative difference {rel.max():.2e}, bitwise-fp32 "
              f"{int((d == ref.astype(np.float32)).sum())} of {d.size}")
    assert ref.min() > 0 and rel.max() <= 1e-6, rel.max()
    g.close()


def test_primary_is_the_monte_carlo_expectation(gpu):
    torch = gpu
    ids, rho = inputs.ellipsoid_phantom(40, 1.5, seed=12)
    geo = dict(sod_mm=300.0, sdd_mm=600.0, nu=32, nv=32, pu_mm=4.0, pv_mm=4.0, step_mm=0.6,
               flags=0)
    g = mcx.Projector(0)
    g.load_phantom(ids, rho, 1.5)
    g.set_geometry(**geo)
    g.set_spectrum(*inputs.kramers_spectrum(120, 2.0))
    g.set_detector_response(np.ones(200, np.float32))      # counting: Poisson counts
    # 16 x 16 rays per pixel: the pixels an ellipsoid's edge crosses need a fine
    # rule before its error drops below the Monte Carlo noise of n photons
    det = _det(torch, g, geo, 0.9, 16)
    n = 20_000_000
    say("Monte Carlo primary against eq. (7)", n)
    p, _ = g.project(0.9, n, 3)
    counts = p.astype(np.float64) / 2 ** 20
    exp = n * det
    z = (counts - exp) / np.sqrt(exp)
    say(f"max |z| {np.abs(z).max():.2f}, total ratio {counts.sum() / exp.sum():.6f}")
    assert np.abs(z).max() < 5.5
    assert abs(counts.sum() / exp.sum() - 1) < 5 / np.sqrt(exp.sum())
    g.close()


def test_interp_angles_bitwise(gpu):
    torch = gpu
    rng = np.random.default_rng(5)
    sim = rng.uniform(0, 10, size=(45, 33, 17)).astype(np.float32)
    g = mcx.Projector(0)
    d_sim = torch.from_numpy(sim).cuda()
    d_full = torch.full((90, 33, 17), -1.0, dtype=torch.float32, device="cuda:0")
    say("interpolation of every other angle")
    mcx.mc_interp_angles_async(g.ctx, d_sim, 45, 33 * 17, d_full)
    torch.cuda.synchronize()
    assert np.array_equal(d_full.cpu().numpy(), oracle.interp_angles(sim))
    g.close()
