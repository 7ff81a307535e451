"""The reconstruction side of the iterative scatter correction (section II-E,
its flowchart and eq. (8)) on the GPU against the oracle (oracle/recon.py),
and the whole loop on a small scan: one correction pass must bring the
reconstruction closer to the scatter-free one.

Tolerances: the kernels compute in fp64 and store fp32, so each stored value
is the oracle's fp64 result rounded once (rel 2^-24), up to fp64 summation
order.  The backprojection sums fp32-stored filtered values q over angles,
so its error is bounded by 2^-24 times the sum of |terms|, itself at most
pi * max|q| * max(R^2 / L^2) (the weights 1/2 (2 pi / n) sum over n angles).
"""
import math

import numpy as np
import pytest

from oracle import recon
from paper_2201_13191_amd import correction, inputs, mcx
from test_gpu_parity import say

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    return torch


def _ctx(geo):
    g = mcx.Projector(0)
    g.set_geometry(**geo)
    return g


GEO = dict(sod_mm=300.0, sdd_mm=520.0, nu=45, nv=38, pu_mm=2.5, pv_mm=2.2, snu=45, snv=38,
           step_mm=1.0, flags=0)
# the library holds geometry and voxel size as fp32: the oracle gets the same values
GEO32 = {k: (float(np.float32(v)) if isinstance(v, float) else v) for k, v in GEO.items()}


def _ball_projections(n_ang, geo, centre, radius, mu):
    """Exact line integrals of a uniform ball through each pixel centre."""
    R, D = geo["sod_mm"], geo["sdd_mm"]
    nu, nv, pu, pv = geo["nu"], geo["nv"], geo["pu_mm"], geo["pv_mm"]
    u = -nu * pu / 2 + (np.arange(nu) + 0.5) * pu
    v = -nv * pv / 2 + (np.arange(nv) + 0.5) * pv
    out = np.zeros((n_ang, nv, nu))
    c = np.asarray(centre, np.float64)
    for i in range(n_ang):
        b = 2 * math.pi * i / n_ang
        S = np.array([R * math.cos(b), R * math.sin(b), 0.0])
        ax = -S / R
        eu = np.array([-math.sin(b), math.cos(b), 0.0])
        U_, V_ = np.meshgrid(u, v, indexing="xy")
        P = S + D * ax + U_[..., None] * eu + V_[..., None] * np.array([0, 0, 1.0])
        d = P - S
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        m = S - c
        bq = np.sum(d * m, axis=-1)
        disc = bq * bq - (np.dot(m, m) - radius * radius)
        out[i] = mu * 2.0 * np.sqrt(np.maximum(disc, 0.0))
    return out.astype(np.float32)


def test_line_integrals_and_eq8():
    torch = _torch()
    rng = np.random.default_rng(11)
    n_ang = 5
    I0 = rng.uniform(0.5, 2.0, (GEO["nv"], GEO["nu"])).astype(np.float32)
    I = (I0[None] * rng.uniform(1e-3, 1.0, (n_ang,) + I0.shape)).astype(np.float32)
    I[0, 0, :4] = 0.0                                   # dead pixels clamp to 1e-30
    ip = rng.uniform(1e-3, 1.0, I.shape).astype(np.float32)
    is_ = rng.uniform(0.0, 0.5, I.shape).astype(np.float32)
    g = _ctx(GEO)
    d = {k: torch.from_numpy(v).cuda() for k, v in dict(I=I, I0=I0, ip=ip, is_=is_).items()}
    a = torch.empty_like(d["I"])
    c = torch.empty_like(d["I"])
    say("line integrals and eq. (8)", I.shape)
    mcx.mc_line_integrals_async(g.ctx, d["I"], d["I0"], a)
    mcx.mc_scatter_correct_async(g.ctx, a, d["ip"], d["is_"], c)
    torch.cuda.synchronize()
    a_o = recon.line_integrals(I, I0[None])
    c_o = recon.scatter_correct(a.cpu().numpy(), ip, is_)
    np.testing.assert_allclose(a.cpu().numpy(), a_o, rtol=2 * U, atol=1e-12)
    np.testing.assert_allclose(c.cpu().numpy(), c_o, rtol=2 * U, atol=1e-12)
    g.close()


@pytest.mark.parametrize("n_ang,vol", [(24, (20, 26, 30)), (7, (9, 11, 13))])
def test_fdk_matches_oracle(n_ang, vol):
    """Ball projections plus noise (ragged volume and panel sizes): the
    filtered projections (the library's d_tmp), the backprojection of those
    same values, and the whole FDK against the oracle."""
    torch = _torch()
    rng = np.random.default_rng(n_ang)
    proj = _ball_projections(n_ang, GEO, (6.0, -4.0, 3.0), 18.0, 0.02)
    proj += rng.normal(0, 0.01, proj.shape).astype(np.float32)
    h = float(np.float32(2.3))
    g = _ctx(GEO)
    d_p = torch.from_numpy(proj).cuda()
    d_q = torch.empty_like(d_p)
    d_v = torch.empty(vol, dtype=torch.float32, device="cuda")
    say("fdk", n_ang, vol)
    mcx.mc_fdk_async(g.ctx, d_p, d_q, d_v, h)
    torch.cuda.synchronize()
    q_o = recon.fdk_filter(proj, GEO32)
    q_g = d_q.cpu().numpy()
    np.testing.assert_allclose(q_g, q_o, rtol=2 * U, atol=1e-12 * np.abs(q_o).max())
    R = GEO["sod_mm"]
    rmax = 0.5 * h * math.hypot(vol[1], vol[2])
    bound = math.pi * np.abs(q_o).max() * (R / (R - rmax)) ** 2
    v_g = d_v.cpu().numpy()
    v_bp = recon.fdk_backproject(q_g, GEO32, vol, h)      # same fp32 q: order and final rounding
    np.testing.assert_allclose(v_g, v_bp, rtol=2 * U, atol=1e-12 * bound)
    v_o = recon.fdk(proj, GEO32, vol, h)
    np.testing.assert_allclose(v_g, v_o, rtol=2 * U, atol=2 * U * bound)
    g.close()


def test_fdk_reconstructs_offset_ball():
    """Orientation check on an object off the axis: the FDK of the library's
    own Monte Carlo primary of a water ball (radius 8 mm at (14, -9, 11) mm)
    puts the ball where the phantom has it -- FDK and projector agree on the
    orbit's direction and the panel's axes.  Around the true centre the mean
    attenuation is water's at 60 keV; around each of the seven mirror images
    of the centre it is that of air."""
    torch = _torch()
    n, h = 40, 2.0
    c = (np.arange(n) + 0.5) * h - n * h / 2
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    cen = np.array([14.0, -9.0, 11.0])
    ball = (X - cen[0]) ** 2 + (Y - cen[1]) ** 2 + (Z - cen[2]) ** 2 <= 8.0 ** 2
    ids = ball.astype(np.uint8)
    rho = np.where(ball, 1.0, 0.0).astype(np.float32)
    geo = dict(sod_mm=300.0, sdd_mm=600.0, nu=96, nv=96, pu_mm=2.0, pv_mm=2.0, snu=24, snv=24,
               step_mm=h, flags=0)
    spec = inputs.mono_spectrum(60.0)
    obj = correction.make_context(geo, spec, ids, rho, h)
    air = correction.make_context(geo, spec, np.zeros_like(ids), np.zeros_like(rho), h)
    try:
        stream = torch.cuda.current_stream()
        n_ang = 90
        say("fdk of an offset ball from the Monte Carlo primary", n_ang)
        p, _ = correction.project(obj, range(n_ang), n_ang, 10_000_000, 3, stream)
        I0 = torch.empty((geo["nv"], geo["nu"]), dtype=torch.float32, device="cuda")
        mcx.mc_primary_expected_async(air.ctx, 0.0, 2, I0, stream)
        a = torch.empty_like(p)
        mcx.mc_line_integrals_async(obj.ctx, p.contiguous(), I0, a, stream)
        v = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        mcx.mc_fdk_async(obj.ctx, a, torch.empty_like(a), v, h, stream)
        torch.cuda.synchronize()
        vh = v.cpu().numpy().astype(np.float64)
        pe, coh, inc, _ = mcx.mc_get_tables(obj.ctx, 2)
        mu_w = 0.1 * float(pe[1][59] + coh[1][59] + inc[1][59])  # per mm at 60 keV (grid 1 + j)
    finally:
        obj.close()
        air.close()
    means = {}
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                m = (X - sx * cen[0]) ** 2 + (Y - sy * cen[1]) ** 2 + (Z - sz * cen[2]) ** 2 <= 25
                means[(sx, sy, sz)] = float(vh[m].mean()) / mu_w
    say("mean attenuation / water's around the centre and its mirror images", means)
    # noise of a 70-voxel mean here: about 1 % of water's attenuation
    assert abs(means[(1, 1, 1)] - 1.0) < 0.06
    assert all(abs(x) < 0.1 for k, x in means.items() if k != (1, 1, 1))


def test_histogram_otsu_density_bitwise():
    torch = _torch()
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(0.002, 0.001, 30001), rng.normal(0.021, 0.002, 17777)])
    x = x.astype(np.float32).reshape(-1)
    lo, hi = float(np.float32(x.min())), float(np.float32(x.max() * 1.0001))
    g = _ctx(GEO)
    d_x = torch.from_numpy(x).cuda()
    hist = torch.empty(256, dtype=torch.int32, device="cuda")
    say("histogram and density", x.size)
    mcx.mc_histogram_async(g.ctx, d_x, lo, hi, 256, hist)
    torch.cuda.synchronize()
    h_g = hist.cpu().numpy()
    h_o = recon.histogram(x, lo, hi, 256)
    assert np.array_equal(h_g.astype(np.int64), h_o)
    # the product's Otsu split (vectorised) equals the oracle's loop
    thr = correction.otsu_threshold(h_g, lo, hi)
    t = recon.otsu_bin(h_o)
    assert thr == lo + (hi - lo) * t / 256
    thr32 = float(np.float32(thr))
    mu_rho = float(np.float32(0.2059))
    ids = torch.empty(x.shape, dtype=torch.uint8, device="cuda")
    rho = torch.empty(x.shape, dtype=torch.float32, device="cuda")
    mcx.mc_to_density_async(g.ctx, d_x, thr32, mu_rho, 1, float(np.float32(0.02)), ids, rho)
    torch.cuda.synchronize()
    ids_o, rho_o = recon.to_density(x, thr32, mu_rho, 1, air_rho=float(np.float32(0.001205)),
                                    step=float(np.float32(0.02)))
    assert np.array_equal(ids.cpu().numpy(), ids_o)
    assert np.array_equal(rho.cpu().numpy(), rho_o)
    g.close()


def test_correction_loop_reduces_error():
    """A small scan (32^3 ellipsoids, 60 angles): one pass of the loop with
    the scatter estimated on a 4x coarser grid brings the reconstruction
    closer to the scatter-free one (lower MSE, higher NCC)."""
    _torch()
    args = correction.parse(["--size", "32", "--voxel-mm", "3", "--panel", "64",
                             "--pixel-mm", "4", "--angles", "60", "--n-measured", "20000000",
                             "--n-estimate", "2000000", "--iterations", "1"])
    say("correction loop", vars(args))
    res = correction.run(args)
    u, c = res["uncorrected"], res["iterations"][0]
    say("uncorrected", u, "corrected", c)
    assert all(np.isfinite(list(c.values())))
    assert c["mse"] < u["mse"] and c["ncc"] > u["ncc"]
    # the scatter's low-frequency error (cupping, lowered attenuation) shrinks
    assert c["rel_l2_smooth"] < u["rel_l2_smooth"]
    assert abs(c["mean_ratio"] - 1) < abs(u["mean_ratio"] - 1)
