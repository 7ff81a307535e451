"""GPU parity of the point-detector scatter estimator (eq. (3)-(5), splitting
and Russian roulette of section II-C-1) against the oracle's.

Both sides follow the same arithmetic; the angular laws' normalisations are
evaluated differently (the oracle in extended precision, the GPU by a Taylor
series or the fp64 closed form), so a score can differ by one least
significant bit of its Q43.20 tally in rare cases.  The bar: scatter images
within rel-L2 1e-9 (the tolerance of the transport is 5e-3), pseudo-particle
counts (scored, killed by roulette, chord steps) equal, and the primary image
bitwise equal to the analog run's.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import check_images, pair, rel_l2, say

pytestmark = pytest.mark.gpu

PD_REL = 1e-9


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    mcx.load()
    return torch


MODES = [(oracle.SCORE_POINT, mcx.MC_SCORE_POINT), (oracle.SCORE_POINT_MIXED, mcx.MC_SCORE_POINT_MIXED)]


def _run(name, ids, rho, h, geo, spec, n, seed, split, rr, angle=0.3, layout=None,
         modes=MODES[0]):
    o, g = pair(ids, rho, h, geo, spec)
    if layout is not None:
        g.set_layout(layout)
        g.load_phantom(ids, rho, h)
    say(name, "analog GPU")
    pa, sa = g.project(angle, n, seed)
    for side, mode in zip((o, g), modes):
        side.set_estimator(mode, split, rr)
    say(name, f"estimator {modes[1]} split {split} rr {rr}, {n} photons")
    g.stats(True)
    pg, sg = g.project(angle, n, seed)
    st_g = g.stats()
    g.stats(False)
    o.stats()
    po, so = o.project(angle, n, seed, threads=8)
    st_o = o.stats()
    r = rel_l2(sg, so)
    say(name, f"scatter rel-L2 {r:.3e}, differing bins {int((sg != so).sum())}, "
              f"scores {st_g['pd_scores']} / {st_o['pd_scores']}, killed {st_g['pd_killed']}, "
              f"chord steps {st_g['pd_steps']}")
    assert np.array_equal(pg, pa), name                 # primary unchanged by the scorer
    assert np.array_equal(pg, po), name
    assert so.sum() > 0 and r <= PD_REL, (name, r)
    assert st_g["pd_scores"] == st_o["pd_scores"], name
    assert st_g["pd_killed"] == st_o["pd_killed"], name
    assert st_g["pd_steps"] == st_o["pd_steps"], name
    g.close()
    return sg, so


@pytest.mark.parametrize("modes", MODES, ids=["point", "mixed"])
def test_pd_cylinder(gpu, modes):
    w = inputs.workload("cylinder64")
    _run("cylinder64", w["ids"], w["rho"], w["voxel_mm"], w["geometry"], w["spectrum"],
         100_000, 0, 4, 0.0, modes=modes)


@pytest.mark.parametrize("modes", MODES, ids=["point", "mixed"])
@pytest.mark.parametrize("layout", [mcx.MC_LAYOUT_PALETTE_LANE, mcx.MC_LAYOUT_PALETTE_SHARED,
                                    mcx.MC_LAYOUT_GENERIC])
def test_pd_layouts_with_roulette(gpu, layout, modes):
    ids, rho = inputs.ellipsoid_phantom(48, 1.0, seed=31)
    geo = dict(sod_mm=300.0, sdd_mm=600.0, nu=64, nv=48, pu_mm=2.0, pv_mm=2.0, snu=16, snv=12,
               step_mm=0.7, flags=0)
    _run(f"ellipsoids48 layout {layout}", ids, rho, 1.0, geo, inputs.kramers_spectrum(120, 2.0),
         60_000, 5, 6, 0.02, layout=layout, modes=modes)


def test_pd_long_steps_and_iron(gpu):
    """Steps longer than a voxel (clamped gathers), an iron insert, low energies
    (Compton normalisation below a = 0.1 by the series), Rayleigh-heavy."""
    ids, rho = inputs.ellipsoid_phantom(40, 1.0, seed=8, materials=(1, 2, 3), iron_insert=True)
    geo = dict(sod_mm=200.0, sdd_mm=400.0, nu=40, nv=40, pu_mm=4.0, pv_mm=4.0, snu=10, snv=10,
               step_mm=1.7, flags=0)
    for modes in MODES:
        _run("iron, long steps", ids, rho, 1.0, geo, inputs.kramers_spectrum(60, 0.5), 50_000, 9,
             3, 0.0, angle=1.1, modes=modes)


def test_pd_full_size_subrange(gpu):
    """The 256^3 benchmark object and panel: a photon sub-range in the middle of
    the id range, split 8, against the oracle's image of the same photons."""
    torch = gpu
    w = inputs.workload("ellipsoids256_poly")
    o, g = pair(w["ids"], w["rho"], w["voxel_mm"], w["geometry"], w["spectrum"])
    for side, mode in zip((o, g), MODES[1]):
        side.set_estimator(mode, 8, 0.0)
    geo = w["geometry"]
    a, m = 50_000_123, 20_000
    say("256^3 point detector sub-range", a, m)
    p = torch.zeros((geo["nv"], geo["nu"]), dtype=torch.int64, device="cuda:0")
    s = torch.zeros((geo["snv"], geo["snu"]), dtype=torch.int64, device="cuda:0")
    mcx.mc_project_range_async(g.ctx, w["angle"], a, m, w["seed"], p, s)
    torch.cuda.synchronize()
    po, so = o.project_range(w["angle"], a, m, w["seed"])
    r = rel_l2(s.cpu().numpy(), so)
    say("256^3 sub-range scatter rel-L2", r)
    assert np.array_equal(p.cpu().numpy(), po)
    assert so.sum() > 0 and r <= PD_REL
    g.close()


def test_pd_bench_configuration_subrange(gpu):
    """The benchmark's point-detector configuration (512^3 object, 2048^2 panel,
    mixed estimator, split 20, 1 keV roulette) in the launch shape bench.py
    times: a photon sub-range against the oracle's image of the same photons,
    with equal scored, killed and chord-step counts; then the same sub-range on
    the shape the autotuner picks for this leg (shared palette table, two
    blocks per CU), bitwise equal to the first."""
    torch = gpu
    w = inputs.workload("ellipsoids512_hires")
    o, g = pair(w["ids"], w["rho"], w["voxel_mm"], w["geometry"], w["spectrum"])
    g.set_launch(256, 0, 58)
    for side, mode in zip((o, g), MODES[1]):
        side.set_estimator(mode, 20, 1.0)
    geo = w["geometry"]
    a, m = 500_000_321, 5_000
    say("512^3 point detector (bench configuration) sub-range", a, m)
    p = torch.zeros((geo["nv"], geo["nu"]), dtype=torch.int64, device="cuda:0")
    s = torch.zeros((geo["snv"], geo["snu"]), dtype=torch.int64, device="cuda:0")
    g.stats(True)
    mcx.mc_project_range_async(g.ctx, w["angle"], a, m, w["seed"], p, s)
    torch.cuda.synchronize()
    st_g = g.stats()
    g.stats(False)
    o.stats()
    po, so = o.project_range(w["angle"], a, m, w["seed"])
    st_o = o.stats()
    sg = s.cpu().numpy()
    r = rel_l2(sg, so)
    say("512^3 sub-range scatter rel-L2", r, "differing bins", int((sg != so).sum()),
        "scores", st_g["pd_scores"], "killed", st_g["pd_killed"])
    assert np.array_equal(p.cpu().numpy(), po)
    assert so.sum() > 0 and r <= PD_REL
    for k in ("pd_scores", "pd_killed", "pd_steps"):
        assert st_g[k] == st_o[k], k
    assert st_g["pd_killed"] > 0
    g.set_layout(mcx.MC_LAYOUT_PALETTE_SHARED)
    g.set_launch(256, 2, 44)
    say("512^3 point detector sub-range, shared palette, 2 blocks per CU")
    p2, s2 = torch.zeros_like(p), torch.zeros_like(s)
    mcx.mc_project_range_async(g.ctx, w["angle"], a, m, w["seed"], p2, s2)
    torch.cuda.synchronize()
    assert g.layout()[0] == mcx.MC_LAYOUT_PALETTE_SHARED
    assert torch.equal(p2, p) and torch.equal(s2, s)
    g.close()


def test_pd_launch_shapes_and_ranges(gpu):
    torch = gpu
    w = inputs.workload("cylinder64")
    g = mcx.Projector(0)
    g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*inputs.kramers_spectrum(100, 1.0))
    g.set_estimator(mcx.MC_SCORE_POINT_MIXED, 5, 0.01)
    say("point detector launch shapes")
    ref = g.project(0.7, 150_000, 11)
    for block, bpc, spr in [(64, 1, 1), (128, 2, 7), (192, 0, 64), (256, 0, 33)]:
        g.set_launch(block, bpc, spr)
        pg, sg = g.project(0.7, 150_000, 11)
        assert np.array_equal(pg, ref[0]) and np.array_equal(sg, ref[1]), (block, bpc, spr)
    g.set_launch(0, 0, 0)
    p = torch.zeros((128, 128), dtype=torch.int64, device="cuda:0")
    s = torch.zeros((128, 128), dtype=torch.int64, device="cuda:0")
    for a, b in [(0, 1), (1, 70_000), (70_000, 150_000)]:
        mcx.mc_project_range_async(g.ctx, 0.7, a, b - a, 11, p, s)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), ref[1]) and np.array_equal(p.cpu().numpy(), ref[0])
    g.close()


def test_pd_batch_needs_analog(gpu):
    torch = gpu
    w = inputs.workload("cylinder64")
    g = mcx.Projector(0)
    g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*w["spectrum"])
    g.set_estimator(mcx.MC_SCORE_POINT, 2, 0.0)
    out = torch.zeros(2 * 128 * 128, dtype=torch.int64, device="cuda:0")
    job = dict(phantom=0, angle_rad=0.0, n_photons=10, seed=0, primary_offset=0,
               scatter_offset=128 * 128)
    with pytest.raises(mcx.MCXError):
        mcx.mc_project_batch(g.ctx, [job], out, out.numel(), flags=0)
    g.set_estimator(mcx.MC_SCORE_ANALOG)
    mcx.mc_project_batch(g.ctx, [job], out, out.numel(), flags=0)
    torch.cuda.synchronize()
    g.close()
