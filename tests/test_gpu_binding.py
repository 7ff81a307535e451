"""GPU parity of the binding effects (S(x,Z) of eq. (1) as null collisions,
Doppler broadening of the Compton line) against the oracle's.

Both sides do the same correctly rounded fp64 arithmetic for the S
acceptance and the Doppler root, so the samplers are compared bitwise; the
transport with the effects on is compared as the analog transport is
(images bitwise equal in practice, the bar the transport's tolerances), with
equal event counts; point-detector images as in the point-detector tests.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import check_images, pair, rel_l2, say

pytestmark = pytest.mark.gpu

FLAGS = [(oracle.PHYS_INCOH_SF, mcx.MC_PHYS_INCOH_SF),
         (oracle.PHYS_DOPPLER, mcx.MC_PHYS_DOPPLER),
         (oracle.PHYS_INCOH_SF | oracle.PHYS_DOPPLER, mcx.MC_PHYS_INCOH_SF | mcx.MC_PHYS_DOPPLER)]
IDS = ["sf", "doppler", "both"]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    mcx.load()
    return torch


@pytest.mark.parametrize("flags", FLAGS, ids=IDS)
@pytest.mark.parametrize("mat,e", [(1, 2.0), (1, 60.0), (4, 30.0), (4, 150.0), (3, 500.0)])
def test_compton_collision_sampler_bitwise(gpu, flags, mat, e):
    o = oracle.Oracle()
    g = mcx.Projector(0)
    o.set_physics(flags[0])
    g.set_physics(flags[1])
    n = 200_000
    say("Compton collision sampler", flags[1], mat, e)
    co, eo = o.test_sample(oracle.PROC_COMPTON, mat, e, n, seed=41)
    cg, eg = g.test_sample(mcx.MC_PROC_COMPTON, mat, e, n, 41)
    null = int((co == 2.0).sum())
    say(f"cos mismatches {int((co != cg).sum())}, energy mismatches {int((eo != eg).sum())}, "
        f"null {null}")
    assert np.array_equal(co, cg) and np.array_equal(eo, eg)
    if flags[1] & mcx.MC_PHYS_INCOH_SF:
        assert null > 0
    g.close()


def _transport(name, ids, rho, h, geo, spec, n, seed, phys, layout=None, est=None, angle=0.4):
    o, g = pair(ids, rho, h, geo, spec)
    for side, f in zip((o, g), phys):
        side.set_physics(f)
    if layout is not None:
        g.set_layout(layout)
        g.load_phantom(ids, rho, h)
    if est is not None:
        o.set_estimator(est[0], 6, 0.0)
        g.set_estimator(est[1], 6, 0.0)
    say(name, f"physics {phys[1]}, {n} photons, layout {layout}, estimator {est}")
    g.stats(True)
    pg, sg = g.project(angle, n, seed)
    st_g = g.stats()
    g.stats(False)
    o.stats()
    po, so = o.project(angle, n, seed, threads=8)
    st_o = o.stats()
    check_images(name, pg, sg, po, so)
    say(name, f"bitwise primary {np.array_equal(pg, po)} scatter {np.array_equal(sg, so)}; "
              f"null collisions {st_g['null_collisions']} / {st_o['null_collisions']}, "
              f"compton {st_g['compton']} / {st_o['compton']}")
    for k in ("null_collisions", "compton", "rayleigh", "photo", "primary_hits"):
        assert st_g[k] == st_o[k], (name, k, st_g[k], st_o[k])
    if est is not None:
        assert st_g["pd_scores"] == st_o["pd_scores"]
    g.close()
    return pg, sg


@pytest.mark.parametrize("flags", FLAGS, ids=IDS)
def test_binding_cylinder(gpu, flags):
    w = inputs.workload("cylinder64")
    _transport("cylinder64", w["ids"], w["rho"], w["voxel_mm"], w["geometry"], w["spectrum"],
               200_000, 3, flags)


@pytest.mark.parametrize("layout", [mcx.MC_LAYOUT_PALETTE_LANE, mcx.MC_LAYOUT_PALETTE_SHARED,
                                    mcx.MC_LAYOUT_GENERIC])
def test_binding_layouts(gpu, layout):
    ids, rho = inputs.ellipsoid_phantom(48, 1.0, seed=31, iron_insert=True)
    geo = dict(sod_mm=300.0, sdd_mm=600.0, nu=64, nv=48, pu_mm=2.0, pv_mm=2.0, snu=16, snv=12,
               step_mm=1.0, flags=0)
    _transport("ellipsoids48 + iron", ids, rho, 1.0, geo, inputs.kramers_spectrum(120, 2.0),
               100_000, 9, FLAGS[2], layout=layout)


@pytest.mark.parametrize("est", [(oracle.SCORE_POINT, mcx.MC_SCORE_POINT),
                                 (oracle.SCORE_POINT_MIXED, mcx.MC_SCORE_POINT_MIXED)],
                         ids=["point", "mixed"])
def test_binding_point_detector(gpu, est):
    w = inputs.workload("cylinder64")
    pg, sg = _transport("cylinder64 PD", w["ids"], w["rho"], w["voxel_mm"], w["geometry"],
                        w["spectrum"], 60_000, 5, FLAGS[2], est=est)
    assert sg.sum() > 0


def test_binding_batch_matches_single(gpu):
    """Batch jobs with the effects on are bitwise the single projections."""
    import torch
    w = inputs.workload("cylinder64")
    g = mcx.Projector(0)
    g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*w["spectrum"])
    g.set_physics(mcx.MC_PHYS_INCOH_SF | mcx.MC_PHYS_DOPPLER)
    geo = g.geometry
    np_, ns_ = geo["nu"] * geo["nv"], geo["snu"] * geo["snv"]
    jobs = [dict(phantom=0, angle_rad=0.5 * i, n_photons=n, seed=70 + i,
                 primary_offset=i * (np_ + ns_), scatter_offset=i * (np_ + ns_) + np_)
            for i, n in enumerate([50_000, 1, 80_000, 30_000])]
    total = len(jobs) * (np_ + ns_)
    out = torch.zeros(total, dtype=torch.int64, device="cuda:0")
    say("binding batch", len(jobs))
    mcx.mc_project_batch(g.ctx, jobs, out, total, flags=mcx.MC_BATCH_GRAPH)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    for j in jobs:
        p, s = g.project(j["angle_rad"], j["n_photons"], j["seed"])
        assert np.array_equal(host[j["primary_offset"]:j["primary_offset"] + np_], p.ravel())
        assert np.array_equal(host[j["scatter_offset"]:j["scatter_offset"] + ns_], s.ravel())
    g.close()
