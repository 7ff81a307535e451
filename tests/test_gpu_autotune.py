"""Autotuners: every timed launch shape reproduces the same images (none
rejected), the winner is applied, a second call is served from the cache, and
the tuned launch's images equal the oracle's (single projections and
batches)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def test_autotune_and_cache(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    w = inputs.workload("cylinder64")
    g = mcx.Projector(0)
    g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*inputs.kramers_spectrum(100, 1.0))
    ref = g.project(0.2, 200_000, 5)
    cache = str(tmp_path / "tune.jsonl")
    say("autotune")
    t = mcx.mc_autotune(g.ctx, 0.2, 200_000, 5, cache)
    say("autotune result", t)
    # 3 block sizes x 2 blocks per CU x 5 event batches x 2 table layouts
    assert t["from_cache"] == 0 and t["candidates"] == 72 and t["rejected"] == 0
    assert t["block"] in (64, 128, 256) and 36 <= t["event_batch"] <= 58
    assert t["table_layout"] in (mcx.MC_LAYOUT_PALETTE_LANE, mcx.MC_LAYOUT_PALETTE_SHARED)
    p, s = g.project(0.2, 200_000, 5)          # runs with the tuned shape
    assert np.array_equal(p, ref[0]) and np.array_equal(s, ref[1])
    o = oracle.Oracle()
    o.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    o.set_geometry(**w["geometry"])
    o.set_spectrum(*inputs.kramers_spectrum(100, 1.0))
    po, so = o.project(0.2, 200_000, 5, threads=8)
    assert np.array_equal(p, po) and np.array_equal(s, so)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["block"] == t["block"]
    t2 = mcx.mc_autotune(g.ctx, 0.2, 200_000, 5, cache)
    assert t2["from_cache"] == 1 and (t2["block"], t2["event_batch"], t2["table_layout"]) == \
        (t["block"], t["event_batch"], t["table_layout"])
    assert g.layout()[0] == t["table_layout"]


def test_autotune_batch_and_cache(tmp_path):
    """Batch autotuner on a job table of several objects (uneven sizes, one
    with more than 32 palette entries): all candidates bitwise equal, the
    tuned shape applied to mc_project_batch (graph replay too), one job equal
    to the oracle, and the second call served from the cache."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    geo = dict(sod_mm=400.0, sdd_mm=800.0, nu=48, nv=40, pu_mm=2.0, pv_mm=2.0, snu=12, snv=10,
               step_mm=0.8, flags=0)
    spec = inputs.kramers_spectrum(110, 1.5)
    rng = np.random.default_rng(4)
    keys = rng.integers(0, 60, size=(9, 14, 17))
    objs = [(*inputs.ellipsoid_phantom(40, 1.5, seed=5), 1.5),
            (*inputs.cylinder_phantom(32, 2.0, radius_mm=20.0), 2.0),
            ((keys % 5).astype(np.uint8), (0.1 + 0.013 * keys).astype(np.float32), 3.0)]
    g = mcx.Projector(0)
    g.set_spectrum(*spec)
    g.set_geometry(**geo)
    g.load_phantom(*objs[0])
    handles = [0] + [mcx.mc_phantom_add(g.ctx, *o) for o in objs[1:]]
    assert mcx.mc_get_batch_info(g.ctx)[0] == 3
    np_, ns_ = geo["nu"] * geo["nv"], geo["snu"] * geo["snv"]
    jobs = [dict(phantom=handles[i % 3], angle_rad=0.3 * i, n_photons=n, seed=50 + i,
                 primary_offset=i * (np_ + ns_), scatter_offset=i * (np_ + ns_) + np_)
            for i, n in enumerate([60_000, 150_000, 1, 40_000, 90_000, 7, 120_000, 30_000])]
    total = len(jobs) * (np_ + ns_)
    ref = torch.zeros(total, dtype=torch.int64, device="cuda:0")
    mcx.mc_project_batch(g.ctx, jobs, ref, total, flags=0)
    torch.cuda.synchronize()
    out = torch.zeros_like(ref)
    cache = str(tmp_path / "tune_batch.jsonl")
    say("autotune batch")
    t = mcx.mc_autotune_batch(g.ctx, jobs, out, total, cache)
    say("autotune batch result", t)
    # 2 table layouts x 2 block sizes x 3 grid sizes x 3 event batches
    assert t["from_cache"] == 0 and t["candidates"] == 36 and t["rejected"] == 0
    assert torch.equal(out, ref)
    out.fill_(-1)
    mcx.mc_project_batch(g.ctx, jobs, out, total, flags=mcx.MC_BATCH_GRAPH)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    j = jobs[4]
    o = oracle.Oracle()
    o.load_phantom(*objs[j["phantom"]])
    o.set_geometry(**geo)
    o.set_spectrum(*spec)
    po, so = o.project(j["angle_rad"], j["n_photons"], j["seed"], threads=8)
    host = out.cpu().numpy()
    assert np.array_equal(host[j["primary_offset"]:j["primary_offset"] + np_].reshape(po.shape), po)
    assert np.array_equal(host[j["scatter_offset"]:j["scatter_offset"] + ns_].reshape(so.shape), so)
    t2 = mcx.mc_autotune_batch(g.ctx, jobs, out, total, cache)
    assert t2["from_cache"] == 1 and (t2["block"], t2["blocks_per_cu"], t2["event_batch"]) == \
        (t["block"], t["blocks_per_cu"], t["event_batch"])
    g.close()
