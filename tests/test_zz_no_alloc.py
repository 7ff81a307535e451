"""The allocation-free batch entry point (mc_project_batch_static) against
mc_project_batch: two calls in a row, the second with fewer jobs, photons and
objects; each call's whole output buffer must be bitwise equal to the
allocating entry point's, and one job to the oracle."""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx

pytestmark = pytest.mark.gpu

GEO = dict(sod_mm=400.0, sdd_mm=800.0, nu=48, nv=40, pu_mm=2.0, pv_mm=2.0, snu=12, snv=10,
           step_mm=0.8, flags=0)


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _jobs(handles, counts, seed0):
    np_, ns_ = GEO["nu"] * GEO["nv"], GEO["snu"] * GEO["snv"]
    jobs, off = [], 0
    for i, n in enumerate(counts):
        jobs.append(dict(phantom=handles[i % len(handles)], angle_rad=0.41 * i + 0.1,
                         n_photons=n, seed=seed0 + 3 * i, primary_offset=off,
                         scatter_offset=off + np_))
        off += np_ + ns_ + 5
    return jobs, off


def test_static_batch_matches_allocating_batch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    spec = inputs.kramers_spectrum(110, 1.5)
    objs = [(*inputs.cylinder_phantom(32, 2.0, radius_mm=20.0), 2.0),
            (*inputs.ellipsoid_phantom(40, 1.5, seed=5), 1.5),
            (*inputs.ellipsoid_phantom(24, 2.5, seed=6), 2.5)]
    g = mcx.Projector(0)
    g.set_spectrum(*spec)
    g.set_geometry(**GEO)
    g.load_phantom(*objs[0])
    handles = [0] + [mcx.mc_phantom_add(g.ctx, *o) for o in objs[1:]]
    stream = torch.cuda.current_stream()
    cases = [(handles, [50_000, 1, 0, 120_003, 777, 64, 33_000, 90_001], 100),
             (handles[:2], [20_000, 5, 3_333], 900)]
    for call, (hs, counts, seed0) in enumerate(cases):
        jobs, total = _jobs(hs, counts, seed0)
        say("no-alloc batch call", call, "jobs", len(jobs), "photons", sum(counts))
        ref = torch.full((total,), 7, dtype=torch.int64, device="cuda:0")
        out = torch.full((total,), -9, dtype=torch.int64, device="cuda:0")
        mcx.mc_project_batch(g.ctx, jobs, ref, total, flags=0, stream=stream)
        mcx.mc_project_batch_static(g.ctx, jobs, out, total, stream=stream)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), call
        assert int(out.sum()) > 0
    # the last call's second job against the oracle
    j = jobs[0]
    o = oracle.Oracle()
    o.load_phantom(*objs[j["phantom"]])
    o.set_geometry(**GEO)
    o.set_spectrum(*spec)
    po, so = o.project(j["angle_rad"], j["n_photons"], j["seed"], threads=8)
    host = out.cpu().numpy()
    np_, ns_ = GEO["nu"] * GEO["nv"], GEO["snu"] * GEO["snv"]
    assert np.array_equal(host[j["primary_offset"]:j["primary_offset"] + np_].reshape(po.shape), po)
    assert np.array_equal(host[j["scatter_offset"]:j["scatter_offset"] + ns_].reshape(so.shape), so)
    g.close()


def test_static_batch_limits():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    g = mcx.Projector(0)
    g.set_spectrum(*inputs.mono_spectrum(60.0))
    g.set_geometry(**GEO)
    a, b = inputs.cylinder_phantom(16, 2.0)
    g.load_phantom(a, b, 2.0)
    np_, ns_ = GEO["nu"] * GEO["nv"], GEO["snu"] * GEO["snv"]
    out = torch.zeros(np_ + ns_, dtype=torch.int64, device="cuda:0")
    job = dict(phantom=0, angle_rad=0.0, n_photons=10, seed=0, primary_offset=0,
               scatter_offset=np_)
    # a fresh context has no device tables yet: the entry point will not allocate them
    with pytest.raises(mcx.MCXError) as err:
        mcx.mc_project_batch_static(g.ctx, [job], out, np_ + ns_)
    assert err.value.code == mcx.MC_E_STATE
    g.project(0.0, 10, 0)
    with pytest.raises(mcx.MCXError):
        mcx.mc_project_batch_static(g.ctx, [job] * (mcx.MC_STATIC_MAX_JOBS + 1), out, np_ + ns_)
    with pytest.raises(mcx.MCXError):      # images outside the buffer
        mcx.mc_project_batch_static(g.ctx, [dict(job, scatter_offset=np_ + 1)], out, np_ + ns_)
    mcx.mc_project_batch_static(g.ctx, [job], out, np_ + ns_)
    torch.cuda.synchronize()
    g.close()
