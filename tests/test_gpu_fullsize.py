"""GPU parity at full workload sizes, in the launch configuration bench.py times.

The oracle cannot run 1e8 - 1e9 photons inside a test, so the full-size runs
are checked on what it can compute: per-history records of photons sampled
across the whole id range, and the image of a sub-range of photons; plus
properties that hold at any size (the full image equals the sum of its
photon sub-ranges, bitwise).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import check_histories, check_images, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    return torch


@pytest.mark.parametrize("name", ["ellipsoids256_poly", "ellipsoids512_hires"])
def test_full_size_workload(torch_gpu, name):
    torch = torch_gpu
    say("full size", name, "generating inputs")
    w = inputs.workload(name)
    n = w["n_photons"]
    geo = w["geometry"]
    g = mcx.Projector(0)
    o = oracle.Oracle()
    for side in (g, o):
        side.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
        side.set_geometry(**geo)
        side.set_spectrum(*w["spectrum"])
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    shp_p, shp_s = (geo["nv"], geo["nu"]), (geo["snv"], geo["snu"])
    p = torch.empty(shp_p, dtype=torch.int64, device=dev)
    s = torch.empty(shp_s, dtype=torch.int64, device=dev)
    say(name, f"full projection, {n} photons")
    mcx.mc_project_async(g.ctx, w["angle"], n, w["seed"], p, s, stream)
    # the same photons as three ranges, accumulated
    p2 = torch.zeros_like(p)
    s2 = torch.zeros_like(s)
    cut = [0, n // 3, n // 3 + 12345, n]
    for a, b in zip(cut[:-1], cut[1:]):
        mcx.mc_project_range_async(g.ctx, w["angle"], a, b - a, w["seed"], p2, s2, stream)
    torch.cuda.synchronize()
    assert torch.equal(p, p2) and torch.equal(s, s2)
    assert int(p.sum()) > 0 and int(s.sum()) > 0

    # sampled histories across the whole id range
    rng = np.random.default_rng(123)
    starts = np.sort(rng.integers(0, n - 2000, size=10))
    for a in starts:
        a = int(a)
        say(name, "histories", a, a + 2000)
        check_histories(f"{name}@{a}", g.debug_histories(w["angle"], a, 2000, w["seed"]),
                        o.debug_histories(w["angle"], a, 2000, w["seed"]))

    # the image of a sub-range, somewhere in the middle of the id range
    a, m = n // 2 + 777, 200_000
    say(name, "sub-range image", a, a + m)
    pr = torch.zeros_like(p)
    sr = torch.zeros_like(s)
    mcx.mc_project_range_async(g.ctx, w["angle"], a, m, w["seed"], pr, sr, stream)
    torch.cuda.synchronize()
    po, so = o.project_range(w["angle"], a, m, w["seed"])
    check_images(f"{name}[{a}:{a + m}]", pr.cpu().numpy(), sr.cpu().numpy(), po, so)
    g.close()


def _host_threads():
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def test_full_image_256_equals_oracle(torch_gpu):
    """The whole 1e8-photon projection of the 256^3 polychromatic workload,
    every pixel of both images, against the oracle's image of the same photons
    (threaded over photon ranges, which sums to the sequential oracle's image)."""
    torch = torch_gpu
    w = inputs.workload("ellipsoids256_poly")
    n, geo = w["n_photons"], w["geometry"]
    g = mcx.Projector(0)
    o = oracle.Oracle()
    for side in (g, o):
        side.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
        side.set_geometry(**geo)
        side.set_spectrum(*w["spectrum"])
    p = torch.empty((geo["nv"], geo["nu"]), dtype=torch.int64, device="cuda:0")
    s = torch.empty((geo["snv"], geo["snu"]), dtype=torch.int64, device="cuda:0")
    say("ellipsoids256_poly whole image on the GPU", n)
    mcx.mc_project_async(g.ctx, w["angle"], n, w["seed"], p, s)
    torch.cuda.synchronize()
    threads = _host_threads()
    say("ellipsoids256_poly whole image on the oracle,", threads, "threads")
    po, so = o.project(w["angle"], n, w["seed"], threads=threads)
    pg, sg = p.cpu().numpy(), s.cpu().numpy()
    check_images("ellipsoids256_poly whole image", pg, sg, po, so)
    say("bitwise", bool(np.array_equal(pg, po) and np.array_equal(sg, so)))
    g.close()
