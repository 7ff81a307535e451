"""The march probe (the gather ceiling the benchmark reports the transport
against) marches every ray exactly as the transport's fixed-step rule does:
on an object of zero density no photon interacts, so the oracle's step count
for photons 0 .. n-1 is the number of voxel gathers of rays 0 .. n-1, which
the probe returns as its step count and, when every voxel holds material
id 1 in the generic layout (code 1, density bits even), as its code sum.  Sums do not depend on the
refill batch or launch shape; palette layouts give the same step counts."""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import say

pytestmark = pytest.mark.gpu

GEO = dict(sod_mm=300.0, sdd_mm=700.0, nu=40, nv=24, pu_mm=3.0, pv_mm=4.0, snu=20, snv=12,
           step_mm=0.7, flags=0)


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    return torch


@pytest.mark.parametrize("angle", [0.0, 0.9, 2.3])
def test_probe_steps_equal_oracle(torch_gpu, angle):
    torch = torch_gpu
    ids = np.ones((50, 21, 37), np.uint8)
    rho = np.zeros((50, 21, 37), np.float32)
    n, seed = 200_000, 11
    spec = inputs.kramers_spectrum(90, 1.0)
    o = oracle.Oracle()
    o.load_phantom(ids, rho, 1.3)
    o.set_geometry(**GEO)
    o.set_spectrum(*spec)
    o.project(angle, n, seed, threads=8)
    steps = o.stats()["steps"]
    say("probe", angle, "oracle steps", steps)
    g = mcx.Projector(0)
    g.set_layout(mcx.MC_LAYOUT_GENERIC)
    g.load_phantom(ids, rho, 1.3)
    g.set_geometry(**GEO)
    g.set_spectrum(*spec)
    sums = []
    for refill in (1, 16, 64):
        for block in (64, 256):
            g.set_launch(block=block)
            d = torch.zeros(2, dtype=torch.int64, device="cuda")
            mcx.mc_march_probe_async(g.ctx, angle, n, seed, refill, d)
            torch.cuda.synchronize()
            sums += d.tolist()
    assert steps > 0 and all(s == steps for s in sums), (steps, sums)


def test_probe_layouts_and_errors(torch_gpu):
    torch = torch_gpu
    w = inputs.workload("cylinder64")
    out = []
    for layout in (mcx.MC_LAYOUT_PALETTE_LANE, mcx.MC_LAYOUT_PALETTE_SHARED):
        g = mcx.Projector(0)
        g.set_layout(layout)
        g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
        g.set_geometry(**w["geometry"])
        g.set_spectrum(*w["spectrum"])
        d = torch.zeros(2, dtype=torch.int64, device="cuda")
        say("probe layout", layout)
        mcx.mc_march_probe_async(g.ctx, 0.4, 300_000, 3, 8, d)
        torch.cuda.synchronize()
        out.append(tuple(d.tolist()))
        with pytest.raises(mcx.MCXError):
            mcx.mc_march_probe_async(g.ctx, 0.4, 10, 3, 65, d)
        with pytest.raises(mcx.MCXError):
            mcx.mc_march_probe_async(g.ctx, 0.4, 10, 3, 8, None)
    assert out[0] == out[1] and out[0][1] > 0


def _probe_pixels(n, seed, n_pix):
    """Pixel of each add of the tally probe, written from its definition in
    the header (32-bit arithmetic in uint64 with explicit wrap)."""
    m = (1 << 32) - 1
    i = np.arange(n, dtype=np.uint64)
    s = np.uint64((seed ^ (seed >> 32)) & m)
    x = ((i & np.uint64(m)) ^ s ^ (((i >> np.uint64(32)) * np.uint64(0x9E3779B9)) & np.uint64(m)))
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7feb352d)) & np.uint64(m)
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846ca68b)) & np.uint64(m)
    x ^= x >> np.uint64(16)
    return ((x * np.uint64(n_pix)) >> np.uint64(32)).astype(np.int64)


@pytest.mark.parametrize("n,n_pix", [(1, 1), (1_000_003, 4099), (3_000_000, 512 * 512)])
def test_atomic_probe_histogram(torch_gpu, n, n_pix):
    """Every add lands on the pixel the definition gives: the image equals the
    host histogram, also when added onto a non-zero image."""
    torch = torch_gpu
    say("atomic probe", n, n_pix)
    ctx = mcx.mc_create(0)
    try:
        seed = 0x1234_5678_9ABC
        img = torch.full((n_pix,), 7, dtype=torch.int64, device="cuda")
        mcx.mc_atomic_probe_async(ctx, n, seed, img, n_pix)
        torch.cuda.synchronize()
        ref = np.bincount(_probe_pixels(n, seed, n_pix), minlength=n_pix) + 7
        assert np.array_equal(img.cpu().numpy(), ref)
        with pytest.raises(mcx.MCXError):
            mcx.mc_atomic_probe_async(ctx, n, seed, img, 0)
    finally:
        mcx.mc_destroy(ctx)
