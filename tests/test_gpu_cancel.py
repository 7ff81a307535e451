"""Cancellation (mc_cancel): a long projection stops early, every kernel exits
normally, and the images hold exactly photons 0 .. m-1 (bitwise a run of m
photons, m read from the statistics); a blocking call cancelled from another
thread returns MC_E_CANCELLED; after clearing the flag projections run in full."""
import threading
import time

import numpy as np
import pytest

from paper_2201_13191_amd import inputs, mcx
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def _ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    w = inputs.workload("cylinder64")
    g = mcx.Projector(0)
    g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*w["spectrum"])
    return torch, g


def _rate(g):
    t = time.perf_counter()
    g.project(0.3, 20_000_000, 1)
    return 20_000_000 / (time.perf_counter() - t)


def test_cancel_async_keeps_a_prefix():
    torch, g = _ctx()
    n = int(min(4.0 * _rate(g), 3e10))          # about four seconds of work
    geo = g.geometry
    dp = torch.zeros(geo["nv"] * geo["nu"], dtype=torch.int64, device="cuda")
    ds = torch.zeros(geo["snv"] * geo["snu"], dtype=torch.int64, device="cuda")
    say("cancel an async projection of", n, "photons")
    g.stats(True)
    t0 = time.perf_counter()
    mcx.mc_project_async(g.ctx, 0.3, n, 5, dp, ds)
    time.sleep(0.4)
    g.cancel(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = g.stats()
    g.stats(False)
    g.cancel(False)
    m = st["histories"]
    say(f"stopped after {elapsed:.2f} s with {m} of {n} photons")
    assert 0 < m < n and elapsed < 2.5
    p, s = g.project(0.3, m, 5)
    assert np.array_equal(dp.cpu().numpy(), p.ravel())
    assert np.array_equal(ds.cpu().numpy(), s.ravel())
    g.close()


def test_cancel_blocking_call_from_another_thread():
    torch, g = _ctx()
    n = int(min(4.0 * _rate(g), 3e10))
    out = {}

    def run():
        try:
            g.project(0.3, n, 9)
            out["code"] = 0
        except mcx.MCXError as e:
            out["code"] = e.code

    say("cancel a blocking projection of", n, "photons")
    th = threading.Thread(target=run)
    t0 = time.perf_counter()
    th.start()
    time.sleep(0.4)
    g.cancel(True)
    th.join(timeout=60)
    elapsed = time.perf_counter() - t0
    g.cancel(False)
    say(f"returned {out.get('code')} after {elapsed:.2f} s")
    assert not th.is_alive() and out.get("code") == mcx.MC_E_CANCELLED and elapsed < 2.5
    # cleared: a projection runs in full and equals a fresh context's
    p, s = g.project(0.2, 300_000, 4)
    torch2, g2 = _ctx()
    p2, s2 = g2.project(0.2, 300_000, 4)
    assert np.array_equal(p, p2) and np.array_equal(s, s2)
    g.close()
    g2.close()
