"""Autotuner: every timed launch shape reproduces the same images (none
rejected), the winner is applied, and a second call is served from the cache."""
import json
import os

import numpy as np
import pytest

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
    assert t["from_cache"] == 0 and t["candidates"] == 60 and t["rejected"] == 0
    assert t["block"] in (64, 128, 256) and 48 <= t["event_batch"] <= 60
    assert t["table_layout"] in (mcx.MC_LAYOUT_PALETTE_LANE, mcx.MC_LAYOUT_PALETTE_SHARED)
    p, s = g.project(0.2, 200_000, 5)          # runs with the tuned shape
    assert np.array_equal(p, ref[0]) and np.array_equal(s, ref[1])
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["block"] == t["block"]
    t2 = mcx.mc_autotune(g.ctx, 0.2, 200_000, 5, cache)
    assert t2["from_cache"] == 1 and (t2["block"], t2["event_batch"], t2["table_layout"]) == \
        (t["block"], t["event_batch"], t["table_layout"])
    assert g.layout()[0] == t["table_layout"]
