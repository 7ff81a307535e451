"""End-to-end run of the learned-part pipeline at toy size: data generation
with the batched launch, normalisation, training, held-out evaluation."""
import math

import pytest

from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def test_pipeline_toy(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    from paper_2201_13191_amd import learned
    say("learned pipeline toy")
    out = learned.main(["--phantoms", "4", "--angles", "2", "--test-phantoms", "2",
                        "--test-angles", "1", "--n-in", "200000", "--n-tgt", "2000000",
                        "--n-ref", "8000000", "--ref-batches", "4", "--epochs", "2",
                        "--batch", "2", "--out", str(tmp_path / "l.json")])
    assert out["pairs"] == 8 and len(out["losses"]) == 2
    for k in ("raw_cubic", "sg_cubic", "unet"):
        assert math.isfinite(out["rel_rms"][k]["raw_mean"])
    assert 0 < out["reference_noise_rel"] < 1
    assert out["plain_mc"]["histories_per_s"] > 1e8
