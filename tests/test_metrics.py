"""Metric pins: closed forms and exact special cases."""
import numpy as np

from paper_2201_13191_amd import metrics as M


def test_rel_l2_and_mse():
    b = np.array([3.0, 4.0])
    assert M.rel_l2(b, b) == 0.0
    assert abs(M.rel_l2(b * 1.1, b) - 0.1) < 1e-12
    assert abs(M.mse([1, 2, 3], [1, 2, 5]) - 4.0 / 3.0) < 1e-12


def test_ncc_properties():
    x = np.random.default_rng(0).normal(size=1000)
    assert abs(M.ncc(x, 3 * x + 2) - 1.0) < 1e-12
    assert abs(M.ncc(x, -x) + 1.0) < 1e-12


def test_cnr_closed_form():
    img = np.zeros((4, 4))
    img[:2] = [[5, 5, 5, 5], [5, 5, 5, 5]]
    img[2:] = [[1, -1, 1, -1], [1, -1, 1, -1]]
    roi = np.zeros((4, 4), bool)
    roi[:2] = True
    assert abs(M.cnr(img, roi, ~roi) - 5.0) < 1e-12


def test_debiased_rel_rms_recovers_true_error():
    rng = np.random.default_rng(1)
    s = 100.0 + 20.0 * np.sin(np.linspace(0, 6, 4096))         # noise-free image
    a = s * 1.02                                               # 2 % off
    batches = s + rng.normal(0, 30.0, size=(8, s.size))        # noisy reference batches
    raw = M.rel_l2(a, batches.mean(axis=0))
    deb = M.debiased_rel_rms(a, batches)
    assert raw > 0.05                      # the raw figure is dominated by the reference's noise
    assert abs(deb - 0.02) < 0.004


def test_pair_rel_rms_recovers_noise_level():
    """Two independent noisy estimates of a known image: the pair estimate
    equals the known rel-RMS of either one (Gaussian noise of known sigma)."""
    rng = np.random.default_rng(2)
    s = 50.0 + 10.0 * np.cos(np.linspace(0, 9, 200_000))
    sigma = 7.0
    a = s + rng.normal(0, sigma, s.size)
    b = s + rng.normal(0, sigma, s.size)
    true_r = sigma * np.sqrt(s.size) / np.linalg.norm(s)
    assert abs(M.pair_rel_rms(a, b) / true_r - 1) < 0.01
    assert M.pair_rel_rms(s, s) == 0.0
