"""Image metrics used to score scatter estimates (host-side evaluation).

* rel_l2(a, b) = ||a - b|| / ||b|| over the image (b is the reference).
* debiased_rel_rms(a, batches): the reference b is the mean of B independent
  photon-range batches; their spread estimates the reference's own noise
  V_b = sum_p Var(b_p), and ((||a - b||^2 - V_b) / (||b||^2 - V_b))^(1/2)
  estimates ||a - s|| / ||s|| against the noise-free image s when a is
  independent of b (negative estimates clip to 0).
* pair_rel_rms(a, b): the rel-RMS of either of two independent estimates of
  equal precision against the noise-free image.
* The paper's quantitative measures (section II-E, eq. (9)-(11)): MSE, the
  normalised cross-correlation NCC and the contrast-to-noise ratio CNR of a
  region of interest against a background region.
"""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float("inf")


def batch_mean_and_noise(batches):
    """Mean image of B independent equal-size batches and the summed variance
    of that mean over pixels."""
    x = np.asarray(batches, np.float64)
    B = x.shape[0]
    if B < 2:
        raise ValueError("need at least two batches")
    mean = x.mean(axis=0)
    var_of_mean = x.var(axis=0, ddof=1).sum() / B
    return mean, float(var_of_mean)


def debiased_rel_rms(a, batches):
    b, vb = batch_mean_and_noise(batches)
    a = np.asarray(a, np.float64)
    num = np.sum((a - b) ** 2) - vb
    den = np.sum(b ** 2) - vb
    if den <= 0:
        return float("inf")
    return float(np.sqrt(max(num, 0.0) / den))


def pair_rel_rms(a, b):
    """rel-RMS ||a - s|| / ||s|| of one estimate against the noise-free image s,
    from two independent estimates a, b of equal precision: E||a - b||^2 = 2V
    and E(||a||^2 + ||b||^2) / 2 = ||s||^2 + V, so
    r^2 = (||a - b||^2 / 2) / ((||a||^2 + ||b||^2) / 2 - ||a - b||^2 / 2)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    v = float(np.sum((a - b) ** 2)) / 2.0
    s2 = float(np.sum(a ** 2) + np.sum(b ** 2)) / 2.0 - v
    return float(np.sqrt(v / s2)) if s2 > 0 else float("inf")


def mse(x1, x2):
    x1 = np.asarray(x1, np.float64)
    x2 = np.asarray(x2, np.float64)
    return float(np.mean((x1 - x2) ** 2))


def ncc(x1, x2):
    x1 = np.asarray(x1, np.float64).ravel()
    x2 = np.asarray(x2, np.float64).ravel()
    d1, d2 = x1 - x1.mean(), x2 - x2.mean()
    return float(np.mean(d1 * d2) / (x1.std() * x2.std()))


def cnr(img, roi, background):
    """|mean(ROI) - mean(background)| / std(background); roi and background
    are boolean masks or index expressions into img."""
    img = np.asarray(img, np.float64)
    r, bg = img[roi], img[background]
    return float(abs(r.mean() - bg.mean()) / bg.std())
