"""Oracle of the paper's scatter post-processing (TEST INFRASTRUCTURE ONLY).

Section II-C-3/4 of the paper smooths noisy MC scatter images with a cubic
Savitzky-Golay filter and up-samples low-resolution projections with cubic
interpolation.  Readings (the paper gives neither window nor boundary rule
nor the cubic kernel):

* Savitzky-Golay: the least-squares polynomial of degree `order` over a
  window of `window` samples, evaluated at the window centre, applied along
  image rows and then along columns (separable); samples beyond an edge are
  mirrored about the edge sample (x[-k] = x[k]).
* Cubic up-sampling by an integer factor f: Keys' cubic convolution kernel
  with a = -0.5, output sample i at input coordinate (i + 0.5)/f - 0.5
  (pixel centres aligned), neighbours beyond an edge clamped to the edge.

fp64, plain loops over the definition.
"""
import numpy as np


def savgol_coefficients(window, order):
    """Weights c[j], j = -h..h, such that sum_j c[j] x[i+j] is the value at 0 of
    the least-squares polynomial of degree `order` through (j, x[i+j])."""
    if window % 2 != 1 or window <= order:
        raise ValueError("window must be odd and larger than the order")
    h = window // 2
    j = np.arange(-h, h + 1, dtype=np.float64)
    A = np.vander(j, order + 1, increasing=True)          # columns 1, j, j^2, ...
    # least squares: p = (A^T A)^-1 A^T x; value at 0 is p[0]
    P = np.linalg.solve(A.T @ A, A.T)
    return P[0]


def _mirror(i, n):
    """Index reflected about the edge samples into [0, n)."""
    if n == 1:
        return 0
    period = 2 * (n - 1)
    i = i % period
    return i if i < n else period - i


def savgol_1d(x, window, order):
    x = np.asarray(x, dtype=np.float64)
    c = savgol_coefficients(window, order)
    h = window // 2
    n = len(x)
    out = np.zeros(n)
    for i in range(n):
        s = 0.0
        for k in range(-h, h + 1):
            s += c[k + h] * x[_mirror(i + k, n)]
        out[i] = s
    return out


def savgol_2d(img, window, order):
    img = np.asarray(img, dtype=np.float64)
    rows = np.array([savgol_1d(r, window, order) for r in img])
    return np.array([savgol_1d(c, window, order) for c in rows.T]).T


def keys_kernel(t, a=-0.5):
    t = abs(t)
    if t <= 1.0:
        return (a + 2.0) * t ** 3 - (a + 3.0) * t ** 2 + 1.0
    if t < 2.0:
        return a * t ** 3 - 5.0 * a * t ** 2 + 8.0 * a * t - 4.0 * a
    return 0.0


def upsample_1d(x, f):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    out = np.zeros(n * f)
    for i in range(n * f):
        u = (i + 0.5) / f - 0.5
        i0 = int(np.floor(u))
        s = 0.0
        for m in range(i0 - 1, i0 + 3):
            s += keys_kernel(u - m) * x[min(max(m, 0), n - 1)]
        out[i] = s
    return out


def upsample_2d(img, f):
    img = np.asarray(img, dtype=np.float64)
    rows = np.array([upsample_1d(r, f) for r in img])
    return np.array([upsample_1d(c, f) for c in rows.T]).T
