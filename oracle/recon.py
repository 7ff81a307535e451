"""Oracle of the iterative scatter correction's reconstruction side (TEST
INFRASTRUCTURE ONLY): what the paper's correction loop (section II-E, its
flowchart and eq. (8)) needs besides the Monte Carlo itself.

* Line integrals: a = -ln(I / I0), I the measured intensity, I0 the flat
  field (the unattenuated primary).
* FBP: the Feldkamp-Davis-Kress cone-beam filtered backprojection for the
  circular orbit of the projector (source at sod (cos b, sin b, 0), panel at
  sdd, u along (-sin b, cos b, 0), v along z), full 2 pi scan of n equally
  spaced angles b_i = 2 pi i / n.  The projections are taken to a virtual
  panel through the rotation axis (coordinates scaled by sod / sdd), weighted
  by sod / sqrt(sod^2 + a^2 + b^2), filtered along rows with the discrete
  Ram-Lak kernel of sampling interval t (h(0) = 1/(4 t^2), h(odd n) =
  -1/(n pi t)^2, h(even n) = 0, times t), and backprojected with weight
  sod^2 / L^2 (L the voxel's distance from the source along the central ray)
  and bilinear interpolation between pixel centres (zero outside the panel):
  f(x) = 1/2 * (2 pi / n) * sum_i w_i(x) q_i(a(x), b(x)).
* Otsu's threshold: the histogram split that maximises the between-class
  variance.
* Volume to density: voxels above the threshold become the object's material
  with density mu / (mu/rho)(E_eff); the others air.
* Eq. (8): c = a - ln(Ip / (Ip + Is)).

fp64, plain loops over the definitions.  Pins: tests/test_oracle_recon.py; the
FDK cosine pre-weight is part of the definition but not separately pinned (on
the pins' balls it moves the reconstruction by less than 0.1 %).
"""
import numpy as np


def line_integrals(I, I0):
    I = np.asarray(I, np.float64)
    I0 = np.asarray(I0, np.float64)
    return -np.log(np.maximum(I, 1e-30) / I0)


def scatter_correct(a, ip, is_):
    """Eq. (8)."""
    ip = np.asarray(ip, np.float64)
    return np.asarray(a, np.float64) - np.log(ip / (ip + np.asarray(is_, np.float64)))


def ramp_kernel(n, t):
    """Discrete Ram-Lak kernel h[k], k = -(n-1) .. n-1, for sampling interval t."""
    k = np.arange(-(n - 1), n)
    h = np.zeros(k.shape, np.float64)
    h[k == 0] = 1.0 / (4.0 * t * t)
    odd = (k % 2) != 0
    h[odd] = -1.0 / (k[odd] * np.pi * t) ** 2
    return h


def fdk_filter(proj, geo):
    """The FDK's weighting and filtering: proj[n_ang][nv][nu] line integrals ->
    the filtered projections q on the virtual panel through the axis."""
    proj = np.asarray(proj, np.float64)
    n_ang, nv, nu = proj.shape
    R, D = float(geo["sod_mm"]), float(geo["sdd_mm"])
    pu, pv = float(geo["pu_mm"]), float(geo["pv_mm"])
    s = R / D
    tu = pu * s                                  # virtual-panel pitch along u
    a = (-nu * pu / 2 + (np.arange(nu) + 0.5) * pu) * s
    b = (-nv * pv / 2 + (np.arange(nv) + 0.5) * pv) * s
    A, B = np.meshgrid(a, b, indexing="xy")
    weight = R / np.sqrt(R * R + A * A + B * B)
    h = ramp_kernel(nu, tu)
    q = np.zeros_like(proj)
    for i in range(n_ang):
        pw = proj[i] * weight
        for r in range(nv):
            q[i, r] = np.convolve(pw[r], h, mode="full")[nu - 1:2 * nu - 1] * tu
    return q


def fdk_backproject(q, geo, vol_shape, voxel_mm):
    """The FDK's distance-weighted backprojection of filtered projections
    q[n_ang][nv][nu] at b_i = 2 pi i / n_ang -> mu[nz][ny][nx]."""
    q = np.asarray(q, np.float64)
    n_ang, nv, nu = q.shape
    R, D = float(geo["sod_mm"]), float(geo["sdd_mm"])
    pu, pv = float(geo["pu_mm"]), float(geo["pv_mm"])
    s = R / D
    nz, ny, nx = vol_shape
    xs = (np.arange(nx) + 0.5) * voxel_mm - nx * voxel_mm / 2
    ys = (np.arange(ny) + 0.5) * voxel_mm - ny * voxel_mm / 2
    zs = (np.arange(nz) + 0.5) * voxel_mm - nz * voxel_mm / 2
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    f = np.zeros(vol_shape, np.float64)
    for i in range(n_ang):
        beta = 2.0 * np.pi * i / n_ang
        cb, sb = np.cos(beta), np.sin(beta)
        L = R - (X * cb + Y * sb)
        av = R * (-X * sb + Y * cb) / L
        bv = R * Z / L
        fu = (av / s + nu * pu / 2) / pu - 0.5      # continuous pixel index, centres at integers
        fv = (bv / s + nv * pv / 2) / pv - 0.5
        iu0 = np.floor(fu).astype(int)
        iv0 = np.floor(fv).astype(int)
        wu = fu - iu0
        wv = fv - iv0
        val = np.zeros_like(f)
        for du, wgt_u in ((0, 1 - wu), (1, wu)):
            for dv, wgt_v in ((0, 1 - wv), (1, wv)):
                iu, iv = iu0 + du, iv0 + dv
                ok = (iu >= 0) & (iu < nu) & (iv >= 0) & (iv < nv)
                val += np.where(ok, q[i, np.clip(iv, 0, nv - 1), np.clip(iu, 0, nu - 1)], 0.0) * \
                    wgt_u * wgt_v
        f += (R * R) / (L * L) * val
    return 0.5 * (2.0 * np.pi / n_ang) * f


def fdk(proj, geo, vol_shape, voxel_mm):
    """proj[n_ang][nv][nu] line integrals at b_i = 2 pi i / n_ang -> mu[nz][ny][nx]
    (per mm), the volume centred on the origin with cubic voxels."""
    return fdk_backproject(fdk_filter(proj, geo), geo, vol_shape, voxel_mm)


def histogram(x, lo, hi, bins):
    """Counts of x in [lo, hi) split into equal bins (values outside dropped;
    bin of v = floor((v - lo) / (hi - lo) * bins))."""
    x = np.asarray(x, np.float64).ravel()
    k = np.floor((x - lo) / (hi - lo) * bins).astype(np.int64)
    k = k[(k >= 0) & (k < bins)]
    return np.bincount(k, minlength=bins)


def otsu_bin(counts):
    """Otsu: the first bin t maximising w0 w1 (m0 - m1)^2, class 0 = bins < t."""
    c = np.asarray(counts, np.float64)
    idx = np.arange(len(c), dtype=np.float64)
    best, arg = -1.0, 1
    for t in range(1, len(c)):
        w0, w1 = c[:t].sum(), c[t:].sum()
        if w0 == 0 or w1 == 0:
            continue
        m0 = (c[:t] * idx[:t]).sum() / w0
        m1 = (c[t:] * idx[t:]).sum() / w1
        v = w0 * w1 * (m0 - m1) ** 2
        if v > best:
            best, arg = v, t
    return arg


def to_density(mu, threshold, mu_rho_cm2g, material, air_rho=0.001205, step=0.005):
    """Voxels with mu >= threshold become `material` with density
    mu / (mu/rho) (mu per mm, mu/rho in cm^2/g), rounded to multiples of
    `step`; the others air (id 0)."""
    mu = np.asarray(mu, np.float64)
    obj = mu >= threshold
    rho = np.where(obj, np.round(mu / (0.1 * mu_rho_cm2g) / step) * step, air_rho)
    ids = np.where(obj, material, 0).astype(np.uint8)
    return ids, rho.astype(np.float32)
