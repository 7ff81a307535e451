"""Seeded synthetic inputs: phantoms, spectra and workload configurations.

This module holds none of the transport arithmetic.  It only builds the
arrays both the GPU library and the oracle consume: voxel material ids and
densities, energy bins with weights, and detector geometry.  Randomness comes
from numpy's Philox bit generator seeded per configuration.

Stand-ins for the paper's data (its voxelised engines, cylinder head and
cement objects; the Geant4 source spectrum) which are not available:
  * objects: a water cylinder (small case) and random ellipsoids of water,
    aluminium and a bone-like calcium mix, optionally with an iron insert,
    shaped after the industrial mixed-material objects of section III;
  * spectrum: Kramers' law bremsstrahlung, (kVp - E)/E per 1 keV bin, behind
    an aluminium filter whose attenuation is a two-term fit (photoelectric
    E^-3 term plus a constant) -- an input recipe, not the transport physics.
"""
from __future__ import annotations

import numpy as np

AIR_RHO = 0.001205

DEFAULT_MATERIALS = [
    dict(z_eff=7.64, z_over_a=0.49919, rho_default=0.001205, name="air"),
    dict(z_eff=7.42, z_over_a=0.55508, rho_default=1.0, name="water"),
    dict(z_eff=13.0, z_over_a=0.48181, rho_default=2.699, name="aluminium"),
    dict(z_eff=13.8, z_over_a=0.51480, rho_default=1.92, name="bone_ca"),
    dict(z_eff=26.0, z_over_a=0.46557, rho_default=7.874, name="iron"),
]


def _centres(n, h):
    return ((np.arange(n, dtype=np.float64) + 0.5) * h - n * h / 2.0)


def cylinder_phantom(n=64, h=1.0, radius_mm=25.0, material=1, density=1.0):
    """Cube of n^3 voxels of edge h; a cylinder along z of the given material
    where x^2 + y^2 <= r^2 at the voxel centre, air elsewhere."""
    c = _centres(n, h)
    X, Y = np.meshgrid(c, c, indexing="xy")          # [y][x]
    inside = (X * X + Y * Y) <= radius_mm * radius_mm
    ids = np.zeros((n, n, n), np.uint8)
    rho = np.full((n, n, n), AIR_RHO, np.float32)
    ids[:, inside] = material
    rho[:, inside] = density
    return ids, rho


def box_phantom(nx, ny, nz, material, density):
    """Homogeneous box: every voxel the same material and density."""
    return (np.full((nz, ny, nx), material, np.uint8),
            np.full((nz, ny, nx), density, np.float32))


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_phantom(n, h, seed, n_ellipsoids=20, materials=(1, 2, 3),
                      density_range=(0.9, 2.7), iron_insert=False,
                      shape=None):
    """Random ellipsoids painted in order (later ones overwrite) in air.

    Centres uniform in the central 80% of the box, semi-axes uniform in
    [0.05, 0.25] of the box edge, orientation a uniform random rotation,
    material uniform over `materials`, density uniform in `density_range`.
    With `iron_insert`, an iron cylinder (rho 7.874, r = 5 mm) along z through
    the centre is painted last.  `shape` = (nz, ny, nx) overrides n^3.
    """
    rng = np.random.Generator(np.random.Philox(seed))
    nz, ny, nx = shape if shape is not None else (n, n, n)
    ext = np.array([nx, ny, nz], np.float64) * h          # box edges (x, y, z)
    ids = np.zeros((nz, ny, nx), np.uint8)
    rho = np.full((nz, ny, nx), AIR_RHO, np.float32)
    cx, cy, cz = _centres(nx, h), _centres(ny, h), _centres(nz, h)
    for _ in range(n_ellipsoids):
        centre = (rng.random(3) - 0.5) * 0.8 * ext
        semi = rng.uniform(0.05, 0.25, 3) * ext.min()
        R = _random_rotation(rng)
        mat = int(rng.choice(np.asarray(materials)))
        dens = np.float32(rng.uniform(*density_range))
        r = semi.max()
        lo = np.searchsorted(cx, centre[0] - r), np.searchsorted(cy, centre[1] - r), \
            np.searchsorted(cz, centre[2] - r)
        hi = np.searchsorted(cx, centre[0] + r), np.searchsorted(cy, centre[1] + r), \
            np.searchsorted(cz, centre[2] + r)
        if min(b - a for a, b in zip(lo, hi)) <= 0:
            continue
        zz, yy, xx = np.meshgrid(cz[lo[2]:hi[2]] - centre[2], cy[lo[1]:hi[1]] - centre[1],
                                 cx[lo[0]:hi[0]] - centre[0], indexing="ij")
        # body coordinates: R^T (p - c)
        bx = R[0, 0] * xx + R[1, 0] * yy + R[2, 0] * zz
        by = R[0, 1] * xx + R[1, 1] * yy + R[2, 1] * zz
        bz = R[0, 2] * xx + R[1, 2] * yy + R[2, 2] * zz
        inside = (bx / semi[0]) ** 2 + (by / semi[1]) ** 2 + (bz / semi[2]) ** 2 <= 1.0
        sub_ids = ids[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub_rho = rho[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub_ids[inside] = mat
        sub_rho[inside] = dens
    if iron_insert:
        X, Y = np.meshgrid(cx, cy, indexing="xy")
        inside = (X * X + Y * Y) <= 25.0
        ids[:, inside] = 4
        rho[:, inside] = 7.874
    return ids, rho


def kramers_spectrum(kvp=150, al_mm=2.0, bin_kev=1.0):
    """Bins [k, k+1) keV with centres k + 0.5 for k = 1 .. kVp-1; weights
    (kVp - E)/E * exp(-mu_Al(E) t) with mu_Al/rho ~ 26583/E^3 + 0.1434 cm^2/g
    (a two-term fit used only to shape this synthetic input), rho_Al 2.699."""
    lo = np.arange(1.0, float(kvp), bin_kev)
    e = lo + 0.5 * bin_kev
    mu_rho = 26583.0 / e ** 3 + 0.1434
    w = (kvp - e) / e * np.exp(-mu_rho * 2.699 * (al_mm / 10.0))
    w = np.where(e < kvp, w, 0.0)
    return e.astype(np.float32), w.astype(np.float32)


def mono_spectrum(e_kev):
    return np.array([e_kev], np.float32), np.array([1.0], np.float32)


# --------------------------------------------------------------- workloads
def workload(name: str):
    """Concrete inputs of a named workload: dict with ids, rho, voxel_mm,
    geometry (keyword dict), spectrum (e, w), n_photons, seed, angle."""
    if name == "cylinder64":
        ids, rho = cylinder_phantom(64, 1.0)
        return dict(name=name, ids=ids, rho=rho, voxel_mm=1.0,
                    geometry=dict(sod_mm=500.0, sdd_mm=1000.0, nu=128, nv=128, pu_mm=1.0,
                                  pv_mm=1.0, snu=128, snv=128, step_mm=0.5, flags=0),
                    spectrum=mono_spectrum(60.0), n_photons=1_000_000, seed=0, angle=0.0)
    if name == "ellipsoids256_poly":
        ids, rho = ellipsoid_phantom(256, 0.5, seed=1)
        return dict(name=name, ids=ids, rho=rho, voxel_mm=0.5,
                    geometry=dict(sod_mm=500.0, sdd_mm=1000.0, nu=512, nv=512, pu_mm=0.4,
                                  pv_mm=0.4, snu=512, snv=512, step_mm=0.5, flags=0),
                    spectrum=kramers_spectrum(150, 2.0), n_photons=100_000_000, seed=0,
                    angle=0.0)
    if name == "ellipsoids512_hires":
        ids, rho = ellipsoid_phantom(512, 0.25, seed=2, materials=(1, 2, 3),
                                     iron_insert=True)
        return dict(name=name, ids=ids, rho=rho, voxel_mm=0.25,
                    geometry=dict(sod_mm=500.0, sdd_mm=1000.0, nu=2048, nv=2048, pu_mm=0.2,
                                  pv_mm=0.2, snu=256, snv=256, step_mm=0.25, flags=0),
                    spectrum=kramers_spectrum(150, 2.0), n_photons=1_000_000_000, seed=0,
                    angle=0.0)
    raise KeyError(name)


def batch_workload():
    """Batched launch: 360 angles x 1e7 photons of the 256^3 benchmark object,
    plus 16 random-ellipsoid objects of uneven size (64^3 .. 384^3 at 0.5 mm,
    one projection each at a random angle, 1e6 .. 5e7 photons log-uniform).
    Geometry and spectrum of the benchmark.  Returns dict with phantoms (list
    of (ids, rho, voxel_mm)), jobs (list of dicts: phantom, angle_rad,
    n_photons, seed), geometry, spectrum."""
    base = workload("ellipsoids256_poly")
    phantoms = [(base["ids"], base["rho"], base["voxel_mm"])]
    rng = np.random.Generator(np.random.Philox(360))
    sizes = [int(round(v / 8.0)) * 8 for v in np.linspace(64, 384, 16)]
    jobs = [dict(phantom=0, angle_rad=float(np.float32(2.0 * np.pi * k / 360.0)),
                 n_photons=10_000_000, seed=1000 + k) for k in range(360)]
    for i, n in enumerate(sizes):
        ids, rho = ellipsoid_phantom(n, 0.5, seed=100 + i)
        phantoms.append((ids, rho, 0.5))
        jobs.append(dict(phantom=i + 1, angle_rad=float(np.float32(rng.uniform(0, 2 * np.pi))),
                         n_photons=int(round(10 ** rng.uniform(6.0, np.log10(5e7)))),
                         seed=2000 + i))
    return dict(name="batch360_uneven16", phantoms=phantoms, jobs=jobs,
                geometry=base["geometry"], spectrum=base["spectrum"])

