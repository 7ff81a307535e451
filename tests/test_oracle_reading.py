"""The oracle's march reading against the plain reading of the fixed-step march.

The paper fixes only that the ray-march step is a free parameter (section
II-C-2).  The oracle (and the GPU kernel, bitwise) follow a reading that
makes every image exact per seed: step voxels at the nominal step centres
(k + 1/2) * step added up in fp32 with re-anchoring every 4 steps, and the
optical depth summed on the 2^-32 grid.  The plain reading takes the true
midpoint of each (clipped) step and sums mu * length in fp64 with no
anchoring (oracle/mco.c, march_plain; selected with mco_set_reading).  Both
are the same discretisation up to rounding, except that the clipped last
step looks up its voxel at the nominal centre in one and at its true
midpoint in the other.

Here both readings run the same photons with the same seeds and must agree
within the parity tolerances of the transport: primary rel-L2 <= 1e-3,
scatter rel-RMS <= 0.5 % at equal photon count, >= 99.9 % of histories with
identical records (scatterings, end code, first interaction type).  With a
step longer than a voxel the last-step difference matters more: there the
records, the primary and the total scatter still meet the tolerances and the
scatter image does on 8 x 8 pixel blocks; the per-pixel figure is printed.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13191_amd import inputs


def _both(w, n, n_rec, threads=8):
    out = []
    for reading in (oracle.READING_GRID, oracle.READING_PLAIN):
        o = oracle.Oracle()
        o.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
        o.set_geometry(**w["geometry"])
        o.set_spectrum(*w["spectrum"])
        o.set_reading(reading)
        p, s = o.project(w["angle"], n, w["seed"], threads=threads)
        n_int, _, end, first = o.debug_histories(w["angle"], 0, n_rec, w["seed"])
        out.append((p.astype(np.float64), s.astype(np.float64), n_int, end, first))
    return out


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _random_case(step_mm):
    base = inputs.workload("cylinder64")
    ids, rho = inputs.ellipsoid_phantom(48, 1.5, seed=77)
    return dict(ids=ids, rho=rho, voxel_mm=1.5, angle=0.7, seed=5,
                geometry=dict(base["geometry"], step_mm=step_mm),
                spectrum=inputs.workload("ellipsoids256_poly")["spectrum"])


CASES = [("cylinder64", 1_000_000), ("ellipsoids256_poly", 1_000_000),
         ("ellipsoids512_hires", 400_000), ("random48_step0.37", 1_000_000)]


@pytest.mark.parametrize("name,n", CASES, ids=[c[0] for c in CASES])
def test_grid_reading_matches_plain_reading(oracle_lib, name, n):
    w = _random_case(0.37) if name.startswith("random48") else inputs.workload(name)
    (p0, s0, n0, e0, f0), (p1, s1, n1, e1, f1) = _both(w, n, 100_000)
    same = np.mean((n0 == n1) & (e0 == e1) & (f0 == f1))
    rp, rs = _rel(p0, p1), _rel(s0, s1)
    print(f"{name}: primary rel-L2 {rp:.2e}, scatter rel-RMS {rs:.2e}, records {same:.6f}")
    assert p1.sum() > 0 and s1.sum() > 0
    assert rp <= 1e-3
    assert rs <= 5e-3
    assert same >= 0.999


def test_long_step_readings(oracle_lib):
    """Step 1.53 voxels: the clipped last step's lookup point differs."""
    w = _random_case(2.3)
    (p0, s0, n0, e0, f0), (p1, s1, n1, e1, f1) = _both(w, 1_000_000, 100_000)
    same = np.mean((n0 == n1) & (e0 == e1) & (f0 == f1))
    blocks = lambda s: s.reshape(16, 8, 16, 8).sum(axis=(1, 3))
    rs_px, rs_blk = _rel(s0, s1), _rel(blocks(s0), blocks(s1))
    print(f"step 2.3 mm: primary {_rel(p0, p1):.2e}, scatter per pixel {rs_px:.2e}, "
          f"8x8 blocks {rs_blk:.2e}, records {same:.6f}")
    assert same >= 0.999
    assert _rel(p0, p1) <= 1e-3
    assert abs(s0.sum() / s1.sum() - 1) <= 5e-3
    assert rs_blk <= 5e-3
