"""ctypes binding of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package.  It loads oracle/liboracle_mco.so (built by oracle/build.py) and
shares nothing with the GPU library.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_mco.so")
# A test may point the binding at a deliberately broken build of the oracle to
# show that the pins catch it (tests/test_oracle_mutations.py).
_OVERRIDE = os.environ.get("MCO_ORACLE_LIB")

NO_SCATTER = 1
PROC_SOURCE_ENERGY, PROC_RAYLEIGH, PROC_COMPTON, PROC_SOURCE_DIR = 0, 1, 2, 3
END_PRIMARY, END_SCATTER, END_MISSED, END_PHOTO, END_CUTOFF, END_CAP = range(6)
FIRST_NONE, FIRST_PHOTO, FIRST_RAYLEIGH, FIRST_COMPTON = range(4)
READING_GRID, READING_PLAIN = 0, 1
SCORE_ANALOG, SCORE_POINT, SCORE_POINT_MIXED = 0, 1, 2
PHYS_INCOH_SF, PHYS_DOPPLER = 1, 2      # binding effects (set_physics)


class Material(C.Structure):
    _fields_ = [("z_eff", C.c_float), ("z_over_a", C.c_float),
                ("rho_default", C.c_float), ("name", C.c_char * 16)]


class Geometry(C.Structure):
    _fields_ = [("sod_mm", C.c_float), ("sdd_mm", C.c_float),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("pu_mm", C.c_float), ("pv_mm", C.c_float),
                ("snu", C.c_int32), ("snv", C.c_int32),
                ("step_mm", C.c_float), ("flags", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "histories", "steps", "flights", "photo", "rayleigh", "compton",
        "primary_hits", "scatter_hits", "cutoff_kills", "cap_hits",
        "pd_scores", "pd_killed", "pd_steps", "null_collisions")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _OVERRIDE or LIB_PATH
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.mco_create.argtypes = [C.POINTER(P)]
        L.mco_destroy.argtypes = [P]
        L.mco_destroy.restype = None
        L.mco_last_error.argtypes = [P]
        L.mco_last_error.restype = C.c_char_p
        L.mco_set_materials.argtypes = [P, C.POINTER(Material), C.c_int]
        L.mco_load_phantom.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int, C.c_float]
        L.mco_set_geometry.argtypes = [P, C.POINTER(Geometry)]
        L.mco_set_spectrum.argtypes = [P, P, P, C.c_int]
        L.mco_set_detector_response.argtypes = [P, P, C.c_int]
        L.mco_project_range.argtypes = [P, C.c_float, C.c_uint64, C.c_uint64, C.c_uint64, P, P]
        L.mco_project.argtypes = [P, C.c_float, C.c_uint64, C.c_uint64, P, P]
        L.mco_project_mt.argtypes = [P, C.c_float, C.c_uint64, C.c_uint64, P, P, C.c_int]
        L.mco_debug_histories.argtypes = [P, C.c_float, C.c_uint64, C.c_uint64, C.c_uint64,
                                          P, P, P, P]
        L.mco_debug_paths.argtypes = [P, C.c_float, C.c_uint64, C.c_uint64, C.c_uint64,
                                      P, P, P]
        L.mco_set_reading.argtypes = [P, C.c_int]
        L.mco_set_estimator.argtypes = [P, C.c_int, C.c_int, C.c_double]
        L.mco_set_physics.argtypes = [P, C.c_uint32]
        L.mco_primary_expected.argtypes = [P, C.c_float, C.c_int, P]
        L.mco_interp_angles.argtypes = [P, C.c_int, C.c_int64, P]
        L.mco_pd_pdf.argtypes = [P, C.c_int, C.c_int, C.c_float, C.c_double,
                                 C.POINTER(C.c_double), C.POINTER(C.c_float)]
        L.mco_pd_score_event.argtypes = [P, C.c_float, C.c_uint64, C.c_uint64, C.c_int, P, P,
                                         C.c_float, C.c_int, C.c_int, P]
        L.mco_test_rotate.argtypes = [P, C.c_float, C.c_double, P]
        L.mco_test_rotate.restype = None
        L.mco_test_sample.argtypes = [P, C.c_int, C.c_int, C.c_float, C.c_uint64,
                                      C.c_uint64, P, P]
        L.mco_detector_pixel.argtypes = [P, C.c_float, P, P, C.POINTER(C.c_int),
                                         C.POINTER(C.c_int)]
        L.mco_get_tables.argtypes = [P, C.POINTER(C.c_int), P, P, P, P]
        L.mco_cross_sections.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.mco_sigma_kn.argtypes = [C.c_double]
        L.mco_sigma_kn.restype = C.c_double
        L.mco_get_stats.argtypes = [P, C.POINTER(Stats)]
        L.mco_philox4x32_10.argtypes = [P, P, P]
        L.mco_philox4x32_10.restype = None
        L.mco_uniform_batch.argtypes = [P, C.c_uint64, P]
        L.mco_uniform_batch.restype = None
        L.mco_tally_scale.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


class Oracle:
    """One oracle context: materials, phantom, geometry, spectrum, eta."""

    def __init__(self):
        self._L = lib()
        h = C.c_void_p()
        rc = self._L.mco_create(C.byref(h))
        if rc:
            raise OracleError(rc, "create")
        self._h = h
        self.geometry = None

    def close(self):
        if self._h:
            self._L.mco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise OracleError(rc, self._L.mco_last_error(self._h).decode())

    # ---- state
    def set_materials(self, mats):
        arr = (Material * len(mats))()
        for i, m in enumerate(mats):
            arr[i] = Material(m["z_eff"], m["z_over_a"], m.get("rho_default", 1.0),
                              m.get("name", "").encode()[:15])
        self._check(self._L.mco_set_materials(self._h, arr, len(mats)))

    def load_phantom(self, ids, rho, voxel_mm):
        ids = np.ascontiguousarray(ids, dtype=np.uint8)
        rho = np.ascontiguousarray(rho, dtype=np.float32)
        nz, ny, nx = ids.shape
        self._check(self._L.mco_load_phantom(self._h, _ptr(ids), _ptr(rho), nx, ny, nz,
                                             float(voxel_mm)))
        self.shape = (nz, ny, nx)

    def set_geometry(self, **g):
        geo = Geometry(g["sod_mm"], g["sdd_mm"], g["nu"], g["nv"], g["pu_mm"], g["pv_mm"],
                       g.get("snu", g["nu"]), g.get("snv", g["nv"]), g["step_mm"],
                       g.get("flags", 0))
        self._check(self._L.mco_set_geometry(self._h, C.byref(geo)))
        self.geometry = dict(g, snu=geo.snu, snv=geo.snv)

    def set_spectrum(self, e_kev, w):
        e = np.ascontiguousarray(e_kev, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self._L.mco_set_spectrum(self._h, _ptr(e), _ptr(w), len(e)))

    def set_detector_response(self, eta):
        eta = np.ascontiguousarray(eta, dtype=np.float32)
        self._check(self._L.mco_set_detector_response(self._h, _ptr(eta), len(eta)))

    # ---- transport
    def _images(self):
        g = self.geometry
        return (np.zeros((g["nv"], g["nu"]), np.int64),
                np.zeros((g["snv"], g["snu"]), np.int64))

    def project(self, angle, n, seed, threads=1):
        p, s = self._images()
        if threads > 1:
            self._check(self._L.mco_project_mt(self._h, angle, n, seed, _ptr(p), _ptr(s),
                                               threads))
        else:
            self._check(self._L.mco_project(self._h, angle, n, seed, _ptr(p), _ptr(s)))
        return p, s

    def project_range(self, angle, first, n, seed, primary=None, scatter=None):
        if primary is None:
            primary, scatter = self._images()
        self._check(self._L.mco_project_range(self._h, angle, first, n, seed,
                                              _ptr(primary), _ptr(scatter)))
        return primary, scatter

    def debug_histories(self, angle, first, m, seed):
        n_int = np.zeros(m, np.uint16)
        steps = np.zeros(m, np.uint32)
        end = np.zeros(m, np.uint8)
        first_t = np.zeros(m, np.uint8)
        self._check(self._L.mco_debug_histories(self._h, angle, first, m, seed, _ptr(n_int),
                                                _ptr(steps), _ptr(end), _ptr(first_t)))
        return n_int, steps, end, first_t

    def debug_paths(self, angle, first, m, seed):
        """(first interaction point [m,3] (NaN if none), crossed pixel iv*nu+iu
        (-1 if none), energy at the end of the history) per history."""
        x1 = np.zeros((m, 3), np.float32)
        pix = np.zeros(m, np.int32)
        e_end = np.zeros(m, np.float32)
        self._check(self._L.mco_debug_paths(self._h, angle, first, m, seed, _ptr(x1),
                                            _ptr(pix), _ptr(e_end)))
        return x1, pix, e_end

    def set_reading(self, reading):
        self._check(self._L.mco_set_reading(self._h, reading))

    def set_physics(self, flags):
        """Binding effects: PHYS_INCOH_SF (S(x,Z) of eq. (1) as null
        collisions) | PHYS_DOPPLER (broadened Compton energies)."""
        self._check(self._L.mco_set_physics(self._h, int(flags)))

    def set_estimator(self, mode, split=1, rr_kev=0.0):
        """SCORE_ANALOG, or SCORE_POINT: the point-detector estimator of eq.
        (3)-(5) with `split` pseudo-particles per scattering and Russian
        roulette below rr_kev (0: off)."""
        self._check(self._L.mco_set_estimator(self._h, mode, split, float(rr_kev)))

    def primary_expected(self, angle, sub=2):
        """Eq. (7): expected primary tally per emitted photon (keV), [nv][nu] fp64."""
        g = self.geometry
        out = np.zeros((g["nv"], g["nu"]), np.float64)
        self._check(self._L.mco_primary_expected(self._h, angle, sub, _ptr(out)))
        return out

    def pd_pdf(self, process, material, e_kev, lam):
        """(pdf per unit scattering cosine, scattered energy) of the point
        detector's angular law for PROC_RAYLEIGH or PROC_COMPTON."""
        pdf, e2 = C.c_double(), C.c_float()
        self._check(self._L.mco_pd_pdf(self._h, process, material, e_kev, float(lam),
                                       C.byref(pdf), C.byref(e2)))
        return pdf.value, e2.value

    def pd_score_event(self, angle, seed, pid, n_prior, o, d, e_kev, material, process,
                       scatter=None):
        """Adds one scattering event's point-detector scores to a scatter image."""
        if scatter is None:
            scatter = self._images()[1]
        o = np.ascontiguousarray(o, dtype=np.float32)
        d = np.ascontiguousarray(d, dtype=np.float32)
        self._check(self._L.mco_pd_score_event(self._h, angle, seed, pid, n_prior, _ptr(o),
                                               _ptr(d), e_kev, material, process,
                                               _ptr(scatter)))
        return scatter

    def test_sample(self, process, material, e_kev, n, seed):
        cos = np.zeros(n, np.float32)
        e = np.zeros(n, np.float32)
        self._check(self._L.mco_test_sample(self._h, process, material, e_kev, n, seed,
                                            _ptr(cos), _ptr(e)))
        return cos, e

    def detector_pixel(self, angle, p, d):
        p = np.ascontiguousarray(p, dtype=np.float32)
        d = np.ascontiguousarray(d, dtype=np.float32)
        iu, iv = C.c_int(), C.c_int()
        self._check(self._L.mco_detector_pixel(self._h, angle, _ptr(p), _ptr(d),
                                               C.byref(iu), C.byref(iv)))
        return iu.value, iv.value

    def tables(self, n_mat):
        J = C.c_int()
        self._check(self._L.mco_get_tables(self._h, C.byref(J), None, None, None, None))
        J = J.value
        # the oracle writes every material it holds (at most 16): room for all
        pe, coh, inc = (np.zeros((16, J), np.float32) for _ in range(3))
        eta = np.zeros(J, np.float32)
        self._check(self._L.mco_get_tables(self._h, C.byref(C.c_int()), _ptr(pe), _ptr(coh),
                                           _ptr(inc), _ptr(eta)))
        return pe[:n_mat].copy(), coh[:n_mat].copy(), inc[:n_mat].copy(), eta

    def stats(self):
        s = Stats()
        self._check(self._L.mco_get_stats(self._h, C.byref(s)))
        return {n: getattr(s, n) for n, _ in Stats._fields_}


def cross_sections(z_eff, z_over_a, e_kev):
    out = np.zeros(3, np.float64)
    rc = lib().mco_cross_sections(z_eff, z_over_a, e_kev, _ptr(out))
    if rc:
        raise OracleError(rc, "cross_sections")
    return out


def sigma_kn(e_kev):
    return lib().mco_sigma_kn(e_kev)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().mco_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    out = np.zeros(x.shape, np.float32)
    lib().mco_uniform_batch(_ptr(x), x.size, _ptr(out))
    return out


def rotate(d, cos_theta, phi):
    """The transport's direction update after one scattering."""
    d = np.ascontiguousarray(d, dtype=np.float32)
    out = np.zeros(3, np.float32)
    lib().mco_test_rotate(_ptr(d), float(cos_theta), float(phi), _ptr(out))
    return out


def tally_scale():
    return lib().mco_tally_scale()


def interp_angles(sim):
    """Every-other-angle scatter maps [n_sim, ...] -> the full set [2 n_sim, ...]."""
    sim = np.ascontiguousarray(sim, dtype=np.float32)
    n_sim = sim.shape[0]
    n_pix = sim[0].size
    full = np.zeros((2 * n_sim,) + sim.shape[1:], np.float32)
    rc = lib().mco_interp_angles(_ptr(sim), n_sim, n_pix, _ptr(full))
    if rc:
        raise OracleError(rc, "interp_angles")
    return full
