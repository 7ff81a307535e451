"""ctypes binding of libmcx (include/mcx.h): argument marshalling only.

Every function of the C ABI is exposed under the same name (mc_create,
mc_load_phantom, mc_set_geometry, mc_set_spectrum, mc_project, ...); the
`Projector` class bundles one context.  All transport runs in the library's
HIP kernels; there is no CPU fallback: if libmcx.so is missing or cannot be
loaded, every call raises.  PyTorch, when used, only supplies device memory
(tensor data pointers) and streams.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MCX_LIB", os.path.join(HERE, "libmcx.so"))   # MCX_LIB: a variant build

MC_OK, MC_E_INVALID_ARG, MC_E_STATE, MC_E_OOM, MC_E_OVERFLOW, MC_E_DEVICE = 0, -1, -2, -3, -4, -6
MC_E_CANCELLED = -7
MC_NO_SCATTER = 1
MC_PROC_SOURCE_ENERGY, MC_PROC_RAYLEIGH, MC_PROC_COMPTON, MC_PROC_SOURCE_DIR = 0, 1, 2, 3
MC_END_PRIMARY, MC_END_SCATTER, MC_END_MISSED, MC_END_PHOTO, MC_END_CUTOFF, MC_END_CAP = range(6)

EXPORTS = ["mc_create", "mc_destroy", "mc_last_error", "mc_set_materials", "mc_load_phantom",
           "mc_set_geometry", "mc_set_spectrum", "mc_set_detector_response", "mc_project",
           "mc_project_async", "mc_project_range_async", "mc_debug_histories", "mc_test_sample",
           "mc_set_stats", "mc_get_stats", "mc_get_tables", "mc_set_layout", "mc_get_layout",
           "mc_set_launch", "mc_tally_scale", "mc_phantom_add", "mc_project_batch",
           "mc_get_shape", "mc_autotune", "mc_tally_to_float_async", "mc_savgol_async",
           "mc_upsample_cubic_async", "mc_savgol_weights", "mc_nn_conv3x3_async",
           "mc_nn_conv3x3_wgrad_async", "mc_nn_bias_grad_async", "mc_nn_flip_weights_async",
           "mc_nn_pool2_async", "mc_nn_upsample2_async", "mc_nn_mse_async", "mc_nn_adam_async",
           "mc_nn_relu_mask_async", "mc_nn_cast_bf16_async", "mc_nn_pack_channel_async",
           "mc_march_probe_async", "mc_cell_map", "mc_flip2d_async", "mc_atomic_probe_async",
           "mc_make_kramers", "mc_project_batch_static", "mc_set_estimator", "mc_set_physics", "mc_cancel",
           "mc_set_batch_launch", "mc_get_batch_info", "mc_autotune_batch",
           "mc_primary_expected_async", "mc_interp_angles_async", "mc_line_integrals_async",
           "mc_scatter_correct_async", "mc_fdk_async", "mc_histogram_async",
           "mc_to_density_async"]
MC_BATCH_GRAPH = 1
MC_LAYOUT_AUTO, MC_LAYOUT_PALETTE_LANE, MC_LAYOUT_PALETTE_SHARED, MC_LAYOUT_GENERIC = 0, 1, 2, 3


class mc_material(C.Structure):
    _fields_ = [("z_eff", C.c_float), ("z_over_a", C.c_float),
                ("rho_default", C.c_float), ("name", C.c_char * 16)]


class mc_geometry(C.Structure):
    _fields_ = [("sod_mm", C.c_float), ("sdd_mm", C.c_float),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("pu_mm", C.c_float), ("pv_mm", C.c_float),
                ("snu", C.c_int32), ("snv", C.c_int32),
                ("step_mm", C.c_float), ("flags", C.c_uint32)]


class mc_job(C.Structure):
    _fields_ = [("phantom", C.c_int32), ("angle_rad", C.c_float), ("n_photons", C.c_uint64),
                ("seed", C.c_uint64), ("primary_offset", C.c_uint64),
                ("scatter_offset", C.c_uint64)]


class mc_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("event_batch", C.c_int32),
                ("table_layout", C.c_int32),
                ("from_cache", C.c_int32), ("candidates", C.c_int32), ("rejected", C.c_int32),
                ("ms", C.c_double), ("histories_per_s", C.c_double)]


class mc_conv3x3(C.Structure):
    _fields_ = [("x", C.c_void_p), ("ldx", C.c_int32), ("xoff", C.c_int32), ("w", C.c_void_p),
                ("bias", C.c_void_p), ("y", C.c_void_p), ("ldy", C.c_int32), ("yoff", C.c_int32),
                ("yf", C.c_void_p), ("mask", C.c_void_p), ("ldm", C.c_int32), ("moff", C.c_int32),
                ("n", C.c_int32), ("h", C.c_int32), ("w_", C.c_int32), ("cin", C.c_int32),
                ("cout", C.c_int32), ("relu", C.c_int32), ("accumulate", C.c_int32)]


class mc_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "histories", "steps", "flights", "photo", "rayleigh", "compton",
        "primary_hits", "scatter_hits", "cutoff_kills", "cap_hits", "skipped_steps",
        "pd_scores", "pd_killed", "pd_steps", "null_collisions")]


class MCXError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmcx status {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libmcx.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MCXError(MC_E_STATE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P, U64, F, I = C.c_void_p, C.c_uint64, C.c_float, C.c_int
    sig = {
        "mc_create": ([C.POINTER(P), I], I),
        "mc_destroy": ([P], None),
        "mc_last_error": ([P], C.c_char_p),
        "mc_set_materials": ([P, C.POINTER(mc_material), I], I),
        "mc_load_phantom": ([P, P, P, I, I, I, F], I),
        "mc_set_geometry": ([P, C.POINTER(mc_geometry)], I),
        "mc_set_spectrum": ([P, P, P, I], I),
        "mc_set_detector_response": ([P, P, I], I),
        "mc_project": ([P, F, U64, U64, P, P], I),
        "mc_project_async": ([P, F, U64, U64, P, P, P], I),
        "mc_project_range_async": ([P, F, U64, U64, U64, P, P, P], I),
        "mc_march_probe_async": ([P, F, U64, U64, I, P, P], I),
        "mc_atomic_probe_async": ([P, U64, U64, P, U64, P], I),
        "mc_make_kramers": ([C.c_double, C.c_double, C.c_double, P, P, I, C.POINTER(C.c_int)], I),
        "mc_cell_map": ([P, I, I, I, P], I),
        "mc_flip2d_async": ([P, P, P, I, I, I, I, F, F, P], I),
        "mc_debug_histories": ([P, F, U64, U64, U64, P, P, P, P], I),
        "mc_test_sample": ([P, I, I, F, U64, U64, P, P], I),
        "mc_set_stats": ([P, I], I),
        "mc_get_stats": ([P, C.POINTER(mc_stats)], I),
        "mc_get_tables": ([P, C.POINTER(I), C.POINTER(I), P, P, P, P], I),
        "mc_set_layout": ([P, I], I),
        "mc_get_layout": ([P, C.POINTER(I), C.POINTER(I)], I),
        "mc_set_launch": ([P, I, I, I], I),
        "mc_tally_scale": ([], C.c_double),
        "mc_phantom_add": ([P, P, P, I, I, I, F, C.POINTER(I)], I),
        "mc_project_batch": ([P, C.POINTER(mc_job), I, P, U64, C.c_uint32, P], I),
        "mc_project_batch_static": ([P, C.POINTER(mc_job), I, P, U64, P], I),
        "mc_set_estimator": ([P, I, I, C.c_double], I),
        "mc_set_physics": ([P, C.c_uint32], I),
        "mc_cancel": ([P, I], I),
        "mc_set_batch_launch": ([P, I, I, I], I),
        "mc_primary_expected_async": ([P, F, I, P, P], I),
        "mc_line_integrals_async": ([P, P, U64, P, U64, P, P], I),
        "mc_scatter_correct_async": ([P, P, P, P, U64, P, P], I),
        "mc_fdk_async": ([P, P, I, P, P, I, I, I, F, P], I),
        "mc_histogram_async": ([P, P, U64, F, F, I, P, P], I),
        "mc_to_density_async": ([P, P, U64, F, F, I, F, P, P, P], I),
        "mc_interp_angles_async": ([P, P, I, U64, P, P], I),
        "mc_get_batch_info": ([P, C.POINTER(I), C.POINTER(U64), C.POINTER(I)], I),
        "mc_autotune_batch": ([P, C.POINTER(mc_job), I, P, U64, C.c_char_p, C.POINTER(mc_tuning)], I),
        "mc_get_shape": ([P] + [C.POINTER(I)] * 7, I),
        "mc_tally_to_float_async": ([P, P, P, U64, C.c_double, P], I),
        "mc_savgol_async": ([P, P, P, P, I, I, I, I, P], I),
        "mc_upsample_cubic_async": ([P, P, P, I, I, I, P], I),
        "mc_savgol_weights": ([I, I, P], I),
        "mc_nn_conv3x3_async": ([P, C.POINTER(mc_conv3x3), P], I),
        "mc_nn_conv3x3_wgrad_async": ([P, P, I, I, P, I, I, I, I, I, I, I, I, P, P, P], I),
        "mc_nn_bias_grad_async": ([P, P, I, I, I, I, P, I, P, P], I),
        "mc_nn_flip_weights_async": ([P, P, P, I, I, I, I, P], I),
        "mc_nn_pool2_async": ([P, P, I, I, P, I, I, I, I, I, I, I, I, P], I),
        "mc_nn_upsample2_async": ([P, P, I, I, P, I, I, I, I, I, I, I, I, P], I),
        "mc_nn_mse_async": ([P, P, I, P, U64, P, I, I, F, P, P], I),
        "mc_nn_adam_async": ([P, P, P, P, P, P, U64, F, F, F, F, I, F, P], I),
        "mc_nn_relu_mask_async": ([P, P, I, I, P, I, I, U64, I, P], I),
        "mc_nn_cast_bf16_async": ([P, P, P, U64, P], I),
        "mc_nn_pack_channel_async": ([P, P, U64, F, P, I, I, P], I),
        "mc_autotune": ([P, F, U64, U64, C.c_char_p, C.POINTER(mc_tuning)], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _np(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    return C.c_void_p(t if isinstance(t, int) else t.data_ptr())


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return C.c_void_p(s)
    return C.c_void_p(s.cuda_stream)


# ---- the C ABI under its own names -------------------------------------------------
def mc_create(device=0):
    h = C.c_void_p()
    rc = load().mc_create(C.byref(h), device)
    if rc:
        raise MCXError(rc, f"mc_create(device={device}) failed")
    return h


def mc_destroy(ctx):
    load().mc_destroy(ctx)


def mc_last_error(ctx):
    return load().mc_last_error(ctx).decode()


def _check(ctx, rc):
    if rc:
        raise MCXError(rc, mc_last_error(ctx))


def mc_set_materials(ctx, materials):
    arr = (mc_material * len(materials))()
    for i, m in enumerate(materials):
        arr[i] = mc_material(m["z_eff"], m["z_over_a"], m.get("rho_default", 1.0),
                             m.get("name", "").encode()[:15])
    _check(ctx, load().mc_set_materials(ctx, arr, len(materials)))


def mc_load_phantom(ctx, ids, rho, voxel_mm):
    ids = np.ascontiguousarray(ids, dtype=np.uint8)
    rho = np.ascontiguousarray(rho, dtype=np.float32)
    nz, ny, nx = ids.shape
    _check(ctx, load().mc_load_phantom(ctx, _np(ids), _np(rho), nx, ny, nz, float(voxel_mm)))


def mc_phantom_add(ctx, ids, rho, voxel_mm):
    ids = np.ascontiguousarray(ids, dtype=np.uint8)
    rho = np.ascontiguousarray(rho, dtype=np.float32)
    nz, ny, nx = ids.shape
    h = C.c_int()
    _check(ctx, load().mc_phantom_add(ctx, _np(ids), _np(rho), nx, ny, nz, float(voxel_mm),
                                      C.byref(h)))
    return h.value


def mc_project_batch(ctx, jobs, d_out, out_elems, flags=MC_BATCH_GRAPH, stream=None):
    """jobs: sequence of dicts with phantom, angle_rad, n_photons, seed,
    primary_offset, scatter_offset; d_out: device int64 buffer (torch tensor)."""
    arr = (mc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = mc_job(j["phantom"], j["angle_rad"], j["n_photons"], j["seed"],
                        j["primary_offset"], j["scatter_offset"])
    _check(ctx, load().mc_project_batch(ctx, arr, len(jobs), _dev(d_out), out_elems, flags,
                                        _stream(stream)))


MC_SCORE_ANALOG, MC_SCORE_POINT, MC_SCORE_POINT_MIXED = 0, 1, 2
MC_PHYS_INCOH_SF, MC_PHYS_DOPPLER = 1, 2


def mc_cancel(ctx, on=True):
    """Stop (on) the context's running and queued transport launches, or clear
    the request (off); safe to call from another thread during a call."""
    _check(ctx, load().mc_cancel(ctx, 1 if on else 0))


def mc_set_physics(ctx, flags):
    """Binding effects: MC_PHYS_INCOH_SF | MC_PHYS_DOPPLER (0: Klein-Nishina)."""
    _check(ctx, load().mc_set_physics(ctx, int(flags)))


def mc_set_estimator(ctx, mode, split=1, rr_kev=0.0):
    """MC_SCORE_ANALOG, or MC_SCORE_POINT: the point-detector scatter estimator
    with `split` pseudo-particles per scattering and roulette below rr_kev."""
    _check(ctx, load().mc_set_estimator(ctx, mode, split, float(rr_kev)))


MC_STATIC_MAX_JOBS = 1024
MC_STATIC_MAX_PHANTOMS = 64


def mc_project_batch_static(ctx, jobs, d_out, out_elems, stream=None):
    """mc_project_batch without device allocation (tables in the library's
    fixed device array; calls on one GPU must not overlap)."""
    arr = (mc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = mc_job(j["phantom"], j["angle_rad"], j["n_photons"], j["seed"],
                        j["primary_offset"], j["scatter_offset"])
    _check(ctx, load().mc_project_batch_static(ctx, arr, len(jobs), _dev(d_out), out_elems,
                                               _stream(stream)))


def mc_set_geometry(ctx, sod_mm, sdd_mm, nu, nv, pu_mm, pv_mm, step_mm, snu=None, snv=None,
                    flags=0):
    g = mc_geometry(sod_mm, sdd_mm, nu, nv, pu_mm, pv_mm, snu or nu, snv or nv, step_mm, flags)
    _check(ctx, load().mc_set_geometry(ctx, C.byref(g)))
    return g


def mc_set_spectrum(ctx, e_kev, w):
    e = np.ascontiguousarray(e_kev, dtype=np.float32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(ctx, load().mc_set_spectrum(ctx, _np(e), _np(w), len(e)))


def mc_set_detector_response(ctx, eta):
    eta = np.ascontiguousarray(eta, dtype=np.float32)
    _check(ctx, load().mc_set_detector_response(ctx, _np(eta), len(eta)))


def mc_project(ctx, angle, n_photons, seed, primary, scatter):
    """Blocking; primary/scatter are host int64 numpy arrays written in place."""
    assert primary.dtype == np.int64 and scatter.dtype == np.int64
    assert primary.flags.c_contiguous and scatter.flags.c_contiguous
    _check(ctx, load().mc_project(ctx, angle, n_photons, seed, _np(primary), _np(scatter)))


def mc_project_async(ctx, angle, n_photons, seed, d_primary, d_scatter, stream=None):
    _check(ctx, load().mc_project_async(ctx, angle, n_photons, seed, _dev(d_primary),
                                        _dev(d_scatter), _stream(stream)))


def mc_cell_map(codes):
    """codes: uint8 [nz, ny, nx] -> uint16 cell words [ceil(nz/4), ceil(ny/4), ceil(nx/4)]."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    nz, ny, nx = codes.shape
    out = np.zeros(((nz + 3) // 4, (ny + 3) // 4, (nx + 3) // 4), np.uint16)
    rc = load().mc_cell_map(_np(codes), nx, ny, nz, _np(out))
    if rc:
        raise MCXError(rc, "bad cell-map arguments")
    return out


def mc_atomic_probe_async(ctx, n_adds, seed, d_image, n_pixels, stream=None):
    _check(ctx, load().mc_atomic_probe_async(ctx, n_adds, seed, _dev(d_image), n_pixels,
                                             _stream(stream)))


def mc_march_probe_async(ctx, angle, n_rays, seed, refill_batch, d_sum, stream=None):
    _check(ctx, load().mc_march_probe_async(ctx, angle, n_rays, seed, refill_batch, _dev(d_sum),
                                            _stream(stream)))


def mc_project_range_async(ctx, angle, first, n, seed, d_primary, d_scatter, stream=None):
    _check(ctx, load().mc_project_range_async(ctx, angle, first, n, seed, _dev(d_primary),
                                              _dev(d_scatter), _stream(stream)))


def mc_debug_histories(ctx, angle, first, m, seed):
    n_int = np.zeros(m, np.uint16)
    steps = np.zeros(m, np.uint32)
    end = np.zeros(m, np.uint8)
    first_t = np.zeros(m, np.uint8)
    _check(ctx, load().mc_debug_histories(ctx, angle, first, m, seed, _np(n_int), _np(steps),
                                          _np(end), _np(first_t)))
    return n_int, steps, end, first_t


def mc_test_sample(ctx, process, material, e_kev, n, seed):
    cos = np.zeros(n, np.float32)
    e = np.zeros(n, np.float32)
    _check(ctx, load().mc_test_sample(ctx, process, material, e_kev, n, seed, _np(cos), _np(e)))
    return cos, e


def mc_set_stats(ctx, enable):
    _check(ctx, load().mc_set_stats(ctx, int(bool(enable))))


def mc_get_stats(ctx):
    s = mc_stats()
    _check(ctx, load().mc_get_stats(ctx, C.byref(s)))
    return {n: getattr(s, n) for n, _ in mc_stats._fields_}


def mc_get_tables(ctx, n_mat=None):
    """(pe, coh, inc, eta): [n_mat][J] tables of every material of the context
    (the first n_mat rows when n_mat is given) and eta[J]."""
    J, M = C.c_int(), C.c_int()
    _check(ctx, load().mc_get_tables(ctx, C.byref(J), C.byref(M), None, None, None, None))
    J, M = J.value, M.value
    if n_mat is not None and not 1 <= n_mat <= M:
        raise ValueError(f"the context has {M} materials, asked for {n_mat}")
    pe, coh, inc = (np.zeros((M, J), np.float32) for _ in range(3))
    eta = np.zeros(J, np.float32)
    _check(ctx, load().mc_get_tables(ctx, C.byref(C.c_int()), C.byref(C.c_int()), _np(pe),
                                     _np(coh), _np(inc), _np(eta)))
    k = M if n_mat is None else n_mat
    return pe[:k].copy(), coh[:k].copy(), inc[:k].copy(), eta


def mc_set_layout(ctx, layout):
    _check(ctx, load().mc_set_layout(ctx, layout))


def mc_get_layout(ctx):
    lay, npal = C.c_int(), C.c_int()
    _check(ctx, load().mc_get_layout(ctx, C.byref(lay), C.byref(npal)))
    return lay.value, npal.value


def mc_set_launch(ctx, block=0, blocks_per_cu=0, event_batch=0):
    _check(ctx, load().mc_set_launch(ctx, block, blocks_per_cu, event_batch))


def mc_get_shape(ctx):
    v = [C.c_int() for _ in range(7)]
    _check(ctx, load().mc_get_shape(ctx, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def mc_autotune(ctx, angle, n_photons, seed, cache_path=None):
    t = mc_tuning()
    path = cache_path.encode() if cache_path else None
    _check(ctx, load().mc_autotune(ctx, angle, n_photons, seed, path, C.byref(t)))
    return {n: getattr(t, n) for n, _ in mc_tuning._fields_}


def mc_primary_expected_async(ctx, angle, sub, d_out, stream=None):
    """Eq. (7): expected primary keV per emitted photon into device fp32 [nv, nu]."""
    _check(ctx, load().mc_primary_expected_async(ctx, angle, sub, _dev(d_out), _stream(stream)))


def mc_interp_angles_async(ctx, d_sim, n_sim, n_pix, d_full, stream=None):
    """Every-other-angle scatter maps [n_sim, n_pix] -> [2 n_sim, n_pix] (device fp32)."""
    _check(ctx, load().mc_interp_angles_async(ctx, _dev(d_sim), n_sim, n_pix, _dev(d_full),
                                              _stream(stream)))


def mc_line_integrals_async(ctx, d_I, d_I0, d_a, stream=None):
    """a = -ln(I / I0) (device fp32; I0 one projection, repeated)."""
    _check(ctx, load().mc_line_integrals_async(ctx, _dev(d_I), d_I.numel(), _dev(d_I0),
                                               d_I0.numel(), _dev(d_a), _stream(stream)))


def mc_scatter_correct_async(ctx, d_a, d_ip, d_is, d_c, stream=None):
    """Eq. (8): c = a - ln(Ip / (Ip + Is)) (device fp32, same sizes)."""
    _check(ctx, load().mc_scatter_correct_async(ctx, _dev(d_a), _dev(d_ip), _dev(d_is),
                                                d_a.numel(), _dev(d_c), _stream(stream)))


def mc_fdk_async(ctx, d_proj, d_tmp, d_vol, voxel_mm, stream=None):
    """FDK of d_proj [n_ang, nv, nu] into d_vol [nz, ny, nx] (device fp32)."""
    n_ang = d_proj.shape[0]
    nz, ny, nx = d_vol.shape
    _check(ctx, load().mc_fdk_async(ctx, _dev(d_proj), n_ang, _dev(d_tmp), _dev(d_vol), nx, ny,
                                    nz, voxel_mm, _stream(stream)))


def mc_histogram_async(ctx, d_x, lo, hi, bins, d_hist, stream=None):
    _check(ctx, load().mc_histogram_async(ctx, _dev(d_x), d_x.numel(), lo, hi, bins, _dev(d_hist),
                                          _stream(stream)))


def mc_to_density_async(ctx, d_mu, threshold, mu_rho, material, step, d_ids, d_rho, stream=None):
    _check(ctx, load().mc_to_density_async(ctx, _dev(d_mu), d_mu.numel(), threshold, mu_rho,
                                           material, step, _dev(d_ids), _dev(d_rho),
                                           _stream(stream)))


def mc_set_batch_launch(ctx, block=0, blocks_per_cu=0, event_batch=0):
    _check(ctx, load().mc_set_batch_launch(ctx, block, blocks_per_cu, event_batch))


def mc_get_batch_info(ctx):
    n, v, p = C.c_int(), C.c_uint64(), C.c_int()
    _check(ctx, load().mc_get_batch_info(ctx, C.byref(n), C.byref(v), C.byref(p)))
    return n.value, v.value, p.value


def mc_autotune_batch(ctx, jobs, d_out, out_elems, cache_path=None):
    """Batch autotuner: jobs as for mc_project_batch; d_out is overwritten."""
    arr = (mc_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = mc_job(j["phantom"], j["angle_rad"], j["n_photons"], j["seed"],
                        j["primary_offset"], j["scatter_offset"])
    t = mc_tuning()
    path = cache_path.encode() if cache_path else None
    _check(ctx, load().mc_autotune_batch(ctx, arr, len(jobs), _dev(d_out), out_elems, path,
                                         C.byref(t)))
    return {n: getattr(t, n) for n, _ in mc_tuning._fields_}


def mc_tally_to_float_async(ctx, d_in, d_out, n, scale, stream=None):
    _check(ctx, load().mc_tally_to_float_async(ctx, _dev(d_in), _dev(d_out), n, scale,
                                               _stream(stream)))


def mc_savgol_async(ctx, d_in, d_out, d_tmp, nx, ny, window, order, stream=None):
    _check(ctx, load().mc_savgol_async(ctx, _dev(d_in), _dev(d_out), _dev(d_tmp), nx, ny, window,
                                       order, _stream(stream)))


def mc_upsample_cubic_async(ctx, d_in, d_out, nx, ny, factor, stream=None):
    _check(ctx, load().mc_upsample_cubic_async(ctx, _dev(d_in), _dev(d_out), nx, ny, factor,
                                               _stream(stream)))


def mc_flip2d_async(ctx, d_in, d_out, nx, ny, flip_x, flip_y, alpha=1.0, beta=0.0, stream=None):
    _check(ctx, load().mc_flip2d_async(ctx, _dev(d_in), _dev(d_out), nx, ny, int(flip_x),
                                       int(flip_y), float(alpha), float(beta), _stream(stream)))


def mc_make_kramers(kvp, al_mm=0.0, bin_kev=1.0):
    """(bin centres, weights) as float32 arrays; see include/mcx.h."""
    n = C.c_int(0)
    rc = load().mc_make_kramers(kvp, al_mm, bin_kev, None, None, 0, C.byref(n))
    if rc:
        raise MCXError(rc, "bad spectrum parameters")
    e, w = np.zeros(n.value, np.float32), np.zeros(n.value, np.float32)
    rc = load().mc_make_kramers(kvp, al_mm, bin_kev, _np(e), _np(w), n.value, C.byref(n))
    if rc:
        raise MCXError(rc, "bad spectrum parameters")
    return e, w


def mc_savgol_weights(window, order):
    w = np.zeros(window, np.float32)
    rc = load().mc_savgol_weights(window, order, _np(w))
    if rc:
        raise MCXError(rc, "bad window/order")
    return w


def _p(t):
    return None if t is None else (t if isinstance(t, int) else t.data_ptr())


def mc_nn_conv3x3_async(ctx, x, ldx, xoff, w, bias, y, ldy, yoff, n, h, w_, cin, cout, relu=0,
                        yf=None, mask=None, ldm=0, moff=0, accumulate=0, stream=None):
    a = mc_conv3x3(_p(x), ldx, xoff, _p(w), _p(bias), _p(y), ldy, yoff, _p(yf), _p(mask), ldm,
                   moff, n, h, w_, cin, cout, int(relu), int(accumulate))
    _check(ctx, load().mc_nn_conv3x3_async(ctx, C.byref(a), _stream(stream)))


def mc_nn_conv3x3_wgrad_async(ctx, x, ldx, xoff, dy, ldy, yoff, n, h, w, cin, cout, splits,
                              workspace, dw, stream=None):
    _check(ctx, load().mc_nn_conv3x3_wgrad_async(ctx, _p(x), ldx, xoff, _p(dy), ldy, yoff, n, h,
                                                 w, cin, cout, splits, _p(workspace), _p(dw),
                                                 _stream(stream)))


def mc_nn_bias_grad_async(ctx, dy, ldy, yoff, npix, c, workspace, rows, db, stream=None):
    _check(ctx, load().mc_nn_bias_grad_async(ctx, _p(dy), ldy, yoff, npix, c, _p(workspace), rows,
                                             _p(db), _stream(stream)))


def mc_nn_flip_weights_async(ctx, w, wt, cout, cin, cout_pad, cin_pad, stream=None):
    _check(ctx, load().mc_nn_flip_weights_async(ctx, _p(w), _p(wt), cout, cin, cout_pad, cin_pad,
                                                _stream(stream)))


def mc_nn_pool2_async(ctx, x, ldx, xoff, y, ldy, yoff, n, h, w, c, backward=0, accumulate=0,
                      stream=None):
    _check(ctx, load().mc_nn_pool2_async(ctx, _p(x), ldx, xoff, _p(y), ldy, yoff, n, h, w, c,
                                         int(backward), int(accumulate), _stream(stream)))


def mc_nn_upsample2_async(ctx, x, ldx, xoff, y, ldy, yoff, n, h, w, c, backward=0, accumulate=0,
                          stream=None):
    _check(ctx, load().mc_nn_upsample2_async(ctx, _p(x), ldx, xoff, _p(y), ldy, yoff, n, h, w, c,
                                             int(backward), int(accumulate), _stream(stream)))


def mc_nn_mse_async(ctx, out, ldo, target, n, grad, ldg, goff, gscale, partial, stream=None):
    _check(ctx, load().mc_nn_mse_async(ctx, _p(out), ldo, _p(target), n, _p(grad), ldg, goff,
                                       gscale, _p(partial), _stream(stream)))


def mc_nn_adam_async(ctx, p, g, m, v, pb, n, lr, b1, b2, eps, step, gscale=1.0, stream=None):
    _check(ctx, load().mc_nn_adam_async(ctx, _p(p), _p(g), _p(m), _p(v), _p(pb), n, lr, b1, b2,
                                        eps, step, gscale, _stream(stream)))


def mc_nn_relu_mask_async(ctx, g, ldg, goff, y, ldy, yoff, npix, c, stream=None):
    _check(ctx, load().mc_nn_relu_mask_async(ctx, _p(g), ldg, goff, _p(y), ldy, yoff, npix, c,
                                             _stream(stream)))


def mc_nn_cast_bf16_async(ctx, x, out, n, stream=None):
    _check(ctx, load().mc_nn_cast_bf16_async(ctx, _p(x), _p(out), n, _stream(stream)))


def mc_nn_pack_channel_async(ctx, x, npix, scale, out, ld, coff, stream=None):
    _check(ctx, load().mc_nn_pack_channel_async(ctx, _p(x), npix, scale, _p(out), ld, coff,
                                                _stream(stream)))


def mc_tally_scale():
    return load().mc_tally_scale()


# ---- convenience wrapper ---------------------------------------------------------
class Projector:
    """One libmcx context with its geometry remembered for image shapes."""

    def __init__(self, device=0):
        self.ctx = mc_create(device)
        self.geometry = None

    def close(self):
        if self.ctx:
            mc_destroy(self.ctx)
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may be torn down before this
        # object (and module globals cleared): the process's end releases the
        # context then
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_materials(self, mats):
        mc_set_materials(self.ctx, mats)

    def load_phantom(self, ids, rho, voxel_mm):
        mc_load_phantom(self.ctx, ids, rho, voxel_mm)

    def set_geometry(self, **g):
        geo = mc_set_geometry(self.ctx, g["sod_mm"], g["sdd_mm"], g["nu"], g["nv"], g["pu_mm"],
                              g["pv_mm"], g["step_mm"], g.get("snu"), g.get("snv"),
                              g.get("flags", 0))
        self.geometry = dict(g, snu=geo.snu, snv=geo.snv)

    def set_spectrum(self, e, w):
        mc_set_spectrum(self.ctx, e, w)

    def set_detector_response(self, eta):
        mc_set_detector_response(self.ctx, eta)

    def images(self):
        g = self.geometry
        return (np.zeros((g["nv"], g["nu"]), np.int64), np.zeros((g["snv"], g["snu"]), np.int64))

    def project(self, angle, n, seed):
        p, s = self.images()
        mc_project(self.ctx, angle, n, seed, p, s)
        return p, s

    def debug_histories(self, angle, first, m, seed):
        return mc_debug_histories(self.ctx, angle, first, m, seed)

    def test_sample(self, process, material, e_kev, n, seed):
        return mc_test_sample(self.ctx, process, material, e_kev, n, seed)

    def tables(self, n_mat=None):
        return mc_get_tables(self.ctx, n_mat)

    def set_estimator(self, mode, split=1, rr_kev=0.0):
        mc_set_estimator(self.ctx, mode, split, rr_kev)

    def set_physics(self, flags):
        mc_set_physics(self.ctx, flags)

    def cancel(self, on=True):
        mc_cancel(self.ctx, on)

    def set_layout(self, layout):
        mc_set_layout(self.ctx, layout)

    def layout(self):
        return mc_get_layout(self.ctx)

    def set_launch(self, block=0, blocks_per_cu=0, event_batch=0):
        mc_set_launch(self.ctx, block, blocks_per_cu, event_batch)

    def stats(self, enable=None):
        if enable is not None:
            mc_set_stats(self.ctx, enable)
            return None
        return mc_get_stats(self.ctx)
