"""Thin ctypes binding of libpbr.so (include/pbr.h).

Functions carry the C names and only marshal arguments: device buffers are torch tensors
(``tensor.data_ptr()``), the stream is torch's current HIP stream.  Every step of the path runs
in the library's HIP kernels; there is no Python or CPU fallback, and loading fails loudly when
the library has not been built.

``Renderer`` bundles one context with the caller-owned buffers the C ABI asks for (field
workspace, Q32.32 sensor accumulator, exit-record buffer).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbr.so")
CHECKED_LIB_PATH = os.path.join(_HERE, "libpbr_checked.so")  # bounds-checked trace kernels

PBR_OK, PBR_ERR_ARG, PBR_ERR_STATE, PBR_ERR_HIP, PBR_ERR_WORKSPACE, PBR_ERR_OVERFLOW = 0, -1, -2, -3, -4, -5
PBR_ERR_BOUNDS = -6
(PBR_RAY_DEPOSITED, PBR_RAY_OFF_SENSOR, PBR_RAY_BLOCKED_APERTURE, PBR_RAY_BLOCKED_LENS,
 PBR_RAY_TIR, PBR_RAY_STEP_LIMIT, PBR_RAY_MISSED) = range(7)
PBR_NUM_STATUS = 7
PBR_CLEAR_FIRST, PBR_RECORD_EXITS, PBR_PREC_FP64_ALL, PBR_PREC_SHOCK_FP64, PBR_SURROGATE = 1, 2, 4, 8, 16
PBR_LANE_REFILL = 32
PBR_SOURCE_SUMS = 64
PBR_MIE = 128
PBR_SOURCE_ORDER = 256
PBR_MAX_SURFACES = 16
PBR_SURF_REFRACT, PBR_SURF_MIRROR, PBR_SURF_APERTURE, PBR_SURF_LENSLETS = 0, 1, 2, 3
PBR_MIE_TABLE_SIZE = 2049
PBR_NOALLOC_MAX_CHUNK = 1 << 20
PBR_SURR_PARAMS = 200710
PBR_FMT_RAW_U64, PBR_FMT_F32, PBR_FMT_U16 = 0, 1, 2

EXPORTED = ["pbr_create", "pbr_destroy", "pbr_last_error", "pbr_set_stream", "pbr_checked_build",
            "pbr_field_workspace_bytes", "pbr_trace_workspace_bytes", "pbr_set_trace_workspace",
            "pbr_set_density_field", "pbr_set_optics",
            "pbr_set_sensor", "pbr_get_derived", "pbr_set_exit_recording",
            "pbr_emit_and_trace", "pbr_calibrate_precision", "pbr_brick_flags",
            "pbr_read_image", "pbr_read_ray_exits",
            "pbr_batch_workspace_bytes", "pbr_batch_create", "pbr_batch_destroy", "pbr_batch_last_error",
            "pbr_batch_get_config", "pbr_batch_configure", "pbr_batch_run", "pbr_batch_autotune",
            "pbr_surrogate_create", "pbr_surrogate_destroy", "pbr_surrogate_last_error",
            "pbr_surrogate_set_params", "pbr_surrogate_get_params", "pbr_surrogate_forward",
            "pbr_surrogate_gradients", "pbr_surrogate_adam_step", "pbr_surrogate_train",
            "pbr_surrogate_tile_map", "pbr_set_surrogate", "pbr_probe_u64_atomics",
            "pbr_set_source_sums", "pbr_dot_map_workspace_bytes", "pbr_dot_displacement_map",
            "pbr_bos_theory_map", "pbr_displace_sources", "pbr_mie_table", "pbr_mie_workspace_bytes",
            "pbr_set_mie", "pbr_set_optical_chain", "pbr_field_workspace_bytes_nodes",
            "pbr_set_density_field_nodes", "pbr_surrogate_blob_bytes", "pbr_surrogate_save",
            "pbr_surrogate_load", "pbr_probe_fma_rate",
            "pbr_probe_read_bandwidth", "pbr_probe_lds_bandwidth", "pbr_emit_and_trace_noalloc",
            "pbr_surrogate_workspace_bytes", "pbr_surrogate_train_workspace_bytes",
            "pbr_set_source_order", "pbr_source_order_morton_workspace_bytes", "pbr_source_order_morton"]


class PbrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pbr error {code}: {msg}")
        self.code = code


class pbr_optics(C.Structure):
    _fields_ = [("z_front_vertex", C.c_double), ("focal_length", C.c_double),
                ("f_number", C.c_double), ("thickness", C.c_double), ("n_glass", C.c_double),
                ("clear_radius", C.c_double), ("z_focus", C.c_double)]


class pbr_sensor(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_double),
                ("z_sensor", C.c_double), ("wavelength", C.c_double), ("sigma_px", C.c_double),
                ("dtau_with_pi", C.c_int32), ("reserved", C.c_int32)]


class pbr_derived(C.Structure):
    _fields_ = [("n_inf", C.c_double), ("lens_radius", C.c_double), ("thickness", C.c_double),
                ("aperture_radius", C.c_double), ("clear_radius", C.c_double),
                ("z_sensor", C.c_double), ("magnification", C.c_double), ("sigma_px", C.c_double),
                ("footprint_r", C.c_int32), ("max_steps", C.c_int32)]


class pbr_stats(C.Structure):
    _fields_ = [("rays", C.c_uint64), ("status", C.c_uint64 * PBR_NUM_STATUS),
                ("entered_volume", C.c_uint64), ("rkn_steps", C.c_uint64),
                ("rkn_steps_fp64", C.c_uint64), ("trace_ms", C.c_double),
                ("box_ms", C.c_double), ("box_launches", C.c_uint64), ("surrogate_rays", C.c_uint64)]


class pbr_precision_report(C.Structure):
    _fields_ = [("n_bricks", C.c_int64), ("n_steep", C.c_int64), ("n_fp64", C.c_int64),
                ("grad_threshold", C.c_double), ("grad_max", C.c_double), ("max_err_px", C.c_double),
                ("tol_px", C.c_double), ("steps_per_sample", C.c_int32), ("rays_per_brick", C.c_int32)]


class pbr_source_sum(C.Structure):
    _fields_ = [("sum_x", C.c_int64), ("sum_y", C.c_int64), ("hits", C.c_uint64), ("reserved", C.c_uint64)]


class pbr_surface(C.Structure):
    _fields_ = [("type", C.c_int32), ("reserved", C.c_int32), ("z", C.c_double), ("radius", C.c_double),
                ("clear", C.c_double), ("n_after", C.c_double), ("pitch", C.c_double)]


class pbr_optical_chain(C.Structure):
    _fields_ = [("n_surfaces", C.c_int32), ("reserved", C.c_int32), ("aim_z", C.c_double),
                ("aim_radius", C.c_double), ("s", pbr_surface * PBR_MAX_SURFACES)]


class pbr_mie(C.Structure):
    _fields_ = [("diameter", C.c_double), ("m_re", C.c_double), ("m_im", C.c_double), ("wavelength", C.c_double),
                ("laser_dir", C.c_double * 3)]


class pbr_map_grid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("dx", C.c_double), ("dy", C.c_double),
                ("z_dots", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32)]


class pbr_batch_item(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("src_dev", C.c_void_p), ("n_src", C.c_int64),
                ("rays_per_src", C.c_int32), ("flags", C.c_uint32), ("seed", C.c_uint64), ("ds", C.c_double)]


class pbr_batch_config(C.Structure):
    _fields_ = [("box_block", C.c_int32), ("unit_rays", C.c_int32), ("tile", C.c_int32),
                ("reserved", C.c_int32), ("round_rays", C.c_int64), ("max_round_rays", C.c_int64),
                ("min_round_rays", C.c_int64), ("rounds", C.c_int32), ("pad", C.c_int32)]


class pbr_batch_stats(C.Structure):
    _fields_ = [("rays", C.c_uint64), ("status", C.c_uint64 * PBR_NUM_STATUS), ("rkn_steps", C.c_uint64),
                ("run_ms", C.c_double), ("rounds", C.c_int32), ("images", C.c_int32),
                ("rkn_steps_nodes", C.c_uint64)]


class pbr_surrogate_train_config(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("lr_max", C.c_float), ("lr_min", C.c_float),
                ("tol_px", C.c_double), ("tiles", C.c_int32), ("min_tile_samples", C.c_int32),
                ("shuffle_seed", C.c_uint64)]


class pbr_surrogate_report(C.Structure):
    _fields_ = [("train_samples", C.c_int64), ("val_samples", C.c_int64), ("val_eligible", C.c_int64),
                ("val_rim_mismatches", C.c_int64), ("steps", C.c_int32), ("eligible_tiles", C.c_int32), ("loss_first_epoch", C.c_double),
                ("loss_last_epoch", C.c_double), ("val_median_px", C.c_double), ("val_p99_px", C.c_double),
                ("val_max_px", C.c_double), ("val_max_eligible_px", C.c_double), ("sample_ms", C.c_double),
                ("train_ms", C.c_double), ("validate_ms", C.c_double)]


RAY_EXIT_DTYPE = np.dtype([("ray_id", "<i8"), ("status", "<i4"), ("n_steps", "<i4"),
                           ("entered", "<i4"), ("reserved", "<i4"), ("vol_exit_pos", "<f8", 3),
                           ("vol_exit_dir", "<f8", 3), ("sensor_px", "<f8", 2)])

_lib = None


def load(path: str = LIB_PATH):
    """Loads libpbr.so (after torch, so both share one HIP runtime).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds the process to torch's HIP runtime first)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1812_05902_amd.build` "
                           "(there is no fallback path)")
    l = C.CDLL(path)
    P, I, I64, U32, U64, D = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    sig = {
        "pbr_create": (I, [C.POINTER(P), I, P]),
        "pbr_destroy": (None, [P]),
        "pbr_last_error": (C.c_char_p, [P]),
        "pbr_set_stream": (I, [P, P]),
        "pbr_checked_build": (I, []),
        "pbr_field_workspace_bytes": (C.c_size_t, [I, I, I]),
        "pbr_trace_workspace_bytes": (C.c_size_t, [I64]),
        "pbr_set_trace_workspace": (I, [P, P, C.c_size_t]),
        "pbr_set_density_field": (I, [P, P, I, I, I, P, P, D, D, P, C.c_size_t]),
        "pbr_set_density_field_nodes": (I, [P, P, I, I, I, P, P, D, D, P, C.c_size_t]),
        "pbr_field_workspace_bytes_nodes": (C.c_size_t, [I, I, I]),
        "pbr_set_optics": (I, [P, C.POINTER(pbr_optics)]),
        "pbr_set_sensor": (I, [P, C.POINTER(pbr_sensor), P]),
        "pbr_get_derived": (I, [P, C.POINTER(pbr_derived)]),
        "pbr_set_exit_recording": (I, [P, I64, I64, I64, P]),
        "pbr_emit_and_trace": (I, [P, P, I64, C.c_int32, U64, D, U32, C.POINTER(pbr_stats)]),
        "pbr_emit_and_trace_noalloc": (I, [P, P, I64, C.c_int32, U64, D, U32, I64, C.POINTER(pbr_stats)]),
        "pbr_calibrate_precision": (I, [P, D, D, C.c_int32, U64, D, C.POINTER(pbr_precision_report)]),
        "pbr_brick_flags": (I, [P, P, I64, I]),
        "pbr_read_image": (I, [P, I, P, D]),
        "pbr_batch_workspace_bytes": (C.c_size_t, [P, I, I64]),
        "pbr_batch_create": (I, [C.POINTER(P), P, I, P, C.c_size_t, P]),
        "pbr_batch_destroy": (None, [P]),
        "pbr_batch_last_error": (C.c_char_p, [P]),
        "pbr_batch_get_config": (I, [P, C.POINTER(pbr_batch_config)]),
        "pbr_batch_configure": (I, [P, C.POINTER(pbr_batch_config)]),
        "pbr_batch_run": (I, [P, C.POINTER(pbr_batch_stats)]),
        "pbr_batch_autotune": (I, [P, C.c_char_p, C.c_int32, C.POINTER(pbr_batch_config), C.POINTER(C.c_double)]),
        "pbr_read_ray_exits": (I, [P, P, I64, I64]),
        "pbr_surrogate_workspace_bytes": (C.c_size_t, [I64, I64]),
        "pbr_surrogate_train_workspace_bytes": (C.c_size_t, [I64, I64, C.c_int32, C.c_int32, C.c_int32]),
        "pbr_surrogate_create": (I, [C.POINTER(P), I, P, U64, I64, I64, P, C.c_size_t]),
        "pbr_surrogate_destroy": (None, [P]),
        "pbr_surrogate_last_error": (C.c_char_p, [P]),
        "pbr_surrogate_set_params": (I, [P, P, I64]),
        "pbr_surrogate_get_params": (I, [P, P, I64]),
        "pbr_surrogate_forward": (I, [P, P, I64, P]),
        "pbr_surrogate_gradients": (I, [P, P, P, I64, P, C.POINTER(D)]),
        "pbr_surrogate_adam_step": (I, [P, P, P, I64, C.c_float, C.c_int32, C.POINTER(D)]),
        "pbr_surrogate_train": (I, [P, P, P, I64, C.c_int32, P, I64, C.c_int32, U64, U64, D,
                                    C.POINTER(pbr_surrogate_train_config), P, C.c_size_t,
                                    C.POINTER(pbr_surrogate_report)]),
        "pbr_surrogate_tile_map": (I, [P, P, P, I64]),
        "pbr_set_surrogate": (I, [P, P]),
        "pbr_surrogate_blob_bytes": (C.c_size_t, [P]),
        "pbr_surrogate_save": (I, [P, P, C.c_size_t]),
        "pbr_surrogate_load": (I, [P, P, P, C.c_size_t]),
        "pbr_probe_u64_atomics": (I, [I, I64, I64, C.POINTER(D)]),
        "pbr_probe_fma_rate": (I, [I, I, C.POINTER(D)]),
        "pbr_probe_read_bandwidth": (I, [I, I64, I64, I, C.POINTER(D)]),
        "pbr_probe_lds_bandwidth": (I, [I, C.POINTER(D)]),
        "pbr_set_source_sums": (I, [P, P, I64]),
        "pbr_set_source_order": (I, [P, P, I64]),
        "pbr_source_order_morton_workspace_bytes": (C.c_size_t, [I64]),
        "pbr_source_order_morton": (I, [P, P, I64, P, P, C.c_size_t]),
        "pbr_dot_map_workspace_bytes": (C.c_size_t, [I, I]),
        "pbr_dot_displacement_map": (I, [P, P, P, P, I64, C.POINTER(pbr_map_grid), P, C.c_size_t, P]),
        "pbr_bos_theory_map": (I, [P, C.POINTER(pbr_map_grid), C.c_int32, P]),
        "pbr_displace_sources": (I, [P, P, P, I64, P, I, I, I, P, P, D, C.c_int32]),
        "pbr_mie_table": (I, [C.POINTER(pbr_mie), D, P, C.c_int32]),
        "pbr_mie_workspace_bytes": (C.c_size_t, []),
        "pbr_set_mie": (I, [P, C.POINTER(pbr_mie), P, C.c_size_t]),
        "pbr_set_optical_chain": (I, [P, C.POINTER(pbr_optical_chain)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(l, name)
        fn.restype = res
        fn.argtypes = args
    _lib = l
    return l


def _check(ctx, code):
    if code != PBR_OK:
        msg = _lib.pbr_last_error(ctx)
        raise PbrError(code, msg.decode() if msg else "")


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ------------------------------------------------------------------ C names (marshalling only)

def pbr_create(device: int = 0, stream=None):
    l = load()
    h = C.c_void_p()
    code = l.pbr_create(C.byref(h), int(device), stream)
    if code != PBR_OK:
        raise PbrError(code, l.pbr_last_error(None).decode())
    return h


def pbr_destroy(ctx):
    load().pbr_destroy(ctx)


def pbr_set_stream(ctx, stream):
    _check(ctx, load().pbr_set_stream(ctx, stream))


def pbr_field_workspace_bytes(nx, ny, nz) -> int:
    return int(load().pbr_field_workspace_bytes(nx, ny, nz))


def pbr_trace_workspace_bytes(rays_per_chunk) -> int:
    return int(load().pbr_trace_workspace_bytes(int(rays_per_chunk)))


def pbr_set_trace_workspace(ctx, ws):
    _check(ctx, load().pbr_set_trace_workspace(ctx, _dptr(ws), ws.numel() * ws.element_size()))


def pbr_set_density_field(ctx, rho, origin, spacing, K, rho_inf, ws, nodes=False):
    nz, ny, nx = rho.shape
    o = (C.c_double * 3)(*origin)
    s = (C.c_double * 3)(*spacing)
    fn = load().pbr_set_density_field_nodes if nodes else load().pbr_set_density_field
    _check(ctx, fn(ctx, _dptr(rho), nx, ny, nz, o, s, float(K), float(rho_inf), _dptr(ws),
                   ws.numel() * ws.element_size()))


def pbr_field_workspace_bytes_nodes(nx, ny, nz) -> int:
    return int(load().pbr_field_workspace_bytes_nodes(nx, ny, nz))


def pbr_set_optics(ctx, optics: pbr_optics):
    _check(ctx, load().pbr_set_optics(ctx, C.byref(optics)))


def pbr_set_sensor(ctx, sensor: pbr_sensor, accum):
    _check(ctx, load().pbr_set_sensor(ctx, C.byref(sensor), _dptr(accum)))


def pbr_get_derived(ctx) -> pbr_derived:
    d = pbr_derived()
    _check(ctx, load().pbr_get_derived(ctx, C.byref(d)))
    return d


def pbr_set_exit_recording(ctx, first, stride, max_records, buf):
    _check(ctx, load().pbr_set_exit_recording(ctx, int(first), int(stride), int(max_records), _dptr(buf)))


def pbr_emit_and_trace(ctx, src, rays_per_src, seed, ds, flags=0, want_stats=False):
    st = pbr_stats() if want_stats else None
    n_src = 0 if src is None else int(src.shape[0])
    _check(ctx, load().pbr_emit_and_trace(ctx, _dptr(src), n_src, int(rays_per_src), int(seed),
                                          float(ds), int(flags), C.byref(st) if st is not None else None))
    return st


def pbr_emit_and_trace_noalloc(ctx, src, rays_per_src, seed, ds, flags=0, rays_per_chunk=0, want_stats=False):
    """pbr_emit_and_trace with the ray states in the library's static device array (no allocation)."""
    st = pbr_stats() if want_stats else None
    n_src = 0 if src is None else int(src.shape[0])
    _check(ctx, load().pbr_emit_and_trace_noalloc(ctx, _dptr(src), n_src, int(rays_per_src), int(seed),
                                                  float(ds), int(flags), int(rays_per_chunk),
                                                  C.byref(st) if st is not None else None))
    return st


def pbr_calibrate_precision(ctx, tol_px, steep_frac, rays_per_brick, seed, ds) -> pbr_precision_report:
    rep = pbr_precision_report()
    _check(ctx, load().pbr_calibrate_precision(ctx, float(tol_px), float(steep_frac), int(rays_per_brick),
                                               int(seed), float(ds), C.byref(rep)))
    return rep


def pbr_brick_flags(ctx, n_bricks, flags=None) -> np.ndarray:
    """Reads the per-brick FP64 flags, or writes ``flags`` (uint8 array) when given."""
    arr = np.zeros(int(n_bricks), dtype=np.uint8) if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    _check(ctx, load().pbr_brick_flags(ctx, arr.ctypes.data_as(C.c_void_p), int(n_bricks), 0 if flags is None else 1))
    return arr


def pbr_read_image(ctx, fmt, out, gain=0.0):
    _check(ctx, load().pbr_read_image(ctx, int(fmt), _dptr(out), float(gain)))


def pbr_read_ray_exits(ctx, first, count) -> np.ndarray:
    out = np.zeros(int(count), dtype=RAY_EXIT_DTYPE)
    _check(ctx, load().pbr_read_ray_exits(ctx, out.ctypes.data_as(C.c_void_p), int(first), int(count)))
    return out


def pbr_set_source_sums(ctx, sums, capacity):
    _check(ctx, load().pbr_set_source_sums(ctx, _dptr(sums), int(capacity)))


def pbr_set_source_order(ctx, order, n_src):
    _check(ctx, load().pbr_set_source_order(ctx, _dptr(order), int(n_src)))


def pbr_source_order_morton_workspace_bytes(n_src) -> int:
    return int(load().pbr_source_order_morton_workspace_bytes(int(n_src)))


def pbr_source_order_morton(ctx, src, n_src, order, ws):
    _check(ctx, load().pbr_source_order_morton(ctx, _dptr(src), int(n_src), _dptr(order), _dptr(ws),
                                               ws.numel() * ws.element_size()))


def pbr_dot_map_workspace_bytes(nx, ny) -> int:
    return int(load().pbr_dot_map_workspace_bytes(int(nx), int(ny)))


def map_grid(x0, y0, dx, dy, nx, ny, z_dots) -> pbr_map_grid:
    return pbr_map_grid(float(x0), float(y0), float(dx), float(dy), float(z_dots), int(nx), int(ny))


def pbr_dot_displacement_map(ctx, with_sums, without_sums, src, grid: pbr_map_grid, ws, out):
    n_src = 0 if src is None else int(src.shape[0])
    _check(ctx, load().pbr_dot_displacement_map(ctx, _dptr(with_sums), _dptr(without_sums), _dptr(src), n_src,
                                                C.byref(grid), _dptr(ws), ws.numel() * ws.element_size(),
                                                _dptr(out)))


def pbr_bos_theory_map(ctx, grid: pbr_map_grid, samples, out):
    _check(ctx, load().pbr_bos_theory_map(ctx, C.byref(grid), int(samples), _dptr(out)))


def pbr_displace_sources(ctx, src_in, src_out, vel, origin, spacing, dt, substeps):
    nz, ny, nx = (int(v) for v in vel.shape[:3])
    o = (C.c_double * 3)(*origin)
    s = (C.c_double * 3)(*spacing)
    n_src = 0 if src_in is None else int(src_in.shape[0])
    _check(ctx, load().pbr_displace_sources(ctx, _dptr(src_in), _dptr(src_out), n_src, _dptr(vel), nx, ny, nz,
                                            o, s, float(dt), int(substeps)))


def optical_chain(surfaces, aim_z, aim_radius) -> pbr_optical_chain:
    """surfaces: list of (type, z, radius, clear, n_after, pitch)."""
    ch = pbr_optical_chain()
    ch.n_surfaces = len(surfaces)
    ch.aim_z, ch.aim_radius = float(aim_z), float(aim_radius)
    for k, (t, z, r, c, n, p) in enumerate(surfaces):
        ch.s[k] = pbr_surface(int(t), 0, float(z), float(r), float(c), float(n), float(p))
    return ch


def pbr_set_optical_chain(ctx, chain):
    _check(ctx, load().pbr_set_optical_chain(ctx, None if chain is None else C.byref(chain)))


def mie_params(diameter, m, wavelength, laser_dir) -> pbr_mie:
    m = complex(m)
    return pbr_mie(float(diameter), m.real, m.imag, float(wavelength), (C.c_double * 3)(*laser_dir))


def pbr_mie_table(mie: pbr_mie, n_medium, n=PBR_MIE_TABLE_SIZE) -> np.ndarray:
    out = np.zeros(int(n))
    code = load().pbr_mie_table(C.byref(mie), float(n_medium), out.ctypes.data_as(C.c_void_p), int(n))
    if code != PBR_OK:
        raise PbrError(code, _lib.pbr_last_error(None).decode())
    return out


def pbr_mie_workspace_bytes() -> int:
    return int(load().pbr_mie_workspace_bytes())


def pbr_set_mie(ctx, mie, table):
    nbytes = 0 if table is None else table.numel() * table.element_size()
    _check(ctx, load().pbr_set_mie(ctx, None if mie is None else C.byref(mie), _dptr(table), nbytes))


# ------------------------------------------------------------------ convenience wrapper

def stats_dict(st: pbr_stats) -> dict:
    return dict(rays=int(st.rays), status=[int(x) for x in st.status],
                entered_volume=int(st.entered_volume), rkn_steps=int(st.rkn_steps),
                rkn_steps_fp64=int(st.rkn_steps_fp64),
                trace_ms=float(st.trace_ms), box_ms=float(st.box_ms),
                box_launches=int(st.box_launches), surrogate_rays=int(st.surrogate_rays))


class Renderer:
    """One context plus the buffers it needs, on torch's current device and stream."""

    def __init__(self, device=None, rays_per_chunk=1 << 22):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = pbr_create(self.device.index, C.c_void_p(self.stream.cuda_stream))
        nb = pbr_trace_workspace_bytes(rays_per_chunk)
        self.trace_ws = torch.empty(nb // 8, dtype=torch.int64, device=self.device)
        pbr_set_trace_workspace(self.ctx, self.trace_ws)
        self.ws = None
        self.accum = None
        self.rec = None
        self.width = self.height = 0

    def close(self):
        if getattr(self, "ctx", None) is not None:
            pbr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_density_field(self, rho, origin, spacing, K, rho_inf, nodes=False):
        """nodes=True: the node layout (16 B per node) for fine grids."""
        torch = self.torch
        rho = torch.as_tensor(rho, dtype=torch.float32, device=self.device).contiguous()
        nz, ny, nx = rho.shape
        nb = pbr_field_workspace_bytes_nodes(nx, ny, nz) if nodes else pbr_field_workspace_bytes(nx, ny, nz)
        if self.ws is None or self.ws.numel() * 4 < nb:
            self.ws = torch.empty((nb + 3) // 4, dtype=torch.float32, device=self.device)
        pbr_set_density_field(self.ctx, rho, origin, spacing, K, rho_inf, self.ws, nodes=nodes)
        self.grid_shape = (nx, ny, nz)
        self._rho_keepalive = rho  # until the stream passes field preparation

    def set_optics(self, z_front_vertex, focal_length, f_number, thickness=0.0, n_glass=1.5,
                   clear_radius=0.0, z_focus=0.0):
        o = pbr_optics(z_front_vertex, focal_length, f_number, thickness, n_glass, clear_radius, z_focus)
        pbr_set_optics(self.ctx, o)

    def set_sensor(self, width, height, pitch, z_sensor=float("nan"), wavelength=532e-9,
                   sigma_px=0.0, dtau_with_pi=False):
        torch = self.torch
        s = pbr_sensor(int(width), int(height), pitch, z_sensor, wavelength, sigma_px,
                       int(bool(dtau_with_pi)), 0)
        if self.accum is None or self.accum.numel() != width * height:
            self.accum = torch.zeros(int(height), int(width), dtype=torch.int64, device=self.device)
        pbr_set_sensor(self.ctx, s, self.accum)
        self.width, self.height = int(width), int(height)

    def set_exit_recording(self, first, stride, max_records):
        torch = self.torch
        nbytes = int(max_records) * RAY_EXIT_DTYPE.itemsize
        self.rec = torch.zeros(max(nbytes, 8) // 8, dtype=torch.int64, device=self.device)
        self.rec_max = int(max_records)
        pbr_set_exit_recording(self.ctx, first, stride, max_records, self.rec)

    def derived(self) -> dict:
        d = pbr_get_derived(self.ctx)
        return {k: getattr(d, k) for k, _ in pbr_derived._fields_}

    def emit_and_trace(self, src, rays_per_src, seed, ds, flags=0, stats=False):
        torch = self.torch
        src = torch.as_tensor(src, dtype=torch.float32, device=self.device).contiguous()
        st = pbr_emit_and_trace(self.ctx, src, rays_per_src, seed, ds, flags, want_stats=stats)
        self._src_keepalive = src
        return stats_dict(st) if st is not None else None

    def calibrate_precision(self, ds, tol_px=1e-3, steep_frac=0.1, rays_per_brick=64, seed=12345) -> dict:
        rep = pbr_calibrate_precision(self.ctx, tol_px, steep_frac, rays_per_brick, seed, ds)
        return {k: getattr(rep, k) for k, _ in pbr_precision_report._fields_}

    def brick_flags(self, flags=None) -> np.ndarray:
        nb = [(n - 1 + 7) // 8 for n in self.grid_shape]
        return pbr_brick_flags(self.ctx, nb[0] * nb[1] * nb[2], flags)

    def read_image(self, fmt=PBR_FMT_RAW_U64, gain=0.0):
        torch = self.torch
        dt = {PBR_FMT_RAW_U64: torch.int64, PBR_FMT_F32: torch.float32, PBR_FMT_U16: torch.int16}[fmt]
        out = torch.empty(self.height, self.width, dtype=dt, device=self.device)
        pbr_read_image(self.ctx, fmt, out, gain)
        return out

    def set_source_sums(self, n_src):
        """Allocates and clears per-source hit sums for n_src sources (int64 tensor [n_src][4]:
        sum_x, sum_y, hits, reserved) and sets them on the context; traces with PBR_SOURCE_SUMS
        add into them."""
        self.sums = self.torch.zeros(int(n_src), 4, dtype=self.torch.int64, device=self.device)
        pbr_set_source_sums(self.ctx, self.sums, n_src)
        return self.sums

    def morton_order(self, src):
        """Permutation of the sources (int64 tensor [n_src]) sorting their positions in the field
        box by Morton code; for set_source_order."""
        torch = self.torch
        src = torch.as_tensor(src, dtype=torch.float32, device=self.device).contiguous()
        n = src.shape[0]
        nb = pbr_source_order_morton_workspace_bytes(n)
        if nb == 0:
            raise PbrError(PBR_ERR_ARG, "too many sources for a Morton order")
        ws = torch.empty(max(nb, 8) // 8, dtype=torch.int64, device=self.device)
        order = torch.empty(n, dtype=torch.int64, device=self.device)
        pbr_source_order_morton(self.ctx, src, n, order, ws)
        self._order_keepalive = (src, ws)
        return order

    def set_source_order(self, order):
        """Traces with PBR_SOURCE_ORDER take the sources in this order (int64 tensor [n_src], a
        permutation); None clears it."""
        if order is None:
            pbr_set_source_order(self.ctx, None, 0)
            self.src_order = None
            return
        self.src_order = self.torch.as_tensor(order, dtype=self.torch.int64, device=self.device).contiguous()
        pbr_set_source_order(self.ctx, self.src_order, self.src_order.shape[0])

    def dot_displacement_map(self, with_sums, without_sums, src, grid):
        """Bilinear map of per-dot displacements (float32 tensor [ny][nx][2], pixels);
        grid = (x0, y0, dx, dy, nx, ny, z_dots)."""
        torch = self.torch
        g = map_grid(*grid)
        src = torch.as_tensor(src, dtype=torch.float32, device=self.device).contiguous()
        ws = torch.empty(max(pbr_dot_map_workspace_bytes(g.nx, g.ny) // 8, 1), dtype=torch.int64, device=self.device)
        out = torch.empty(g.ny, g.nx, 2, dtype=torch.float32, device=self.device)
        pbr_dot_displacement_map(self.ctx, with_sums, without_sums, src, g, ws, out)
        self._map_keepalive = (src, ws)
        return out

    def bos_theory_map(self, grid, samples=None):
        """Eq. 9 on the grid (float32 tensor [ny][nx][2], pixels); samples defaults to four per
        cell of the box depth."""
        g = map_grid(*grid)
        if samples is None:
            samples = 4 * (self.grid_shape[2] - 1)
        out = self.torch.empty(g.ny, g.nx, 2, dtype=self.torch.float32, device=self.device)
        pbr_bos_theory_map(self.ctx, g, samples, out)
        return out

    def set_optical_chain(self, surfaces, aim_z=0.0, aim_radius=0.0):
        """General optical chain (sec. 3.3) in place of the singlet; surfaces = list of
        (type, z, radius, clear, n_after, pitch); None restores the singlet."""
        pbr_set_optical_chain(self.ctx, None if surfaces is None else optical_chain(surfaces, aim_z, aim_radius))

    def set_mie(self, diameter, m, wavelength, laser_dir):
        """Mie weighting of later traces with PBR_MIE (sec. 3.1): particle diameter (m), relative
        index m (complex), laser wavelength (m) and propagation direction; None clears it."""
        if diameter is None:
            pbr_set_mie(self.ctx, None, None)
            return
        self.mie_table = self.torch.empty(PBR_MIE_TABLE_SIZE, dtype=self.torch.float64, device=self.device)
        pbr_set_mie(self.ctx, mie_params(diameter, m, wavelength, laser_dir), self.mie_table)

    def displace_sources(self, src, vel, origin, spacing, dt, substeps=4):
        """Sources of the second frame of a PIV pair: src advanced by the velocity field vel
        (float32 [nz][ny][nx][3], m/s) over dt; returns a new float32 tensor [n][4]."""
        torch = self.torch
        src = torch.as_tensor(src, dtype=torch.float32, device=self.device).contiguous()
        vel = torch.as_tensor(vel, dtype=torch.float32, device=self.device).contiguous()
        out = torch.empty_like(src)
        pbr_displace_sources(self.ctx, src, out, vel, origin, spacing, dt, substeps)
        self._vel_keepalive = (src, vel)
        return out

    def read_ray_exits(self, first=0, count=None):
        if count is None:
            count = self.rec_max - first
        return pbr_read_ray_exits(self.ctx, first, count)

    @classmethod
    def from_scene(cls, scene, rho=None, device=None, rays_per_chunk=1 << 22, nodes=False):
        """Renderer with field, optics and sensor of an ``inputs.Scene`` (nodes: node layout)."""
        from . import inputs
        r = cls(device, rays_per_chunk=rays_per_chunk)
        if rho is None:
            rho = inputs.density(scene)
        r.set_density_field(rho, scene.origin, scene.spacing, scene.K, scene.rho_inf, nodes=nodes)
        r.set_optics(scene.z_lens, scene.focal_length, scene.f_number, scene.thickness,
                     scene.n_glass, scene.clear_radius, scene.z_focus)
        r.set_sensor(scene.width, scene.height, scene.pitch, scene.z_sensor, scene.wavelength,
                     scene.sigma_px, scene.dtau_with_pi)
        return r


def u64_image_to_numpy(t) -> np.ndarray:
    """int64 tensor holding uint64 Q32.32 values -> numpy uint64."""
    return t.cpu().numpy().view(np.uint64)


def u16_image_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint16)


def trace_scene(scene, flags=PBR_CLEAR_FIRST, stats=True, record=None, rho=None, src=None, nodes=False,
                rays_per_chunk=1 << 22):
    """Convenience: render a scene; ``record`` = (first, stride, max) for exit records.
    Returns (renderer, stats dict, records or None)."""
    from . import inputs
    r = Renderer.from_scene(scene, rho=rho, nodes=nodes, rays_per_chunk=rays_per_chunk)
    if record is not None:
        r.set_exit_recording(*record)
        flags |= PBR_RECORD_EXITS
    if src is None:
        src = inputs.sources(scene)
    st = r.emit_and_trace(src, scene.rays_per_src, scene.ray_seed, scene.ds, flags, stats=stats)
    recs = r.read_ray_exits() if record is not None else None
    return r, st, recs


# ------------------------------------------------------------------ batches

def _bcheck(b, code):
    if code != PBR_OK:
        msg = _lib.pbr_batch_last_error(b)
        raise PbrError(code, msg.decode() if msg else "")


def pbr_batch_workspace_bytes(items, round_rays) -> int:
    arr = (pbr_batch_item * len(items))(*items)
    return int(load().pbr_batch_workspace_bytes(C.cast(arr, C.c_void_p), len(items), int(round_rays)))


def pbr_batch_create(items, ws, stream):
    arr = (pbr_batch_item * len(items))(*items)
    h = C.c_void_p()
    code = load().pbr_batch_create(C.byref(h), C.cast(arr, C.c_void_p), len(items), _dptr(ws),
                                   ws.numel() * ws.element_size(), stream)
    if code != PBR_OK:
        raise PbrError(code, _lib.pbr_batch_last_error(None).decode())
    return h


def pbr_batch_destroy(b):
    load().pbr_batch_destroy(b)


def pbr_batch_get_config(b) -> pbr_batch_config:
    c = pbr_batch_config()
    _bcheck(b, load().pbr_batch_get_config(b, C.byref(c)))
    return c


def pbr_batch_configure(b, cfg: pbr_batch_config):
    _bcheck(b, load().pbr_batch_configure(b, C.byref(cfg)))


def pbr_batch_run(b, want_stats=True):
    st = pbr_batch_stats() if want_stats else None
    _bcheck(b, load().pbr_batch_run(b, C.byref(st) if st is not None else None))
    return st


def pbr_batch_autotune(b, cache_path=None, probe_rounds=1):
    c = pbr_batch_config()
    rate = C.c_double()
    _bcheck(b, load().pbr_batch_autotune(b, None if cache_path is None else str(cache_path).encode(),
                                         int(probe_rounds), C.byref(c), C.byref(rate)))
    return c, float(rate.value)


def config_dict(c: pbr_batch_config) -> dict:
    return {k: getattr(c, k) for k, _ in pbr_batch_config._fields_ if k not in ("reserved", "pad")}


class Batch:
    """Many ``Renderer`` images traced in one graph-captured launch sequence."""

    def __init__(self, renderers, sources, rays_per_src, seeds, ds, flags=PBR_CLEAR_FIRST,
                 round_rays=1 << 22):
        import torch
        self.torch = torch
        self.renderers = list(renderers)
        dev = self.renderers[0].device
        self.src = [torch.as_tensor(s, dtype=torch.float32, device=dev).contiguous() for s in sources]
        n = len(self.renderers)
        rps = rays_per_src if isinstance(rays_per_src, (list, tuple)) else [rays_per_src] * n
        seeds = seeds if isinstance(seeds, (list, tuple)) else [seeds] * n
        dss = ds if isinstance(ds, (list, tuple)) else [ds] * n
        flg = flags if isinstance(flags, (list, tuple)) else [flags] * n
        self.items = [pbr_batch_item(r.ctx.value, s.data_ptr() if s.numel() else 0, int(s.shape[0]), int(k),
                                     int(f), int(sd), float(d))
                      for r, s, k, sd, d, f in zip(self.renderers, self.src, rps, seeds, dss, flg)]
        nb = pbr_batch_workspace_bytes(self.items, round_rays)
        self.ws = torch.empty((nb + 255) // 256 * 32, dtype=torch.int64, device=dev)
        self.h = pbr_batch_create(self.items, self.ws, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))

    def run(self, stats=True):
        st = pbr_batch_run(self.h, stats)
        if st is None:
            return None
        return dict(rays=int(st.rays), status=[int(x) for x in st.status], rkn_steps=int(st.rkn_steps),
                    run_ms=float(st.run_ms), rounds=int(st.rounds), images=int(st.images),
                    rkn_steps_nodes=int(st.rkn_steps_nodes))

    def config(self) -> dict:
        return config_dict(pbr_batch_get_config(self.h))

    def configure(self, **kw):
        c = pbr_batch_get_config(self.h)
        for k, v in kw.items():
            setattr(c, k, v)
        pbr_batch_configure(self.h, c)

    def autotune(self, cache_path=None, probe_rounds=1):
        c, rate = pbr_batch_autotune(self.h, cache_path, probe_rounds)
        return config_dict(c), rate

    def close(self):
        if getattr(self, "h", None) is not None:
            pbr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ ray surrogate network

def _scheck(sg, code):
    if code != PBR_OK:
        msg = _lib.pbr_surrogate_last_error(sg)
        raise PbrError(code, msg.decode() if msg else "")


def pbr_surrogate_workspace_bytes(max_rows, ray_chunk) -> int:
    return int(load().pbr_surrogate_workspace_bytes(int(max_rows), int(ray_chunk)))


def pbr_surrogate_train_workspace_bytes(n_train_rays, n_val_rays, batch, epochs, tiles) -> int:
    return int(load().pbr_surrogate_train_workspace_bytes(int(n_train_rays), int(n_val_rays), int(batch),
                                                          int(epochs), int(tiles)))


def pbr_surrogate_create(device, stream, init_seed, max_rows, ray_chunk, ws):
    h = C.c_void_p()
    code = load().pbr_surrogate_create(C.byref(h), int(device), stream, int(init_seed), int(max_rows),
                                       int(ray_chunk), _dptr(ws), ws.numel() * ws.element_size())
    if code != PBR_OK:
        raise PbrError(code, _lib.pbr_surrogate_last_error(None).decode())
    return h


def pbr_surrogate_destroy(sg):
    load().pbr_surrogate_destroy(sg)


def pbr_surrogate_set_params(sg, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _scheck(sg, load().pbr_surrogate_set_params(sg, p.ctypes.data_as(C.c_void_p), p.size))


def pbr_surrogate_get_params(sg) -> np.ndarray:
    p = np.zeros(PBR_SURR_PARAMS, dtype=np.float32)
    _scheck(sg, load().pbr_surrogate_get_params(sg, p.ctypes.data_as(C.c_void_p), p.size))
    return p


def pbr_surrogate_forward(sg, x, y):
    _scheck(sg, load().pbr_surrogate_forward(sg, _dptr(x), int(x.shape[0]), _dptr(y)))


def pbr_surrogate_gradients(sg, x, t, want_grad=True):
    g = np.zeros(PBR_SURR_PARAMS, dtype=np.float32) if want_grad else None
    loss = C.c_double()
    _scheck(sg, load().pbr_surrogate_gradients(sg, _dptr(x), _dptr(t), int(x.shape[0]),
                                               g.ctypes.data_as(C.c_void_p) if g is not None else None,
                                               C.byref(loss)))
    return float(loss.value), g


def pbr_surrogate_adam_step(sg, x, t, lr, step, want_loss=False):
    loss = C.c_double()
    _scheck(sg, load().pbr_surrogate_adam_step(sg, _dptr(x), _dptr(t), int(x.shape[0]), float(lr), int(step),
                                               C.byref(loss) if want_loss else None))
    return float(loss.value) if want_loss else None


def pbr_surrogate_train(sg, ctx, train_src, train_rays_per_src, val_src, val_rays_per_src, train_seed, val_seed,
                        ds, cfg: pbr_surrogate_train_config, ws) -> pbr_surrogate_report:
    rep = pbr_surrogate_report()
    _scheck(sg, load().pbr_surrogate_train(sg, ctx, _dptr(train_src), int(train_src.shape[0]),
                                           int(train_rays_per_src), _dptr(val_src), int(val_src.shape[0]),
                                           int(val_rays_per_src), int(train_seed), int(val_seed), float(ds),
                                           C.byref(cfg), _dptr(ws), ws.numel() * ws.element_size(),
                                           C.byref(rep)))
    return rep


def pbr_surrogate_tile_map(sg, tiles):
    ok = np.zeros(tiles * tiles, dtype=np.uint8)
    err = np.zeros(tiles * tiles, dtype=np.float32)
    _scheck(sg, load().pbr_surrogate_tile_map(sg, ok.ctypes.data_as(C.c_void_p), err.ctypes.data_as(C.c_void_p),
                                              tiles * tiles))
    return ok.reshape(tiles, tiles), err.reshape(tiles, tiles)


def pbr_surrogate_save(sg) -> bytes:
    n = int(load().pbr_surrogate_blob_bytes(sg))
    buf = C.create_string_buffer(max(n, 1))
    _scheck(sg, load().pbr_surrogate_save(sg, buf, n))
    return buf.raw[:n]


def pbr_surrogate_load(sg, ctx, blob: bytes):
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _scheck(sg, load().pbr_surrogate_load(sg, ctx, buf, len(blob)))


def pbr_set_surrogate(ctx, sg):
    _check(ctx, load().pbr_set_surrogate(ctx, sg))


class Surrogate:
    """The ray surrogate network on torch's current device and stream."""

    def __init__(self, device=None, init_seed=0, max_rows=0, ray_chunk=1 << 22):
        """max_rows: rows per training or forward pass; ray_chunk: the largest trace chunk (rays)
        of the renderers the surrogate is attached to (53 bytes of device buffers per ray)."""
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        stream = torch.cuda.current_stream(self.device)
        nb = pbr_surrogate_workspace_bytes(max_rows, ray_chunk)
        if nb == 0:
            raise PbrError(PBR_ERR_ARG, "max_rows or ray_chunk out of range")
        self.ws = torch.empty(nb // 8, dtype=torch.int64, device=self.device)
        self.h = pbr_surrogate_create(self.device.index, C.c_void_p(stream.cuda_stream), init_seed, max_rows,
                                      ray_chunk, self.ws)
        self.tiles = 0

    def _dev(self, a):
        return self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()

    def set_params(self, p):
        pbr_surrogate_set_params(self.h, p)

    def params(self) -> np.ndarray:
        return pbr_surrogate_get_params(self.h)

    def forward(self, x):
        x = self._dev(x)
        y = self.torch.empty_like(x)
        pbr_surrogate_forward(self.h, x, y)
        return y

    def gradients(self, x, t):
        return pbr_surrogate_gradients(self.h, self._dev(x), self._dev(t))

    def adam_step(self, x, t, lr, step, want_loss=False):
        return pbr_surrogate_adam_step(self.h, self._dev(x), self._dev(t), lr, step, want_loss)

    def train(self, renderer, train_src, train_rays_per_src, val_src, val_rays_per_src, train_seed, val_seed, ds,
              batch=4096, epochs=4, lr_max=1e-3, lr_min=1e-5, tol_px=0.01, tiles=64, min_tile_samples=8,
              shuffle_seed=1) -> dict:
        cfg = pbr_surrogate_train_config(int(batch), int(epochs), float(lr_max), float(lr_min), float(tol_px),
                                         int(tiles), int(min_tile_samples), int(shuffle_seed))
        tr, va = self._dev(train_src), self._dev(val_src)
        nb = pbr_surrogate_train_workspace_bytes(tr.shape[0] * train_rays_per_src, va.shape[0] * val_rays_per_src,
                                                 batch, epochs, tiles)
        ws = self.torch.empty(max(nb, 8) // 8, dtype=self.torch.int64, device=self.device)
        rep = pbr_surrogate_train(self.h, renderer.ctx, tr, train_rays_per_src, va, val_rays_per_src, train_seed,
                                  val_seed, ds, cfg, ws)
        del ws
        self.tiles = int(tiles)
        return {k: getattr(rep, k) for k, _ in pbr_surrogate_report._fields_}

    def tile_map(self):
        return pbr_surrogate_tile_map(self.h, self.tiles)

    # offset of the int32 tile count in the blob: magic 8, version 4, parameter count 4, scene key 104,
    # geometry 9 x 8, scaling 12 x 4
    _BLOB_TILES_AT = 8 + 4 + 4 + 104 + 72 + 48

    def save(self) -> bytes:
        """The trained surrogate as a self-checking blob (weights, Adam state, scaling, tile map)."""
        return pbr_surrogate_save(self.h)

    def load(self, renderer, blob: bytes):
        """Restores a saved surrogate for ``renderer``, which must hold its training scene."""
        pbr_surrogate_load(self.h, renderer.ctx, blob)
        self.tiles = int(np.frombuffer(blob, dtype="<i4", count=1, offset=self._BLOB_TILES_AT)[0])

    def attach(self, renderer):
        pbr_set_surrogate(renderer.ctx, self.h)
        renderer._surrogate_keepalive = self

    def close(self):
        if getattr(self, "h", None) is not None:
            pbr_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pbr_probe_u64_atomics(device=0, n_slots=1 << 20, n_updates=1 << 28) -> float:
    """Updates per second of 64-bit atomic additions (calibration probe)."""
    rate = C.c_double()
    code = load().pbr_probe_u64_atomics(int(device), int(n_slots), int(n_updates), C.byref(rate))
    if code != PBR_OK:
        raise PbrError(code, "atomic probe failed")
    return float(rate.value)


def pbr_probe_fma_rate(device=0, fp64=False) -> float:
    """Vector FMA rate of the device, FLOP/s (FP32 without packed instructions, or FP64)."""
    v = C.c_double()
    code = load().pbr_probe_fma_rate(int(device), int(bool(fp64)), C.byref(v))
    if code != PBR_OK:
        raise PbrError(code, "FMA-rate probe failed")
    return float(v.value)


def pbr_probe_read_bandwidth(device=0, buffer_bytes=1 << 20, total_bytes=1 << 34, scattered=False) -> float:
    """Read bandwidth, bytes/s, from a buffer of buffer_bytes (L2-resident when small, HBM when large)."""
    v = C.c_double()
    code = load().pbr_probe_read_bandwidth(int(device), int(buffer_bytes), int(total_bytes), int(bool(scattered)),
                                           C.byref(v))
    if code != PBR_OK:
        raise PbrError(code, "read-bandwidth probe failed")
    return float(v.value)


def pbr_probe_lds_bandwidth(device=0) -> float:
    """LDS read bandwidth, bytes/s."""
    v = C.c_double()
    code = load().pbr_probe_lds_bandwidth(int(device), C.byref(v))
    if code != PBR_OK:
        raise PbrError(code, "LDS-bandwidth probe failed")
    return float(v.value)
