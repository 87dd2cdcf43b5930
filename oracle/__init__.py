"""Python access to the FP64 CPU oracle (``oracle.c``).

Test infrastructure: only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It shares no code with the GPU library (``paper_1812_05902_amd``); both
take their inputs from the seeded generators in ``paper_1812_05902_amd.inputs``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

GRID, LINEAR_N, N2_LINEAR, BUMP = 0, 1, 2, 3
DEPOSITED, OFF_SENSOR, BLOCKED_APERTURE, BLOCKED_LENS, TIR, STEP_LIMIT, MISSED = range(7)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (ISO C11, no floating-point contraction, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O2", "-fPIC", "-shared",
                               "-fopenmp", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("field_mode", C.c_int32),
        ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
        ("K", C.c_double), ("rho_inf", C.c_double),
        ("ana", C.c_double * 10),
        ("z_lens", C.c_double), ("focal_length", C.c_double), ("f_number", C.c_double),
        ("n_glass", C.c_double), ("thickness", C.c_double), ("clear_radius", C.c_double),
        ("z_focus", C.c_double),
        ("width", C.c_int32), ("height", C.c_int32), ("dtau_with_pi", C.c_int32), ("pad0", C.c_int32),
        ("pitch", C.c_double), ("z_sensor", C.c_double), ("wavelength", C.c_double),
        ("sigma_px", C.c_double),
        ("ds", C.c_double), ("seed", C.c_uint64),
        ("max_steps", C.c_int32), ("pad1", C.c_int32),
    ]


class Ray(C.Structure):
    _fields_ = [
        ("ray_id", C.c_int64), ("status", C.c_int32), ("n_steps", C.c_int32),
        ("entered", C.c_int32), ("pad", C.c_int32),
        ("lens_point", C.c_double * 2), ("dir0", C.c_double * 3),
        ("vol_exit_pos", C.c_double * 3), ("vol_exit_dir", C.c_double * 3),
        ("sensor_px", C.c_double * 2),
    ]


class Surface(C.Structure):
    _fields_ = [("type", C.c_int32), ("reserved", C.c_int32), ("z", C.c_double), ("radius", C.c_double),
                ("clear", C.c_double), ("n_after", C.c_double), ("pitch", C.c_double)]


SURF_REFRACT, SURF_MIRROR, SURF_APERTURE, SURF_LENSLETS = range(4)


RAY_DTYPE = np.dtype([
    ("ray_id", "<i8"), ("status", "<i4"), ("n_steps", "<i4"), ("entered", "<i4"), ("pad", "<i4"),
    ("lens_point", "<f8", 2), ("dir0", "<f8", 3), ("vol_exit_pos", "<f8", 3),
    ("vol_exit_dir", "<f8", 3), ("sensor_px", "<f8", 2),
])
assert RAY_DTYPE.itemsize == C.sizeof(Ray)

_lib = None


def lib():
    global _lib
    if _lib is None:
        l = C.CDLL(build())
        P = C.c_void_p
        l.orc_create.restype = P
        l.orc_create.argtypes = [C.POINTER(Cfg), P]
        l.orc_destroy.argtypes = [P]
        l.orc_derived.argtypes = [P, P]
        l.orc_splitmix64.restype = C.c_uint64
        l.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        l.orc_ray_uniforms.argtypes = [C.c_uint64, C.c_int64, C.c_int64, P]
        l.orc_field_eval.argtypes = [P, P, P]
        l.orc_rkn_step.argtypes = [P, P, P, C.c_double]
        l.orc_rkn_integrate.argtypes = [P, P, P, C.c_double, C.c_int64]
        l.orc_refract.restype = C.c_int
        l.orc_refract.argtypes = [P, P, C.c_double, C.c_double, P]
        l.orc_lens_to_sensor.restype = C.c_int
        l.orc_lens_to_sensor.argtypes = [P, P, P, P]
        l.orc_trace_ray.restype = C.c_int
        l.orc_trace_ray.argtypes = [P, P, C.c_int64, C.c_int32, P]
        l.orc_pixel_fraction.restype = C.c_double
        l.orc_pixel_fraction.argtypes = [C.c_double, C.c_int, C.c_double]
        l.orc_render.restype = C.c_int
        l.orc_render.argtypes = [P, P, C.c_int64, C.c_int32, P, P, P, C.c_int]
        l.orc_trace_ids.restype = C.c_int
        l.orc_trace_ids.argtypes = [P, P, C.c_int32, P, C.c_int64, P, C.c_int]
        l.orc_num_threads.restype = C.c_int
        l.orc_readout_u16.argtypes = [P, C.c_int64, C.c_double, P]
        _lib = l
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))


def ray_uniforms(seed: int, s: int, j: int):
    out = np.zeros(2)
    lib().orc_ray_uniforms(seed, s, j, _ptr(out))
    return out


def readout_u16(q: np.ndarray, gain: float = 0.0) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.zeros(q.shape, dtype=np.uint16)
    lib().orc_readout_u16(_ptr(q), q.size, float(gain), _ptr(out))
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def pixel_fraction(x: float, i: int, sigma: float) -> float:
    return float(lib().orc_pixel_fraction(x, i, sigma))


def refract(u, N, n1, n2):
    u = np.ascontiguousarray(u, dtype=np.float64)
    N = np.ascontiguousarray(N, dtype=np.float64)
    out = np.zeros(3)
    tir = lib().orc_refract(_ptr(u), _ptr(N), n1, n2, _ptr(out))
    return (None if tir else out)


class OracleScene:
    """A prepared oracle scene (field node values + derived optics)."""

    def __init__(self, cfg: Cfg, rho: np.ndarray | None = None):
        self.cfg = cfg
        self._rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float32)
        if cfg.field_mode == GRID:
            assert self._rho is not None and self._rho.size == cfg.nx * cfg.ny * cfg.nz
        self.h = lib().orc_create(C.byref(cfg), None if self._rho is None else _ptr(self._rho))
        d = np.zeros(11)
        lib().orc_derived(self.h, _ptr(d))
        (self.R, self.z_sensor, self.M, self.sigma_px, self.n_inf, self.step, self.a,
         r_fp, self.t, self.clear, max_steps) = d.tolist()
        self.r_fp = int(r_fp)
        self.max_steps = int(max_steps)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # --- pieces
    def field(self, R):
        R = np.ascontiguousarray(R, dtype=np.float64)
        out = np.zeros(4)
        lib().orc_field_eval(self.h, _ptr(R), _ptr(out))
        return out

    def rkn_step(self, R, T, h):
        R = np.array(R, dtype=np.float64)
        T = np.array(T, dtype=np.float64)
        lib().orc_rkn_step(self.h, _ptr(R), _ptr(T), h)
        return R, T

    def rkn_integrate(self, R, T, h, nsteps):
        R = np.array(R, dtype=np.float64)
        T = np.array(T, dtype=np.float64)
        lib().orc_rkn_integrate(self.h, _ptr(R), _ptr(T), h, int(nsteps))
        return R, T

    def lens_to_sensor(self, P, u):
        P = np.ascontiguousarray(P, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        px = np.zeros(2)
        st = lib().orc_lens_to_sensor(self.h, _ptr(P), _ptr(u), _ptr(px))
        return st, px

    def trace_ray(self, src4, s, j):
        src4 = np.ascontiguousarray(src4, dtype=np.float32)
        r = np.zeros(1, dtype=RAY_DTYPE)
        lib().orc_trace_ray(self.h, _ptr(src4), int(s), int(j), _ptr(r))
        return r[0]

    def trace_ids(self, src, rays_per_src, ids, n_threads=0):
        src = np.ascontiguousarray(src, dtype=np.float32)
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        out = np.zeros(len(ids), dtype=RAY_DTYPE)
        lib().orc_trace_ids(self.h, _ptr(src), int(rays_per_src), _ptr(ids), len(ids), _ptr(out),
                            int(n_threads))
        return out

    def set_chain(self, surfaces, aim_z, aim_r):
        """General optical chain (``orc_set_chain``): surfaces = list of (type, z, radius, clear,
        n_after, pitch); [] restores the built-in singlet."""
        arr = (Surface * max(len(surfaces), 1))()
        for k, (t, z, r, c, n, p) in enumerate(surfaces):
            arr[k] = Surface(int(t), 0, float(z), float(r), float(c), float(n), float(p))
        l = lib()
        l.orc_set_chain.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_double]
        l.orc_set_chain(self.h, C.cast(arr, C.c_void_p), len(surfaces), float(aim_z), float(aim_r))

    def chain_to_sensor(self, P, u):
        P = np.ascontiguousarray(P, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        px = np.zeros(2)
        l = lib()
        l.orc_chain_to_sensor.restype = C.c_int
        l.orc_chain_to_sensor.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        st = l.orc_chain_to_sensor(self.h, _ptr(P), _ptr(u), _ptr(px))
        return st, px

    def set_mie(self, table, laser_dir):
        """Weights every ray by the Mie table at its scattering angle (``orc_set_mie``);
        table=None clears it."""
        l = lib()
        l.orc_set_mie.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        k = np.ascontiguousarray(laser_dir, dtype=np.float64)
        if table is None:
            l.orc_set_mie(self.h, None, 0, _ptr(k))
            return
        t = np.ascontiguousarray(table, dtype=np.float64)
        l.orc_set_mie(self.h, _ptr(t), len(t), _ptr(k))

    def mie_weight(self, u):
        l = lib()
        l.orc_mie_weight.restype = C.c_double
        l.orc_mie_weight.argtypes = [C.c_void_p, C.c_void_p]
        return float(l.orc_mie_weight(self.h, _ptr(np.ascontiguousarray(u, dtype=np.float64))))

    def render(self, src, rays_per_src, n_threads=0, want_float=True):
        """Returns (uint64 Q32.32 image [H][W], float64 image or None, counts[8])."""
        src = np.ascontiguousarray(src, dtype=np.float32)
        W, H = self.cfg.width, self.cfg.height
        q = np.zeros((H, W), dtype=np.uint64)
        f = np.zeros((H, W), dtype=np.float64) if want_float else None
        counts = np.zeros(8, dtype=np.uint64)
        lib().orc_render(self.h, _ptr(src), src.shape[0], int(rays_per_src), _ptr(q),
                         None if f is None else _ptr(f), _ptr(counts), int(n_threads))
        return q, f, counts


def cfg_from_scene(scene, field_mode: int = GRID, ana=None, **over) -> Cfg:
    """Oracle configuration for an ``inputs.Scene`` (field recipe given by its density grid)."""
    c = Cfg()
    c.nx, c.ny, c.nz = scene.nx, scene.ny, scene.nz
    c.field_mode = field_mode
    c.origin = (C.c_double * 3)(*scene.origin)
    c.spacing = (C.c_double * 3)(*scene.spacing)
    c.K = scene.K
    c.rho_inf = scene.rho_inf
    if ana is not None:
        a = list(ana) + [0.0] * (10 - len(ana))
        c.ana = (C.c_double * 10)(*a)
    c.z_lens = scene.z_lens
    c.focal_length = scene.focal_length
    c.f_number = scene.f_number
    c.n_glass = scene.n_glass
    c.thickness = scene.thickness
    c.clear_radius = scene.clear_radius
    c.z_focus = scene.z_focus
    c.width, c.height = scene.width, scene.height
    c.dtau_with_pi = int(bool(scene.dtau_with_pi))
    c.pitch = scene.pitch
    c.z_sensor = scene.z_sensor
    c.wavelength = scene.wavelength
    c.sigma_px = scene.sigma_px
    c.ds = scene.ds
    c.seed = scene.ray_seed
    c.max_steps = 0
    for k, v in over.items():
        setattr(c, k, v)
    return c


def scene_oracle(scene, rho=None, **over) -> OracleScene:
    """Grid-mode oracle for a scene; builds the density from the seeded generator if absent."""
    if rho is None:
        from paper_1812_05902_amd import inputs
        rho = inputs.density(scene)
    return OracleScene(cfg_from_scene(scene, **over), rho)


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = math.sqrt(float((b * b).sum()))
    return math.sqrt(float(((a - b) ** 2).sum())) / (den if den > 0 else 1.0)
