"""C-ABI checks that need no GPU: the library loads, exports every function include/pbr.h
declares, validates its inputs, and derives the same optics as the oracle (two independent
derivations: the library uses the paraxial system matrix, the oracle a marginal-ray trace)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1812_05902_amd import inputs, pbr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # host-only contexts never dereference device pointers


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pbr.LIB_PATH):
        from paper_1812_05902_amd import build
        build.build()
    return pbr.load()


def _declared():
    txt = open(os.path.join(ROOT, "include", "pbr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pbr_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_function(lib):
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pbr.EXPORTED) == names


def test_struct_sizes_match_header_layout(lib):
    # the record layout is part of the ABI: 8 + 4*4 + 6*8 + 2*8 bytes
    assert pbr.RAY_EXIT_DTYPE.itemsize == 88
    assert C.sizeof(pbr.pbr_optics) == 56
    assert C.sizeof(pbr.pbr_sensor) == 48
    assert C.sizeof(pbr.pbr_stats) == 8 * (1 + 7 + 3) + 8 * 3 + 8
    assert C.sizeof(pbr.pbr_precision_report) == 8 * 7 + 8


def test_binding_structs_match_c_compiler_layout(tmp_path):
    """Every ctypes mirror of a header struct has the size and field offsets the C compiler gives
    the header's definition (gcc on the header itself), and the record dtype matches its struct."""
    import subprocess
    structs = [v for k, v in vars(pbr).items()
               if k.startswith("pbr_") and isinstance(v, type) and issubclass(v, C.Structure)]
    assert len(structs) >= 10
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pbr.h"', "int main(void) {"]
    for st in structs + ["pbr_ray_exit"]:
        name = st if isinstance(st, str) else st.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        fields = (pbr.RAY_EXIT_DTYPE.names if isinstance(st, str) else [f for f, _ in st._fields_])
        for f in fields:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for st in structs:
        assert int(got[st.__name__]) == C.sizeof(st), st.__name__
        for f, _ in st._fields_:
            assert int(got[f"{st.__name__}.{f}"]) == getattr(st, f).offset, (st.__name__, f)
    assert int(got["pbr_ray_exit"]) == pbr.RAY_EXIT_DTYPE.itemsize
    for f in pbr.RAY_EXIT_DTYPE.names:
        assert int(got[f"pbr_ray_exit.{f}"]) == pbr.RAY_EXIT_DTYPE.fields[f][1], f


def test_binding_constants_match_the_header(tmp_path):
    """Every constant include/pbr.h defines (error codes, statuses, flags, formats, limits) has the
    value the C compiler gives it in the binding."""
    import subprocess
    names = [n for n in re.findall(r"^#define (PBR_\w+)\s", open(os.path.join(ROOT, "include", "pbr.h")).read(),
                                   flags=re.M) if n != "PBR_H"]
    assert len(names) >= 30
    lines = ['#include <stdio.h>', '#include "pbr.h"', "int main(void) {"]
    lines += [f'printf("{n} %lld\\n", (long long)({n}));' for n in names]
    lines.append("return 0; }")
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for n in names:
        assert int(got[n]) == getattr(pbr, n), n


def test_batch_structs_and_workspace(lib):
    assert C.sizeof(pbr.pbr_batch_item) == 48
    assert C.sizeof(pbr.pbr_batch_config) == 48
    assert C.sizeof(pbr.pbr_batch_stats) == 8 * 9 + 8 + 8 + 8
    it = pbr.pbr_batch_item(FAKE, FAKE, 1000, 100, 1, 1, 1e-4)
    nb = pbr.pbr_batch_workspace_bytes([it, it], 1 << 20)
    assert nb >= (1 << 20) * 64 and nb % 256 == 0
    assert pbr.pbr_batch_workspace_bytes([it], 10) == 0
    # creation refuses host-only contexts before touching the device
    h = _host_ctx(lib)
    try:
        it = pbr.pbr_batch_item(h.value, FAKE, 10, 10, 1, 1, 1e-4)
        arr = (pbr.pbr_batch_item * 1)(it)
        b = C.c_void_p()
        assert lib.pbr_batch_create(C.byref(b), C.cast(arr, C.c_void_p), 1, FAKE, 1 << 30, None) == pbr.PBR_ERR_ARG
        assert "GPU" in lib.pbr_batch_last_error(None).decode()
        assert lib.pbr_batch_create(C.byref(b), None, 0, FAKE, 1 << 30, None) == pbr.PBR_ERR_ARG
    finally:
        lib.pbr_destroy(h)


def test_workspace_bytes(lib):
    # 128 bytes of trilinear coefficients per cell, then 4 + 1 bytes per brick of 8^3 cells,
    # each part rounded up to 256 bytes
    up = lambda v: (v + 255) // 256 * 256
    for n in (32, 512):
        nb = ((n - 1 + 7) // 8) ** 3
        want = up(up(up((n - 1) ** 3 * 128) + 4 * nb) + nb)
        assert pbr.pbr_field_workspace_bytes(n, n, n) == want
    assert pbr.pbr_field_workspace_bytes(1, 4, 4) == 0
    # 64 bytes of ray state per ray of a chunk, at least 256 rays
    assert pbr.pbr_trace_workspace_bytes(1 << 22) == (1 << 22) * 64
    assert pbr.pbr_trace_workspace_bytes(10) == 256 * 64


def _host_ctx(lib):
    h = C.c_void_p()
    assert lib.pbr_create(C.byref(h), -1, None) == pbr.PBR_OK
    return h


def _set_field(lib, h, nx=32, ny=32, nz=32, origin=(0, 0, 0.1), spacing=(1e-3,) * 3, K=2.26e-4,
               rho_inf=1.2, ws=FAKE, ws_bytes=None, rho=FAKE):
    o = (C.c_double * 3)(*origin)
    s = (C.c_double * 3)(*spacing)
    if ws_bytes is None:
        ws_bytes = max(pbr.pbr_field_workspace_bytes(nx, ny, nz), 16)
    return lib.pbr_set_density_field(h, rho, nx, ny, nz, o, s, K, rho_inf, ws, ws_bytes)


def _err(lib, h):
    return lib.pbr_last_error(h).decode()


def test_null_context_and_create_errors(lib):
    assert lib.pbr_set_optics(None, None) == pbr.PBR_ERR_ARG
    assert lib.pbr_emit_and_trace(None, None, 0, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_ARG
    assert lib.pbr_create(None, 0, None) == pbr.PBR_ERR_ARG
    assert "null" in lib.pbr_last_error(None).decode()
    lib.pbr_destroy(None)


def test_field_validation(lib):
    h = _host_ctx(lib)
    try:
        assert _set_field(lib, h, nx=1) == pbr.PBR_ERR_ARG
        assert _set_field(lib, h, spacing=(1e-3, 0.0, 1e-3)) == pbr.PBR_ERR_ARG
        assert _set_field(lib, h, origin=(0, math.nan, 0)) == pbr.PBR_ERR_ARG
        assert _set_field(lib, h, K=-1.0) == pbr.PBR_ERR_ARG
        assert _set_field(lib, h, ws_bytes=100) == pbr.PBR_ERR_WORKSPACE
        assert "workspace" in _err(lib, h)
        assert _set_field(lib, h, ws=FAKE + 4) == pbr.PBR_ERR_ARG  # misaligned
        assert _set_field(lib, h, rho=None) == pbr.PBR_ERR_ARG
        assert _set_field(lib, h) == pbr.PBR_OK
    finally:
        lib.pbr_destroy(h)


def _optics(**kw):
    d = dict(z_front_vertex=0.5, focal_length=0.05, f_number=8.0, thickness=0.0, n_glass=1.5,
             clear_radius=0.0, z_focus=0.0)
    d.update(kw)
    return pbr.pbr_optics(**d)


def _sensor(**kw):
    d = dict(width=256, height=256, pitch=20e-6, z_sensor=math.nan, wavelength=532e-9,
             sigma_px=0.0, dtau_with_pi=0, reserved=0)
    d.update(kw)
    return pbr.pbr_sensor(**d)


def test_optics_and_sensor_validation(lib):
    h = _host_ctx(lib)
    try:
        for bad in (dict(focal_length=0.0), dict(f_number=-1.0), dict(n_glass=1.0),
                    dict(thickness=1.0), dict(clear_radius=1e-4), dict(z_focus=math.inf)):
            assert lib.pbr_set_optics(h, C.byref(_optics(**bad))) == pbr.PBR_ERR_ARG, bad
        assert lib.pbr_set_optics(h, C.byref(_optics())) == pbr.PBR_OK
        for bad in (dict(width=0), dict(height=20000), dict(pitch=0.0), dict(wavelength=-1.0),
                    dict(z_sensor=math.inf)):
            assert lib.pbr_set_sensor(h, C.byref(_sensor(**bad)), FAKE) == pbr.PBR_ERR_ARG, bad
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE + 4) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), None) == pbr.PBR_ERR_ARG
    finally:
        lib.pbr_destroy(h)


def test_call_order_and_trace_validation(lib):
    h = _host_ctx(lib)
    try:
        st = pbr.pbr_stats()
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_STATE
        d = pbr.pbr_derived()
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_ERR_STATE
        assert lib.pbr_read_image(h, 0, FAKE, 0.0) == pbr.PBR_ERR_STATE
        assert lib.pbr_read_ray_exits(h, None, 0, 1) == pbr.PBR_ERR_STATE
        assert _set_field(lib, h) == pbr.PBR_OK
        assert lib.pbr_set_optics(h, C.byref(_optics())) == pbr.PBR_OK
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE) == pbr.PBR_OK
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_STATE
        assert "trace workspace" in _err(lib, h)
        assert lib.pbr_set_trace_workspace(h, None, 1 << 20) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_trace_workspace(h, FAKE + 8, 1 << 20) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_trace_workspace(h, FAKE, 1000) == pbr.PBR_ERR_WORKSPACE
        assert lib.pbr_set_trace_workspace(h, FAKE, 1 << 20) == pbr.PBR_OK
        # argument errors come before the host-only state error
        assert lib.pbr_emit_and_trace(h, FAKE, -1, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 0, 0, 1e-4, 0, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 0.0, 0, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, math.nan, 0, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace(h, None, 5, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, 1 << 9, None) == pbr.PBR_ERR_ARG
        # 2^32 rays could overflow one pixel of the Q32.32 sensor
        assert lib.pbr_emit_and_trace(h, FAKE, 1 << 20, 1 << 12, 0, 1e-4, 1, C.byref(st)) == pbr.PBR_ERR_OVERFLOW
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_STATE
        # lens inside or before the box
        assert lib.pbr_set_optics(h, C.byref(_optics(z_front_vertex=0.12))) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_ARG
        assert "beyond" in _err(lib, h)
        # exit recording
        assert lib.pbr_set_exit_recording(h, -1, 1, 1, FAKE) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_exit_recording(h, 0, 0, 1, FAKE) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_exit_recording(h, 0, 1, 5, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_exit_recording(h, 0, 1, 5, FAKE) == pbr.PBR_OK
        assert lib.pbr_read_ray_exits(h, None, 3, 5) == pbr.PBR_ERR_ARG
        # spot too wide for the deposit window
        assert lib.pbr_set_sensor(h, C.byref(_sensor(sigma_px=4.0)), FAKE) == pbr.PBR_OK
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_ERR_ARG
    finally:
        lib.pbr_destroy(h)


@pytest.mark.parametrize("make", [inputs.tiny_bos,
                                  lambda: inputs.turbulence_bos(n=16, n_src=1, rays_per_src=1),
                                  lambda: inputs.tomo_piv_shock(n=8, n_src=1, rays_per_src=1),
                                  lambda: inputs.tiny_bos().replace(dtau_with_pi=True, f_number=4.0)])
def test_derived_optics_match_oracle(lib, make):
    sc = make()
    h = _host_ctx(lib)
    try:
        assert _set_field(lib, h, nx=sc.nx, ny=sc.ny, nz=sc.nz, origin=sc.origin, spacing=sc.spacing,
                          K=sc.K, rho_inf=sc.rho_inf) == pbr.PBR_OK
        o = _optics(z_front_vertex=sc.z_lens, focal_length=sc.focal_length, f_number=sc.f_number,
                    thickness=sc.thickness, n_glass=sc.n_glass, clear_radius=sc.clear_radius,
                    z_focus=sc.z_focus)
        assert lib.pbr_set_optics(h, C.byref(o)) == pbr.PBR_OK
        s = _sensor(width=sc.width, height=sc.height, pitch=sc.pitch, z_sensor=sc.z_sensor,
                    wavelength=sc.wavelength, sigma_px=sc.sigma_px, dtau_with_pi=int(sc.dtau_with_pi))
        assert lib.pbr_set_sensor(h, C.byref(s), FAKE) == pbr.PBR_OK
        d = pbr.pbr_derived()
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_OK
    finally:
        lib.pbr_destroy(h)
    oc = oracle.OracleScene(oracle.cfg_from_scene(sc, field_mode=oracle.BUMP, ana=[1, 0, 1, 0, 0, 0]))
    assert d.n_inf == pytest.approx(oc.n_inf, rel=1e-15)
    assert d.lens_radius == pytest.approx(oc.R, rel=1e-13)
    assert d.thickness == pytest.approx(oc.t, rel=1e-15)
    assert d.aperture_radius == pytest.approx(oc.a, rel=1e-15)
    assert d.clear_radius == pytest.approx(oc.clear, rel=1e-15)
    assert d.z_sensor == pytest.approx(oc.z_sensor, rel=1e-12)
    assert d.magnification == pytest.approx(oc.M, rel=1e-10)
    assert d.sigma_px == pytest.approx(oc.sigma_px, rel=1e-10)
    assert d.footprint_r == oc.r_fp


def test_surrogate_entry_points_validate_before_device_work(lib):
    h = C.c_void_p()
    need = lib.pbr_surrogate_workspace_bytes(0, 1 << 12)
    assert lib.pbr_surrogate_create(C.byref(h), 0, None, 1, -5, 1 << 12, FAKE, need) == pbr.PBR_ERR_ARG
    assert h.value is None
    assert b"max_rows" in lib.pbr_surrogate_last_error(None)
    assert lib.pbr_surrogate_create(None, 0, None, 1, 0, 0, FAKE, need) == pbr.PBR_ERR_ARG
    assert lib.pbr_surrogate_create(C.byref(h), 0, None, 1, 0, -1, FAKE, need) == pbr.PBR_ERR_ARG
    assert lib.pbr_surrogate_create(C.byref(h), 0, None, 1, 0, 1 << 12, None, need) == pbr.PBR_ERR_ARG
    assert lib.pbr_surrogate_create(C.byref(h), 0, None, 1, 0, 1 << 12, FAKE + 16, need) == pbr.PBR_ERR_ARG
    assert b"256-byte" in lib.pbr_surrogate_last_error(None)
    # the workspace check comes before any device call (this container has no GPU)
    assert lib.pbr_surrogate_create(C.byref(h), 0, None, 1, 0, 1 << 12, FAKE, need - 1) == pbr.PBR_ERR_WORKSPACE
    assert h.value is None
    for fn, args in (("pbr_surrogate_set_params", (None, 0)), ("pbr_surrogate_get_params", (None, 0)),
                     ("pbr_surrogate_forward", (None, 0, None)),
                     ("pbr_surrogate_gradients", (None, None, 64, None, None)),
                     ("pbr_surrogate_tile_map", (None, None, 0))):
        assert getattr(lib, fn)(None, *args) == pbr.PBR_ERR_ARG, fn
    lib.pbr_surrogate_destroy(None)
    ctx = _host_ctx(lib)
    try:
        assert lib.pbr_set_surrogate(ctx, None) == pbr.PBR_OK  # detaching needs nothing
        # tracing with PBR_SURROGATE and nothing attached is a state error, found before any launch
        assert _set_field(lib, ctx) == pbr.PBR_OK
        o = _optics(z_front_vertex=0.5, focal_length=0.05, f_number=8.0)
        assert lib.pbr_set_optics(ctx, C.byref(o)) == pbr.PBR_OK
        s = _sensor(width=64, height=64, pitch=20e-6)
        assert lib.pbr_set_sensor(ctx, C.byref(s), FAKE) == pbr.PBR_OK
        st = pbr.pbr_stats()
        code = lib.pbr_emit_and_trace(ctx, FAKE, 1, 1, 1, 1e-4, pbr.PBR_SURROGATE, C.byref(st))
        assert code == pbr.PBR_ERR_STATE
        assert b"no surrogate attached" in lib.pbr_last_error(ctx)
    finally:
        lib.pbr_destroy(ctx)


def test_bos_check_entry_points_validate_before_device_work(lib):
    """Per-source sums, the dot displacement map and the eq. 9 map: argument and state errors
    come before any device work (host-only context)."""
    assert pbr.pbr_dot_map_workspace_bytes(64, 32) == 64 * 32 * 24
    assert pbr.pbr_dot_map_workspace_bytes(0, 5) == 0 and pbr.pbr_dot_map_workspace_bytes(5, 4097) == 0
    h = _host_ctx(lib)
    try:
        g = pbr.map_grid(-0.01, -0.01, 1e-3, 1e-3, 21, 21, 0.0)
        ws = pbr.pbr_dot_map_workspace_bytes(21, 21)
        # sums: set, errors, and the trace checks that use them
        assert lib.pbr_set_source_sums(h, None, 4) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_source_sums(h, FAKE, -1) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_source_sums(h, FAKE + 4, 4) == pbr.PBR_ERR_ARG
        assert _set_field(lib, h) == pbr.PBR_OK
        assert lib.pbr_set_optics(h, C.byref(_optics())) == pbr.PBR_OK
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE) == pbr.PBR_OK
        assert lib.pbr_set_trace_workspace(h, FAKE, 1 << 20) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 3, 8, 0, 1e-4, pbr.PBR_SOURCE_SUMS, None) == pbr.PBR_ERR_STATE
        assert "source_sums" in _err(lib, h)
        assert lib.pbr_set_source_sums(h, FAKE, 2) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 3, 8, 0, 1e-4, pbr.PBR_SOURCE_SUMS, None) == pbr.PBR_ERR_WORKSPACE
        assert lib.pbr_emit_and_trace(h, FAKE, 2, (1 << 25) + 1, 0, 1e-4, pbr.PBR_SOURCE_SUMS,
                                      None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace(h, FAKE, 2, 8, 0, 1e-4, pbr.PBR_SOURCE_SUMS, None) == pbr.PBR_ERR_STATE
        assert "host-only" in _err(lib, h)
        # displacement map
        dm = lib.pbr_dot_displacement_map
        assert dm(h, FAKE, FAKE, FAKE, 5, None, FAKE, ws, FAKE) == pbr.PBR_ERR_ARG
        for bad in (pbr.map_grid(0, 0, 0.0, 1e-3, 4, 4, 0), pbr.map_grid(0, 0, 1e-3, 1e-3, 0, 4, 0),
                    pbr.map_grid(0, 0, 1e-3, 1e-3, 4, 5000, 0), pbr.map_grid(math.nan, 0, 1e-3, 1e-3, 4, 4, 0)):
            assert dm(h, FAKE, FAKE, FAKE, 5, C.byref(bad), FAKE, ws, FAKE) == pbr.PBR_ERR_ARG
        assert dm(h, FAKE, FAKE, FAKE, -1, C.byref(g), FAKE, ws, FAKE) == pbr.PBR_ERR_ARG
        assert dm(h, None, FAKE, FAKE, 5, C.byref(g), FAKE, ws, FAKE) == pbr.PBR_ERR_ARG
        assert dm(h, FAKE, FAKE, FAKE + 8, 5, C.byref(g), FAKE, ws, FAKE) == pbr.PBR_ERR_ARG
        assert dm(h, FAKE, FAKE, FAKE, 5, C.byref(g), FAKE, ws - 1, FAKE) == pbr.PBR_ERR_WORKSPACE
        assert dm(h, FAKE, FAKE, FAKE, 5, C.byref(g), FAKE, ws, FAKE) == pbr.PBR_ERR_STATE
        # eq. 9 map
        tm = lib.pbr_bos_theory_map
        assert tm(h, C.byref(g), 0, FAKE) == pbr.PBR_ERR_ARG
        assert tm(h, C.byref(g), 65537, FAKE) == pbr.PBR_ERR_ARG
        assert tm(h, C.byref(g), 64, None) == pbr.PBR_ERR_ARG
        assert tm(h, C.byref(pbr.map_grid(0, 0, 1e-3, 1e-3, 4, 4, 0.2)), 64, FAKE) == pbr.PBR_ERR_ARG
        assert "in front" in _err(lib, h)
        assert tm(h, C.byref(g), 64, FAKE) == pbr.PBR_ERR_STATE
    finally:
        lib.pbr_destroy(h)
    h = _host_ctx(lib)
    try:  # the eq. 9 map needs field, optics and sensor
        assert lib.pbr_bos_theory_map(h, C.byref(g), 64, FAKE) == pbr.PBR_ERR_STATE
    finally:
        lib.pbr_destroy(h)


def test_piv_displacement_validates_before_device_work(lib):
    h = _host_ctx(lib)
    try:
        o = (C.c_double * 3)(0, 0, 0)
        s = (C.c_double * 3)(1e-3, 1e-3, 1e-3)
        bad = (C.c_double * 3)(1e-3, 0.0, 1e-3)
        nan = (C.c_double * 3)(math.nan, 0, 0)
        f = lib.pbr_displace_sources
        assert f(None, FAKE, FAKE, 1, FAKE, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, -1, FAKE, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, None, FAKE, 1, FAKE, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE + 4, FAKE, 1, FAKE, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, None, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE + 2, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 1, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 70000, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 2000, 2000, 2000, o, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 4, o, bad, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 4, nan, s, 1e-3, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 4, o, s, math.inf, 4) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 4, o, s, 1e-3, 0) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 4, o, s, 1e-3, 4097) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, FAKE, 1, FAKE, 4, 4, 4, o, s, 1e-3, 4) == pbr.PBR_ERR_STATE
        assert "host-only" in _err(lib, h)
    finally:
        lib.pbr_destroy(h)


@pytest.mark.parametrize("d,m,lam", [(1e-6, 1.47 + 0j, 532e-9), (10e-6, 1.59 + 0.002j, 532e-9),
                                     (50e-9, 1.5 + 0j, 532e-9), (3e-6, 2.0 + 1.0j, 1064e-9)])
def test_mie_table_matches_oracle(lib, d, m, lam):
    """The library's host Mie series (C++) against the oracle's (numpy), both from Bohren &
    Huffman's formulas: the normalised intensity table agrees to 1e-9."""
    from oracle import mie
    n_med = 1.000277
    got = pbr.pbr_mie_table(pbr.mie_params(d, m, lam, (1, 0, 0)), n_med)
    want = mie.intensity_table(m, mie.size_parameter(d, lam, n_med), pbr.PBR_MIE_TABLE_SIZE)
    assert got.max() == 1.0
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12)


def test_mie_entry_points_validate(lib):
    with pytest.raises(pbr.PbrError):
        pbr.pbr_mie_table(pbr.mie_params(-1e-6, 1.5, 532e-9, (1, 0, 0)), 1.0)
    with pytest.raises(pbr.PbrError):
        pbr.pbr_mie_table(pbr.mie_params(1e-6, 1.5 - 0.1j, 532e-9, (1, 0, 0)), 1.0)
    with pytest.raises(pbr.PbrError):
        pbr.pbr_mie_table(pbr.mie_params(1e-6, 1.5, 532e-9, (0, 0, 0)), 1.0)
    with pytest.raises(pbr.PbrError):
        pbr.pbr_mie_table(pbr.mie_params(1e-2, 1.5, 532e-9, (1, 0, 0)), 1.0)  # x ~ 6e4
    with pytest.raises(pbr.PbrError):
        pbr.pbr_mie_table(pbr.mie_params(1e-6, 1.5, 532e-9, (1, 0, 0)), 1.0, n=1)
    assert pbr.pbr_mie_workspace_bytes() == 8 * pbr.PBR_MIE_TABLE_SIZE
    h = _host_ctx(lib)
    try:
        good = pbr.mie_params(1e-6, 1.47, 532e-9, (1, 0, 0))
        ws = pbr.pbr_mie_workspace_bytes()
        assert lib.pbr_set_mie(h, C.byref(good), FAKE, ws) == pbr.PBR_ERR_STATE  # no field yet
        assert _set_field(lib, h) == pbr.PBR_OK
        assert lib.pbr_set_mie(h, C.byref(pbr.mie_params(1e-6, 0.0, 532e-9, (1, 0, 0))), FAKE, ws) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_mie(h, C.byref(good), None, ws) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_mie(h, C.byref(good), FAKE + 4, ws) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_mie(h, C.byref(good), FAKE, ws - 8) == pbr.PBR_ERR_WORKSPACE
        assert lib.pbr_set_mie(h, C.byref(good), FAKE, ws) == pbr.PBR_ERR_STATE
        assert "host-only" in _err(lib, h)
        assert lib.pbr_set_mie(h, None, None, 0) == pbr.PBR_OK  # off
        assert lib.pbr_set_optics(h, C.byref(_optics())) == pbr.PBR_OK
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE) == pbr.PBR_OK
        assert lib.pbr_set_trace_workspace(h, FAKE, 1 << 20) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, pbr.PBR_MIE, None) == pbr.PBR_ERR_STATE
        assert "Mie" in _err(lib, h)
    finally:
        lib.pbr_destroy(h)


def test_optical_chain_validates(lib):
    R = pbr.PBR_SURF_REFRACT
    h = _host_ctx(lib)
    try:
        def setc(surfs, aim_z=0.5, aim_r=0.003):
            ch = pbr.optical_chain(surfs, aim_z, aim_r)
            return lib.pbr_set_optical_chain(h, C.byref(ch))
        assert lib.pbr_set_optical_chain(None, None) == pbr.PBR_ERR_ARG
        assert setc([]) == pbr.PBR_ERR_ARG
        bad = pbr.optical_chain([(R, 0.5, 0.0, 0.01, 1.5, 0.0)], 0.5, 0.003)
        bad.n_surfaces = 17
        assert lib.pbr_set_optical_chain(h, C.byref(bad)) == pbr.PBR_ERR_ARG
        assert setc([(7, 0.5, 0.0, 0.01, 1.5, 0.0)]) == pbr.PBR_ERR_ARG
        assert setc([(R, 0.5, 0.0, 0.0, 1.5, 0.0)]) == pbr.PBR_ERR_ARG
        assert setc([(R, math.nan, 0.0, 0.01, 1.5, 0.0)]) == pbr.PBR_ERR_ARG
        assert setc([(pbr.PBR_SURF_LENSLETS, 0.5, 1e-4, 0.01, 1.5, 0.0)]) == pbr.PBR_ERR_ARG
        assert setc([(pbr.PBR_SURF_LENSLETS, 0.5, 4e-5, 0.01, 1.5, 1e-4)]) == pbr.PBR_ERR_ARG
        assert setc([(R, 0.5, 0.0, 0.01, 1.5, 0.0)], aim_r=0.0) == pbr.PBR_ERR_ARG
        assert setc([(R, 0.5, 0.05, 0.01, 1.5, 0.0), (R, 0.505, -0.05, 0.01, 0.0, 0.0)]) == pbr.PBR_OK
        # a chain needs an explicit sensor plane and spot
        assert _set_field(lib, h) == pbr.PBR_OK
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE) == pbr.PBR_OK
        d = pbr.pbr_derived()
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_ERR_STATE
        assert lib.pbr_set_sensor(h, C.byref(_sensor(z_sensor=0.6, sigma_px=0.5)), FAKE) == pbr.PBR_OK
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_OK
        assert d.footprint_r == 2 and d.z_sensor == 0.6 and math.isnan(d.magnification)
        assert d.aperture_radius == 0.003
        # singlet-only calls refuse the chain
        assert lib.pbr_set_trace_workspace(h, FAKE, 1 << 20) == pbr.PBR_OK
        rep = pbr.pbr_precision_report()
        assert lib.pbr_calibrate_precision(h, 1e-3, 0.1, 8, 1, 1e-4, C.byref(rep)) == pbr.PBR_ERR_STATE
        g = pbr.map_grid(-0.01, -0.01, 1e-3, 1e-3, 4, 4, 0.0)
        assert lib.pbr_bos_theory_map(h, C.byref(g), 16, FAKE) == pbr.PBR_ERR_STATE
        # emission target before the box
        assert setc([(R, 0.5, 0.0, 0.01, 1.5, 0.0)], aim_z=0.12) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, 0, None) == pbr.PBR_ERR_ARG
        # back to the singlet
        assert lib.pbr_set_optical_chain(h, None) == pbr.PBR_OK
        assert lib.pbr_get_derived(h, C.byref(d)) == pbr.PBR_ERR_STATE  # no pbr_set_optics yet
    finally:
        lib.pbr_destroy(h)


def test_node_layout_workspace_and_limits(lib):
    """Node layout: 16 bytes per node, then the brick tables; the paths that need per-cell records
    refuse it before any device work."""
    up = lambda v: (v + 255) // 256 * 256
    for n in (32, 257):
        nb = ((n - 1 + 7) // 8) ** 3
        assert pbr.pbr_field_workspace_bytes_nodes(n, n, n) == up(up(up(n ** 3 * 16) + 4 * nb) + nb)
    assert pbr.pbr_field_workspace_bytes_nodes(1, 4, 4) == 0
    assert pbr.pbr_field_workspace_bytes_nodes(64, 64, 64) < pbr.pbr_field_workspace_bytes(64, 64, 64) / 7
    h = _host_ctx(lib)
    try:
        o = (C.c_double * 3)(0, 0, 0.1)
        sp = (C.c_double * 3)(1e-3, 1e-3, 1e-3)
        need = pbr.pbr_field_workspace_bytes_nodes(32, 32, 32)
        f = lib.pbr_set_density_field_nodes
        assert f(h, FAKE, 32, 32, 32, o, sp, 2.26e-4, 1.2, FAKE, need - 1) == pbr.PBR_ERR_WORKSPACE
        assert f(h, FAKE, 1, 32, 32, o, sp, 2.26e-4, 1.2, FAKE, need) == pbr.PBR_ERR_ARG
        assert f(h, FAKE, 32, 32, 32, o, sp, 2.26e-4, 1.2, FAKE, need) == pbr.PBR_OK
        assert lib.pbr_set_optics(h, C.byref(_optics())) == pbr.PBR_OK
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE) == pbr.PBR_OK
        assert lib.pbr_set_trace_workspace(h, FAKE, 1 << 20) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, pbr.PBR_LANE_REFILL, None) == pbr.PBR_ERR_STATE
        assert "per-cell" in _err(lib, h)
        # shock FP64 steps and their calibration take the node layout (this context is host-only)
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, pbr.PBR_PREC_SHOCK_FP64, None) == pbr.PBR_ERR_STATE
        assert "host-only" in _err(lib, h)
        rep = pbr.pbr_precision_report()
        assert lib.pbr_calibrate_precision(h, 1e-3, 0.1, 8, 1, 1e-4, C.byref(rep)) == pbr.PBR_ERR_STATE
        assert "host-only" in _err(lib, h)
        # the per-cell field lifts the lane-refill restriction
        assert _set_field(lib, h) == pbr.PBR_OK
        assert lib.pbr_emit_and_trace(h, FAKE, 1, 1, 0, 1e-4, pbr.PBR_LANE_REFILL, None) == pbr.PBR_ERR_STATE
        assert "host-only" in _err(lib, h)
    finally:
        lib.pbr_destroy(h)


def test_noalloc_trace_validates_before_device_work(lib):
    """pbr_emit_and_trace_noalloc: the chunk range first, then the checks of pbr_emit_and_trace
    (a host-only context reaches the state error only after every argument passed)."""
    assert lib.pbr_emit_and_trace_noalloc(None, FAKE, 1, 1, 0, 1e-4, 0, 0, None) == pbr.PBR_ERR_ARG
    h = _host_ctx(lib)
    try:
        assert _set_field(lib, h) == pbr.PBR_OK
        assert lib.pbr_set_optics(h, C.byref(_optics())) == pbr.PBR_OK
        assert lib.pbr_set_sensor(h, C.byref(_sensor()), FAKE) == pbr.PBR_OK
        for bad in (pbr.PBR_NOALLOC_MAX_CHUNK + 1, 255, 1, -1):
            assert lib.pbr_emit_and_trace_noalloc(h, FAKE, 1, 1, 0, 1e-4, 0, bad, None) == pbr.PBR_ERR_ARG
            assert "rays_per_chunk" in _err(lib, h)
        assert lib.pbr_emit_and_trace_noalloc(h, FAKE, 1, 0, 0, 1e-4, 0, 0, None) == pbr.PBR_ERR_ARG
        assert lib.pbr_emit_and_trace_noalloc(h, FAKE, 1, 1, 0, 0.0, 0, 256, None) == pbr.PBR_ERR_ARG
        # no trace workspace is needed: the remaining error is the host-only context
        for chunk in (0, 256, pbr.PBR_NOALLOC_MAX_CHUNK):
            assert lib.pbr_emit_and_trace_noalloc(h, FAKE, 1, 1, 0, 1e-4, 0, chunk, None) == pbr.PBR_ERR_STATE
            assert "host-only" in _err(lib, h)
    finally:
        lib.pbr_destroy(h)


def test_surrogate_workspace_sizes(lib):
    """Persistent workspace: parameters, moments and bf16 copies (fixed), 8.4 kB per training row
    (transposed bf16 activations and errors of three layers, row-block sums), 53 B per trace-chunk ray
    and a 1 MiB tile map, each part rounded up to 256 B; training workspace: 88 B samples per ray,
    shuffles, losses and per-tile validation maxima."""
    ws = lib.pbr_surrogate_workspace_bytes
    base = ws(64, 0)
    assert base > 1 << 20
    assert ws(0, 0) == ws(65536, 0)          # 0 rows means 65536
    assert ws(100, 0) == ws(128, 0)          # rows round up to 64
    per_row = (ws(64 + 64 * 1024, 0) - base) / (64 * 1024)
    # 6 x 256 x 2 (transposed bf16 activations and errors) + 4 x 256 x 4 (pre-activations)
    # + 4224 x 4 / 16 (row-block sums) + 4224 x 4 / 256 (their group sums) + 3 x 6 x 4
    assert abs(per_row - 8362) < 1
    per_ray = (ws(64, 1 << 20) - base) / (1 << 20)
    assert abs(per_ray - 53) < 1e-3
    assert ws(-1, 0) == 0 and ws(1 << 25, 0) == 0 and ws(64, -1) == 0
    tw = lib.pbr_surrogate_train_workspace_bytes
    t0 = tw(1 << 20, 1 << 18, 4096, 8, 64)
    # samples of both sets dominate: 88 B per ray
    assert 88 * ((1 << 20) + (1 << 18)) < t0 < 110 * ((1 << 20) + (1 << 18))
    assert tw(1 << 20, 1 << 18, 4096, 8, 64) < tw(1 << 20, 1 << 18, 4096, 8, 1024)
    assert tw(0, 1, 64, 1, 1) == 0 and tw(1, 1, 100, 1, 1) == 0 and tw(1, 1, 64, 0, 1) == 0
    assert tw(1, 1, 64, 1, 1025) == 0
    assert tw((1 << 31) - 1, 1, 64, 1 << 20, 1) == 0  # more than 2^30 Adam steps


def test_source_order_entry_points_validate_before_device_work(lib):
    """The source order: setter arguments, the Morton order's workspace size and its state and
    argument errors, and a trace with PBR_SOURCE_ORDER that has no matching order, all found on
    the host."""
    ws = lib.pbr_source_order_morton_workspace_bytes
    assert ws(-1) == 0 and ws(1 << 31) == 0
    assert ws(0) > 0
    # keys in and out and the identity (8 bytes each per source) plus the sort's own scratch
    assert ws(1 << 20) >= 3 * 8 * (1 << 20)
    assert ws(1 << 20) < ws(1 << 21)
    ctx = _host_ctx(lib)
    try:
        assert lib.pbr_set_source_order(ctx, None, -1) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_source_order(ctx, None, 5) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_source_order(ctx, FAKE + 4, 5) == pbr.PBR_ERR_ARG
        assert lib.pbr_set_source_order(ctx, None, 0) == pbr.PBR_OK
        order = lib.pbr_source_order_morton
        assert order(ctx, FAKE, 10, FAKE, FAKE, ws(10)) == pbr.PBR_ERR_STATE  # no field
        assert b"no field" in lib.pbr_last_error(ctx)
        assert _set_field(lib, ctx) == pbr.PBR_OK
        assert order(ctx, FAKE, -1, FAKE, FAKE, ws(10)) == pbr.PBR_ERR_ARG
        assert order(ctx, None, 10, FAKE, FAKE, ws(10)) == pbr.PBR_ERR_ARG
        assert order(ctx, FAKE + 8, 10, FAKE, FAKE, ws(10)) == pbr.PBR_ERR_ARG  # float4 sources
        assert order(ctx, FAKE, 10, FAKE, FAKE, ws(10)) == pbr.PBR_ERR_STATE    # host-only context
        o = _optics(z_front_vertex=0.5, focal_length=0.05, f_number=8.0)
        assert lib.pbr_set_optics(ctx, C.byref(o)) == pbr.PBR_OK
        s = _sensor(width=64, height=64, pitch=20e-6)
        assert lib.pbr_set_sensor(ctx, C.byref(s), FAKE) == pbr.PBR_OK
        st = pbr.pbr_stats()
        code = lib.pbr_emit_and_trace(ctx, FAKE, 3, 1, 1, 1e-4, pbr.PBR_SOURCE_ORDER, C.byref(st))
        assert code == pbr.PBR_ERR_STATE and b"no source order" in lib.pbr_last_error(ctx)
        assert lib.pbr_set_source_order(ctx, FAKE, 4) == pbr.PBR_OK
        code = lib.pbr_emit_and_trace(ctx, FAKE, 3, 1, 1, 1e-4, pbr.PBR_SOURCE_ORDER, C.byref(st))
        assert code == pbr.PBR_ERR_ARG and b"4 sources" in lib.pbr_last_error(ctx)
    finally:
        lib.pbr_destroy(ctx)


def test_checked_build_has_the_same_entry_points(lib):
    """libpbr_checked.so (index tests on the trace kernels' device accesses) exports every declared
    function and says that it is the checked build; the regular library says that it is not."""
    if not os.path.exists(pbr.CHECKED_LIB_PATH):
        from paper_1812_05902_amd import build
        build.build()
    chk = C.CDLL(pbr.CHECKED_LIB_PATH)
    for n in _declared():
        assert hasattr(chk, n), n
    assert chk.pbr_checked_build() == 1
    assert lib.pbr_checked_build() == 0
