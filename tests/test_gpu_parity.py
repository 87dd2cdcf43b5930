"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Bar: per-ray sensor hits within 1e-4 px and images within 1e-3 relative L2 for the FP32 path;
per-ray hits within 1e-7 px for the all-FP64 path.  Integer work (ray status, step counts, the
Q32.32 image of one render vs another, readout) is compared exactly, except for rays sitting on
a decision boundary within rounding (counted and bounded)."""
import math

import numpy as np
import pytest

import oracle
from paper_1812_05902_amd import inputs, pbr

pytestmark = pytest.mark.gpu

TOL_PX = 1e-4
TOL_PX_FP64 = 1e-7


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pbr.load()
    return torch


def _compare_records(gpu, ref, tol_px, max_boundary_frac=1e-4, label=""):
    """Per-ray comparison; returns (max px error, number of status mismatches)."""
    assert len(gpu) == len(ref)
    assert np.array_equal(gpu["ray_id"], ref["ray_id"])
    same = gpu["status"] == ref["status"]
    mism = int((~same).sum())
    assert mism <= max(1, int(max_boundary_frac * len(gpu))), f"{label}: {mism} status mismatches"
    both = same & ((gpu["status"] == pbr.PBR_RAY_DEPOSITED) | (gpu["status"] == pbr.PBR_RAY_OFF_SENSOR))
    err = np.abs(gpu["sensor_px"][both] - ref["sensor_px"][both]).max() if both.any() else 0.0
    ent = same & (gpu["entered"] == 1) & (gpu["status"] != pbr.PBR_RAY_STEP_LIMIT)
    assert np.array_equal(gpu["entered"], ref["entered"])
    if ent.any():
        assert np.abs(gpu["n_steps"][ent] - ref["n_steps"][ent]).max() <= 1, label
        assert np.abs(gpu["vol_exit_pos"][ent] - ref["vol_exit_pos"][ent]).max() < 1e-8, label
        assert np.abs(gpu["vol_exit_dir"][ent] - ref["vol_exit_dir"][ent]).max() < 1e-7, label
    assert err <= tol_px, f"{label}: max sensor error {err:.3e} px > {tol_px:.1e}"
    return float(err), mism


def _render_all(torch, scene, flags=0, src=None, nodes=False):
    if src is None:
        src = inputs.sources(scene)
    n = scene.n_rays
    r, st, recs = pbr.trace_scene(scene, flags=pbr.PBR_CLEAR_FIRST | flags, stats=True,
                                  record=(0, 1, max(n, 1)), src=src, nodes=nodes)
    return r, st, recs, src


def test_tiny_bos_rays_and_image_match_oracle(torch):
    sc = inputs.tiny_bos()
    r, st, recs, src = _render_all(torch, sc)
    o = oracle.scene_oracle(sc)
    ref = o.trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    err, mism = _compare_records(recs, ref, TOL_PX, label="tiny_bos")
    print(f"tiny_bos: max |dpx| = {err:.3e}, status mismatches = {mism}")
    # counters
    assert st["rays"] == sc.n_rays
    assert sum(st["status"]) == sc.n_rays
    counts = np.bincount(ref["status"], minlength=7)
    assert np.abs(np.array(st["status"]) - counts).sum() <= 2 * mism
    assert st["rkn_steps"] == pytest.approx(int(ref["n_steps"].sum()), abs=2 * sc.n_rays * 1e-3 + 10)
    # image
    img = pbr.u64_image_to_numpy(r.read_image(pbr.PBR_FMT_RAW_U64))
    q, f, _ = o.render(src, sc.rays_per_src)
    rel = oracle.rel_l2(img.astype(np.float64), q.astype(np.float64))
    print(f"tiny_bos: image rel L2 = {rel:.3e}")
    assert rel <= 1e-3
    assert oracle.rel_l2(img.astype(np.float64) / 2 ** 32, f) <= 1e-3


def test_render_is_bitwise_deterministic(torch):
    sc = inputs.tiny_bos()
    src = inputs.sources(sc)
    r = pbr.Renderer.from_scene(sc)
    imgs = []
    for _ in range(3):
        r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
        imgs.append(pbr.u64_image_to_numpy(r.read_image()))
    assert np.array_equal(imgs[0], imgs[1]) and np.array_equal(imgs[0], imgs[2])
    # integer deposits accumulate exactly: the first half of the sources rendered twice without
    # clearing is twice the half image, and differs from the full image
    r.emit_and_trace(src[:500], sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
    half = pbr.u64_image_to_numpy(r.read_image())
    r.emit_and_trace(src[:500], sc.rays_per_src, sc.ray_seed, sc.ds, 0)
    twice = pbr.u64_image_to_numpy(r.read_image())
    assert half.sum() > 0 and not np.array_equal(half, imgs[0])
    assert np.array_equal(twice, half * np.uint64(2))


def test_fp64_path_matches_oracle_tightly(torch):
    sc = inputs.tiny_bos().replace(n_src=200)
    r, st, recs, src = _render_all(torch, sc, flags=pbr.PBR_PREC_FP64_ALL)
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    err, _ = _compare_records(recs, ref, TOL_PX_FP64, label="tiny_bos fp64")
    print(f"fp64 path: max |dpx| = {err:.3e}")


def test_ragged_sizes_and_empty(torch):
    sc = inputs.tiny_bos().replace(n_src=333, rays_per_src=37)
    r, st, recs, src = _render_all(torch, sc)
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    _compare_records(recs, ref, TOL_PX, label="ragged")
    # strided records of a second call, ragged tail
    r.set_exit_recording(5, 97, 200)
    r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                     pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS)
    recs2 = r.read_ray_exits()
    ids = 5 + 97 * np.arange(200)
    ok = ids < sc.n_rays
    assert np.array_equal(recs2["ray_id"][ok], ids[ok])
    assert np.array_equal(recs2["sensor_px"][ok], recs["sensor_px"][ids[ok]])
    # no sources: nothing deposited, counters zero
    st0 = r.emit_and_trace(src[:0], sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST, stats=True)
    assert st0["rays"] == 0 and sum(st0["status"]) == 0
    assert int(pbr.u64_image_to_numpy(r.read_image()).sum()) == 0


@pytest.mark.parametrize("nodes", [False, True], ids=["cells", "nodes"])
@pytest.mark.parametrize("ds, half", [(4.0e-3, 0.024), (1.2e-3, 0.040), (2.0e-2, 0.024)])
def test_long_steps_and_rays_along_the_faces_match_oracle(torch, ds, half, nodes):
    """Steps longer than a cell (ds = 4 mm on 1.6 mm cells: up to 2.5 cells per step, so the
    interior margin is three cells on every axis; ds = 20 mm: about 12 cells per step, five
    interior cells per axis, three steps per ray) and, with ds = 1.2 mm, dots spread beyond the box
    so that many rays enter or leave through the side faces and travel next to them: both the
    integer interior test and the end-point test near the faces are exercised, in FP32 and FP64."""
    sc = inputs.tiny_bos().replace(n_src=300, rays_per_src=40, ds=ds,
                                   src_region=((-half, half), (-half, half), (0.0, 0.0)))
    r, st, recs, src = _render_all(torch, sc, nodes=nodes)
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    err, mism = _compare_records(recs, ref, TOL_PX, label=f"ds {ds}")
    n_in = int((ref["entered"] == 1).sum())
    print(f"{'nodes' if nodes else 'cells'}, ds {ds * 1e3:.1f} mm, dots +-{half * 1e3:.0f} mm: {n_in} of "
          f"{sc.n_rays} rays entered, max |dpx| = {err:.3e}, status mismatches = {mism}")
    assert n_in > sc.n_rays // 4
    _, _, recs64, _ = _render_all(torch, sc, flags=pbr.PBR_PREC_FP64_ALL, src=src, nodes=nodes)
    _compare_records(recs64, ref, 1e-6 if nodes else TOL_PX_FP64, label=f"ds {ds} fp64")


@pytest.mark.parametrize("nodes", [False, True], ids=["cells", "nodes"])
def test_single_ray_and_sources_inside_box(torch, nodes):
    """PIV: particles inside the density box (shock field on a 48^3 grid), plus the one-ray case."""
    sc = inputs.tomo_piv_shock(n=48, n_src=300, rays_per_src=40).replace(width=512, height=512,
                                                                         pitch=40e-6)
    r, st, recs, src = _render_all(torch, sc, nodes=nodes)
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    both = (recs["status"] == ref["status"]) & (recs["status"] == 0)
    d = np.abs(recs["sensor_px"][both] - ref["sensor_px"][both]).max(axis=1)
    print(f"piv shock 48^3: max {d.max():.3e} px, p99.9 {np.quantile(d, 0.999):.3e} px")
    assert np.quantile(d, 0.999) <= TOL_PX
    assert d.max() <= 1e-2
    r64, _, recs64, _ = _render_all(torch, sc, flags=pbr.PBR_PREC_FP64_ALL, src=src, nodes=nodes)
    _compare_records(recs64, ref, 1e-6, label="piv fp64")
    one = sc.replace(n_src=1, rays_per_src=1)
    _, st1, rec1, src1 = _render_all(torch, one, src=src[:1], nodes=nodes)
    ref1 = oracle.scene_oracle(one).trace_ids(src1, 1, np.arange(1))
    _compare_records(rec1, ref1, TOL_PX, label="one ray")


def test_readout_formats(torch):
    sc = inputs.tiny_bos().replace(n_src=300)
    src = inputs.sources(sc)
    r = pbr.Renderer.from_scene(sc)
    r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
    q = pbr.u64_image_to_numpy(r.read_image(pbr.PBR_FMT_RAW_U64))
    f = r.read_image(pbr.PBR_FMT_F32).cpu().numpy()
    assert np.array_equal(f, (q.astype(np.float64) / 2 ** 32).astype(np.float32))
    u = pbr.u16_image_to_numpy(r.read_image(pbr.PBR_FMT_U16))
    assert np.array_equal(u, oracle.readout_u16(q))
    assert u.max() == 65535
    u2 = pbr.u16_image_to_numpy(r.read_image(pbr.PBR_FMT_U16, gain=1000.0))
    assert np.array_equal(u2, oracle.readout_u16(q, 1000.0))


def test_derived_step_limit_and_stats(torch):
    sc = inputs.tiny_bos()
    r = pbr.Renderer.from_scene(sc)
    src = inputs.sources(sc)[:10]
    st = r.emit_and_trace(src, 10, 1, sc.ds, pbr.PBR_CLEAR_FIRST, stats=True)
    d = r.derived()
    o = oracle.scene_oracle(sc)
    assert d["max_steps"] == o.max_steps
    assert st["trace_ms"] > 0.0
    assert st["entered_volume"] == 100


def test_turbulence_bos_full_size_sampled(torch):
    """The benchmarked workload at full size (128^3 turbulence, 5e7 rays, 1024^2 sensor), in the
    launch configuration the benchmark times: 1000 strided rays against the oracle, and the
    image total against the deposited ray count (each ray deposits its spot mass, at least
    1 - 1e-6 of it inside the window for sigma = 0.4 px and r = 2)."""
    sc = inputs.turbulence_bos()
    rho = inputs.density(sc)
    src = inputs.sources(sc)
    stride = sc.n_rays // 1000 - 1
    r, st, recs = pbr.trace_scene(sc, rho=rho, src=src, record=(17, stride, 1000), rays_per_chunk=1 << 24)
    assert st["box_launches"] == 3  # 16 777 216-ray chunks, as the benchmark runs them
    assert st["rays"] == sc.n_rays == sum(st["status"])
    o = oracle.scene_oracle(sc, rho=rho)
    ref = o.trace_ids(src, sc.rays_per_src, recs["ray_id"])
    err, _ = _compare_records(recs, ref, TOL_PX, label="turbulence_bos full")
    print(f"turbulence_bos full: max |dpx| over 1000 rays = {err:.3e}; trace {st['trace_ms']:.1f} ms")
    img = pbr.u64_image_to_numpy(r.read_image())
    total = img.astype(np.float64).sum() / 2 ** 32
    ndep = st["status"][pbr.PBR_RAY_DEPOSITED]
    assert total <= ndep * (1 + 1e-6)
    assert total >= 0.99 * ndep


@pytest.mark.parametrize("make", [lambda: inputs.tiny_bos().replace(n_src=333, rays_per_src=37),
                                  lambda: inputs.tomo_piv_shock(n=48, n_src=3000, rays_per_src=50).replace(
                                      width=512, height=512, pitch=40e-6)],
                         ids=["tiny_bos_ragged", "piv_shock_48"])
def test_lane_refill_equals_one_thread_per_ray(torch, make):
    """The persistent integration kernel whose lanes take a new ray as soon as theirs leaves the box
    gives the same exit states, step counts and image, bit for bit, as one thread per ray; with
    chunks smaller than the image (several launches, each draining its own queue)."""
    sc = make()
    src = inputs.sources(sc)
    out = []
    for flags in (pbr.PBR_LANE_REFILL, 0):
        r2 = pbr.Renderer(rays_per_chunk=40000)
        r2.set_density_field(inputs.density(sc), sc.origin, sc.spacing, sc.K, sc.rho_inf)
        r2.set_optics(sc.z_lens, sc.focal_length, sc.f_number, sc.thickness, sc.n_glass, sc.clear_radius,
                      sc.z_focus)
        r2.set_sensor(sc.width, sc.height, sc.pitch, sc.z_sensor, sc.wavelength, sc.sigma_px, sc.dtau_with_pi)
        r2.set_exit_recording(0, 1, sc.n_rays)
        st = r2.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                               pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | flags, stats=True)
        out.append((pbr.u64_image_to_numpy(r2.read_image()), r2.read_ray_exits(), st))
        r2.close()
    (img_a, rec_a, st_a), (img_b, rec_b, st_b) = out
    print(f"refill: {st_a['box_ms']:.3f} ms, one thread per ray: {st_b['box_ms']:.3f} ms "
          f"({st_a['box_launches']} launches, {st_a['rkn_steps']} steps)")
    assert np.array_equal(img_a, img_b)
    for f in pbr.RAY_EXIT_DTYPE.names:
        assert np.array_equal(rec_a[f], rec_b[f]), f
    assert st_a["status"] == st_b["status"] and st_a["rkn_steps"] == st_b["rkn_steps"]


def test_non_finite_density_is_refused(torch):
    """A NaN or an infinity anywhere in the density grid fails pbr_set_density_field (both
    layouts) and leaves no field set."""
    sc = inputs.tiny_bos()
    for bad in (float("nan"), float("inf")):
        rho = inputs.density(sc).copy()
        rho[17, 3, 29] = bad
        for nodes in (False, True):
            r = pbr.Renderer()
            with pytest.raises(pbr.PbrError, match="non-finite"):
                r.set_density_field(rho, sc.origin, sc.spacing, sc.K, sc.rho_inf, nodes=nodes)
            with pytest.raises(pbr.PbrError):
                r.derived()
            r.close()


@pytest.mark.parametrize("ds", [1.6e-3, 0.8e-3])
def test_node_layout_cell_by_cell_moves_match_oracle(torch, ds):
    """Node layout with steps of about one cell (1.6 mm cells) through a strong bump (ten times
    the tiny scene's amplitude), dots spread over +-40 mm so that rays cross x and y faces in both
    directions: the integration moves to a face neighbour on most stage points, reusing the four
    corners of the shared face, and steps jump cells diagonally too.  Every ray against the oracle
    at 1e-4 px (FP32) and 1e-6 px (FP64)."""
    sc = inputs.tiny_bos().replace(n_src=600, rays_per_src=40, ds=ds,
                                   src_region=((-0.04, 0.04), (-0.04, 0.04), (0.0, 0.0)),
                                   field_params=dict(inputs.tiny_bos().field_params, amp=1.0))
    r, st, recs, src = _render_all(torch, sc, nodes=True)
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    err, mism = _compare_records(recs, ref, TOL_PX, label=f"nodes ds {ds}")
    ent = ref["entered"] == 1
    d = ref["dir0"][ent]
    print(f"nodes, ds {ds * 1e3:.1f} mm: {int(ent.sum())} rays entered ({(d[:, 0] > 0).sum()} towards +x, "
          f"{(d[:, 0] < 0).sum()} -x, {(d[:, 1] > 0).sum()} +y, {(d[:, 1] < 0).sum()} -y), max |dpx| {err:.3e}, "
          f"status mismatches {mism}")
    assert (d[:, 0] > 0.02).sum() > 1000 and (d[:, 0] < -0.02).sum() > 1000
    assert (d[:, 1] > 0.02).sum() > 1000 and (d[:, 1] < -0.02).sum() > 1000
    _, _, recs64, _ = _render_all(torch, sc, flags=pbr.PBR_PREC_FP64_ALL, src=src, nodes=True)
    _compare_records(recs64, ref, 1e-6, label=f"nodes ds {ds} fp64")


def test_source_weights_outside_the_unit_range(torch):
    """Weights beyond [0, 1] count as the nearer end and NaN as 0 on the device as in the oracle:
    the image of weights (1.7, -0.3, NaN, 0.25, ...) equals that of (1, 0, 0, 0.25, ...) bit for
    bit and matches the oracle's render of the out-of-range weights."""
    sc = inputs.tiny_bos().replace(n_src=200, rays_per_src=50)
    src = inputs.sources(sc)
    w = np.resize(np.array([1.7, -0.3, np.nan, 0.25, 1.0, 0.6], dtype=np.float32), sc.n_src)
    a = src.copy()
    a[:, 3] = w
    b = src.copy()
    b[:, 3] = np.where(np.isnan(w), 0.0, np.clip(w, 0.0, 1.0)).astype(np.float32)
    r = pbr.Renderer.from_scene(sc)
    imgs = []
    for s in (a, b):
        r.emit_and_trace(s, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
        imgs.append(pbr.u64_image_to_numpy(r.read_image()))
    assert np.array_equal(imgs[0], imgs[1])
    q, _, _ = oracle.scene_oracle(sc).render(a, sc.rays_per_src, want_float=False)
    rel = oracle.rel_l2(imgs[0].astype(np.float64), q.astype(np.float64))
    print(f"out-of-range weights: image rel L2 vs oracle {rel:.2e}")
    assert rel <= 1e-3
