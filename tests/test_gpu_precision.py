"""GPU: the precision policy for steep-gradient (shock) cells, and the Tomo-PIV shock workload.

FP64 integration steps are taken only inside bricks whose measured FP32 error exceeds the
tolerance; these tests check the calibration finds the shock, that flagged bricks switch the
step precision (and nothing else), and the FP32 / mixed / FP64 errors against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1812_05902_amd import inputs, pbr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pbr.load()
    return torch


def _shock(n=64, n_src=200, rays=50):
    return inputs.tomo_piv_shock(n=n, n_src=n_src, rays_per_src=rays).replace(width=512, height=512,
                                                                              pitch=40e-6)


def _trace(r, sc, src, flags, nrec):
    r.set_exit_recording(0, 1, nrec)
    st = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                          pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | flags, stats=True)
    return st, r.read_ray_exits(), pbr.u64_image_to_numpy(r.read_image())


@pytest.mark.parametrize("nodes", [False, True], ids=["cells", "nodes"])
def test_calibration_finds_the_shock_bricks(torch, nodes):
    sc = _shock()
    r = pbr.Renderer.from_scene(sc, nodes=nodes)
    rep = r.calibrate_precision(sc.ds, tol_px=1e-3, steep_frac=0.1)
    print("calibration (tol 1e-3 px):", rep)
    assert rep["n_steep"] > 0
    flags = r.brick_flags()
    nb = [(n - 1 + 7) // 8 for n in (sc.nx, sc.ny, sc.nz)]
    assert flags.size == nb[0] * nb[1] * nb[2]
    assert int(flags.sum()) == rep["n_fp64"]
    # every steep brick touches the shock plane x = 0 (bricks bx = 3, 4 of 8 at 64^3)
    rep0 = r.calibrate_precision(sc.ds, tol_px=0.0, steep_frac=0.1)
    f0 = r.brick_flags().reshape(nb[2], nb[1], nb[0])
    bx = np.nonzero(f0.any(axis=(0, 1)))[0]
    assert rep0["n_fp64"] == rep0["n_steep"] > 0
    assert set(bx.tolist()) <= {2, 3, 4, 5}, bx
    assert rep0["max_err_px"] == rep["max_err_px"]


@pytest.mark.parametrize("nodes", [False, True], ids=["cells", "nodes"])
def test_mixed_precision_switches_only_the_step_precision(torch, nodes):
    sc = _shock()
    src = inputs.sources(sc)
    r = pbr.Renderer.from_scene(sc, nodes=nodes)
    st32, rec32, img32 = _trace(r, sc, src, 0, sc.n_rays)
    # no bricks flagged: the shock-FP64 flag changes nothing
    r.calibrate_precision(sc.ds, tol_px=1e9)
    stm0, recm0, imgm0 = _trace(r, sc, src, pbr.PBR_PREC_SHOCK_FP64, sc.n_rays)
    assert stm0["rkn_steps_fp64"] == 0 and np.array_equal(imgm0, img32)
    # steep bricks flagged: part of the steps run in FP64
    r.calibrate_precision(sc.ds, tol_px=0.0, steep_frac=0.1)
    stm, recm, imgm = _trace(r, sc, src, pbr.PBR_PREC_SHOCK_FP64, sc.n_rays)
    assert 0 < stm["rkn_steps_fp64"] < stm["rkn_steps"]
    stm2, _, imgm2 = _trace(r, sc, src, pbr.PBR_PREC_SHOCK_FP64, sc.n_rays)
    assert np.array_equal(imgm, imgm2)  # deterministic
    # every brick flagged: the mixed kernel reproduces the all-FP64 path
    r.brick_flags(np.ones_like(r.brick_flags()))
    sta, reca, _ = _trace(r, sc, src, pbr.PBR_PREC_SHOCK_FP64, sc.n_rays)
    st64, rec64, _ = _trace(r, sc, src, pbr.PBR_PREC_FP64_ALL, sc.n_rays)
    assert sta["rkn_steps_fp64"] == sta["rkn_steps"] == st64["rkn_steps"]
    ok = (reca["status"] == 0) & (rec64["status"] == 0)
    assert np.abs(reca["sensor_px"][ok] - rec64["sensor_px"][ok]).max() < 1e-8
    # against the oracle: FP32, mixed and FP64 all within the bar; FP64 far tighter
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, np.arange(sc.n_rays))
    errs = {}
    for name, rec in (("fp32", rec32), ("mixed", recm), ("fp64", rec64)):
        both = (rec["status"] == ref["status"]) & (rec["status"] == 0)
        errs[name] = float(np.abs(rec["sensor_px"][both] - ref["sensor_px"][both]).max())
    print("shock 64^3 max |dpx| vs oracle:", errs)
    assert errs["fp32"] <= 1e-4 and errs["mixed"] <= 1e-4 and errs["fp64"] <= 1e-7


def test_tomo_piv_shock_full_grid_sampled(torch):
    """The Tomo-PIV shock field at its full 512^3 grid, 2048^2 sensor and 1e4 rays per particle,
    for the first 2000 particles (2e7 rays): 500 strided rays against the oracle, FP32 and
    mixed precision after calibration at 1e-3 px, and the 16-bit readout."""
    sc = inputs.tomo_piv_shock().replace(n_src=2000)
    rho = inputs.density(sc)
    src = inputs.sources(sc)
    r = pbr.Renderer.from_scene(sc, rho=rho)
    rep = r.calibrate_precision(sc.ds, tol_px=1e-3, steep_frac=0.1)
    print("calibration 512^3:", rep)
    stride = sc.n_rays // 500
    r.set_exit_recording(7, stride, 500)
    st = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                          pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_PREC_SHOCK_FP64, stats=True)
    rec = r.read_ray_exits()
    u16 = pbr.u16_image_to_numpy(r.read_image(pbr.PBR_FMT_U16))
    assert u16.max() == 65535
    o = oracle.scene_oracle(sc, rho=rho)
    ref = o.trace_ids(src, sc.rays_per_src, rec["ray_id"])
    same = rec["status"] == ref["status"]
    assert (~same).sum() <= 1
    both = same & (rec["status"] == 0)
    d = np.abs(rec["sensor_px"][both] - ref["sensor_px"][both]).max(axis=1)
    print(f"tomo_piv_shock 512^3 ({both.sum()} rays): max {d.max():.3e} px, p99 {np.quantile(d, 0.99):.3e} px; "
          f"{st['rays'] / st['trace_ms'] * 1e3:.3e} rays/s, fp64 steps {st['rkn_steps_fp64']}")
    assert np.quantile(d, 0.99) <= 2e-5
    assert d.max() <= 1e-4
    # a tolerance below what FP32 reaches in the steep bricks flags some of them, so that the mixed
    # kernel takes FP64 steps at the full grid: same rays, same bars
    rep2 = r.calibrate_precision(sc.ds, tol_px=1e-7, steep_frac=0.1)
    st2 = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                           pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_PREC_SHOCK_FP64, stats=True)
    rec2 = r.read_ray_exits()
    assert np.array_equal(rec2["ray_id"], rec["ray_id"])
    same2 = rec2["status"] == ref["status"]
    assert (~same2).sum() <= 1
    both2 = same2 & (rec2["status"] == 0)
    d2 = np.abs(rec2["sensor_px"][both2] - ref["sensor_px"][both2]).max(axis=1)
    print(f"calibrated at 1e-7 px: {rep2['n_fp64']} of {rep2['n_steep']} steep bricks FP64, "
          f"{st2['rkn_steps_fp64']} FP64 steps of {st2['rkn_steps']}; max {d2.max():.3e} px, "
          f"{st2['rays'] / st2['trace_ms'] * 1e3:.3e} rays/s")
    assert rep2["n_fp64"] > 0 and st2["rkn_steps_fp64"] > 0
    assert abs(st2["rkn_steps"] - st["rkn_steps"]) <= 1e-6 * st["rkn_steps"]  # a few exits a step apart
    assert np.quantile(d2, 0.99) <= 2e-5
    assert d2.max() <= 1e-4


def test_tomo_piv_full_image_node_layout_sampled(torch):
    """The benchmarked Tomo-PIV image as the benchmark renders it: all 1e5 particles x 1e4 rays on
    the 512^3 node-layout field, 16 777 216-ray chunks, 2048^2 sensor read out as 16-bit; 1000
    strided rays against the oracle (the same bars as the per-cell test above), the 16-bit image
    against the oracle's readout of the device's Q32.32 image (an exact integer transform), and the
    light of the image against the deposited ray count."""
    sc = inputs.tomo_piv_shock()
    rho = inputs.density(sc)
    src = inputs.sources(sc)
    r = pbr.Renderer.from_scene(sc, rho=rho, nodes=True, rays_per_chunk=1 << 24)
    stride = sc.n_rays // 1000
    r.set_exit_recording(7, stride, 1000)
    st = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS,
                          stats=True)
    assert st["box_launches"] == 60 and st["rays"] == sc.n_rays == sum(st["status"])
    rec = r.read_ray_exits()
    q = pbr.u64_image_to_numpy(r.read_image())
    u16 = pbr.u16_image_to_numpy(r.read_image(pbr.PBR_FMT_U16))
    assert np.array_equal(u16, oracle.readout_u16(q)) and u16.max() == 65535
    total = q.astype(np.float64).sum() / 2 ** 32
    ndep = st["status"][pbr.PBR_RAY_DEPOSITED]
    assert 0.99 * ndep <= total <= ndep * (1 + 1e-6)
    o = oracle.scene_oracle(sc, rho=rho)
    ref = o.trace_ids(src, sc.rays_per_src, rec["ray_id"])
    same = rec["status"] == ref["status"]
    assert (~same).sum() <= 1
    both = same & (rec["status"] == 0)
    d = np.abs(rec["sensor_px"][both] - ref["sensor_px"][both]).max(axis=1)
    print(f"tomo_piv 512^3 nodes, full image ({both.sum()} sampled rays): max {d.max():.3e} px, "
          f"p99 {np.quantile(d, 0.99):.3e} px; {st['rays'] / st['trace_ms'] * 1e3:.3e} rays/s")
    assert both.sum() > 800
    assert np.quantile(d, 0.99) <= 2e-5
    assert d.max() <= 1e-4
    # shock FP64 steps on the node layout: calibrated below what FP32 reaches in the steep bricks,
    # the mixed kernel takes part of the steps in FP64; the sampled rays stay within the bars
    rep2 = r.calibrate_precision(sc.ds, tol_px=1e-7, steep_frac=0.1)
    st3 = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                           pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_PREC_SHOCK_FP64, stats=True)
    rec3 = r.read_ray_exits()
    same3 = rec3["status"] == ref["status"]
    assert (~same3).sum() <= 1
    both3 = same3 & (rec3["status"] == 0)
    d3 = np.abs(rec3["sensor_px"][both3] - ref["sensor_px"][both3]).max(axis=1)
    print(f"nodes, calibrated at 1e-7 px: {rep2['n_fp64']} of {rep2['n_steep']} steep bricks FP64, "
          f"{st3['rkn_steps_fp64']} FP64 steps; max {d3.max():.3e} px, {st3['rays'] / st3['trace_ms'] * 1e3:.3e} rays/s")
    assert rep2["n_fp64"] > 0 and st3["rkn_steps_fp64"] > 0
    assert np.quantile(d3, 0.99) <= 2e-5 and d3.max() <= 1e-4
    # the same image with the sources taken in Morton order, as the benchmark traces them: the
    # same bits, records and counts
    r.set_source_order(r.morton_order(src))
    st2 = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                           pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_SOURCE_ORDER, stats=True)
    print(f"Morton order: {st2['rays'] / st2['trace_ms'] * 1e3:.3e} rays/s")
    assert np.array_equal(pbr.u64_image_to_numpy(r.read_image()), q)
    rec2 = r.read_ray_exits()
    for f in pbr.RAY_EXIT_DTYPE.names:
        assert np.array_equal(rec2[f], rec[f]), f
    assert st2["status"] == st["status"] and st2["rkn_steps"] == st["rkn_steps"]
