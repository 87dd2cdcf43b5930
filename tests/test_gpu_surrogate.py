"""GPU: the ray surrogate network's own kernels against the FP64 oracle of the network (in its
bfloat16-emulation mode: the same roundings at the same places), then the trained surrogate inside
the trace: fallback map, exit error against the tracer in pixels, and what it gains in time."""
import numpy as np
import pytest

from oracle import mlp
from paper_1812_05902_amd import inputs, pbr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pbr.load()
    return torch


def _params32(seed):
    """Oracle initialisation rounded to the FP32 master weights both sides then use."""
    v = mlp.flatten(mlp.init_params(seed)).astype(np.float32)
    return v, mlp.unflatten(v.astype(np.float64))


def _batch(rows, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(rows, 6)).astype(np.float32)
    t = rng.normal(size=(rows, 6)).astype(np.float32)
    return x, t


@pytest.mark.parametrize("rows", [64, 200, 1000])
def test_forward_matches_oracle(torch, rows):
    v, p = _params32(11)
    s = pbr.Surrogate(init_seed=0, max_rows=256)  # 1000 rows: several passes and a ragged tail
    s.set_params(v)
    assert np.array_equal(s.params(), v)
    x, _ = _batch(rows, 5)
    y = s.forward(x).cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(p, x.astype(np.float64), bf=True)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"rows {rows}: forward max rel err {err:.3g}")
    assert err <= 1e-3
    s.close()


def test_gradients_match_oracle(torch):
    v, p = _params32(12)
    s = pbr.Surrogate(init_seed=0, max_rows=512)
    s.set_params(v)
    x, t = _batch(320, 6)  # five 64-row groups
    loss, g = s.gradients(x, t)
    y, cache = mlp.forward(p, x.astype(np.float64), bf=True)
    L, dy = mlp.loss_and_grad_y(y, t.astype(np.float64))
    gr = mlp.backward(p, cache, dy, bf=True)
    assert loss == pytest.approx(L, rel=1e-3)
    gg = mlp.unflatten(g.astype(np.float64))
    for k in mlp.PARAM_ORDER:
        rel = np.linalg.norm(gg[k] - gr[k]) / np.linalg.norm(gr[k])
        # element by element: within 2% of the element or 1e-3 of the tensor's largest entry (the
        # bfloat16 roundings match the oracle's, only the FP32 summation order differs)
        d = np.abs(gg[k] - gr[k])
        bound = 2e-2 * np.abs(gr[k]) + 1e-3 * np.abs(gr[k]).max()
        worst = float((d / bound).max())
        print(f"{k}: grad rel err {rel:.3g}, worst element at {worst:.3g} of its bound")
        assert rel <= 1e-2, k
        assert worst <= 1.0, k
    # the bfloat16 roundings are where the oracle puts them: against the pure-FP64 gradient the
    # difference is of bfloat16 size, far above the emulation's agreement for the hidden weights
    y64, c64 = mlp.forward(p, x.astype(np.float64))
    g64 = mlp.backward(p, c64, mlp.loss_and_grad_y(y64, t.astype(np.float64))[1])
    rel64 = np.linalg.norm(gg["W3"] - g64["W3"]) / np.linalg.norm(g64["W3"])
    rel_bf = np.linalg.norm(gg["W3"] - gr["W3"]) / np.linalg.norm(gr["W3"])
    print(f"W3 vs FP64 {rel64:.3g}, vs bf16 emulation {rel_bf:.3g}")
    assert rel_bf < rel64
    s.close()


def test_adam_steps_match_oracle(torch):
    v, p = _params32(13)
    s = pbr.Surrogate(init_seed=0, max_rows=256)
    s.set_params(v)
    x, t = _batch(128, 7)
    w = mlp.flatten(p)
    m = np.zeros_like(w)
    q = np.zeros_like(w)
    for step in range(1, 4):
        s.adam_step(x, t, 1e-3, step)
        pp = mlp.unflatten(w)
        y, cache = mlp.forward(pp, x.astype(np.float64), bf=True)
        g = mlp.flatten(mlp.backward(pp, cache, mlp.loss_and_grad_y(y, t.astype(np.float64))[1], bf=True))
        w, m, q = mlp.adam_step(w, g, m, q, step, lr=1e-3)
    got = s.params().astype(np.float64)
    d_gpu, d_orc = got - v.astype(np.float64), w - v.astype(np.float64)
    rel = np.linalg.norm(d_gpu - d_orc) / np.linalg.norm(d_orc)
    print(f"3 Adam steps: update rel err {rel:.3g}")
    assert rel <= 1e-2
    s.close()


def test_argument_errors(torch):
    s = pbr.Surrogate(init_seed=0, max_rows=128)
    x, t = _batch(100, 1)
    with pytest.raises(pbr.PbrError, match="multiple of 64"):
        s.gradients(x, t)
    with pytest.raises(pbr.PbrError, match="expected 200710"):
        s.set_params(np.zeros(10, np.float32))
    with pytest.raises(pbr.PbrError, match="not trained"):
        s.tiles = 1
        s.tile_map()
    r = pbr.Renderer(rays_per_chunk=1 << 12)
    with pytest.raises(pbr.PbrError, match="not trained"):
        s.attach(r)
    s.close()
    r.close()


def _tiny_renderer(sc, chunk=1 << 18):
    r = pbr.Renderer(rays_per_chunk=chunk)
    r.set_density_field(inputs.density(sc), sc.origin, sc.spacing, sc.K, sc.rho_inf)
    r.set_optics(sc.z_lens, sc.focal_length, sc.f_number, sc.thickness, sc.n_glass, sc.clear_radius, sc.z_focus)
    r.set_sensor(sc.width, sc.height, sc.pitch, sc.z_sensor, sc.wavelength, sc.sigma_px, sc.dtau_with_pi)
    return r


@pytest.fixture(scope="module")
def trained(torch):
    """Gaussian-bump BOS scene (32^3): a surrogate trained on 2e5 tracer rays, validated on 1e5
    others."""
    sc = inputs.tiny_bos()
    r = _tiny_renderer(sc, chunk=1 << 22)
    tr = inputs.sources(sc.replace(n_src=2000, src_seed=501))
    va = inputs.sources(sc.replace(n_src=1000, src_seed=502))
    s = pbr.Surrogate(init_seed=3, max_rows=1 << 16)
    rep = s.train(r, tr, 100, va, 100, train_seed=50, val_seed=52, ds=sc.ds, batch=2048, epochs=30,
                  lr_max=2e-3, lr_min=2e-5, tol_px=0.01, tiles=16, min_tile_samples=8)
    print("train report:", rep)
    yield sc, r, s, rep
    s.close()
    r.close()


def test_surrogate_in_the_trace(torch, trained):
    """Render 5e5 unseen rays with and without the surrogate: fallback map, exit error against the
    tracer ray by ray, untouched rays outside the eligible tiles, image difference."""
    sc, r, s, rep = trained
    assert rep["train_samples"] > 100000 and rep["val_samples"] > 50000
    assert rep["loss_last_epoch"] < 0.05 * rep["loss_first_epoch"]
    ok, err = s.tile_map()
    print("eligible tiles", int(ok.sum()), "of", ok.size)
    assert rep["eligible_tiles"] == int(ok.sum()) > 0
    assert np.all(err[ok.astype(bool)] <= 0.01)
    assert rep["val_max_eligible_px"] <= 0.01

    ev = inputs.sources(sc.replace(n_src=5000, src_seed=503))
    n_rays = 5000 * 100
    r.set_exit_recording(0, 1, n_rays)
    st_t = r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS, stats=True)
    img_t = pbr.u64_image_to_numpy(r.read_image()).astype(np.float64)
    rec_t = r.read_ray_exits()
    s.attach(r)
    st_s = r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_SURROGATE,
                            stats=True)
    img_s = pbr.u64_image_to_numpy(r.read_image()).astype(np.float64)
    rec_s = r.read_ray_exits()
    print("tracer", st_t, "\nsurrogate", st_s)
    assert st_s["surrogate_rays"] > 0
    assert sum(st_s["status"]) == n_rays
    surr = (rec_s["entered"] == 1) & (rec_s["n_steps"] == 0) & (rec_t["n_steps"] > 0)
    assert int(surr.sum()) == st_s["surrogate_rays"]
    both = surr & (rec_s["status"] == 0) & (rec_t["status"] == 0)
    e = np.hypot(*(rec_s["sensor_px"][both] - rec_t["sensor_px"][both]).T)
    rim = int((surr & (rec_s["status"] != rec_t["status"])).sum())
    print(f"surrogate rays {surr.sum()}: exit error vs tracer median {np.median(e):.3g} px, "
          f"p99 {np.quantile(e, 0.99):.3g}, max {e.max():.3g}; status differs on {rim}")
    # every ray through the network lands within 0.01 px of the tracer's hit, and rays whose
    # aperture or lens status would change stay with the tracer (rim tiles are never eligible)
    assert e.max() <= 0.01
    assert rim <= max(1, int(1e-4 * surr.sum()))
    # rays outside eligible tiles are traced exactly as without the surrogate
    rest = ~surr
    assert np.array_equal(rec_s["sensor_px"][rest], rec_t["sensor_px"][rest])
    rel = np.linalg.norm(img_s - img_t) / np.linalg.norm(img_t)
    print(f"image rel L2 surrogate vs tracer {rel:.3g}")
    assert rel < 1e-2
    # with the sources in a random order (chunks and waves made of other rays) every ray through the
    # network or the tracer gives the same bits: image, records and counts
    order = np.random.default_rng(5).permutation(len(ev))
    r.set_source_order(torch.as_tensor(order))
    st_o = r.emit_and_trace(ev, 100, 51, sc.ds,
                            pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_SURROGATE | pbr.PBR_SOURCE_ORDER,
                            stats=True)
    assert np.array_equal(pbr.u64_image_to_numpy(r.read_image()).astype(np.float64), img_s)
    rec_o = r.read_ray_exits()
    for f in pbr.RAY_EXIT_DTYPE.names:
        assert np.array_equal(rec_o[f], rec_s[f]), f
    assert st_o["status"] == st_s["status"] and st_o["surrogate_rays"] == st_s["surrogate_rays"]
    r.set_source_order(None)
    r.set_exit_recording(0, 1, 0)


def test_surrogate_gain_over_the_tracer(torch, trained):
    """What the trained network gains: on 5e6 rays (two trace chunks of up to 2^22 rays) the
    integration steps drop to the rays left to the tracer and the whole trace (emission, network or
    integration, lens, deposit) takes less time than with the tracer alone.  (The rays left to the
    tracer in a chunk take as long as their longest path: a fixed cost per chunk, which large
    chunks amortise.)"""
    sc, r, s, rep = trained
    s.attach(r)
    ev = torch.as_tensor(inputs.sources(sc.replace(n_src=50000, src_seed=504)), device="cuda")
    t_ms, s_ms = [], []
    for _ in range(3):
        st_t = r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST, stats=True)
        st_s = r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE, stats=True)
        t_ms.append(st_t["trace_ms"])
        s_ms.append(st_s["trace_ms"])
    print(f"5e6 rays: tracer {min(t_ms):.2f} ms ({st_t['rkn_steps']} steps), with the surrogate "
          f"{min(s_ms):.2f} ms ({st_s['rkn_steps']} steps, {st_s['surrogate_rays']} rays through the "
          f"network): {min(t_ms) / min(s_ms):.2f}x")
    assert st_s["surrogate_rays"] > 0.9 * st_t["entered_volume"]
    assert st_s["rkn_steps"] < 0.05 * st_t["rkn_steps"]
    assert min(s_ms) < 0.8 * min(t_ms)


def test_surrogate_buffers_bound_the_trace_chunk(torch, trained):
    """The surrogate's inference buffers are sized at creation for trace chunks of 2^22 rays: a
    context whose chunk is larger is refused (WORKSPACE) before any launch; the allocation-free
    trace with a chunk inside that size runs the network and renders the same image as the
    workspace trace."""
    sc, r, s, rep = trained
    s.attach(r)
    ev = torch.as_tensor(inputs.sources(sc.replace(n_src=3000, src_seed=505)), device="cuda")
    flags = pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE
    st_ws = r.emit_and_trace(ev, 100, 51, sc.ds, flags, stats=True)
    img_ws = pbr.u64_image_to_numpy(r.read_image())
    st_na = pbr.stats_dict(pbr.pbr_emit_and_trace_noalloc(r.ctx, ev, 100, 51, sc.ds, flags, 1 << 20,
                                                          want_stats=True))
    img_na = pbr.u64_image_to_numpy(r.read_image())
    assert st_na["surrogate_rays"] == st_ws["surrogate_rays"] > 0
    assert np.array_equal(img_na, img_ws)
    big = torch.empty(pbr.pbr_trace_workspace_bytes(1 << 23) // 8, dtype=torch.int64, device="cuda")
    pbr.pbr_set_trace_workspace(r.ctx, big)
    try:
        with pytest.raises(pbr.PbrError, match="trace chunks of at most") as ei:
            r.emit_and_trace(ev, 100, 51, sc.ds, flags)
        assert ei.value.code == pbr.PBR_ERR_WORKSPACE
    finally:
        pbr.pbr_set_trace_workspace(r.ctx, r.trace_ws)
    assert np.array_equal(pbr.u64_image_to_numpy(r.read_image()), img_ws)  # the refused call left no trace


def test_save_and_load(torch, trained):
    """A saved surrogate loaded into a fresh context of the same scene gives the same parameters,
    tile map and image bit for bit; another field, a damaged blob or another step length is refused."""
    sc, r, s, rep = trained
    blob = s.save()
    r2 = _tiny_renderer(sc, chunk=1 << 22)
    s2 = pbr.Surrogate(max_rows=1 << 16)
    s2.load(r2, blob)
    assert np.array_equal(s2.params(), s.params())
    assert np.array_equal(s2.tile_map()[0], s.tile_map()[0])
    assert np.array_equal(s2.tile_map()[1], s.tile_map()[1])
    assert s2.save() == blob
    s.attach(r)
    s2.attach(r2)
    ev = inputs.sources(sc.replace(n_src=2000, src_seed=506))
    st1 = r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE, stats=True)
    st2 = r2.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE, stats=True)
    assert st1["surrogate_rays"] == st2["surrogate_rays"] > 0
    assert np.array_equal(r.read_image().cpu().numpy(), r2.read_image().cpu().numpy())
    print(f"blob {len(blob)} bytes; {st2['surrogate_rays']} rays through the loaded surrogate, same image")
    with pytest.raises(pbr.PbrError, match="steps of"):
        r2.emit_and_trace(ev, 100, 51, 2 * sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE)
    bad = bytearray(blob)
    bad[len(bad) // 2] ^= 1
    s3 = pbr.Surrogate(max_rows=1024)
    with pytest.raises(pbr.PbrError, match="checksum"):
        s3.load(r2, bytes(bad))
    with pytest.raises(pbr.PbrError, match="not a surrogate"):
        s3.load(r2, b"x" * 64)
    other = sc.replace(field_params=dict(sc.field_params, amp=0.11))
    r3 = _tiny_renderer(other)
    with pytest.raises(pbr.PbrError, match="differ"):
        s3.load(r3, blob)
    for x in (s2, s3, r2, r3):
        x.close()


def test_scene_change_invalidates_the_surrogate(torch, trained):
    sc, r, s, rep = trained
    s.attach(r)
    ev = inputs.sources(sc.replace(n_src=10, src_seed=505))
    r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE)
    r.set_optics(sc.z_lens, sc.focal_length, sc.f_number, sc.thickness, sc.n_glass, sc.clear_radius, sc.z_focus)
    with pytest.raises(pbr.PbrError, match="no longer matches"):
        r.emit_and_trace(ev, 100, 51, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SURROGATE)
    with pytest.raises(pbr.PbrError, match="changed since"):
        s.attach(r)


def test_training_is_deterministic(torch):
    """Two trainings with the same seeds give the same parameters bit for bit (fixed-order
    reductions everywhere: split-K slices and row-block partial sums are added in index order).
    About 34 steps per epoch, so each epoch replays the 16-step graph twice and the one-step graph
    for the rest, and three epochs cycle through both order buffers."""
    sc = inputs.tiny_bos()
    r = _tiny_renderer(sc)
    tr = inputs.sources(sc.replace(n_src=700, src_seed=601))
    va = inputs.sources(sc.replace(n_src=200, src_seed=602))
    out = []
    for _ in range(2):
        s = pbr.Surrogate(init_seed=4, max_rows=1024)
        rep = s.train(r, tr, 50, va, 20, train_seed=60, val_seed=62, ds=sc.ds, batch=1024, epochs=3,
                      tiles=8, min_tile_samples=4)
        spe = rep["train_samples"] // 1024
        assert spe % 16 != 0 and spe > 16 and rep["steps"] == 3 * spe
        out.append((s.params(), rep, s.tile_map()[0]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1]["loss_last_epoch"] == out[1][1]["loss_last_epoch"]
    assert np.array_equal(out[0][2], out[1][2])
    r.close()


def test_surrogate_at_the_256_turbulence_scale(torch):
    """The surrogate workload's own scene and training set: 256^3 turbulence field, 1e7 training and
    1e6 validation rays, 8 epochs; then 2e6 unseen rays (2000 dots x 1000) rendered with and
    without the network, every second ray recorded: every ray the network takes lands within
    0.01 px of the tracer's hit, rim status changes stay within 1e-4 of them, the rays left to the
    tracer are traced exactly as without the network, and the images agree to 1e-2 rel. L2."""
    ev, tr, va = inputs.surrogate_turbulence()
    rho = inputs.density(ev)
    r = pbr.Renderer.from_scene(ev, rho=rho, rays_per_chunk=1 << 22)
    s = pbr.Surrogate(init_seed=7, max_rows=1 << 18, ray_chunk=1 << 22)
    rep = s.train(r, inputs.sources(tr), tr.rays_per_src, inputs.sources(va), va.rays_per_src, tr.ray_seed,
                  va.ray_seed, ev.ds, batch=4096, epochs=8, lr_max=1e-3, lr_min=1e-5, tol_px=0.01, tiles=64,
                  min_tile_samples=8)
    print("256^3 training:", {k: rep[k] for k in ("train_samples", "steps", "loss_first_epoch", "loss_last_epoch",
                                                  "eligible_tiles", "val_p99_px", "val_max_eligible_px")})
    assert rep["train_samples"] > 9_000_000 and rep["loss_last_epoch"] < 0.02 * rep["loss_first_epoch"]
    assert rep["eligible_tiles"] > 1000 and rep["val_max_eligible_px"] <= 0.01
    sc = ev.replace(n_src=2000, src_seed=530)
    src = torch.as_tensor(inputs.sources(sc), device="cuda").contiguous()
    r.set_exit_recording(0, 2, sc.n_rays // 2)
    r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS)
    img_t = pbr.u64_image_to_numpy(r.read_image()).astype(np.float64)
    rec_t = r.read_ray_exits()
    s.attach(r)
    st = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds,
                          pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS | pbr.PBR_SURROGATE, stats=True)
    img_s = pbr.u64_image_to_numpy(r.read_image()).astype(np.float64)
    rec_s = r.read_ray_exits()
    surr = (rec_s["entered"] == 1) & (rec_s["n_steps"] == 0) & (rec_t["n_steps"] > 0)
    both = surr & (rec_s["status"] == 0) & (rec_t["status"] == 0)
    e = np.hypot(*(rec_s["sensor_px"][both] - rec_t["sensor_px"][both]).T)
    rim = int((surr & (rec_s["status"] != rec_t["status"])).sum())
    rel = np.linalg.norm(img_s - img_t) / np.linalg.norm(img_t)
    print(f"256^3: {st['surrogate_rays']} of {sc.n_rays} rays through the network; on {both.sum()} recorded: "
          f"median {np.median(e):.2e} px, p99 {np.quantile(e, 0.99):.2e}, max {e.max():.2e}; rim {rim}; "
          f"image rel L2 {rel:.2e}")
    assert st["surrogate_rays"] > 0.5 * sc.n_rays and both.sum() > 0.4 * len(rec_s)
    assert e.max() <= 0.01
    assert rim <= max(1, int(1e-4 * surr.sum()))
    assert np.array_equal(rec_s["sensor_px"][~surr], rec_t["sensor_px"][~surr])
    assert rel < 1e-2
    s.close()
    r.close()
