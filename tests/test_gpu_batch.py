"""GPU: batches of uneven images in one graph-captured launch sequence.

Image k of a batch must equal, bit for bit, the same image rendered alone (integer deposits and
identical per-ray arithmetic), for every configuration the autotuner may pick, on graph replays,
and when images are split across rounds."""
import numpy as np
import pytest

from paper_1812_05902_amd import inputs, pbr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pbr.load()
    return torch


def _small_batch(n=6):
    """Uneven images shaped like the 64-image workload, scaled down: grids 17-41^3, 20-300
    particles, 30-400 rays each, sensors 64-256 px."""
    out = []
    rng = np.random.default_rng(77)
    for i, sc in enumerate(inputs.batch_scenes(n_images=n, seed_base=4100)):
        g = int(rng.choice([17, 25, 41]))
        w = int(rng.choice([64, 128, 256]))
        org, sp = inputs._centred_box((g, g, g), (0.1, 0.1, 0.1), 0.0)
        fp = sc.field_params
        if sc.field == "turbulence":
            fp = dict(fp, kmax=min(fp["kmax"], (g - 1) // 2 - 1))
        out.append(sc.replace(nx=g, ny=g, nz=g, origin=org, spacing=sp, field_params=fp,
                              n_src=int(rng.integers(20, 300)), rays_per_src=int(rng.integers(30, 400)),
                              width=w, height=w, pitch=10e-6 * 2048 / w))
    return out


def _renderers(scenes, nodes=None):
    rs = []
    for i, sc in enumerate(scenes):
        r = pbr.Renderer(rays_per_chunk=1 << 16)
        r.set_density_field(inputs.density(sc), sc.origin, sc.spacing, sc.K, sc.rho_inf,
                            nodes=bool(nodes[i]) if nodes is not None else False)
        r.set_optics(sc.z_lens, sc.focal_length, sc.f_number, sc.thickness, sc.n_glass, sc.clear_radius,
                     sc.z_focus)
        r.set_sensor(sc.width, sc.height, sc.pitch, sc.z_sensor, sc.wavelength, sc.sigma_px, sc.dtau_with_pi)
        rs.append(r)
    return rs


def test_batch_equals_single_renders_bitwise(torch):
    scenes = _small_batch()
    srcs = [inputs.sources(sc) for sc in scenes]
    singles = _renderers(scenes)
    ref, ref_st = [], []
    for r, sc, s in zip(singles, scenes, srcs):
        ref_st.append(r.emit_and_trace(s, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST, stats=True))
        ref.append(pbr.u64_image_to_numpy(r.read_image()))
    rs = _renderers(scenes)
    b = pbr.Batch(rs, srcs, [sc.rays_per_src for sc in scenes], [sc.ray_seed for sc in scenes],
                  [sc.ds for sc in scenes], round_rays=1 << 16)
    print("batch config:", b.config())

    def check(tag):
        st = b.run()
        for k, r in enumerate(rs):
            img = pbr.u64_image_to_numpy(r.read_image())
            assert np.array_equal(img, ref[k]), f"{tag}: image {k} differs"
        assert st["rays"] == sum(sc.n_rays for sc in scenes)
        assert st["status"] == [sum(x["status"][j] for x in ref_st) for j in range(7)]
        assert st["rkn_steps"] == sum(x["rkn_steps"] for x in ref_st)
        return st

    st = check("first run (capture)")
    print("rounds", st["rounds"], "run_ms", st["run_ms"])
    check("graph replay")
    cfg = b.config()
    for bb, ur, tl in ((256, 256, 16), (64, 128, 32), (256, 64, 16)):
        b.configure(box_block=bb, unit_rays=ur, tile=tl, round_rays=cfg["min_round_rays"])
        st = check(f"config {bb}/{ur}/{tl} min round")
        assert st["rounds"] >= 1


def test_batch_records_and_accumulate(torch):
    scenes = _small_batch(3)
    srcs = [inputs.sources(sc) for sc in scenes]
    single = _renderers(scenes[:1])[0]
    single.set_exit_recording(0, 3, 500)
    single.emit_and_trace(srcs[0], scenes[0].rays_per_src, scenes[0].ray_seed, scenes[0].ds,
                          pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS)
    rec_ref = single.read_ray_exits()
    rs = _renderers(scenes)
    rs[0].set_exit_recording(0, 3, 500)
    b = pbr.Batch(rs, srcs, [sc.rays_per_src for sc in scenes], [sc.ray_seed for sc in scenes],
                  [sc.ds for sc in scenes],
                  flags=[pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS, pbr.PBR_CLEAR_FIRST, 0])
    rs[2].emit_and_trace(srcs[2], scenes[2].rays_per_src, scenes[2].ray_seed, scenes[2].ds, pbr.PBR_CLEAR_FIRST)
    once = pbr.u64_image_to_numpy(rs[2].read_image())
    b.run()
    rec = rs[0].read_ray_exits()
    for f in pbr.RAY_EXIT_DTYPE.names:
        bad = np.nonzero(np.any((rec[f] != rec_ref[f]).reshape(len(rec), -1), axis=1))[0]
        assert bad.size == 0, (f, bad[:10], rec[bad[:3]], rec_ref[bad[:3]], scenes[0].n_rays)
    # the third item accumulates onto what its sensor held: twice the single image
    assert np.array_equal(pbr.u64_image_to_numpy(rs[2].read_image()), once * np.uint64(2))


def test_autotune_and_cache(torch, tmp_path):
    scenes = _small_batch(4)
    srcs = [inputs.sources(sc) for sc in scenes]
    rs = _renderers(scenes)
    b = pbr.Batch(rs, srcs, [sc.rays_per_src for sc in scenes], [sc.ray_seed for sc in scenes],
                  [sc.ds for sc in scenes], round_rays=1 << 17)
    cache = tmp_path / "tune.txt"
    cfg, rate = b.autotune(cache_path=cache, probe_rounds=1)
    print("autotune:", cfg, rate, "rays/ms")
    assert rate > 0 and cache.exists()
    assert len(cache.read_text().strip().splitlines()) == 1
    b.configure(box_block=256 if cfg["box_block"] == 64 else 64)
    cfg2, rate2 = b.autotune(cache_path=cache)  # from the cache, no re-timing
    assert cfg2 == cfg and rate2 == pytest.approx(rate, rel=1e-5)
    assert len(cache.read_text().strip().splitlines()) == 1
    # a tuned batch still renders the same images
    singles = _renderers(scenes)
    st = b.run()
    for k, (r, sc, s) in enumerate(zip(singles, scenes, srcs)):
        r.emit_and_trace(s, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
        assert np.array_equal(pbr.u64_image_to_numpy(rs[k].read_image()), pbr.u64_image_to_numpy(r.read_image()))
    assert st["rays"] == sum(sc.n_rays for sc in scenes)


def test_batch_refuses_contexts_changed_since_creation(torch):
    """A batch replays launch parameters taken from its contexts at creation: after a context's
    sensor or exit recording changes, running (or tuning) the batch fails with STATE instead of
    tracing through stale pointers; a new batch over the changed contexts runs."""
    scenes = _small_batch(2)
    srcs = [inputs.sources(sc) for sc in scenes]
    rs = _renderers(scenes)
    mk = lambda: pbr.Batch(rs, srcs, [sc.rays_per_src for sc in scenes], [sc.ray_seed for sc in scenes],
                           [sc.ds for sc in scenes], round_rays=1 << 16)
    b = mk()
    b.run()
    sc = scenes[1]
    rs[1].set_sensor(sc.width // 2, sc.height // 2, sc.pitch, sc.z_sensor, sc.wavelength, sc.sigma_px,
                     sc.dtau_with_pi)
    for call in (b.run, lambda: b.autotune(probe_rounds=1)):
        with pytest.raises(pbr.PbrError) as ei:
            call()
        assert ei.value.code == pbr.PBR_ERR_STATE
    b.close()
    b = mk()
    b.run()
    rs[0].set_exit_recording(0, 1, 10)
    with pytest.raises(pbr.PbrError) as ei:
        b.run()
    assert ei.value.code == pbr.PBR_ERR_STATE
    b.close()


def test_batch_mixes_field_layouts(torch):
    """Images stored per node and per cell in one batch (two persistent integration kernels per
    round, one queue each): every image equals its single render in the same layout bit for bit,
    before and after tuning, and a node image's records match the oracle (1e-4 px)."""
    import oracle
    scenes = _small_batch(5)
    nodes = [False, True, True, False, True]
    srcs = [inputs.sources(sc) for sc in scenes]
    singles = _renderers(scenes, nodes)
    ref = []
    for r, sc, s in zip(singles, scenes, srcs):
        r.emit_and_trace(s, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
        ref.append(pbr.u64_image_to_numpy(r.read_image()))
    rs = _renderers(scenes, nodes)
    k = 1
    rs[k].set_exit_recording(0, 1, scenes[k].n_rays)
    flags = [pbr.PBR_CLEAR_FIRST | (pbr.PBR_RECORD_EXITS if i == k else 0) for i in range(len(scenes))]
    b = pbr.Batch(rs, srcs, [s.rays_per_src for s in scenes], [s.ray_seed for s in scenes],
                  [s.ds for s in scenes], flags=flags, round_rays=1 << 16)
    st = b.run()
    print(f"\nmixed-layout batch: {st['rounds']} rounds, config {b.config()}")
    assert st["rounds"] > 1
    for i, r in enumerate(rs):
        assert np.array_equal(pbr.u64_image_to_numpy(r.read_image()), ref[i]), f"image {i} (nodes={nodes[i]})"
    rec = rs[k].read_ray_exits()
    ids = np.arange(scenes[k].n_rays)
    o = oracle.scene_oracle(scenes[k]).trace_ids(srcs[k], scenes[k].rays_per_src, ids)
    same = rec["status"] == o["status"]
    dep = same & (o["status"] == oracle.DEPOSITED)
    err = np.abs(rec["sensor_px"][dep] - o["sensor_px"][dep]).max()
    print(f"node image {k}: {dep.sum()} deposited rays, max |dpx| vs oracle {err:.2e}")
    assert same.mean() > 0.999 and dep.sum() > 0.5 * len(ids) and err <= 1e-4
    b.autotune(probe_rounds=1)
    b.run()
    for i, r in enumerate(rs):
        assert np.array_equal(pbr.u64_image_to_numpy(r.read_image()), ref[i]), f"tuned image {i}"
    b.close()


def _batch_vs_oracle(scenes, k, stride, tol_px=1e-4):
    """Renders the scenes as one batch with exit records on image k (every stride-th ray) and
    compares image k's records and image with the oracle's."""
    import oracle
    srcs = [inputs.sources(sc) for sc in scenes]
    rs = _renderers(scenes)
    sc = scenes[k]
    nrec = (sc.n_rays + stride - 1) // stride
    rs[k].set_exit_recording(0, stride, nrec)
    flags = [pbr.PBR_CLEAR_FIRST | (pbr.PBR_RECORD_EXITS if i == k else 0) for i in range(len(scenes))]
    b = pbr.Batch(rs, srcs, [s.rays_per_src for s in scenes], [s.ray_seed for s in scenes],
                  [s.ds for s in scenes], flags=flags, round_rays=1 << 20)
    st = b.run()
    rec = rs[k].read_ray_exits()
    img = pbr.u64_image_to_numpy(rs[k].read_image()).astype(np.float64)
    o = oracle.scene_oracle(sc)
    ids = np.arange(0, sc.n_rays, stride)
    ref = o.trace_ids(srcs[k], sc.rays_per_src, ids)
    assert np.array_equal(rec["ray_id"], ids)
    same = rec["status"] == ref["status"]
    dep = same & (ref["status"] == oracle.DEPOSITED)
    err = np.abs(rec["sensor_px"][dep] - ref["sensor_px"][dep]).max()
    print(f"\nbatch of {len(scenes)} ({st['rounds']} rounds), image {k}: {sc.nx}^3 grid, {sc.width}^2 sensor, "
          f"{sc.n_rays} rays; {dep.sum()} sampled deposited rays, max |dpx| vs oracle {err:.2e}, "
          f"status mismatches {(~same).sum()}", flush=True)
    assert same.mean() > 0.999
    assert dep.sum() > 0.5 * len(ids)
    assert err <= tol_px
    b.close()
    return img, o, srcs[k]


def test_batch_image_and_records_match_oracle(torch):
    """Image 1 of a small uneven batch: every ray's record against the oracle's trace (1e-4 px),
    and the image against the oracle's Q32.32 render (rel. L2 1e-3)."""
    import oracle
    scenes = _small_batch(3)
    img, o, src = _batch_vs_oracle(scenes, 1, 1)
    q, _, _ = o.render(src, scenes[1].rays_per_src, want_float=False)
    rel = oracle.rel_l2(img, q.astype(np.float64))
    print(f"image rel L2 vs oracle {rel:.2e}")
    assert rel <= 1e-3


def test_full_size_batch64_image_matches_oracle_on_sampled_rays(torch):
    """Three images of the 64-image workload at full size (their grids, sensors, particle and
    ray counts) in one batch; the largest is checked against the oracle on about 1500 strided
    rays."""
    scenes = inputs.batch_scenes(64)[:3]
    k = int(np.argmax([sc.nx * 1000 + sc.width for sc in scenes]))
    stride = max(1, scenes[k].n_rays // 1500)
    _batch_vs_oracle(scenes, k, stride)
