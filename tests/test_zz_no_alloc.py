"""The allocation-free trace entry point, pbr_emit_and_trace_noalloc (ray states in the library's
static device array), against pbr_emit_and_trace (ray states in the context's trace workspace) on
the same context and sources: images bit for bit (integer deposits), exit records and counters
equal, on two calls in a row, the second with fewer sources and a smaller chunk."""
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


def _trace(torch, r, sc, src, chunk, noalloc):
    flags = pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS
    r.rec.zero_()
    if noalloc:
        st = pbr.stats_dict(pbr.pbr_emit_and_trace_noalloc(r.ctx, src, sc.rays_per_src, sc.ray_seed, sc.ds, flags,
                                                           chunk, want_stats=True))
    else:
        st = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, flags, stats=True)
    n = int(src.shape[0]) * sc.rays_per_src
    return st, pbr.u64_image_to_numpy(r.read_image()), r.read_ray_exits(0, n)


@pytest.mark.parametrize("nodes", [False, True], ids=["cells", "nodes"])
def test_noalloc_trace_equals_the_workspace_trace(torch, nodes):
    sc = inputs.tiny_bos()
    src_all = torch.as_tensor(inputs.sources(sc), device="cuda").contiguous()
    r = pbr.Renderer.from_scene(sc, nodes=nodes, rays_per_chunk=1 << 16)
    r.set_exit_recording(0, 1, sc.n_rays)
    # two calls in a row: all sources in one static chunk, then fewer sources over several chunks
    for n_src, chunk in ((sc.n_src, 0), (sc.n_src // 3 + 7, 4096 + 64)):
        print(f"noalloc check: nodes={nodes} n_src={n_src} rays_per_src={sc.rays_per_src} chunk={chunk}", flush=True)
        src = src_all[:n_src].contiguous()
        st_ref, img_ref, rec_ref = _trace(torch, r, sc, src, chunk, noalloc=False)
        st, img, rec = _trace(torch, r, sc, src, chunk, noalloc=True)
        assert img.sum() > 0
        assert np.array_equal(img, img_ref)
        assert rec.tobytes() == rec_ref.tobytes()
        for k in ("rays", "status", "entered_volume", "rkn_steps"):
            assert st[k] == st_ref[k], k
        assert st["box_ms"] == 0.0
        want = -(-n_src * sc.rays_per_src // (chunk or pbr.PBR_NOALLOC_MAX_CHUNK))
        assert st["box_launches"] == want
    r.close()


def test_noalloc_rejects_chunks_beyond_the_static_array(torch):
    sc = inputs.tiny_bos().replace(n_src=4, rays_per_src=64)
    r = pbr.Renderer.from_scene(sc)
    src = torch.as_tensor(inputs.sources(sc), device="cuda").contiguous()
    for bad in (pbr.PBR_NOALLOC_MAX_CHUNK + 1, 255, -1):
        with pytest.raises(pbr.PbrError) as ei:
            pbr.pbr_emit_and_trace_noalloc(r.ctx, src, sc.rays_per_src, sc.ray_seed, sc.ds, 0, bad)
        assert ei.value.code == pbr.PBR_ERR_ARG
        assert "rays_per_chunk" in str(ei.value)
    r.close()
