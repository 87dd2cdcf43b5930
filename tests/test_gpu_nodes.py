"""GPU parity of the node field layout (16 bytes per node; the integration kernel forms each cell's
coefficients from its corners): rays and images against the oracle and against the per-cell layout,
in FP32 and FP64, and the sec. 4 check on a node field."""
import numpy as np
import pytest

import oracle
from oracle import bos
from paper_1812_05902_amd import inputs, pbr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("flags,tol_oracle", [(0, 1e-4), (pbr.PBR_PREC_FP64_ALL, 1e-5)])
def test_node_layout_matches_oracle_and_cell_layout(flags, tol_oracle):
    sc = inputs.tiny_bos()
    src = inputs.sources(sc)
    rec = (0, 7, sc.n_rays // 7 + 1)
    rn, stn, recn = pbr.trace_scene(sc, src=src, record=rec, nodes=True, flags=pbr.PBR_CLEAR_FIRST | flags)
    rc, stc, recc = pbr.trace_scene(sc, src=src, record=rec, flags=pbr.PBR_CLEAR_FIRST | flags)
    ids = np.arange(0, sc.n_rays, 7)
    ref = oracle.scene_oracle(sc).trace_ids(src, sc.rays_per_src, ids)
    got = recn[: len(ids)]
    same = (got["status"] == ref["status"]) & (ref["status"] == oracle.DEPOSITED)
    err = np.abs(got["sensor_px"][same] - ref["sensor_px"][same]).max()
    both = (recn["status"] == recc["status"]) & (recc["status"] == pbr.PBR_RAY_DEPOSITED)
    dcell = np.abs(recn["sensor_px"][both] - recc["sensor_px"][both]).max()
    img = pbr.u64_image_to_numpy(rn.read_image()).astype(np.float64)
    q, _, _ = oracle.scene_oracle(sc).render(src, sc.rays_per_src, want_float=False)
    rel = oracle.rel_l2(img, q.astype(np.float64))
    print(f"\nnodes, flags {flags}: max |dpx| vs oracle {err:.2e}, vs cell layout {dcell:.2e}, image rel L2 {rel:.2e}, "
          f"{stn['rkn_steps']} steps (cells {stc['rkn_steps']})")
    assert same.mean() > 0.9
    assert err <= tol_oracle
    assert dcell <= tol_oracle
    assert rel <= 1e-3


def test_bos_check_on_a_node_field():
    """The Fig. 4 pipeline with the node layout: per-dot displacements equal the per-cell layout's
    to 1e-5 px, and the eq. 9 map matches the oracle."""
    import torch
    sc = inputs.bos_slice(n=129, n_src=400, rays_per_src=100)
    src = inputs.sources(sc)
    grid = (-0.02, -0.02, 6.5e-4, 6.5e-4, 62, 62, 0.0)
    disp = []
    for nodes in (False, True):
        maps = []
        sums = []
        for s in (sc, sc.replace(field="uniform", field_params=dict(rho0=sc.rho_inf))):
            r = pbr.Renderer.from_scene(s, nodes=nodes)
            t = r.set_source_sums(sc.n_src)
            r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST | pbr.PBR_SOURCE_SUMS)
            sums.append(t.cpu().numpy())
            if s is sc:
                maps.append(r.bos_theory_map(grid, 4 * (sc.nz - 1)).cpu().numpy().astype(np.float64))
        disp.append(bos.means_from_sums(sums[0]) - bos.means_from_sums(sums[1]))
        if nodes:
            want = bos.theory_map(oracle.scene_oracle(sc), grid, 4 * (sc.nz - 1))
            big = np.abs(want).max()
            err = np.abs(maps[0] - want).max()
            assert err <= 1e-4 * big, (err, big)
    ok = np.isfinite(disp[0][:, 0]) & np.isfinite(disp[1][:, 0])
    d = np.abs(disp[0][ok] - disp[1][ok]).max()
    print(f"\nper-dot displacement, node vs cell layout: max |d| {d:.2e} px over {ok.sum()} dots; eq. 9 map err {err:.2e}")
    assert ok.sum() > 350
    assert d <= 1e-5
