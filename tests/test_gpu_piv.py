"""GPU parity of PIV frame pairs (sec. 1): particle displacement by a prescribed velocity field
against the oracle, and the two frames of a pair rendered with one seed."""
import numpy as np
import pytest

import oracle
from oracle import bos, piv
from paper_1812_05902_amd import inputs, pbr

pytestmark = pytest.mark.gpu


def _ulps(a, b):
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b).max()


@pytest.mark.parametrize("kind,substeps", [("vortex", 4), ("rotation", 1), ("shear", 7)])
def test_displacement_matches_oracle(kind, substeps):
    import torch
    p = dict(vortex=dict(gamma=0.05, rc=0.01, centre=(0.003, -0.002), u=(0.2, 0.0, 0.05)),
             rotation=dict(omega=20.0, centre=(0.0, 0.01)), shear=dict(gamma=30.0))[kind]
    vel, org, sp = inputs.velocity_field(kind, 33, **p)
    sc = inputs.tomo_piv_shock(n=8, n_src=5001)
    src = inputs.sources(sc)
    src[::97, 2] += 0.03  # some particles beyond the velocity grid
    src[:, 3] = np.linspace(0.1, 1.0, len(src), dtype=np.float32)
    want = piv.displace_sources(src, vel, org, sp, 2e-3, substeps).astype(np.float32)
    r = pbr.Renderer()
    got = r.displace_sources(src, vel, org, sp, 2e-3, substeps).cpu().numpy()
    moved = np.abs(want[:, :2] - src[:, :2]).max()
    print(f"\n{kind}: max displacement {moved * 1e3:.3f} mm, max difference {_ulps(got, want)} ulp")
    assert moved > 1e-5
    assert _ulps(got, want) <= 1
    # in place
    t = torch.as_tensor(src, device=r.device).contiguous()
    pbr.pbr_displace_sources(r.ctx, t, t, torch.as_tensor(vel, device=r.device).contiguous(), org, sp, 2e-3, substeps)
    assert np.array_equal(t.cpu().numpy(), got)
    # empty list: nothing to do, no error
    pbr.pbr_displace_sources(r.ctx, t[:0], t[:0], torch.as_tensor(vel, device=r.device), org, sp, 2e-3, substeps)


def _pair_scene():
    return inputs.tomo_piv_shock(n=64, n_src=400, rays_per_src=64).replace(width=512, height=512, pitch=40e-6)


def test_pair_second_frame_matches_oracle():
    """Frame B of a vortex pair, rendered from the GPU-displaced particles, against the oracle's
    render of the oracle-displaced particles (same seed as frame A)."""
    sc = _pair_scene()
    src = inputs.sources(sc)
    vel, org, sp = inputs.velocity_field("vortex", 33, gamma=0.05, rc=0.01)
    r = pbr.Renderer.from_scene(sc)
    b_src = r.displace_sources(src, vel, org, sp, 2e-3, 4)
    r.emit_and_trace(b_src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST)
    img = pbr.u64_image_to_numpy(r.read_image()).astype(np.float64)
    o_src = piv.displace_sources(src, vel, org, sp, 2e-3, 4).astype(np.float32)
    q, _, _ = oracle.scene_oracle(sc).render(o_src, sc.rays_per_src, want_float=False)
    rel = oracle.rel_l2(img, q.astype(np.float64))
    print(f"\nframe B image rel L2 vs oracle {rel:.2e}")
    assert rel <= 1e-3


def test_pair_is_noise_free():
    """Zero velocity: frame B is frame A bit for bit (one seed, one aperture point per ray in both
    frames).  Uniform in-plane motion of particles on the focused plane: every particle image moves
    by M dx / pitch (the image is inverted, M < 0), measured from per-particle hit means."""
    import torch
    sc = _pair_scene().replace(src_region=((-0.004, 0.004), (-0.004, 0.004), (0.0, 0.0)))
    sc = sc.replace(field="uniform", field_params=dict(rho0=sc.rho_inf))
    src = inputs.sources(sc)
    r = pbr.Renderer.from_scene(sc)
    flags = pbr.PBR_CLEAR_FIRST | pbr.PBR_SOURCE_SUMS
    sums_a = r.set_source_sums(sc.n_src)
    r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, flags)
    img_a = r.read_image().cpu().numpy()
    a = sums_a.cpu().numpy()
    zero, org, sp = inputs.velocity_field("uniform", 5, u=(0.0, 0.0, 0.0))
    b0 = r.displace_sources(src, zero, org, sp, 1e-3)
    r.set_source_sums(sc.n_src)
    r.emit_and_trace(b0, sc.rays_per_src, sc.ray_seed, sc.ds, flags)
    assert np.array_equal(r.read_image().cpu().numpy(), img_a)
    dx = 50e-6
    move, org, sp = inputs.velocity_field("uniform", 5, u=(dx / 1e-3, 0.0, 0.0))
    b1 = r.displace_sources(src, move, org, sp, 1e-3)
    sums_b = r.set_source_sums(sc.n_src)
    r.emit_and_trace(b1, sc.rays_per_src, sc.ray_seed, sc.ds, flags)
    b = sums_b.cpu().numpy()
    ok = (a[:, 2] > 0) & (b[:, 2] > 0)
    assert ok.mean() > 0.95
    d = b[ok, :2] / 2.0 ** 24 / b[ok, 2:3] - a[ok, :2] / 2.0 ** 24 / a[ok, 2:3]
    M = r.derived()["magnification"]
    want = M * dx / sc.pitch
    print(f"\nimage displacement {d[:, 0].mean():.4f} px (spread {d[:, 0].std():.1e}), M dx / pitch = {want:.4f}")
    assert abs(want) > 0.2
    assert np.abs(d[:, 0] - want).max() <= 0.005 * abs(want)
    assert np.abs(d[:, 1]).max() <= 0.005 * abs(want)
