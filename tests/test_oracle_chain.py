"""Pins of the general optical chain of the oracle (sec. 3.3: mirrors, lenses and windows,
apertures, lens arrays as in a plenoptic camera): the built-in singlet rebuilt as a chain, a
flat window's lateral shift in closed form, a concave mirror returning every ray from its centre
of curvature, lenslets focusing at the thick-lens back focal distance, and the blocking rules."""
import math

import numpy as np
import pytest

import oracle
from oracle import SURF_APERTURE, SURF_LENSLETS, SURF_MIRROR, SURF_REFRACT
from paper_1812_05902_amd import inputs


@pytest.fixture(scope="module", autouse=True)
def oracle_lib():
    oracle.build()


def _uniform(sc):
    return sc.replace(field="uniform", field_params=dict(rho0=sc.rho_inf))


def singlet_chain(o, sc):
    """The built-in lens (aperture stop in the front-vertex plane, symmetric biconvex singlet)."""
    zl = sc.z_lens
    return [(SURF_APERTURE, zl, 0.0, o.a, 0.0, 0.0),
            (SURF_REFRACT, zl, o.R, o.clear, sc.n_glass, 0.0),
            (SURF_REFRACT, zl + o.t, -o.R, o.clear, 0.0, 0.0)]


def test_singlet_as_a_chain_equals_the_builtin_lens():
    sc = inputs.tiny_bos().replace(n_src=60, rays_per_src=20)
    src = inputs.sources(sc)
    o = oracle.scene_oracle(sc)
    ids = np.arange(sc.n_rays)
    ref = o.trace_ids(src, sc.rays_per_src, ids)
    o.set_chain(singlet_chain(o, sc), sc.z_lens, o.a)
    got = o.trace_ids(src, sc.rays_per_src, ids)
    assert np.array_equal(got["status"], ref["status"])
    ok = ref["status"] == oracle.DEPOSITED
    assert ok.sum() > 0.9 * sc.n_rays
    assert np.abs(got["sensor_px"][ok] - ref["sensor_px"][ok]).max() < 1e-9


def test_flat_window_shift_closed_form():
    """A slab of index n and thickness t shifts a ray tilted by theta sideways by
    t (tan theta - tan theta'), n sin theta' = n0 sin theta, and keeps its direction."""
    sc = _uniform(inputs.tiny_bos()).replace(z_sensor=1.0)
    o = oracle.scene_oracle(sc)
    n0, n, t, zw = o.n_inf, 1.52, 0.012, 0.3
    o.set_chain([(SURF_REFRACT, zw, 0.0, 0.5, n, 0.0), (SURF_REFRACT, zw + t, 0.0, 0.5, 0.0, 0.0)], 0.3, 0.01)
    P = np.array([0.001, -0.002, 0.2])
    for th in (0.0, 0.1, 0.3, 0.6):
        u = np.array([math.sin(th), 0.0, math.cos(th)])
        st, px = o.chain_to_sensor(P, u)
        assert st == oracle.DEPOSITED
        thp = math.asin(n0 * math.sin(th) / n)
        x_straight = P[0] + (1.0 - P[2]) * math.tan(th)
        x_want = x_straight - t * (math.tan(th) - math.tan(thp))
        assert (px[0] - 0.5 * sc.width) * sc.pitch == pytest.approx(x_want, abs=1e-13)
        assert (px[1] - 0.5 * sc.height) * sc.pitch == pytest.approx(P[1], abs=1e-13)


def test_concave_mirror_returns_rays_through_its_centre():
    """Every ray from the centre of curvature meets the mirror along the normal and comes back
    through the centre: on a sensor plane through the centre all rays land at one point."""
    sc = _uniform(inputs.tiny_bos())
    zm, R = 0.6, -0.2  # centre of curvature at z = 0.4, in front of the mirror
    sc = sc.replace(z_sensor=zm + R)
    o = oracle.scene_oracle(sc)
    o.set_chain([(SURF_MIRROR, zm, R, 0.05, 0.0, 0.0)], zm, 0.02)
    rng = np.random.default_rng(3)
    C = np.array([0.0, 0.0, zm + R])
    for _ in range(50):
        v = np.array([*rng.uniform(-0.15, 0.15, 2), 1.0])
        st, px = o.chain_to_sensor(C, v / np.linalg.norm(v))
        assert st == oracle.DEPOSITED
        np.testing.assert_allclose(px, [0.5 * sc.width, 0.5 * sc.height], atol=1e-9)
    # a plane mirror: angle of reflection equals the angle of incidence
    o.set_chain([(SURF_MIRROR, zm, 0.0, 0.05, 0.0, 0.0)], zm, 0.02)
    u = np.array([0.1, 0.05, 1.0]) / np.linalg.norm([0.1, 0.05, 1.0])
    P = np.array([0.0, 0.0, zm + R])
    st, px = o.chain_to_sensor(P, u)
    # out and back over the same height difference: lateral travel doubles
    d = 2 * (zm - P[2]) * u[:2] / u[2]
    np.testing.assert_allclose((px - [0.5 * sc.width, 0.5 * sc.height]) * sc.pitch, d, atol=1e-13)


def test_lenslets_focus_at_the_back_focal_distance():
    """Plano-convex lenslets (curved side first, radius r, index n, thickness tt) in a medium of
    index n0, on a square grid: a ray along a lenslet's axis goes straight; paraxial rays parallel
    to it cross that axis at the back focal distance n0 r/(n - n0) - tt n0/n behind the flat side."""
    n, r, tt, pitch, za = 1.5, 2e-4, 5e-5, 1e-4, 0.3
    sc = _uniform(inputs.tiny_bos()).replace(pitch=1e-6, width=2000, height=2000)
    n0 = oracle.scene_oracle(sc).n_inf
    bfd = n0 * r / (n - n0) - tt * n0 / n
    sc = sc.replace(z_sensor=za + tt + bfd)
    o = oracle.scene_oracle(sc)
    o.set_chain([(SURF_LENSLETS, za, r, 0.01, n, pitch), (SURF_REFRACT, za + tt, 0.0, 0.01, 0.0, 0.0)], za, 0.01)
    centre = np.array([0.5 * sc.width, 0.5 * sc.height])
    for k in (0, 3, -2):
        cx = k * pitch
        st, px = o.chain_to_sensor(np.array([cx, 0.0, 0.2]), np.array([0.0, 0.0, 1.0]))
        assert st == oracle.DEPOSITED
        np.testing.assert_allclose((px - centre) * sc.pitch, [cx, 0.0], atol=1e-15)
        for h in (1e-7, -2e-7):
            st, px = o.chain_to_sensor(np.array([cx + h, 0.0, 0.2]), np.array([0.0, 0.0, 1.0]))
            assert st == oracle.DEPOSITED
            # transverse aberration of the focused ray: third order in h/r
            assert abs((px[0] - centre[0]) * sc.pitch - cx) < 2 * abs(h) * (h / r) ** 2 * 10
    # a ray that crosses into the neighbouring cell inside the lenslet is blocked
    st, _ = o.chain_to_sensor(np.array([0.0, 0.0, 0.2]), np.array([0.6, 0.0, 0.8]))
    assert st == oracle.BLOCKED_LENS


def test_aperture_and_rim_blocking_and_tir():
    sc = _uniform(inputs.tiny_bos()).replace(z_sensor=1.0)
    o = oracle.scene_oracle(sc)
    o.set_chain([(SURF_APERTURE, 0.3, 0.0, 0.004, 0.0, 0.0), (SURF_REFRACT, 0.31, 0.0, 0.005, 1.5, 0.0)], 0.3, 0.004)
    st, _ = o.chain_to_sensor(np.array([0.0039, 0.0, 0.2]), np.array([0.0, 0.0, 1.0]))
    assert st == oracle.DEPOSITED
    st, _ = o.chain_to_sensor(np.array([0.0041, 0.0, 0.2]), np.array([0.0, 0.0, 1.0]))
    assert st == oracle.BLOCKED_APERTURE
    u = np.array([0.3, 0.0, 1.0]) / math.hypot(0.3, 1.0)  # passes the stop, misses the 5 mm rim
    st, _ = o.chain_to_sensor(np.array([0.0, 0.0, 0.29]), u)
    assert st == oracle.BLOCKED_LENS
    # glass to air beyond the critical angle: total internal reflection
    o.set_chain([(SURF_REFRACT, 0.3, 0.0, 0.05, 1.5, 0.0), (SURF_REFRACT, 0.31, 0.03, 0.05, 0.0, 0.0)], 0.3, 0.01)
    st, _ = o.chain_to_sensor(np.array([0.0, 0.024, 0.2]), np.array([0.0, 0.0, 1.0]))
    assert st == oracle.TIR
