"""Pins of the PIV frame-pair oracle: particle displacement by a prescribed velocity field (RK4 on
the trilinearly interpolated field) against exact solutions — translation, shear, solid-body
rotation with fourth-order convergence — and the edge extension outside the velocity grid."""
import math

import numpy as np
import pytest

import oracle
from oracle import piv
from paper_1812_05902_amd import inputs


@pytest.fixture(scope="module", autouse=True)
def oracle_lib():
    oracle.build()


def _particles(n=200, seed=3, box=((-0.05, 0.05), (-0.05, 0.05), (-0.015, 0.015))):
    rng = np.random.default_rng(seed)
    src = np.ones((n, 4), np.float32)
    for a in range(3):
        src[:, a] = rng.uniform(*box[a], n)
    src[:, 3] = rng.uniform(0.2, 1.0, n).astype(np.float32)
    return src


def test_uniform_translation_is_exact():
    vel, org, sp = inputs.velocity_field("uniform", 9, u=(1.5, -0.75, 0.25))
    src = _particles()
    out = piv.displace_sources(src, vel, org, sp, 2e-4, 3)
    want = src[:, :3].astype(np.float64) + 2e-4 * np.array([1.5, -0.75, 0.25])
    np.testing.assert_allclose(out[:, :3], want, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(out[:, 3], src[:, 3].astype(np.float64))


def test_outside_the_grid_takes_the_nearest_face_value():
    vel, org, sp = inputs.velocity_field("uniform", 5, region=((-0.01, 0.01),) * 3, u=(0.5, 0.0, -1.0))
    src = _particles(50, box=((-0.05, 0.05), (-0.05, 0.05), (0.02, 0.04)))  # all beyond the grid
    out = piv.displace_sources(src, vel, org, sp, 1e-3, 2)
    np.testing.assert_allclose(out[:, :3] - src[:, :3], np.tile([5e-4, 0.0, -1e-3], (50, 1)), atol=1e-15)


def test_shear_is_exact():
    """u = (gamma y, 0, 0): y stays put, x moves by gamma y dt (RK4 is exact for this field)."""
    vel, org, sp = inputs.velocity_field("shear", 17, gamma=40.0)
    src = _particles()
    out = piv.displace_sources(src, vel, org, sp, 1e-3, 4)
    y = src[:, 1].astype(np.float64)
    np.testing.assert_allclose(out[:, 0], src[:, 0] + 40.0 * y * 1e-3, rtol=0, atol=1e-14)
    np.testing.assert_allclose(out[:, 1:3], src[:, 1:3].astype(np.float64), rtol=0, atol=1e-15)


def _rotation_error(substeps):
    omega, dt = 50.0, 0.02  # one radian
    vel, org, sp = inputs.velocity_field("rotation", 11, omega=omega, centre=(0.004, -0.003))
    src = _particles(100, seed=5, box=((-0.03, 0.03), (-0.03, 0.03), (-0.01, 0.01)))
    out = piv.displace_sources(src, vel, org, sp, dt, substeps)
    c = np.array([0.004, -0.003])
    d = src[:, :2].astype(np.float64) - c
    a = omega * dt
    ex = c + np.stack([d[:, 0] * math.cos(a) - d[:, 1] * math.sin(a), d[:, 0] * math.sin(a) + d[:, 1] * math.cos(a)], 1)
    assert np.abs(out[:, 2] - src[:, 2]).max() < 1e-15
    return np.abs(out[:, :2] - ex).max()


def test_rotation_matches_exact_solution_at_fourth_order():
    """Solid-body rotation (a linear field, so the trilinear interpolation is exact) by one radian:
    RK4's phase error is n (w h)^5 / 120 radians for n steps of w h, and halving h cuts it ~16
    times (checked at 4 and 8 steps; the float32 velocity nodes set a floor near 1e-9 m)."""
    r_max = math.hypot(0.034, 0.033)
    e4, e8 = _rotation_error(4), _rotation_error(8)
    assert e8 <= 1.1 * 8 * (1 / 8) ** 5 / 120 * r_max + 2e-9
    assert 13 < e4 / e8 < 19, (e4, e8)
