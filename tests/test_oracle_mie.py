"""Pins of the Mie oracle (sec. 3.1, Bohren & Huffman's series): the Rayleigh limit (efficiency and
angular shape in closed form), the optical theorem, the scattered energy as the integral of the
amplitude functions over all directions, no absorption without an imaginary index, and the
extinction paradox (Q_ext -> 2) for large spheres."""
import numpy as np
import pytest

from oracle import mie


def test_rayleigh_limit():
    """x << 1: Q_sca = (8/3) x^4 |(m^2-1)/(m^2+2)|^2 and i(theta) proportional to (1 + cos^2)/2."""
    m, x = 1.5 + 0.0j, 0.01
    K = (m * m - 1) / (m * m + 2)
    qext, qsca = mie.efficiencies(m, x)
    assert qsca == pytest.approx(8.0 / 3.0 * x ** 4 * abs(K) ** 2, rel=1e-3)
    t = mie.intensity_table(m, x, 181)
    th = np.linspace(0, np.pi, 181)
    np.testing.assert_allclose(t, (1 + np.cos(th) ** 2) / 2, rtol=1e-3)


def test_optical_theorem():
    """Q_ext = 4/x^2 Re S(0), with S1(0) = S2(0)."""
    for m, x in ((1.33 + 0j, 3.0), (1.59 + 0.01j, 12.5), (2.0 + 1.0j, 0.7)):
        S1, S2 = mie.amplitudes(m, x, np.array([1.0]))
        assert S1[0] == pytest.approx(S2[0], rel=1e-12)
        qext, _ = mie.efficiencies(m, x)
        assert qext == pytest.approx(4.0 / x ** 2 * S1[0].real, rel=1e-10)


@pytest.mark.parametrize("m,x", [(1.33 + 0j, 2.0), (1.59 + 0j, 8.0), (1.5 + 0.1j, 5.0)])
def test_scattered_energy_is_the_integral_of_the_amplitudes(m, x):
    """Q_sca = 1/x^2 int_0^pi (|S1|^2 + |S2|^2) sin(theta) dtheta: ties the angular functions
    pi_n, tau_n and the series weights to the coefficient sum."""
    nodes, weights = np.polynomial.legendre.leggauss(400)  # in mu = cos(theta)
    S1, S2 = mie.amplitudes(m, x, nodes)
    integral = np.sum(weights * (np.abs(S1) ** 2 + np.abs(S2) ** 2)) / x ** 2
    _, qsca = mie.efficiencies(m, x)
    assert integral == pytest.approx(qsca, rel=1e-9)


def test_no_absorption_for_a_real_index():
    for x in (0.5, 4.0, 40.0):
        qext, qsca = mie.efficiencies(1.45 + 0j, x)
        assert qext == pytest.approx(qsca, rel=1e-10)
    qext, qsca = mie.efficiencies(1.45 + 0.05j, 4.0)
    assert qext > qsca * 1.01


def test_extinction_paradox():
    qext, _ = mie.efficiencies(1.33 + 0j, 800.0)
    assert abs(qext - 2.0) < 0.03


def test_table_normalised_and_forward_peaked_for_piv_particles():
    """A 1 um oil droplet in air at 532 nm (x ~ 5.9): largest weight 1, forward scattering
    strongest, side scattering (where a PIV camera looks) orders of magnitude weaker."""
    x = mie.size_parameter(1e-6, 532e-9, 1.000277)
    t = mie.intensity_table(1.47 + 0j, x)
    assert t.max() == 1.0 and t[0] == 1.0
    assert t[len(t) // 2] < 1e-2
    assert (t > 0).all()


def test_render_weights_each_ray_by_its_scattering_angle():
    """With a Mie table set, the oracle's image total is the sum over deposited rays of
    (source weight x table value at acos(u0 . k)) times the spot mass inside the window; a table
    of ones reproduces the unweighted image bit for bit; the interpolation hits table nodes exactly."""
    import oracle
    from paper_1812_05902_amd import inputs
    oracle.build()
    sc = inputs.tiny_bos().replace(n_src=40, rays_per_src=16, field="uniform", field_params=dict(rho0=1.2))
    src = inputs.sources(sc)
    o = oracle.scene_oracle(sc)
    q0, f0, _ = o.render(src, sc.rays_per_src)
    o.set_mie(np.ones(33), (1.0, 0.0, 0.0))
    q1, _, _ = o.render(src, sc.rays_per_src)
    assert np.array_equal(q0, q1)
    t = mie.intensity_table(1.47 + 0j, 5.9, 33)
    o.set_mie(t, (0.0, 2.0, 0.0))  # direction normalised inside
    for k in (0, 7, 16, 32):
        th = k * np.pi / 32
        assert o.mie_weight([np.sin(th), np.cos(th), 0.0]) == pytest.approx(t[k], rel=1e-12)
    _, f2, _ = o.render(src, sc.rays_per_src)
    ids = np.arange(sc.n_rays)
    rec = o.trace_ids(src, sc.rays_per_src, ids)
    dep = rec["status"] == oracle.DEPOSITED
    w = np.array([o.mie_weight(u) for u in rec["dir0"][dep]])
    # uniform field and a 3-sigma window: nearly all of each spot lands in the window
    assert f2.sum() == pytest.approx(w.sum(), rel=2e-3)
    assert f2.sum() < 0.5 * f0.sum()


@pytest.mark.parametrize("m,x", [(1.33 + 0j, 3.0), (1.59 + 0.01j, 8.0), (1.5 + 0.1j, 0.7), (1.47 + 0j, 25.0)])
def test_series_against_spherical_bessel_and_legendre_functions(m, x):
    """The recurrences of the oracle against the closed definitions, evaluated another way:
    a_n, b_n from Riccati-Bessel functions psi_n(z) = z j_n(z), xi_n(x) = x h_n^(1)(x) (scipy's
    spherical Bessel functions, complex argument m x), and pi_n = P_n'(mu),
    tau_n = mu P_n'(mu) - (1 - mu^2) P_n''(mu) from numpy's Legendre polynomials."""
    from numpy.polynomial import legendre as L
    from scipy.special import spherical_jn, spherical_yn
    a, b = mie.coefficients(m, x)
    n = np.arange(1, len(a) + 1)

    def psi(z):
        return z * spherical_jn(n, z)

    def dpsi(z):
        return spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)

    h = spherical_jn(n, x) + 1j * spherical_yn(n, x)
    dh = spherical_jn(n, x, derivative=True) + 1j * spherical_yn(n, x, derivative=True)
    xi, dxi = x * h, h + x * dh
    mx = m * x
    A = (m * psi(mx) * dpsi(x) - psi(x) * dpsi(mx)) / (m * psi(mx) * dxi - xi * dpsi(mx))
    B = (psi(mx) * dpsi(x) - m * psi(x) * dpsi(mx)) / (psi(mx) * dxi - m * xi * dpsi(mx))
    big = max(np.abs(a).max(), np.abs(b).max())
    assert np.abs(A - a).max() <= 1e-10 * big
    assert np.abs(B - b).max() <= 1e-10 * big
    mu = np.cos(np.linspace(0.0, np.pi, 37))
    S1 = np.zeros(mu.shape, complex)
    S2 = np.zeros(mu.shape, complex)
    for k in n:
        P = L.Legendre.basis(int(k))
        pk = P.deriv(1)(mu)
        tk = mu * pk - (1 - mu * mu) * P.deriv(2)(mu)
        f = (2 * k + 1) / (k * (k + 1))
        S1 += f * (A[k - 1] * pk + B[k - 1] * tk)
        S2 += f * (A[k - 1] * tk + B[k - 1] * pk)
    s1, s2 = mie.amplitudes(m, x, mu)
    scale = max(np.abs(S1).max(), np.abs(S2).max())
    assert np.abs(S1 - s1).max() <= 1e-9 * scale
    assert np.abs(S2 - s2).max() <= 1e-9 * scale


def test_weight_is_linear_in_the_scattering_angle_between_nodes():
    """orc_mie_weight between table nodes: a table linear in theta (t_k = theta_k / pi) gives
    exactly theta / pi at any angle, and a table of theta_k^2 gives the chord value
    theta^2 + (theta - theta_k)(theta_k+1 - theta) at points between nodes; an interpolation in
    cos(theta), or an index off by one, fails both."""
    import oracle
    from paper_1812_05902_amd import inputs
    oracle.build()
    sc = inputs.tiny_bos().replace(n_src=1, rays_per_src=1)
    o = oracle.scene_oracle(sc)
    n = 33
    nodes = np.arange(n) * (np.pi / (n - 1))
    rng = np.random.default_rng(4)
    th = np.concatenate([rng.uniform(0, np.pi, 200), [0.0, np.pi, nodes[5] + 1e-9, nodes[31] - 1e-9]])
    laser = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    e1 = np.cross(laser, [1.0, 0.0, 0.0])
    e1 /= np.linalg.norm(e1)
    o.set_mie(nodes / np.pi, laser * 3.0)
    for t in th:
        u = np.cos(t) * laser + np.sin(t) * e1
        assert o.mie_weight(u) == pytest.approx(t / np.pi, abs=1e-12)
    o.set_mie(nodes ** 2, laser)
    for t in th[:200]:
        k = min(int(t / (np.pi / (n - 1))), n - 2)
        want = t * t + (t - nodes[k]) * (nodes[k + 1] - t)
        u = np.cos(t) * laser + np.sin(t) * e1
        assert o.mie_weight(u) == pytest.approx(want, abs=1e-10)
