"""Oracle of the Mie-scattering radiance of sec. 3.1 (the paper computes it following Bohren &
Huffman, "Absorption and Scattering of Light by Small Particles", 1983, ch. 4): the amplitude
functions S1, S2 of a homogeneous sphere from the series of the scattering coefficients a_n, b_n,
and the table of angular intensity the ray weights are looked up in.

Test infrastructure only (see the package docstring).  Plain FP64 numpy, written from the series:
  size parameter x = pi d n_medium / lambda, relative index m, y = m x;
  D_n(y) = psi_n'(y) / psi_n(y) by the downward recurrence D_{n-1} = n/y - 1/(D_n + n/y);
  Riccati-Bessel psi_n, chi_n by the upward recurrence f_n = (2n-1)/x f_{n-1} - f_{n-2}
  (psi_{-1} = cos x, psi_0 = sin x, chi_{-1} = -sin x, chi_0 = cos x), xi_n = psi_n - i chi_n;
  a_n = ((D_n/m + n/x) psi_n - psi_{n-1}) / ((D_n/m + n/x) xi_n - xi_{n-1}),
  b_n = ((m D_n + n/x) psi_n - psi_{n-1}) / ((m D_n + n/x) xi_n - xi_{n-1});
  pi_n(mu) = (2n-1)/(n-1) mu pi_{n-1} - n/(n-1) pi_{n-2} (pi_0 = 0, pi_1 = 1),
  tau_n = n mu pi_n - (n+1) pi_{n-1};
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n), S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n);
  Q_ext = 2/x^2 sum (2n+1) Re(a_n + b_n), Q_sca = 2/x^2 sum (2n+1) (|a_n|^2 + |b_n|^2).
Series length n_stop = round(x + 4 x^(1/3) + 2) (Wiscombe's criterion).
"""
from __future__ import annotations

import numpy as np

TABLE_SIZE = 2049


def coefficients(m: complex, x: float):
    """a_n, b_n for n = 1 .. n_stop."""
    m = complex(m)
    nstop = int(round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    y = m * x
    nmx = int(max(nstop, abs(y))) + 16
    D = np.zeros(nmx + 1, dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / y - 1.0 / (D[n] + n / y)
    a = np.zeros(nstop, dtype=np.complex128)
    b = np.zeros(nstop, dtype=np.complex128)
    psi_m2, psi_m1 = np.cos(x), np.sin(x)      # psi_{-1}, psi_0
    chi_m2, chi_m1 = -np.sin(x), np.cos(x)     # chi_{-1}, chi_0
    for n in range(1, nstop + 1):
        psi = (2 * n - 1) / x * psi_m1 - psi_m2
        chi = (2 * n - 1) / x * chi_m1 - chi_m2
        xi, xi_m1 = complex(psi, -chi), complex(psi_m1, -chi_m1)
        da = D[n] / m + n / x
        db = m * D[n] + n / x
        a[n - 1] = (da * psi - psi_m1) / (da * xi - xi_m1)
        b[n - 1] = (db * psi - psi_m1) / (db * xi - xi_m1)
        psi_m2, psi_m1 = psi_m1, psi
        chi_m2, chi_m1 = chi_m1, chi
    return a, b


def amplitudes(m: complex, x: float, mu):
    """S1(mu), S2(mu) at mu = cos(theta) (array)."""
    a, b = coefficients(m, x)
    mu = np.asarray(mu, dtype=np.float64)
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros(mu.shape, dtype=np.complex128)
    pi_m1 = np.zeros(mu.shape)    # pi_0
    pi_n = np.ones(mu.shape)      # pi_1
    for n in range(1, len(a) + 1):
        if n > 1:
            pi_new = (2 * n - 1) / (n - 1) * mu * pi_n - n / (n - 1) * pi_m1
            pi_m1, pi_n = pi_n, pi_new
        tau = n * mu * pi_n - (n + 1) * pi_m1
        f = (2 * n + 1) / (n * (n + 1))
        S1 += f * (a[n - 1] * pi_n + b[n - 1] * tau)
        S2 += f * (a[n - 1] * tau + b[n - 1] * pi_n)
    return S1, S2


def efficiencies(m: complex, x: float):
    """(Q_ext, Q_sca)."""
    a, b = coefficients(m, x)
    n = np.arange(1, len(a) + 1)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * (a + b).real)
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(qext), float(qsca)


def size_parameter(diameter: float, wavelength: float, n_medium: float) -> float:
    return float(np.pi * diameter * n_medium / wavelength)


def intensity_table(m: complex, x: float, n: int = TABLE_SIZE):
    """Unpolarised scattered intensity (|S1|^2 + |S2|^2) / 2 at theta_k = k pi / (n - 1),
    divided by its largest value (so every ray weight stays in [0, 1])."""
    th = np.arange(n) * (np.pi / (n - 1))
    S1, S2 = amplitudes(m, x, np.cos(th))
    i = 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2)
    return i / i.max()
