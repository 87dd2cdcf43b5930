// Mie-scattering intensity of a homogeneous sphere (sec. 3.1, after Bohren & Huffman, 1983,
// ch. 4), computed on the host once per particle type: the series of the scattering
// coefficients a_n, b_n (Riccati-Bessel functions by upward recurrence, the logarithmic derivative
// of the inner solution by downward recurrence) and the amplitude functions S1, S2 from the
// angular functions pi_n, tau_n.  Output: the unpolarised intensity (|S1|^2 + |S2|^2) / 2 at
// n_angles equally spaced scattering angles over [0, pi], divided by its maximum.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace pbr {
namespace host {

bool mie_intensity_table(std::complex<double> m, double x, int n_angles, double *out)
{
    using cplx = std::complex<double>;
    if (!(x > 0.0) || n_angles < 2) return false;
    const int terms = (int)std::lround(x + 4.0 * std::cbrt(x) + 2.0);  // Wiscombe's series length
    const cplx mx = m * x;
    const int start = (int)std::max((double)terms, std::abs(mx)) + 16;
    // D_k(mx) = psi_k'(mx) / psi_k(mx), from D_start = 0 downwards (stable for any m)
    std::vector<cplx> logd((size_t)start + 1, cplx(0.0, 0.0));
    for (int k = start; k > 0; --k) {
        const cplx q = (double)k / mx;
        logd[(size_t)k - 1] = q - 1.0 / (logd[(size_t)k] + q);
    }
    std::vector<cplx> an((size_t)terms), bn((size_t)terms);
    double psi_prev2 = std::cos(x), psi_prev = std::sin(x);    // psi_{-1}, psi_0
    double chi_prev2 = -std::sin(x), chi_prev = std::cos(x);   // chi_{-1}, chi_0
    for (int k = 1; k <= terms; ++k) {
        const double c = (2.0 * k - 1.0) / x;
        const double psi = c * psi_prev - psi_prev2;
        const double chi = c * chi_prev - chi_prev2;
        const cplx xi(psi, -chi), xi_prev(psi_prev, -chi_prev);
        const cplx ta = logd[(size_t)k] / m + (double)k / x;
        const cplx tb = m * logd[(size_t)k] + (double)k / x;
        an[(size_t)k - 1] = (ta * psi - psi_prev) / (ta * xi - xi_prev);
        bn[(size_t)k - 1] = (tb * psi - psi_prev) / (tb * xi - xi_prev);
        psi_prev2 = psi_prev; psi_prev = psi;
        chi_prev2 = chi_prev; chi_prev = chi;
    }
    double peak = 0.0;
    for (int t = 0; t < n_angles; ++t) {
        const double mu = std::cos((double)t * (3.14159265358979323846 / (double)(n_angles - 1)));
        cplx s1(0.0, 0.0), s2(0.0, 0.0);
        double pi_prev = 0.0, pi_cur = 1.0;  // pi_0, pi_1
        for (int k = 1; k <= terms; ++k) {
            if (k > 1) {
                const double pn = (2.0 * k - 1.0) / (k - 1.0) * mu * pi_cur - (double)k / (k - 1.0) * pi_prev;
                pi_prev = pi_cur;
                pi_cur = pn;
            }
            const double tau = k * mu * pi_cur - (k + 1.0) * pi_prev;
            const double wgt = (2.0 * k + 1.0) / (k * (k + 1.0));
            s1 += wgt * (an[(size_t)k - 1] * pi_cur + bn[(size_t)k - 1] * tau);
            s2 += wgt * (an[(size_t)k - 1] * tau + bn[(size_t)k - 1] * pi_cur);
        }
        out[t] = 0.5 * (std::norm(s1) + std::norm(s2));
        peak = std::max(peak, out[t]);
    }
    if (!(peak > 0.0) || !std::isfinite(peak)) return false;
    for (int t = 0; t < n_angles; ++t) out[t] /= peak;
    return true;
}

}  // namespace host
}  // namespace pbr
