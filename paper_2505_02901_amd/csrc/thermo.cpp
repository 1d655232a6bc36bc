// Finite-temperature Lanczos method (Jaklic and Prelovsek 1994; the
// thermodynamics examples of Sec. 4.6): R random start vectors per block, M
// Lanczos steps each, and the Gauss quadrature of the recurrence,
//   <r| f(H) |r> ~ sum_j w_j f(eps_j)   (eps_j Ritz values, w_j squared first
//   components of the Ritz vectors of T),
// summed over recurrences with weight D_block / R:
//   Z(T) = sum_r W_r sum_j w_rj exp(-eps_rj / T),
//   E(T) = <H>,  C(T) = (<H^2> - <H>^2) / T^2.
// Host arithmetic on the tridiagonal matrices returned by the batched
// Lanczos driver; exponents are shifted by the lowest Ritz value overall.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "xdg_internal.hpp"

namespace xdg {

int ftlm_thermo(int n_rec, int m, const double *alpha, const double *beta, const double *weight,
                int n_temp, const double *temps, double *energy, double *heat, double *log_z) {
    if (n_rec < 1 || m < 1 || !alpha || !beta || !weight || n_temp < 0 ||
        (n_temp > 0 && (!temps || !energy || !heat || !log_z))) {
        set_error("ftlm: bad arguments");
        return XDG_EINVAL;
    }
    for (int t = 0; t < n_temp; ++t)
        if (!(temps[t] > 0.0)) {
            set_error("ftlm: temperature %d is %g (must be > 0)", t, temps[t]);
            return XDG_EINVAL;
        }
    std::vector<std::vector<double>> ev(n_rec), w(n_rec);
    double e_min = INFINITY;
    for (int r = 0; r < n_rec; ++r) {
        const double *a = alpha + (size_t)r * m, *b = beta + (size_t)r * m;
        // a breakdown (invariant subspace) ends the recurrence
        int mm = m;
        for (int j = 0; j + 1 < m; ++j)
            if (b[j] <= 1e-13 * std::max(1.0, std::fabs(a[j])) || !std::isfinite(b[j])) {
                mm = j + 1;
                break;
            }
        tridiag_spectral_weights(mm, a, b, ev[r], w[r]);
        e_min = std::min(e_min, ev[r][0]);
    }
    for (int t = 0; t < n_temp; ++t) {
        const double T = temps[t];
        double z = 0.0, e1 = 0.0, e2 = 0.0;
        for (int r = 0; r < n_rec; ++r)
            for (size_t j = 0; j < ev[r].size(); ++j) {
                const double x = ev[r][j] - e_min;
                const double f = weight[r] * w[r][j] * std::exp(-x / T);
                z += f;
                e1 += f * x;
                e2 += f * x * x;
            }
        const double mean = e1 / z;
        energy[t] = mean + e_min;
        heat[t] = (e2 / z - mean * mean) / (T * T);
        log_z[t] = std::log(z) - e_min / T;
    }
    return XDG_OK;
}

// Spectral function from a Lanczos recurrence started at phi (continued
// fraction of the resolvent; the dynamical examples of Sec. 4.4):
//   G(z) = |phi|^2 / (z - a_0 - b_0^2 / (z - a_1 - b_1^2 / (...))),
//   z = omega + e0 + i eta,  S(omega) = -Im G(z) / pi.
// The fraction is evaluated from the bottom; a breakdown ends it.
int spectral_cf(int m, const double *alpha, const double *beta, double norm2, double e0,
                int n_w, const double *omega, double eta, double *out) {
    if (m < 1 || !alpha || !beta || n_w < 0 || (n_w > 0 && (!omega || !out)) || !(eta > 0.0)) {
        set_error("spectral: bad arguments (need m >= 1, eta > 0)");
        return XDG_EINVAL;
    }
    int mm = m;
    for (int j = 0; j + 1 < m; ++j)
        if (beta[j] <= 1e-13 * std::max(1.0, std::fabs(alpha[j])) || !std::isfinite(beta[j])) {
            mm = j + 1;
            break;
        }
    for (int k = 0; k < n_w; ++k) {
        const std::complex<double> z(omega[k] + e0, eta);
        std::complex<double> t = z - alpha[mm - 1];
        for (int j = mm - 2; j >= 0; --j) t = z - alpha[j] - beta[j] * beta[j] / t;
        out[k] = -std::imag(norm2 / t) / M_PI;
    }
    return XDG_OK;
}

}  // namespace xdg
