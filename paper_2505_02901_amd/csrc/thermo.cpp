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

// Canonical TPQ thermodynamics from microcanonical sequences (Sec. 4.6,
// after Sugiura and Shimizu 2013).  With h = H/N and |phi_k> = (l - h)^k |psi>
// for a unit |psi>, the moments M_n = <psi|(l - h)^n|psi> follow from the
// normalised sequence |k> = |phi_k> / sqrt(q_k):
//   q_0 = 1,  q_{k+1} = q_k <k|(l - h)^2|k> = q_k (l^2 - 2 l u_k + u2_k),
//   M_{2k} = q_k,  M_{2k+1} = q_k (l - u_k).
// The canonical state e^{-beta H / 2}|psi> = e^{-x l / 2} e^{x (l - h) / 2}|psi>,
// x = N beta, then has
//   <(l - h)^j> = S_j / S_0,  S_j = sum_n M_{n+j} x^n / n!,
//   <psi| e^{-beta H} |psi> = e^{-x l} S_0,
// with every sum over the moments that K steps give (n + j <= 2K).  The
// ensemble sums numerators and denominators over the sequences with their
// weights; the sums run in log space.  A series whose last kept term is not
// below 1e-12 of its sum is not converged at that temperature: NaN there.
int tpq_thermo(int n_rec, int n_steps, const double *u, const double *u2, double l, int n_sites,
               const double *weight, int n_temp, const double *temps, double *energy,
               double *heat, double *log_z) {
    if (n_rec < 1 || n_steps < 1 || !u || !u2 || !weight || n_sites < 1 || !std::isfinite(l) ||
        n_temp < 0 || (n_temp > 0 && (!temps || !energy || !heat || !log_z))) {
        set_error("tpq: bad arguments");
        return XDG_EINVAL;
    }
    for (int t = 0; t < n_temp; ++t)
        if (!(temps[t] > 0.0)) {
            set_error("tpq: temperature %d is %g (must be > 0)", t, temps[t]);
            return XDG_EINVAL;
        }
    const int K = n_steps;
    // log moments per sequence; -inf for a zero moment (the sequence ended
    // in an eigenvector of h with eigenvalue l: every later moment is zero)
    std::vector<std::vector<double>> lm(n_rec, std::vector<double>(2 * (size_t)K + 1, -INFINITY));
    for (int r = 0; r < n_rec; ++r) {
        const double *ur = u + (size_t)r * K, *u2r = u2 + (size_t)r * K;
        if (!(weight[r] > 0.0)) {
            set_error("tpq: weight %d is %g (must be > 0)", r, weight[r]);
            return XDG_EINVAL;
        }
        double lq = 0.0;   // log q_k
        for (int k = 0; k < K; ++k) {
            const double a = l - ur[k];
            if (a < 0.0) {
                set_error("tpq: l = %g is below <k|H/N|k> = %g (sequence %d, step %d)", l, ur[k],
                          r, k);
                return XDG_EINVAL;
            }
            lm[r][2 * k] = lq;
            lm[r][2 * k + 1] = a > 0.0 ? lq + std::log(a) : -INFINITY;
            const double q = l * l - 2.0 * l * ur[k] + u2r[k];
            if (!(q > 0.0)) break;
            lq += std::log(q);
            if (k + 1 == K) lm[r][2 * K] = lq;
        }
    }
    const double N = (double)n_sites;
    for (int t = 0; t < n_temp; ++t) {
        const double x = N / temps[t], lx = std::log(x);
        // log of sum_r w_r S_j^(r), j = 0, 1, 2, and the convergence test
        double ls[3];
        bool ok = true;
        for (int j = 0; j < 3; ++j) {
            const int nmax = 2 * K - j;
            double mx = -INFINITY;
            for (int r = 0; r < n_rec; ++r)
                for (int n = 0; n <= nmax; ++n)
                    mx = std::max(mx, std::log(weight[r]) + lm[r][n + j] + n * lx -
                                          std::lgamma(n + 1.0));
            double s = 0.0, last = 0.0;
            for (int r = 0; r < n_rec; ++r)
                for (int n = 0; n <= nmax; ++n) {
                    const double e = std::exp(std::log(weight[r]) + lm[r][n + j] + n * lx -
                                              std::lgamma(n + 1.0) - mx);
                    s += e;
                    if (n == nmax) last += e;
                }
            ls[j] = mx + std::log(s);
            if (last > 1e-12 * s) ok = false;
        }
        const double a1 = std::exp(ls[1] - ls[0]), a2 = std::exp(ls[2] - ls[0]);
        energy[t] = ok ? N * (l - a1) : NAN;
        heat[t] = ok ? x * x * (a2 - a1 * a1) : NAN;
        log_z[t] = ok ? ls[0] - x * l : NAN;
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
