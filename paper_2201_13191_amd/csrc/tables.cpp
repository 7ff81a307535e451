// Cross-section, spectrum and response tables of the transport (host side).
//
// Interaction coefficients per material on the 1 keV grid E_j = 1 + j, in
// cm^2/g, evaluated in x87 extended precision and rounded once to fp32:
//   - Compton: N_A (Z/A) sigma_KN(E), sigma_KN the integral over the sphere
//     of the Klein-Nishina cross section, eq. (1) with S(q,Z) = 1;
//   - Rayleigh: the integral of eq. (2) with the screened form factor
//     F(x,Z) = Z / (1 + b x^2)^2, x = sin(theta/2)/lambda, b = (2 pi r_Z)^2,
//     r_Z = 0.885 a0 Z^(-1/3) (a Thomas-Fermi screening radius; the paper's
//     Hubbell tables are replaced by this parametric form);
//   - photoelectric: N_A (Z/A) C Z^3 / E^3 with one constant C (per-electron
//     Z^3/E^3 scaling; no absorption edges).
#include "tables.hpp"

#include <cmath>
#include <utility>

namespace mcx {
namespace {

constexpr long double kPi = 3.141592653589793238462643383279502884L;
constexpr long double kRe = 2.8179403262e-13L;     // classical electron radius, cm (CODATA)
constexpr long double kMec2 = 510.99895L;          // keV
constexpr long double kAvogadro = 6.02214076e23L;  // 1/mol
constexpr long double kHc = 12.398419843320026L;   // keV * Angstrom
constexpr long double kBohr = 0.529177210903L;     // Angstrom
constexpr long double kPhoto = 3.2e-23L;           // cm^2 keV^3 per electron, times Z^3

// Klein-Nishina total cross section per electron (cm^2).
long double klein_nishina_total(long double e_kev) {
    const long double k = e_kev / kMec2;
    const long double d = 1.0L + 2.0L * k;
    const long double ln = std::log1p(2.0L * k);
    const long double first = (1.0L + k) / (k * k) * (2.0L * (1.0L + k) / d - ln / k);
    const long double second = ln / (2.0L * k);
    const long double third = (1.0L + 3.0L * k) / (d * d);
    return 2.0L * kPi * kRe * kRe * (first + second - third);
}

// (1/V) * integral_0^V (1 + cos^2(theta(v))) (1 + b v)^-4 dv with B = b V,
// cos(theta) = 1 - 2 v / V.  Power series in B below 0.1, closed form in
// w = 1 + b v above.
long double coherent_shape(long double B) {
    if (B < 0.1L) {
        long double sum = 0.0L;
        long double pw = 1.0L;
        for (int i = 0; i <= 40; ++i) {
            const long double c3 = (long double)(i + 1) * (i + 2) * (i + 3) / 6.0L;
            const long double t =
                c3 * pw * (2.0L / (i + 1) - 4.0L / (i + 2) + 4.0L / (i + 3));
            sum += (i % 2 == 0) ? t : -t;
            pw *= B;
        }
        return sum;
    }
    const long double r1 = 1.0L / (1.0L + B);
    const long double r2 = r1 * r1;
    const long double r3 = r2 * r1;
    const long double m0 = (1.0L - r3) / 3.0L;
    const long double m1 = 1.0L / 6.0L - r2 / 2.0L + r3 / 3.0L;
    const long double m2 = 1.0L / 3.0L - r1 + r2 - r3 / 3.0L;
    return 2.0L * m0 / B - 4.0L * m1 / (B * B) + 4.0L * m2 / (B * B * B);
}

long double screening_b(long double z) {
    const long double r = 0.885L * kBohr / std::cbrt(z);
    const long double t = 2.0L * kPi * r;
    return t * t;
}

}  // namespace

void kn_norm_series(double *c, int n) {
    // K(a) = 2 [A + B + C + D] with A = 2 (1 + a)^2 / (a^2 (1 + 2a)),
    // B = -(1 + a) ln(1 + 2a) / a^3, C = ln(1 + 2a) / (2a), D = -(1 + 3a) / (1 + 2a)^2;
    // with 1/(1+2a) = sum g_k a^k, ln(1+2a) = sum l_k a^k, 1/(1+2a)^2 = sum h_k a^k the
    // coefficient of a^k is 2 [2 (g_{k+2} + 2 g_{k+1} + g_k) - (l_{k+3} + l_{k+2})
    // + l_{k+1} / 2 - h_k - 3 h_{k-1}] (the negative powers cancel).
    auto g = [](int k) { return k < 0 ? 0.0L : std::pow(-2.0L, (long double)k); };
    auto l = [](int k) {
        return k < 1 ? 0.0L : ((k % 2) ? 1.0L : -1.0L) * std::pow(2.0L, (long double)k) / k;
    };
    auto h = [](int k) { return k < 0 ? 0.0L : (k + 1) * std::pow(-2.0L, (long double)k); };
    for (int k = 0; k < n; ++k)
        c[k] = (double)(2.0L * (2.0L * (g(k + 2) + 2.0L * g(k + 1) + g(k)) -
                                (l(k + 3) + l(k + 2)) + l(k + 1) / 2.0L - h(k) - 3.0L * h(k - 1)));
}

void coherent_series(double *d, int n) {
    for (int i = 0; i < n; ++i) {
        const long double c3 = (long double)(i + 1) * (i + 2) * (i + 3) / 6.0L;
        const long double t = c3 * (2.0L / (i + 1) - 4.0L / (i + 2) + 4.0L / (i + 3));
        d[i] = (double)((i % 2 == 0) ? t : -t);
    }
}

void attenuation_coefficients(double z_eff, double z_over_a, double e_kev, double out[3]) {
    const long double z = z_eff, e = e_kev;
    const long double electrons = kAvogadro * (long double)z_over_a;
    out[0] = (double)(electrons * kPhoto * z * z * z / (e * e * e));
    const long double inv_lambda = e / kHc;
    const long double B = screening_b(z) * inv_lambda * inv_lambda;
    out[1] = (double)(electrons * 2.0L * kPi * kRe * kRe * z * coherent_shape(B));
    out[2] = (double)(electrons * klein_nishina_total(e));
}

int table_length(float e_max_kev) { return (int)std::floor(e_max_kev) + 2; }

void build_tables(const Material *mats, int n_mat, int J, const float *eta_user, int n_eta,
                  std::vector<float> &pe, std::vector<float> &coh, std::vector<float> &inc,
                  std::vector<float> &eta) {
    pe.assign((size_t)n_mat * J, 0.0f);
    coh.assign((size_t)n_mat * J, 0.0f);
    inc.assign((size_t)n_mat * J, 0.0f);
    eta.assign((size_t)J, 0.0f);
    for (int m = 0; m < n_mat; ++m) {
        const long double z = mats[m].z_eff;
        const long double electrons = kAvogadro * (long double)mats[m].z_over_a;
        const long double b = screening_b(z);
        for (int j = 0; j < J; ++j) {
            const long double e = (long double)(1 + j);
            const size_t o = (size_t)m * J + j;
            pe[o] = (float)(electrons * kPhoto * z * z * z / (e * e * e));
            const long double inv_lambda = e / kHc;
            coh[o] = (float)(electrons * 2.0L * kPi * kRe * kRe * z *
                             coherent_shape(b * inv_lambda * inv_lambda));
            inc[o] = (float)(electrons * klein_nishina_total(e));
        }
    }
    for (int j = 0; j < J; ++j)
        eta[j] = eta_user ? eta_user[j < n_eta ? j : n_eta - 1] : (float)(1 + j);
}

double rayleigh_b(float z_eff) {
    const double r = 0.885 * 0.529177210903 / std::cbrt((double)z_eff);
    const double t = 6.283185307179586 * r;
    return t * t;
}

double compton_pz_scale(float z_eff) {
    // hbar / r_Z for the screening radius r_Z = 0.885 a0 Z^(-1/3): (a0 / r_Z)
    // atomic units of momentum, one of which is m c / 137.035999084
    return (std::cbrt((double)z_eff) / 0.885) / 137.035999084;
}

void savgol_weights(int window, int order, float *w) {
    // least-squares polynomial of degree `order` on offsets -h..h, value at 0:
    // row 0 of (A^T A)^-1 A^T with A[j][k] = j^k, solved by Gauss-Jordan in
    // long double on the (order+1)^2 normal matrix
    const int h = window / 2, m = order + 1;
    long double N[16][16] = {}, inv[16][16] = {};
    for (int r = 0; r < m; ++r)
        for (int cc = 0; cc < m; ++cc) {
            long double s = 0.0L;
            for (int j = -h; j <= h; ++j) s += std::pow((long double)j, r + cc);
            N[r][cc] = s;
        }
    for (int r = 0; r < m; ++r) inv[r][r] = 1.0L;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (std::fabs(N[r][col]) > std::fabs(N[piv][col])) piv = r;
        for (int cc = 0; cc < m; ++cc) {
            std::swap(N[col][cc], N[piv][cc]);
            std::swap(inv[col][cc], inv[piv][cc]);
        }
        const long double d = N[col][col];
        for (int cc = 0; cc < m; ++cc) {
            N[col][cc] /= d;
            inv[col][cc] /= d;
        }
        for (int r = 0; r < m; ++r) {
            if (r == col) continue;
            const long double f = N[r][col];
            for (int cc = 0; cc < m; ++cc) {
                N[r][cc] -= f * N[col][cc];
                inv[r][cc] -= f * inv[col][cc];
            }
        }
    }
    for (int j = -h; j <= h; ++j) {
        long double s = 0.0L;
        for (int k = 0; k < m; ++k) s += inv[0][k] * std::pow((long double)j, k);
        w[j + h] = (float)s;
    }
}

void spectrum_thresholds(const float *w, int n, std::vector<uint64_t> &thr) {
    thr.resize(n);
    double total = 0.0;
    for (int k = 0; k < n; ++k) total += (double)w[k];
    double run = 0.0;
    for (int k = 0; k < n; ++k) {
        run += (double)w[k];
        thr[k] = (k + 1 == n) ? (uint64_t(1) << 32)
                              : (uint64_t)std::floor(run / total * 4294967296.0);
    }
}

}  // namespace mcx
