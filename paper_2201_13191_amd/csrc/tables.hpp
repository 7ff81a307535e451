// Host-side table generation for the transport kernel (see tables.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace mcx {

struct Material {
    float z_eff;
    float z_over_a;
};

// Unrounded {mu_pe, mu_coh, mu_incoh} / rho in cm^2/g at one energy.
void attenuation_coefficients(double z_eff, double z_over_a, double e_kev, double out[3]);

// Grid length for spectra up to e_max: E_j = 1 + j keV, j < J, J = floor(e_max) + 2,
// so both neighbours of every reachable energy are on the grid.
int table_length(float e_max_kev);

// fp32 tables [n_mat][J] and eta[J] (user eta on the same grid, last value
// repeated; NULL -> eta(E) = E).
void build_tables(const Material *mats, int n_mat, int J, const float *eta_user, int n_eta,
                  std::vector<float> &pe, std::vector<float> &coh, std::vector<float> &inc,
                  std::vector<float> &eta);

// Screening constant b = (2 pi 0.885 a0 Z^(-1/3))^2 [A^2] of the Rayleigh sampler (fp64).
double rayleigh_b(float z_eff);

// Momentum scale p0 / (m c) of the 1s-like Compton profile of a material: the
// orbital of the Rayleigh screening radius (fp64).
double compton_pz_scale(float z_eff);

// Spectrum bin thresholds on 32-bit draws: thr[k] = floor(W_k / W * 2^32) of the
// cumulative weight, thr[n-1] = 2^32; the bin of draw x is the first k with x < thr[k].
void spectrum_thresholds(const float *w, int n, std::vector<uint64_t> &thr);

// Taylor coefficients c[0 .. n) of K(a) = sigma_KN / (pi r_e^2), a = E / mc^2: the
// integral over the scattering cosine of the bracket of eq. (1) (S = 1).  Used
// where the closed form cancels (small a).
void kn_norm_series(double *c, int n);

// Coefficients d[0 .. n) of the power series in B of the coherent shape
// (1/V) int_0^V (1 + cos^2) (1 + b v)^-4 dv, B = b V, used below B = 0.1.
void coherent_series(double *d, int n);

// Savitzky-Golay weights (window odd <= 31, order < window): value at the
// window centre of the least-squares polynomial, as fp32.
void savgol_weights(int window, int order, float *w);

}  // namespace mcx
