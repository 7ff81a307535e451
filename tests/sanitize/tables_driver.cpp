// Drives the library's host-side table generation (tables.cpp) over its whole
// input range for an AddressSanitizer / UndefinedBehaviorSanitizer build.
// Prints "ok" and exits 0 when the outputs are finite and of the right sizes.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2201_13191_amd/csrc/tables.hpp"

using namespace mcx;

int main() {
    const Material mats[5] = {{7.64f, 0.49919f}, {7.42f, 0.55508f}, {13.0f, 0.48181f},
                              {13.8f, 0.5148f},  {26.0f, 0.46557f}};
    for (float emax : {1.0f, 1.5f, 150.0f, 999.9f, 1000.0f}) {
        const int J = table_length(emax);
        std::vector<float> pe, coh, inc, eta;
        build_tables(mats, 5, J, nullptr, 0, pe, coh, inc, eta);
        std::vector<float> user(37, 2.0f);
        build_tables(mats, 5, J, user.data(), (int)user.size(), pe, coh, inc, eta);
        if ((int)pe.size() != 5 * J || (int)eta.size() != J) return 1;
        for (size_t i = 0; i < pe.size(); ++i)
            if (!std::isfinite(pe[i]) || !std::isfinite(coh[i]) || !std::isfinite(inc[i])) return 2;
    }
    double out[3];
    for (double e = 1.0; e <= 1000.0; e *= 1.7) attenuation_coefficients(7.42, 0.555, e, out);
    for (float z = 1.0f; z <= 100.0f; z += 7.5f)
        if (!(rayleigh_b(z) > 0.0) || !(compton_pz_scale(z) > 0.0)) return 3;
    std::vector<float> w = {0.0f, 1.0f, 3.0f, 0.0f, 2.0f};
    std::vector<uint64_t> thr;
    spectrum_thresholds(w.data(), (int)w.size(), thr);
    if (thr.size() != w.size() || thr.back() != (uint64_t)1 << 32) return 4;
    double kn[30], cs[41];
    kn_norm_series(kn, 30);
    coherent_series(cs, 41);
    float sg[31];
    for (int win = 1; win <= 31; win += 2)
        for (int order = 0; order < win && order <= 5; ++order) savgol_weights(win, order, sg);
    std::printf("ok\n");
    return 0;
}
