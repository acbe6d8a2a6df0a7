// Host-only driver for the operator-table builders, built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Exercises
// every builder for every supported order and checks finiteness, the exact
// symmetry T(-o) = T(o)^T of the translation bank and the sparsity of the
// gradient table.  Exit status 0 = all checks passed.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "operators.h"

int main(int argc, char** argv) {
    const int pmax = argc > 1 ? std::atoi(argv[1]) : fmmops::kMaxOrder - 1;
    int bad = 0;
    for (int p = 1; p <= pmax; ++p) {
        const int K = fmmops::ncoef(p);
        std::vector<double> bank(343ull * K * K), m2m(8ull * K * K), l2l(8ull * K * K);
        fmmops::build_m2l_bank(p, bank.data());
        fmmops::build_m2m(p, m2m.data());
        fmmops::build_l2l(p, l2l.data());
        for (double v : bank) bad += !std::isfinite(v);
        for (double v : m2m) bad += !std::isfinite(v);
        for (double v : l2l) bad += !std::isfinite(v);
        // T(-o) = T(o)^T for every offset
        double amax = 0, dmax = 0;
        for (int o = 0; o < 343; ++o) {
            const int on = 342 - o;  // index of -o
            for (int r = 0; r < K; ++r)
                for (int k = 0; k < K; ++k) {
                    const double a = bank[(size_t)o * K * K + (size_t)r * K + k];
                    const double b = bank[(size_t)on * K * K + (size_t)k * K + r];
                    amax = std::fmax(amax, std::fabs(a));
                    dmax = std::fmax(dmax, std::fabs(a - b));
                }
        }
        if (dmax > 1e-13 * amax) {
            std::printf("p=%d: bank asymmetry %g\n", p, dmax / amax);
            ++bad;
        }
        std::vector<int32_t> gi(3ull * p * p * 4);
        std::vector<double> gc(3ull * p * p * 4);
        fmmops::build_grad_table(p, gi.data(), gc.data());
        for (size_t i = 0; i < gi.size(); ++i)
            if (gi[i] < -1 || gi[i] >= K || !std::isfinite(gc[i])) ++bad;
        std::vector<double> rho(K);
        const double r[3] = {0.31, -0.22, 0.4};
        fmmops::eval_rho(p, r, rho.data());
        for (double v : rho) bad += !std::isfinite(v);
        if (p <= 6 || p == pmax) {
            std::vector<double> lat((size_t)K * K);
            fmmops::build_lattice(p, lat.data());
            for (double v : lat) bad += !std::isfinite(v);
        }
    }
    std::printf("host operator checks: %d failures\n", bad);
    return bad ? 1 : 0;
}
