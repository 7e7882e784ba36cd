// Host sanitizer driver for the ensemble statistics of libtgf (test
// infrastructure): the lattice normalisation, the coupling with its
// jackknife, the slice-charge correlator and the susceptibility, with valid
// and invalid arguments.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tgf.h"

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);    \
            fails++;                                                              \
        }                                                                         \
    } while (0)

int main() {
    double v = 0, e = 0;
    for (int Lt : {6, 12, 18, 48})
        for (double c : {0.3, 0.4}) {
            CHECK(tgf_latt_norm(c, Lt, 3, &v) == TGF_OK && std::isfinite(v) && v > 0);
        }
    CHECK(tgf_latt_norm(0.3, 0, 3, &v) != TGF_OK);
    CHECK(tgf_latt_norm(0.3, 1000, 3, &v) != TGF_OK);
    CHECK(tgf_latt_norm(0.3, 12, 3, nullptr) != TGF_OK);
    const int n = 37, T = 18;
    std::vector<double> t2E(n), Q(n), q(n * T), C(T), Ce(T);
    for (int k = 0; k < n; k++) {
        t2E[k] = 0.1 + 0.001 * k;
        Q[k] = (k % 5 == 0) ? 1.02 : 0.01 * (k % 3);
        for (int x = 0; x < T; x++) q[k * T + x] = 0.01 * std::sin(0.3 * (k + x));
    }
    CHECK(tgf_coupling(t2E.data(), Q.data(), n, 0.3, 12, 3, &v, &e) == TGF_OK && std::isfinite(v));
    CHECK(tgf_coupling(t2E.data(), Q.data(), n, 0.3, 12, 3, &v, nullptr) == TGF_OK);
    std::vector<double> Qbig(n, 2.0);
    CHECK(tgf_coupling(t2E.data(), Qbig.data(), n, 0.3, 12, 3, &v, &e) == TGF_E_STATE);
    CHECK(tgf_coupling(t2E.data(), Q.data(), 0, 0.3, 12, 3, &v, &e) != TGF_OK);
    CHECK(tgf_charge_correlator(q.data(), Q.data(), n, T, T, C.data(), Ce.data()) == TGF_OK);
    CHECK(tgf_charge_correlator(q.data(), Q.data(), n, T, T, C.data(), nullptr) == TGF_OK);
    CHECK(tgf_charge_correlator(q.data(), Q.data(), n, T, T - 1, C.data(), Ce.data()) != TGF_OK);
    CHECK(tgf_susceptibility(Q.data(), n, 1e4, &v, &e) == TGF_OK && std::isfinite(v));
    CHECK(tgf_susceptibility(Q.data(), 1, 1e4, &v, &e) == TGF_OK);
    CHECK(tgf_susceptibility(Q.data(), n, 0.0, &v, &e) != TGF_OK);
    CHECK(tgf_stats_last_error() != nullptr);
    std::printf("stats driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
