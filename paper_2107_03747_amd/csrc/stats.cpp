// stats.cpp -- ensemble statistics of the twisted gradient-flow coupling
// (host FP64; inputs are the per-configuration observables that tgf_flow and
// tgf_slice_charge return).
//
//   lattice normalisation  N^{-1}(c, Lt) = c^4/128 sum_{mu != nu} sum'_q
//        exp(-c^2 Lt^2 qhat^2 / 4) sin^2(q_nu) cos^2(q_mu / 2) / qhat^2,
//        q_mu = 2 pi n_mu / Lt, n_mu = 0..Lt-1, qhat_mu = 2 sin(q_mu / 2); the
//        prime drops the momenta whose two twisted-plane components both have
//        Lt q_i a multiple of 2 pi N, i.e. n_i = 0 mod N (sec. 3.1, eq. latt_norm)
//   coupling  lambda_TGF = N(c, Lt) <t^2 E delta_Q> / (3 <delta_Q>),
//        delta_Q = 1 iff |Q| < 0.5 (sec. 3.1, eq. lambdat_latt)
//   correlator  C(x0) = <q(x0) q(0) delta_Q> / <delta_Q> with the slice charge
//        q(x0) of sec. 4 (eq. qcorr), averaged over the origin
//   susceptibility  chi = <Q^2> / V over all configurations (sec. 4.2)
// Errors are delete-one jackknife over configurations.
#include <cmath>
#include <string>
#include <vector>

#include "../../include/tgf.h"

namespace {
thread_local std::string s_err;
tgf_status bad(tgf_status s, const char *m) {
    s_err = m;
    return s;
}
}  // namespace

extern "C" {

tgf_status tgf_latt_norm(double c, int32_t Lt, int32_t N, double *out) {
    if (!out || !(c > 0) || Lt < 1 || N < 1) return bad(TGF_E_INVAL, "bad argument");
    if (Lt > 512) return bad(TGF_E_UNSUPPORTED, "Lt > 512");
    const double pi = 3.14159265358979323846;
    const double a = 0.25 * c * c * (double)Lt * (double)Lt;
    std::vector<double> s2(Lt), c2(Lt), h(Lt), e(Lt);
    for (int n = 0; n < Lt; n++) {
        const double q = 2.0 * pi * n / Lt;
        s2[n] = std::sin(q) * std::sin(q);
        c2[n] = std::cos(0.5 * q) * std::cos(0.5 * q);
        h[n] = 4.0 * std::sin(0.5 * q) * std::sin(0.5 * q);
        e[n] = std::exp(-a * h[n]);
    }
    double sum = 0;
    for (int n3 = 0; n3 < Lt; n3++)
        for (int n2 = 0; n2 < Lt; n2++) {
            double part = 0;
            for (int n1 = 0; n1 < Lt; n1++)
                for (int n0 = 0; n0 < Lt; n0++) {
                    // Lt q_i = 2 pi n_i a multiple of 2 pi N in both twisted directions
                    if (n0 % N == 0 && n1 % N == 0) continue;
                    const double qh = h[n0] + h[n1] + h[n2] + h[n3];
                    const double C = c2[n0] + c2[n1] + c2[n2] + c2[n3];
                    // sum_{mu != nu} s2_nu c2_mu = sum_nu s2_nu (C - c2_nu)
                    const double w = s2[n0] * (C - c2[n0]) + s2[n1] * (C - c2[n1]) +
                                     s2[n2] * (C - c2[n2]) + s2[n3] * (C - c2[n3]);
                    part += e[n0] * e[n1] * e[n2] * e[n3] * w / qh;
                }
            sum += part;
        }
    const double inv = std::pow(c, 4) / 128.0 * sum;
    if (!(inv > 0)) return bad(TGF_E_NONFINITE, "normalisation sum vanished");
    *out = 1.0 / inv;
    return TGF_OK;
}

tgf_status tgf_coupling(const double *t2E, const double *Q, int32_t n, double c, int32_t Lt,
                        int32_t N, double *lambda, double *err) {
    if (!t2E || !Q || !lambda || n < 1) return bad(TGF_E_INVAL, "bad argument");
    double norm;
    tgf_status s = tgf_latt_norm(c, Lt, N, &norm);
    if (s) return s;
    double se = 0, sd = 0;
    for (int k = 0; k < n; k++) {
        const double d = std::fabs(Q[k]) < 0.5 ? 1.0 : 0.0;
        se += t2E[k] * d;
        sd += d;
    }
    if (sd == 0) return bad(TGF_E_STATE, "no configuration with |Q| < 0.5");
    *lambda = norm * se / (3.0 * sd);
    if (err) {
        double m = 0, v = 0;
        int used = 0;
        std::vector<double> jk(n);
        for (int k = 0; k < n; k++) {
            const double d = std::fabs(Q[k]) < 0.5 ? 1.0 : 0.0;
            const double sdk = sd - d;
            if (sdk == 0) { jk[k] = NAN; continue; }
            jk[k] = norm * (se - t2E[k] * d) / (3.0 * sdk);
            m += jk[k];
            used++;
        }
        if (used < 2) {
            *err = NAN;
        } else {
            m /= used;
            for (int k = 0; k < n; k++)
                if (!std::isnan(jk[k])) v += (jk[k] - m) * (jk[k] - m);
            *err = std::sqrt((double)(used - 1) / used * v);
        }
    }
    return TGF_OK;
}

tgf_status tgf_charge_correlator(const double *q, const double *Q, int32_t n, int32_t T,
                                 int32_t ld, double *C, double *err) {
    if (!q || !Q || !C || n < 1 || T < 1 || ld < T) return bad(TGF_E_INVAL, "bad argument");
    std::vector<double> ck((size_t)n * T, 0.0), d(n);
    double sd = 0;
    for (int k = 0; k < n; k++) {
        d[k] = std::fabs(Q[k]) < 0.5 ? 1.0 : 0.0;
        sd += d[k];
        const double *qk = q + (size_t)k * ld;
        for (int x = 0; x < T; x++) {
            double s = 0;
            for (int y = 0; y < T; y++) s += qk[(y + x) % T] * qk[y];
            ck[(size_t)k * T + x] = s / T;
        }
    }
    if (sd == 0) return bad(TGF_E_STATE, "no configuration with |Q| < 0.5");
    for (int x = 0; x < T; x++) {
        double s = 0;
        for (int k = 0; k < n; k++) s += d[k] * ck[(size_t)k * T + x];
        C[x] = s / sd;
        if (err) {
            std::vector<double> jk;
            for (int k = 0; k < n; k++) {
                if (sd - d[k] == 0) continue;
                jk.push_back((s - d[k] * ck[(size_t)k * T + x]) / (sd - d[k]));
            }
            if (jk.size() < 2) {
                err[x] = NAN;
            } else {
                double m = 0, v = 0;
                for (double j : jk) m += j;
                m /= jk.size();
                for (double j : jk) v += (j - m) * (j - m);
                err[x] = std::sqrt((double)(jk.size() - 1) / jk.size() * v);
            }
        }
    }
    return TGF_OK;
}

tgf_status tgf_susceptibility(const double *Q, int32_t n, double V, double *chi, double *err) {
    if (!Q || !chi || n < 1 || !(V > 0)) return bad(TGF_E_INVAL, "bad argument");
    double s = 0;
    for (int k = 0; k < n; k++) s += Q[k] * Q[k];
    *chi = s / n / V;
    if (err) {
        if (n < 2) {
            *err = NAN;
        } else {
            // delete-one estimates (s - Q_k^2) / ((n - 1) V); their mean is chi
            double v = 0;
            for (int k = 0; k < n; k++) {
                const double j = (s - Q[k] * Q[k]) / (n - 1) / V - *chi;
                v += j * j;
            }
            *err = std::sqrt((double)(n - 1) / n * v);
        }
    }
    return TGF_OK;
}

const char *tgf_stats_last_error(void) { return s_err.c_str(); }

}  // extern "C"
