/* Host sanitizer driver for the FP64 oracle (test infrastructure): runs every
 * oracle entry point -- measurement, force, densities, RK3 steps, whole flows
 * with a short last step, hybrid over-relaxation, SU(N) flows, the Philox and
 * SU(2) samplers -- on small lattices with ragged extents and several twist
 * tensors, and checks return codes and finiteness.  Built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_sanitizers.py. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

void oracle_set_threads(int n);
int oracle_measure(const cplx *links, const int dims[4], const int twist[6], const int base[4],
                   double *out);
int oracle_force(const cplx *links, const int dims[4], const int twist[6], const int base[4],
                 cplx *F);
void oracle_expm(const cplx *A, cplx *out);
int oracle_densities(const cplx *links, const int dims[4], const int twist[6], const int base[4],
                     double *e, double *q);
int oracle_rk3_step(cplx *links, const int dims[4], const int twist[6], const int base[4],
                    double eps);
int oracle_flow(cplx *links, const int dims[4], const int twist[6], const int base[4],
                double eps, double t0, double t_end, double meas_dt, double *rows, int max_rows);
int oracle_mc(cplx *links, const int dims[4], const int twist[6], const int base[4], double beta,
              int n_hybrid, int n_or, unsigned long long seed, unsigned int sweep0,
              unsigned int cfg);
int oracle_or_sweeps(cplx *links, const int dims[4], const int twist[6], const int base[4], int n);
void oracle_su2_samples(double alpha, unsigned long long seed, int n, double *out);
void oracle_philox(const unsigned int ctr[4], unsigned int k0, unsigned int k1,
                   unsigned int out[4]);
int oracle_sun_measure(const cplx *U, int nc, const int dims[4], const int twist[6],
                       const int base[4], double *out);
int oracle_sun_expm(int nc, const cplx *A, cplx *out);
int oracle_sun_flow(cplx *U, int nc, const int dims[4], const int twist[6], const int base[4],
                    double eps, double t0, double t_end, double meas_dt, double *rows,
                    int max_rows);

static unsigned long long rng = 88172645463325252ull;
static double urand(void) {   /* xorshift64, uniform in (-1, 1) */
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 4503599627370496.0 - 1.0;
}

static int fails = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);      \
            fails++;                                                           \
        }                                                                      \
    } while (0)

/* exp(A) for A = i a H, H Hermitian traceless random N x N */
static void random_group_element(int nc, double a, cplx *out) {
    cplx A[64];
    for (int i = 0; i < nc; i++)
        for (int j = i; j < nc; j++) {
            double re = urand(), im = (i == j) ? 0.0 : urand();
            A[i * nc + j] = re + I * im;
            A[j * nc + i] = re - I * im;
        }
    cplx tr = 0;
    for (int i = 0; i < nc; i++) tr += A[i * nc + i];
    for (int i = 0; i < nc; i++) A[i * nc + i] -= tr / nc;
    for (int k = 0; k < nc * nc; k++) A[k] *= I * a;
    if (nc == 3)
        oracle_expm(A, out);
    else
        CHECK(oracle_sun_expm(nc, A, out) == 0);
}

static cplx *field(int nc, const int d[4], double a) {
    long V = (long)d[0] * d[1] * d[2] * d[3];
    cplx *U = malloc(sizeof(cplx) * V * 4 * nc * nc);
    for (long k = 0; k < V * 4; k++) random_group_element(nc, a, U + k * nc * nc);
    return U;
}

static int finite_all(const double *x, long n) {
    for (long k = 0; k < n; k++)
        if (!isfinite(x[k])) return 0;
    return 1;
}

int main(void) {
    oracle_set_threads(2);
    const int dims[][4] = {{2, 2, 4, 4}, {3, 3, 5, 7}, {4, 2, 6, 2}};
    const int twists[][6] = {{1, 0, 0, 0, 0, 0}, {1, 2, 1, 2, 1, 2}, {0, 0, 0, 0, 0, 0}};
    const int base[4] = {0, 0, 0, 0};
    double rows[64 * 6], out[4];
    for (int g = 0; g < 3; g++)
        for (int w = 0; w < 3; w++) {
            const int *d = dims[g];
            long V = (long)d[0] * d[1] * d[2] * d[3];
            cplx *U = field(3, d, 0.4);
            CHECK(oracle_measure(U, d, twists[w], base, out) == 0 && finite_all(out, 4));
            cplx *F = malloc(sizeof(cplx) * V * 4 * 9);
            CHECK(oracle_force(U, d, twists[w], base, F) == 0);
            CHECK(finite_all((const double *)F, V * 4 * 9 * 2));
            free(F);
            double *e = malloc(sizeof(double) * V), *q = malloc(sizeof(double) * V);
            CHECK(oracle_densities(U, d, twists[w], base, e, q) == 0);
            CHECK(finite_all(e, V) && finite_all(q, V));
            free(e);
            free(q);
            CHECK(oracle_rk3_step(U, d, twists[w], base, 0.02) == 0);
            int nr = oracle_flow(U, d, twists[w], base, 0.02, 0.02, 0.075, 0.02, rows, 64);
            CHECK(nr >= 3 && finite_all(rows, nr * 6));
            free(U);
        }
    /* Monte Carlo: heat bath and over-relaxation on even extents */
    {
        const int d[4] = {2, 2, 4, 4};
        cplx *U = field(3, d, 0.5);
        CHECK(oracle_mc(U, d, twists[0], base, 3.0, 2, 2, 12345ull, 0u, 1u) == 0);
        CHECK(oracle_or_sweeps(U, d, twists[1], base, 2) == 0);
        CHECK(oracle_mc(U, d, twists[0], base, 3.0, 1, 1, 1ull, 0u, 0u) == 0);
        const int odd[4] = {3, 2, 4, 4};
        CHECK(oracle_mc(U, odd, twists[0], base, 3.0, 1, 1, 1ull, 0u, 0u) == -1);
        CHECK(oracle_measure(U, d, twists[0], base, out) == 0 && finite_all(out, 4));
        free(U);
    }
    /* SU(N) flows */
    for (int nc = 2; nc <= 5; nc += 3) {
        const int d[4] = {2, 3, 4, 2};
        const int tw[6] = {1, 0, 0, 0, 0, nc - 1};
        cplx *U = field(nc, d, 0.3);
        CHECK(oracle_sun_measure(U, nc, d, tw, base, out) == 0 && finite_all(out, 4));
        int nr = oracle_sun_flow(U, nc, d, tw, base, 0.02, 0.0, 0.05, 0.02, rows, 64);
        CHECK(nr >= 3 && finite_all(rows, nr * 6));
        free(U);
    }
    /* samplers */
    {
        unsigned int ctr[4] = {1, 2, 3, 4}, r[4];
        oracle_philox(ctr, 7u, 9u, r);
        double y[4 * 64];
        oracle_su2_samples(0.7, 5ull, 64, y);
        oracle_su2_samples(30.0, 5ull, 64, y);
        CHECK(finite_all(y, 4 * 64));
    }
    /* invalid geometry */
    {
        const int bad[4] = {0, 2, 2, 2};
        CHECK(oracle_measure(NULL, bad, twists[0], base, out) != 0);
    }
    printf("oracle driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
