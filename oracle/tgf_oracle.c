/*
 * tgf_oracle.c -- plain, slow, FP64 CPU oracle for the twisted Wilson flow.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * helper with the GPU library; the two meet only in the canonical link layout.
 *
 * Paper: E. I. Bribian, J. Dasilva Golan, M. Garcia Perez, A. Ramos,
 * "Memory efficient finite volume schemes with twisted boundary conditions"
 * (arXiv 2107.03747).  What is computed, and where it is defined:
 *
 *   geometry        L^2 x (3L)^2 torus, links U_mu(n) in SU(3)      sec. 3.1
 *   twist factors   Z_{mu nu}(n) != 1 only on the plaquettes at the
 *                   twist site of the twisted plane, Z_12 = Z_21^* =
 *                   exp(2 pi i/3)                                   sec. 3.1
 *   Wilson action   S_W = 3b sum_n sum_{mu!=nu} Tr[1 - Z^* P]       sec. 3.1
 *   flow            the Wilson-flow discretisation of the gradient
 *                   flow equation (sec. 1, sec. 3.1), integrated with
 *                   Luscher's third-order Runge-Kutta scheme
 *   clover E        E_cl = 1/2 Tr[G^cl G^cl], G^cl from four twisted
 *                   leaves (eq. gmunu)                              sec. 3.1
 *   charge Q        (1/16 pi^2) sum_n Tr{G^cl G~^cl}  (eq. qlatt)   sec. 3.1
 *   Monte Carlo     hybrid over-relaxation: one heat-bath sweep, then
 *                   over-relaxation sweeps (Cabibbo-Marinari SU(2)
 *                   subgroups, checkerboard, Philox4x32-10)         sec. 3.1
 *
 * Readings where the paper is silent (both paths adopt them):
 *   - The twist site "x1 = x2 = 1" is 1-based; 0-based it is n_mu = n_nu = 0.
 *     For the relocation test the twist site is a parameter (base[]).
 *   - "- c.c." in G^cl is minus the Hermitian adjoint of the whole sum, no
 *     trace subtraction (parity unpinned: a convention both paths adopt,
 *     which nothing outside them fixes).
 *   - E sums Tr G_{mu nu} G_{mu nu} over all ordered pairs with weight 1/2.
 *   - G~_{mu nu} = 1/2 eps_{mu nu rho sigma} G_{rho sigma}, eps_{0123} = +1.
 *   - The force is F = -P_ah(Omega) (the Lie derivative of g0^2 S_W), which
 *     fixes the meaning of flow time t.
 *   - plaquette = (1/18V) sum_n sum_{mu<nu} Re Tr[Z^* P]; action
 *     s = sum_n sum_{mu<nu} Re Tr[1 - Z^* P]  (= g0^2 S_W / 2).
 *   - Schedule: steps of eps while t + eps <= t_end (+1e-12), then one short
 *     step to t_end; rows at grid multiples of meas_dt and at t_end.
 *   - Monte Carlo (the paper names the algorithm, not its details): beta =
 *     18 b; sweep order mu = 0..3, even then odd sites; subgroups (0,1),
 *     (0,2), (1,2) in turn; the random-number counter layout stated at
 *     mc_sweep.
 *
 * The exponential is scaling-and-squaring with a degree-16 Taylor sum: a
 * different method from the GPU library's.
 *
 * Layout: complex128 [d3][d2][d1][d0][4][3][3], n0 fastest, row-major 3x3.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
typedef struct { cplx a[3][3]; } mat;

typedef struct {
    int d[4];
    long V;
    int tw[4][4];   /* twist tensor n_{mu nu} mod 3, antisymmetric */
    int base[4];    /* coordinates of the twist site */
} lat;

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices                                                */

static mat m_zero(void) { mat r; memset(&r, 0, sizeof r); return r; }

static mat m_eye(void) {
    mat r = m_zero();
    for (int i = 0; i < 3; i++) r.a[i][i] = 1.0;
    return r;
}

static mat m_mul(mat x, mat y) {
    mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += x.a[i][k] * y.a[k][j];
            r.a[i][j] = s;
        }
    return r;
}

static mat m_dag(mat x) {
    mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.a[i][j] = conj(x.a[j][i]);
    return r;
}

static mat m_add(mat x, mat y) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) x.a[i][j] += y.a[i][j];
    return x;
}

static mat m_scale(cplx c, mat x) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) x.a[i][j] *= c;
    return x;
}

static cplx m_tr(mat x) { return x.a[0][0] + x.a[1][1] + x.a[2][2]; }

static double m_fnorm(mat x) {
    double s = 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) s += creal(x.a[i][j] * conj(x.a[i][j]));
    return sqrt(s);
}

/* Traceless anti-Hermitian part: P_ah(M) = (M - M^+)/2 - Tr(M - M^+)/6. */
static mat m_proj_ah(mat m) {
    mat d = m_dag(m);
    mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.a[i][j] = 0.5 * (m.a[i][j] - d.a[i][j]);
    cplx t = m_tr(r) / 3.0;
    for (int i = 0; i < 3; i++) r.a[i][i] -= t;
    return r;
}

/* exp(A): scale A by 2^-s so that ||A/2^s||_F <= 1/4, sum the Taylor
 * series to degree 16, square s times. */
static mat m_exp(mat A) {
    double nrm = m_fnorm(A);
    int s = 0;
    if (nrm > 0.25) s = (int)ceil(log2(nrm / 0.25));
    mat B = m_scale(ldexp(1.0, -s), A);
    mat sum = m_eye(), term = m_eye();
    for (int k = 1; k <= 16; k++) {
        term = m_scale(1.0 / k, m_mul(term, B));
        sum = m_add(sum, term);
    }
    for (int i = 0; i < s; i++) sum = m_mul(sum, sum);
    return sum;
}

/* ------------------------------------------------------------------ */
/* lattice geometry and twist                                          */

static int lat_init(lat *L, const int dims[4], const int twist6[6], const int base[4]) {
    L->V = 1;
    for (int m = 0; m < 4; m++) {
        if (dims[m] < 1) return -1;
        L->d[m] = dims[m];
        L->V *= dims[m];
        L->base[m] = base ? ((base[m] % dims[m]) + dims[m]) % dims[m] : 0;
    }
    memset(L->tw, 0, sizeof L->tw);
    int k = 0;
    for (int m = 0; m < 4; m++)
        for (int n = m + 1; n < 4; n++, k++) {
            int t = twist6 ? ((twist6[k] % 3) + 3) % 3 : 0;
            L->tw[m][n] = t;
            L->tw[n][m] = (3 - t) % 3;
        }
    return 0;
}

static void coords(const lat *L, long i, int n[4]) {
    for (int m = 0; m < 4; m++) { n[m] = (int)(i % L->d[m]); i /= L->d[m]; }
}

static long index_of(const lat *L, const int n[4]) {
    long i = 0;
    for (int m = 3; m >= 0; m--) i = i * L->d[m] + n[m];
    return i;
}

/* site n + s*mu_hat, periodic */
static long step(const lat *L, long i, int mu, int s) {
    int n[4];
    coords(L, i, n);
    n[mu] = ((n[mu] + s) % L->d[mu] + L->d[mu]) % L->d[mu];
    return index_of(L, n);
}

/* Z_{mu nu}(n): exp(2 pi i n_{mu nu}/3) on the twist site of the plane, else 1 */
static cplx zfac(const lat *L, long i, int mu, int nu) {
    if (mu == nu || L->tw[mu][nu] == 0) return 1.0;
    int n[4];
    coords(L, i, n);
    if (n[mu] != L->base[mu] || n[nu] != L->base[nu]) return 1.0;
    return cexp(I * (2.0 * PI * L->tw[mu][nu] / 3.0));
}

static mat U(const cplx *links, long i, int mu) {
    mat r;
    memcpy(&r, links + (i * 4 + mu) * 9, sizeof r);
    return r;
}

/* Link in a signed direction: U_{+mu}(n) = U_mu(n), U_{-mu}(n) = U_mu(n - mu)^+.
 * Directions are encoded as dir = mu (positive) or dir = -(mu+1) (negative). */
static mat Us(const lat *L, const cplx *links, long i, int dir) {
    if (dir >= 0) return U(links, i, dir);
    int mu = -dir - 1;
    return m_dag(U(links, step(L, i, mu, -1), mu));
}

static long shift_s(const lat *L, long i, int dir) {
    return dir >= 0 ? step(L, i, dir, +1) : step(L, i, -dir - 1, -1);
}

/* P_{ab}(n) = U_a(n) U_b(n+a) U_a(n+b)^+ U_b(n)^+ for signed directions a, b */
static mat plaq_s(const lat *L, const cplx *links, long i, int a, int b) {
    mat x = Us(L, links, i, a);
    x = m_mul(x, Us(L, links, shift_s(L, i, a), b));
    x = m_mul(x, m_dag(Us(L, links, shift_s(L, i, b), a)));
    x = m_mul(x, m_dag(Us(L, links, i, b)));
    return x;
}

/* ------------------------------------------------------------------ */
/* force: F_mu(n) = -P_ah(Omega_mu(n))                                 */
/*
 * Omega_mu(n) collects every plaquette of S_W that starts with U_mu(n):
 *   upper:  Z^*_{mu nu}(n)      U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
 *   lower:  Z_{mu nu}(n-nu)     U_mu(n) U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu)
 * (the lower plaquette is P_{mu nu}(n-nu)^+ rotated to start at U_mu(n), so
 * it carries the conjugate of that plaquette's factor Z^*_{mu nu}(n-nu)).
 * With tr(T^a T^b) = -delta_ab/2 and 3b = 1/g0^2 the Lie derivative is
 * g0^2 d_{n,mu} S_W = P_ah(Omega_mu(n)), and the flow is dV/dt = -P_ah(Omega) V.
 */
static mat omega(const lat *L, const cplx *links, long i, int mu) {
    mat om = m_zero();
    mat Umu = U(links, i, mu);
    long ipm = step(L, i, mu, +1);
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        long ipn = step(L, i, nu, +1);
        long imn = step(L, i, nu, -1);
        long ipm_mn = step(L, ipm, nu, -1);
        mat up = m_mul(m_mul(m_mul(Umu, U(links, ipm, nu)), m_dag(U(links, ipn, mu))),
                       m_dag(U(links, i, nu)));
        mat lo = m_mul(m_mul(m_mul(Umu, m_dag(U(links, ipm_mn, nu))), m_dag(U(links, imn, mu))),
                       U(links, imn, nu));
        om = m_add(om, m_scale(conj(zfac(L, i, mu, nu)), up));
        om = m_add(om, m_scale(zfac(L, imn, mu, nu), lo));
    }
    return om;
}

static void force_field(const lat *L, const cplx *links, mat *F) {
    long V = L->V;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++)
        for (int mu = 0; mu < 4; mu++)
            F[i * 4 + mu] = m_scale(-1.0, m_proj_ah(omega(L, links, i, mu)));
}

/* ------------------------------------------------------------------ */
/* observables                                                         */

/* G^cl_{mu nu}(n) per eq. gmunu: -(i/8) { C - C^+ } with C the four
 * twisted leaves Z^*(n)P_{mu nu}(n) + Z^*(n-nu)P_{-nu,mu}(n)
 * + Z^*(n-mu)P_{nu,-mu}(n) + Z^*(n-mu-nu)P_{-mu,-nu}(n). */
static mat clover(const lat *L, const cplx *links, long i, int mu, int nu) {
    if (mu == nu) return m_zero();
    int pm = mu, mm = -(mu + 1), pn = nu, mn = -(nu + 1);
    long i_n = step(L, i, nu, -1), i_m = step(L, i, mu, -1);
    long i_mn = step(L, i_m, nu, -1);
    mat C = m_scale(conj(zfac(L, i, mu, nu)), plaq_s(L, links, i, pm, pn));
    C = m_add(C, m_scale(conj(zfac(L, i_n, mu, nu)), plaq_s(L, links, i, mn, pm)));
    C = m_add(C, m_scale(conj(zfac(L, i_m, mu, nu)), plaq_s(L, links, i, pn, mm)));
    C = m_add(C, m_scale(conj(zfac(L, i_mn, mu, nu)), plaq_s(L, links, i, mm, mn)));
    mat Cd = m_dag(C);
    mat G;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G.a[a][b] = (-I / 8.0) * (C.a[a][b] - Cd.a[a][b]);
    return G;
}

static int levi(int a, int b, int c, int d) {
    int p[4] = {a, b, c, d}, s = 1;
    for (int x = 0; x < 4; x++)
        for (int y = x + 1; y < 4; y++) {
            if (p[x] == p[y]) return 0;
            if (p[x] > p[y]) s = -s;
        }
    return s;
}

/* per-site densities: e(n), q(n), plaquette sum, action density */
static void site_obs(const lat *L, const cplx *links, long i, double out[4]) {
    mat G[4][4];
    for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) G[m][n] = clover(L, links, i, m, n);
    double e = 0, q = 0, p = 0, s = 0;
    for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) {
            e += 0.5 * creal(m_tr(m_mul(G[m][n], G[m][n])));
            for (int r = 0; r < 4; r++)
                for (int t = 0; t < 4; t++) {
                    int eps = levi(m, n, r, t);
                    if (eps) q += 0.5 * eps * creal(m_tr(m_mul(G[m][n], G[r][t])));
                }
        }
    q /= 16.0 * PI * PI;
    for (int m = 0; m < 4; m++)
        for (int n = m + 1; n < 4; n++) {
            double re = creal(conj(zfac(L, i, m, n)) * m_tr(plaq_s(L, links, i, m, n)));
            p += re;
            s += 3.0 - re;
        }
    out[0] = e; out[1] = q; out[2] = p; out[3] = s;
}

static double pairwise_sum(const double *x, long n, long stride) {
    if (n <= 8) {
        double s = 0;
        for (long k = 0; k < n; k++) s += x[k * stride];
        return s;
    }
    long h = n / 2;
    return pairwise_sum(x, h, stride) + pairwise_sum(x + h * stride, n - h, stride);
}

/* out: [E, plaq, Q, action] with E the site average of e(n) */
static int measure(const lat *L, const cplx *links, double out[4]) {
    long V = L->V;
    double *d = (double *)malloc(sizeof(double) * 4 * V);
    if (!d) return -2;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) site_obs(L, links, i, d + 4 * i);
    double e = pairwise_sum(d + 0, V, 4), q = pairwise_sum(d + 1, V, 4);
    double p = pairwise_sum(d + 2, V, 4), s = pairwise_sum(d + 3, V, 4);
    free(d);
    out[0] = e / V;
    out[1] = p / (18.0 * V);
    out[2] = q;
    out[3] = s;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Luscher RK3 step (explicit Z0, Z1, Z2)                              */
/*
 *   W0 = V_t,  Z_i = eps F(W_i)
 *   W1 = exp(Z0/4) W0
 *   W2 = exp(8/9 Z1 - 17/36 Z0) W1
 *   V_{t+eps} = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2
 */
static int rk3_step(const lat *L, cplx *links, double eps) {
    long V = L->V, NL = 4 * V;
    mat *Z0 = (mat *)malloc(sizeof(mat) * NL);
    mat *Z1 = (mat *)malloc(sizeof(mat) * NL);
    mat *Z2 = (mat *)malloc(sizeof(mat) * NL);
    if (!Z0 || !Z1 || !Z2) { free(Z0); free(Z1); free(Z2); return -2; }
    mat *W = (mat *)links;

    force_field(L, links, Z0);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < NL; l++) {
        Z0[l] = m_scale(eps, Z0[l]);
        W[l] = m_mul(m_exp(m_scale(0.25, Z0[l])), W[l]);
    }
    force_field(L, links, Z1);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < NL; l++) {
        Z1[l] = m_scale(eps, Z1[l]);
        mat A = m_add(m_scale(8.0 / 9.0, Z1[l]), m_scale(-17.0 / 36.0, Z0[l]));
        W[l] = m_mul(m_exp(A), W[l]);
    }
    force_field(L, links, Z2);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < NL; l++) {
        Z2[l] = m_scale(eps, Z2[l]);
        mat A = m_add(m_add(m_scale(0.75, Z2[l]), m_scale(-8.0 / 9.0, Z1[l])),
                      m_scale(17.0 / 36.0, Z0[l]));
        W[l] = m_mul(m_exp(A), W[l]);
    }
    free(Z0); free(Z1); free(Z2);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Monte Carlo: hybrid over-relaxation (sec. 3.1: one heat-bath sweep  */
/* followed by n_or over-relaxation sweeps) with Cabibbo-Marinari      */
/* SU(2) subgroups (0,1), (0,2), (1,2), on a checkerboard              */
/*
 * Local action of U_mu(n): -(beta/3) Re Tr[U_mu(n) S] with S the twisted
 * staple sum (Omega = U S above), beta = 18 b (S_W = 3b sum_{mu!=nu} Tr[1 - Z^* P]).
 * A subgroup update U -> A U (A in SU(2) on rows i, j) changes Re Tr[U S] by
 * Re Tr[A W_ij] - Re Tr[W_ij] with W = U S; for A = a0 + i a.sigma,
 * Re Tr[A W_ij] = a . c with c = (W_ii.re + W_jj.re, -(W_ij.im + W_ji.im),
 * W_ji.re - W_ij.re, W_jj.im - W_ii.im).  Heat bath: A = Y C^ with C^ the SU(2)
 * element of c/|c| and Y drawn with density ~ exp(alpha y0), alpha = beta |c|/3
 * (Creutz for alpha < 2, Kennedy-Pendleton otherwise).  Over-relaxation:
 * A = C^ C^, which keeps Re Tr[U S].
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), counter
 * (site, sweep, mu<<24 | subgroup<<16 | attempt, config), key = seed;
 * u = (x + 1/2) 2^-32.
 */
typedef struct { unsigned int v[4]; } u4;

static u4 philox4x32_10(u4 ctr, unsigned int k0, unsigned int k1) {
    const unsigned int M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const unsigned int W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += W0; k1 += W1; }
        unsigned long long p0 = (unsigned long long)M0 * ctr.v[0];
        unsigned long long p1 = (unsigned long long)M1 * ctr.v[2];
        u4 o;
        o.v[0] = (unsigned int)(p1 >> 32) ^ ctr.v[1] ^ k0;
        o.v[1] = (unsigned int)p1;
        o.v[2] = (unsigned int)(p0 >> 32) ^ ctr.v[3] ^ k1;
        o.v[3] = (unsigned int)p0;
        ctr = o;
    }
    return ctr;
}

static double u01(unsigned int x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* y0 with density ~ sqrt(1 - y0^2) exp(alpha y0) on [-1, 1], then a uniform
 * direction for (y1, y2, y3); ctr.v[2] holds mu<<24 | subgroup<<16 */
static void su2_draw(double alpha, u4 ctr, unsigned int k0, unsigned int k1, double y[4]) {
    double y0 = 1.0;
    int ok = 0;
    for (unsigned int att = 0; att < 256 && !ok; att++) {
        u4 c = ctr;
        c.v[2] |= att;
        u4 r = philox4x32_10(c, k0, k1);
        double u1 = u01(r.v[0]), u2 = u01(r.v[1]), u3 = u01(r.v[2]), u4_ = u01(r.v[3]);
        if (alpha < 1e-8) {
            y0 = 2.0 * u1 - 1.0;
            ok = u2 * u2 <= 1.0 - y0 * y0;
        } else if (alpha < 2.0) {            /* Creutz */
            double e = exp(-2.0 * alpha);
            y0 = 1.0 + log(u1 * (1.0 - e) + e) / alpha;
            ok = u2 * u2 <= 1.0 - y0 * y0;
        } else {                             /* Kennedy-Pendleton */
            double cs = cos(2.0 * PI * u2);
            double X = -(log(u1) + cs * cs * log(u3)) / (2.0 * alpha);
            y0 = 1.0 - 2.0 * X;
            ok = u4_ * u4_ <= 1.0 - X;
        }
    }
    if (!ok) { y[0] = 1; y[1] = y[2] = y[3] = 0; return; }
    u4 c = ctr;
    c.v[2] |= 0xFFFFu;
    u4 r = philox4x32_10(c, k0, k1);
    double ct = 2.0 * u01(r.v[0]) - 1.0, ph = 2.0 * PI * u01(r.v[1]);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct)), rr = sqrt(fmax(0.0, 1.0 - y0 * y0));
    y[0] = y0;
    y[1] = rr * st * cos(ph);
    y[2] = rr * st * sin(ph);
    y[3] = rr * ct;
}

/* SU(2) matrix of the unit quaternion a: [[a0 + i a3, a2 + i a1], [-a2 + i a1, a0 - i a3]] */
static void q2m(const double a[4], cplx m[2][2]) {
    m[0][0] = a[0] + I * a[3];
    m[0][1] = a[2] + I * a[1];
    m[1][0] = -a[2] + I * a[1];
    m[1][1] = a[0] - I * a[3];
}

/* left-multiply rows i, j of X by the 2x2 matrix A */
static void rows_mul(mat *X, int i, int j, cplx A[2][2]) {
    for (int k = 0; k < 3; k++) {
        cplx xi = X->a[i][k], xj = X->a[j][k];
        X->a[i][k] = A[0][0] * xi + A[0][1] * xj;
        X->a[j][k] = A[1][0] * xi + A[1][1] * xj;
    }
}

static void update_link(const lat *L, cplx *links, long i, int mu, double beta, int heatbath,
                        unsigned long long seed, unsigned int sweep, unsigned int cfg) {
    mat W = omega(L, links, i, mu);          /* U S with the twist factors */
    mat Um = U(links, i, mu);
    const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int s = 0; s < 3; s++) {
        int a = sub[s][0], b = sub[s][1];
        double c[4];
        c[0] = creal(W.a[a][a]) + creal(W.a[b][b]);
        c[1] = -(cimag(W.a[a][b]) + cimag(W.a[b][a]));
        c[2] = creal(W.a[b][a]) - creal(W.a[a][b]);
        c[3] = cimag(W.a[b][b]) - cimag(W.a[a][a]);
        double k = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + c[3] * c[3]);
        if (!(k > 1e-300)) continue;
        double ch[4] = {c[0] / k, c[1] / k, c[2] / k, c[3] / k};
        cplx C[2][2], A[2][2];
        q2m(ch, C);
        if (heatbath) {
            u4 ctr = {{(unsigned int)i, sweep, ((unsigned int)mu << 24) | ((unsigned int)s << 16), cfg}};
            double y[4];
            su2_draw(beta * k / 3.0, ctr, (unsigned int)seed, (unsigned int)(seed >> 32), y);
            cplx Y[2][2];
            q2m(y, Y);
            for (int p = 0; p < 2; p++)
                for (int q = 0; q < 2; q++) A[p][q] = Y[p][0] * C[0][q] + Y[p][1] * C[1][q];
        } else {
            for (int p = 0; p < 2; p++)
                for (int q = 0; q < 2; q++) A[p][q] = C[p][0] * C[0][q] + C[p][1] * C[1][q];
        }
        rows_mul(&Um, a, b, A);
        rows_mul(&W, a, b, A);
    }
    memcpy(links + (i * 4 + mu) * 9, &Um, sizeof Um);
}

static void mc_sweep(const lat *L, cplx *links, double beta, int heatbath,
                     unsigned long long seed, unsigned int sweep, unsigned int cfg) {
    for (int mu = 0; mu < 4; mu++)
        for (int par = 0; par < 2; par++) {
#pragma omp parallel for schedule(static)
            for (long i = 0; i < L->V; i++) {
                int n[4];
                coords(L, i, n);
                if (((n[0] + n[1] + n[2] + n[3]) & 1) != par) continue;
                update_link(L, links, i, mu, beta, heatbath, seed, sweep, cfg);
            }
        }
}

/* ------------------------------------------------------------------ */
/* exported entry points (ctypes)                                      */

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* out[4] = E (site average of e(n)), plaquette, Q, action s */
int oracle_measure(const cplx *links, const int dims[4], const int twist[6],
                   const int base[4], double out[4]) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
    return measure(&L, links, out);
}

/* F[V][4][3][3] = -P_ah(Omega_mu(n)) */
int oracle_force(const cplx *links, const int dims[4], const int twist[6],
                 const int base[4], cplx *F) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
    force_field(&L, links, (mat *)F);
    return 0;
}

void oracle_expm(const cplx *A, cplx *out) {
    mat a;
    memcpy(&a, A, sizeof a);
    mat r = m_exp(a);
    memcpy(out, &r, sizeof r);
}

/* per-site e(n), q(n) arrays (for density tests) */
int oracle_densities(const cplx *links, const int dims[4], const int twist[6],
                     const int base[4], double *e, double *q) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < L.V; i++) {
        double o[4];
        site_obs(&L, links, i, o);
        e[i] = o[0];
        q[i] = o[1];
    }
    return 0;
}

int oracle_rk3_step(cplx *links, const int dims[4], const int twist[6],
                    const int base[4], double eps) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
    return rk3_step(&L, links, eps);
}

static int on_grid(double t, double dt) {
    if (dt <= 0) return 0;
    double k = floor(t / dt + 0.5);
    return fabs(t - k * dt) <= 1e-9;
}

/*
 * Flow links in place from t0 to t_end with step eps and write rows
 * [t, E, t^2 E, plaq, Q, s] to rows[max_rows][6].
 *   steps:  t_k = t0 + k*eps for every k with t_k <= t_end + 1e-12, then one
 *           short step to t_end if t_end - t_last > 1e-12;
 *   rows:   at t0 if t0 lies on the meas_dt grid, after every step that
 *           ends on the grid, and at t_end (once).
 * Returns the number of rows, or a negative status.
 */
int oracle_flow(cplx *links, const int dims[4], const int twist[6], const int base[4],
                double eps, double t0, double t_end, double meas_dt,
                double *rows, int max_rows) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
    if (!(eps > 0) || t_end < t0) return -1;
    int nr = 0;
    double o[4];
#define EMIT(tt)                                                         \
    do {                                                                 \
        if (nr >= max_rows) return -3;                                   \
        if (measure(&L, links, o)) return -2;                            \
        double *r = rows + 6 * nr++;                                     \
        r[0] = (tt); r[1] = o[0]; r[2] = (tt) * (tt) * o[0];             \
        r[3] = o[1]; r[4] = o[2]; r[5] = o[3];                           \
    } while (0)

    long n_full = 0;
    while (t0 + (n_full + 1) * eps <= t_end + 1e-12) n_full++;
    double t_last = t0 + n_full * eps;
    int has_short = (t_end - t_last) > 1e-12;

    if (on_grid(t0, meas_dt) || (!has_short && n_full == 0)) EMIT(t0);
    for (long k = 1; k <= n_full; k++) {
        if (rk3_step(&L, links, eps)) return -2;
        double t = t0 + k * eps;
        int last = (k == n_full) && !has_short;
        if (on_grid(t, meas_dt) || last) EMIT(t);
    }
    if (has_short) {
        if (rk3_step(&L, links, t_end - t_last)) return -2;
        EMIT(t_end);
    }
#undef EMIT
    return nr;
}

/* n_hybrid times: one heat-bath sweep (index sweep0 + h (1 + n_or)) and n_or
 * over-relaxation sweeps; beta = 18 b.  All extents must be even. */
int oracle_mc(cplx *links, const int dims[4], const int twist[6], const int base[4],
              double beta, int n_hybrid, int n_or, unsigned long long seed,
              unsigned int sweep0, unsigned int cfg) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
    for (int m = 0; m < 4; m++)
        if (dims[m] % 2) return -1;
    unsigned int sw = sweep0;
    for (int h = 0; h < n_hybrid; h++) {
        mc_sweep(&L, links, beta, 1, seed, sw++, cfg);
        for (int o = 0; o < n_or; o++) mc_sweep(&L, links, beta, 0, seed, sw++, cfg);
    }
    return 0;
}

/* over-relaxation sweeps only (no random numbers) */
int oracle_or_sweeps(cplx *links, const int dims[4], const int twist[6], const int base[4],
                     int n) {
    lat L;
    if (lat_init(&L, dims, twist, base)) return -1;
    for (int m = 0; m < 4; m++)
        if (dims[m] % 2) return -1;
    for (int o = 0; o < n; o++) mc_sweep(&L, links, 0.0, 0, 0, 0, 0);
    return 0;
}

/* n draws of the SU(2) heat-bath quaternion for a fixed alpha (sampler test) */
void oracle_su2_samples(double alpha, unsigned long long seed, int n, double *out) {
    for (int k = 0; k < n; k++) {
        u4 ctr = {{(unsigned int)k, 7u, 0u, 0u}};
        su2_draw(alpha, ctr, (unsigned int)seed, (unsigned int)(seed >> 32), out + 4 * k);
    }
}

/* raw Philox4x32-10 output */
void oracle_philox(const unsigned int ctr[4], unsigned int k0, unsigned int k1, unsigned int out[4]) {
    u4 c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
    u4 r = philox4x32_10(c, k0, k1);
    memcpy(out, r.v, sizeof r.v);
}
