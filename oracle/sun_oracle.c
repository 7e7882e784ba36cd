/*
 * sun_oracle.c -- plain, slow, FP64 CPU oracle for the twisted Wilson flow of
 * SU(N) gauge fields, 2 <= N <= 8.
 *
 * TEST INFRASTRUCTURE ONLY.  Independent reference for the GPU library's
 * SU(N) path; it shares no code, header, table or helper with it (the two
 * meet only in the canonical link layout).  It is also independent of the
 * SU(3) oracle in this directory, against which it is checked at N = 3.
 *
 * Paper: arXiv 2107.03747.  The TGF scheme is defined for SU(N) on an
 * l^2 x (N l)^2 box with the short plane twisted, Z_12 = exp(2 pi i k / N), k
 * and N coprime (sec. 1); the Wilson action with twist factors, the clover
 * G_{mu nu} (eq. gmunu) and the charge (eq. qlatt) are those of sec. 3.1 with
 * N colours:
 *   S_W = (N b) sum_n sum_{mu != nu} Tr[1 - Z^*_{mu nu}(n) P_{mu nu}(n)], b = 1/lambda_0
 *   plaquette = (1 / (6 N V)) sum_n sum_{mu<nu} Re Tr[Z^* P]
 *   action    = sum_n sum_{mu<nu} Re Tr[1 - Z^* P]
 *   E = site average of 1/2 sum_{mu,nu} Tr G G,   Q = (1/16 pi^2) sum_n Tr G G~
 *   force F = -P_ah(Omega), P_ah(M) = (M - M^+)/2 - Tr(M - M^+)/(2N)
 * integrated with Luscher's RK3 scheme (explicit Z0, Z1, Z2).  Readings as in
 * the SU(3) oracle: twist site n_mu = n_nu = 0 (parameter base[]), no trace
 * subtraction in G (parity unpinned, a convention), eps_{0123} = +1, the same
 * step schedule.  The twist tensor
 * n_{mu nu} is taken mod N.
 *
 * The exponential is scaling-and-squaring with a term-by-term Taylor sum to
 * degree 20 after scaling to ||A||_F <= 1/8.
 *
 * Layout: complex128 [d3][d2][d1][d0][4][N][N], n0 fastest, row-major N x N.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define NMAX 8

typedef struct { cplx a[NMAX][NMAX]; } matn;

typedef struct {
    int n;          /* colours */
    int d[4];
    long V;
    int tw[4][4];   /* n_{mu nu} mod N, antisymmetric */
    int base[4];
} latn;

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ */
/* N x N complex matrices                                              */

static matn z_zero(void) { matn r; memset(&r, 0, sizeof r); return r; }

static matn z_eye(int n) {
    matn r = z_zero();
    for (int i = 0; i < n; i++) r.a[i][i] = 1.0;
    return r;
}

static matn z_mul(int n, const matn *x, const matn *y) {
    matn r = z_zero();
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            cplx s = 0;
            for (int k = 0; k < n; k++) s += x->a[i][k] * y->a[k][j];
            r.a[i][j] = s;
        }
    return r;
}

static matn z_dag(int n, const matn *x) {
    matn r = z_zero();
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) r.a[i][j] = conj(x->a[j][i]);
    return r;
}

static void z_axpy(int n, cplx c, const matn *x, matn *y) {
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) y->a[i][j] += c * x->a[i][j];
}

static matn z_scale(int n, cplx c, matn x) {
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) x.a[i][j] *= c;
    return x;
}

static cplx z_tr(int n, const matn *x) {
    cplx s = 0;
    for (int i = 0; i < n; i++) s += x->a[i][i];
    return s;
}

static double z_fnorm(int n, const matn *x) {
    double s = 0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) s += creal(x->a[i][j] * conj(x->a[i][j]));
    return sqrt(s);
}

/* traceless anti-Hermitian part */
static matn z_proj_ah(int n, const matn *m) {
    matn r = z_zero();
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) r.a[i][j] = 0.5 * (m->a[i][j] - conj(m->a[j][i]));
    cplx t = z_tr(n, &r) / (double)n;
    for (int i = 0; i < n; i++) r.a[i][i] -= t;
    return r;
}

static matn z_exp(int n, const matn *A) {
    double nrm = z_fnorm(n, A);
    int s = 0;
    if (nrm > 0.125) s = (int)ceil(log2(nrm / 0.125));
    matn B = z_scale(n, ldexp(1.0, -s), *A);
    matn sum = z_eye(n), term = z_eye(n);
    for (int k = 1; k <= 20; k++) {
        term = z_mul(n, &term, &B);
        term = z_scale(n, 1.0 / k, term);
        z_axpy(n, 1.0, &term, &sum);
    }
    for (int i = 0; i < s; i++) sum = z_mul(n, &sum, &sum);
    return sum;
}

/* ------------------------------------------------------------------ */
/* lattice                                                             */

static int latn_init(latn *L, int nc, const int dims[4], const int twist6[6], const int base[4]) {
    if (nc < 2 || nc > NMAX) return -1;
    L->n = nc;
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
        for (int v = m + 1; v < 4; v++, k++) {
            int t = twist6 ? ((twist6[k] % nc) + nc) % nc : 0;
            L->tw[m][v] = t;
            L->tw[v][m] = (nc - t) % nc;
        }
    return 0;
}

static void coords(const latn *L, long i, int x[4]) {
    for (int m = 0; m < 4; m++) { x[m] = (int)(i % L->d[m]); i /= L->d[m]; }
}

static long index_of(const latn *L, const int x[4]) {
    long i = 0;
    for (int m = 3; m >= 0; m--) i = i * L->d[m] + x[m];
    return i;
}

static long hop(const latn *L, long i, int mu, int s) {
    int x[4];
    coords(L, i, x);
    x[mu] = ((x[mu] + s) % L->d[mu] + L->d[mu]) % L->d[mu];
    return index_of(L, x);
}

/* Z_{mu nu}(n) = exp(2 pi i n_{mu nu} / N) on the twist site of the plane */
static cplx zf(const latn *L, long i, int mu, int nu) {
    if (mu == nu || L->tw[mu][nu] == 0) return 1.0;
    int x[4];
    coords(L, i, x);
    if (x[mu] != L->base[mu] || x[nu] != L->base[nu]) return 1.0;
    return cexp(I * (2.0 * PI * L->tw[mu][nu] / L->n));
}

static matn link(const latn *L, const cplx *U, long i, int mu) {
    const int n = L->n;
    matn r = z_zero();
    const cplx *p = U + ((size_t)i * 4 + mu) * n * n;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) r.a[a][b] = p[a * n + b];
    return r;
}

static void put(const latn *L, cplx *U, long i, int mu, const matn *m) {
    const int n = L->n;
    cplx *p = U + ((size_t)i * 4 + mu) * n * n;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) p[a * n + b] = m->a[a][b];
}

/* signed directions: dir = mu (forward) or -(mu+1) (backward) */
static matn link_s(const latn *L, const cplx *U, long i, int dir) {
    if (dir >= 0) return link(L, U, i, dir);
    int mu = -dir - 1;
    matn x = link(L, U, hop(L, i, mu, -1), mu);
    return z_dag(L->n, &x);
}

static long hop_s(const latn *L, long i, int dir) {
    return dir >= 0 ? hop(L, i, dir, +1) : hop(L, i, -dir - 1, -1);
}

/* P_{ab}(n) = U_a(n) U_b(n+a) U_a(n+b)^+ U_b(n)^+, signed directions */
static matn plaq_dir(const latn *L, const cplx *U, long i, int a, int b) {
    const int n = L->n;
    matn x = link_s(L, U, i, a);
    matn y = link_s(L, U, hop_s(L, i, a), b);
    x = z_mul(n, &x, &y);
    y = link_s(L, U, hop_s(L, i, b), a);
    y = z_dag(n, &y);
    x = z_mul(n, &x, &y);
    y = link_s(L, U, i, b);
    y = z_dag(n, &y);
    return z_mul(n, &x, &y);
}

/* Omega_mu(n): every plaquette of S_W that starts with U_mu(n) --
 * upper Z^*_{mu nu}(n) P_{mu nu}(n) and lower Z_{mu nu}(n - nu) times
 * U_mu(n) U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu) */
static matn omega(const latn *L, const cplx *U, long i, int mu) {
    const int n = L->n;
    matn om = z_zero();
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        matn up = plaq_dir(L, U, i, mu, nu);
        z_axpy(n, conj(zf(L, i, mu, nu)), &up, &om);
        long imn = hop(L, i, nu, -1);
        matn lo = plaq_dir(L, U, i, mu, -(nu + 1));   /* U_mu(n) U_-nu(n+mu) ... */
        z_axpy(n, zf(L, imn, mu, nu), &lo, &om);
    }
    return om;
}

/* F_mu(n) = -P_ah(Omega_mu(n)), canonical layout */
static void force_field(const latn *L, const cplx *U, cplx *F) {
    const int n = L->n;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < L->V; i++)
        for (int mu = 0; mu < 4; mu++) {
            matn om = omega(L, U, i, mu);
            matn f = z_proj_ah(n, &om);
            f = z_scale(n, -1.0, f);
            put(L, F, i, mu, &f);
        }
}

/* clover G_{mu nu}(n) = -(i/8)(C - C^+), C the four twisted leaves */
static matn clover(const latn *L, const cplx *U, long i, int mu, int nu) {
    const int n = L->n;
    int pm = mu, mm = -(mu + 1), pn = nu, mn = -(nu + 1);
    long i_n = hop(L, i, nu, -1), i_m = hop(L, i, mu, -1), i_mn = hop(L, i_m, nu, -1);
    matn C = z_zero(), x;
    x = plaq_dir(L, U, i, pm, pn);  z_axpy(n, conj(zf(L, i, mu, nu)), &x, &C);
    x = plaq_dir(L, U, i, mn, pm);  z_axpy(n, conj(zf(L, i_n, mu, nu)), &x, &C);
    x = plaq_dir(L, U, i, pn, mm);  z_axpy(n, conj(zf(L, i_m, mu, nu)), &x, &C);
    x = plaq_dir(L, U, i, mm, mn);  z_axpy(n, conj(zf(L, i_mn, mu, nu)), &x, &C);
    matn G = z_zero();
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) G.a[a][b] = (-I / 8.0) * (C.a[a][b] - conj(C.a[b][a]));
    return G;
}

static int perm_sign(int a, int b, int c, int d) {
    int p[4] = {a, b, c, d}, s = 1;
    for (int x = 0; x < 4; x++)
        for (int y = x + 1; y < 4; y++) {
            if (p[x] == p[y]) return 0;
            if (p[x] > p[y]) s = -s;
        }
    return s;
}

static double tr_prod_re(int n, const matn *a, const matn *b) {
    double s = 0;
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) s += creal(a->a[i][k] * b->a[k][i]);
    return s;
}

/* e(n), q(n), plaquette sum, action density */
static void site_obs(const latn *L, const cplx *U, long i, double out[4]) {
    const int n = L->n;
    static const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    matn G[4][4];
    for (int a = 0; a < 4; a++) G[a][a] = z_zero();
    for (int p = 0; p < 6; p++) {
        int a = pairs[p][0], b = pairs[p][1];
        G[a][b] = clover(L, U, i, a, b);
        G[b][a] = z_scale(n, -1.0, G[a][b]);
    }
    double e = 0, q = 0, pl = 0, s = 0;
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            e += 0.5 * tr_prod_re(n, &G[a][b], &G[a][b]);
            for (int c = 0; c < 4; c++)
                for (int d = 0; d < 4; d++) {
                    int sg = perm_sign(a, b, c, d);
                    if (sg) q += 0.5 * sg * tr_prod_re(n, &G[a][b], &G[c][d]);
                }
        }
    q /= 16.0 * PI * PI;
    for (int p = 0; p < 6; p++) {
        int a = pairs[p][0], b = pairs[p][1];
        matn P = plaq_dir(L, U, i, a, b);
        double re = creal(conj(zf(L, i, a, b)) * z_tr(n, &P));
        pl += re;
        s += n - re;
    }
    out[0] = e; out[1] = q; out[2] = pl; out[3] = s;
}

static double psum(const double *x, long m, long stride) {
    if (m <= 8) {
        double s = 0;
        for (long k = 0; k < m; k++) s += x[k * stride];
        return s;
    }
    long h = m / 2;
    return psum(x, h, stride) + psum(x + h * stride, m - h, stride);
}

static int measure(const latn *L, const cplx *U, double out[4], double *e_out, double *q_out) {
    long V = L->V;
    double *d = (double *)malloc(sizeof(double) * 4 * V);
    if (!d) return -2;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) site_obs(L, U, i, d + 4 * i);
    if (e_out)
        for (long i = 0; i < V; i++) e_out[i] = d[4 * i];
    if (q_out)
        for (long i = 0; i < V; i++) q_out[i] = d[4 * i + 1];
    out[0] = psum(d + 0, V, 4) / V;
    out[1] = psum(d + 2, V, 4) / (6.0 * L->n * V);
    out[2] = psum(d + 1, V, 4);
    out[3] = psum(d + 3, V, 4);
    free(d);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Luscher RK3: W1 = exp(Z0/4) W0, W2 = exp(8/9 Z1 - 17/36 Z0) W1,     */
/* W3 = exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) W2, Z_i = eps F(W_i)           */

static int rk3(const latn *L, cplx *U, double eps) {
    const int n = L->n;
    const size_t NL = (size_t)4 * L->V, E = (size_t)n * n;
    cplx *Z0 = (cplx *)malloc(sizeof(cplx) * NL * E);
    cplx *Z1 = (cplx *)malloc(sizeof(cplx) * NL * E);
    cplx *Z2 = (cplx *)malloc(sizeof(cplx) * NL * E);
    if (!Z0 || !Z1 || !Z2) { free(Z0); free(Z1); free(Z2); return -2; }
    const double c[3][3] = {{0.25, 0, 0}, {-17.0 / 36.0, 8.0 / 9.0, 0}, {17.0 / 36.0, -8.0 / 9.0, 0.75}};
    cplx *Z[3] = {Z0, Z1, Z2};
    for (int st = 0; st < 3; st++) {
        force_field(L, U, Z[st]);
#pragma omp parallel for schedule(static)
        for (long l = 0; l < (long)NL; l++) {
            for (size_t e = 0; e < E; e++) Z[st][l * E + e] *= eps;
            matn A = z_zero();
            for (int k = 0; k <= st; k++)
                for (int a = 0; a < n; a++)
                    for (int b = 0; b < n; b++) A.a[a][b] += c[st][k] * Z[k][l * E + a * n + b];
            matn X = z_exp(n, &A);
            matn W = link(L, U, l / 4, (int)(l % 4));
            W = z_mul(n, &X, &W);
            put(L, U, l / 4, (int)(l % 4), &W);
        }
    }
    free(Z0); free(Z1); free(Z2);
    return 0;
}

static int grid_point(double t, double dt) {
    if (dt <= 0) return 0;
    double k = floor(t / dt + 0.5);
    return fabs(t - k * dt) <= 1e-9;
}

/* ------------------------------------------------------------------ */
/* exported entry points (ctypes)                                      */

int oracle_sun_measure(const cplx *U, int nc, const int dims[4], const int twist[6],
                       const int base[4], double out[4]) {
    latn L;
    if (latn_init(&L, nc, dims, twist, base)) return -1;
    return measure(&L, U, out, NULL, NULL);
}

int oracle_sun_densities(const cplx *U, int nc, const int dims[4], const int twist[6],
                         const int base[4], double *e, double *q) {
    latn L;
    double o[4];
    if (latn_init(&L, nc, dims, twist, base)) return -1;
    return measure(&L, U, o, e, q);
}

int oracle_sun_force(const cplx *U, int nc, const int dims[4], const int twist[6],
                     const int base[4], cplx *F) {
    latn L;
    if (latn_init(&L, nc, dims, twist, base)) return -1;
    force_field(&L, U, F);
    return 0;
}

int oracle_sun_expm(int nc, const cplx *A, cplx *out) {
    if (nc < 2 || nc > NMAX) return -1;
    matn a = z_zero();
    for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) a.a[i][j] = A[i * nc + j];
    matn r = z_exp(nc, &a);
    for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) out[i * nc + j] = r.a[i][j];
    return 0;
}

int oracle_sun_rk3_step(cplx *U, int nc, const int dims[4], const int twist[6],
                        const int base[4], double eps) {
    latn L;
    if (latn_init(&L, nc, dims, twist, base)) return -1;
    return rk3(&L, U, eps);
}

/* rows of [t, E, t^2 E, plaq, Q, action]; same schedule as the SU(3) oracle */
int oracle_sun_flow(cplx *U, int nc, const int dims[4], const int twist[6], const int base[4],
                    double eps, double t0, double t_end, double meas_dt, double *rows,
                    int max_rows) {
    latn L;
    if (latn_init(&L, nc, dims, twist, base)) return -1;
    if (!(eps > 0) || t_end < t0) return -1;
    int nr = 0;
    double o[4];
    long n_full = 0;
    while (t0 + (n_full + 1) * eps <= t_end + 1e-12) n_full++;
    const double t_last = t0 + n_full * eps;
    const int has_short = (t_end - t_last) > 1e-12;
    for (long k = 0; k <= n_full + has_short; k++) {
        double t;
        if (k == 0) {
            t = t0;
        } else if (k <= n_full) {
            if (rk3(&L, U, eps)) return -2;
            t = t0 + k * eps;
        } else {
            if (rk3(&L, U, t_end - t_last)) return -2;
            t = t_end;
        }
        const int last = k == n_full + has_short;
        if (grid_point(t, meas_dt) || last) {
            if (nr >= max_rows) return -3;
            if (measure(&L, U, o, NULL, NULL)) return -2;
            double *r = rows + 6 * nr++;
            r[0] = t; r[1] = o[0]; r[2] = t * t * o[0]; r[3] = o[1]; r[4] = o[2]; r[5] = o[3];
        }
    }
    return nr;
}
