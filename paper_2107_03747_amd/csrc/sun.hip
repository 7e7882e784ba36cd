// sun.hip -- twisted Wilson flow of SU(N) gauge fields, FP64, 2 <= N <= 8,
// for gfx950.
//
// Method (arXiv 2107.03747): the TGF scheme is defined for SU(N) on an
// l^2 x (N l)^2 box whose short plane is twisted by Z = exp(2 pi i k / N)
// (sec. 1); the twisted Wilson action, the clover G (eq. gmunu) and the charge
// (eq. qlatt) are those of sec. 3.1 with N colours.  The flow force is
// F = -P_ah(Omega) with P_ah(M) = (M - M^+)/2 - Tr(M - M^+)/(2N), integrated
// with Luscher's RK3 scheme in the same low-storage form as the SU(3) path,
// X_i = B_i eps F + A_i X_{i-1}, W_{i+1} = exp(X_i) W_i.
//
// Work decomposition ("row per lane"): the N x N matrix of a link is spread
// over N consecutive lanes of a wavefront, lane r holding row r, so a wave
// holds G = floor(64 / N) links.  In a product C = A B every lane forms its
// own row of C: its row of A is local, the rows of B come from the other
// lanes of its group through cross-lane permutes (ds_bpermute).  A^+ enters
// through the column of A that a lane needs (gathered the same way).  No
// matrix ever sits whole in one lane, so N = 8 needs 32 registers per row.
//
// Storage: FP64, [mu][entry][site] with entry = r N + j, the structure of
// arrays of the SU(3) full storage; the RK accumulator X is a full N x N
// matrix per link in the same layout.  A work-group is one tile of 64 sites.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "launch.h"
#include "lattice_dev.h"
#include "layout.h"
#include "su3_dev.h"

namespace tgf {

template <int N>
struct RowN {
    cx<double> e[N];
};

// this lane's place in its group of N lanes
struct Grp {
    int base;   // first lane of the group
    int r;      // row held by this lane
};

template <int N>
__device__ __forceinline__ RowN<N> row_zero() {
    RowN<N> o;
#pragma unroll
    for (int j = 0; j < N; j++) o.e[j] = {0.0, 0.0};
    return o;
}

// the row held by lane src of the wave
template <int N>
__device__ __forceinline__ RowN<N> row_from(const RowN<N> &m, int src) {
    RowN<N> o;
#pragma unroll
    for (int j = 0; j < N; j++) {
        o.e[j].x = __shfl(m.e[j].x, src);
        o.e[j].y = __shfl(m.e[j].y, src);
    }
    return o;
}

// entry r of a row for a lane-dependent r, by selection (no register indexing)
template <int N>
__device__ __forceinline__ cx<double> pick(const RowN<N> &m, int r) {
    cx<double> v = m.e[0];
#pragma unroll
    for (int j = 1; j < N; j++)
        if (r == j) v = m.e[j];
    return v;
}

template <int N>
__device__ __forceinline__ double group_sum(double v, const Grp &g) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < N; k++) s += __shfl(v, g.base + k);
    return s;
}

// row r of A B
template <int N>
__device__ __forceinline__ RowN<N> mm_nn(const RowN<N> &a, const RowN<N> &b, const Grp &g) {
    RowN<N> c = row_zero<N>();
#pragma unroll
    for (int k = 0; k < N; k++) {
        const RowN<N> bk = row_from(b, g.base + k);
#pragma unroll
        for (int j = 0; j < N; j++) c.e[j] = cmadd(c.e[j], a.e[k], bk.e[j]);
    }
    return c;
}

// row r of A B^+: (A B^+)_{rj} = sum_k A_{rk} conj(B_{jk})
template <int N>
__device__ __forceinline__ RowN<N> mm_nd(const RowN<N> &a, const RowN<N> &b, const Grp &g) {
    RowN<N> c;
#pragma unroll
    for (int j = 0; j < N; j++) {
        const RowN<N> bj = row_from(b, g.base + j);
        cx<double> s = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < N; k++) s = cmadd_nc(s, a.e[k], bj.e[k]);
        c.e[j] = s;
    }
    return c;
}

// column r of A: col_k = A_{kr}
template <int N>
__device__ __forceinline__ RowN<N> column(const RowN<N> &a, const Grp &g) {
    RowN<N> col;
#pragma unroll
    for (int k = 0; k < N; k++) col.e[k] = pick(row_from(a, g.base + k), g.r);
    return col;
}

// row r of A^+ B: sum_k conj(A_{kr}) B_k
template <int N>
__device__ __forceinline__ RowN<N> mm_dn(const RowN<N> &a, const RowN<N> &b, const Grp &g) {
    const RowN<N> col = column(a, g);
    RowN<N> c = row_zero<N>();
#pragma unroll
    for (int k = 0; k < N; k++) {
        const RowN<N> bk = row_from(b, g.base + k);
#pragma unroll
        for (int j = 0; j < N; j++) c.e[j] = cmadd_cn(c.e[j], col.e[k], bk.e[j]);
    }
    return c;
}

template <int N>
__device__ __forceinline__ void row_axpy(RowN<N> &y, cx<double> z, const RowN<N> &x) {
#pragma unroll
    for (int j = 0; j < N; j++) y.e[j] = cmadd(y.e[j], z, x.e[j]);
}

// ---------------------------------------------------------------------------
// storage access: row r of link (mu, site); the plane of mu is a uniform base,
// the lane part a 32-bit byte offset (sites per configuration are capped so
// that N^2 planes of one direction span less than 4 GiB)

template <int N>
__device__ __forceinline__ unsigned row_off(int r, int j, int stride, int site) {
    return ((unsigned)(r * N + j) * (unsigned)stride + (unsigned)site) * 16u;
}

template <int N>
__device__ __forceinline__ RowN<N> load_row(gptr<const v2<double>> W, int stride, int mu, int r,
                                            int site) {
    gptr<const v2<double>> q = W + (size_t)(mu * N * N) * stride;
    RowN<N> o;
#pragma unroll
    for (int j = 0; j < N; j++) o.e[j] = ld(q, row_off<N>(r, j, stride, site));
    return o;
}

template <int N>
__device__ __forceinline__ void store_row(gptr<v2<double>> W, int stride, int mu, int r, int site,
                                          const RowN<N> &v) {
    gptr<v2<double>> q = W + (size_t)(mu * N * N) * stride;
#pragma unroll
    for (int j = 0; j < N; j++) st(q, row_off<N>(r, j, stride, site), v.e[j]);
}

// twist exponent n_{mu nu} (mod N, antisymmetric) and Z = exp(2 pi i n / N)
template <int N>
__device__ __forceinline__ int tw_exp(const CfgDesc &c, int mu, int nu) {
    if (mu < nu) return c.tw[plane_index(mu, nu)];
    const int t = c.tw[plane_index(nu, mu)];
    return t ? N - t : 0;
}

template <int N>
__device__ __forceinline__ cx<double> zphase(int t) {
    double s, co;
    sincospi(2.0 * (double)t / (double)N, &s, &co);
    return {co, s};
}

// ---------------------------------------------------------------------------
// flow stage

// Omega_MU(n) = U_MU(n) S, S the twisted staple sum (upper staples times
// Z^*_{mu nu}(n), lower staples times Z_{mu nu}(n - nu))
template <int N, int MU>
__device__ __forceinline__ RowN<N> omega_row(gptr<const v2<double>> W, const CfgDesc &c,
                                             const Geo &g, const Grp &gr, RowN<N> &U) {
    const int st = c.stride, r = gr.r;
    RowN<N> S = row_zero<N>();
    auto add_staples = [&](int nu) {
        const int k = tw_exp<N>(c, MU, nu);
        // upper: U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
        RowN<N> t = mm_nd(load_row<N>(W, st, nu, r, g.i + g.up(MU)),
                          load_row<N>(W, st, MU, r, g.i + g.up(nu)), gr);
        t = mm_nd(t, load_row<N>(W, st, nu, r, g.i), gr);
        cx<double> z = {1.0, 0.0};
        if (k && g.n(MU) == 0 && g.n(nu) == 0) z = cconj(zphase<N>(k));
        row_axpy(S, z, t);
        // lower: (U_mu(n-nu) U_nu(n+mu-nu))^+ U_nu(n-nu)
        const int imn = g.i + g.dn(nu);
        t = mm_nn(load_row<N>(W, st, MU, r, imn), load_row<N>(W, st, nu, r, imn + g.up(MU)), gr);
        t = mm_dn(t, load_row<N>(W, st, nu, r, imn), gr);
        z = {1.0, 0.0};
        if (k && g.n(MU) == 0 && g.back(nu) == 0) z = zphase<N>(k);
        row_axpy(S, z, t);
    };
    if constexpr (N == 3) {
#pragma unroll
        for (int nu = 0; nu < 4; nu++)
            if (nu != MU) add_staples(nu);
    } else {
        // one direction at a time: unrolled, the loads of all six staples are
        // live together and the kernel spills from N = 5 on (and N = 2 keeps
        // two waves per SIMD this way)
#pragma unroll 1
        for (int nu = 0; nu < 4; nu++)
            if (nu != MU) add_staples(nu);
    }
    U = load_row<N>(W, st, MU, r, g.i);
    return mm_nn(U, S, gr);
}

// scale * P_ah(M), row r
template <int N>
__device__ __forceinline__ RowN<N> proj_ah_row(const RowN<N> &m, const Grp &g, double scale) {
    const RowN<N> col = column(m, g);   // col_j = M_{jr}; (M^+)_{rj} = conj(col_j)
    RowN<N> a;
#pragma unroll
    for (int j = 0; j < N; j++)
        a.e[j] = {0.5 * (m.e[j].x - col.e[j].x), 0.5 * (m.e[j].y + col.e[j].y)};
    // the diagonal of (M - M^+)/2 is i Im M_rr; remove the trace part
    const double t = group_sum<N>(pick(m, g.r).y, g) / (double)N;
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (j == g.r) a.e[j].y -= t;
        a.e[j] = {scale * a.e[j].x, scale * a.e[j].y};
    }
    return a;
}

// exp(X) for X anti-Hermitian: scale so that ||Y||_F <= 1/4 (Y = X 2^-s),
// degree-12 Taylor polynomial by Horner's rule as T <- 1 + T Y / k (T is a
// polynomial in Y, so T Y = Y T), then s squarings.  Truncation error
// ||Y||^13 / 13! < 3e-18.
template <int N>
__device__ __forceinline__ RowN<N> exp_row(const RowN<N> &x, const Grp &g) {
    double n2 = 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) n2 = fma(x.e[j].x, x.e[j].x, fma(x.e[j].y, x.e[j].y, n2));
    const double nrm = sqrt(group_sum<N>(n2, g));
    int s = 0;
    if (nrm > 0.25) s = (int)ceil(log2(nrm * 4.0));
    const double f = ldexp(1.0, -s);
    RowN<N> y;
#pragma unroll
    for (int j = 0; j < N; j++) y.e[j] = {f * x.e[j].x, f * x.e[j].y};
    constexpr int M = 12;
    RowN<N> t;
#pragma unroll
    for (int j = 0; j < N; j++) {
        t.e[j] = {y.e[j].x * (1.0 / M), y.e[j].y * (1.0 / M)};
        if (j == g.r) t.e[j].x += 1.0;
    }
    for (int k = M - 1; k >= 1; k--) {
        const RowN<N> ty = mm_nn(t, y, g);
        const double ik = 1.0 / (double)k;
#pragma unroll
        for (int j = 0; j < N; j++) {
            t.e[j] = {ty.e[j].x * ik, ty.e[j].y * ik};
            if (j == g.r) t.e[j].x += 1.0;
        }
    }
    for (int i = 0; i < s; i++) t = mm_nn(t, t, g);
    return t;
}

struct SunStageArgs {
    const CfgDesc *cfgs;
    const int *tile_start;
    int n_act;
    int n_tiles;
    int step;
    int stage;
    double eps;
};

__constant__ double kSunRkA[3] = {0.0, -17.0 / 9.0, -1.0};
__constant__ double kSunRkB[3] = {0.25, 8.0 / 9.0, 0.75};

template <int N, int MU>
__device__ __forceinline__ void sun_link_update(const SunStageArgs &a, const CfgDesc &c, int site,
                                                const Grp &gr) {
    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    gptr<const v2<double>> W = as_global<double>((const void *)(in ? c.W[1] : c.W[0]));
    gptr<v2<double>> Wout = as_global<double>(in ? c.W[0] : c.W[1]);
    gptr<v2<double>> X = as_global<double>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const Geo g = make_geo(c, site);
    RowN<N> U;
    const RowN<N> om = omega_row<N, MU>(W, c, g, gr, U);
    RowN<N> z = proj_ah_row(om, gr, -kSunRkB[a.stage] * eps);   // B eps F, F = -P_ah(Omega)
    if (a.stage > 0) {
        const RowN<N> xo = load_row<N>(X, c.stride, MU, gr.r, site);
        row_axpy(z, cx<double>{kSunRkA[a.stage], 0.0}, xo);
    }
    if (a.stage < 2) store_row<N>(X, c.stride, MU, gr.r, site, z);
    const RowN<N> e = exp_row(z, gr);
    store_row<N>(Wout, c.stride, MU, gr.r, site, mm_nn(e, U, gr));
}

// work-group = one tile of 64 sites; wave w updates direction w for the
// tile's sites, G = 64 / N at a time (lane = g N + r)
template <int N>
__global__ __launch_bounds__(256) void sun_stage_kernel(SunStageArgs a) {
    const int tile = blockIdx.x;
    if (tile >= a.n_tiles) return;
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc c = a.cfgs[ci];
    constexpr int G = 64 / N;
    const int lane = threadIdx.x & 63;
    const int g = lane / N;
    const Grp gr{g * N, lane - g * N};
    const int first = (tile - a.tile_start[ci]) * kTile;
    for (int s0 = 0; s0 < kTile; s0 += G) {
        const int site = first + s0 + g;
        if (g >= G || s0 + g >= kTile || site >= c.V) continue;
        switch (mu) {
            case 0: sun_link_update<N, 0>(a, c, site, gr); break;
            case 1: sun_link_update<N, 1>(a, c, site, gr); break;
            case 2: sun_link_update<N, 2>(a, c, site, gr); break;
            default: sun_link_update<N, 3>(a, c, site, gr); break;
        }
    }
}

// ---------------------------------------------------------------------------
// measurement: clover G (eq. gmunu) from the four twisted leaves, e(n),
// q(n) = (1/4 pi^2)[Tr G01 G23 - Tr G02 G13 + Tr G03 G12], plaquette and action

template <int N>
__device__ __forceinline__ cx<double> leaf_phase(const CfgDesc &c, int mu, int nu, int xm, int xn) {
    const int k = tw_exp<N>(c, mu, nu);
    if (k && xm == 0 && xn == 0) return cconj(zphase<N>(k));
    return {1.0, 0.0};
}

// row r of G_{mu nu}(n); rp += Re of this lane's diagonal entry of Z^* P_{mu nu}(n)
template <int N>
__device__ __forceinline__ RowN<N> clover_row(gptr<const v2<double>> W, const CfgDesc &c,
                                              const Geo &g, const Grp &gr, int mu, int nu,
                                              double &rp) {
    const int st = c.stride, r = gr.r;
    const int i = g.i, ipm = g.i + g.up(mu), ipn = g.i + g.up(nu);
    const int imm = g.i + g.dn(mu), imn = g.i + g.dn(nu);
    RowN<N> C = row_zero<N>();
    // leaf 1: U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
    RowN<N> t = mm_nn(load_row<N>(W, st, mu, r, i), load_row<N>(W, st, nu, r, ipm), gr);
    t = mm_nd(t, load_row<N>(W, st, mu, r, ipn), gr);
    t = mm_nd(t, load_row<N>(W, st, nu, r, i), gr);
    cx<double> z = leaf_phase<N>(c, mu, nu, g.n(mu), g.n(nu));
    row_axpy(C, z, t);
    rp += cmul(z, pick(t, r)).x;
    // leaf 2: U_nu(n-nu)^+ U_mu(n-nu) U_nu(n+mu-nu) U_mu(n)^+
    t = mm_dn(load_row<N>(W, st, nu, r, imn), load_row<N>(W, st, mu, r, imn), gr);
    t = mm_nn(t, load_row<N>(W, st, nu, r, imn + g.up(mu)), gr);
    t = mm_nd(t, load_row<N>(W, st, mu, r, i), gr);
    row_axpy(C, leaf_phase<N>(c, mu, nu, g.n(mu), g.back(nu)), t);
    // leaf 3: U_nu(n) U_mu(n+nu-mu)^+ U_nu(n-mu)^+ U_mu(n-mu)
    t = mm_nd(load_row<N>(W, st, nu, r, i), load_row<N>(W, st, mu, r, ipn + g.dn(mu)), gr);
    t = mm_nd(t, load_row<N>(W, st, nu, r, imm), gr);
    t = mm_nn(t, load_row<N>(W, st, mu, r, imm), gr);
    row_axpy(C, leaf_phase<N>(c, mu, nu, g.back(mu), g.n(nu)), t);
    // leaf 4: (U_nu(n-mu-nu) U_mu(n-mu))^+ U_mu(n-mu-nu) U_nu(n-nu)
    const int imm_mn = imm + g.dn(nu);
    t = mm_nn(load_row<N>(W, st, nu, r, imm_mn), load_row<N>(W, st, mu, r, imm), gr);
    t = mm_dn(t, load_row<N>(W, st, mu, r, imm_mn), gr);
    t = mm_nn(t, load_row<N>(W, st, nu, r, imn), gr);
    row_axpy(C, leaf_phase<N>(c, mu, nu, g.back(mu), g.back(nu)), t);
    // G = -(i/8)(C - C^+): row r of C - C^+ is C_r - conj(column r of C)
    const RowN<N> col = column(C, gr);
    RowN<N> G;
#pragma unroll
    for (int j = 0; j < N; j++) {
        const double wr = C.e[j].x - col.e[j].x, wi = C.e[j].y + col.e[j].y;
        G.e[j] = {0.125 * wi, -0.125 * wr};
    }
    return G;
}

template <int N>
__device__ __forceinline__ double herm_dot(const RowN<N> &a, const RowN<N> &b) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) s = fma(a.e[j].x, b.e[j].x, fma(a.e[j].y, b.e[j].y, s));
    return s;
}

// this lane's share of e(n), q(n), the plaquette sum and the action density:
// for Hermitian G, Tr(G_a G_b) = sum_{r,j} Re G_a,rj conj(G_b,rj), so every
// lane adds its row and the wave sum completes the traces
template <int N>
__device__ __forceinline__ void measure_site_n(gptr<const v2<double>> W, const CfgDesc &c,
                                               const Geo &g, const Grp &gr, double v[4]) {
    // the three dual plane pairs (01,23), (02,13), (03,12), one at a time
    double e = 0.0, q = 0.0, p = 0.0;
#pragma unroll 1
    for (int pr = 0; pr < 3; pr++) {
        const int a1 = pr + 1;                         // planes (0, a1) and (b0, b1)
        const int b0 = pr == 2 ? 1 : (pr == 1 ? 1 : 2);
        const int b1 = pr == 0 ? 3 : (pr == 1 ? 3 : 2);
        const RowN<N> Ga = clover_row<N>(W, c, g, gr, 0, a1, p);
        const RowN<N> Gb = clover_row<N>(W, c, g, gr, b0, b1, p);
        e += herm_dot(Ga, Ga) + herm_dot(Gb, Gb);
        const double d = herm_dot(Ga, Gb);
        q += pr == 1 ? -d : d;
    }
    v[0] += e;
    v[1] += q * 0.025330295910584444;   // 1 / (4 pi^2)
    v[2] += p;
    v[3] += 6.0 - p;   // each lane's share of sum_planes (N - Re Tr Z^* P)
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// work-group = one tile; wave w measures the tile's sites 16 w .. 16 w + 15,
// G at a time; the per-tile sums go to partials[tile][0], slots 1, 2 are zero
// (the layout of the SU(3) measurement, so the same reduction finishes it)
template <int N>
__global__ __launch_bounds__(256) void sun_measure_kernel(const CfgDesc *__restrict__ cfgs,
                                                          const int *__restrict__ tile_start,
                                                          int n_cfg, int n_tiles,
                                                          const MeasSlot *__restrict__ slots,
                                                          double *__restrict__ partials,
                                                          int buf_sel) {
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const int ci = find_cfg(tile_start, n_cfg, tile);
    if (slots[ci].row < 0) return;
    const CfgDesc c = cfgs[ci];
    const int sel = buf_sel < 0 ? c.cur : ((c.cur + buf_sel) & 1);
    gptr<const v2<double>> W = as_global<double>((const void *)(sel ? c.W[1] : c.W[0]));
    constexpr int G = 64 / N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / N;
    const Grp gr{g * N, lane - g * N};
    const int first = (tile - tile_start[ci]) * kTile + 16 * w;
    double v[4] = {0, 0, 0, 0};
    for (int s0 = 0; s0 < 16; s0 += G) {
        const int site = first + s0 + g;
        if (g >= G || s0 + g >= 16 || site >= c.V) continue;
        measure_site_n<N>(W, c, make_geo(c, site), gr, v);
    }
    __shared__ double red[4][4];
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = wave_sum_d(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; k++) red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 12) {
        const int slot = threadIdx.x >> 2, k = threadIdx.x & 3;
        double *o = partials + ((size_t)tile * 3 + slot) * 4 + k;
        *o = slot ? 0.0 : (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
}

// ---------------------------------------------------------------------------
// ingest / export / unitarity checks

// canonical [site][mu][N][N] <-> storage [mu][entry][site]; grid (sites, 4 N^2)
__global__ void sun_pack_kernel(const double2 *__restrict__ src, double2 *__restrict__ W, int V,
                                int stride, int nn) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const int me = blockIdx.y, mu = me / nn, e = me - mu * nn;
    W[(size_t)me * stride + i] = src[((size_t)i * 4 + mu) * nn + e];
}

__global__ void sun_unpack_kernel(const double2 *__restrict__ W, double2 *__restrict__ dst, int V,
                                  int stride, int nn) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const int me = blockIdx.y, mu = me / nn, e = me - mu * nn;
    dst[((size_t)i * 4 + mu) * nn + e] = W[(size_t)me * stride + i];
}

// max |U U^+ - 1| and |det U - 1| for one link held whole by one thread;
// the determinant by Gaussian elimination with partial pivoting
template <int N>
__device__ __forceinline__ void sun_defects(cx<double> (&a)[N][N], double &du, double &dd) {
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) {
            cx<double> s = {i == j ? -1.0 : 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < N; k++) s = cmadd_nc(s, a[i][k], a[j][k]);
            du = fmax(du, fmax(fabs(s.x), fabs(s.y)));
        }
    cx<double> det = {1.0, 0.0};
#pragma unroll
    for (int col = 0; col < N; col++) {
        int p = col;
        double best = a[col][col].x * a[col][col].x + a[col][col].y * a[col][col].y;
#pragma unroll
        for (int r = col + 1; r < N; r++) {
            const double m = a[r][col].x * a[r][col].x + a[r][col].y * a[r][col].y;
            if (m > best) { best = m; p = r; }
        }
#pragma unroll
        for (int r = col + 1; r < N; r++) {
            if (r == p) {
#pragma unroll
                for (int j = 0; j < N; j++) {
                    const cx<double> tmp = a[col][j];
                    a[col][j] = a[r][j];
                    a[r][j] = tmp;
                }
                det = {-det.x, -det.y};
            }
        }
        const cx<double> piv = a[col][col];
        det = cmul(det, piv);
        const double pn = piv.x * piv.x + piv.y * piv.y;
        if (!(pn > 0.0)) {
            det = {0.0, 0.0};
            break;
        }
        const cx<double> inv = {piv.x / pn, -piv.y / pn};
#pragma unroll
        for (int r = col + 1; r < N; r++) {
            const cx<double> f = cmul(a[r][col], inv);
#pragma unroll
            for (int j = col; j < N; j++) a[r][j] = cmadd(a[r][j], cx<double>{-f.x, -f.y}, a[col][j]);
        }
    }
    dd = fmax(dd, fmax(fabs(det.x - 1.0), fabs(det.y)));
    if (!(du <= 1e300) || !(dd <= 1e300)) { du = INFINITY; dd = INFINITY; }   // NaN input
}

// one thread per site (four links), partials[tile][2] as in the SU(3) check
template <int N, bool CANON>
__global__ __launch_bounds__(64) void sun_check_kernel(const void *__restrict__ src, int V,
                                                       int stride, double *__restrict__ partials) {
    const int tile = blockIdx.x;
    const int i = tile * kTile + (int)threadIdx.x;
    double du = 0, dd = 0;
    if (i < V) {
        for (int mu = 0; mu < 4; mu++) {
            cx<double> a[N][N];
            const double2 *s = (const double2 *)src;
#pragma unroll
            for (int r = 0; r < N; r++)
#pragma unroll
                for (int j = 0; j < N; j++) {
                    const double2 v = CANON ? s[((size_t)i * 4 + mu) * N * N + r * N + j]
                                            : s[((size_t)(mu * N * N + r * N + j)) * stride + i];
                    a[r][j] = {v.x, v.y};
                }
            sun_defects<N>(a, du, dd);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        du = fmax(du, __shfl_xor(du, off));
        dd = fmax(dd, __shfl_xor(dd, off));
    }
    if (threadIdx.x == 0) {
        partials[(size_t)tile * 2] = du;
        partials[(size_t)tile * 2 + 1] = dd;
    }
}

// ---------------------------------------------------------------------------
// launchers

template <int N>
static hipError_t stage_n(hipStream_t s, const SunStageArgs &a) {
    hipLaunchKernelGGL(sun_stage_kernel<N>, dim3(a.n_tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stage_sun(int nc, hipStream_t s, const CfgDesc *cfgs, const int *tile_start,
                            int n_act, int n_tiles, int step, int stage, double eps) {
    if (n_tiles <= 0) return hipSuccess;
    const SunStageArgs a{cfgs, tile_start, n_act, n_tiles, step, stage, eps};
    switch (nc) {
        case 2: return stage_n<2>(s, a);
        case 3: return stage_n<3>(s, a);
        case 4: return stage_n<4>(s, a);
        case 5: return stage_n<5>(s, a);
        case 6: return stage_n<6>(s, a);
        case 7: return stage_n<7>(s, a);
        case 8: return stage_n<8>(s, a);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t measure_n(hipStream_t s, const CfgDesc *cfgs, const int *tile_start, int n_cfg,
                            int n_tiles, const MeasSlot *slots, double *partials, int buf_sel) {
    hipLaunchKernelGGL(sun_measure_kernel<N>, dim3(n_tiles), dim3(256), 0, s, cfgs, tile_start,
                       n_cfg, n_tiles, slots, partials, buf_sel);
    return hipGetLastError();
}

hipError_t launch_measure_sun(int nc, hipStream_t s, const CfgDesc *cfgs, const int *tile_start,
                              int n_cfg, int n_tiles, const MeasSlot *slots, double *partials,
                              int buf_sel) {
    if (n_tiles <= 0) return hipSuccess;
    switch (nc) {
        case 2: return measure_n<2>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        case 3: return measure_n<3>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        case 4: return measure_n<4>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        case 5: return measure_n<5>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        case 6: return measure_n<6>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        case 7: return measure_n<7>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        case 8: return measure_n<8>(s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_sun(int nc, hipStream_t s, const void *src, void *W, int V, int stride) {
    const int nn = nc * nc;
    hipLaunchKernelGGL(sun_pack_kernel, dim3((V + 255) / 256, 4 * nn), dim3(256), 0, s,
                       (const double2 *)src, (double2 *)W, V, stride, nn);
    return hipGetLastError();
}

hipError_t launch_unpack_sun(int nc, hipStream_t s, const void *W, void *dst, int V, int stride) {
    const int nn = nc * nc;
    hipLaunchKernelGGL(sun_unpack_kernel, dim3((V + 255) / 256, 4 * nn), dim3(256), 0, s,
                       (const double2 *)W, (double2 *)dst, V, stride, nn);
    return hipGetLastError();
}

template <int N>
static hipError_t check_n(bool canon, hipStream_t s, const void *src, int V, int stride,
                          double *partials) {
    const int ntiles = (V + kTile - 1) / kTile;
    if (canon)
        hipLaunchKernelGGL((sun_check_kernel<N, true>), dim3(ntiles), dim3(64), 0, s, src, V,
                           stride, partials);
    else
        hipLaunchKernelGGL((sun_check_kernel<N, false>), dim3(ntiles), dim3(64), 0, s, src, V,
                           stride, partials);
    return hipGetLastError();
}

hipError_t launch_check_sun(int nc, bool canon, hipStream_t s, const void *src, int V, int stride,
                            double *partials, double *out) {
    hipError_t e;
    switch (nc) {
        case 2: e = check_n<2>(canon, s, src, V, stride, partials); break;
        case 3: e = check_n<3>(canon, s, src, V, stride, partials); break;
        case 4: e = check_n<4>(canon, s, src, V, stride, partials); break;
        case 5: e = check_n<5>(canon, s, src, V, stride, partials); break;
        case 6: e = check_n<6>(canon, s, src, V, stride, partials); break;
        case 7: e = check_n<7>(canon, s, src, V, stride, partials); break;
        case 8: e = check_n<8>(canon, s, src, V, stride, partials); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return launch_check_final(s, partials, (V + kTile - 1) / kTile, out);
}

}  // namespace tgf
