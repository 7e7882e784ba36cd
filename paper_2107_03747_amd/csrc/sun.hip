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
// Work decomposition ("R rows per lane"): the N x N matrix of a link is spread
// over L = N / R consecutive lanes of a wavefront, lane l holding rows
// l R .. l R + R - 1, so a wave holds G = floor(64 / L) links.  In a product
// C = A B every lane forms its own rows of C: its rows of A are local, the
// rows of B held by the other lanes of its group come through cross-lane
// permutes (ds_bpermute), each fetched entry then serving R multiply-adds.
// A^+ enters through the columns of A that a lane needs (gathered the same
// way).  R = N is one thread per link with no permutes; R = 1 keeps the
// fewest registers.  The choice is per context (the SU(N) variants).
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

// rows l R .. l R + R - 1 of an N x N matrix
template <int N, int R>
struct Blk {
    cx<double> e[R][N];
};

// this lane's place in its group of L = N / R lanes
struct Grp {
    int base;   // first lane of the group
    int l;      // index of this lane in the group
};

// global row index of local row i
template <int N, int R>
__device__ __forceinline__ int row_index(const Grp &g, int i) {
    return (N == R) ? i : g.l * R + i;
}

template <int N, int R>
__device__ __forceinline__ Blk<N, R> blk_zero() {
    Blk<N, R> o;
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < N; j++) o.e[i][j] = {0.0, 0.0};
    return o;
}

// the rows held by lane base + q of the group (the block itself when L = 1)
template <int N, int R>
__device__ __forceinline__ Blk<N, R> blk_from(const Blk<N, R> &m, const Grp &g, int q) {
    if constexpr (N == R) {
        return m;
    } else {
        Blk<N, R> o;
        const int src = g.base + q;
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < N; j++) {
                o.e[i][j].x = __shfl(m.e[i][j].x, src);
                o.e[i][j].y = __shfl(m.e[i][j].y, src);
            }
        return o;
    }
}

// entry r of a row for a lane-dependent r, by selection (no register indexing)
template <int N>
__device__ __forceinline__ cx<double> pick(const cx<double> (&row)[N], int r) {
    cx<double> v = row[0];
#pragma unroll
    for (int j = 1; j < N; j++)
        if (r == j) v = row[j];
    return v;
}

template <int N, int R>
__device__ __forceinline__ double group_sum(double v, const Grp &g) {
    if constexpr (N == R) {
        return v;
    } else {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < N / R; q++) s += __shfl(v, g.base + q);
        return s;
    }
}

// own rows of A B
template <int N, int R>
__device__ __forceinline__ Blk<N, R> mm_nn(const Blk<N, R> &a, const Blk<N, R> &b, const Grp &g) {
    Blk<N, R> c = blk_zero<N, R>();
#pragma unroll
    for (int q = 0; q < N / R; q++) {
        const Blk<N, R> bq = blk_from<N, R>(b, g, q);
#pragma unroll
        for (int kk = 0; kk < R; kk++)
#pragma unroll
            for (int i = 0; i < R; i++)
#pragma unroll
                for (int j = 0; j < N; j++)
                    c.e[i][j] = cmadd(c.e[i][j], a.e[i][q * R + kk], bq.e[kk][j]);
    }
    return c;
}

// own rows of A B^+: (A B^+)_{ij} = sum_k A_{ik} conj(B_{jk})
template <int N, int R>
__device__ __forceinline__ Blk<N, R> mm_nd(const Blk<N, R> &a, const Blk<N, R> &b, const Grp &g) {
    Blk<N, R> c;
#pragma unroll
    for (int q = 0; q < N / R; q++) {
        const Blk<N, R> bq = blk_from<N, R>(b, g, q);
#pragma unroll
        for (int jj = 0; jj < R; jj++)
#pragma unroll
            for (int i = 0; i < R; i++) {
                cx<double> s = {0.0, 0.0};
#pragma unroll
                for (int k = 0; k < N; k++) s = cmadd_nc(s, a.e[i][k], bq.e[jj][k]);
                c.e[i][q * R + jj] = s;
            }
    }
    return c;
}

// columns of A at the own row indices: col_{ik} = A_{k, row(i)}
template <int N, int R>
__device__ __forceinline__ Blk<N, R> column(const Blk<N, R> &a, const Grp &g) {
    Blk<N, R> col;
#pragma unroll
    for (int q = 0; q < N / R; q++) {
        const Blk<N, R> aq = blk_from<N, R>(a, g, q);
#pragma unroll
        for (int kk = 0; kk < R; kk++)
#pragma unroll
            for (int i = 0; i < R; i++) {
                if constexpr (N == R)
                    col.e[i][q * R + kk] = aq.e[kk][i];
                else
                    col.e[i][q * R + kk] = pick<N>(aq.e[kk], row_index<N, R>(g, i));
            }
    }
    return col;
}

// own rows of A^+ B: sum_k conj(A_{k, row(i)}) B_k
template <int N, int R>
__device__ __forceinline__ Blk<N, R> mm_dn(const Blk<N, R> &a, const Blk<N, R> &b, const Grp &g) {
    const Blk<N, R> col = column<N, R>(a, g);
    Blk<N, R> c = blk_zero<N, R>();
#pragma unroll
    for (int q = 0; q < N / R; q++) {
        const Blk<N, R> bq = blk_from<N, R>(b, g, q);
#pragma unroll
        for (int kk = 0; kk < R; kk++)
#pragma unroll
            for (int i = 0; i < R; i++)
#pragma unroll
                for (int j = 0; j < N; j++)
                    c.e[i][j] = cmadd_cn(c.e[i][j], col.e[i][q * R + kk], bq.e[kk][j]);
    }
    return c;
}

// The rows of S taken through an empty asm statement: what computes them is
// done before it, and no load or store moves across it.  Used as a fence
// between staples, so that the compiler does not load the links of later
// staples while earlier ones are still being formed.
template <int N, int R>
__device__ __forceinline__ void pin_blk(Blk<N, R> &S) {
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < N; j++) asm volatile("" : "+v"(S.e[i][j].x), "+v"(S.e[i][j].y)::"memory");
    __builtin_amdgcn_sched_barrier(0);
}

template <int N, int R>
__device__ __forceinline__ void blk_axpy(Blk<N, R> &y, cx<double> z, const Blk<N, R> &x) {
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < N; j++) y.e[i][j] = cmadd(y.e[i][j], z, x.e[i][j]);
}

// ---------------------------------------------------------------------------
// storage access: the own rows of link (mu, site); the plane of mu is a uniform
// base, the lane part a 32-bit byte offset (sites per configuration are capped
// so that the N^2 planes of one direction span less than 4 GiB)

template <int N>
__device__ __forceinline__ unsigned row_off(int r, int j, int stride, int site) {
    return ((unsigned)(r * N + j) * (unsigned)stride + (unsigned)site) * 16u;
}

// SGPR plane base + 32-bit lane offset for every access (sgpr_base,
// lane_here, no 64-bit per-lane address arithmetic) where it measured
// faster over a whole flow: (4,4) +31%, (6,2) +10%, (7,1) +3%; the other
// (N, rows per lane) builds ran up to 24% slower with it.
template <int N, int R>
constexpr bool sun_pin() {
    return (N == 4 && R == 4) || (N == 6 && R == 2) || (N == 7 && R == 1);
}

template <int N, int R>
__device__ __forceinline__ Blk<N, R> load_blk(gptr<const v2<double>> W, int stride, int mu,
                                              const Grp &g, int site) {
    gptr<const v2<double>> q = W + (size_t)(mu * N * N) * stride;
    Blk<N, R> o;
    if constexpr (sun_pin<N, R>()) {
        q = sgpr_base(q);
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < N; j++)
                o.e[i][j] = ld(q, lane_here(row_off<N>(row_index<N, R>(g, i), j, stride, site)));
    } else {
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < N; j++)
                o.e[i][j] = ld(q, row_off<N>(row_index<N, R>(g, i), j, stride, site));
    }
    return o;
}

template <int N, int R>
__device__ __forceinline__ void store_blk(gptr<v2<double>> W, int stride, int mu, const Grp &g,
                                          int site, const Blk<N, R> &v) {
    gptr<v2<double>> q = W + (size_t)(mu * N * N) * stride;
    if constexpr (sun_pin<N, R>()) {
        q = sgpr_base(q);
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < N; j++)
                st(q, lane_here(row_off<N>(row_index<N, R>(g, i), j, stride, site)), v.e[i][j]);
    } else {
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < N; j++)
                st(q, row_off<N>(row_index<N, R>(g, i), j, stride, site), v.e[i][j]);
    }
}

// twist exponent n_{mu nu} (mod N, antisymmetric) and Z = exp(2 pi i n / N)
template <int N>
__device__ __forceinline__ int tw_exp(const CfgDesc &c, int mu, int nu) {
    if (mu < nu) return c.tw[plane_index(mu, nu)];
    const int t = c.tw[plane_index(nu, mu)];
    return t ? N - t : 0;
}

// exp(2 pi i k / N) for N = 2..8, k = 0..N-1 as (cos, sin), the exact values
// rounded to double (evaluated to 60 digits; zeros and units exact).  A table
// read with a wave-uniform index keeps the trigonometric code, and the private
// memory its argument reduction uses, out of the flow kernels.
__constant__ double kTwistPhase[9][8][2] = {
    {  // unused
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // unused
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // N = 2
        {1.0, 0.0}, {-1.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // N = 3
        {1.0, 0.0}, {-0.5, 0.8660254037844386},
        {-0.5, -0.8660254037844386}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // N = 4
        {1.0, 0.0}, {0.0, 1.0},
        {-1.0, 0.0}, {0.0, -1.0},
        {0.0, 0.0}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // N = 5
        {1.0, 0.0}, {0.30901699437494745, 0.9510565162951535},
        {-0.8090169943749475, 0.5877852522924731}, {-0.8090169943749475, -0.5877852522924731},
        {0.30901699437494745, -0.9510565162951535}, {0.0, 0.0},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // N = 6
        {1.0, 0.0}, {0.5, 0.8660254037844386},
        {-0.5, 0.8660254037844386}, {-1.0, 0.0},
        {-0.5, -0.8660254037844386}, {0.5, -0.8660254037844386},
        {0.0, 0.0}, {0.0, 0.0},
    },
    {  // N = 7
        {1.0, 0.0}, {0.6234898018587335, 0.7818314824680298},
        {-0.2225209339563144, 0.9749279121818236}, {-0.9009688679024191, 0.4338837391175581},
        {-0.9009688679024191, -0.4338837391175581}, {-0.2225209339563144, -0.9749279121818236},
        {0.6234898018587335, -0.7818314824680298}, {0.0, 0.0},
    },
    {  // N = 8
        {1.0, 0.0}, {0.7071067811865476, 0.7071067811865476},
        {0.0, 1.0}, {-0.7071067811865476, 0.7071067811865476},
        {-1.0, 0.0}, {-0.7071067811865476, -0.7071067811865476},
        {0.0, -1.0}, {0.7071067811865476, -0.7071067811865476},
    },
};

template <int N>
__device__ __forceinline__ cx<double> zphase(int t) {
    return {kTwistPhase[N][t][0], kTwistPhase[N][t][1]};
}

// ---------------------------------------------------------------------------
// flow stage

// Omega_MU(n) = U_MU(n) S, S the twisted staple sum (upper staples times
// Z^*_{mu nu}(n), lower staples times Z_{mu nu}(n - nu))
template <int N, int R, int MU>
__device__ __forceinline__ Blk<N, R> omega_blk(gptr<const v2<double>> W, const CfgDesc &c,
                                               const Geo &g, const Grp &gr, Blk<N, R> &U) {
    const int st = c.stride;
    Blk<N, R> S = blk_zero<N, R>();
    auto add_staples = [&](int nu) {
        const int k = tw_exp<N>(c, MU, nu);
        // upper: U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
        Blk<N, R> t = mm_nd<N, R>(load_blk<N, R>(W, st, nu, gr, g.i + g.up(MU)),
                                  load_blk<N, R>(W, st, MU, gr, g.i + g.up(nu)), gr);
        t = mm_nd<N, R>(t, load_blk<N, R>(W, st, nu, gr, g.i), gr);
        cx<double> z = {1.0, 0.0};
        if (k && g.n(MU) == 0 && g.n(nu) == 0) z = cconj(zphase<N>(k));
        blk_axpy(S, z, t);
        pin_blk(S);
        // lower: (U_mu(n-nu) U_nu(n+mu-nu))^+ U_nu(n-nu)
        const int imn = g.i + g.dn(nu);
        t = mm_nn<N, R>(load_blk<N, R>(W, st, MU, gr, imn),
                        load_blk<N, R>(W, st, nu, gr, imn + g.up(MU)), gr);
        t = mm_dn<N, R>(t, load_blk<N, R>(W, st, nu, gr, imn), gr);
        z = {1.0, 0.0};
        if (k && g.n(MU) == 0 && g.back(nu) == 0) z = zphase<N>(k);
        blk_axpy(S, z, t);
        pin_blk(S);
    };
    if constexpr ((N == 3 && R == 1) || (N == 2 && R == 2)) {
#pragma unroll
        for (int nu = 0; nu < 4; nu++)
            if (nu != MU) add_staples(nu);
    } else {
        // one direction at a time: unrolled, the loads of all six staples are
        // live together and the larger blocks spill
#pragma unroll 1
        for (int nu = 0; nu < 4; nu++)
            if (nu != MU) add_staples(nu);
    }
    U = load_blk<N, R>(W, st, MU, gr, g.i);
    return mm_nn<N, R>(U, S, gr);
}

// scale * P_ah(M), own rows
template <int N, int R>
__device__ __forceinline__ Blk<N, R> proj_ah_blk(const Blk<N, R> &m, const Grp &g, double scale) {
    const Blk<N, R> col = column<N, R>(m, g);   // (M^+)_{ij} = conj(col_ij)
    Blk<N, R> a;
    double im = 0.0;
#pragma unroll
    for (int i = 0; i < R; i++) {
#pragma unroll
        for (int j = 0; j < N; j++)
            a.e[i][j] = {0.5 * (m.e[i][j].x - col.e[i][j].x), 0.5 * (m.e[i][j].y + col.e[i][j].y)};
        im += pick<N>(m.e[i], row_index<N, R>(g, i)).y;
    }
    // the diagonal of (M - M^+)/2 is i Im M_rr; remove the trace part
    const double t = group_sum<N, R>(im, g) / (double)N;
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < N; j++) {
            if (j == row_index<N, R>(g, i)) a.e[i][j].y -= t;
            a.e[i][j] = {scale * a.e[i][j].x, scale * a.e[i][j].y};
        }
    return a;
}

// exp(X) for X anti-Hermitian: scale so that ||Y||_F <= 1/4 (Y = X 2^-s),
// degree-12 Taylor polynomial by Horner's rule as T <- 1 + T Y / k (T is a
// polynomial in Y, so T Y = Y T), then s squarings.  Truncation error
// ||Y||^13 / 13! < 3e-18.
template <int N, int R>
__device__ __forceinline__ Blk<N, R> exp_blk(const Blk<N, R> &x, const Grp &g) {
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < N; j++)
            n2 = fma(x.e[i][j].x, x.e[i][j].x, fma(x.e[i][j].y, x.e[i][j].y, n2));
    const double nrm = sqrt(group_sum<N, R>(n2, g));
    int s = 0;
    if (nrm > 0.25) s = (int)ceil(log2(nrm * 4.0));
    const double f = ldexp(1.0, -s);
    constexpr int M = 12;
    Blk<N, R> y, t;
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < N; j++) {
            y.e[i][j] = {f * x.e[i][j].x, f * x.e[i][j].y};
            t.e[i][j] = {y.e[i][j].x * (1.0 / M), y.e[i][j].y * (1.0 / M)};
            if (j == row_index<N, R>(g, i)) t.e[i][j].x += 1.0;
        }
    for (int k = M - 1; k >= 1; k--) {
        const Blk<N, R> ty = mm_nn<N, R>(t, y, g);
        const double ik = 1.0 / (double)k;
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < N; j++) {
                t.e[i][j] = {ty.e[i][j].x * ik, ty.e[i][j].y * ik};
                if (j == row_index<N, R>(g, i)) t.e[i][j].x += 1.0;
            }
    }
    for (int i = 0; i < s; i++) t = mm_nn<N, R>(t, t, g);
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

template <int N, int R, int MU>
__device__ __forceinline__ void sun_link_update(const SunStageArgs &a, const CfgDesc &c, int site,
                                                const Grp &gr) {
    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    gptr<const v2<double>> W = as_global<double>((const void *)(in ? c.W[1] : c.W[0]));
    gptr<v2<double>> Wout = as_global<double>(in ? c.W[0] : c.W[1]);
    gptr<v2<double>> X = as_global<double>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const Geo g = make_geo(c, site);
    Blk<N, R> U;
    const Blk<N, R> om = omega_blk<N, R, MU>(W, c, g, gr, U);
    Blk<N, R> z = proj_ah_blk<N, R>(om, gr, -kSunRkB[a.stage] * eps);   // B eps F, F = -P_ah(Omega)
    if (a.stage > 0) {
        const Blk<N, R> xo = load_blk<N, R>(X, c.stride, MU, gr, site);
        blk_axpy(z, cx<double>{kSunRkA[a.stage], 0.0}, xo);
    }
    if (a.stage < 2) store_blk<N, R>(X, c.stride, MU, gr, site, z);
    const Blk<N, R> e = exp_blk<N, R>(z, gr);
    store_blk<N, R>(Wout, c.stride, MU, gr, site, mm_nn<N, R>(e, U, gr));
}

// work-group = one tile of 64 sites; wave w updates direction w for the
// tile's sites, G = 64 / L at a time (lane = g L + l)
template <int N, int R>
__global__ __launch_bounds__(256) void sun_stage_kernel(SunStageArgs a) {
    const int tile = blockIdx.x;
    if (tile >= a.n_tiles) return;
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc &c = a.cfgs[ci];   // in global memory: the twist entries are read with run-time indices
    constexpr int L = N / R, G = 64 / L;
    const int lane = threadIdx.x & 63;
    const int g = lane / L;
    const Grp gr{g * L, lane - g * L};
    const int first = (tile - a.tile_start[ci]) * kTile;
    for (int s0 = 0; s0 < kTile; s0 += G) {
        const int site = first + s0 + g;
        if (g >= G || s0 + g >= kTile || site >= c.V) continue;
        switch (mu) {
            case 0: sun_link_update<N, R, 0>(a, c, site, gr); break;
            case 1: sun_link_update<N, R, 1>(a, c, site, gr); break;
            case 2: sun_link_update<N, R, 2>(a, c, site, gr); break;
            default: sun_link_update<N, R, 3>(a, c, site, gr); break;
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

// own rows of G_{mu nu}(n); rp += Re of this lane's diagonal entries of Z^* P_{mu nu}(n)
template <int N, int R>
__device__ __forceinline__ Blk<N, R> clover_blk(gptr<const v2<double>> W, const CfgDesc &c,
                                                const Geo &g, const Grp &gr, int mu, int nu,
                                                double &rp) {
    const int st = c.stride;
    const int i = g.i, ipm = g.i + g.up(mu), ipn = g.i + g.up(nu);
    const int imm = g.i + g.dn(mu), imn = g.i + g.dn(nu);
    Blk<N, R> C = blk_zero<N, R>();
    // leaf 1: U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
    Blk<N, R> t = mm_nn<N, R>(load_blk<N, R>(W, st, mu, gr, i), load_blk<N, R>(W, st, nu, gr, ipm), gr);
    t = mm_nd<N, R>(t, load_blk<N, R>(W, st, mu, gr, ipn), gr);
    t = mm_nd<N, R>(t, load_blk<N, R>(W, st, nu, gr, i), gr);
    const cx<double> z = leaf_phase<N>(c, mu, nu, g.n(mu), g.n(nu));
    blk_axpy(C, z, t);
    pin_blk(C);
#pragma unroll
    for (int r = 0; r < R; r++) rp += cmul(z, pick<N>(t.e[r], row_index<N, R>(gr, r))).x;
    // leaf 2: U_nu(n-nu)^+ U_mu(n-nu) U_nu(n+mu-nu) U_mu(n)^+
    t = mm_dn<N, R>(load_blk<N, R>(W, st, nu, gr, imn), load_blk<N, R>(W, st, mu, gr, imn), gr);
    t = mm_nn<N, R>(t, load_blk<N, R>(W, st, nu, gr, imn + g.up(mu)), gr);
    t = mm_nd<N, R>(t, load_blk<N, R>(W, st, mu, gr, i), gr);
    blk_axpy(C, leaf_phase<N>(c, mu, nu, g.n(mu), g.back(nu)), t);
    pin_blk(C);
    // leaf 3: U_nu(n) U_mu(n+nu-mu)^+ U_nu(n-mu)^+ U_mu(n-mu)
    t = mm_nd<N, R>(load_blk<N, R>(W, st, nu, gr, i), load_blk<N, R>(W, st, mu, gr, ipn + g.dn(mu)), gr);
    t = mm_nd<N, R>(t, load_blk<N, R>(W, st, nu, gr, imm), gr);
    t = mm_nn<N, R>(t, load_blk<N, R>(W, st, mu, gr, imm), gr);
    blk_axpy(C, leaf_phase<N>(c, mu, nu, g.back(mu), g.n(nu)), t);
    pin_blk(C);
    // leaf 4: (U_nu(n-mu-nu) U_mu(n-mu))^+ U_mu(n-mu-nu) U_nu(n-nu)
    const int imm_mn = imm + g.dn(nu);
    t = mm_nn<N, R>(load_blk<N, R>(W, st, nu, gr, imm_mn), load_blk<N, R>(W, st, mu, gr, imm), gr);
    t = mm_dn<N, R>(t, load_blk<N, R>(W, st, mu, gr, imm_mn), gr);
    t = mm_nn<N, R>(t, load_blk<N, R>(W, st, nu, gr, imn), gr);
    blk_axpy(C, leaf_phase<N>(c, mu, nu, g.back(mu), g.back(nu)), t);
    pin_blk(C);
    // G = -(i/8)(C - C^+): own rows of C - C^+ are C_i - conj(column i of C)
    const Blk<N, R> col = column<N, R>(C, gr);
    Blk<N, R> G;
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int j = 0; j < N; j++) {
            const double wr = C.e[r][j].x - col.e[r][j].x, wi = C.e[r][j].y + col.e[r][j].y;
            G.e[r][j] = {0.125 * wi, -0.125 * wr};
        }
    return G;
}

template <int N, int R>
__device__ __forceinline__ double herm_dot(const Blk<N, R> &a, const Blk<N, R> &b) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int j = 0; j < N; j++) s = fma(a.e[r][j].x, b.e[r][j].x, fma(a.e[r][j].y, b.e[r][j].y, s));
    return s;
}

// this lane's share of e(n), q(n), the plaquette sum and the action density:
// for Hermitian G, Tr(G_a G_b) = sum_{r,j} Re G_a,rj conj(G_b,rj), so every
// lane adds its rows and the wave sum completes the traces
template <int N, int R>
__device__ __forceinline__ void measure_site_n(gptr<const v2<double>> W, const CfgDesc &c,
                                               const Geo &g, const Grp &gr, double v[4]) {
    // the three dual plane pairs (01,23), (02,13), (03,12), one at a time
    double e = 0.0, q = 0.0, p = 0.0;
#pragma unroll 1
    for (int pr = 0; pr < 3; pr++) {
        const int a1 = pr + 1;                         // planes (0, a1) and (b0, b1)
        const int b0 = pr == 2 ? 1 : (pr == 1 ? 1 : 2);
        const int b1 = pr == 0 ? 3 : (pr == 1 ? 3 : 2);
        const Blk<N, R> Ga = clover_blk<N, R>(W, c, g, gr, 0, a1, p);
        const Blk<N, R> Gb = clover_blk<N, R>(W, c, g, gr, b0, b1, p);
        e += herm_dot(Ga, Ga) + herm_dot(Gb, Gb);
        const double d = herm_dot(Ga, Gb);
        q += pr == 1 ? -d : d;
    }
    v[0] += e;
    v[1] += q * 0.025330295910584444;   // 1 / (4 pi^2)
    v[2] += p;
    v[3] += 6.0 * R - p;   // this lane's share of sum_planes (N - Re Tr Z^* P)
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// work-group = one tile of WPB waves; wave w measures the tile's sites
// SPW w .. SPW w + SPW - 1, G at a time (G = 64 / (N/R) sites fill a wave, so
// one wave per tile when a lane holds a whole link, two when it holds half);
// the per-tile sums go to partials[tile][0], slots 1, 2 are zero (the layout
// of the SU(3) measurement, so the same reduction finishes it)
template <int N, int R>
struct MeasShape {
    static constexpr int G = 64 / (N / R);
    static constexpr int WPB = G >= 64 ? 1 : (G >= 32 ? 2 : 4);
    static constexpr int SPW = 64 / WPB;
};

template <int N, int R>
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
    const CfgDesc &c = cfgs[ci];     // in global memory: the twist entries are read with run-time indices
    const int sel = buf_sel < 0 ? c.cur : ((c.cur + buf_sel) & 1);
    gptr<const v2<double>> W = as_global<double>((const void *)(sel ? c.W[1] : c.W[0]));
    constexpr int L = N / R, G = MeasShape<N, R>::G, SPW = MeasShape<N, R>::SPW;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / L;
    const Grp gr{g * L, lane - g * L};
    const int first = (tile - tile_start[ci]) * kTile + SPW * w;
    double v[4] = {0, 0, 0, 0};
    for (int s0 = 0; s0 < SPW; s0 += G) {
        const int site = first + s0 + g;
        if (g >= G || s0 + g >= SPW || site >= c.V) continue;
        measure_site_n<N, R>(W, c, make_geo(c, site), gr, v);
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
        constexpr int WPB = MeasShape<N, R>::WPB;
        const double t = WPB == 1 ? red[0][k]
                       : WPB == 2 ? red[0][k] + red[1][k]
                                  : (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
        *o = slot ? 0.0 : t;
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
// LDS-operand variant.  One row per lane (a link over N consecutive lanes,
// G = 64 / N links per wave), and the right operand of every product is read
// from an LDS slot of the wave that the owning lanes have filled with their
// rows: one 16-byte LDS read per complex multiply-add, against four 4-byte
// cross-lane permutes in the permute variants, and the products run as short
// loops over rows of the operand, so no link matrix is held whole in
// registers.  Each wave owns two slots of G padded link matrices (one complex
// of padding per link puts the G links of a read in different banks).  LDS
// operations of a wave execute in order, so a slot written by a wave is read
// by the same wave without a barrier; the fences below only keep the compiler
// from moving accesses and arithmetic across a fill or a row of a product.

template <int N>
struct LdsShape {
    static constexpr int G = 64 / N;         // links per wave
    static constexpr int LS = N * N + 1;     // complex per link in a slot
    static constexpr int SLOT = G * LS;      // complex per slot
};

template <int N>
struct Row {
    cx<double> e[N];
};

template <int N>
__device__ __forceinline__ Row<N> row_zero() {
    Row<N> o;
#pragma unroll
    for (int j = 0; j < N; j++) o.e[j] = {0.0, 0.0};
    return o;
}

// this lane's row r of its link g: s[0], s[1] the link's matrices in the two slots
template <int N>
struct LaneRow {
    v2<double> *s[2];
    int r;
    int base;   // first lane of the link
};

// Compiler fences.  The products end each row of their operand with one that
// takes the accumulators through an empty asm statement: the arithmetic of
// that row is then done before it, and no load or store moves across it
// (neither in the IR passes nor in the scheduler).  Without them the compiler
// reads a whole operand matrix before the first multiply-add, which holds it
// in registers and spills.
__device__ __forceinline__ void lds_fence() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}
__device__ __forceinline__ void pin(cx<double> &z) {
    asm volatile("" : "+v"(z.x), "+v"(z.y)::"memory");
}
// entry r of a row for this lane's row index r, by selection; the empty asm
// per step keeps the compiler from turning the selection into an indexed
// load from a private copy of the row
template <int N>
__device__ __forceinline__ cx<double> own_entry(const Row<N> &a, int r) {
    cx<double> v = a.e[0];
#pragma unroll
    for (int j = 1; j < N; j++) {
        if (r == j) v = a.e[j];
        asm volatile("" : "+v"(v.x), "+v"(v.y));
    }
    return v;
}

template <int N>
__device__ __forceinline__ void pin_row(Row<N> &c) {
#pragma unroll
    for (int j = 0; j < N; j++) pin(c.e[j]);
    __builtin_amdgcn_sched_barrier(0);
}

// Fill slot k with the own rows.
template <int N>
__device__ __forceinline__ void put(const LaneRow<N> &q, int k, const Row<N> &a) {
    lds_fence();
#pragma unroll
    for (int j = 0; j < N; j++) q.s[k][q.r * N + j] = v2<double>{a.e[j].x, a.e[j].y};
    __builtin_amdgcn_wave_barrier();
    lds_fence();
}

template <int N>
__device__ __forceinline__ cx<double> got(const LaneRow<N> &q, int k, int i, int j) {
    const v2<double> v = q.s[k][i * N + j];
    return {v.x, v.y};
}

// own row of A B, B in slot k
template <int N>
__device__ __forceinline__ Row<N> lmm_nn(const Row<N> &a, const LaneRow<N> &q, int k) {
    Row<N> c = row_zero<N>();
#pragma unroll
    for (int m = 0; m < N; m++) {
#pragma unroll
        for (int j = 0; j < N; j++) c.e[j] = cmadd(c.e[j], a.e[m], got(q, k, m, j));
        pin_row(c);   // one operand row in registers at a time
    }
    return c;
}

// own row of A^+ B with A in slot ka and B in slot kb: sum_m conj(A_{m r}) B_m
template <int N>
__device__ __forceinline__ Row<N> lmm_dn(const LaneRow<N> &q, int ka, int kb) {
    Row<N> c = row_zero<N>();
#pragma unroll
    for (int m = 0; m < N; m++) {
        const cx<double> am = got(q, ka, m, q.r);
#pragma unroll
        for (int j = 0; j < N; j++) c.e[j] = cmadd_cn(c.e[j], am, got(q, kb, m, j));
        pin_row(c);
    }
    return c;
}

// own row of A B^+, B in slot k: sum_m A_m conj(B_{j m})
template <int N>
__device__ __forceinline__ Row<N> lmm_nd(const Row<N> &a, const LaneRow<N> &q, int k) {
    Row<N> c;
#pragma unroll
    for (int j = 0; j < N; j++) {
        cx<double> t = {0.0, 0.0};
#pragma unroll
        for (int m = 0; m < N; m++) t = cmadd_nc(t, a.e[m], got(q, k, j, m));
        pin(t);
        __builtin_amdgcn_sched_barrier(0);
        c.e[j] = t;
    }
    return c;
}

template <int N>
__device__ __forceinline__ double link_sum(double v, const LaneRow<N> &q) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < N; l++) s += __shfl(v, q.base + l);
    return s;
}

template <int N>
__device__ __forceinline__ Row<N> load_row(gptr<const v2<double>> W, int stride, int mu, int r,
                                           int site) {
    gptr<const v2<double>> p = W + (size_t)(mu * N * N) * stride;
    Row<N> o;
#pragma unroll
    for (int j = 0; j < N; j++) o.e[j] = ld(p, row_off<N>(r, j, stride, site));
    return o;
}

template <int N>
__device__ __forceinline__ void store_row(gptr<v2<double>> W, int stride, int mu, int r, int site,
                                          const Row<N> &v) {
    gptr<v2<double>> p = W + (size_t)(mu * N * N) * stride;
#pragma unroll
    for (int j = 0; j < N; j++) st(p, row_off<N>(r, j, stride, site), v.e[j]);
}

template <int N>
__device__ __forceinline__ void row_axpy(Row<N> &y, cx<double> z, const Row<N> &x) {
#pragma unroll
    for (int j = 0; j < N; j++) y.e[j] = cmadd(y.e[j], z, x.e[j]);
}

// own row of Omega_MU(n) = U_MU(n) S (as omega_blk); U gets the own row of
// U_MU(n).  Upper and lower staples in two loops over nu: in one loop body the
// compiler interleaves their loads and products and runs out of registers.
template <int N>
__device__ __forceinline__ Row<N> omega_row(gptr<const v2<double>> W, const CfgDesc &c,
                                            const Geo &g, const LaneRow<N> &q, int mu,
                                            Row<N> &U) {
    const int st = c.stride, r = q.r;
    Row<N> S = row_zero<N>();
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        // upper: U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+, times Z^*_{mu nu}(n)
        put(q, 1, load_row<N>(W, st, mu, r, g.i + g.up(nu)));
        Row<N> t = lmm_nd<N>(load_row<N>(W, st, nu, r, g.i + g.up(mu)), q, 1);
        put(q, 1, load_row<N>(W, st, nu, r, g.i));
        t = lmm_nd<N>(t, q, 1);
        const int k = tw_exp<N>(c, mu, nu);
        cx<double> z = {1.0, 0.0};
        if (k && g.n(mu) == 0 && g.n(nu) == 0) z = cconj(zphase<N>(k));
        row_axpy(S, z, t);
    }
#pragma unroll 1
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        // lower: (U_mu(n-nu) U_nu(n+mu-nu))^+ U_nu(n-nu), times Z_{mu nu}(n-nu)
        const int imn = g.i + g.dn(nu);
        put(q, 1, load_row<N>(W, st, nu, r, imn + g.up(mu)));
        Row<N> t = lmm_nn<N>(load_row<N>(W, st, mu, r, imn), q, 1);
        put(q, 0, t);
        put(q, 1, load_row<N>(W, st, nu, r, imn));
        t = lmm_dn<N>(q, 0, 1);
        const int k = tw_exp<N>(c, mu, nu);
        cx<double> z = {1.0, 0.0};
        if (k && g.n(mu) == 0 && g.back(nu) == 0) z = zphase<N>(k);
        row_axpy(S, z, t);
    }
    U = load_row<N>(W, st, mu, r, g.i);
    put(q, 1, S);
    return lmm_nn<N>(U, q, 1);
}

// scale * P_ah(M), own row (M's rows are put in slot 0)
template <int N>
__device__ __forceinline__ Row<N> proj_ah_row(const Row<N> &m, const LaneRow<N> &q, double scale) {
    put(q, 0, m);
    Row<N> a;
#pragma unroll
    for (int j = 0; j < N; j++) {
        const cx<double> mj = got(q, 0, j, q.r);           // M_{j r}
        a.e[j] = {0.5 * (m.e[j].x - mj.x), 0.5 * (m.e[j].y + mj.y)};
    }
    const double t = link_sum<N>(got(q, 0, q.r, q.r).y, q) / (double)N;   // Im M_rr
#pragma unroll
    for (int j = 0; j < N; j++) {
        if (j == q.r) a.e[j].y -= t;
        a.e[j] = {scale * a.e[j].x, scale * a.e[j].y};
    }
    return a;
}

// exp(X), X anti-Hermitian: the scaling, degree and squarings of exp_blk; the
// scaled argument Y stays in slot 0 for the whole Horner loop
template <int N>
__device__ __forceinline__ Row<N> exp_row(const Row<N> &x, const LaneRow<N> &q) {
    double n2 = 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) n2 = fma(x.e[j].x, x.e[j].x, fma(x.e[j].y, x.e[j].y, n2));
    const double nrm = sqrt(link_sum<N>(n2, q));
    int s = 0;
    if (nrm > 0.25) s = (int)ceil(log2(nrm * 4.0));
    const double f = ldexp(1.0, -s);
    constexpr int M = 12;
    Row<N> y, t;
#pragma unroll
    for (int j = 0; j < N; j++) {
        y.e[j] = {f * x.e[j].x, f * x.e[j].y};
        t.e[j] = {y.e[j].x * (1.0 / M), y.e[j].y * (1.0 / M)};
        if (j == q.r) t.e[j].x += 1.0;
    }
    put(q, 0, y);
    for (int k = M - 1; k >= 1; k--) {
        const Row<N> ty = lmm_nn<N>(t, q, 0);
        const double ik = 1.0 / (double)k;
#pragma unroll
        for (int j = 0; j < N; j++) {
            t.e[j] = {ty.e[j].x * ik, ty.e[j].y * ik};
            if (j == q.r) t.e[j].x += 1.0;
        }
    }
    for (int i = 0; i < s; i++) {
        put(q, 1, t);
        t = lmm_nn<N>(t, q, 1);
    }
    return t;
}

template <int N>
__device__ __forceinline__ void sun_link_update_lds(const SunStageArgs &a, const CfgDesc &c,
                                                    int site, int mu, const LaneRow<N> &q) {
    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    gptr<const v2<double>> W = as_global<double>((const void *)(in ? c.W[1] : c.W[0]));
    gptr<v2<double>> Wout = as_global<double>(in ? c.W[0] : c.W[1]);
    gptr<v2<double>> X = as_global<double>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const Geo g = make_geo(c, site);
    Row<N> U;
    const Row<N> om = omega_row<N>(W, c, g, q, mu, U);
    Row<N> z = proj_ah_row<N>(om, q, -kSunRkB[a.stage] * eps);   // B eps F, F = -P_ah(Omega)
    if (a.stage > 0) {
        const Row<N> xo = load_row<N>(X, c.stride, mu, q.r, site);
        row_axpy(z, cx<double>{kSunRkA[a.stage], 0.0}, xo);
    }
    if (a.stage < 2) store_row<N>(X, c.stride, mu, q.r, site, z);
    const Row<N> e = exp_row<N>(z, q);
    put(q, 1, U);
    store_row<N>(Wout, c.stride, mu, q.r, site, lmm_nn<N>(e, q, 1));
}

// work-group = one tile of 64 sites; wave w updates direction w for the
// tile's sites, G at a time (lane = g N + r)
template <int N>
__global__ __launch_bounds__(256) void sun_stage_lds_kernel(SunStageArgs a) {
    constexpr int G = LdsShape<N>::G, SLOT = LdsShape<N>::SLOT, LS = LdsShape<N>::LS;
    __shared__ v2<double> lds[4][2][SLOT];
    const int tile = blockIdx.x;
    if (tile >= a.n_tiles) return;
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc &c = a.cfgs[ci];   // in global memory: the twist entries are read with run-time indices
    const int lane = threadIdx.x & 63;
    const int g = lane / N;
    if (g >= G) return;                      // lanes past the last whole link
    const LaneRow<N> q{{&lds[mu][0][g * LS], &lds[mu][1][g * LS]}, lane - g * N, g * N};
    const int first = (tile - a.tile_start[ci]) * kTile;
#pragma unroll 1
    for (int s0 = 0; s0 < kTile; s0 += G) {
        const int site = first + s0 + g;
        if (s0 + g >= kTile || site >= c.V) continue;
        sun_link_update_lds<N>(a, c, site, mu, q);
    }
}

// measurement: own row of G_{mu nu}(n) (as clover_blk)
template <int N>
__device__ __forceinline__ Row<N> clover_row(gptr<const v2<double>> W, const CfgDesc &c,
                                             const Geo &g, const LaneRow<N> &q, int mu, int nu,
                                             double &rp) {
    const int st = c.stride, r = q.r;
    const int i = g.i, ipm = g.i + g.up(mu), ipn = g.i + g.up(nu);
    const int imm = g.i + g.dn(mu), imn = g.i + g.dn(nu);
    Row<N> C = row_zero<N>();
    // leaf 1: U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
    put(q, 1, load_row<N>(W, st, nu, r, ipm));
    Row<N> t = lmm_nn<N>(load_row<N>(W, st, mu, r, i), q, 1);
    put(q, 1, load_row<N>(W, st, mu, r, ipn));
    t = lmm_nd<N>(t, q, 1);
    put(q, 1, load_row<N>(W, st, nu, r, i));
    t = lmm_nd<N>(t, q, 1);
    const cx<double> z = leaf_phase<N>(c, mu, nu, g.n(mu), g.n(nu));
    row_axpy(C, z, t);
    pin_row(C);
    rp += cmul(z, own_entry<N>(t, r)).x;
    // leaf 2: U_nu(n-nu)^+ U_mu(n-nu) U_nu(n+mu-nu) U_mu(n)^+
    put(q, 0, load_row<N>(W, st, nu, r, imn));
    put(q, 1, load_row<N>(W, st, mu, r, imn));
    t = lmm_dn<N>(q, 0, 1);
    put(q, 1, load_row<N>(W, st, nu, r, imn + g.up(mu)));
    t = lmm_nn<N>(t, q, 1);
    put(q, 1, load_row<N>(W, st, mu, r, i));
    t = lmm_nd<N>(t, q, 1);
    row_axpy(C, leaf_phase<N>(c, mu, nu, g.n(mu), g.back(nu)), t);
    pin_row(C);
    // leaf 3: U_nu(n) U_mu(n+nu-mu)^+ U_nu(n-mu)^+ U_mu(n-mu)
    put(q, 1, load_row<N>(W, st, mu, r, ipn + g.dn(mu)));
    t = lmm_nd<N>(load_row<N>(W, st, nu, r, i), q, 1);
    put(q, 1, load_row<N>(W, st, nu, r, imm));
    t = lmm_nd<N>(t, q, 1);
    put(q, 1, load_row<N>(W, st, mu, r, imm));
    t = lmm_nn<N>(t, q, 1);
    row_axpy(C, leaf_phase<N>(c, mu, nu, g.back(mu), g.n(nu)), t);
    pin_row(C);
    // leaf 4: (U_nu(n-mu-nu) U_mu(n-mu))^+ U_mu(n-mu-nu) U_nu(n-nu)
    const int imm_mn = imm + g.dn(nu);
    put(q, 1, load_row<N>(W, st, mu, r, imm));
    t = lmm_nn<N>(load_row<N>(W, st, nu, r, imm_mn), q, 1);
    put(q, 0, t);
    put(q, 1, load_row<N>(W, st, mu, r, imm_mn));
    t = lmm_dn<N>(q, 0, 1);
    put(q, 1, load_row<N>(W, st, nu, r, imn));
    t = lmm_nn<N>(t, q, 1);
    row_axpy(C, leaf_phase<N>(c, mu, nu, g.back(mu), g.back(nu)), t);
    pin_row(C);
    // G = -(i/8)(C - C^+): own row of C - C^+ is C_r - conj(column r of C)
    put(q, 0, C);
    Row<N> Gr;
#pragma unroll
    for (int j = 0; j < N; j++) {
        const cx<double> cj = got(q, 0, j, r);             // C_{j r}
        const double wr = C.e[j].x - cj.x, wi = C.e[j].y + cj.y;
        Gr.e[j] = {0.125 * wi, -0.125 * wr};
    }
    return Gr;
}

template <int N>
__device__ __forceinline__ double row_dot(const Row<N> &a, const Row<N> &b) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < N; j++) s = fma(a.e[j].x, b.e[j].x, fma(a.e[j].y, b.e[j].y, s));
    return s;
}

// this lane's share of e(n), q(n), the plaquette sum and the action density
// (as measure_site_n)
template <int N>
__device__ __forceinline__ void measure_site_lds(gptr<const v2<double>> W, const CfgDesc &c,
                                                 const Geo &g, const LaneRow<N> &q, double v[4]) {
    double e = 0.0, qq = 0.0, p = 0.0;
#pragma unroll 1
    for (int pr = 0; pr < 3; pr++) {
        const int a1 = pr + 1;
        const int b0 = pr == 2 ? 1 : (pr == 1 ? 1 : 2);
        const int b1 = pr == 0 ? 3 : (pr == 1 ? 3 : 2);
        const Row<N> Ga = clover_row<N>(W, c, g, q, 0, a1, p);
        const Row<N> Gb = clover_row<N>(W, c, g, q, b0, b1, p);
        e += row_dot(Ga, Ga) + row_dot(Gb, Gb);
        const double d = row_dot(Ga, Gb);
        qq += pr == 1 ? -d : d;
    }
    v[0] += e;
    v[1] += qq * 0.025330295910584444;   // 1 / (4 pi^2)
    v[2] += p;
    v[3] += 6.0 - p;
}

template <int N>
__global__ __launch_bounds__(256) void sun_measure_lds_kernel(const CfgDesc *__restrict__ cfgs,
                                                              const int *__restrict__ tile_start,
                                                              int n_cfg, int n_tiles,
                                                              const MeasSlot *__restrict__ slots,
                                                              double *__restrict__ partials,
                                                              int buf_sel) {
    constexpr int G = LdsShape<N>::G, SLOT = LdsShape<N>::SLOT, LS = LdsShape<N>::LS;
    constexpr int WPB = MeasShape<N, 1>::WPB, SPW = MeasShape<N, 1>::SPW;
    __shared__ v2<double> lds[WPB][2][SLOT];
    __shared__ double red[4][4];
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const int ci = find_cfg(tile_start, n_cfg, tile);
    if (slots[ci].row < 0) return;
    const CfgDesc &c = cfgs[ci];     // in global memory: the twist entries are read with run-time indices
    const int sel = buf_sel < 0 ? c.cur : ((c.cur + buf_sel) & 1);
    gptr<const v2<double>> W = as_global<double>((const void *)(sel ? c.W[1] : c.W[0]));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / N;
    const int gg = g < G ? g : 0;            // lanes past the last link: no slot
    const LaneRow<N> q{{&lds[w][0][gg * LS], &lds[w][1][gg * LS]}, lane - g * N, g * N};
    const int first = (tile - tile_start[ci]) * kTile + SPW * w;
    double v[4] = {0, 0, 0, 0};
    if (g < G) {
        for (int s0 = 0; s0 < SPW; s0 += G) {
            const int site = first + s0 + g;
            if (s0 + g >= SPW || site >= c.V) continue;
            measure_site_lds<N>(W, c, make_geo(c, site), q, v);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = wave_sum_d(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; k++) red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 12) {
        const int slot = threadIdx.x >> 2, k = threadIdx.x & 3;
        double *o = partials + ((size_t)tile * 3 + slot) * 4 + k;
        const double t = WPB == 1 ? red[0][k]
                       : WPB == 2 ? red[0][k] + red[1][k]
                                  : (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
        *o = slot ? 0.0 : t;
    }
}

// ---------------------------------------------------------------------------
// launchers.  The variants of each N in order (variant 0 is the default):
// the first entry is the fastest measured on the benchmark boxes (about 10^6
// sites of 4x4x4Nx4N, stage launch): one thread per link for N = 2..4, the
// LDS-operand variant from N = 5 (3.1x to 8.1x the permute variants there).

// Variant table: rows per lane of the permute variants, or kLds for the
// LDS-operand variant (one row per lane).
constexpr int kLds = 16;

__host__ __device__ constexpr int sun_code(int nc, int v) {
    // N = 2: 2, 1, LDS    3: 3, 1, LDS    4: 4, 2, 1, LDS    5, 7, 8: LDS, 1    6: LDS, 2, 1
    return nc == 2 ? (v == 0 ? 2 : (v == 1 ? 1 : kLds))
         : nc == 3 ? (v == 0 ? 3 : (v == 1 ? 1 : kLds))
         : nc == 4 ? (v == 0 ? 4 : (v == 1 ? 2 : (v == 2 ? 1 : kLds)))
         : nc == 6 ? (v == 0 ? kLds : (v == 1 ? 2 : 1))
         : (v == 0 ? kLds : 1);
}

int sun_variant_count(int nc) {
    switch (nc) {
        case 2: case 3: case 6: return 3;
        case 4: return 4;
        case 5: case 7: case 8: return 2;
        default: return 0;
    }
}

int sun_rows_per_lane(int nc, int v) {
    if (v < 0) v = 0;
    if (v >= sun_variant_count(nc)) return 0;
    const int code = sun_code(nc, v);
    return code == kLds ? 1 : code;
}

int sun_variant_lds(int nc, int v) {
    if (v < 0) v = 0;
    if (v >= sun_variant_count(nc)) return -1;
    return sun_code(nc, v) == kLds ? 1 : 0;
}

template <int N, int R>
static hipError_t stage_nr(hipStream_t s, const SunStageArgs &a) {
    if constexpr (R == kLds)
        hipLaunchKernelGGL((sun_stage_lds_kernel<N>), dim3(a.n_tiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((sun_stage_kernel<N, R>), dim3(a.n_tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int N, int R>
static hipError_t measure_nr(hipStream_t s, const CfgDesc *cfgs, const int *tile_start, int n_cfg,
                             int n_tiles, const MeasSlot *slots, double *partials, int buf_sel) {
    if constexpr (R == kLds)
        hipLaunchKernelGGL((sun_measure_lds_kernel<N>), dim3(n_tiles),
                           dim3(64 * MeasShape<N, 1>::WPB), 0, s, cfgs, tile_start, n_cfg, n_tiles,
                           slots, partials, buf_sel);
    else
        hipLaunchKernelGGL((sun_measure_kernel<N, R>), dim3(n_tiles),
                           dim3(64 * MeasShape<N, R>::WPB), 0, s, cfgs, tile_start, n_cfg, n_tiles,
                           slots, partials, buf_sel);
    return hipGetLastError();
}

// F(N, R) for every (N, code) pair the variant table can name
#define TGF_SUN_DISPATCH(F, ...)                                                  \
    switch (nc * 32 + sun_code(nc, variant < 0 ? 0 : variant)) {                  \
        case 2 * 32 + 1: return F<2, 1>(__VA_ARGS__);                             \
        case 2 * 32 + 2: return F<2, 2>(__VA_ARGS__);                             \
        case 2 * 32 + kLds: return F<2, kLds>(__VA_ARGS__);                       \
        case 3 * 32 + 1: return F<3, 1>(__VA_ARGS__);                             \
        case 3 * 32 + 3: return F<3, 3>(__VA_ARGS__);                             \
        case 3 * 32 + kLds: return F<3, kLds>(__VA_ARGS__);                       \
        case 4 * 32 + 1: return F<4, 1>(__VA_ARGS__);                             \
        case 4 * 32 + 2: return F<4, 2>(__VA_ARGS__);                             \
        case 4 * 32 + 4: return F<4, 4>(__VA_ARGS__);                             \
        case 4 * 32 + kLds: return F<4, kLds>(__VA_ARGS__);                       \
        case 5 * 32 + 1: return F<5, 1>(__VA_ARGS__);                             \
        case 5 * 32 + kLds: return F<5, kLds>(__VA_ARGS__);                       \
        case 6 * 32 + 1: return F<6, 1>(__VA_ARGS__);                             \
        case 6 * 32 + 2: return F<6, 2>(__VA_ARGS__);                             \
        case 6 * 32 + kLds: return F<6, kLds>(__VA_ARGS__);                       \
        case 7 * 32 + 1: return F<7, 1>(__VA_ARGS__);                             \
        case 7 * 32 + kLds: return F<7, kLds>(__VA_ARGS__);                       \
        case 8 * 32 + 1: return F<8, 1>(__VA_ARGS__);                             \
        case 8 * 32 + kLds: return F<8, kLds>(__VA_ARGS__);                       \
        default: return hipErrorInvalidValue;                                     \
    }

hipError_t launch_stage_sun(int nc, int variant, hipStream_t s, const CfgDesc *cfgs,
                            const int *tile_start, int n_act, int n_tiles, int step, int stage,
                            double eps) {
    if (n_tiles <= 0) return hipSuccess;
    if (variant >= sun_variant_count(nc)) return hipErrorInvalidValue;
    const SunStageArgs a{cfgs, tile_start, n_act, n_tiles, step, stage, eps};
    TGF_SUN_DISPATCH(stage_nr, s, a)
}

hipError_t launch_measure_sun(int nc, int variant, hipStream_t s, const CfgDesc *cfgs,
                              const int *tile_start, int n_cfg, int n_tiles, const MeasSlot *slots,
                              double *partials, int buf_sel) {
    if (n_tiles <= 0) return hipSuccess;
    if (variant >= sun_variant_count(nc)) return hipErrorInvalidValue;
    TGF_SUN_DISPATCH(measure_nr, s, cfgs, tile_start, n_cfg, n_tiles, slots, partials, buf_sel)
}

#undef TGF_SUN_DISPATCH

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
