// kernels.hip -- HIP kernels of the twisted Wilson flow for gfx950 (CDNA4).
//
// Method (arXiv 2107.03747, sec. 3.1): the Wilson action with twist factors
// Z_{mu nu}(n) on the plaquettes of the twist site, its gradient flow
// integrated with Luscher's third-order Runge-Kutta scheme in the low-storage
// form
//     X_i = B_i eps F(W_i) + A_i X_{i-1},   W_{i+1} = exp(X_i) W_i,
//     (A, B) = (0, 1/4), (-17/9, 8/9), (-1, 3/4),
// (identical to exp(Z0/4), exp(8/9 Z1 - 17/36 Z0), exp(3/4 Z2 - 8/9 Z1 +
// 17/36 Z0)), force F = -P_ah(Omega) with Omega the twisted staple sum, and
// the clover observables of eq. gmunu / eq. qlatt.
//
// Work decomposition: a "tile" is 64 consecutive sites of one configuration
// (one wavefront in the site mapping).  Tiles of all configurations of a
// batch are numbered consecutively; a wavefront finds its configuration by a
// wave-uniform binary search in the tile prefix table, so one launch covers
// the whole batch.  Each stage is one launch: links are read from one
// ping-pong buffer and written to the other, so no stage reads what another
// work-group of the same launch writes.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "launch.h"
#include "lattice_dev.h"
#include "layout.h"
#include "measure_dev.h"
#include "su3_dev.h"

namespace tgf {

// RK stage tail for one link, from Z = B eps F in the 8-real form:
// X = Z + A X_old; W_out = exp(X) W_in, formed as W_in + (exp(X) - 1) W_in so
// that FP32 rounding has no preferred direction (su3_expm1).
template <class R, int NE, class LK>
__device__ __forceinline__ void update_link_z(const LK &W, gptr<v2<R>> Wout,
                                              gptr<v2<R>> X, int stride, int mu, int i,
                                              Alg<R> Z, R a, int stage, int reunit) {
    if (stage > 0) {
        R o[8];
        ld_alg8<R>(X, mu, stride, i, o);
#pragma unroll
        for (int k = 0; k < 8; k++) Z.a[k] = fma(a, o[k], Z.a[k]);
    }
    if (stage < 2) st_alg8<R>(X, mu, stride, i, Z.a);
    constexpr int ROWS = NE == 9 ? 3 : 2;
    const M3<R> D = su3_expm1<R, ROWS>(Z);
    const M3<R> U = W.own(mu, i);
    M3<R> N = mul_add_expm1<R, ROWS>(D, U);
    if (reunit) reunitarise(N);
    store_link<R, NE>(Wout, stride, mu, i, N);
}

// RK stage tail from Omega: B eps F = -B eps P_ah(Omega).
template <class R, int NE>
__device__ __forceinline__ void update_link(const Links<R, NE> &W, gptr<v2<R>> Wout,
                                            gptr<v2<R>> X, int stride, int mu, int i,
                                            const M3<R> &Omega, R beps, R a, int stage,
                                            int reunit) {
    update_link_z<R, NE>(W, Wout, X, stride, mu, i, proj_ah(Omega, -beps), a, stage, reunit);
}

__constant__ double kRkA[3] = {0.0, -17.0 / 9.0, -1.0};
__constant__ double kRkB[3] = {0.25, 8.0 / 9.0, 0.75};

struct StageArgs {
    const CfgDesc *cfgs;
    const int *tile_start;
    int n_act;
    int n_tiles;
    const int *blk_start;   // LDS-staged variants: work-groups of CfgDesc::blk sites
    int n_blocks;
    int step;
    int stage;
    double eps;
    int reunit_every;   // FP64 reunitarisation every this many steps (0 = never)
    int xcd;        // 1: remap blocks so each XCD owns a contiguous tile range
};

// Reunitarise at the end of this step of configuration c?  Steps are counted
// from the load of the configuration (reunit_phase = steps done before this
// flow call, modulo reunit_every), so the schedule does not depend on how a
// caller splits a flow into calls.
__device__ __forceinline__ int reunit_now(const StageArgs &a, const CfgDesc &c) {
    return a.stage == 2 && a.reunit_every > 0 &&
           (c.reunit_phase + a.step + 1) % a.reunit_every == 0;
}

// Lower staples of link MU summed, Omega_MU += U_MU(n) S, then the RK update
// (MU is a template argument so that acc[] is never indexed at run time).
template <class R, int NE, int MU>
__device__ __forceinline__ void site_lower_update(const Links<R, NE> &W, gptr<v2<R>> Wout,
                                                  gptr<v2<R>> X, const CfgDesc &c, const Geo &g,
                                                  M3<R> &om, R beps, R ac, const StageArgs &a) {
    M3<R> S;
    m_zero(S);
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == MU) continue;
        acc_lower_staple(S, W, c, g, MU, nu);
    }
    m_acc_mul_nn(om, W(MU, g.i), S);
    update_link<R, NE>(W, Wout, X, c.stride, MU, g.i, om, beps, ac, a.stage, reunit_now(a, c));
}

// One thread per site: the six upper plaquettes feed both of their links
// (P_{nu mu} = P_{mu nu}^+), the twelve lower staples are summed per link
// before the single U_mu(n) S product.
template <class R, int NE>
__global__ __launch_bounds__(256) void stage_site_kernel(StageArgs a) {
    const int nb = (a.n_tiles + 3) >> 2;
    const int b = remap_block(blockIdx.x, nb, a.xcd);
    if (b >= nb) return;
    const int tile = b * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tile >= a.n_tiles) return;
    const int ci = find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc c = a.cfgs[ci];
    const int i = (tile - a.tile_start[ci]) * kTile + (threadIdx.x & 63);
    if (i >= c.V) return;

    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    const Links<R, NE> W{as_global<R>((const void *)(in ? c.W[1] : c.W[0])), c.stride};
    gptr<v2<R>> Wout = as_global<R>(in ? c.W[0] : c.W[1]);
    gptr<v2<R>> X = as_global<R>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const R beps = (R)(kRkB[a.stage] * eps);
    const R ac = (R)kRkA[a.stage];
    const Geo g = make_geo(c, i);

    M3<R> acc[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) m_zero(acc[mu]);
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int nu = mu + 1; nu < 4; nu++) {
            M3<R> P = upper_plaq(W, c, g, mu, nu);
            m_acc(acc[mu], P);
            m_acc_scaled_dag(acc[nu], cx<R>{R(1), R(0)}, P);
        }
    site_lower_update<R, NE, 0>(W, Wout, X, c, g, acc[0], beps, ac, a);
    site_lower_update<R, NE, 1>(W, Wout, X, c, g, acc[1], beps, ac, a);
    site_lower_update<R, NE, 2>(W, Wout, X, c, g, acc[2], beps, ac, a);
    site_lower_update<R, NE, 3>(W, Wout, X, c, g, acc[3], beps, ac, a);
}

// Site variant with su(3) force accumulators.  Each upper plaquette
// Z^* P_{mu nu}(n) enters its two links with opposite signs (P_ah(P^+) =
// -P_ah(P)) in the raw 8-real form (r2_raw: no third row, no per-term
// projection); each link's sum is projected once (raw_to_alg).  Lower staples:
// FP32 forms each closed loop U_mu(n) x staple in two rows and adds its raw
// form the same way (fewer operations, no 3x3 sum, 188 instead of 240
// registers); FP64 sums the three staples as 3x3 matrices and multiplies the
// sum by U_mu(n) once, which runs 1.5% faster at its one wave per SIMD.
template <class R, int NE, int MU, class LK>
__device__ __forceinline__ void site_alg_update(const LK &W, gptr<v2<R>> Wout,
                                                gptr<v2<R>> X, const CfgDesc &c, const Geo &g,
                                                const R f[8], R beps, R ac,
                                                const StageArgs &a) {
    Alg<R> Z;
    if constexpr (sizeof(R) == 4) {
        R k[8];
#pragma unroll
        for (int t = 0; t < 8; t++) k[t] = f[t];
#pragma unroll
        for (int nu = 0; nu < 4; nu++) {
            if (nu == MU) continue;
            // U_mu(n) times the lower staple is the closed loop
            // U_mu(n) U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu), an SU(3) matrix
            // times a cube root of unity: two rows, raw form
            const int imn = g.i + g.dn(nu);
            R2<R> P = r2_of(W.own(MU, g.i));
            P = r2_mul_nd(P, W(nu, imn + g.up(MU)));
            P = r2_mul_nd(P, W(MU, imn));
            P = r2_mul_nn(P, W(nu, imn));
            const int kt = twist_exp(c, MU, nu);
            // the loop is U_nu(n-nu)^+ P_{mu nu}(n-nu)^+ U_nu(n-nu): its factor is
            // Z_{mu nu}, the conjugate of the Z^* on the plaquette
            if (kt && g.n(MU) == 0 && g.back(nu) == 0) r2_scale(P, omega_pow<R>(kt));
            R r[8];
            r2_raw(P, r);
#pragma unroll
            for (int t = 0; t < 8; t++) k[t] += r[t];
        }
        Z = raw_to_alg(k, -beps);
    } else {
        M3<R> S;
        m_zero(S);
#pragma unroll
        for (int nu = 0; nu < 4; nu++) {
            if (nu == MU) continue;
            acc_lower_staple(S, W, c, g, MU, nu);
        }
        const Alg<R> lo = proj_ah(mul_nn(W.own(MU, g.i), S), R(1));
        Z = raw_to_alg(f, -beps);
#pragma unroll
        for (int k = 0; k < 8; k++) Z.a[k] = fma(-beps, lo.a[k], Z.a[k]);
    }
    update_link_z<R, NE>(W, Wout, X, c.stride, MU, g.i, Z, ac, a.stage, reunit_now(a, c));
}

// The force of the four links of site g.i from raw su(3) accumulators, then
// the four RK updates; W is the link accessor (global memory, or LDS-staged).
template <class R, int NE, class LK>
__device__ __forceinline__ void site_alg_work(const LK &W, gptr<v2<R>> Wout, gptr<v2<R>> X,
                                              const CfgDesc &c, const Geo &g, R beps, R ac,
                                              const StageArgs &a) {
    const int i = g.i;
    R f[4][8];
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int k = 0; k < 8; k++) f[mu][k] = R(0);
#pragma unroll
    for (int mu = 0, p = 0; mu < 4; mu++)
#pragma unroll
        for (int nu = mu + 1; nu < 4; nu++, p++) {
            // rows 0,1 of U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+, times Z^*; a
            // cube root of unity keeps the third row conj(row0 x row1)
            R2<R> P = r2_of(W.own(mu, i));
            P = r2_mul_nn(P, W(nu, i + g.up(mu)));
            P = r2_mul_nd(P, W(mu, i + g.up(nu)));
            P = r2_mul_nd(P, W.own(nu, i));
            const int k = c.tw[p];
            if (k && g.n(mu) == 0 && g.n(nu) == 0) r2_scale(P, cconj(omega_pow<R>(k)));
            R r[8];
            r2_raw(P, r);
#pragma unroll
            for (int t = 0; t < 8; t++) {
                f[mu][t] += r[t];
                f[nu][t] -= r[t];
            }
        }
    site_alg_update<R, NE, 0>(W, Wout, X, c, g, f[0], beps, ac, a);
    site_alg_update<R, NE, 1>(W, Wout, X, c, g, f[1], beps, ac, a);
    site_alg_update<R, NE, 2>(W, Wout, X, c, g, f[2], beps, ac, a);
    site_alg_update<R, NE, 3>(W, Wout, X, c, g, f[3], beps, ac, a);
}

// site_alg_work with in-wave plaquette reuse (FP32): a lane's lower staple
// term of link mu in plane nu is the conjugated plaquette of site n - nu;
// when that site lies in the same wave for every active lane (the (n0, n1)
// directions when a 64-site wave holds whole planes), its raw form is pulled
// from that lane right after it is formed, and conjugated by one link:
//   link mu < nu: -U_nu(n-nu)^+ [Z^*P_{mu nu}](n-nu) U_nu(n-nu),
//   link nu > mu: +U_mu(n-mu)^+ [Z^*P_{mu nu}](n-mu) U_mu(n-mu)   (raw forms).
// Other lower terms are formed directly.  The choice depends only on the
// work-group shape of the configuration, so a configuration's result does not
// depend on the batch around it.
template <class R, int NE, class LK>
__device__ __forceinline__ void site_wave_work(const LK &W, gptr<v2<R>> Wout, gptr<v2<R>> X,
                                               const CfgDesc &c, const Geo &g, R beps, R ac,
                                               const StageArgs &a, int nw) {
    // nw: active lanes of this wave, holding sites tb .. tb + nw - 1
    const int i = g.i;
    const int tb = i - (int)(threadIdx.x & 63);        // first site of this wave
    R f[4][8];
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int k = 0; k < 8; k++) f[mu][k] = R(0);
    unsigned done = 0;                                  // bit 4 mu + nu: lower term (mu, nu)
#pragma unroll
    for (int mu = 0, p = 0; mu < 4; mu++)
#pragma unroll
        for (int nu = mu + 1; nu < 4; nu++, p++) {
            R2<R> P = r2_of(W.own(mu, i));
            P = r2_mul_nn(P, W(nu, i + g.up(mu)));
            P = r2_mul_nd(P, W(mu, i + g.up(nu)));
            P = r2_mul_nd(P, W.own(nu, i));
            const int k = c.tw[p];
            if (k && g.n(mu) == 0 && g.n(nu) == 0) r2_scale(P, cconj(omega_pow<R>(k)));
            R r[8];
            r2_raw(P, r);
#pragma unroll
            for (int t = 0; t < 8; t++) {
                f[mu][t] += r[t];
                f[nu][t] -= r[t];
            }
            const int imn = i + g.dn(nu);
            if (__all((unsigned)(imn - tb) < (unsigned)nw)) {
                R an[8], cc[8];
#pragma unroll
                for (int t = 0; t < 8; t++) an[t] = __shfl(r[t], imn - tb);
                conj_raw(W(nu, imn), an, cc);
#pragma unroll
                for (int t = 0; t < 8; t++) f[mu][t] -= cc[t];
                done |= 1u << (4 * mu + nu);
            }
            const int imm = i + g.dn(mu);
            if (__all((unsigned)(imm - tb) < (unsigned)nw)) {
                R an[8], cc[8];
#pragma unroll
                for (int t = 0; t < 8; t++) an[t] = __shfl(r[t], imm - tb);
                conj_raw(W(mu, imm), an, cc);
#pragma unroll
                for (int t = 0; t < 8; t++) f[nu][t] += cc[t];
                done |= 1u << (4 * nu + mu);
            }
        }
    // the remaining lower terms grouped by direction nu: U_nu(n - nu), which
    // closes all three loops of that direction, is fetched and its third row
    // rebuilt once; the scheduling fences keep the groups from being
    // interleaved (without them: 168 registers and a spill instead of 147)
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        unsigned todo = 0;
#pragma unroll
        for (int mu = 0; mu < 4; mu++)
            if (mu != nu && !((done >> (4 * mu + nu)) & 1u)) todo |= 1u << mu;
        if (!todo) continue;
        __builtin_amdgcn_sched_barrier(0);
        const int imn = i + g.dn(nu);
        const M3<R> V = W(nu, imn);
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            if (mu == nu || !((todo >> mu) & 1u)) continue;
            R2<R> P = r2_of(W.own(mu, i));
            P = r2_mul_nd(P, W(nu, imn + g.up(mu)));
            P = r2_mul_nd(P, W(mu, imn));
            P = r2_mul_nn(P, V);
            const int kt = twist_exp(c, mu, nu);
            if (kt && g.n(mu) == 0 && g.back(nu) == 0) r2_scale(P, omega_pow<R>(kt));
            R r[8];
            r2_raw(P, r);
#pragma unroll
            for (int t = 0; t < 8; t++) f[mu][t] += r[t];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    const int rn = reunit_now(a, c);
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
        update_link_z<R, NE>(W, Wout, X, c.stride, mu, i, raw_to_alg(f[mu], -beps), ac, a.stage,
                             rn);
}

template <class R, int NE>
__device__ __forceinline__ void site_alg_body(const StageArgs &a) {
    const int nb = (a.n_tiles + 3) >> 2;
    const int b = remap_block(blockIdx.x, nb, a.xcd);
    if (b >= nb) return;
    const int tile = b * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tile >= a.n_tiles) return;
    const int ci = find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc c = a.cfgs[ci];
    const int i = (tile - a.tile_start[ci]) * kTile + (threadIdx.x & 63);
    if (i >= c.V) return;

    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    const Links<R, NE> W{as_global<R>((const void *)(in ? c.W[1] : c.W[0])), c.stride};
    gptr<v2<R>> Wout = as_global<R>(in ? c.W[0] : c.W[1]);
    gptr<v2<R>> X = as_global<R>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const R beps = (R)(kRkB[a.stage] * eps);
    const R ac = (R)kRkA[a.stage];
    site_alg_work<R, NE>(W, Wout, X, c, make_geo(c, i), beps, ac, a);
}

// ---------------------------------------------------------------------------
// LDS-staged site variant.  A work-group owns blk consecutive sites of one
// configuration (blk <= 256 per configuration, CfgDesc::blk: whole (n0, n1)
// planes where they fit, so that the neighbours in directions 0 and 1 are
// always in the block); it first copies their four links into LDS as 16-byte
// units ([mu][unit][site]: FP32 entry pairs, and entry 8 alone for the full
// storage; FP64 one complex entry per unit), then every link a wave needs is
// read from LDS when all of its active lanes find the link's site inside the
// block, and from global memory otherwise.  Wave w holds sites base + 64 w +
// lane (lanes past the block end are idle).  LDS per work-group: 48 KB (FP32
// 12-real), 72 KB (FP32 full), 144 KB (FP64).  (Staging full matrices for the
// 12-real storage, so that its third rows are rebuilt once per link, ran 15%
// slower.)

template <class R, int NE>
struct StagedLinks {
    typedef R U16 __attribute__((ext_vector_type(16 / sizeof(R))));
    static constexpr int NU = sizeof(R) == 8 ? NE : (NE == 9 ? 4 : 3);   // units per link
    Links<R, NE> gl;
    const U16 *s16;           // [mu][unit][kBlock]
    const v2<R> *s8;          // [mu][kBlock], FP32 full storage entry 8
    int base;                 // first site of the block
    int nblk;                 // sites in the block
    // a link of this lane's own site: always in LDS
    __device__ __forceinline__ M3<R> own(int mu, int i) const { return fetch(mu, i, true); }
    __device__ __forceinline__ M3<R> operator()(int mu, int j) const {
        return fetch(mu, j, __all((unsigned)(j - base) < (unsigned)nblk));
    }
    __device__ __forceinline__ M3<R> fetch(int mu, int j, bool from_lds) const {
        // the 16-byte units come from LDS or from global memory; the matrix
        // (and the 12-real third row) is assembled once after the branch
        const unsigned k = (unsigned)(j - base);
        constexpr bool kE8 = sizeof(R) == 4 && NE == 9;
        U16 u[NU];
        v2<R> e8;
        if (from_lds) {
            const U16 *q = s16 + mu * NU * kBlock + k;
#pragma unroll
            for (int e = 0; e < NU; e++) u[e] = q[e * kBlock];
            if constexpr (kE8) e8 = s8[mu * kBlock + k];
        } else {
            gptr<const char> q = (gptr<const char>)(gl.p + (size_t)(mu * NE) * gl.stride);
            const size_t pl = (size_t)gl.stride * 16u;
            const unsigned off = (unsigned)j * 16u;
#pragma unroll
            for (int e = 0; e < NU; e++) u[e] = *(gptr<const U16>)(q + e * pl + off);
            if constexpr (kE8)
                e8 = *(gptr<const v2<R>>)((gptr<const char>)(gl.p + (size_t)(mu * 9 + 8) * gl.stride) +
                                          lane_off<R>(j));
        }
        M3<R> U;
        if constexpr (sizeof(R) == 4) {
            U.e[0][0] = {u[0].x, u[0].y};
            U.e[0][1] = {u[0].z, u[0].w};
            U.e[0][2] = {u[1].x, u[1].y};
            U.e[1][0] = {u[1].z, u[1].w};
            U.e[1][1] = {u[2].x, u[2].y};
            U.e[1][2] = {u[2].z, u[2].w};
            if constexpr (NE == 9) {
                U.e[2][0] = {u[3].x, u[3].y};
                U.e[2][1] = {u[3].z, u[3].w};
                U.e[2][2] = {e8.x, e8.y};
            }
        } else {
#pragma unroll
            for (int e = 0; e < NE; e++) U.e[e / 3][e % 3] = {u[e].x, u[e].y};
        }
        if constexpr (NE == 6) rebuild_row2(U);
        return U;
    }
};

template <class R, int NE>
__device__ __forceinline__ void site_lds_body(const StageArgs &a) {
    typedef typename StagedLinks<R, NE>::U16 U16;
    constexpr int NU = StagedLinks<R, NE>::NU;
    constexpr bool kE8 = sizeof(R) == 4 && NE == 9;
    __shared__ U16 s16[4 * NU * kBlock];
    __shared__ v2<R> s8[kE8 ? 4 * kBlock : 1];

    const int b = remap_block(blockIdx.x, a.n_blocks, a.xcd);
    if (b >= a.n_blocks) return;                           // whole work-group
    const int ci = find_cfg(a.blk_start, a.n_act, b);      // work-group uniform
    const CfgDesc c = a.cfgs[ci];
    const int base = block_order(b - a.blk_start[ci], c) * c.blk;
    const int nblk = min(c.blk, c.V - base);               // sites base .. base + nblk - 1
    const int i = base + (int)threadIdx.x;

    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    const Links<R, NE> G{as_global<R>((const void *)(in ? c.W[1] : c.W[0])), c.stride};
    if ((int)threadIdx.x < nblk) {
        // unit u of link (mu, i) sits at byte (mu NE stride 2 sizeof(R)) +
        // u stride 16 + 16 i (the FP32 pairs of entry_index; FP64 entries)
        gptr<const char> q = (gptr<const char>)G.p;
        const size_t pl = (size_t)c.stride * 16u;
        const unsigned u = (unsigned)i * 16u;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            gptr<const char> qm = q + (size_t)(mu * NE) * c.stride * (2 * sizeof(R));
#pragma unroll
            for (int e = 0; e < NU; e++)
                s16[(mu * NU + e) * kBlock + threadIdx.x] = *(gptr<const U16>)(qm + e * pl + u);
            if constexpr (kE8) {
                const cx<R> z = ld(G.p + (size_t)(mu * 9 + 8) * c.stride, lane_off<R>(i));
                s8[mu * kBlock + threadIdx.x] = v2<R>{z.x, z.y};
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x >= nblk) return;

    const StagedLinks<R, NE> W{G, s16, s8, base, nblk};
    gptr<v2<R>> Wout = as_global<R>(in ? c.W[0] : c.W[1]);
    gptr<v2<R>> X = as_global<R>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const R beps = (R)(kRkB[a.stage] * eps);
    const R ac = (R)kRkA[a.stage];
    // 12-real storage reuses in-wave plaquettes (stage launch -1.4%); for the
    // full storages the plain site_alg_work measured faster
    if constexpr (sizeof(R) == 4 && NE == 6) {
        const int nw = min(64, nblk - (int)(threadIdx.x & ~63u));
        site_wave_work<R, NE>(W, Wout, X, c, make_geo(c, i), beps, ac, a, nw);
    } else {
        site_alg_work<R, NE>(W, Wout, X, c, make_geo(c, i), beps, ac, a);
    }
}

// Waves per SIMD: FP32 12-real three (147 registers, none spilled; three
// 48 KB blocks per CU), FP32 full two (72 KB blocks), FP64 one (144 KB).
// With the in-block neighbours in LDS the third 12-real wave pays: 6.5%
// shorter stage launches than the two-wave build, where without LDS a third
// wave brought as many L2 misses as it hid.
template <class R, int NE>
__global__ __launch_bounds__(256, sizeof(R) == 8 ? 1 : (NE == 6 ? 3 : 2))
void stage_site_lds_kernel(StageArgs a) {
    site_lds_body<R, NE>(a);
}

// Lower staple terms of link MU (from the block's plaquettes in LDS where the
// whole wave finds them there, else formed directly) and the RK update.
template <class R, int NE, int MU, class U16>
__device__ __forceinline__ void plq_update(const Links<R, NE> &W, gptr<v2<R>> Wout, gptr<v2<R>> X,
                                           const CfgDesc &c, const Geo &g, const Alg<R> &f,
                                           R beps, R ac, const StageArgs &a, const U16 *sA,
                                           int base, int staged) {
    constexpr int NA = 8 * (int)sizeof(R) / 16;
    Alg<R> Z = f;
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == MU) continue;
        const int imn = g.i + g.dn(nu);
        const unsigned k = (unsigned)(imn - base);
        R A8[8];
        if (staged && __all(k < (unsigned)kBlock)) {
            const int p = MU < nu ? (MU == 0 ? nu - 1 : (MU == 1 ? nu + 1 : 5))
                                      : (nu == 0 ? MU - 1 : (nu == 1 ? MU + 1 : 5));
            const U16 *q = sA + p * NA * kBlock + k;
            R am[8];
#pragma unroll
            for (int u = 0; u < NA; u++) {
                const U16 v = q[u * kBlock];
                if constexpr (sizeof(R) == 4) {
                    am[4 * u] = v.x; am[4 * u + 1] = v.y; am[4 * u + 2] = v.z; am[4 * u + 3] = v.w;
                } else {
                    am[2 * u] = v.x; am[2 * u + 1] = v.y;
                }
            }
            conj_alg(W(nu, imn), am, A8);
            const R sg = MU < nu ? R(-1) : R(1);
#pragma unroll
            for (int t = 0; t < 8; t++) A8[t] *= sg;
        } else {
            R2<R> P = r2_of(W(MU, g.i));
            P = r2_mul_nd(P, W(nu, imn + g.up(MU)));
            P = r2_mul_nd(P, W(MU, imn));
            P = r2_mul_nn(P, W(nu, imn));
            const int kt = twist_exp(c, MU, nu);
            if (kt && g.n(MU) == 0 && g.back(nu) == 0) r2_scale(P, omega_pow<R>(kt));
            r2_proj_ah(P, R(1), A8);
        }
#pragma unroll
        for (int t = 0; t < 8; t++) Z.a[t] += A8[t];
    }
#pragma unroll
    for (int t = 0; t < 8; t++) Z.a[t] *= -beps;
    update_link_z<R, NE>(W, Wout, X, c.stride, MU, g.i, Z, ac, a.stage, reunit_now(a, c));
}

// ---------------------------------------------------------------------------
// Plaquette-sharing site variant.  A work-group owns 256 consecutive sites of
// one configuration.  Each lane first forms its six upper plaquettes
// A_{mu nu}(n) = P_ah(Z^* P_{mu nu}(n)) (two-row products, as site_alg) and
// keeps them in LDS ([plane][16-byte unit][site]); after a barrier, a lower
// staple term of link mu in plane nu whose plaquette P_{mu nu}(n-nu) belongs
// to a site of the block (all active lanes of the wave) is taken from there:
//   P_ah(U_mu(n) x lower staple) = -/+ U_nu(n-nu)^+ A_{min max}(n-nu) U_nu(n-nu)
// (- for mu < nu, + for mu > nu; P_ah is linear and commutes with the
// conjugation), one link load and one conjugation instead of three links and
// three two-row products.  Other lower terms are formed directly.  Work-groups
// whose tiles span two configurations skip the LDS (no barrier).

template <class R, int NE>
__device__ __forceinline__ void site_plq_body(const StageArgs &a) {
    typedef R U16 __attribute__((ext_vector_type(16 / sizeof(R))));
    constexpr int NA = 8 * (int)sizeof(R) / 16;      // 16-byte units per su(3) element
    __shared__ U16 sA[6 * NA * kBlock];

    const int nb = (a.n_tiles + 3) >> 2;
    const int b = remap_block(blockIdx.x, nb, a.xcd);
    if (b >= nb) return;                                   // whole work-group
    const int t0 = b * 4;
    const int tile = t0 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci0 = find_cfg(a.tile_start, a.n_act, t0);
    const int staged = t0 + 3 < a.n_tiles && find_cfg(a.tile_start, a.n_act, t0 + 3) == ci0;
    if (!staged && tile >= a.n_tiles) return;
    const int ci = staged ? ci0 : find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc c = a.cfgs[ci];
    const int i = (tile - a.tile_start[ci]) * kTile + (threadIdx.x & 63);
    const int base = (t0 - a.tile_start[ci]) * kTile;

    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    const Links<R, NE> W{as_global<R>((const void *)(in ? c.W[1] : c.W[0])), c.stride};
    const Geo g = make_geo(c, i < c.V ? i : 0);

    Alg<R> f[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int k = 0; k < 8; k++) f[mu].a[k] = R(0);
    if (i < c.V) {
#pragma unroll
        for (int mu = 0, p = 0; mu < 4; mu++)
#pragma unroll
            for (int nu = mu + 1; nu < 4; nu++, p++) {
                R2<R> P = r2_of(W(mu, i));
                P = r2_mul_nn(P, W(nu, i + g.up(mu)));
                P = r2_mul_nd(P, W(mu, i + g.up(nu)));
                P = r2_mul_nd(P, W(nu, i));
                const int k = c.tw[p];
                if (k && g.n(mu) == 0 && g.n(nu) == 0) r2_scale(P, cconj(omega_pow<R>(k)));
                R A8[8];
                r2_proj_ah(P, R(1), A8);
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    f[mu].a[t] += A8[t];
                    f[nu].a[t] -= A8[t];
                }
                if (staged) {
                    U16 *o = sA + p * NA * kBlock + threadIdx.x;
#pragma unroll
                    for (int u = 0; u < NA; u++) {
                        U16 v;
                        if constexpr (sizeof(R) == 4) {
                            v.x = A8[4 * u]; v.y = A8[4 * u + 1]; v.z = A8[4 * u + 2]; v.w = A8[4 * u + 3];
                        } else {
                            v.x = A8[2 * u]; v.y = A8[2 * u + 1];
                        }
                        o[u * kBlock] = v;
                    }
                }
            }
    }
    if (staged) __syncthreads();
    if (i >= c.V) return;

    gptr<v2<R>> Wout = as_global<R>(in ? c.W[0] : c.W[1]);
    gptr<v2<R>> X = as_global<R>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const R beps = (R)(kRkB[a.stage] * eps);
    const R ac = (R)kRkA[a.stage];
    plq_update<R, NE, 0>(W, Wout, X, c, g, f[0], beps, ac, a, sA, base, staged);
    plq_update<R, NE, 1>(W, Wout, X, c, g, f[1], beps, ac, a, sA, base, staged);
    plq_update<R, NE, 2>(W, Wout, X, c, g, f[2], beps, ac, a, sA, base, staged);
    plq_update<R, NE, 3>(W, Wout, X, c, g, f[3], beps, ac, a, sA, base, staged);
}

template <class R, int NE>
__global__ __launch_bounds__(256, sizeof(R) == 8 ? 1 : (NE == 6 ? 3 : 2))
void stage_site_plq_kernel(StageArgs a) {
    site_plq_body<R, NE>(a);
}

// Register budgets: FP64 keeps the whole working set in 512 registers (one
// wave per SIMD); FP32 is capped at 256 (two waves per SIMD).
template <class R, int NE>
__global__ __launch_bounds__(256) void stage_site_alg_kernel(StageArgs a) {
    site_alg_body<R, NE>(a);
}

template <class R, int NE>
__global__ __launch_bounds__(256, 2) void stage_site_alg2_kernel(StageArgs a) {
    site_alg_body<R, NE>(a);
}

// the same with at most 168 registers, so three waves share a SIMD (the
// compiler spills the excess to scratch)
template <class R, int NE>
__global__ __launch_bounds__(256, 3) void stage_site_alg3_kernel(StageArgs a) {
    site_alg_body<R, NE>(a);
}

// One thread per link: a work-group is one tile of 64 sites x 4 directions,
// wave w handles direction mu = w for the 64 sites (mu is a compile-time
// constant inside the body, so all coordinate arrays stay in registers).
template <class R, int NE, int MU>
__device__ __forceinline__ void link_body(const StageArgs &a, const CfgDesc &c, int i) {
    const int in = (c.cur + 3 * a.step + a.stage) & 1;
    const Links<R, NE> W{as_global<R>((const void *)(in ? c.W[1] : c.W[0])), c.stride};
    gptr<v2<R>> Wout = as_global<R>(in ? c.W[0] : c.W[1]);
    gptr<v2<R>> X = as_global<R>(c.X);
    const double eps = a.step < c.n_full ? a.eps : c.eps_last;
    const R beps = (R)(kRkB[a.stage] * eps);
    const R ac = (R)kRkA[a.stage];
    const Geo g = make_geo(c, i);

    M3<R> S;
    m_zero(S);
#pragma unroll
    for (int nu = 0; nu < 4; nu++) {
        if (nu == MU) continue;
        m_acc(S, upper_staple(W, c, g, MU, nu));
        m_acc(S, lower_staple(W, c, g, MU, nu));
    }
    M3<R> Om = mul_nn(W(MU, i), S);
    update_link<R, NE>(W, Wout, X, c.stride, MU, i, Om, beps, ac, a.stage, reunit_now(a, c));
}

template <class R, int NE>
__global__ __launch_bounds__(256) void stage_link_kernel(StageArgs a) {
    const int b = remap_block(blockIdx.x, a.n_tiles, a.xcd);
    if (b >= a.n_tiles) return;
    const int tile = b;
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = find_cfg(a.tile_start, a.n_act, tile);
    const CfgDesc c = a.cfgs[ci];
    const int i = (tile - a.tile_start[ci]) * kTile + (threadIdx.x & 63);
    if (i >= c.V) return;
    switch (mu) {
        case 0: link_body<R, NE, 0>(a, c, i); break;
        case 1: link_body<R, NE, 1>(a, c, i); break;
        case 2: link_body<R, NE, 2>(a, c, i); break;
        default: link_body<R, NE, 3>(a, c, i); break;
    }
}

// ---------------------------------------------------------------------------
// measurement: clover G (eq. gmunu), e(n), q(n), plaquette, action (measure_dev.h)

template <class R, int NE>
__global__ __launch_bounds__(192) void measure_kernel(const CfgDesc *__restrict__ cfgs,
                                                      const int *__restrict__ tile_start, int n_cfg,
                                                      int n_tiles, const MeasSlot *__restrict__ slots,
                                                      double *__restrict__ partials, int buf_sel) {
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const int pair = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ci = find_cfg(tile_start, n_cfg, tile);
    if (slots[ci].row < 0) return;
    const CfgDesc c = cfgs[ci];
    const int tb = (tile - tile_start[ci]) * kTile;            // site of lane 0
    const int i = tb + (threadIdx.x & 63);
    double v[4] = {0, 0, 0, 0};
    if (i < c.V) {
        const int sel = buf_sel < 0 ? c.cur : ((c.cur + buf_sel) & 1);
        const Links<R, NE> W{as_global<R>((const void *)(sel ? c.W[1] : c.W[0])), c.stride};
        const Geo g = make_geo(c, i);
        const int nw = min(kTile, c.V - tb);
        switch (pair) {
            case 0: measure_pair<R, 0>(W, c, g, v, tb, nw); break;
            case 1: measure_pair<R, 1>(W, c, g, v, tb, nw); break;
            default: measure_pair<R, 2>(W, c, g, v, tb, nw); break;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) {
        double *o = partials + ((size_t)tile * 3 + pair) * 4;
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
}

// ---------------------------------------------------------------------------
// Topological charge per slice: q(s) = (1/16 pi^2) sum_{n : n_dir = s} Tr G G~
// (eq. qlatt restricted to one slice).  Block (b, s) takes the sites
// 256 b .. 256 b + 255 of slice s, one per thread; the sites of a slice are
// enumerated over the three other directions in increasing order.  FP64
// partials, summed in a fixed order.
template <class R, int NE>
__global__ __launch_bounds__(256) void slice_charge_kernel(const CfgDesc *__restrict__ cfgs, int ci,
                                                           int dir, double *__restrict__ partials) {
    const CfgDesc &c = cfgs[ci];   // read in place (c.d is indexed at run time)
    const int s = blockIdx.y;
    const int S = c.V / c.d[dir];
    // the other three directions, increasing
    const int o0 = dir == 0 ? 1 : 0;
    const int o1 = dir <= 1 ? 2 : 1;
    const int o2 = dir == 3 ? 2 : 3;
    // site stride of direction m (no private array indexed at run time)
    auto stride_of = [&](int m) {
        return m == 0 ? 1 : m == 1 ? c.d[0] : m == 2 ? c.d[0] * c.d[1] : c.d[0] * c.d[1] * c.d[2];
    };
    double q = 0;
    const int j = blockIdx.x * 256 + (int)threadIdx.x;
    if (j < S) {
        const int da = c.d[o0], db = c.d[o1];
        const int na = j % da, r = j / da;
        const int nb = r % db, nc = r / db;
        const int i = na * stride_of(o0) + nb * stride_of(o1) + nc * stride_of(o2) + s * stride_of(dir);
        const Links<R, NE> W{as_global<R>((const void *)(c.cur ? c.W[1] : c.W[0])), c.stride};
        const Geo g = make_geo(c, i);
        double v0[4], v1[4], v2[4];   // lanes do not hold consecutive sites: leaves formed link by link
        measure_pair<R, 0>(W, c, g, v0);
        measure_pair<R, 1>(W, c, g, v1);
        measure_pair<R, 2>(W, c, g, v2);
        q = (v0[1] + v1[1]) + v2[1];
    }
    q = wave_sum(q);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[(size_t)s * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per-site densities of configuration ci: e(n) = sum_{mu<nu} Tr G^2 and
// q(n) = (1/16 pi^2) Tr G G~, from the three dual plane pairs, written to
// FP64 arrays in site order (either may be null).
template <class R, int NE>
__global__ __launch_bounds__(256) void density_kernel(const CfgDesc *__restrict__ cfgs, int ci,
                                                      double *__restrict__ e_out,
                                                      double *__restrict__ q_out) {
    const CfgDesc c = cfgs[ci];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.V) return;
    const Links<R, NE> W{as_global<R>((const void *)(c.cur ? c.W[1] : c.W[0])), c.stride};
    const Geo g = make_geo(c, i);
    const int tb = i - (int)(threadIdx.x & 63), nw = min(64, c.V - tb);   // lanes = sites tb ..
    double v0[4], v1[4], v2[4];
    measure_pair<R, 0>(W, c, g, v0, tb, nw);
    measure_pair<R, 1>(W, c, g, v1, tb, nw);
    measure_pair<R, 2>(W, c, g, v2, tb, nw);
    if (e_out) e_out[i] = (v0[0] + v1[0]) + v2[0];
    if (q_out) q_out[i] = (v0[1] + v1[1]) + v2[1];
}

__global__ void slice_finalize_kernel(const double *__restrict__ partials, int n_slices, int chunks,
                                      double *__restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    double t = 0;
    for (int k = 0; k < chunks; k++) t += partials[(size_t)s * chunks + k];
    out[s] = t;
}

// One work-group per configuration: fixed-order sum of its tile partials.
__global__ __launch_bounds__(256) void finalize_kernel(const CfgDesc *__restrict__ cfgs,
                                                       const int *__restrict__ tile_start,
                                                       const MeasSlot *__restrict__ slots,
                                                       const double *__restrict__ partials,
                                                       double *__restrict__ rows, int n_cfg_total,
                                                       int *__restrict__ flag, int nc) {
    const int ci = blockIdx.x;
    const MeasSlot sl = slots[ci];
    if (sl.row < 0) return;
    const CfgDesc &c = cfgs[ci];
    const int t0 = tile_start[ci] * 3, t1 = tile_start[ci + 1] * 3;   // (tile, pair) slots
    double tot[4];
    sum_tile_partials(partials, t0, t1, tot);
    if (threadIdx.x == 0) {
        const double V = (double)c.V;
        const double E = tot[0] / V;
        double *r = rows + ((size_t)sl.row * n_cfg_total + c.user) * 6;
        r[0] = sl.t;
        r[1] = E;
        r[2] = sl.t * sl.t * E;
        r[3] = tot[2] / (6.0 * nc * V);
        r[4] = tot[1];
        r[5] = tot[3];
        if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2]) || !isfinite(tot[3]))
            *flag = 1;
    }
}

// ---------------------------------------------------------------------------
// ingest / export / checks

template <class R, int NE>
__global__ __launch_bounds__(256) void unpack_kernel(const cx<R> *__restrict__ W,
                                                     double2 *__restrict__ dst, int V, int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (i >= V) return;
    M3<double> U;
#pragma unroll
    for (int e = 0; e < NE; e++) {
        cx<R> v = W[entry_index<R, NE>(mu, e, stride, i)];
        U.e[e / 3][e % 3] = {(double)v.x, (double)v.y};
    }
    if constexpr (NE == 6) rebuild_row2(U);
    double2 *d = dst + ((size_t)i * 4 + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; e++) d[e] = make_double2(U.e[e / 3][e % 3].x, U.e[e / 3][e % 3].y);
}

__device__ __forceinline__ double finite_or_inf(double v) { return (v <= DBL_MAX) ? v : INFINITY; }

__device__ __forceinline__ void su3_defects(const M3<double> &U, double &du, double &dd) {
    double m = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double re = (i == j) ? -1.0 : 0.0, im = 0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                re += U.e[i][k].x * U.e[j][k].x + U.e[i][k].y * U.e[j][k].y;
                im += U.e[i][k].y * U.e[j][k].x - U.e[i][k].x * U.e[j][k].y;
            }
            m = fmax(m, finite_or_inf(sqrt(re * re + im * im)));
        }
    cx<double> c0 = csub(cmul(U.e[1][1], U.e[2][2]), cmul(U.e[1][2], U.e[2][1]));
    cx<double> c1 = csub(cmul(U.e[1][2], U.e[2][0]), cmul(U.e[1][0], U.e[2][2]));
    cx<double> c2 = csub(cmul(U.e[1][0], U.e[2][1]), cmul(U.e[1][1], U.e[2][0]));
    cx<double> det = cmul(U.e[0][0], c0);
    det = cmadd(det, U.e[0][1], c1);
    det = cmadd(det, U.e[0][2], c2);
    du = m;
    dd = finite_or_inf(sqrt((det.x - 1) * (det.x - 1) + det.y * det.y));
}

// Unitarity defects of stored links, per tile (the canonical inputs of a
// load are checked by ingest_batch_kernel).
template <class R, int NE>
__global__ __launch_bounds__(256) void check_kernel(const void *__restrict__ src, int V, int stride,
                                                    double *__restrict__ partials) {
    const int tile = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = tile * kTile + (threadIdx.x & 63);
    double du = 0, dd = 0;
    if (i < V) {
        for (int mu = 0; mu < 4; mu++) {
            M3<double> U;
            const cx<R> *q = (const cx<R> *)src;
#pragma unroll
            for (int e = 0; e < NE; e++) {
                cx<R> v = q[entry_index<R, NE>(mu, e, stride, i)];
                U.e[e / 3][e % 3] = {(double)v.x, (double)v.y};
            }
            if constexpr (NE == 6) rebuild_row2(U);
            double a, b;
            su3_defects(U, a, b);
            du = fmax(du, a);
            dd = fmax(dd, b);
        }
    }
    du = wave_max(du);
    dd = wave_max(dd);
    const int ntiles = (V + kTile - 1) / kTile;
    if ((threadIdx.x & 63) == 0 && tile < ntiles) {
        partials[(size_t)tile * 2] = du;
        partials[(size_t)tile * 2 + 1] = dd;
    }
}

// Batched ingest: one launch checks and packs the canonical links of every
// configuration of a load call (srcs[k] is configuration k's input; the tile
// table numbers their tiles in order, as for a flow).  A work-group takes one
// 64-site tile.  Its input, 64 sites x 4 links x 9 complex doubles, is one
// contiguous 36 KB range: it arrives through coalesced 16-byte loads (four
// consecutive lanes read 64 consecutive bytes) into LDS, one pad slot after
// every site so that the reads below spread over the banks.  Thread
// (site, mu) then checks its link in FP64 (the defects of check_kernel) and
// writes it, in the context's storage, into the configuration's idle buffer
// W[cur ^ 1] with full 16-byte unit stores; the caller makes that buffer
// current only when every link of the batch passed, so a rejected load
// changes no stored state.  The per-tile maxima of the two defects go to
// partials[2 tile], partials[2 tile + 1].
template <class R, int NE>
__global__ __launch_bounds__(256) void ingest_batch_kernel(const double2 *const *__restrict__ srcs,
                                                           const CfgDesc *__restrict__ cfgs,
                                                           const int *__restrict__ tile_start,
                                                           int n_cfg, int n_tiles,
                                                           double *__restrict__ partials) {
    constexpr int kEnt = 36, kPad = kEnt + 1;   // complex entries per site, LDS slots per site
    __shared__ v2<double> lds[kTile * kPad];
    __shared__ double red[4][2];
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;                           // whole work-group
    const int ci = find_cfg(tile_start, n_cfg, tile);
    const CfgDesc &c = cfgs[ci];
    const int i0 = (tile - tile_start[ci]) * kTile;
    const int ns = min(kTile, c.V - i0);                   // sites i0 .. i0 + ns - 1
    gptr<const v2<double>> src = as_global<double>((const void *)srcs[ci]) + (size_t)i0 * kEnt;
    const int n_el = ns * kEnt;
#pragma unroll
    for (int k = 0; k < kEnt * kTile / 256; k++) {
        const int g = k * 256 + (int)threadIdx.x;
        if (g < n_el) {
            const int st = g / kEnt;
            lds[st * kPad + (g - st * kEnt)] = src[g];
        }
    }
    __syncthreads();
    const int site = threadIdx.x & 63, mu = threadIdx.x >> 6;
    double du = 0, dd = 0;
    if (site < ns) {
        const v2<double> *q = lds + site * kPad + mu * 9;
        M3<double> U;
        M3<R> V;
#pragma unroll
        for (int e = 0; e < 9; e++) {
            const v2<double> v = q[e];
            U.e[e / 3][e % 3] = {v.x, v.y};
            V.e[e / 3][e % 3] = {(R)v.x, (R)v.y};
        }
        su3_defects(U, du, dd);
        store_link<R, NE>(as_global<R>(c.cur ? c.W[0] : c.W[1]), c.stride, mu, i0 + site, V);
    }
    du = wave_max(du);
    dd = wave_max(dd);
    if ((threadIdx.x & 63) == 0) {
        red[mu][0] = du;
        red[mu][1] = dd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[(size_t)tile * 2] = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
        partials[(size_t)tile * 2 + 1] = fmax(fmax(red[0][1], red[1][1]), fmax(red[2][1], red[3][1]));
    }
}

// one work-group per configuration: the maxima over its tiles
__global__ __launch_bounds__(256) void check_batch_final_kernel(const double *__restrict__ partials,
                                                                const int *__restrict__ tile_start,
                                                                double *__restrict__ out) {
    const int k = blockIdx.x;
    double a = 0, b = 0;
    for (int t = tile_start[k] + (int)threadIdx.x; t < tile_start[k + 1]; t += blockDim.x) {
        a = fmax(a, partials[(size_t)t * 2]);
        b = fmax(b, partials[(size_t)t * 2 + 1]);
    }
    a = wave_max(a);
    b = wave_max(b);
    __shared__ double red[4][2];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w][0] = a; red[w][1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * k] = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
        out[2 * k + 1] = fmax(fmax(red[0][1], red[1][1]), fmax(red[2][1], red[3][1]));
    }
}

__global__ __launch_bounds__(256) void check_final_kernel(const double *__restrict__ partials,
                                                          int ntiles, double *__restrict__ out) {
    double a = 0, b = 0;
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        a = fmax(a, partials[(size_t)t * 2]);
        b = fmax(b, partials[(size_t)t * 2 + 1]);
    }
    a = wave_max(a);
    b = wave_max(b);
    __shared__ double red[4][2];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w][0] = a; red[w][1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
        out[1] = fmax(fmax(red[0][1], red[1][1]), fmax(red[2][1], red[3][1]));
    }
}

__global__ void fill_int_kernel(int *dst, int n, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
}

__global__ __launch_bounds__(256) void copy_kernel(const float4 *__restrict__ src,
                                                   float4 *__restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t step = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += step) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launchers

const char *variant_name(int v) {
    switch (v) {
        case V_SITE: return "site";
        case V_LINK: return "link";
        case V_SITE_XCD: return "site_xcd";
        case V_LINK_XCD: return "link_xcd";
        case V_SITE_ALG: return "site_alg";
        case V_SITE_ALG_XCD: return "site_alg_xcd";
        case V_SITE_ALG3: return "site_alg3";
        case V_SITE_ALG3_XCD: return "site_alg3_xcd";
        case V_SITE_LDS: return "site_lds";
        case V_SITE_LDS_XCD: return "site_lds_xcd";
        case V_SITE_PLQ: return "site_plq";
        case V_SITE_PLQ_XCD: return "site_plq_xcd";
        default: return "?";
    }
}

template <class R, int NE>
static hipError_t launch_stage_t(int variant, hipStream_t s, const StageArgs &a) {
    const bool xcd = variant == V_SITE_XCD || variant == V_LINK_XCD || variant == V_SITE_ALG_XCD || variant == V_SITE_ALG3_XCD ||
                     variant == V_SITE_LDS_XCD || variant == V_SITE_PLQ_XCD;
    StageArgs b = a;
    b.xcd = xcd ? 1 : 0;
    const int site_blocks = xcd ? ((a.n_tiles + 3) / 4 + 7) / 8 * 8 : (a.n_tiles + 3) / 4;
    const int tile_blocks = xcd ? (a.n_tiles + 7) / 8 * 8 : a.n_tiles;
    const int lds_blocks = xcd ? (a.n_blocks + 7) / 8 * 8 : a.n_blocks;
    if (variant == V_SITE || variant == V_SITE_XCD) {
        hipLaunchKernelGGL((stage_site_kernel<R, NE>), dim3(site_blocks), dim3(256), 0, s, b);
    } else if (variant == V_SITE_ALG || variant == V_SITE_ALG_XCD) {
        if constexpr (sizeof(R) == 8)
            hipLaunchKernelGGL((stage_site_alg_kernel<R, NE>), dim3(site_blocks), dim3(256), 0, s, b);
        else
            hipLaunchKernelGGL((stage_site_alg2_kernel<R, NE>), dim3(site_blocks), dim3(256), 0, s,
                               b);
    } else if (variant == V_SITE_ALG3 || variant == V_SITE_ALG3_XCD) {
        hipLaunchKernelGGL((stage_site_alg3_kernel<R, NE>), dim3(site_blocks), dim3(256), 0, s, b);
    } else if (variant == V_SITE_LDS || variant == V_SITE_LDS_XCD) {
        if (lds_blocks > 0)
            hipLaunchKernelGGL((stage_site_lds_kernel<R, NE>), dim3(lds_blocks), dim3(256), 0, s,
                               b);
    } else if (variant == V_SITE_PLQ || variant == V_SITE_PLQ_XCD) {
        hipLaunchKernelGGL((stage_site_plq_kernel<R, NE>), dim3(site_blocks), dim3(256), 0, s, b);
    } else {
        hipLaunchKernelGGL((stage_link_kernel<R, NE>), dim3(tile_blocks), dim3(256), 0, s, b);
    }
    return hipGetLastError();
}

hipError_t launch_stage(int variant, Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs,
                        const int *tile_start, int n_act, int n_tiles, const int *blk_start,
                        int n_blocks, int step, int stage, double eps, int reunit_every) {
    if (n_tiles <= 0) return hipSuccess;
    StageArgs a{cfgs, tile_start, n_act, n_tiles, blk_start, n_blocks, step, stage, eps,
                reunit_every, 0};
    if (p == P_F64) return launch_stage_t<double, 9>(variant, s, a);
    if (c12) return launch_stage_t<float, 6>(variant, s, a);
    return launch_stage_t<float, 9>(variant, s, a);
}

hipError_t launch_measure(Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs,
                          const int *tile_start, int n_cfg, int n_tiles, const MeasSlot *slots,
                          double *partials, int buf_sel) {
    if (n_tiles <= 0) return hipSuccess;
    dim3 grid(n_tiles);
    if (p == P_F64)
        hipLaunchKernelGGL((measure_kernel<double, 9>), grid, dim3(192), 0, s, cfgs, tile_start,
                           n_cfg, n_tiles, slots, partials, buf_sel);
    else if (c12)
        hipLaunchKernelGGL((measure_kernel<float, 6>), grid, dim3(192), 0, s, cfgs, tile_start,
                           n_cfg, n_tiles, slots, partials, buf_sel);
    else
        hipLaunchKernelGGL((measure_kernel<float, 9>), grid, dim3(192), 0, s, cfgs, tile_start,
                           n_cfg, n_tiles, slots, partials, buf_sel);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, const CfgDesc *cfgs, const int *tile_start, int n_cfg,
                           const MeasSlot *slots, const double *partials, double *rows,
                           int n_cfg_total, int *flag, int nc) {
    if (n_cfg <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(n_cfg), dim3(256), 0, s, cfgs, tile_start, slots,
                       partials, rows, n_cfg_total, flag, nc);
    return hipGetLastError();
}

hipError_t launch_unpack(Prec p, bool c12, hipStream_t s, const void *W, void *dst, int V,
                         int stride) {
    dim3 grid((V + 255) / 256, 4);
    double2 *out = (double2 *)dst;
    if (p == P_F64)
        hipLaunchKernelGGL((unpack_kernel<double, 9>), grid, dim3(256), 0, s,
                           (const cx<double> *)W, out, V, stride);
    else if (c12)
        hipLaunchKernelGGL((unpack_kernel<float, 6>), grid, dim3(256), 0, s,
                           (const cx<float> *)W, out, V, stride);
    else
        hipLaunchKernelGGL((unpack_kernel<float, 9>), grid, dim3(256), 0, s,
                           (const cx<float> *)W, out, V, stride);
    return hipGetLastError();
}

hipError_t launch_check(Prec p, bool c12, hipStream_t s, const void *src, int V, int stride,
                        double *partials, double *out) {
    const int ntiles = (V + kTile - 1) / kTile;
    dim3 grid((ntiles + 3) / 4);
    if (p == P_F64)
        hipLaunchKernelGGL((check_kernel<double, 9>), grid, dim3(256), 0, s, src, V, stride,
                           partials);
    else if (c12)
        hipLaunchKernelGGL((check_kernel<float, 6>), grid, dim3(256), 0, s, src, V, stride,
                           partials);
    else
        hipLaunchKernelGGL((check_kernel<float, 9>), grid, dim3(256), 0, s, src, V, stride,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_check_final(s, partials, ntiles, out);
}

hipError_t launch_ingest_batch(Prec p, bool c12, hipStream_t s, const void *srcs,
                               const CfgDesc *cfgs, const int *tile_start, int n_cfg, int n_tiles,
                               double *partials, double *out) {
    if (n_tiles <= 0) return hipSuccess;
    const double2 *const *sp = (const double2 *const *)srcs;
    if (p == P_F64)
        hipLaunchKernelGGL((ingest_batch_kernel<double, 9>), dim3(n_tiles), dim3(256), 0, s, sp,
                           cfgs, tile_start, n_cfg, n_tiles, partials);
    else if (c12)
        hipLaunchKernelGGL((ingest_batch_kernel<float, 6>), dim3(n_tiles), dim3(256), 0, s, sp,
                           cfgs, tile_start, n_cfg, n_tiles, partials);
    else
        hipLaunchKernelGGL((ingest_batch_kernel<float, 9>), dim3(n_tiles), dim3(256), 0, s, sp,
                           cfgs, tile_start, n_cfg, n_tiles, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(check_batch_final_kernel, dim3(n_cfg), dim3(256), 0, s, partials,
                       tile_start, out);
    return hipGetLastError();
}

hipError_t launch_check_final(hipStream_t s, const double *partials, int ntiles, double *out) {
    hipLaunchKernelGGL(check_final_kernel, dim3(1), dim3(256), 0, s, partials, ntiles, out);
    return hipGetLastError();
}

hipError_t launch_slice_charge(Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs, int ci,
                               int dir, int n_slices, int slice_sites, double *partials,
                               double *out) {
    const int chunks = (slice_sites + 255) / 256;
    dim3 grid(chunks, n_slices);
    if (p == P_F64)
        hipLaunchKernelGGL((slice_charge_kernel<double, 9>), grid, dim3(256), 0, s, cfgs, ci, dir,
                           partials);
    else if (c12)
        hipLaunchKernelGGL((slice_charge_kernel<float, 6>), grid, dim3(256), 0, s, cfgs, ci, dir,
                           partials);
    else
        hipLaunchKernelGGL((slice_charge_kernel<float, 9>), grid, dim3(256), 0, s, cfgs, ci, dir,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(slice_finalize_kernel, dim3((n_slices + 63) / 64), dim3(64), 0, s, partials,
                       n_slices, chunks, out);
    return hipGetLastError();
}

hipError_t launch_densities(Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs, int ci, int V,
                            double *e_out, double *q_out) {
    dim3 grid((V + 255) / 256);
    if (p == P_F64)
        hipLaunchKernelGGL((density_kernel<double, 9>), grid, dim3(256), 0, s, cfgs, ci, e_out,
                           q_out);
    else if (c12)
        hipLaunchKernelGGL((density_kernel<float, 6>), grid, dim3(256), 0, s, cfgs, ci, e_out,
                           q_out);
    else
        hipLaunchKernelGGL((density_kernel<float, 9>), grid, dim3(256), 0, s, cfgs, ci, e_out,
                           q_out);
    return hipGetLastError();
}

hipError_t launch_fill_int(hipStream_t s, int *dst, int n, int value) {
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, void *dst, const void *src, size_t bytes) {
    size_t n = bytes / 16;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const float4 *)src,
                       (float4 *)dst, n);
    return hipGetLastError();
}

}  // namespace tgf
