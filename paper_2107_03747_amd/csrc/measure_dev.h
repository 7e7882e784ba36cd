// measure_dev.h -- device side of the measurement (arXiv 2107.03747,
// sec. 3.1 eq. gmunu and eq. qlatt): the clover field strength G_{mu nu}(n)
// from the four twisted leaves, its per-site energy and charge densities,
// the plaquette, FP64 wavefront sums and the fixed-order sum of per-tile
// partials.  Templated on the link accessor (any type with
// M3<R> operator()(int mu, int site)), so the same arithmetic serves the
// context's storage layouts and canonical caller links.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "lattice_dev.h"
#include "layout.h"
#include "su3_dev.h"

namespace tgf {

template <class R>
struct Herm {   // Hermitian 3x3: diag reals + upper off-diagonals
    R d[3];
    cx<R> o[3];   // 01, 02, 12
};

template <class R>
__device__ __forceinline__ R tr_herm2(const Herm<R> &a, const Herm<R> &b) {
    R s = a.d[0] * b.d[0] + a.d[1] * b.d[1] + a.d[2] * b.d[2];
    R o = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) o += a.o[k].x * b.o[k].x + a.o[k].y * b.o[k].y;
    return s + R(2) * o;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// rows 0,1 of U^+
template <class R>
__device__ __forceinline__ R2<R> r2_dag(const M3<R> &U) {
    R2<R> r;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) r.e[i][j] = cconj(U.e[j][i]);
    return r;
}

// A leaf (or a sum of leaves) C enters G only through K = C - C^+.  Leaves
// are carried in 9 reals: the raw form of su3_dev.h, k[0..5] = K01, K02, K12
// (complex), k[6] = Im C00 - Im C22, k[7] = Im C11 - Im C22 (the traceless
// part of K, on which conj_raw acts), and k[8] = Im Tr C, which conjugation
// leaves alone.

// 9-real form of a leaf L in SU(3) x Z_3 given by rows 0, 1 (row 2 =
// conj(row0 x row1)), after multiplying by z where twisted; returns Re Tr L.
template <class R>
__device__ __forceinline__ R leaf_raw9(R2<R> L, bool twisted, cx<R> z, R k[9]) {
    if (twisted) r2_scale(L, z);   // z in Z_3: z L is again in SU(3)
    const cx<R> *a = L.e[0], *b = L.e[1];
    r2_raw(L, k);
    // L22 = conj(a0 b1 - a1 b0)
    const R re22 = fma(a[0].x, b[1].x, fma(-a[0].y, b[1].y, fma(-a[1].x, b[0].x, a[1].y * b[0].y)));
    const R im22 = fma(-a[0].x, b[1].y, fma(-a[0].y, b[1].x, fma(a[1].x, b[0].y, a[1].y * b[0].x)));
    k[8] = a[0].y + b[1].y + im22;
    return a[0].x + b[1].x + re22;
}

// 9-real form of U^+ C U from that of C.
template <class R>
__device__ __forceinline__ void conj_raw9(const M3<R> &U, const R k[9], R out[9]) {
    conj_raw(U, k, out);
    out[8] = k[8];
}

// G = -(i/8) K of the leaf sum in 9-real form: G_aa = Im C_aa / 4,
// G_ab = -(i/8) K_ab.
template <class R>
__device__ __forceinline__ Herm<R> g_of_raw9(const R k[9]) {
    Herm<R> G;
    const R q = R(0.125), third = R(1.0 / 3.0);
    G.d[0] = R(0.25) * third * fma(R(2), k[6], k[8] - k[7]);
    G.d[1] = R(0.25) * third * fma(R(2), k[7], k[8] - k[6]);
    G.d[2] = R(0.25) * third * (k[8] - k[6] - k[7]);
#pragma unroll
    for (int t = 0; t < 3; t++) G.o[t] = {q * k[2 * t + 1], -q * k[2 * t]};
    return G;
}

// Clover G_{mu nu}(n) of eq. gmunu: -(i/8)(C - C^+), C the four leaves, each
// with Z^*_{mu nu} of its base site; also returns Re Tr of leaf 1 (the
// plaquette).  Leaves 2, 3 and 4 are plaquettes of the sites n - nu, n - mu
// and n - mu - nu carried to n: leaf 2 = U_nu(n-nu)^+ P(n-nu) U_nu(n-nu), and
// leaves 3 + 4 = U_mu(n-mu)^+ [leaf 1 + leaf 2](n-mu) U_mu(n-mu).  When lanes
// hold consecutive sites (tb = site of lane 0, nw active lanes; tb < 0: they
// do not) and every active lane finds site n - nu (n - mu) in the wave, the
// leaf sum of that site is taken from its lane and conjugated; otherwise the
// leaves are formed link by link.
template <class R, class LK>
__device__ __forceinline__ Herm<R> clover_G(const LK &W, const CfgDesc &c, const Geo &g, int mu,
                                            int nu, R &retr_plaq, int tb, int nw) {
    const int i = g.i;
    const int i_m = i + g.dn(mu), i_n = i + g.dn(nu);
    const int i_mn = i_m + g.dn(nu);
    const int k = twist_exp(c, mu, nu);
    const int nm = g.back(mu);
    const int nn = g.back(nu);
    const cx<R> zs = cconj(omega_pow<R>(k));
    R2<R> L;
    R s[9], t[9], u[9];
    // leaf 1: Z^*(n) U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
    L = r2_of(W(mu, i));
    L = r2_mul_nn(L, W(nu, i + g.up(mu)));
    L = r2_mul_nd(L, W(mu, i + g.up(nu)));
    L = r2_mul_nd(L, W(nu, i));
    retr_plaq = leaf_raw9(L, k && g.n(mu) == 0 && g.n(nu) == 0, zs, s);
    // leaf 2: Z^*(n-nu) U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu) U_mu(n)^+
    if (tb >= 0 && __all((unsigned)(i_n - tb) < (unsigned)nw)) {
#pragma unroll
        for (int x = 0; x < 9; x++) u[x] = __shfl(s[x], i_n - tb);
        conj_raw9(W(nu, i_n), u, t);
    } else {
        L = r2_dag(W(nu, i_n));
        L = r2_mul_nn(L, W(mu, i_n));
        L = r2_mul_nn(L, W(nu, i_n + g.up(mu)));
        L = r2_mul_nd(L, W(mu, i));
        leaf_raw9(L, k && g.n(mu) == 0 && nn == 0, zs, t);
    }
#pragma unroll
    for (int x = 0; x < 9; x++) s[x] += t[x];
    if (tb >= 0 && __all((unsigned)(i_m - tb) < (unsigned)nw)) {
        // leaves 3 + 4 from the leaf sum of site n - mu
#pragma unroll
        for (int x = 0; x < 9; x++) u[x] = __shfl(s[x], i_m - tb);
        conj_raw9(W(mu, i_m), u, t);
#pragma unroll
        for (int x = 0; x < 9; x++) s[x] += t[x];
    } else {
        // leaf 3: Z^*(n-mu) U_nu(n) U_mu(n-mu+nu)^+ U_nu(n-mu)^+ U_mu(n-mu)
        L = r2_of(W(nu, i));
        L = r2_mul_nd(L, W(mu, i_m + g.up(nu)));
        L = r2_mul_nd(L, W(nu, i_m));
        L = r2_mul_nn(L, W(mu, i_m));
        leaf_raw9(L, k && nm == 0 && g.n(nu) == 0, zs, t);
#pragma unroll
        for (int x = 0; x < 9; x++) s[x] += t[x];
        // leaf 4: Z^*(n-mu-nu) U_mu(n-mu)^+ U_nu(n-mu-nu)^+ U_mu(n-mu-nu) U_nu(n-nu)
        L = r2_dag(W(mu, i_m));
        L = r2_mul_nd(L, W(nu, i_mn));
        L = r2_mul_nn(L, W(mu, i_mn));
        L = r2_mul_nn(L, W(nu, i_n));
        leaf_raw9(L, k && nm == 0 && nn == 0, zs, t);
#pragma unroll
        for (int x = 0; x < 9; x++) s[x] += t[x];
    }
    return g_of_raw9(s);
}

// Measurement: a work-group is one tile of 64 sites x the three dual plane
// pairs (01,23), (02,13), (03,12); wave w computes the two clovers of pair w,
// their e(n), plaquette and action densities and the pair's term of
// q(n) = (1/4 pi^2)[Tr G01 G23 - Tr G02 G13 + Tr G03 G12], reduced in FP64
// over the wave into partials[tile][pair][4].
template <class R, int PAIR, class LK>
__device__ __forceinline__ void measure_pair(const LK &W, const CfgDesc &c, const Geo &g,
                                             double out[4], int tb = -1, int nw = 0) {
    constexpr int a0 = 0, a1 = PAIR + 1;                       // (0,1) (0,2) (0,3)
    constexpr int b0 = PAIR == 0 ? 2 : 1;
    constexpr int b1 = PAIR == 2 ? 2 : 3;                      // (2,3) (1,3) (1,2)
    R p1, p2;
    Herm<R> Ga = clover_G<R>(W, c, g, a0, a1, p1, tb, nw);
    Herm<R> Gb = clover_G<R>(W, c, g, b0, b1, p2, tb, nw);
    const R x = tr_herm2(Ga, Gb);
    out[0] = (double)(tr_herm2(Ga, Ga) + tr_herm2(Gb, Gb));
    out[1] = (double)(PAIR == 1 ? -x : x) * (1.0 / (4.0 * M_PI * M_PI));
    out[2] = (double)(p1 + p2);
    out[3] = (double)((R(3) - p1) + (R(3) - p2));
}

// Fixed-order sum of the (tile, pair) partials [t0, t1) of one configuration
// (4 doubles each: e, q, plaquette, action) by a 256-thread work-group:
// strided per-thread sums, wavefront sums, then the four waves in a fixed
// order.  Valid in thread 0.
__device__ __forceinline__ void sum_tile_partials(const double *__restrict__ partials, int t0,
                                                  int t1, double tot[4]) {
    double acc[4] = {0, 0, 0, 0};
    for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 4; k++) acc[k] += partials[(size_t)t * 4 + k];
    }
    __shared__ double red[4][4];
#pragma unroll
    for (int k = 0; k < 4; k++) acc[k] = wave_sum(acc[k]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 4; k++) red[w][k] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; k++) tot[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
}

}  // namespace tgf
