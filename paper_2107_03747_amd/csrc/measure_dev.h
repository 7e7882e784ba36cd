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

// C += z L for a leaf L in SU(3) given by rows 0,1 (row 2 = conj(row0 x row1));
// returns Re Tr(z L).
template <class R>
__device__ __forceinline__ R acc_leaf(M3<R> &C, R2<R> L, bool twisted, cx<R> z) {
    if (twisted) r2_scale(L, z);   // z in Z_3: z L is again in SU(3)
    M3<R> F = r2_full(L);
    m_acc(C, F);
    return F.e[0][0].x + F.e[1][1].x + F.e[2][2].x;
}

// Clover G_{mu nu}(n) of eq. gmunu: -(i/8)(C - C^+), C the four leaves, each
// with Z^*_{mu nu} of its base site; also returns Re Tr of leaf 1 (the plaquette).
template <class R, class LK>
__device__ __forceinline__ Herm<R> clover_G(const LK &W, const CfgDesc &c, const Geo &g, int mu,
                                            int nu, R &retr_plaq) {
    const int i = g.i;
    const int i_m = i + g.dn(mu), i_n = i + g.dn(nu);
    const int i_mn = i_m + g.dn(nu);
    const int k = twist_exp(c, mu, nu);
    const int nm = g.back(mu);
    const int nn = g.back(nu);
    const cx<R> zs = cconj(omega_pow<R>(k));
    M3<R> C;
    m_zero(C);
    R2<R> L;
    // leaf 1: Z^*(n) U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+
    L = r2_of(W(mu, i));
    L = r2_mul_nn(L, W(nu, i + g.up(mu)));
    L = r2_mul_nd(L, W(mu, i + g.up(nu)));
    L = r2_mul_nd(L, W(nu, i));
    retr_plaq = acc_leaf(C, L, k && g.n(mu) == 0 && g.n(nu) == 0, zs);
    // leaf 2: Z^*(n-nu) U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu) U_mu(n)^+
    L = r2_dag(W(nu, i_n));
    L = r2_mul_nn(L, W(mu, i_n));
    L = r2_mul_nn(L, W(nu, i_n + g.up(mu)));
    L = r2_mul_nd(L, W(mu, i));
    acc_leaf(C, L, k && g.n(mu) == 0 && nn == 0, zs);
    // leaf 3: Z^*(n-mu) U_nu(n) U_mu(n-mu+nu)^+ U_nu(n-mu)^+ U_mu(n-mu)
    L = r2_of(W(nu, i));
    L = r2_mul_nd(L, W(mu, i_m + g.up(nu)));
    L = r2_mul_nd(L, W(nu, i_m));
    L = r2_mul_nn(L, W(mu, i_m));
    acc_leaf(C, L, k && nm == 0 && g.n(nu) == 0, zs);
    // leaf 4: Z^*(n-mu-nu) U_mu(n-mu)^+ U_nu(n-mu-nu)^+ U_mu(n-mu-nu) U_nu(n-nu)
    L = r2_dag(W(mu, i_m));
    L = r2_mul_nd(L, W(nu, i_mn));
    L = r2_mul_nn(L, W(mu, i_mn));
    L = r2_mul_nn(L, W(nu, i_n));
    acc_leaf(C, L, k && nm == 0 && nn == 0, zs);
    // G = -(i/8)(C - C^+)
    Herm<R> G;
    const R q = R(0.125);
#pragma unroll
    for (int a = 0; a < 3; a++) G.d[a] = R(2) * q * C.e[a][a].y;
    const int ia[3] = {0, 0, 1}, ib[3] = {1, 2, 2};
#pragma unroll
    for (int t = 0; t < 3; t++) {
        cx<R> u = C.e[ia[t]][ib[t]], v = C.e[ib[t]][ia[t]];
        // C_ab - conj(C_ba), times -i/8
        R dr = u.x - v.x, di = u.y + v.y;
        G.o[t] = {q * di, -q * dr};
    }
    return G;
}

// Measurement: a work-group is one tile of 64 sites x the three dual plane
// pairs (01,23), (02,13), (03,12); wave w computes the two clovers of pair w,
// their e(n), plaquette and action densities and the pair's term of
// q(n) = (1/4 pi^2)[Tr G01 G23 - Tr G02 G13 + Tr G03 G12], reduced in FP64
// over the wave into partials[tile][pair][4].
template <class R, int PAIR, class LK>
__device__ __forceinline__ void measure_pair(const LK &W, const CfgDesc &c, const Geo &g,
                                             double out[4]) {
    constexpr int a0 = 0, a1 = PAIR + 1;                       // (0,1) (0,2) (0,3)
    constexpr int b0 = PAIR == 0 ? 2 : 1;
    constexpr int b1 = PAIR == 2 ? 2 : 3;                      // (2,3) (1,3) (1,2)
    R p1, p2;
    Herm<R> Ga = clover_G<R>(W, c, g, a0, a1, p1);
    Herm<R> Gb = clover_G<R>(W, c, g, b0, b1, p2);
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
