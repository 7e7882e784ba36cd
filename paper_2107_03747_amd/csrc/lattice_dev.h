// lattice_dev.h -- device-side building blocks shared by the flow and the
// Monte Carlo kernels: global-address-space accessors of the link storage,
// site geometry, twist factors, link loads/stores, FP64 reunitarisation and
// the twisted plaquettes and staples of the Wilson action (arXiv 2107.03747,
// sec. 3.1).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "layout.h"
#include "su3_dev.h"

namespace tgf {

constexpr int kTile = 64;

// Pointers into the workspace in the global address space: loads and stores
// become global_* instructions with a uniform (SGPR) base and a 32-bit
// per-lane offset, instead of flat instructions with 64-bit per-lane addresses.
// The element type is a built-in two-lane vector (re, im) with the size and
// alignment of cx<R>, so a complex number moves with one 8- or 16-byte access.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class R>
using v2 = R __attribute__((ext_vector_type(2)));

template <class R>
__device__ __forceinline__ gptr<v2<R>> as_global(void *p) {
    return (gptr<v2<R>>)p;
}
template <class R>
__device__ __forceinline__ gptr<const v2<R>> as_global(const void *p) {
    return (gptr<const v2<R>>)p;
}
// Element k of an entry plane: `plane` is uniform (one SGPR pair), the lane
// part is a 32-bit byte offset, so the access is a single global_load/store
// with an SGPR base and a VGPR offset (sites per configuration are capped so
// that every offset fits in 32 bits).
template <class R>
__device__ __forceinline__ unsigned lane_off(int i) {
    return (unsigned)i * (unsigned)sizeof(v2<R>);
}
template <class R>
__device__ __forceinline__ cx<R> ld(gptr<const v2<R>> plane, unsigned off) {
    const v2<R> v = *(gptr<const v2<R>>)((gptr<const char>)plane + off);
    return {v.x, v.y};
}
template <class R>
__device__ __forceinline__ cx<R> ld(gptr<v2<R>> plane, unsigned off) {
    const v2<R> v = *(gptr<const v2<R>>)((gptr<const char>)plane + off);
    return {v.x, v.y};
}
template <class R>
__device__ __forceinline__ void st(gptr<v2<R>> plane, unsigned off, cx<R> z) {
    v2<R> v;
    v.x = z.x;
    v.y = z.y;
    *(gptr<v2<R>>)((gptr<char>)plane + off) = v;
}

// Non-temporal (streaming) stores and loads for data that no other lane of
// the same launch touches again: link and accumulator outputs, accumulator
// inputs.  They keep the per-XCD L2 for the neighbour links that are re-read
// (stage launch with LDS staging: FP32 12-real -3%, FP64 -6%).
template <class T>
__device__ __forceinline__ void st_stream(gptr<T> p, T v) {
    __builtin_nontemporal_store(v, p);
}
template <class T>
__device__ __forceinline__ T ld_stream(gptr<const T> p) {
    return __builtin_nontemporal_load(p);
}
template <class R>
__device__ __forceinline__ void st_nt(gptr<v2<R>> plane, unsigned off, cx<R> z) {
    v2<R> v;
    v.x = z.x;
    v.y = z.y;
    st_stream((gptr<v2<R>>)((gptr<char>)plane + off), v);
}
template <class R>
__device__ __forceinline__ cx<R> ld_nt(gptr<const v2<R>> plane, unsigned off) {
    const v2<R> v = ld_stream((gptr<const v2<R>>)((gptr<const char>)plane + off));
    return {v.x, v.y};
}

// ---------------------------------------------------------------------------
// geometry

struct Geo {
    // scalar members (no arrays), so a runtime direction index never turns
    // the struct into addressable private or LDS memory
    int d0, d1, d2, d3;
    int s1, s2, s3;       // index strides (s0 = 1)
    int n0, n1, n2, n3;   // coordinates of this site
    int i;                // site index
    __host__ __device__ __forceinline__ int d(int mu) const {
        return mu == 0 ? d0 : (mu == 1 ? d1 : (mu == 2 ? d2 : d3));
    }
    __host__ __device__ __forceinline__ int s(int mu) const {
        return mu == 0 ? 1 : (mu == 1 ? s1 : (mu == 2 ? s2 : s3));
    }
    __host__ __device__ __forceinline__ int n(int mu) const {
        return mu == 0 ? n0 : (mu == 1 ? n1 : (mu == 2 ? n2 : n3));
    }
    __host__ __device__ __forceinline__ int up(int mu) const {        // delta to n + mu
        return n(mu) == d(mu) - 1 ? -(d(mu) - 1) * s(mu) : s(mu);
    }
    __host__ __device__ __forceinline__ int dn(int mu) const {        // delta to n - mu
        return n(mu) == 0 ? (d(mu) - 1) * s(mu) : -s(mu);
    }
    __host__ __device__ __forceinline__ int back(int mu) const {      // coordinate n_mu - 1 (periodic)
        return n(mu) == 0 ? d(mu) - 1 : n(mu) - 1;
    }
};

__host__ __device__ __forceinline__ Geo make_geo(const CfgDesc &c, int i) {
    Geo g;
    g.i = i;
    g.d0 = c.d[0]; g.d1 = c.d[1]; g.d2 = c.d[2]; g.d3 = c.d[3];
    g.s1 = c.d[0];
    g.s2 = c.d[0] * c.d[1];
    g.s3 = g.s2 * c.d[2];
    int r = i;
    g.n0 = r % c.d[0]; r /= c.d[0];
    g.n1 = r % c.d[1]; r /= c.d[1];
    g.n2 = r % c.d[2];
    g.n3 = r / c.d[2];
    return g;
}

__host__ __device__ __forceinline__ int plane_index(int mu, int nu) {
    // (0,1)->0 (0,2)->1 (0,3)->2 (1,2)->3 (1,3)->4 (2,3)->5, mu < nu
    return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5);
}

// twist exponent of Z_{mu nu} (antisymmetric mod 3)
__device__ __forceinline__ int twist_exp(const CfgDesc &c, int mu, int nu) {
    if (mu < nu) return c.tw[plane_index(mu, nu)];
    int t = c.tw[plane_index(nu, mu)];
    return t ? 3 - t : 0;
}

// omega^k, omega = exp(2 pi i / 3)
template <class R>
__device__ __forceinline__ cx<R> omega_pow(int k) {
    const R h = R(0.86602540378443864676);
    if (k == 1) return {R(-0.5), h};
    if (k == 2) return {R(-0.5), -h};
    return {R(1), R(0)};
}

template <class R>
__device__ __forceinline__ void m_scale(M3<R> &A, cx<R> z) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) A.e[i][j] = cmul(z, A.e[i][j]);
}

// XCD-contiguous block order: the hardware deals consecutive work-groups to
// the eight XCDs in turn, so block b runs on XCD b mod 8; mapping it to
// logical block (b mod 8) * per + b / 8 gives each XCD (and its L2) one
// contiguous range of tiles.  The grid is padded to 8 * per blocks.
__host__ __device__ __forceinline__ int remap_block(int b, int nb, int xcd) {
    if (!xcd) return b;
    int per = (nb + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

// wave-uniform: which config (exec order) holds tile t (also the block
// table of the LDS-staged variants)
__host__ __device__ __forceinline__ int find_cfg(const int *__restrict__ tile_start, int n, int t) {
    int lo = 0, hi = n;   // tile_start[lo] <= t < tile_start[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Launch order of a configuration's LDS-staged work-groups: its j-th
// work-group takes block block_order(j, c), the sites blk * block_order(j, c)
// onwards.  In site order (c.chunk = 0) a block's neighbours in direction 3
// are d0 d1 d2 / blk blocks away; on large boxes that is more work-groups
// than an XCD holds at a time, so the neighbour links have left its L2 when
// they are read.  There the n3 slices are cut into columns of c.chunk blocks
// (along n2) and each column is walked through all n3 before the next: the
// direction-3 neighbours are c.chunk blocks away.  A one-to-one map of
// 0 .. V/blk - 1; needs d0 d1 d2 to be a multiple of blk * c.chunk.
__host__ __device__ __forceinline__ int block_order(int j, const CfgDesc &c) {
    if (!c.chunk) return j;
    const int slice = c.d[0] * c.d[1] * c.d[2] / c.blk;   // blocks per n3 slice
    const int col = c.chunk * c.d[3];                     // blocks per column
    const int k = j / col, r = j - k * col;
    const int n3 = r / c.chunk;
    return n3 * slice + k * c.chunk + (r - n3 * c.chunk);
}

// A wave-uniform pointer taken through readfirstlane: the result is known to
// be uniform (an SGPR pair) and opaque to re-association, so that
// `sgpr_base(uniform) + lane offset` stays a global access with an SGPR base
// and a 32-bit VGPR offset instead of 64-bit per-lane pointer arithmetic.
// The argument must be the same in every active lane.
template <class T>
__device__ __forceinline__ gptr<T> sgpr_base(gptr<T> p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (gptr<T>)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
// A per-lane 32-bit offset re-materialised where it is used, so that the
// instruction selector sees `SGPR base + zero-extended 32-bit offset` in the
// same block as the access (a copy hoisted into another block arrives as a
// 64-bit value and forces 64-bit address arithmetic).
__device__ __forceinline__ unsigned lane_here(unsigned off) {
    asm volatile("" : "+v"(off));
    return off;
}

// ---------------------------------------------------------------------------
// link storage: [mu][entry][stride] complex
//
// PIN (FP64): every entry plane's base goes through sgpr_base and the lane
// offset through lane_here, so every access uses SGPR-base addressing.  The
// Monte Carlo kernel uses it (+6% link updates/s from fewer 64-bit address
// operations); the flow kernels measured equal or up to 2.5% slower with it
// and keep the plain form.

template <class R, int NE, bool PIN = false>
struct Links {
    gptr<const v2<R>> p;
    int stride;
    __device__ __forceinline__ M3<R> own(int mu, int i) const { return (*this)(mu, i); }
    __device__ __forceinline__ M3<R> operator()(int mu, int i) const {
        M3<R> U;
        if constexpr (PIN && sizeof(R) == 8) {
            gptr<const v2<R>> q = p + (size_t)(mu * NE) * stride;
            const unsigned u = lane_here(lane_off<R>(i));
#pragma unroll
            for (int e = 0; e < NE; e++) U.e[e / 3][e % 3] = ld(sgpr_base(q + (size_t)e * stride), u);
            if constexpr (NE == 6) rebuild_row2(U);
        } else if constexpr (sizeof(R) == 4) {
            // entry pairs: three (12-real) or four 16-byte loads, and for the
            // full storage entry 8 alone (entry_index)
            typedef R R4 __attribute__((ext_vector_type(4)));
            gptr<const char> q = (gptr<const char>)(p + (size_t)(mu * NE) * stride);
            const unsigned u = (unsigned)i * 16u;
            const size_t pl = (size_t)stride * 16u;
            const R4 a = *(gptr<const R4>)(q + u);
            const R4 b = *(gptr<const R4>)(q + pl + u);
            const R4 c = *(gptr<const R4>)(q + 2 * pl + u);
            U.e[0][0] = {a.x, a.y};
            U.e[0][1] = {a.z, a.w};
            U.e[0][2] = {b.x, b.y};
            U.e[1][0] = {b.z, b.w};
            U.e[1][1] = {c.x, c.y};
            U.e[1][2] = {c.z, c.w};
            if constexpr (NE == 9) {
                const R4 d = *(gptr<const R4>)(q + 3 * pl + u);
                U.e[2][0] = {d.x, d.y};
                U.e[2][1] = {d.z, d.w};
                U.e[2][2] = ld(p + (size_t)(mu * 9 + 8) * stride, lane_off<R>(i));
            } else {
                rebuild_row2(U);
            }
        } else {
            // entry planes are uniform bases, the site index the lane offset
            gptr<const v2<R>> q = p + (size_t)(mu * NE) * stride;
            const unsigned u = lane_off<R>(i);
            U.e[0][0] = ld(q, u);
            U.e[0][1] = ld(q + (size_t)stride, u);
            U.e[0][2] = ld(q + (size_t)2 * stride, u);
            U.e[1][0] = ld(q + (size_t)3 * stride, u);
            U.e[1][1] = ld(q + (size_t)4 * stride, u);
            U.e[1][2] = ld(q + (size_t)5 * stride, u);
            if constexpr (NE == 9) {
                U.e[2][0] = ld(q + (size_t)6 * stride, u);
                U.e[2][1] = ld(q + (size_t)7 * stride, u);
                U.e[2][2] = ld(q + (size_t)8 * stride, u);
            } else {
                rebuild_row2(U);
            }
        }
        return U;
    }
};

template <class R, int NE, bool PIN = false>
__device__ __forceinline__ void store_link(gptr<v2<R>> p, int stride, int mu, int i,
                                           const M3<R> &U) {
    if constexpr (PIN && sizeof(R) == 8) {
        gptr<v2<R>> q = p + (size_t)(mu * NE) * stride;
        const unsigned u = lane_here(lane_off<R>(i));
#pragma unroll
        for (int e = 0; e < NE; e++) st_nt(sgpr_base(q + (size_t)e * stride), u, U.e[e / 3][e % 3]);
        return;
    } else if constexpr (sizeof(R) == 4) {
        typedef R R4 __attribute__((ext_vector_type(4)));
        gptr<char> q = (gptr<char>)(p + (size_t)(mu * NE) * stride);
        const unsigned u = (unsigned)i * 16u;
        const size_t pl = (size_t)stride * 16u;
        R4 a, b, c;
        a.x = U.e[0][0].x; a.y = U.e[0][0].y; a.z = U.e[0][1].x; a.w = U.e[0][1].y;
        b.x = U.e[0][2].x; b.y = U.e[0][2].y; b.z = U.e[1][0].x; b.w = U.e[1][0].y;
        c.x = U.e[1][1].x; c.y = U.e[1][1].y; c.z = U.e[1][2].x; c.w = U.e[1][2].y;
        st_stream((gptr<R4>)(q + u), a);
        st_stream((gptr<R4>)(q + pl + u), b);
        st_stream((gptr<R4>)(q + 2 * pl + u), c);
        if constexpr (NE == 9) {
            R4 d;
            d.x = U.e[2][0].x; d.y = U.e[2][0].y; d.z = U.e[2][1].x; d.w = U.e[2][1].y;
            st_stream((gptr<R4>)(q + 3 * pl + u), d);
            const v2<R> e8 = {U.e[2][2].x, U.e[2][2].y};
            st_stream((gptr<v2<R>>)((gptr<char>)(p + (size_t)(mu * 9 + 8) * stride) + lane_off<R>(i)),
                      e8);
        }
        return;
    } else {
        gptr<v2<R>> q = p + (size_t)(mu * NE) * stride;
        const unsigned u = lane_off<R>(i);
        st_nt(q, u, U.e[0][0]);
        st_nt(q + (size_t)stride, u, U.e[0][1]);
        st_nt(q + (size_t)2 * stride, u, U.e[0][2]);
        st_nt(q + (size_t)3 * stride, u, U.e[1][0]);
        st_nt(q + (size_t)4 * stride, u, U.e[1][1]);
        st_nt(q + (size_t)5 * stride, u, U.e[1][2]);
        if constexpr (NE == 9) {
            st_nt(q + (size_t)6 * stride, u, U.e[2][0]);
            st_nt(q + (size_t)7 * stride, u, U.e[2][1]);
            st_nt(q + (size_t)8 * stride, u, U.e[2][2]);
        }
    }
}

// The 8 reals of an su(3) element in a buffer of records [record][4 complex]
// [site] (the RK accumulator X, the plaquette algebra A).  FP32 pairs the
// complex slots, [record][2][site][4 reals], so the record moves with two
// 16-byte accesses; FP64 keeps four 16-byte planes.
template <class R, bool NT = true>
__device__ __forceinline__ void ld_alg8(gptr<const v2<R>> base, int rec, int stride, int i,
                                        R out[8]) {
    if constexpr (sizeof(R) == 4) {
        typedef R R4 __attribute__((ext_vector_type(4)));
        gptr<const char> q = (gptr<const char>)(base + (size_t)(rec * 4) * stride);
        const unsigned u = (unsigned)i * 16u;
        gptr<const R4> pa = (gptr<const R4>)(q + u);
        gptr<const R4> pb = (gptr<const R4>)(q + (size_t)stride * 16u + u);
        R4 a, b;
        if constexpr (NT) {
            a = ld_stream(pa);
            b = ld_stream(pb);
        } else {
            a = *pa;
            b = *pb;
        }
        out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
        out[4] = b.x; out[5] = b.y; out[6] = b.z; out[7] = b.w;
    } else {
        gptr<const v2<R>> q = base + (size_t)(rec * 4) * stride;
        const unsigned u = lane_off<R>(i);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const cx<R> v = NT ? ld_nt(q + (size_t)t * stride, u) : ld(q + (size_t)t * stride, u);
            out[2 * t] = v.x;
            out[2 * t + 1] = v.y;
        }
    }
}

template <class R>
__device__ __forceinline__ void st_alg8(gptr<v2<R>> base, int rec, int stride, int i,
                                        const R v[8]) {
    if constexpr (sizeof(R) == 4) {
        typedef R R4 __attribute__((ext_vector_type(4)));
        gptr<char> q = (gptr<char>)(base + (size_t)(rec * 4) * stride);
        const unsigned u = (unsigned)i * 16u;
        R4 a, b;
        a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
        b.x = v[4]; b.y = v[5]; b.z = v[6]; b.w = v[7];
        st_stream((gptr<R4>)(q + u), a);
        st_stream((gptr<R4>)(q + (size_t)stride * 16u + u), b);
    } else {
        gptr<v2<R>> q = base + (size_t)(rec * 4) * stride;
        const unsigned u = lane_off<R>(i);
#pragma unroll
        for (int t = 0; t < 4; t++) st_nt(q + (size_t)t * stride, u, cx<R>{v[2 * t], v[2 * t + 1]});
    }
}

// FP64 reunitarisation: normalise row 0, orthogonalise and normalise row 1,
// row 2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void reunitarise(M3<R> &U) {
    double a[3][2], b[3][2];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        a[k][0] = (double)U.e[0][k].x; a[k][1] = (double)U.e[0][k].y;
        b[k][0] = (double)U.e[1][k].x; b[k][1] = (double)U.e[1][k].y;
    }
    double na = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) na += a[k][0] * a[k][0] + a[k][1] * a[k][1];
    na = 1.0 / sqrt(na);
#pragma unroll
    for (int k = 0; k < 3; k++) { a[k][0] *= na; a[k][1] *= na; }
    double dr = 0, di = 0;   // conj(a) . b
#pragma unroll
    for (int k = 0; k < 3; k++) {
        dr += a[k][0] * b[k][0] + a[k][1] * b[k][1];
        di += a[k][0] * b[k][1] - a[k][1] * b[k][0];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        b[k][0] -= dr * a[k][0] - di * a[k][1];
        b[k][1] -= dr * a[k][1] + di * a[k][0];
    }
    double nb = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) nb += b[k][0] * b[k][0] + b[k][1] * b[k][1];
    nb = 1.0 / sqrt(nb);
#pragma unroll
    for (int k = 0; k < 3; k++) { b[k][0] *= nb; b[k][1] *= nb; }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        // (a x b)_k = a_k1 b_k2 - a_k2 b_k1, then conjugate
        double cr = a[k1][0] * b[k2][0] - a[k1][1] * b[k2][1] - (a[k2][0] * b[k1][0] - a[k2][1] * b[k1][1]);
        double ci = a[k1][0] * b[k2][1] + a[k1][1] * b[k2][0] - (a[k2][0] * b[k1][1] + a[k2][1] * b[k1][0]);
        U.e[0][k] = {(R)a[k][0], (R)a[k][1]};
        U.e[1][k] = {(R)b[k][0], (R)b[k][1]};
        U.e[2][k] = {(R)cr, (R)(-ci)};
    }
}

// ---------------------------------------------------------------------------
// staples

// Upper plaquette P_{mu nu}(n) = U_mu(n) U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+,
// multiplied by its twist factor Z^*_{mu nu}(n).
template <class R, int NE, bool PN>
__device__ __forceinline__ M3<R> upper_plaq(const Links<R, NE, PN> &W, const CfgDesc &c,
                                            const Geo &g, int mu, int nu) {
    // P is in SU(3): rows 0,1 by two-row products, row 2 = conj(row0 x row1)
    R2<R> A = r2_of(W(mu, g.i));
    A = r2_mul_nn(A, W(nu, g.i + g.up(mu)));
    A = r2_mul_nd(A, W(mu, g.i + g.up(nu)));
    A = r2_mul_nd(A, W(nu, g.i));
    M3<R> P = r2_full(A);
    int k = twist_exp(c, mu, nu);
    if (k && g.n(mu) == 0 && g.n(nu) == 0) m_scale(P, cconj(omega_pow<R>(k)));
    return P;
}

// Upper staple U_nu(n+mu) U_mu(n+nu)^+ U_nu(n)^+ times Z^*_{mu nu}(n).
template <class R, int NE, bool PN>
__device__ __forceinline__ M3<R> upper_staple(const Links<R, NE, PN> &W, const CfgDesc &c,
                                              const Geo &g, int mu, int nu) {
    M3<R> A = mul_nd(W(nu, g.i + g.up(mu)), W(mu, g.i + g.up(nu)));
    A = mul_nd(A, W(nu, g.i));
    int k = twist_exp(c, mu, nu);
    if (k && g.n(mu) == 0 && g.n(nu) == 0) m_scale(A, cconj(omega_pow<R>(k)));
    return A;
}

// Lower staple U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu) times Z_{mu nu}(n-nu):
// the plaquette P_{mu nu}(n-nu) enters the action with Z^*, and it contains
// U_mu(n)^+, so its contribution to Omega_mu(n) is the adjoint.
template <class R, int NE, bool PN>
__device__ __forceinline__ M3<R> lower_staple(const Links<R, NE, PN> &W, const CfgDesc &c,
                                              const Geo &g, int mu, int nu) {
    int imn = g.i + g.dn(nu);
    M3<R> T = mul_nn(W(mu, imn), W(nu, imn + g.up(mu)));
    M3<R> L = mul_dn(T, W(nu, imn));
    int k = twist_exp(c, mu, nu);
    int nnu = g.back(nu);
    if (k && g.n(mu) == 0 && nnu == 0) m_scale(L, omega_pow<R>(k));
    return L;
}

// S += Z_{mu nu}(n-nu) U_nu(n+mu-nu)^+ U_mu(n-nu)^+ U_nu(n-nu), accumulated in
// place; the twist factor is folded into T = U_mu(n-nu) U_nu(n+mu-nu) as
// z T^+ U = (conj(z) T)^+ U, so twisted and untwisted lanes run the same code.
template <class R, class LK>
__device__ __forceinline__ void acc_lower_staple(M3<R> &S, const LK &W,
                                                 const CfgDesc &c, const Geo &g, int mu, int nu) {
    const int imn = g.i + g.dn(nu);
    M3<R> T = mul_nn(W(mu, imn), W(nu, imn + g.up(mu)));
    const int k = twist_exp(c, mu, nu);
    if (k && g.n(mu) == 0 && g.back(nu) == 0) m_scale(T, cconj(omega_pow<R>(k)));
    m_acc_mul_dn(S, T, W(nu, imn));
}

}  // namespace tgf
