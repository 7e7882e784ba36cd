// su3_dev.h -- device SU(3) arithmetic for the twisted Wilson flow (gfx950).
//
// Complex numbers are {re, im} pairs of R = float or double.  A link is kept
// in registers as a full 3x3 matrix; in memory it is structure-of-arrays
// (see layout.h).  Products are written out with fused multiply-adds; the
// compiler keeps them in scalar (non-packed) FP32/FP64 VALU instructions.
#pragma once

#include <hip/hip_runtime.h>

namespace tgf {

template <class R>
struct alignas(2 * sizeof(R)) cx {
    R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> cmake(R x, R y) { return {x, y}; }

template <class R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }

template <class R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }

template <class R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.x, -a.y}; }

template <class R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}

// acc + a*b
template <class R>
__device__ __forceinline__ cx<R> cmadd(cx<R> acc, cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}

// acc + a*conj(b)
template <class R>
__device__ __forceinline__ cx<R> cmadd_nc(cx<R> acc, cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y))};
}

// acc + conj(a)*b
template <class R>
__device__ __forceinline__ cx<R> cmadd_cn(cx<R> acc, cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y))};
}

// acc + conj(a)*conj(b)
template <class R>
__device__ __forceinline__ cx<R> cmadd_cc(cx<R> acc, cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(-a.x, b.y, fma(-a.y, b.x, acc.y))};
}

template <class R>
struct M3 {
    cx<R> e[3][3];
};

template <class R>
__device__ __forceinline__ void m_zero(M3<R> &a) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) a.e[i][j] = {R(0), R(0)};
}

// C = A B
template <class R>
__device__ __forceinline__ M3<R> mul_nn(const M3<R> &A, const M3<R> &B) {
    M3<R> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = cmul(A.e[i][0], B.e[0][j]);
            s = cmadd(s, A.e[i][1], B.e[1][j]);
            s = cmadd(s, A.e[i][2], B.e[2][j]);
            C.e[i][j] = s;
        }
    return C;
}

// C = A B^+
template <class R>
__device__ __forceinline__ M3<R> mul_nd(const M3<R> &A, const M3<R> &B) {
    M3<R> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = {R(0), R(0)};
            s = cmadd_nc(s, A.e[i][0], B.e[j][0]);
            s = cmadd_nc(s, A.e[i][1], B.e[j][1]);
            s = cmadd_nc(s, A.e[i][2], B.e[j][2]);
            C.e[i][j] = s;
        }
    return C;
}

// C = A^+ B
template <class R>
__device__ __forceinline__ M3<R> mul_dn(const M3<R> &A, const M3<R> &B) {
    M3<R> C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = {R(0), R(0)};
            s = cmadd_cn(s, A.e[0][i], B.e[0][j]);
            s = cmadd_cn(s, A.e[1][i], B.e[1][j]);
            s = cmadd_cn(s, A.e[2][i], B.e[2][j]);
            C.e[i][j] = s;
        }
    return C;
}

// acc += z * A
template <class R>
__device__ __forceinline__ void m_acc_scaled(M3<R> &acc, cx<R> z, const M3<R> &A) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) acc.e[i][j] = cmadd(acc.e[i][j], z, A.e[i][j]);
}

// acc += A^+ B  (the product accumulated straight into acc)
template <class R>
__device__ __forceinline__ void m_acc_mul_dn(M3<R> &acc, const M3<R> &A, const M3<R> &B) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = acc.e[i][j];
            s = cmadd_cn(s, A.e[0][i], B.e[0][j]);
            s = cmadd_cn(s, A.e[1][i], B.e[1][j]);
            s = cmadd_cn(s, A.e[2][i], B.e[2][j]);
            acc.e[i][j] = s;
        }
}

// acc += A B
template <class R>
__device__ __forceinline__ void m_acc_mul_nn(M3<R> &acc, const M3<R> &A, const M3<R> &B) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = acc.e[i][j];
            s = cmadd(s, A.e[i][0], B.e[0][j]);
            s = cmadd(s, A.e[i][1], B.e[1][j]);
            s = cmadd(s, A.e[i][2], B.e[2][j]);
            acc.e[i][j] = s;
        }
}

// acc += A
template <class R>
__device__ __forceinline__ void m_acc(M3<R> &acc, const M3<R> &A) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) acc.e[i][j] = cadd(acc.e[i][j], A.e[i][j]);
}

// acc += (z A)^+ = conj(z) A^+
template <class R>
__device__ __forceinline__ void m_acc_scaled_dag(M3<R> &acc, cx<R> z, const M3<R> &A) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) acc.e[i][j] = cmadd_cc(acc.e[i][j], z, A.e[j][i]);
}

// conj(aj bk - ak bj), one entry of a conjugated cross product, as one
// multiply and three fused multiply-adds per real part (the form with two
// complex products and a subtraction takes five).
template <class R>
__device__ __forceinline__ cx<R> cross_conj(cx<R> aj, cx<R> bk, cx<R> ak, cx<R> bj) {
    const R re = fma(aj.x, bk.x, fma(-aj.y, bk.y, fma(-ak.x, bj.x, ak.y * bj.y)));
    const R im = fma(-aj.x, bk.y, fma(-aj.y, bk.x, fma(ak.x, bj.y, ak.y * bj.x)));
    return {re, im};
}

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void rebuild_row2(M3<R> &U) {
    const cx<R> *a = U.e[0], *b = U.e[1];
    // (a x b)_0 = a1 b2 - a2 b1, (a x b)_1 = a2 b0 - a0 b2, (a x b)_2 = a0 b1 - a1 b0
    U.e[2][0] = cross_conj(a[1], b[2], a[2], b[1]);
    U.e[2][1] = cross_conj(a[2], b[0], a[0], b[2]);
    U.e[2][2] = cross_conj(a[0], b[1], a[1], b[0]);
}

// ---------------------------------------------------------------------------
// su(3) algebra element X (anti-Hermitian, traceless) as 8 reals:
//   a[0..1] = X01, a[2..3] = X02, a[4..5] = X12, a[6] = Im X00, a[7] = Im X11,
//   X10 = -conj(X01), ..., X22 = -i (a[6] + a[7]).
template <class R>
struct Alg {
    R a[8];
};

// Traceless anti-Hermitian part P_ah(M) = (M - M^+)/2 - Tr(M - M^+)/6, times s.
template <class R>
__device__ __forceinline__ Alg<R> proj_ah(const M3<R> &M, R s) {
    Alg<R> X;
    R h = R(0.5) * s;
    X.a[0] = h * (M.e[0][1].x - M.e[1][0].x);
    X.a[1] = h * (M.e[0][1].y + M.e[1][0].y);
    X.a[2] = h * (M.e[0][2].x - M.e[2][0].x);
    X.a[3] = h * (M.e[0][2].y + M.e[2][0].y);
    X.a[4] = h * (M.e[1][2].x - M.e[2][1].x);
    X.a[5] = h * (M.e[1][2].y + M.e[2][1].y);
    R tr3 = (M.e[0][0].y + M.e[1][1].y + M.e[2][2].y) * R(1.0 / 3.0);
    X.a[6] = s * (M.e[0][0].y - tr3);
    X.a[7] = s * (M.e[1][1].y - tr3);
    return X;
}

// ---------------------------------------------------------------------------
// Two-row arithmetic for products that stay in SU(3): rows 0 and 1 of a
// product are computed, the third row of an SU(3) matrix is conj(row0 x row1).

template <class R>
struct R2 {   // rows 0 and 1 of a 3x3 matrix
    cx<R> e[2][3];
};

// rows 0,1 of A B (A given by its rows 0,1)
template <class R>
__device__ __forceinline__ R2<R> r2_mul_nn(const R2<R> &A, const M3<R> &B) {
    R2<R> C;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = cmul(A.e[i][0], B.e[0][j]);
            s = cmadd(s, A.e[i][1], B.e[1][j]);
            s = cmadd(s, A.e[i][2], B.e[2][j]);
            C.e[i][j] = s;
        }
    return C;
}

// rows 0,1 of A B^+
template <class R>
__device__ __forceinline__ R2<R> r2_mul_nd(const R2<R> &A, const M3<R> &B) {
    R2<R> C;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = {R(0), R(0)};
            s = cmadd_nc(s, A.e[i][0], B.e[j][0]);
            s = cmadd_nc(s, A.e[i][1], B.e[j][1]);
            s = cmadd_nc(s, A.e[i][2], B.e[j][2]);
            C.e[i][j] = s;
        }
    return C;
}

template <class R>
__device__ __forceinline__ void r2_scale(R2<R> &A, cx<R> z) {
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) A.e[i][j] = cmul(z, A.e[i][j]);
}

// full SU(3) matrix from rows 0,1
template <class R>
__device__ __forceinline__ M3<R> r2_full(const R2<R> &A) {
    M3<R> U;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) U.e[i][j] = A.e[i][j];
    rebuild_row2(U);
    return U;
}

template <class R>
__device__ __forceinline__ R2<R> r2_of(const M3<R> &A) {
    R2<R> r;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) r.e[i][j] = A.e[i][j];
    return r;
}

// s * P_ah(P) for P in SU(3) given by rows 0,1; the entries of row 2 that the
// projection needs (P20, P21, Im P22) come from row2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void r2_proj_ah(const R2<R> &P, R s, R out[8]) {
    const cx<R> *a = P.e[0], *b = P.e[1];
    cx<R> p20 = cross_conj(a[1], b[2], a[2], b[1]);
    cx<R> p21 = cross_conj(a[2], b[0], a[0], b[2]);
    // Im P22 = -Im(a0 b1 - a1 b0)
    R im22 = fma(-a[0].x, b[1].y, fma(-a[0].y, b[1].x, fma(a[1].x, b[0].y, a[1].y * b[0].x)));
    R h = R(0.5) * s;
    out[0] = h * (a[1].x - b[0].x);
    out[1] = h * (a[1].y + b[0].y);
    out[2] = h * (a[2].x - p20.x);
    out[3] = h * (a[2].y + p20.y);
    out[4] = h * (b[2].x - p21.x);
    out[5] = h * (b[2].y + p21.y);
    R tr3 = (a[0].y + b[1].y + im22) * R(1.0 / 3.0);
    out[6] = s * (a[0].y - tr3);
    out[7] = s * (b[1].y - tr3);
}

// ---------------------------------------------------------------------------
// Raw anti-Hermitian form (8 reals) of the force terms.  For a matrix M,
//   k[0..5] = z01, z02, z12 with z_ij = M_ij - conj(M_ji)   (complex pairs),
//   k[6] = u = Im M_00 - Im M_22,   k[7] = v = Im M_11 - Im M_22,
// so that
//   P_ah(M) = { z_ij / 2 ;  diagonal i (2u - v)/3, i (2v - u)/3, -(sum) }.
// The form is linear in M and odd under M -> M^+, and the traceless part of
// M - M^+ is what conjugation by a unitary U acts on (conj_raw), so force
// terms are summed in it and halved and projected once per link
// (raw_to_alg) instead of once per term.

// Raw form of P in SU(3) (times a cube root of unity) given by rows 0, 1: the
// row-2 entries enter through row2 = conj(row0 x row1):
//   z02 = P02 - conj(P20) = a2 - (a1 b2 - a2 b1),
//   z12 = P12 - conj(P21) = b2 - (a2 b0 - a0 b2),
//   Im P22 = -Im(a0 b1 - a1 b0).
template <class R>
__device__ __forceinline__ void r2_raw(const R2<R> &P, R k[8]) {
    const cx<R> *a = P.e[0], *b = P.e[1];
    k[0] = a[1].x - b[0].x;
    k[1] = a[1].y + b[0].y;
    k[2] = fma(-a[1].x, b[2].x, fma(a[1].y, b[2].y, fma(a[2].x, b[1].x, fma(-a[2].y, b[1].y, a[2].x))));
    k[3] = fma(-a[1].x, b[2].y, fma(-a[1].y, b[2].x, fma(a[2].x, b[1].y, fma(a[2].y, b[1].x, a[2].y))));
    k[4] = fma(-a[2].x, b[0].x, fma(a[2].y, b[0].y, fma(a[0].x, b[2].x, fma(-a[0].y, b[2].y, b[2].x))));
    k[5] = fma(-a[2].x, b[0].y, fma(-a[2].y, b[0].x, fma(a[0].x, b[2].y, fma(a[0].y, b[2].x, b[2].y))));
    const R im22 = fma(-a[0].x, b[1].y, fma(-a[0].y, b[1].x, fma(a[1].x, b[0].y, a[1].y * b[0].x)));
    k[6] = a[0].y - im22;
    k[7] = b[1].y - im22;
}

// s * P_ah(M) in the 8-real su(3) form from the raw form of M.
template <class R>
__device__ __forceinline__ Alg<R> raw_to_alg(const R k[8], R s) {
    Alg<R> X;
    const R h = R(0.5) * s, t = s * R(1.0 / 3.0);
#pragma unroll
    for (int j = 0; j < 6; j++) X.a[j] = h * k[j];
    X.a[6] = t * fma(R(2), k[6], -k[7]);
    X.a[7] = t * fma(R(2), k[7], -k[6]);
    return X;
}

// Raw form of U^+ M U from the raw form k of M: with T the traceless part of
// M - M^+ (off-diagonals z_ij, diagonal 2i (2u - v)/3, 2i (2v - u)/3, ...),
// B = T U, C = U^+ B (upper off-diagonals and the first two diagonal entries;
// C is traceless, so Im C_22 = -(Im C_00 + Im C_11)).
template <class R>
__device__ __forceinline__ void conj_raw(const M3<R> &U, const R k[8], R c[8]) {
    const cx<R> x01 = {k[0], k[1]}, x02 = {k[2], k[3]}, x12 = {k[4], k[5]};
    const R w = R(2.0 / 3.0);
    const R d0 = w * fma(R(2), k[6], -k[7]), d1 = w * fma(R(2), k[7], -k[6]);
    const R d2 = -(d0 + d1);
    M3<R> B;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        cx<R> t = {-d0 * U.e[0][j].y, d0 * U.e[0][j].x};
        t = cmadd(t, x01, U.e[1][j]);
        t = cmadd(t, x02, U.e[2][j]);
        B.e[0][j] = t;
        t = {-d1 * U.e[1][j].y, d1 * U.e[1][j].x};
        t = cmadd(t, cx<R>{-x01.x, x01.y}, U.e[0][j]);
        t = cmadd(t, x12, U.e[2][j]);
        B.e[1][j] = t;
        t = {-d2 * U.e[2][j].y, d2 * U.e[2][j].x};
        t = cmadd(t, cx<R>{-x02.x, x02.y}, U.e[0][j]);
        t = cmadd(t, cx<R>{-x12.x, x12.y}, U.e[1][j]);
        B.e[2][j] = t;
    }
    const int ia[3] = {0, 0, 1}, ib[3] = {1, 2, 2};
#pragma unroll
    for (int t = 0; t < 3; t++) {
        cx<R> s = {R(0), R(0)};
#pragma unroll
        for (int m = 0; m < 3; m++) s = cmadd_cn(s, U.e[m][ia[t]], B.e[m][ib[t]]);
        c[2 * t] = s.x;
        c[2 * t + 1] = s.y;
    }
    R im[2];
#pragma unroll
    for (int d = 0; d < 2; d++) {
        R v = 0;
#pragma unroll
        for (int m = 0; m < 3; m++) v = fma(U.e[m][d].x, B.e[m][d].y, fma(-U.e[m][d].y, B.e[m][d].x, v));
        im[d] = v;
    }
    // u' = (Im C00 - Im C22)/2 = Im C00 + Im C11 / 2, v' = Im C11 + Im C00 / 2
    c[6] = fma(R(0.5), im[1], im[0]);
    c[7] = fma(R(0.5), im[0], im[1]);
}

// C = U^+ A U for A in su(3) (8-real form); the result is again in su(3).
template <class R>
__device__ __forceinline__ void conj_alg(const M3<R> &U, const R a[8], R c[8]) {
    // A as a matrix
    const cx<R> x01 = {a[0], a[1]}, x02 = {a[2], a[3]}, x12 = {a[4], a[5]};
    const R d0 = a[6], d1 = a[7], d2 = -(a[6] + a[7]);
    M3<R> B;   // B = A U
#pragma unroll
    for (int j = 0; j < 3; j++) {
        // row 0: i d0 U0j + x01 U1j + x02 U2j
        cx<R> t = {-d0 * U.e[0][j].y, d0 * U.e[0][j].x};
        t = cmadd(t, x01, U.e[1][j]);
        t = cmadd(t, x02, U.e[2][j]);
        B.e[0][j] = t;
        // row 1: -conj(x01) U0j + i d1 U1j + x12 U2j
        t = {-d1 * U.e[1][j].y, d1 * U.e[1][j].x};
        t = cmadd(t, cx<R>{-x01.x, x01.y}, U.e[0][j]);
        t = cmadd(t, x12, U.e[2][j]);
        B.e[1][j] = t;
        // row 2: -conj(x02) U0j - conj(x12) U1j + i d2 U2j
        t = {-d2 * U.e[2][j].y, d2 * U.e[2][j].x};
        t = cmadd(t, cx<R>{-x02.x, x02.y}, U.e[0][j]);
        t = cmadd(t, cx<R>{-x12.x, x12.y}, U.e[1][j]);
        B.e[2][j] = t;
    }
    // C = U^+ B: upper off-diagonals and Im of the first two diagonal entries
    const int ia[3] = {0, 0, 1}, ib[3] = {1, 2, 2};
#pragma unroll
    for (int t = 0; t < 3; t++) {
        cx<R> s = {R(0), R(0)};
#pragma unroll
        for (int k = 0; k < 3; k++) s = cmadd_cn(s, U.e[k][ia[t]], B.e[k][ib[t]]);
        c[2 * t] = s.x;
        c[2 * t + 1] = s.y;
    }
#pragma unroll
    for (int d = 0; d < 2; d++) {
        R im = 0;
#pragma unroll
        for (int k = 0; k < 3; k++) im = fma(U.e[k][d].x, B.e[k][d].y, fma(-U.e[k][d].y, B.e[k][d].x, im));
        c[6 + d] = im;
    }
}

template <class R>
struct ExpTol;
template <>
struct ExpTol<float> {
    static constexpr float tol = 1e-9f;
    static constexpr int kmax = 14;
};
template <>
struct ExpTol<double> {
    static constexpr double tol = 1e-18;
    static constexpr int kmax = 24;
};

// 1/k for the exponential series (k = 0 unused)
__device__ constexpr double kInvK[25] = {
    0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9,
    1.0 / 10, 1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17,
    1.0 / 18, 1.0 / 19, 1.0 / 20, 1.0 / 21, 1.0 / 22, 1.0 / 23, 1.0 / 24};

// exp(X) - 1 for X in su(3), by Cayley-Hamilton: with Q = -i X (Hermitian,
// traceless), Q^3 = c1 Q + c0 with c1 = Tr(Q^2)/2, c0 = det Q, so every power
// Q^k = alpha_k + beta_k Q + gamma_k Q^2 and exp(iQ) = f0 + f1 Q + f2 Q^2 with
// f_j the exponential series of the coefficient recursion
//   alpha' = gamma c0, beta' = alpha + gamma c1, gamma' = beta.
// The series runs until the remainder bound rho^k/k! (rho = ||Q||_F) drops
// below the working precision; for rho > 1 the argument is halved s times and
// the result squared s times ((1 + D)^2 - 1 = 2D + D^2).
//
// The identity is left out (f0 starts at 0) so that the caller can form
// exp(X) U as U + (D U) with one rounding per entry (mul_add_expm1).
// ROWS = 2 returns rows 0 and 1 only (enough to update a 12-real link),
// unless squarings are needed.
template <class R, int ROWS = 3>
__device__ __forceinline__ M3<R> su3_expm1(const Alg<R> &X) {
    // Q = -i X
    R q00 = X.a[6], q11 = X.a[7], q22 = -(X.a[6] + X.a[7]);
    cx<R> q01 = {X.a[1], -X.a[0]}, q02 = {X.a[3], -X.a[2]}, q12 = {X.a[5], -X.a[4]};
    R n01 = q01.x * q01.x + q01.y * q01.y;
    R n02 = q02.x * q02.x + q02.y * q02.y;
    R n12 = q12.x * q12.x + q12.y * q12.y;
    R fro2 = q00 * q00 + q11 * q11 + q22 * q22 + R(2) * (n01 + n02 + n12);

    int s = 0;
    if (fro2 > R(1)) {
        // halve until ||Q||_F <= 1
        R f = fro2;
        while (f > R(1) && s < 30) { f *= R(0.25); s++; }
        const R sc = ldexp(R(1), -s), sc2 = sc * sc;
        q00 *= sc; q11 *= sc; q22 *= sc;
        q01 = {q01.x * sc, q01.y * sc};
        q02 = {q02.x * sc, q02.y * sc};
        q12 = {q12.x * sc, q12.y * sc};
        n01 *= sc2; n02 *= sc2; n12 *= sc2;
        fro2 *= sc2;
    }
    const R c1 = R(0.5) * fro2;
    // det of a Hermitian 3x3: q00 q11 q22 + 2 Re(q01 q12 conj(q02)) - q00|q12|^2 - q11|q02|^2 - q22|q01|^2
    const cx<R> t = cmul(q01, q12);
    const R re3 = t.x * q02.x + t.y * q02.y;
    const R c0 = q00 * q11 * q22 + R(2) * re3 - q00 * n12 - q11 * n02 - q22 * n01;

    // series: term k holds alpha_k/k!, beta_k/k!, gamma_k/k!, weight i^k; the
    // k = 0 term (the identity) is not added
    R al = R(1), be = R(0), ga = R(0);
    cx<R> f0 = {R(0), R(0)}, f1 = {R(0), R(0)}, f2 = {R(0), R(0)};
    const R rho = sqrt(fro2);
    R bound = R(1);
#pragma unroll
    for (int k = 1; k <= ExpTol<R>::kmax; k++) {
        const R inv = (R)kInvK[k];
        bound = bound * rho * inv;
        const R nal = ga * c0 * inv;
        const R nbe = (al + ga * c1) * inv;
        const R nga = be * inv;
        al = nal; be = nbe; ga = nga;
        switch (k & 3) {
            case 0: f0.x += al; f1.x += be; f2.x += ga; break;
            case 1: f0.y += al; f1.y += be; f2.y += ga; break;
            case 2: f0.x -= al; f1.x -= be; f2.x -= ga; break;
            default: f0.y -= al; f1.y -= be; f2.y -= ga; break;
        }
        if (bound < ExpTol<R>::tol) break;
    }

    // Q^2 (Hermitian): diagonal and upper triangle
    const R s00 = q00 * q00 + n01 + n02;
    const R s11 = q11 * q11 + n01 + n12;
    const R s22 = q22 * q22 + n02 + n12;
    // (Q^2)_01 = q00 q01 + q01 q11 + q02 conj(q12)
    cx<R> s01 = {(q00 + q11) * q01.x, (q00 + q11) * q01.y};
    s01 = cmadd_nc(s01, q02, q12);
    // (Q^2)_02 = q00 q02 + q01 q12 + q02 q22
    cx<R> s02 = {(q00 + q22) * q02.x, (q00 + q22) * q02.y};
    s02 = cmadd(s02, q01, q12);
    // (Q^2)_12 = conj(q01) q02 + q11 q12 + q12 q22
    cx<R> s12 = {(q11 + q22) * q12.x, (q11 + q22) * q12.y};
    s12 = cmadd_cn(s12, q01, q02);

    // D = (f0 - 1) + f1 Q + f2 Q^2
    auto ent = [&](cx<R> q, cx<R> sq) { return cmadd(cmul(f1, q), f2, sq); };
    auto dia = [&](R q, R sq) {
        return cx<R>{f0.x + f1.x * q + f2.x * sq, f0.y + f1.y * q + f2.y * sq};
    };
    M3<R> D;
    D.e[0][0] = dia(q00, s00);
    D.e[0][1] = ent(q01, s01);
    D.e[0][2] = ent(q02, s02);
    D.e[1][0] = ent(cconj(q01), cconj(s01));
    D.e[1][1] = dia(q11, s11);
    D.e[1][2] = ent(q12, s12);
    if (ROWS == 3 || s > 0) {
        D.e[2][0] = ent(cconj(q02), cconj(s02));
        D.e[2][1] = ent(cconj(q12), cconj(s12));
        D.e[2][2] = dia(q22, s22);
    }
    for (int i = 0; i < s; i++) {
        M3<R> D2 = mul_nn(D, D);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++)
                D.e[a][b] = cadd(D2.e[a][b], cadd(D.e[a][b], D.e[a][b]));
    }
    return D;
}

// Rows 0 .. ROWS-1 of exp(X) U = U + (D U) with D = exp(X) - 1 (su3_expm1).
// The increment D U is summed on its own (its entries are of the size of X,
// so FP32 keeps its second-order part -|X|^2 U / 2 to a relative 1e-7) and
// added to U last, one rounding per entry.  Any other order loses that part:
// a diagonal 1 - |X|^2/2 rounds to 1 when |X|^2 < 2^-24, and a multiply-add
// chain started from U's entry rounds after its first-order term, after which
// the second-order term is below half an ulp of the running sum and dropped.
// Either way every link gains norm |X|^2 per stage, which shows as a
// plaquette offset growing by ~1e-7 per step until the next reunitarisation.
template <class R, int ROWS>
__device__ __forceinline__ M3<R> mul_add_expm1(const M3<R> &D, const M3<R> &U) {
    M3<R> N;
#pragma unroll
    for (int r = 0; r < ROWS; r++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> s = cmul(D.e[r][0], U.e[0][j]);
            s = cmadd(s, D.e[r][1], U.e[1][j]);
            s = cmadd(s, D.e[r][2], U.e[2][j]);
            N.e[r][j] = cadd(U.e[r][j], s);
        }
    return N;
}

}  // namespace tgf
