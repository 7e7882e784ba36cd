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

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void rebuild_row2(M3<R> &U) {
    const cx<R> *a = U.e[0], *b = U.e[1];
    // (a x b)_0 = a1 b2 - a2 b1, etc.; then conjugate
    cx<R> c0 = csub(cmul(a[1], b[2]), cmul(a[2], b[1]));
    cx<R> c1 = csub(cmul(a[2], b[0]), cmul(a[0], b[2]));
    cx<R> c2 = csub(cmul(a[0], b[1]), cmul(a[1], b[0]));
    U.e[2][0] = cconj(c0);
    U.e[2][1] = cconj(c1);
    U.e[2][2] = cconj(c2);
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

// exp(X) for X in su(3), by Cayley-Hamilton: with Q = -i X (Hermitian,
// traceless), Q^3 = c1 Q + c0 with c1 = Tr(Q^2)/2, c0 = det Q, so every power
// Q^k = alpha_k + beta_k Q + gamma_k Q^2 and exp(iQ) = f0 + f1 Q + f2 Q^2 with
// f_j the exponential series of the coefficient recursion
//   alpha' = gamma c0, beta' = alpha + gamma c1, gamma' = beta.
// The series runs until the remainder bound rho^k/k! (rho = ||Q||_F) drops
// below the working precision; for rho > 1 the argument is halved s times and
// the result squared s times.
template <class R>
__device__ __forceinline__ M3<R> su3_exp(const Alg<R> &X) {
    // Q = -i X
    M3<R> Q;
    Q.e[0][0] = {X.a[6], R(0)};
    Q.e[1][1] = {X.a[7], R(0)};
    Q.e[2][2] = {-(X.a[6] + X.a[7]), R(0)};
    Q.e[0][1] = {X.a[1], -X.a[0]};
    Q.e[0][2] = {X.a[3], -X.a[2]};
    Q.e[1][2] = {X.a[5], -X.a[4]};
    Q.e[1][0] = cconj(Q.e[0][1]);
    Q.e[2][0] = cconj(Q.e[0][2]);
    Q.e[2][1] = cconj(Q.e[1][2]);

    R q00 = Q.e[0][0].x, q11 = Q.e[1][1].x, q22 = Q.e[2][2].x;
    R n01 = Q.e[0][1].x * Q.e[0][1].x + Q.e[0][1].y * Q.e[0][1].y;
    R n02 = Q.e[0][2].x * Q.e[0][2].x + Q.e[0][2].y * Q.e[0][2].y;
    R n12 = Q.e[1][2].x * Q.e[1][2].x + Q.e[1][2].y * Q.e[1][2].y;
    R fro2 = q00 * q00 + q11 * q11 + q22 * q22 + R(2) * (n01 + n02 + n12);

    int s = 0;
    if (fro2 > R(1)) {
        // halve until ||Q||_F <= 1
        R f = fro2;
        while (f > R(1) && s < 30) { f *= R(0.25); s++; }
        R sc = ldexp(R(1), -s);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) { Q.e[i][j].x *= sc; Q.e[i][j].y *= sc; }
        q00 *= sc; q11 *= sc; q22 *= sc;
        R sc2 = sc * sc;
        n01 *= sc2; n02 *= sc2; n12 *= sc2;
        fro2 *= sc2;
    }

    R c1 = R(0.5) * fro2;
    // det of a Hermitian 3x3: q00 q11 q22 + 2 Re(q01 q12 q20) - q00|q12|^2 - q11|q02|^2 - q22|q01|^2
    cx<R> t = cmul(Q.e[0][1], Q.e[1][2]);
    R re3 = t.x * Q.e[0][2].x + t.y * Q.e[0][2].y;  // Re(q01 q12 conj(q02))
    R c0 = q00 * q11 * q22 + R(2) * re3 - q00 * n12 - q11 * n02 - q22 * n01;

    // series: term k holds alpha_k/k!, beta_k/k!, gamma_k/k!, weight i^k
    R al = R(1), be = R(0), ga = R(0);
    cx<R> f0 = {R(1), R(0)}, f1 = {R(0), R(0)}, f2 = {R(0), R(0)};
    R rho = sqrt(fro2);
    R bound = R(1);
    for (int k = 1; k <= ExpTol<R>::kmax; k++) {
        bound = bound * rho / R(k);
        R inv = R(1) / R(k);
        R nal = ga * c0 * inv;
        R nbe = (al + ga * c1) * inv;
        R nga = be * inv;
        al = nal; be = nbe; ga = nga;
        switch (k & 3) {
            case 0: f0.x += al; f1.x += be; f2.x += ga; break;
            case 1: f0.y += al; f1.y += be; f2.y += ga; break;
            case 2: f0.x -= al; f1.x -= be; f2.x -= ga; break;
            default: f0.y -= al; f1.y -= be; f2.y -= ga; break;
        }
        if (bound < ExpTol<R>::tol) break;
    }

    // Q^2 (Hermitian)
    M3<R> Q2 = mul_nn(Q, Q);
    M3<R> E;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<R> v = cmul(f1, Q.e[i][j]);
            v = cmadd(v, f2, Q2.e[i][j]);
            if (i == j) v = cadd(v, f0);
            E.e[i][j] = v;
        }
    for (int i = 0; i < s; i++) E = mul_nn(E, E);
    return E;
}

}  // namespace tgf
