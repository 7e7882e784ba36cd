"""numpy brute force for tiny lattices (test-only, independent of the oracle).

``action`` evaluates s = sum_n sum_{mu<nu} Re Tr[1 - Z^*_{mu nu}(n) P_{mu nu}(n)]
(sec. 3.1, g0^2 S_W / 2) with whole-array shifts; ``fd_force_components``
differentiates it numerically along the eight su(3) generators of a link, so
the oracle's analytic force can be checked against the action it derives
from without reusing any of its staple algebra.  The ``torus_*`` functions
flow fields in the maximal torus of SU(N), where the flow is an ODE for the
link angles, with a classical Runge-Kutta tableau.
"""

import numpy as np

from fields import coords, su3_generators


def _dag(x):
    return np.conj(np.swapaxes(x, -1, -2))


def _shift(A, mu):
    """A(n + mu_hat) in canonical axis order (axis 3 - mu is n_mu)."""
    return np.roll(A, -1, axis=3 - mu)


def action(U, dims, twist=(1, 0, 0, 0, 0, 0), base=(0, 0, 0, 0)):
    """s = sum_n sum_{mu<nu} Re Tr[1 - Z^* P] for SU(N), N = U.shape[-1];
    Z = exp(2 pi i n_{mu nu} / N) on the twist site of each plane."""
    N = U.shape[-1]
    n = coords(dims)
    s = 0.0
    k = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = U[..., mu, :, :] @ _shift(U[..., nu, :, :], mu) \
                @ _dag(_shift(U[..., mu, :, :], nu)) @ _dag(U[..., nu, :, :])
            tr = np.trace(P, axis1=-2, axis2=-1)
            z = np.ones(tr.shape, complex)
            if twist[k] % N:
                on = (n[mu] == base[mu]) & (n[nu] == base[nu])
                z[on] = np.exp(2j * np.pi * (twist[k] % N) / N)
            s += np.sum(N - np.real(np.conj(z) * tr))
            k += 1
    return s


def expm_small(A, terms=30):
    N = A.shape[-1]
    out = np.eye(N, dtype=complex)
    term = np.eye(N, dtype=complex)
    for k in range(1, terms):
        term = term @ A / k
        out = out + term
    return out


def fd_force_components(U, dims, site, mu, twist=(1, 0, 0, 0, 0, 0), h=1e-4, T=None):
    """d/ds s(exp(s T^a) U_mu(site)) at s = 0 for every generator T^a
    (central differences); T defaults to the SU(3) basis."""
    T = su3_generators() if T is None else T
    d = np.zeros(len(T))
    for a in range(len(T)):
        vals = []
        for sgn in (+1, -1):
            V = U.copy()
            V[site + (mu,)] = expm_small(sgn * h * T[a]) @ U[site + (mu,)]
            vals.append(action(V, dims, twist))
        d[a] = (vals[0] - vals[1]) / (2 * h)
    return d


def u_strong(beta, n=256):
    """(1/3) <Re Tr U> under exp((beta/3) Re Tr U) dU on SU(3), by the Weyl
    integration formula (eigenphases t1, t2, t3 = -t1 - t2, weight |Delta|^2);
    the periodic trapezoid rule converges spectrally."""
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    z = [np.exp(1j * t1), np.exp(1j * t2), np.exp(-1j * (t1 + t2))]
    vd = np.abs((z[0] - z[1]) * (z[0] - z[2]) * (z[1] - z[2])) ** 2
    tr = (z[0] + z[1] + z[2]).real
    w = vd * np.exp(beta / 3 * tr)
    return float((tr * w).sum() / w.sum() / 3)


# ----------------------------------------------------------------------------
# The flow on the maximal torus of SU(N): U = diag(e^{i a_1}, ..., e^{i a_N}),
# sum_k a_k = 0.  Plaquettes are diagonal with angles phi_k, the twist factor
# multiplies every entry by e^{i theta_P} (theta_P = 2 pi n_{mu nu} / N on the
# twist site), and the action above is s = sum_P sum_k [1 - cos(phi_k -
# theta_P)].  Moving U_mu(n) along the diagonal generator T = i diag(t)
# (sum t = 0) changes s by t . g with g_k = sum_P +-sin(phi_k - theta_P); the
# flow generator F = i diag(f) obeys tr(T F) = ds for every such T (the
# relation between the force and the action's derivative), so
# f = -(g - mean(g)), and the field never leaves the torus.

# three-stage Runge-Kutta tableaus (c2, a31, a32, (b1, b2, b3)) of third
# order: Luscher's scheme exp(Z0/4), exp(8/9 Z1 - 17/36 Z0),
# exp(3/4 Z2 - 8/9 Z1 + 17/36 Z0) written as a classical method, and others
RK3_TABLEAUS = {
    "luscher": (1 / 4, -2 / 9, 8 / 9, (1 / 4, 0, 3 / 4)),
    "kutta": (1 / 2, -1, 2, (1 / 6, 2 / 3, 1 / 6)),
    "heun": (1 / 3, 0, 2 / 3, (1 / 4, 0, 3 / 4)),
    # third order on the group as well (nodes 1/3, 3/4)
    "group_c2_1/3": (1 / 3, -3 / 16, 15 / 16, (1 / 6, 3 / 10, 8 / 15)),
}


def torus_angles(dims, N, seed, scale):
    """Uniform link angles in [-scale, scale), the last fixed by sum = 0,
    canonical [d3, d2, d1, d0, 4, N] order."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-scale, scale, size=tuple(dims[::-1]) + (4, N - 1))
    return np.concatenate([a, -a.sum(-1, keepdims=True)], axis=-1)


def torus_links(ang):
    N = ang.shape[-1]
    U = np.zeros(ang.shape + (N,), complex)
    for k in range(N):
        U[..., k, k] = np.exp(1j * ang[..., k])
    return U


def torus_velocity(ang, dims, twist=(1, 0, 0, 0, 0, 0), base=(0, 0, 0, 0)):
    """da/dt of every link angle (the flow of the action above on the torus)."""
    N = ang.shape[-1]
    back = lambda A, mu: np.roll(A, 1, axis=3 - mu)     # A(n - mu)
    n = coords(dims)
    g = np.zeros_like(ang)
    p = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a_mu, a_nu = ang[..., mu, :], ang[..., nu, :]
            phi = a_mu + _shift(a_nu, mu) - _shift(a_mu, nu) - a_nu
            theta = np.zeros(phi.shape[:-1])
            if twist[p] % N:
                on = (n[mu] == base[mu]) & (n[nu] == base[nu])
                theta[on] = 2 * np.pi * (twist[p] % N) / N
            sn = np.sin(phi - theta[..., None])
            # U_mu(n) enters P(n) and, daggered, P(n - nu); U_nu(n) enters
            # P(n - mu) and, daggered, P(n)
            g[..., mu, :] += sn - back(sn, nu)
            g[..., nu, :] += back(sn, mu) - sn
            p += 1
    return -(g - g.mean(-1, keepdims=True))


def torus_rk3(ang, dims, h, twist, tableau):
    """One step of the classical three-stage Runge-Kutta method `tableau`."""
    c2, a31, a32, b = tableau
    k1 = torus_velocity(ang, dims, twist)
    k2 = torus_velocity(ang + h * c2 * k1, dims, twist)
    k3 = torus_velocity(ang + h * (a31 * k1 + a32 * k2), dims, twist)
    return ang + h * (b[0] * k1 + b[1] * k2 + b[2] * k3)
