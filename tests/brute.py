"""numpy brute force for tiny lattices (test-only, independent of the oracle).

``action`` evaluates s = sum_n sum_{mu<nu} Re Tr[1 - Z^*_{mu nu}(n) P_{mu nu}(n)]
(sec. 3.1, g0^2 S_W / 2) with whole-array shifts; ``fd_force_components``
differentiates it numerically along the eight su(3) generators of a link, so
the oracle's analytic force can be checked against the action it derives
from without reusing any of its staple algebra.
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
