"""Closed-form SU(N) test fields (numpy, test-only, independent of the oracle
and of the GPU library), layout [d3, d2, d1, d0, 4, N, N]."""

import numpy as np

from fields import coords
from paper_2107_03747_amd import gen


def identity_n(dims, N):
    return gen.identity_n(dims, N).numpy().copy()


def su_n_generators(N):
    """T^a = -i lambda^a / 2 for the N^2 - 1 generalised Gell-Mann matrices
    (tr lambda^a lambda^b = 2 delta_ab), so tr(T^a T^b) = -delta_ab / 2."""
    lam = []
    for j in range(N):
        for k in range(j + 1, N):
            m = np.zeros((N, N), complex)
            m[j, k] = m[k, j] = 1
            lam.append(m)
            m = np.zeros((N, N), complex)
            m[j, k], m[k, j] = -1j, 1j
            lam.append(m)
    for l in range(1, N):
        m = np.zeros((N, N), complex)
        for i in range(l):
            m[i, i] = 1
        m[l, l] = -l
        lam.append(m * np.sqrt(2.0 / (l * (l + 1))))
    return -0.5j * np.array(lam)


def twist_matrices_n(N, k=1):
    """Gamma_a = c_a P^k, Gamma_b = c_b S with the clock P = diag(w^j), the
    shift S e_j = e_{j+1}, w = exp(2 pi i / N): Gamma_a Gamma_b =
    w^k Gamma_b Gamma_a (the twist algebra of sec. 1); the phases c make
    both determinants 1."""
    w = np.exp(2j * np.pi / N)
    P = np.diag(w ** (k * np.arange(N)))
    S = np.zeros((N, N), complex)
    for i in range(N):
        S[(i + 1) % N, i] = 1
    for M in (P, S):
        d = np.linalg.det(M)
        M *= np.exp(-1j * np.angle(d) / N)
    return P, S


def twist_eater_n(dims, N, k=1):
    """Zero-action field of the (0,1) plane twisted by k: U_0 = Gamma_a on
    n0 = 0, U_1 = Gamma_b on n1 = 0, every other link 1."""
    Ga, Gb = twist_matrices_n(N, k)
    U = identity_n(dims, N)
    U[:, :, :, 0, 0] = Ga
    U[:, :, 0, :, 1] = Gb
    return U


def _diag_links(angle, N):
    H = np.zeros(N)
    H[0], H[1] = 1.0, -1.0
    out = np.zeros(angle.shape + (N, N), complex)
    for k in range(N):
        out[..., k, k] = np.exp(1j * angle * H[k])
    return out


def flux_field_n(dims, N, m01=1, m23=1):
    """Constant abelian field strength in the first SU(2) block of SU(N),
    untwisted torus, plaquette angles phi01 = 2 pi m01/(d0 d1) and
    phi23 = 2 pi m23/(d2 d3).  Returns (U, phi01, phi23)."""
    d0, d1, d2, d3 = dims
    n0, n1, n2, n3 = coords(dims)
    p01 = 2 * np.pi * m01 / (d0 * d1)
    p23 = 2 * np.pi * m23 / (d2 * d3)
    U = identity_n(dims, N)
    U[..., 1, :, :] = _diag_links(p01 * n0, N)
    U[..., 0, :, :] = _diag_links(np.where(n0 == d0 - 1, -p01 * d0 * n1, 0.0), N)
    U[..., 3, :, :] = _diag_links(p23 * n2, N)
    U[..., 2, :, :] = _diag_links(np.where(n2 == d2 - 1, -p23 * d2 * n3, 0.0), N)
    return U, p01, p23


def single_mode_n(dims, N, alpha, p, rho):
    """U_rho(n) = exp(i alpha cos(p.n) T), T = diag(1, -1, 0, ...)/2."""
    n0, n1, n2, n3 = coords(dims)
    ph = p[0] * n0 + p[1] * n1 + p[2] * n2 + p[3] * n3
    U = identity_n(dims, N)
    U[..., rho, :, :] = _diag_links(0.5 * alpha * np.cos(ph), N)
    return U


def unitarity_defect_n(U):
    N = U.shape[-1]
    Ud = np.conj(np.swapaxes(U, -1, -2))
    return np.abs(U @ Ud - np.eye(N)).max(), np.abs(np.linalg.det(U) - 1).max()
