"""Ensemble statistics of the twisted gradient-flow coupling -- TEST
INFRASTRUCTURE ONLY (plain numpy, explicit loops where the formula has them).

* theta3(0, ix) both ways of eq. theta3; A(x) of eq. calA; the continuum
  normalisation 128 pi^2 / (N A(pi c^2)) of eq. lambdat;
* the lattice normalisation of eq. latt_norm, written out term by term;
* lambda_TGF of eq. lambdat_latt with delta_Q = [|Q| < 0.5], and the
  correlator of eq. qcorr, with delete-one jackknife errors;
* slice charges q(x0) from the oracle's per-site charge density.
"""

import math

import numpy as np


def theta3(x, terms=60):
    """theta_3(0, ix) = sum_m exp(-pi x m^2)."""
    m = np.arange(-terms, terms + 1)
    return float(np.sum(np.exp(-np.pi * x * m * m)))


def theta3_dual(x, terms=60):
    """The same function by the second form of eq. theta3: x^-1/2 sum_m exp(-pi m^2 / x)."""
    m = np.arange(-terms, terms + 1)
    return float(np.sum(np.exp(-np.pi * m * m / x)) / math.sqrt(x))


def calA(x, N=3):
    t = theta3(x)
    return x * x * t * t * (t * t - theta3(x * N * N) ** 2)


def continuum_norm(c, N=3):
    return 128 * math.pi ** 2 / (N * calA(math.pi * c * c, N))


def latt_norm(c, Lt, N=3):
    """N(c, Lt) by the momentum sum of eq. latt_norm; momenta q = 2 pi n / Lt in
    all four directions; excluded are those whose two twisted-plane (0, 1)
    components have Lt q_i a multiple of 2 pi N (n_i = 0 mod N)."""
    n = np.arange(Lt)
    q = 2 * np.pi * n / Lt
    total = 0.0
    q0, q1, q2 = np.meshgrid(q, q, q, indexing="ij")     # directions 0, 1, 2
    n0, n1 = np.meshgrid(n, n, indexing="ij")
    excluded = (n0 % N == 0) & (n1 % N == 0)   # Lt q_i = 2 pi n_i in 2 pi N Z
    for k3 in range(Lt):                                  # direction 3, one slab at a time
        qq = [q0, q1, q2, np.full_like(q0, q[k3])]
        qhat2 = sum(4 * np.sin(x / 2) ** 2 for x in qq)
        keep = ~np.broadcast_to(excluded[:, :, None], q0.shape)
        w = np.exp(-0.25 * c * c * Lt * Lt * qhat2)
        acc = np.zeros_like(q0)
        for mu in range(4):
            for nu in range(4):
                if mu != nu:
                    acc += np.sin(qq[nu]) ** 2 * np.cos(qq[mu] / 2) ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            term = np.where(keep, w * acc / qhat2, 0.0)
        total += float(term.sum())
    return 1.0 / (c ** 4 / 128 * total)


def coupling(t2E, Q, c, Lt, N=3):
    t2E = np.asarray(t2E, float)
    d = (np.abs(np.asarray(Q, float)) < 0.5).astype(float)
    norm = latt_norm(c, Lt, N)
    lam = norm * np.sum(t2E * d) / (3 * np.sum(d))
    jk = []
    for k in range(len(t2E)):
        keep = np.arange(len(t2E)) != k
        if np.sum(d[keep]) > 0:
            jk.append(norm * np.sum(t2E[keep] * d[keep]) / (3 * np.sum(d[keep])))
    jk = np.array(jk)
    err = math.sqrt((len(jk) - 1) / len(jk) * np.sum((jk - jk.mean()) ** 2))
    return lam, err


def charge_correlator(q, Q):
    q = np.asarray(q, float)
    n, T = q.shape
    d = (np.abs(np.asarray(Q, float)) < 0.5).astype(float)
    ck = np.zeros((n, T))
    for k in range(n):
        for x in range(T):
            ck[k, x] = sum(q[k, (y + x) % T] * q[k, y] for y in range(T)) / T
    C = (d[:, None] * ck).sum(0) / d.sum()
    E = np.zeros(T)
    for x in range(T):
        jk = np.array([(np.sum(d * ck[:, x]) - d[k] * ck[k, x]) / (d.sum() - d[k])
                       for k in range(n) if d.sum() - d[k] > 0])
        E[x] = math.sqrt((len(jk) - 1) / len(jk) * np.sum((jk - jk.mean()) ** 2))
    return C, E


def susceptibility(Q, V):
    """chi = <Q^2>/V (sec. 4.2), delete-one jackknife error."""
    Q = np.asarray(Q, float)
    n = len(Q)
    chi = float(np.mean(Q ** 2) / V)
    jk = np.array([np.mean(np.delete(Q, k) ** 2) / V for k in range(n)])
    err = math.sqrt((n - 1) / n * np.sum((jk - jk.mean()) ** 2))
    return chi, err


def slice_charges(qdens, dims, direction=3):
    """q(x0) = sum of the per-site charge density over the slice n_dir = x0."""
    d0, d1, d2, d3 = dims
    q = np.asarray(qdens).reshape(d3, d2, d1, d0)
    axis = 3 - direction
    other = tuple(a for a in range(4) if a != axis)
    return q.sum(axis=other)
