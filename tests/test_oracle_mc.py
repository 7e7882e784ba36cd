"""Pins of the oracle's Monte Carlo: hybrid over-relaxation (sec. 3.1: one
heat-bath sweep followed by over-relaxation sweeps), SU(2) subgroup updates on
a checkerboard, Philox4x32-10 random numbers.

What fixes each value independently of the oracle's own arithmetic:
  * Philox4x32-10: the known-answer vectors published with the generator
    (Salmon, Moraes, Dror, Shaw, SC'11, Random123 distribution).
  * SU(2) sampler: y0 has density ~ sqrt(1 - y0^2) exp(alpha y0) on [-1, 1]
    (the SU(2) Haar measure times the local Boltzmann weight), whose moments
    are ratios of modified Bessel functions: <y0> = I2(alpha)/I1(alpha); the
    whole distribution is compared with its CDF by quadrature.
  * Over-relaxation leaves the action unchanged link by link.
  * beta = 0 heat bath: Haar measure on SU(3), whose trace moments are
    <Tr U> = 0, <|Tr U|^2> = 1, <(Tr U)^3> = 1 (the SU(3) determinant),
    <|Tr U|^4> = 2.
  * Strong coupling: the mean plaquette equals the one-link expectation
    u(beta) = (1/3) <Re Tr U> under exp((beta/3) Re Tr U) to corrections of
    order u^5; u(beta) is a Weyl-formula integral over the eigenphases.
"""

import numpy as np
import pytest

import oracle
from brute import u_strong
from paper_2107_03747_amd import gen

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    out = oracle.philox(ctr, *key)
    assert [int(x) for x in out] == list(expect)


def _y0_density(alpha):
    from scipy import integrate
    f = lambda y: np.sqrt(max(0.0, 1 - y * y)) * np.exp(alpha * (y - 1))
    z = integrate.quad(f, -1, 1, limit=200)[0]
    return f, z


@pytest.mark.parametrize("alpha", [0.0, 0.7, 1.99, 2.01, 6.0, 40.0])
def test_su2_sampler_moments(alpha):
    """Both branches (Creutz below alpha = 2, Kennedy-Pendleton above) and the
    alpha = 0 (Haar) case: mean, second moment, unit norm, isotropy."""
    from scipy import integrate
    from scipy.special import ive
    n = 200000
    y = oracle.su2_samples(alpha, 4321, n)
    assert np.abs((y ** 2).sum(1) - 1).max() < 1e-14
    f, z = _y0_density(alpha)
    m1 = ive(2, alpha) / ive(1, alpha) if alpha > 0 else 0.0
    m2 = integrate.quad(lambda t: t * t * f(t), -1, 1, limit=200)[0] / z
    sd = np.sqrt(m2 - m1 * m1)
    assert abs(y[:, 0].mean() - m1) < 5 * sd / np.sqrt(n)
    assert abs((y[:, 0] ** 2).mean() - m2) < 5 * np.sqrt(1.0 / n)
    # (y1, y2, y3) uniform on the sphere of radius sqrt(1 - y0^2)
    perp = 1 - m2
    for k in (1, 2, 3):
        assert abs(y[:, k].mean()) < 5 * np.sqrt(perp / 3 / n)
        assert abs((y[:, k] ** 2).mean() - perp / 3) < 5 * np.sqrt(2.0 / n) * perp


@pytest.mark.parametrize("alpha", [1.0, 4.0])
def test_su2_sampler_distribution(alpha):
    """Kolmogorov-Smirnov test of y0 against the exact CDF."""
    from scipy import integrate, stats
    f, z = _y0_density(alpha)
    grid = np.linspace(-1, 1, 4001)
    cdf = np.concatenate([[0], np.cumsum([integrate.quad(f, a, b)[0]
                                          for a, b in zip(grid[:-1], grid[1:])])]) / z
    y0 = oracle.su2_samples(alpha, 99, 50000)[:, 0]
    p = stats.kstest(y0, lambda x: np.interp(x, grid, cdf)).pvalue
    assert p > 1e-4


def _start(dims, kind, seed=7):
    if kind == "near":
        return np.ascontiguousarray(gen.near_identity(dims, 0.4, seed).numpy())
    return np.ascontiguousarray(gen.haar(dims, seed).numpy())


@pytest.mark.parametrize("kind", ["near", "haar"])
@pytest.mark.parametrize("twist", [oracle.PAPER_TWIST, (1, 2, 0, 1, 0, 2)])
def test_overrelaxation_keeps_action(kind, twist):
    dims = (4, 4, 6, 6)
    U = _start(dims, kind)
    before = oracle.measure(U, dims, twist)["action"]
    U0 = U.copy()
    oracle.or_sweeps(U, dims, 3, twist)
    after = oracle.measure(U, dims, twist)["action"]
    assert abs(after - before) <= 1e-12 * abs(before)
    assert np.abs(U - U0).max() > 0.1           # the links did move
    eye = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


def test_heatbath_beta0_is_haar():
    dims = (4, 4, 4, 4)
    U = np.ascontiguousarray(gen.identity(dims).numpy())
    tr = []
    for k in range(40):
        oracle.mc(U, dims, 0.0, 1, 0, seed=5, sweep0=k)
        if k >= 10:
            tr.append(np.trace(U, axis1=-2, axis2=-1).ravel())
    tr = np.concatenate(tr)
    n = len(tr)
    assert abs(tr.mean()) < 5 * np.sqrt(1.0 / n)
    assert abs(np.mean(np.abs(tr) ** 2) - 1) < 5 * np.sqrt(1.0 / n)
    assert abs(np.mean(tr ** 3) - 1) < 5 * np.sqrt(6.0 / n)
    assert abs(np.mean(np.abs(tr) ** 4) - 2) < 5 * np.sqrt(22.0 / n)


def test_u_strong_series():
    # the weak-field end of the one-link integral: u = beta/18 + beta^2/216 + O(beta^3)
    b = 0.05
    assert abs(u_strong(b) - (b / 18 + b * b / 216)) < 1e-6


def test_strong_coupling_plaquette():
    """beta = 18 b = 1.5: <plaq> = u(beta) + O(u^5) (u^5 ~ 1e-5 here)."""
    beta = 1.5
    dims = (6, 6, 6, 6)
    U = np.ascontiguousarray(gen.identity(dims).numpy())
    ps = []
    for k in range(130):
        oracle.mc(U, dims, beta / 18, 1, 2, seed=99, sweep0=3 * k)
        if k >= 30:
            ps.append(oracle.measure(U, dims)["plaq"])
    ps = np.array(ps)
    err = ps.std() / np.sqrt(len(ps))
    assert err < 6e-4
    assert abs(ps.mean() - u_strong(beta)) < 5 * err + 1e-4


def test_mc_deterministic_and_counter_based():
    dims = (4, 4, 6, 6)
    U0 = _start(dims, "near")
    runs = []
    for threads in (1, 8):
        oracle.set_threads(threads)
        V = U0.copy()
        oracle.mc(V, dims, 0.6, 2, 3, seed=11)
        runs.append(V)
    assert np.array_equal(runs[0], runs[1])
    # a chain split in two calls, continuing the sweep counter, is the same chain
    V = U0.copy()
    oracle.mc(V, dims, 0.6, 1, 3, seed=11, sweep0=0)
    oracle.mc(V, dims, 0.6, 1, 3, seed=11, sweep0=4)
    assert np.array_equal(V, runs[0])
    # another seed or config index gives another chain
    for kw in (dict(seed=12), dict(seed=11, cfg=1)):
        W = U0.copy()
        oracle.mc(W, dims, 0.6, 2, 3, **kw)
        assert np.abs(W - runs[0]).max() > 0.1


def test_mc_rejects_odd_extent():
    dims = (4, 4, 5, 6)
    U = np.ascontiguousarray(gen.identity(dims).numpy())
    with pytest.raises(RuntimeError):
        oracle.mc(U, dims, 0.5, 1, 1, seed=1)
