"""Ensemble statistics: pins of the oracle (tests of oracle/stats.py against
closed forms and identities) and the library's host functions against it.

Paper: eq. lambdat, eq. calA, eq. theta3 (sec. 1); eq. latt_norm and
eq. lambdat_latt (sec. 3.1); eq. qcorr (sec. 4).
"""

import math

import numpy as np
import pytest

import fields
import oracle
from oracle import stats

tgf = pytest.importorskip("paper_2107_03747_amd.tgf", reason="libtgf.so not built")


# ---------------------------------------------------------------- oracle pins

@pytest.mark.parametrize("x", [0.05, 0.283, 1.0, 3.7])
def test_theta3_two_forms_agree(x):
    """The two expressions of eq. theta3 (Poisson resummation)."""
    assert stats.theta3(x) == pytest.approx(stats.theta3_dual(x), rel=1e-13)


@pytest.mark.parametrize("c", [0.3, 0.4])
def test_latt_norm_approaches_continuum(c):
    """N(c, Lt) -> 128 pi^2 / (N A(pi c^2)) with O(1/Lt^2) corrections: in the
    continuum the lattice sum becomes theta3^4 minus the excluded modes, i.e.
    A(x)/x^2 -- which pins the mode exclusion and the c^4/128 normalisation."""
    cont = stats.continuum_norm(c)
    d = [stats.latt_norm(c, L) / cont - 1 for L in (12, 24, 48)]
    assert abs(d[2]) < 1e-2
    assert 3.0 < d[0] / d[1] < 5.0 and 3.0 < d[1] / d[2] < 5.0


def test_latt_norm_without_exclusion_is_wrong():
    """Keeping the twisted zero modes changes the answer by O(1): the pin above
    would not pass with a wrong exclusion rule."""
    c, L = 0.3, 24
    cont_all = 128 * math.pi ** 2 / (3 * (math.pi * c * c) ** 2 * stats.theta3(math.pi * c * c) ** 4)
    assert abs(stats.latt_norm(c, L) / cont_all - 1) > 0.05


def test_coupling_is_mean_with_standard_error_when_all_in_sector():
    rng = np.random.default_rng(1)
    t2E = rng.normal(0.2, 0.01, size=40)
    Q = np.zeros(40)
    lam, err = stats.coupling(t2E, Q, 0.3, 12)
    n = stats.latt_norm(0.3, 12)
    assert lam == pytest.approx(n * t2E.mean() / 3, rel=1e-14)
    assert err == pytest.approx(n / 3 * t2E.std(ddof=1) / math.sqrt(40), rel=1e-10)


def test_coupling_filters_topology():
    t2E = np.array([0.1, 0.2, 5.0, 0.3, 7.0])
    Q = np.array([0.1, -0.49, 1.0, 0.2, -0.5])    # |Q| < 0.5 keeps 0, 1, 3
    lam, _ = stats.coupling(t2E, Q, 0.3, 12)
    assert lam == pytest.approx(stats.latt_norm(0.3, 12) * 0.2 / 3, rel=1e-14)


def test_correlator_identities():
    rng = np.random.default_rng(2)
    q = rng.normal(size=(6, 12))
    Q = np.array([0.1, 0.3, 2.0, -0.2, 0.0, 0.7])
    C, E = stats.charge_correlator(q, Q)
    d = np.abs(Q) < 0.5
    tot = q.sum(1)
    assert C.sum() == pytest.approx(np.sum(tot[d] ** 2) / (12 * d.sum()), rel=1e-12)
    assert np.allclose(C[1:], C[1:][::-1], rtol=1e-13)        # C(x) = C(T - x)


def test_slice_charges_sum_to_Q_and_flux_closed_form():
    dims = (4, 4, 6, 6)
    U, p01, p23 = fields.flux_field(dims, 1, 1)
    e, qd = oracle.densities(U, dims, twist=(0,) * 6)
    for direction in (2, 3):
        qs = stats.slice_charges(qd, dims, direction)
        Q = oracle.measure(U, dims, twist=(0,) * 6)["Q"]
        assert qs.sum() == pytest.approx(Q, rel=1e-12)
        # constant density: every slice carries Q / extent
        assert np.allclose(qs, Q / dims[direction], rtol=1e-12)


# ------------------------------------------------- library host code vs oracle

@pytest.mark.parametrize("c,L", [(0.3, 6), (0.3, 12), (0.3, 18), (0.4, 24), (0.3, 9)])
def test_library_latt_norm(c, L):
    assert tgf.latt_norm(c, L) == pytest.approx(stats.latt_norm(c, L), rel=1e-12)


def test_library_coupling_and_correlator():
    rng = np.random.default_rng(3)
    t2E = rng.normal(0.3, 0.02, size=25)
    Q = rng.normal(0, 0.6, size=25)
    lam, err = tgf.coupling(t2E, Q, 0.3, 12)
    lo, eo = stats.coupling(t2E, Q, 0.3, 12)
    assert lam == pytest.approx(lo, rel=1e-13) and err == pytest.approx(eo, rel=1e-10)
    q = rng.normal(size=(25, 18))
    C, E = tgf.charge_correlator(q, Q)
    Co, Eo = stats.charge_correlator(q, Q)
    assert np.allclose(C, Co, rtol=1e-12, atol=1e-15) and np.allclose(E, Eo, rtol=1e-9)


def test_susceptibility_pins():
    """chi = <Q^2>/V; the delete-one jackknife of a mean is the standard
    error of that mean, s(Q^2)/sqrt(n) with the n-1 sample deviation."""
    V = 4 * 4 * 12 * 12
    chi, err = stats.susceptibility([1.0, -1.0] * 10, V)
    assert chi == pytest.approx(1.0 / V, rel=1e-15) and err == pytest.approx(0.0, abs=1e-18)
    rng = np.random.default_rng(11)
    Q = rng.normal(0, 1.3, size=40)
    chi, err = stats.susceptibility(Q, V)
    assert chi == pytest.approx(np.mean(Q ** 2) / V, rel=1e-14)
    assert err == pytest.approx(np.std(Q ** 2, ddof=1) / np.sqrt(len(Q)) / V, rel=1e-10)
    chi_l, err_l = tgf.susceptibility(Q, V)
    assert chi_l == pytest.approx(chi, rel=1e-14) and err_l == pytest.approx(err, rel=1e-10)
    with pytest.raises(tgf.TGFError):
        tgf.susceptibility(Q, 0.0)
    with pytest.raises(tgf.TGFError):
        tgf.susceptibility([], V)


def test_library_stats_errors():
    with pytest.raises(tgf.TGFError) as e:
        tgf.coupling([0.1, 0.2], [1.0, 2.0], 0.3, 12)
    assert e.value.status == tgf.TGF_E_STATE
    with pytest.raises(tgf.TGFError):
        tgf.latt_norm(-0.3, 12)
    with pytest.raises(tgf.TGFError):
        tgf.latt_norm(0.3, 0)
