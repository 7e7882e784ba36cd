"""Sanity of the seeded input generators (paper_2107_03747_amd/gen.py), which
both the oracle and the GPU path take their links from.

* Haar SU(3) (the hot starts of the large-box workload): group membership, and
  the trace moments of the Haar measure on SU(3), <Tr U> = 0, <|Tr U|^2> = 1,
  <(Tr U)^3> = 1, <|Tr U|^4> = 2 (the numbers of singlets in 3, 3 x 3bar,
  3 x 3 x 3 and (3 x 3bar)^2), within 5 standard errors of the sample mean;
  Haar SU(N) for N = 2, 4: <|Tr U|^2> = 1 and det U = 1.
* near-identity links U = exp(i eps H), H = sum_a h_a lambda_a / 2 with
  Gaussian h_a: det U = 1 and <Re Tr U> / 3 = 1 - (2/3) eps^2 + (5/36) eps^4
  + O(eps^6) (from <Tr H^2> = 4 and <Tr H^4> = 10 for the SU(3) generators in
  the fundamental representation).
* determinism: the same seed gives the same links (for the Haar generators
  with the same chunk size: each chunk draws its own normals, so the chunk
  size is part of the draw order; the near-identity generators draw all
  coefficients at once).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2107_03747_amd import gen  # noqa: E402


def _tr(U):
    return np.trace(U, axis1=-2, axis2=-1)


def _group_defects(U):
    N = U.shape[-1]
    eye = np.eye(N)
    du = np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - eye).max()
    dd = np.abs(np.linalg.det(U) - 1).max()
    return du, dd


def _within(sample, expect, k=5.0):
    m = sample.mean()
    se = sample.std() / np.sqrt(sample.size)
    return abs(m - expect) <= k * se + 1e-12, (m, expect, se)


def test_haar_su3_moments():
    U = gen.su3_haar(400_000, seed=123).numpy()
    du, dd = _group_defects(U)
    assert du < 1e-13 and dd < 1e-13
    t = _tr(U)
    for sample, expect in ((t.real, 0.0), (t.imag, 0.0), (np.abs(t) ** 2, 1.0),
                           ((t ** 3).real, 1.0), ((t ** 3).imag, 0.0), (np.abs(t) ** 4, 2.0)):
        ok, info = _within(sample, expect)
        assert ok, info


def test_haar_lattice_is_the_matrix_generator():
    dims = (2, 2, 4, 4)
    U = gen.haar(dims, seed=7).numpy()
    assert U.shape == (4, 4, 2, 2, 4, 3, 3)
    du, dd = _group_defects(U)
    assert du < 1e-13 and dd < 1e-13
    assert np.array_equal(U, gen.haar(dims, seed=7).numpy())
    assert not np.array_equal(U, gen.haar(dims, seed=8).numpy())


@pytest.mark.parametrize("N", [2, 4])
def test_haar_sun_moments(N):
    U = gen.haar_n((4, 4, 8, 8), N, seed=11).numpy().reshape(-1, N, N)
    du, dd = _group_defects(U)
    assert du < 1e-12 and dd < 1e-12
    ok, info = _within(np.abs(_tr(U)) ** 2, 1.0)
    assert ok, info


def test_near_identity_scale():
    eps = 0.1
    U = gen.near_identity((8, 8, 16, 16), eps, seed=5).numpy().reshape(-1, 3, 3)
    du, dd = _group_defects(U)
    assert du < 1e-13 and dd < 1e-13
    expect = 1 - (2.0 / 3.0) * eps ** 2 + (5.0 / 36.0) * eps ** 4
    ok, info = _within(_tr(U).real / 3, expect)
    assert ok, info
    # a generator that dropped the 1/2 of lambda_a / 2 (or used eps^2) fails:
    assert abs(info[0] - (1 - (8.0 / 3.0) * eps ** 2)) > 10 * info[2]
    same = gen.near_identity((8, 8, 16, 16), eps, seed=5, chunk=1000).numpy().reshape(-1, 3, 3)
    assert np.array_equal(U, same)


def test_near_identity_sun_group():
    U = gen.near_identity_n((2, 2, 8, 8), 4, 0.3, seed=3).numpy().reshape(-1, 4, 4)
    du, dd = _group_defects(U)
    assert du < 1e-13 and dd < 1e-13
