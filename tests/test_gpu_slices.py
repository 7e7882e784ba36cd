"""GPU: topological charge per slice (sec. 4) against the oracle's charge
density summed over slices, and the ensemble coupling computed end to end
from GPU flows against the same from oracle flows."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle                                      # noqa: E402
from oracle import stats                           # noqa: E402
from paper_2107_03747_amd import gen, tgf          # noqa: E402

oracle.set_threads(16)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-4), ("f32c12", 1e-4)])
def test_slice_charge_matches_oracle(storage, tol):
    dims_list = [(4, 4, 12, 12), (3, 3, 5, 7), (6, 6, 18, 18)]
    links = [gen.near_identity(d, 0.9, seed=60 + k).numpy().copy() for k, d in enumerate(dims_list)]
    f = tgf.Flow(dims_list, storage)
    f.load_all([torch.from_numpy(l).cuda() for l in links])
    f.flow(0.01, 0.05, 0.0)
    for direction in (3, 2, 0):
        qs = f.slice_charge(direction)
        tot = f.measure()[:, tgf.OBS_FIELDS.index("Q")]
        for k, d in enumerate(dims_list):
            U = f.store(k).cpu().numpy()
            _, qd = oracle.densities(U, d)
            ref = stats.slice_charges(qd, d, direction)
            got = qs[k, : d[direction]]
            print(f"  {storage} dir {direction} {d}: max |dq| {np.abs(got - ref).max():.3g}", flush=True)
            assert np.abs(got - ref).max() <= tol
            assert np.all(qs[k, d[direction]:] == 0)
            assert got.sum() == pytest.approx(tot[k], abs=tol * d[direction])


def test_coupling_end_to_end():
    """Four 4x4x12x12 configurations flowed to sqrt(8t) = 0.3 * 12 on the GPU
    (FP64), lambda_TGF and the slice-charge correlator vs the oracle's flows."""
    dims = (4, 4, 12, 12)
    L_t, c = 12, 0.3
    t_end = (c * L_t) ** 2 / 8
    links = [gen.near_identity(dims, 0.5, seed=70 + k).numpy().copy() for k in range(4)]
    f = tgf.Flow([dims] * 4, "f64")
    f.load_all([torch.from_numpy(l).cuda() for l in links])
    rows = f.flow(0.02, t_end, 0.0)
    t2E = rows[-1, :, tgf.OBS_FIELDS.index("t2E")]
    Q = rows[-1, :, tgf.OBS_FIELDS.index("Q")]
    qs = f.slice_charge(3)
    ref_rows = [oracle.flow(l.copy(), dims, 0.02, t_end, 0.0)[-1] for l in links]
    rt2E = np.array([r[2] for r in ref_rows])
    rQ = np.array([r[4] for r in ref_rows])
    assert np.allclose(t2E, rt2E, rtol=1e-12)
    lam, err = tgf.coupling(t2E, Q, c, L_t)
    lo, eo = stats.coupling(rt2E, rQ, c, L_t)
    assert lam == pytest.approx(lo, rel=1e-11)
    C, _ = tgf.charge_correlator(qs, Q)
    assert np.isfinite(C).all()
    V = float(np.prod(dims))
    chi, _ = tgf.susceptibility(Q, V)
    chi_o, _ = stats.susceptibility(rQ, V)
    assert chi == pytest.approx(chi_o, rel=1e-9, abs=1e-18)
