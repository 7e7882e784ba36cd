"""GPU: general SU(N) flow (the TGF scheme for SU(N), sec. 1; action, clover
and charge of sec. 3.1 with N colours) against the SU(N) oracle, through the
C ABI (tgf_create_sun).

Bars (FP64 path, as for SU(3)): t^2 E relative 1e-12 over rows with t > 0,
plaquette 1e-13, Q 1e-10 absolute, action relative 1e-12, final links 1e-12.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import fields_n                                     # noqa: E402
import oracle                                       # noqa: E402
from paper_2107_03747_amd import gen, tgf           # noqa: E402

oracle.set_threads(16)
OBS = tgf.OBS_FIELDS


def _compare_rows(rows, ref, label):
    assert rows.shape[0] == ref.shape[0], (rows.shape, ref.shape)
    t = ref[:, 0]
    pos = t > 0
    rel = np.abs(rows[:, OBS.index("t2E")] - ref[:, 2])[pos] / np.abs(ref[:, 2][pos])
    dpl = np.abs(rows[:, OBS.index("plaq")] - ref[:, 3]).max()
    dq = np.abs(rows[:, OBS.index("Q")] - ref[:, 4]).max()
    dact = (np.abs(rows[:, OBS.index("action")] - ref[:, 5]) / np.abs(ref[:, 5])).max()
    print(f"  {label}: max rel t2E {rel.max() if rel.size else 0:.3g}  max |dplaq| {dpl:.3g}  "
          f"max |dQ| {dq:.3g}  rel action {dact:.3g}", flush=True)
    assert np.allclose(rows[:, 0], t, rtol=0, atol=1e-12)
    if rel.size:
        assert rel.max() <= 1e-12
    assert dpl <= 1e-13 and dq <= 1e-10 and dact <= 1e-12


def _flow_both(N, dims_list, twists, starts, eps, t_end, meas_dt):
    """Every stage variant (rows per lane, permutes or LDS operands) of SU(N)
    against the oracle."""
    refs = []
    for k, (d, tw, s) in enumerate(zip(dims_list, twists, starts)):
        U = s.copy()
        ref = oracle.sun_flow(U, d, eps, t_end[k] if np.ndim(t_end) else t_end, meas_dt, twist=tw)
        refs.append((ref, U))
    nv = tgf.tgf_sun_variant_count(N)
    assert nv >= 1
    for v in range(nv):
        f = tgf.Flow([(d, t) for d, t in zip(dims_list, twists)], "f64", nc=N)
        f.set_variant(v)
        f.load_all([torch.from_numpy(s.copy()).cuda() for s in starts])
        rows = f.flow(eps, t_end, meas_dt)
        rpl = tgf.tgf_sun_rows_per_lane(N, v)
        kind = "LDS operands" if tgf.tgf_sun_variant_lds(N, v) == 1 else "permutes"
        for k, (d, tw) in enumerate(zip(dims_list, twists)):
            ref, U = refs[k]
            n = ref.shape[0]
            _compare_rows(rows[:n, k], ref, f"SU({N}) rows/lane {rpl} ({kind}) {d} twist {tw[0]}")
            got = f.store(k).cpu().numpy()
            dl = np.abs(got - U).max()
            print(f"    final links max |dU| {dl:.3g}", flush=True)
            assert dl <= 1e-12
            du, dd = f.unitarity(k)
            assert du < 1e-13 and dd < 1e-13
    return [U for _, U in refs]


@pytest.mark.parametrize("N,k", [(2, 1), (3, 1), (4, 1), (4, 3), (5, 2), (6, 1), (7, 3), (8, 3)])
def test_sun_flow_matches_oracle(N, k):
    """The TGF geometry l^2 x (N l)^2 with l = 2 (l = 4 for N = 2), the short
    plane twisted by k; near-identity links; 5 steps plus a short one."""
    l = 4 if N == 2 else 2
    d = (l, l, N * l, N * l)
    s = gen.near_identity_n(d, N, 0.4, seed=10 + N).numpy()
    _flow_both(N, [d], [(k, 0, 0, 0, 0, 0)], [s], 0.02, 0.11, 0.04)


@pytest.mark.parametrize("N", [3, 4, 6])
def test_sun_hot_start_and_ragged(N):
    """Haar starts, a ragged box (V not a multiple of 64) and several twisted
    planes, in one batch."""
    dims_list = [(3, 2, 5, 3), (2, 2, 2 * N, 2 * N)]
    twists = [(1, 0, N - 1, 1, 0, 2 % N), (1, 0, 0, 0, 0, 0)]
    starts = [gen.haar_n(d, N, seed=20 + j).numpy() for j, d in enumerate(dims_list)]
    _flow_both(N, dims_list, twists, starts, 0.01, [0.05, 0.03], 0.01)


def test_general_n3_equals_su3_path():
    """At N = 3 the general kernels and the SU(3)-specialised kernels compute
    the same flow (different arithmetic order)."""
    d = (4, 4, 12, 12)
    s = torch.from_numpy(gen.near_identity(d, 0.4, seed=5).numpy()).cuda()
    a = tgf.Flow([d], "f64")
    a.load(0, s)
    ra = a.flow(0.02, 0.2, 0.05)
    b = tgf.Flow([d], "f64", nc=3)
    b.load(0, s)
    rb = b.flow(0.02, 0.2, 0.05)
    assert ra.shape == rb.shape
    pos = ra[:, 0, 0] > 0
    rel = np.abs(ra[pos, 0, 2] - rb[pos, 0, 2]) / np.abs(ra[pos, 0, 2])
    assert rel.max() <= 1e-12
    assert (a.store(0) - b.store(0)).abs().max().item() <= 1e-12


@pytest.mark.parametrize("N,k", [(4, 3), (5, 2)])
def test_sun_twist_eater_is_fixed(N, k):
    d = (2, 2, 2 * N, 2 * N)
    U = fields_n.twist_eater_n(d, N, k)
    f = tgf.Flow([(d, (k, 0, 0, 0, 0, 0))], "f64", nc=N)
    f.load(0, torch.from_numpy(U).cuda())
    rows = f.flow(0.05, 0.2, 0.1)
    assert np.abs(rows[:, 0, OBS.index("E")]).max() < 1e-14
    assert np.abs(rows[:, 0, OBS.index("plaq")] - 1).max() < 1e-14
    assert np.abs(f.store(0).cpu().numpy() - U).max() < 1e-13


def test_sun_graph_and_direct_launches_agree():
    N, d = 4, (2, 2, 8, 8)
    s = torch.from_numpy(gen.near_identity_n(d, N, 0.5, seed=3).numpy()).cuda()
    outs = []
    for flags in (0, tgf.TGF_NO_GRAPH):
        f = tgf.Flow([d], "f64", nc=N)
        f.load(0, s)
        outs.append((f.flow(0.02, 0.1, 0.02, flags=flags), f.store(0)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])


def test_sun_errors():
    N, d = 4, (2, 2, 8, 8)
    with pytest.raises(tgf.TGFError):
        tgf.Flow([(d, (4, 0, 0, 0, 0, 0))], "f64", nc=N)          # twist >= N
    with pytest.raises(tgf.TGFError):
        tgf.Flow([d], "f32c12", nc=N)                              # FP64 only
    f = tgf.Flow([d], "f64", nc=N)
    bad = gen.near_identity_n(d, N, 0.5, seed=3)
    bad[0, 0, 0, 0, 0, 0, 0] += 1e-6
    with pytest.raises(tgf.TGFError) as e:
        f.load(0, bad.cuda())
    assert e.value.status == tgf.TGF_E_NOT_SU3
    f.load(0, gen.near_identity_n(d, N, 0.5, seed=3).cuda())
    for call in (lambda: f.mc(0.5, 1, 1), lambda: f.slice_charge(3)):
        with pytest.raises(tgf.TGFError) as e:
            call()
        assert e.value.status == tgf.TGF_E_UNSUPPORTED
    with pytest.raises(tgf.TGFError) as e:
        f.set_variant(tgf.tgf_sun_variant_count(N))
    assert e.value.status == tgf.TGF_E_INVAL
    v = f.autotune(None)                                           # times the rows-per-lane variants
    assert 0 <= v < tgf.tgf_sun_variant_count(N)
    f.set_variant(-1)
