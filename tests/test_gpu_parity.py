"""GPU parity: libtgf.so (through the C ABI) against the FP64 CPU oracle.

Bars (relative error of t^2 E over rows with t > 0): <= 1e-12 for the FP64
path, <= 1e-5 for both FP32 storages (the stated precision targets).  The
plaquette bar is 1e-13 (FP64) / 1e-6 (FP32) absolute and Q's 1e-10 / 1e-4.
The plaquette is an average over 6V plaquettes, so unbiased FP32 roundings
of the links cancel in it; what remains is a systematic drift of the link
norms off SU(3).  The link update is formed as U + (exp(X) - 1) U, so its
roundings have no preferred direction (forming exp(X) first rounded its
diagonal 1 - |X|^2/2 to 1 whenever |X|^2 < 2^-24 and grew every link's norm
by |X|^2 per stage, a plaquette offset of ~1e-6 after ten steps).  The FP32
unitarity bar, 2e-6, is the largest defect of a link after <= 30 stages of
unbiased roundings since the last reunitarisation (sqrt(30) x 1e-7 per
stage, about 3.5 standard deviations over the 147 456 links).  Workloads: synthetic seeded links of the shapes
the paper flows (L x L x 3L x 3L, twist n_01 = 1, sec. 3.1), eps = 0.01.
Full sizes beyond the oracle's reach are covered by properties in
test_gpu_properties.py.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle                                      # noqa: E402
import fields                                      # noqa: E402
from paper_2107_03747_amd import gen, tgf          # noqa: E402

oracle.set_threads(16)

TOL = {"f64": dict(t2E=1e-12, plaq=1e-13, Q=1e-10),
       "f32": dict(t2E=1e-5, plaq=1e-6, Q=1e-4),
       "f32c12": dict(t2E=1e-5, plaq=1e-6, Q=1e-4)}
COL = {n: k for k, n in enumerate(tgf.OBS_FIELDS)}


def say(*a):
    print(*a, flush=True)


def gpu_flow(dims_list, storage, links_list, eps, t_end, meas_dt, reunit=0, flags=0,
             variant=None, twist=None):
    say(f"  gpu_flow {storage} dims={dims_list} t_end={t_end} meas_dt={meas_dt} "
        f"reunit={reunit} flags={flags} variant={variant}")
    geoms = [(d, twist or tgf.PAPER_TWIST) for d in dims_list]
    f = tgf.Flow(geoms, storage)
    if variant is not None:
        f.set_variant(variant)
    f.load_all([torch.from_numpy(l).cuda() for l in links_list])
    rows = f.flow(eps, t_end, meas_dt, reunit, flags)
    return rows, f


def compare(rows_gpu, rows_ref, storage, label=""):
    tol = TOL[storage]
    assert rows_gpu.shape[0] == rows_ref.shape[0], (rows_gpu.shape, rows_ref.shape)
    assert np.allclose(rows_gpu[:, COL["t"]], rows_ref[:, 0], rtol=0, atol=1e-12)
    pos = rows_ref[:, 0] > 0
    e_rel = np.abs(rows_gpu[pos, COL["t2E"]] - rows_ref[pos, 2]) / np.abs(rows_ref[pos, 2])
    d_pl = np.abs(rows_gpu[:, COL["plaq"]] - rows_ref[:, 3])
    d_q = np.abs(rows_gpu[:, COL["Q"]] - rows_ref[:, 4])
    say(f"  {label} {storage}: max rel t2E {e_rel.max() if e_rel.size else 0:.3g}  "
        f"max |dplaq| {d_pl.max():.3g}  max |dQ| {d_q.max():.3g}")
    if e_rel.size:
        assert e_rel.max() <= tol["t2E"], e_rel
    assert d_pl.max() <= tol["plaq"]
    assert d_q.max() <= tol["Q"]
    return e_rel.max() if e_rel.size else 0.0


# ---------------------------------------------------------------------------
# small box: 4x4x12x12, U = exp(i 0.3 H), eps 0.01 to t = 0.32, t^2 E every 0.02

D1 = (4, 4, 12, 12)


@pytest.fixture(scope="module")
def d1():
    U = gen.near_identity(D1, 0.3, seed=1).numpy().copy()
    ref = oracle.flow(U.copy(), D1, 0.01, 0.32, 0.02)
    return U, ref


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_d1_parity(d1, storage):
    U, ref = d1
    rows, _ = gpu_flow([D1], storage, [U], 0.01, 0.32, 0.02)
    assert rows.shape[0] == 17
    compare(rows[:, 0], ref, storage, "D1")


# ---------------------------------------------------------------------------
# 8x8x24x24, near-identity (eps 0.3), eps 0.01 to c = 0.3 (t = 0.72), every 0.04

D2 = (8, 8, 24, 24)


@pytest.fixture(scope="module")
def d2():
    U = gen.near_identity(D2, 0.3, seed=2).numpy().copy()
    ref = oracle.flow(U.copy(), D2, 0.01, 0.72, 0.04)
    return U, ref


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_d2_parity(d2, storage):
    U, ref = d2
    rows, f = gpu_flow([D2], storage, [U], 0.01, 0.72, 0.04,
                       reunit=10 if storage != "f64" else 0)
    compare(rows[:, 0], ref, storage, "D2")
    du, dd = f.unitarity(0)
    say(f"  D2 {storage}: unitarity defects {du:.3g} {dd:.3g}")
    bar = 1e-13 if storage == "f64" else 2e-6
    assert du < bar and dd < bar


# ---------------------------------------------------------------------------
# 16x16x48x48 (the paper's largest lattice), Haar hot start: first steps

D3 = (16, 16, 48, 48)


@pytest.fixture(scope="module")
def d3():
    U = gen.haar(D3, seed=3).numpy().copy()
    ref = oracle.flow(U.copy(), D3, 0.01, 0.02, 0.01)
    return U, ref


@pytest.mark.parametrize("storage", ["f64", "f32c12"])
def test_d3_first_steps(d3, storage):
    U, ref = d3
    rows, _ = gpu_flow([D3], storage, [U], 0.01, 0.02, 0.01)
    compare(rows[:, 0], ref, storage, "D3")


# ---------------------------------------------------------------------------
# ragged sizes, degenerate extents, other twists, short final step

@pytest.mark.parametrize("dims,twist", [
    ((3, 3, 5, 7), (1, 0, 0, 0, 0, 0)),        # V = 315: ragged tiles
    ((2, 2, 2, 2), (1, 0, 0, 0, 0, 0)),        # n + mu = n - mu
    ((6, 6, 18, 18), (2, 0, 0, 0, 0, 0)),      # conjugate twist
    ((4, 3, 5, 2), (1, 2, 0, 0, 1, 1)),        # several twisted planes
    ((4, 4, 12, 12), (0, 0, 0, 0, 0, 0)),      # periodic
])
@pytest.mark.parametrize("storage", ["f64", "f32c12"])
def test_odd_shapes(dims, twist, storage):
    U = gen.haar(dims, seed=17).numpy().copy() if np.prod(dims) < 400 else \
        gen.near_identity(dims, 0.5, seed=17).numpy().copy()
    ref = oracle.flow(U.copy(), dims, 0.01, 0.035, 0.02, twist=twist)
    rows, _ = gpu_flow([dims], storage, [U], 0.01, 0.035, 0.02, twist=twist)
    assert np.allclose(rows[:, 0, 0], [0.0, 0.02, 0.035])
    compare(rows[:, 0], ref, storage, f"{dims}")


def test_no_step_and_short_step_only():
    dims = (4, 4, 12, 12)
    U = gen.near_identity(dims, 0.3, seed=5).numpy().copy()
    f = tgf.Flow([dims], "f64")
    f.load(0, torch.from_numpy(U).cuda(), t0=0.3)
    rows = f.flow(0.01, 0.3, 0.02)
    ref = oracle.flow(U.copy(), dims, 0.01, 0.3, 0.02, t0=0.3)
    compare(rows[:, 0], ref, "f64", "no-step")
    rows = f.flow(0.01, 0.304, 0.0)
    ref = oracle.flow(U.copy(), dims, 0.01, 0.304, 0.0, t0=0.3)
    compare(rows[:, 0], ref, "f64", "short-only")
    assert abs(f.time(0) - 0.304) < 1e-15


# ---------------------------------------------------------------------------
# batch: mixed L, different t_end, equals the solo runs

def test_batch_matches_solo_and_oracle():
    dims = [(6, 6, 18, 18), (4, 4, 12, 12), (3, 3, 5, 7)]
    links = [gen.near_identity(d, e, seed=40 + k).numpy().copy()
             for k, (d, e) in enumerate(zip(dims, (0.2, 0.3, 0.4)))]
    t_end = [0.405, 0.2, 0.125]
    for storage in ("f64", "f32c12"):
        f = tgf.Flow(dims, storage)
        f.load_all([torch.from_numpy(l).cuda() for l in links])
        rows = f.flow(0.01, t_end, 0.1, reunit_every=10)
        for k, d in enumerate(dims):
            g = tgf.Flow([d], storage)
            g.load(0, torch.from_numpy(links[k]).cuda())
            solo = g.flow(0.01, t_end[k], 0.1, reunit_every=10)
            n = solo.shape[0]
            assert np.array_equal(rows[:n, k], solo[:, 0]), (storage, d)
            # configs that finished early repeat their last row
            assert all(np.array_equal(rows[r, k], solo[-1, 0]) for r in range(n, rows.shape[0]))
            if storage == "f64":
                ref = oracle.flow(links[k].copy(), d, 0.01, t_end[k], 0.1)
                compare(solo[:, 0], ref, storage, f"batch {d}")


# ---------------------------------------------------------------------------
# execution modes and determinism

def test_graph_direct_timing_identical_and_deterministic():
    U = gen.near_identity(D2, 0.3, seed=9).numpy().copy()
    out = []
    for flags in (0, 0, tgf.TGF_NO_GRAPH, tgf.TGF_TIMING):
        rows, f = gpu_flow([D2], "f64", [U], 0.01, 0.1, 0.05, flags=flags)
        out.append((rows, f.store(0).cpu().numpy()))
        if flags == tgf.TGF_TIMING:
            tm = f.timing()
            assert tm["stage_launches"] == 30 and tm["stage_ms"] > 0
            V = np.prod(D2)
            assert tm["stage_bytes"] == pytest.approx(10 * V * 4480)
    for rows, links in out[1:]:
        assert np.array_equal(rows, out[0][0])
        assert np.array_equal(links, out[0][1])


def test_graph_replay_matches_eager():
    """The cached graph is replayed on later flows with eager work and
    synchronisations in between; every replay equals the eager result."""
    U = torch.from_numpy(gen.near_identity(D1, 0.4, seed=12).numpy().copy()).cuda()
    f = tgf.Flow([D1], "f32c12")
    eager = []
    for _ in range(2):
        f.load(0, U)
        eager.append(f.flow(0.01, 0.1, 0.05, flags=tgf.TGF_NO_GRAPH))
    for _ in range(4):
        f.load(0, U)
        junk = torch.randn(1 << 20, device="cuda").sum()     # eager work in between
        torch.cuda.synchronize()
        rows = f.flow(0.01, 0.1, 0.05)
        assert np.array_equal(rows, eager[0])
        del junk


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_variants_agree(storage):
    U = gen.near_identity(D1, 0.4, seed=13).numpy().copy()
    base, _ = gpu_flow([D1], storage, [U], 0.01, 0.1, 0.05, variant=0)
    tol = 1e-13 if storage == "f64" else 2e-6
    for v in range(1, tgf.tgf_variant_count()):
        rows, _ = gpu_flow([D1], storage, [U], 0.01, 0.1, 0.05, variant=v)
        rel = np.abs(rows[1:, 0, COL["t2E"]] - base[1:, 0, COL["t2E"]]) / np.abs(base[1:, 0, COL["t2E"]])
        assert rel.max() <= tol, (v, rel)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_lds_staged_variant_batch(storage):
    """The LDS-staged site variants (staged links; staged plaquettes reused as
    lower staple terms) on a batch whose work-groups straddle two
    configurations (the unstaged path), whose last tiles are ragged, whose
    (n0, n1) planes do and do not divide the 256-site block, with several
    twisted planes; every configuration against the oracle."""
    names = tgf.variant_names()
    dims_list = [(4, 4, 12, 12), (3, 5, 4, 7), (10, 10, 6, 6), (6, 6, 18, 18)]
    twists = [tgf.PAPER_TWIST, (1, 0, 2, 1, 0, 2), (2, 1, 0, 0, 1, 0), tgf.PAPER_TWIST]
    Us = [gen.near_identity(d, 0.35, seed=40 + k).numpy().copy() for k, d in enumerate(dims_list)]
    refs = [oracle.flow(U.copy(), d, 0.02, 0.1, 0.05, twist=tw)
            for U, d, tw in zip(Us, dims_list, twists)]
    for name in ("site_lds", "site_lds_xcd", "site_plq", "site_plq_xcd"):
        say(f"  variant {name}")
        f = tgf.Flow(list(zip(dims_list, twists)), storage)
        f.set_variant(names.index(name))
        f.load_all([torch.from_numpy(U).cuda() for U in Us])
        rows = f.flow(0.02, 0.1, 0.05)
        for k, d in enumerate(dims_list):
            compare(rows[:refs[k].shape[0], k], refs[k], storage, f"{name} {d}")


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_all_planes_twisted_plane_tiles(storage):
    """8x8 (n0, n1) planes fill a 64-site tile exactly, so the 12-real site
    kernel takes its lower staple terms in directions 0 and 1 from the
    plaquettes of neighbouring lanes; every plane twisted (n_{mu nu} = 1 or
    2), so each such term carries a twist factor of its own plane.  Default
    variant and both LDS block orders, against the oracle."""
    dims = (8, 8, 4, 6)
    twist = (1, 2, 1, 2, 1, 2)
    U = gen.near_identity(dims, 0.35, seed=77).numpy().copy()
    ref = oracle.flow(U.copy(), dims, 0.02, 0.1, 0.05, twist=twist)
    names = tgf.variant_names()
    for v in (None, names.index("site_lds"), names.index("site_lds_xcd")):
        rows, _ = gpu_flow([dims], storage, [U], 0.02, 0.1, 0.05, variant=v, twist=twist)
        compare(rows[:, 0], ref, storage, f"all planes twisted, variant {v}")


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_block_shapes_per_extent(storage):
    """The paper's mixed-L workload (Table A.1; the benchmark batch mixes
    L = 6, 8, 10) with the LDS-staged kernel at the whole-plane work-group
    shapes (252, 256, 200 sites) and at 256 sites for every L: each
    configuration against the oracle; FP64 and FP32 full shapes give the same
    bits (LDS or global memory, same arithmetic), and a configuration's result
    does not depend on the batch around it."""
    dims_list = [(6, 6, 18, 18), (8, 8, 24, 24), (10, 10, 30, 30)]
    Us = [gen.near_identity(d, 0.3, seed=60 + k).numpy().copy() for k, d in enumerate(dims_list)]
    refs = [oracle.flow(U.copy(), d, 0.02, 0.06, 0.02) for U, d in zip(Us, dims_list)]
    names = tgf.variant_names()
    out = {}
    for shapes in ("planes", "256"):
        f = tgf.Flow(dims_list, storage)
        f.set_variant(names.index("site_lds_xcd"))
        if shapes == "256":
            for k in range(len(dims_list)):
                f.set_block(k, 256)
        say(f"  {storage} shapes {[f.block(k) for k in range(len(dims_list))]}")
        f.load_all([torch.from_numpy(U).cuda() for U in Us])
        rows = f.flow(0.02, 0.06, 0.02, 10)
        for k, d in enumerate(dims_list):
            compare(rows[:, k], refs[k], storage, f"shapes {shapes} {d}")
        out[shapes] = rows
    if storage != "f32c12":
        assert np.array_equal(out["planes"], out["256"])
    # batch = solo, bitwise, at the whole-plane shapes
    for k, d in enumerate(dims_list):
        g = tgf.Flow([d], storage)
        g.set_variant(names.index("site_lds_xcd"))
        g.load(0, torch.from_numpy(Us[k]).cuda())
        solo = g.flow(0.02, 0.06, 0.02, 10)
        assert np.array_equal(solo[:, 0], out["planes"][:, k]), d


def test_autotune_per_extent(tmp_path):
    """The autotuner keeps the LDS-staged kernel unless another is 2% faster,
    and picks each extent class's work-group shape from {whole planes, 256}."""
    dims_list = [(6, 6, 18, 18), (8, 8, 24, 24), (10, 10, 30, 30)]
    Us = [torch.from_numpy(gen.near_identity(d, 0.3, seed=70 + k).numpy().copy()).cuda()
          for k, d in enumerate(dims_list)]
    f = tgf.Flow(dims_list * 2, "f32c12")
    f.load_all(Us * 2)
    cache = str(tmp_path / "tune.txt")
    v = f.autotune(cache)
    names = tgf.variant_names()
    say(f"  autotune: {names[v]}, shapes {[f.block(k) for k in range(6)]}")
    assert names[v].endswith("_xcd") and names[v] not in ("site_plq_xcd",)
    for k in range(3):
        assert f.block(k) == f.block(k + 3)
        assert f.block(k) in ({252, 256}, {256}, {200, 256})[k]
    g = tgf.Flow(dims_list * 2, "f32c12")
    g.load_all(Us * 2)
    assert g.autotune(cache) == v
    assert [g.block(k) for k in range(6)] == [f.block(k) for k in range(6)]


def test_resume_is_bitwise():
    U = torch.from_numpy(gen.near_identity(D1, 0.3, seed=14).numpy().copy()).cuda()
    a = tgf.Flow([D1], "f64")
    a.load(0, U)
    ra = a.flow(0.01, 0.2, 0.1)
    b = tgf.Flow([D1], "f64")
    b.load(0, U)
    b.flow(0.01, 0.1, 0.1)
    rb = b.flow(0.01, 0.2, 0.1)
    assert np.array_equal(ra[-1], rb[-1])
    assert torch.equal(a.store(0), b.store(0))


def test_store_load_roundtrip():
    U = torch.from_numpy(gen.haar(D1, seed=15).numpy().copy()).cuda()
    f = tgf.Flow([D1], "f64")
    f.load(0, U)
    assert torch.equal(f.store(0), U)
    g = tgf.Flow([D1], "f32c12")
    g.load(0, U)
    assert (g.store(0) - U).abs().max().item() < 1e-6


def test_autotune_picks_a_variant(tmp_path):
    U = torch.from_numpy(gen.near_identity(D2, 0.3, seed=16).numpy().copy()).cuda()
    f = tgf.Flow([D2], "f32c12")
    f.load(0, U)
    cache = str(tmp_path / "tune.txt")
    v = f.autotune(cache)
    assert 0 <= v < tgf.tgf_variant_count()
    # variants whose result depends on the rest of the batch are never chosen
    assert tgf.variant_names()[v] not in ("site_plq", "site_plq_xcd")
    g = tgf.Flow([D2], "f32c12")
    g.load(0, U)
    assert g.autotune(cache) == v          # read back from the cache
    # tuning does not change the state
    r1 = f.flow(0.01, 0.05, 0.0)
    h = tgf.Flow([D2], "f32c12")
    h.load(0, U)
    h.set_variant(v)
    h.set_block(0, f.block(0))
    assert np.array_equal(r1, h.flow(0.01, 0.05, 0.0))
