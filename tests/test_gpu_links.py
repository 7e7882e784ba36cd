"""Element-wise GPU parity of the flowed links and of the per-site densities,
the integrator against Luscher's tableau on torus fields, the LDS-staging
race check, failure injection and the reunitarisation schedule across calls
(all through the C ABI).

Links (sec. 3.1, the Wilson flow): the GPU's links after one RK3 step and
after the full 4x4x12x12 flow are compared entry by entry with the oracle's
(oracle.rk3_step / oracle.flow, which flow the array in place).  Bars:
  FP64   1e-13 absolute per entry (both sides are exact to rounding; their
         exponentials and summation orders differ, so a few hundred roundings
         of 1.1e-16 separate them);
  FP32   a link entry (|U_ij| <= 1) leaves every RK stage through a chain of
         about a dozen multiply-adds, each rounded to half an FP32 ulp
         (<= 2^-25 = 3e-8), plus the input rounding: <= 4e-7 per stage.  One
         step (3 stages) is bounded by 1.2e-6, bar 1.5e-6.  Over the 32-step
         flow the unbiased roundings add as a random walk (the exponential is
         formed as U + (exp(X) - 1) U, so no direction is preferred):
         sqrt(96) x 4e-7 = 4e-6, with a factor 2.5 for the largest of the
         73 728 entries, bar 1e-5.
Densities (eq. gmunu, eq. qlatt): e(n) and q(n) per site against
oracle.densities on the same links, FP64 1e-13 absolute, FP32 5e-6 (e, of
size <= 1 here, from a clover built of four-link leaves in FP32) and 1e-7
(q, which carries 1/(4 pi^2)).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import brute                                       # noqa: E402
import oracle                                      # noqa: E402
from paper_2107_03747_amd import gen, tgf          # noqa: E402

oracle.set_threads(16)

D1 = (4, 4, 12, 12)
LINK_BAR_1 = {"f64": 1e-13, "f32": 1.5e-6, "f32c12": 1.5e-6}
LINK_BAR_FLOW = {"f64": 1e-13, "f32": 1e-5, "f32c12": 1e-5}
DENS_BAR = {"f64": (1e-13, 1e-13), "f32": (5e-6, 1e-7), "f32c12": (5e-6, 1e-7)}


def say(*a):
    print(*a, flush=True)


def variant_index(name):
    return None if name is None else tgf.variant_names().index(name)


def gpu_links(dims, storage, U, eps, t_end, variant=None, twist=tgf.PAPER_TWIST, reunit=0):
    f = tgf.Flow([(dims, twist)], storage)
    if variant is not None:
        f.set_variant(variant_index(variant))
    f.load(0, torch.from_numpy(U).cuda())
    f.flow(eps, t_end, 0.0, reunit)
    out = f.store(0)
    torch.cuda.synchronize()
    return out.cpu().numpy(), f


@pytest.mark.parametrize("variant", [None, "site_lds", "site_lds_xcd"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_links_after_one_step(storage, variant):
    U = gen.near_identity(D1, 0.3, seed=1).numpy().copy()
    ref = U.copy()
    oracle.rk3_step(ref, D1, 0.01)
    got, _ = gpu_links(D1, storage, U, 0.01, 0.01, variant)
    d = np.abs(got - ref).max()
    say(f"  one step {storage} {variant}: max |dU| {d:.3g}")
    assert d <= LINK_BAR_1[storage]


@pytest.mark.parametrize("variant", [None, "site_lds", "site_lds_xcd"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_links_after_full_flow(storage, variant):
    U = gen.near_identity(D1, 0.3, seed=1).numpy().copy()
    ref = U.copy()
    oracle.flow(ref, D1, 0.01, 0.32, 0.0)
    got, _ = gpu_links(D1, storage, U, 0.01, 0.32, variant)
    d = np.abs(got - ref).max()
    say(f"  32 steps {storage} {variant}: max |dU| {d:.3g}")
    assert d <= LINK_BAR_FLOW[storage]


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_links_every_plane_twisted(storage):
    """8x8 planes fill a wave (the 12-real kernel's in-wave plaquette reuse)
    and every plane carries its own twist: links entry by entry after 5 steps."""
    dims, twist = (8, 8, 4, 6), (1, 2, 1, 2, 1, 2)
    U = gen.near_identity(dims, 0.35, seed=77).numpy().copy()
    ref = U.copy()
    oracle.flow(ref, dims, 0.02, 0.1, 0.0, twist=twist)
    for v in (None, "site_lds", "site_lds_xcd"):
        got, _ = gpu_links(dims, storage, U, 0.02, 0.1, v, twist)
        d = np.abs(got - ref).max()
        say(f"  every plane twisted {storage} {v}: max |dU| {d:.3g}")
        # 5 steps: between the one-step and the 32-step bars
        assert d <= (1e-13 if storage == "f64" else 5e-6)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_links_column_launch_order(storage):
    """A box whose n3 slice spans more than 64 LDS work-groups (16x16x72:
    72 blocks of 256 sites) runs them in columns of 12 blocks along n2, each
    column through all n3 (block_order): links entry by entry against the
    oracle after two steps, and the same box in a batch with a site-order
    box (8x8x24x24) gives bitwise its solo links."""
    dims, other = (16, 16, 72, 4), (8, 8, 24, 24)
    U = gen.near_identity(dims, 0.3, seed=91).numpy().copy()
    W = gen.near_identity(other, 0.3, seed=92).numpy().copy()
    ref = U.copy()
    oracle.flow(ref, dims, 0.01, 0.02, 0.0)
    got, _ = gpu_links(dims, storage, U, 0.01, 0.02, "site_lds_xcd")
    d = np.abs(got - ref).max()
    say(f"  column order {storage}: max |dU| {d:.3g}")
    assert d <= (1e-13 if storage == "f64" else 3e-6)      # two steps
    f = tgf.Flow([other, dims], storage)
    f.set_variant(variant_index("site_lds_xcd"))
    f.load_all([torch.from_numpy(W).cuda(), torch.from_numpy(U).cuda()])
    f.flow(0.01, 0.02, 0.0, 0)
    assert np.array_equal(f.store(1).cpu().numpy(), got)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
@pytest.mark.parametrize("twist", [tgf.PAPER_TWIST, (1, 2, 1, 2, 1, 2)])
def test_torus_flow_is_luschers_tableau(storage, twist):
    """The GPU integrator against a reference that does not go through the
    oracle: on links in the maximal torus of SU(3) the flow is an ODE for the
    angles (tests/brute.py, from the action), and Luscher's RK3 is there the
    classical tableau c = (0, 1/4, 2/3), b = (1/4, 0, 3/4).  Two steps of 0.05
    on a hot torus field (angles up to 2.5), 8x8 planes that fill a wave; the
    other third-order tableaus lie 1e-5 and more away."""
    dims, h = (8, 8, 4, 6), 0.05
    ang = brute.torus_angles(dims, 3, seed=41, scale=2.5)
    refs = {}
    for name, tab in brute.RK3_TABLEAUS.items():
        a = ang
        for _ in range(2):
            a = brute.torus_rk3(a, dims, h, twist, tab)
        refs[name] = brute.torus_links(a)
    got, _ = gpu_links(dims, storage, brute.torus_links(ang), h, 2 * h, None, twist)
    d = {k: np.abs(got - r).max() for k, r in refs.items()}
    say(f"  torus {storage} {twist}: " + " ".join(f"{k} {v:.3g}" for k, v in d.items()))
    assert d["luscher"] <= (1e-13 if storage == "f64" else 3e-6)
    assert min(v for k, v in d.items() if k != "luscher") > 1e-5


def test_large_box_one_step_vs_oracle():
    """The 32x32x96x96 Haar box of the benchmark's large leg (9.4M sites,
    column launch order, site_lds_xcd): one RK3 step, every link entry of
    the FP64, FP32 full and FP32 12-real flows against the oracle's step."""
    dims = (32, 32, 96, 96)
    U = gen.haar(dims, seed=5, device="cuda")
    ref = U.cpu().numpy().copy()
    say("  D5: oracle step (16 threads)")
    oracle.rk3_step(ref, dims, 0.01)
    ref_dev = torch.from_numpy(ref).cuda()
    del ref
    for storage in ("f64", "f32", "f32c12"):
        f = tgf.Flow([dims], storage)
        f.set_variant(variant_index("site_lds_xcd"))
        f.load(0, U)
        f.flow(0.01, 0.01, 0.0, 10)
        d = (f.store(0) - ref_dev).abs().max().item()
        say(f"  D5 one step {storage}: max |dU| {d:.3g}")
        assert d <= LINK_BAR_1[storage]
        del f
        torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
@pytest.mark.parametrize("case", ["d1", "twisted"])
def test_densities(storage, case):
    if case == "d1":
        dims, twist, U = D1, tgf.PAPER_TWIST, gen.near_identity(D1, 0.3, seed=1).numpy().copy()
    else:
        dims, twist = (8, 8, 4, 6), (1, 2, 1, 2, 1, 2)
        U = gen.near_identity(dims, 0.35, seed=77).numpy().copy()
    f = tgf.Flow([(dims, twist)], storage)
    f.load(0, torch.from_numpy(U).cuda())
    e_bar, q_bar = DENS_BAR[storage]
    for step in range(2):
        if step == 1:
            # after a flow, on the GPU's own links (stored back in FP64)
            f.flow(0.02, 0.1, 0.0)
            U = f.store(0).cpu().numpy()
        e, q = f.densities(0)
        torch.cuda.synchronize()
        e, q = e.cpu().numpy(), q.cpu().numpy()
        # the FP32 storages hold the links rounded to FP32: the oracle reads
        # the same rounded links back (store), so only the measurement differs
        ref_links = f.store(0).cpu().numpy() if storage != "f64" else U
        er, qr = oracle.densities(ref_links, dims, twist)
        de, dq = np.abs(e - er).max(), np.abs(q - qr).max()
        say(f"  densities {case} {storage} t={'0' if step == 0 else '0.1'}: max |de| {de:.3g} "
            f"(max e {np.abs(er).max():.3g}), max |dq| {dq:.3g} (max q {np.abs(qr).max():.3g})")
        assert de <= e_bar and dq <= q_bar
        # the densities sum to the measured observables
        m = f.measure()[0]
        cols = {n: k for k, n in enumerate(tgf.OBS_FIELDS)}
        assert abs(e.mean() - m[cols["E"]]) <= 1e-12 * max(1.0, abs(m[cols["E"]]))
        assert abs(q.sum() - m[cols["Q"]]) <= 1e-10


@pytest.mark.parametrize("storage", ["f64", "f32", "f32c12"])
def test_lds_staging_is_bitwise(storage):
    """Race check: a kernel reading its block's links from LDS and one reading
    them from global memory run the same arithmetic, so a missing barrier or
    a stale LDS entry would show as a bit difference.  FP64 and FP32 full: the
    global-memory site kernel (two block orders, two register budgets) against
    the LDS-staged one (two block orders).  12-real: the LDS kernel (in-wave
    plaquette reuse) in both block orders, and the global-memory kernels among
    themselves.  Rows and stored links bitwise, on a batch with ragged tiles,
    work-groups straddling configurations and three twist patterns."""
    dims_list = [(4, 4, 12, 12), (3, 5, 4, 7), (10, 10, 6, 6), (6, 6, 18, 18)]
    twists = [tgf.PAPER_TWIST, (1, 0, 2, 1, 0, 2), (2, 1, 0, 0, 1, 0), tgf.PAPER_TWIST]
    Us = [torch.from_numpy(gen.near_identity(d, 0.35, seed=40 + k).numpy().copy()).cuda()
          for k, d in enumerate(dims_list)]
    if storage == "f32c12":
        groups = [("site_lds", "site_lds_xcd"),
                  ("site_alg", "site_alg_xcd", "site_alg3", "site_alg3_xcd")]
    else:
        groups = [("site_alg", "site_alg_xcd", "site_alg3", "site_alg3_xcd", "site_lds",
                   "site_lds_xcd")]
    for group in groups:
        first = None
        for name in group:
            f = tgf.Flow(list(zip(dims_list, twists)), storage)
            f.set_variant(variant_index(name))
            f.load_all(Us)
            rows = f.flow(0.02, 0.1, 0.05, 10)
            links = [f.store(k).cpu() for k in range(len(dims_list))]
            if first is None:
                first = (name, rows, links)
                continue
            say(f"  {storage}: {name} vs {first[0]}")
            assert np.array_equal(rows, first[1]), name
            for k in range(len(dims_list)):
                assert torch.equal(links[k], first[2][k]), (name, k)


@pytest.mark.parametrize("storage", ["f64", "f32c12"])
def test_nonfinite_after_flow(storage):
    """Failure injection from the host: a NaN written into a stored link of the
    caller-owned workspace spreads through the stencil, and the flow reports
    TGF_E_NONFINITE (every kernel still runs to its end)."""
    U = torch.from_numpy(gen.near_identity(D1, 0.3, seed=5).numpy().copy()).cuda()
    f = tgf.Flow([D1], storage)
    f.load(0, U)
    f.flow(0.01, 0.02, 0.0)
    off, nb = f.link_buffer(0)
    assert off % 256 == 0 and off + nb <= f.workspace.numel()
    dt = torch.float64 if storage == "f64" else torch.float32
    w = f.workspace[off:off + nb].view(dt)
    w[5] = float("nan")                      # one real part of one link entry
    torch.cuda.synchronize()
    with pytest.raises(tgf.TGFError) as ei:
        f.flow(0.01, 0.05, 0.01)
    assert ei.value.status == tgf.TGF_E_NONFINITE
    with pytest.raises(tgf.TGFError) as ei:
        f.measure()
    assert ei.value.status == tgf.TGF_E_NONFINITE
    # a fresh load recovers the context
    f.load(0, U)
    rows = f.flow(0.01, 0.02, 0.0)
    assert np.isfinite(rows).all()


@pytest.mark.parametrize("storage", ["f32", "f32c12"])
def test_reunit_schedule_across_calls(storage):
    """Reunitarisation every 10 steps counts steps from the load, so a flow
    split into calls of any length (7 + 16 + 9 steps, or 3 at a time) gives
    the same links and rows, bitwise, as one call."""
    U = torch.from_numpy(gen.near_identity(D1, 0.3, seed=14).numpy().copy()).cuda()
    one = tgf.Flow([D1], storage)
    one.load(0, U)
    r_one = one.flow(0.01, 0.32, 0.0, 10)
    l_one = one.store(0).cpu()
    for cuts in ((0.07, 0.23), tuple(0.03 * k for k in range(1, 11))):
        f = tgf.Flow([D1], storage)
        f.load(0, U)
        for t in cuts:
            f.flow(0.01, t, 0.0, 10)
        r = f.flow(0.01, 0.32, 0.0, 10)
        assert torch.equal(f.store(0).cpu(), l_one), cuts
        # observables (t itself is summed differently: t0 + k eps per call)
        assert np.array_equal(r[-1, 0, [1, 3, 4, 5]], r_one[-1, 0, [1, 3, 4, 5]]), cuts
    # and reunitarisation does act: without it the links differ
    g = tgf.Flow([D1], storage)
    g.load(0, U)
    g.flow(0.01, 0.32, 0.0, 0)
    assert not torch.equal(g.store(0).cpu(), l_one)
