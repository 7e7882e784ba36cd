"""Maximum sizes: boxes of 137M and 196M sites, where the kernels' 32-bit
per-lane byte offsets (16-byte units, site index x 16) pass 2^31.

The flow (sec. 3.1) commutes with translations along the untwisted directions
2 and 3: the twist factor of the (0,1) planes sits at n0 = n1 = 0 for every
n2, n3, and nothing else in the action depends on position.  So a box built
of K x K copies of an 8x8x24x24 configuration along directions 2 and 3 flows
into K x K copies of the flowed 8x8x24x24 box.  Here the copies are compared
with the small box flowed alone, bit for bit: the LDS-staged stage kernel
works on blocks of four whole (n0, n1) planes, which tile 24 planes, so every
site of every copy takes the arithmetic of its counterpart in the small box
(the same in-wave plaquette reuse, the same lower terms formed directly), and
the links it reads hold the same bits.  The small box is checked against the
oracle's RK3 step entry by entry (bars of the one-step link parity).  Rows:
t^2 E and the plaquette are averages, equal to the small box's up to the
order of the FP64 sums; Q and the action are sums, K^2 times the small box's.

Sizes: FP32 12-real on 8x8x1752x1752 (196 M sites, lane offsets up to
3.1e9; 100 GB workspace + 113 GB of canonical links), FP32 full on
8x8x1464x1464 (137 M sites, lane offsets up to 2.2e9; 97 + 79 GB).  The FP64
storage would need 272 GB at the 2^31 crossing and is left to the host audit
of the same offset code (tests/sanitize/index_audit.cpp), which also covers
boxes at the site cap of 2^28 - 256.

SU(N) (FP64, N^2 entry planes per direction, sites capped at 2^28 / N^2 -
256 so that a lane's offset into a direction's planes fits in 32 bits): boxes
just under the cap, SU(5) on 2x2x1630x1640 (10.7 M sites) and SU(8) on
2x2x1008x1040 (4.19 M sites), whose largest offsets are 4.28e9 and 4.29e9 of
2^32, built of copies of 2x2x10x10 and 2x2x16x16 fields; every stage variant
(LDS operands, cross-lane permutes) flows them bitwise like the small box,
whose step is checked against the SU(N) oracle (1e-12).  The SU(N) kernels
take no position-dependent path (no wave votes), so every copy's arithmetic
is that of the small box.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle                                      # noqa: E402
from paper_2107_03747_amd import gen, tgf          # noqa: E402

oracle.set_threads(16)

SMALL = (8, 8, 24, 24)
COPIES = {"f32c12": 73, "f32": 61}
LINK_BAR_1 = 1.5e-6
COL = {k: i for i, k in enumerate(tgf.OBS_FIELDS)}


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("storage", ["f32c12", "f32"])
def test_replicated_box_flows_like_its_copy(storage):
    K = COPIES[storage]
    big = (SMALL[0], SMALL[1], SMALL[2] * K, SMALL[3] * K)
    V = int(np.prod(big))
    assert V * 16 > 1 << 31 and V <= (1 << 28) - 256
    ws = tgf.workspace_bytes([big], storage)
    links_bytes = V * 4 * 9 * 16
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < ws + links_bytes + (4 << 30):
        pytest.skip(f"needs {(ws + links_bytes) / 1e9:.0f} GB of device memory, "
                    f"{free / 1e9:.0f} GB free")

    U = gen.near_identity(SMALL, 0.3, seed=7)
    ref = U.numpy().copy()
    oracle.rk3_step(ref, SMALL, 0.01)

    say(f"  small {SMALL} {storage}: one step with rows at t = 0, 0.01")
    fs = tgf.Flow([SMALL], storage)
    fs.load(0, U.cuda())
    rows_s = fs.flow(0.01, 0.01, 0.01)
    small = fs.store(0)
    torch.cuda.synchronize()
    d = np.abs(small.cpu().numpy() - ref).max()
    say(f"  small vs oracle: max |dU| {d:.3g}")
    assert d <= LINK_BAR_1
    fs.close()

    say(f"  big {big} ({V} sites, {ws / 1e9:.1f} GB workspace) {storage}: load")
    links = U.cuda().repeat(K, K, 1, 1, 1, 1, 1)
    fb = tgf.Flow([big], storage)
    fb.load(0, links)
    say("  big: flow one step")
    rows_b = fb.flow(0.01, 0.01, 0.01)
    say("  big: store")
    fb.store(0, out=links)
    torch.cuda.synchronize()
    fb.close()
    del fb
    torch.cuda.empty_cache()

    say("  big: compare the copies with the small box")
    bv = links.view(K, SMALL[3], K, SMALL[2], -1)
    sv = small.view(SMALL[3], 1, SMALL[2], -1)
    differing = 0
    for a in range(K):
        differing += int((bv[a] != sv).any(dim=-1).sum().item())
    say(f"  copies: {K * K}, sites differing from the small box: {differing}")
    assert differing == 0

    assert rows_b.shape == rows_s.shape == (2, 1, 6)
    rb, rs = rows_b[:, 0], rows_s[:, 0]
    n = K * K
    assert np.array_equal(rb[:, COL["t"]], rs[:, COL["t"]])
    pos = rs[:, COL["t"]] > 0                       # t^2 E vanishes at t = 0
    for col, scale, rows in (("t2E", 1, pos), ("E", 1, slice(None)), ("plaq", 1, slice(None)),
                             ("action", n, slice(None))):
        b, s_ = rb[rows, COL[col]], scale * rs[rows, COL[col]]
        rel = np.abs(b - s_) / np.abs(s_)
        say(f"  rows {col}: max rel {rel.max():.3g}")
        assert rel.max() <= 1e-11, (col, rb[:, COL[col]], rs[:, COL[col]])
    dq = np.abs(rb[:, COL["Q"]] - n * rs[:, COL["Q"]])
    say(f"  rows Q: {rb[:, COL['Q']]} vs {n} x {rs[:, COL['Q']]}")
    assert dq.max() <= 1e-9 * n
    del links
    torch.cuda.empty_cache()


SUN_CASES = {5: ((2, 2, 10, 10), 2, (163, 164)), 8: ((2, 2, 16, 16), 3, (63, 65))}


@pytest.mark.parametrize("N", [5, 8])
def test_sun_replicated_box_at_the_site_cap(N):
    small_dims, k, (k2, k3) = SUN_CASES[N]
    twist = (k, 0, 0, 0, 0, 0)
    big = (small_dims[0], small_dims[1], small_dims[2] * k2, small_dims[3] * k3)
    V = int(np.prod(big))
    cap = (1 << 28) // (N * N) - 256
    assert 0.99 * cap < V <= cap
    links_bytes = V * 4 * N * N * 16
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 4 * links_bytes + (4 << 30):       # workspace (3 x links) + links
        pytest.skip(f"needs {4 * links_bytes / 1e9:.0f} GB of device memory")

    U = gen.near_identity_n(small_dims, N, 0.4, seed=70 + N)
    ref = U.numpy().copy()
    oracle.sun_rk3_step(ref, small_dims, 0.01, twist=twist)
    for v in range(tgf.tgf_sun_variant_count(N)):
        kind = "LDS operands" if tgf.tgf_sun_variant_lds(N, v) == 1 else "permutes"
        say(f"  SU({N}) variant {v} ({kind}): small {small_dims}")
        fs = tgf.Flow([(small_dims, twist)], "f64", nc=N)
        fs.set_variant(v)
        fs.load(0, U.cuda())
        rows_s = fs.flow(0.01, 0.01, 0.01)
        small = fs.store(0)
        torch.cuda.synchronize()
        d = np.abs(small.cpu().numpy() - ref).max()
        say(f"  small vs oracle: max |dU| {d:.3g}")
        assert d <= 1e-12
        fs.close()

        say(f"  big {big} ({V} sites, cap {cap}): load, one step, store")
        links = U.cuda().repeat(k3, k2, 1, 1, 1, 1, 1)
        fb = tgf.Flow([(big, twist)], "f64", nc=N)
        fb.set_variant(v)
        fb.load(0, links)
        rows_b = fb.flow(0.01, 0.01, 0.01)
        fb.store(0, out=links)
        torch.cuda.synchronize()
        fb.close()
        del fb
        torch.cuda.empty_cache()
        bv = links.view(k3, small_dims[3], k2, small_dims[2], -1)
        sv = small.view(small_dims[3], 1, small_dims[2], -1)
        differing = sum(int((bv[a] != sv).any(dim=-1).sum().item()) for a in range(k3))
        say(f"  copies: {k2 * k3}, sites differing from the small box: {differing}")
        assert differing == 0
        rb, rs = rows_b[:, 0], rows_s[:, 0]
        for col in ("E", "plaq"):
            rel = np.abs(rb[:, COL[col]] - rs[:, COL[col]]) / np.abs(rs[:, COL[col]])
            assert rel.max() <= 1e-11, (col, rb[:, COL[col]], rs[:, COL[col]])
        rel = np.abs(rb[:, COL["action"]] - k2 * k3 * rs[:, COL["action"]]) / np.abs(
            k2 * k3 * rs[:, COL["action"]])
        assert rel.max() <= 1e-11
        del links
        torch.cuda.empty_cache()
