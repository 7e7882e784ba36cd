"""C-ABI boundary checks that need no GPU: the library loads, exports every
function include/tgf.h declares, and rejects bad arguments on the host
before anything is enqueued (the validation paths return before any HIP
call, so they run on a machine without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgf.h")

tgf = pytest.importorskip("paper_2107_03747_amd.tgf",
                          reason="libtgf.so not built (python -m paper_2107_03747_amd.build)")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tgf_\w+)\s*\(", text)))


def test_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(tgf.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in tgf.h but not exported"
    assert set(names) == set(tgf.EXPORTED)


def test_workspace_bytes_validation():
    g = tgf.make_geoms([(4, 4, 12, 12)])
    assert tgf.tgf_workspace_bytes(1, g, tgf.TGF_F64_FULL) > 0
    assert tgf.tgf_workspace_bytes(0, g, tgf.TGF_F64_FULL) == 0
    assert tgf.tgf_workspace_bytes(1, g, 7) == 0
    assert tgf.tgf_workspace_bytes(1, tgf.make_geoms([(1, 4, 12, 12)]), 0) == 0
    assert tgf.tgf_workspace_bytes(1, tgf.make_geoms([((4, 4, 12, 12), (3, 0, 0, 0, 0, 0))]),
                                   0) == 0
    assert tgf.tgf_workspace_bytes(1, tgf.make_geoms([(2048, 2048, 512, 2)]), 0) == 0


def test_workspace_sizes_scale_with_storage():
    g = [(8, 8, 24, 24)]
    V = 8 * 8 * 24 * 24
    f64 = tgf.workspace_bytes(g, "f64")
    f32 = tgf.workspace_bytes(g, "f32")
    c12 = tgf.workspace_bytes(g, "f32c12")
    # two link buffers + X: (2*4*9 + 4*4) complex/site, 16 bytes each in FP64, 8 in FP32
    assert f64 - f32 == pytest.approx(V * (2 * 4 * 9 + 4 * 4) * 8, abs=4096)
    assert f32 - c12 == pytest.approx(V * (2 * 4 * 3 * 8), abs=4096)
    # per-site storage: 1408 / 704 / 512 bytes (the shared tables are a small
    # constant on top: descriptors, partials, rows, schedule)
    g2 = [(8, 8, 24, 48)]
    for st, per_site in (("f64", 1408), ("f32", 704), ("f32c12", 512)):
        assert tgf.workspace_bytes(g2, st) - tgf.workspace_bytes(g, st) == pytest.approx(
            V * per_site, rel=0.01)


FAKE = 1 << 40   # an aligned address; validation never dereferences it


def make_ctx(st=tgf.TGF_F64_FULL, geoms=((4, 4, 12, 12),)):
    g = tgf.make_geoms(list(geoms))
    need = tgf.tgf_workspace_bytes(len(geoms), g, st)
    ctx = ctypes.c_void_p()
    rc = tgf.tgf_create(ctypes.byref(ctx), len(geoms), g, st, ctypes.c_void_p(FAKE), need, None)
    return rc, ctx, need


def test_create_errors():
    g = tgf.make_geoms([(4, 4, 12, 12)])
    need = tgf.tgf_workspace_bytes(1, g, 0)
    ctx = ctypes.c_void_p()
    assert tgf.tgf_create(ctypes.byref(ctx), 1, g, 0, ctypes.c_void_p(FAKE), need - 1,
                          None) == tgf.TGF_E_SIZE
    assert b"too small" in tgf.tgf_last_error()
    assert tgf.tgf_create(ctypes.byref(ctx), 1, g, 0, ctypes.c_void_p(FAKE + 8), need,
                          None) == tgf.TGF_E_INVAL
    assert tgf.tgf_create(ctypes.byref(ctx), 1, g, 0, None, need, None) == tgf.TGF_E_INVAL
    assert tgf.tgf_create(ctypes.byref(ctx), 0, g, 0, ctypes.c_void_p(FAKE), need,
                          None) == tgf.TGF_E_INVAL
    assert tgf.tgf_create(None, 1, g, 0, ctypes.c_void_p(FAKE), need, None) == tgf.TGF_E_INVAL
    assert tgf.tgf_create(ctypes.byref(ctx), 1, g, 9, ctypes.c_void_p(FAKE), need,
                          None) == tgf.TGF_E_INVAL


def test_state_and_argument_errors_before_any_enqueue():
    rc, ctx, _ = make_ctx()
    assert rc == tgf.TGF_OK and ctx
    try:
        obs = (tgf.tgf_obs * 4)()
        te = (ctypes.c_double * 1)(0.1)
        p = tgf.tgf_flow_params(0.01, te, 0.0, 0, 0)
        nr = ctypes.c_int32()
        # nothing loaded yet
        assert tgf.tgf_flow(ctx, ctypes.byref(p), obs, 4, ctypes.byref(nr)) == tgf.TGF_E_STATE
        assert tgf.tgf_measure(ctx, obs) == tgf.TGF_E_STATE
        assert tgf.tgf_store_links(ctx, 0, ctypes.c_void_p(FAKE)) == tgf.TGF_E_STATE
        assert tgf.tgf_autotune(ctx, None) == tgf.TGF_E_STATE
        d2 = (ctypes.c_double * 2)()
        assert tgf.tgf_unitarity(ctx, 0, d2) == tgf.TGF_E_STATE
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        assert tgf.tgf_link_buffer(ctx, 0, ctypes.byref(off), ctypes.byref(nb)) == tgf.TGF_E_STATE
        assert tgf.tgf_link_buffer(ctx, 0, None, ctypes.byref(nb)) == tgf.TGF_E_INVAL
        assert tgf.tgf_link_buffer(ctx, 2, ctypes.byref(off), ctypes.byref(nb)) == tgf.TGF_E_INVAL
        assert tgf.tgf_densities(ctx, 0, ctypes.c_void_p(FAKE), None) == tgf.TGF_E_STATE
        assert tgf.tgf_densities(ctx, -1, ctypes.c_void_p(FAKE), None) == tgf.TGF_E_INVAL
        # bad flow parameters
        for eps in (0.0, -0.01, float("nan"), float("inf")):
            p = tgf.tgf_flow_params(eps, te, 0.0, 0, 0)
            assert tgf.tgf_flow(ctx, ctypes.byref(p), obs, 4, ctypes.byref(nr)) == tgf.TGF_E_INVAL
        p = tgf.tgf_flow_params(0.01, te, -1.0, 0, 0)
        assert tgf.tgf_flow(ctx, ctypes.byref(p), obs, 4, ctypes.byref(nr)) == tgf.TGF_E_INVAL
        p = tgf.tgf_flow_params(0.01, te, 0.0, -2, 0)
        assert tgf.tgf_flow(ctx, ctypes.byref(p), obs, 4, ctypes.byref(nr)) == tgf.TGF_E_INVAL
        p = tgf.tgf_flow_params(0.01, None, 0.0, 0, 0)
        assert tgf.tgf_flow(ctx, ctypes.byref(p), obs, 4, ctypes.byref(nr)) == tgf.TGF_E_INVAL
        p = tgf.tgf_flow_params(0.01, te, 0.0, 0, 0)
        assert tgf.tgf_flow(ctx, ctypes.byref(p), obs, 0, ctypes.byref(nr)) == tgf.TGF_E_SIZE
        # bad loads (host checks come before the device check)
        assert tgf.tgf_load_links(ctx, 0, None, 0.0) == tgf.TGF_E_INVAL
        assert tgf.tgf_load_links(ctx, 0, ctypes.c_void_p(FAKE), -1.0) == tgf.TGF_E_INVAL
        assert tgf.tgf_load_links(ctx, 0, ctypes.c_void_p(FAKE), float("nan")) == tgf.TGF_E_INVAL
        assert tgf.tgf_load_links(ctx, 1, ctypes.c_void_p(FAKE), 0.0) == tgf.TGF_E_INVAL
        assert tgf.tgf_load_links(ctx, -1, ctypes.c_void_p(FAKE), 0.0) == tgf.TGF_E_INVAL
        assert tgf.tgf_store_links(ctx, 0, None) == tgf.TGF_E_INVAL
        t = ctypes.c_double(-1)
        assert tgf.tgf_get_time(ctx, 0, ctypes.byref(t)) == tgf.TGF_OK and t.value == 0.0
        assert tgf.tgf_get_time(ctx, 3, ctypes.byref(t)) == tgf.TGF_E_INVAL
        assert tgf.tgf_set_variant(ctx, 99) == tgf.TGF_E_INVAL
        assert tgf.tgf_set_variant(ctx, 1) == tgf.TGF_OK and tgf.tgf_get_variant(ctx) == 1
        assert tgf.tgf_set_variant(ctx, -1) == tgf.TGF_OK
        assert tgf.tgf_stream_copy(ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE + 4), 16,
                                   None) == tgf.TGF_E_INVAL
    finally:
        tgf.tgf_destroy(ctx)


def test_block_shapes_default_to_whole_planes():
    """LDS work-groups hold whole (n0, n1) planes of the L x L x 3L x 3L boxes
    when at least half the 256 threads get work, else 256 sites."""
    dims = [(6, 6, 18, 18), (8, 8, 24, 24), (10, 10, 30, 30), (12, 12, 36, 36), (16, 16, 48, 48),
            (32, 32, 96, 96), (3, 5, 4, 7), (9, 20, 4, 4), (20, 20, 4, 4)]
    want = [252, 256, 200, 144, 256, 256, 255, 180, 256]
    rc, ctx, _ = make_ctx(tgf.TGF_F32_C12, dims)
    assert rc == tgf.TGF_OK
    try:
        v = ctypes.c_int32()
        for k, w in enumerate(want):
            assert tgf.tgf_get_block(ctx, k, ctypes.byref(v)) == tgf.TGF_OK and v.value == w, k
        assert tgf.tgf_set_block(ctx, 0, 256) == tgf.TGF_OK
        assert tgf.tgf_get_block(ctx, 0, ctypes.byref(v)) == tgf.TGF_OK and v.value == 256
        assert tgf.tgf_set_block(ctx, 0, 0) == tgf.TGF_OK
        assert tgf.tgf_get_block(ctx, 0, ctypes.byref(v)) == tgf.TGF_OK and v.value == 252
        for bad in (63, 257, -1):
            assert tgf.tgf_set_block(ctx, 0, bad) == tgf.TGF_E_INVAL
        assert tgf.tgf_set_block(ctx, len(dims), 256) == tgf.TGF_E_INVAL
        assert tgf.tgf_get_block(ctx, 0, None) == tgf.TGF_E_INVAL
    finally:
        tgf.tgf_destroy(ctx)


def test_null_context_is_rejected():
    obs = (tgf.tgf_obs * 1)()
    assert tgf.tgf_measure(None, obs) == tgf.TGF_E_INVAL
    assert tgf.tgf_load_links(None, 0, ctypes.c_void_p(FAKE), 0.0) == tgf.TGF_E_INVAL
    assert tgf.tgf_densities(None, 0, None, None) == tgf.TGF_E_INVAL
    tgf.tgf_destroy(None)


def test_variant_table():
    names = tgf.variant_names()
    assert names[:2] == ["site", "link"] and len(names) == tgf.tgf_variant_count()


def test_su3_site_cap():
    """Sites per SU(3) configuration are capped at 2^28 - 256, so that every
    per-lane byte offset of the kernels (16-byte units) fits in 32 bits; the
    workspace size of a box at the cap is formed in 64 bits."""
    at_cap = tgf.make_geoms([(16, 16, 1024, 1023)])       # 268 173 312 sites
    over = tgf.make_geoms([(16, 16, 1024, 1024)])         # 2^28
    for st, per_site in ((tgf.TGF_F32_C12, 512), (tgf.TGF_F32_FULL, 704), (tgf.TGF_F64_FULL, 1408)):
        b = tgf.tgf_workspace_bytes(1, at_cap, st)
        assert b >= 16 * 16 * 1024 * 1023 * per_site > 1 << 32
        assert tgf.tgf_workspace_bytes(1, over, st) == 0
    ctx = ctypes.c_void_p()
    assert tgf.tgf_create(ctypes.byref(ctx), 1, over, tgf.TGF_F32_C12, ctypes.c_void_p(FAKE),
                          1 << 40, None) == tgf.TGF_E_INVAL
    assert b"too large" in tgf.tgf_last_error() and not ctx.value


def test_sun_workspace_and_create_validation():
    g = tgf.make_geoms([((4, 4, 16, 16), (3, 0, 0, 0, 0, 0))])
    F64 = tgf.TGF_F64_FULL
    V = 4 * 4 * 16 * 16
    b2 = tgf.tgf_workspace_bytes_sun(2, 1, tgf.make_geoms([(4, 4, 16, 16)]), F64)
    for nc in (4, 8):
        b = tgf.tgf_workspace_bytes_sun(nc, 1, tgf.make_geoms([(4, 4, 16, 16)]), F64)
        # two link buffers + X, each 4 nc^2 complex128 per site (shared regions cancel)
        assert b - b2 == pytest.approx(V * 3 * 4 * (nc * nc - 4) * 16, abs=4096)
    assert tgf.tgf_workspace_bytes_sun(4, 1, g, F64) > 0          # twist 3 < 4
    assert tgf.tgf_workspace_bytes_sun(3, 1, g, F64) == 0         # twist 3 >= 3
    assert tgf.tgf_workspace_bytes_sun(1, 1, g, F64) == 0
    assert tgf.tgf_workspace_bytes_sun(9, 1, g, F64) == 0
    assert tgf.tgf_workspace_bytes_sun(4, 1, g, tgf.TGF_F32_C12) == 0
    # sites per configuration capped at 2^28 / nc^2 - 256
    big = tgf.make_geoms([(64, 64, 64, 64)])
    assert tgf.tgf_workspace_bytes_sun(2, 1, big, F64) > 0
    assert tgf.tgf_workspace_bytes_sun(8, 1, big, F64) == 0
    ctx = ctypes.c_void_p()
    assert tgf.tgf_create_sun(ctypes.byref(ctx), 9, 1, g, F64, ctypes.c_void_p(FAKE), 1 << 40,
                              None) == tgf.TGF_E_INVAL
    assert tgf.tgf_create_sun(ctypes.byref(ctx), 4, 1, g, tgf.TGF_F32_FULL,
                              ctypes.c_void_p(FAKE), 1 << 40, None) == tgf.TGF_E_UNSUPPORTED
    assert tgf.tgf_create_sun(ctypes.byref(ctx), 4, 1, g, F64, ctypes.c_void_p(FAKE), 1024,
                              None) == tgf.TGF_E_SIZE
    assert not ctx.value
