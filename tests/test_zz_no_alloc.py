"""The allocation-free measurement (tgf_measure_noalloc) against tgf_measure on
a TGF_F64_FULL context holding the same links, through the C ABI: two calls
in a row on one stream, the second on a smaller lattice (the fixed scratch
array keeps the first call's partials, which must not leak into the second).
The two paths share the measurement arithmetic, the partial layout and the
reduction order, so they agree to the FP64 bar (1e-12 relative, Q 1e-10
absolute) and in practice bit for bit."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2107_03747_amd import gen, tgf          # noqa: E402

COLS = {n: k for k, n in enumerate(tgf.OBS_FIELDS)}


def noalloc(dims, twist, U, t, stream):
    g = tgf.make_geoms([(dims, twist)])
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    stream.wait_stream(torch.cuda.current_stream())
    tgf.check(tgf.tgf_measure_noalloc(g, ctypes.c_void_p(U.data_ptr()), float(t),
                                      ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(stream.cuda_stream)))
    stream.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_context_measure():
    cases = [((8, 8, 24, 24), tgf.PAPER_TWIST, 0.3, "near"),
             ((3, 5, 4, 7), (1, 0, 2, 1, 0, 2), 0.05, "haar")]
    s = torch.cuda.Stream()
    for k, (dims, twist, t, kind) in enumerate(cases):
        print(f"  case {dims} twist {twist} t {t}", flush=True)
        if kind == "near":
            U = gen.near_identity(dims, 0.3, seed=90 + k, device="cuda")
        else:
            U = gen.haar(dims, seed=90 + k, device="cuda")
        f = tgf.Flow([(dims, twist)], "f64")
        f.load(0, U, t0=t)
        ref = f.measure()[0]
        got = noalloc(dims, twist, U, t, s)
        print(f"    context {ref}\n    noalloc {got}  bitwise {np.array_equal(got, ref)}",
              flush=True)
        for name in ("t", "E", "t2E", "plaq", "action"):
            a, b = got[COLS[name]], ref[COLS[name]]
            assert abs(a - b) <= 1e-12 * max(abs(b), 1e-300), (name, a, b)
        assert abs(got[COLS["Q"]] - ref[COLS["Q"]]) <= 1e-10


def test_noalloc_rejects_on_the_host():
    s = torch.cuda.Stream()
    out = torch.zeros(6, dtype=torch.float64, device="cuda")
    U = gen.identity((4, 4, 4, 4), device="cuda")
    P = ctypes.c_void_p
    big = tgf.make_geoms([(4096, 4096, 2, 2)])       # 2^26 sites > TGF_NOALLOC_MAX_SITES
    assert tgf.tgf_measure_noalloc(big, P(U.data_ptr()), 0.0, P(out.data_ptr()),
                                   P(s.cuda_stream)) == tgf.TGF_E_SIZE
    bad = tgf.make_geoms([((4, 4, 4, 4), (3, 0, 0, 0, 0, 0))])
    assert tgf.tgf_measure_noalloc(bad, P(U.data_ptr()), 0.0, P(out.data_ptr()),
                                   P(s.cuda_stream)) == tgf.TGF_E_INVAL
    g = tgf.make_geoms([((4, 4, 4, 4), (0, 0, 0, 0, 0, 0))])
    assert tgf.tgf_measure_noalloc(g, None, 0.0, P(out.data_ptr()),
                                   P(s.cuda_stream)) == tgf.TGF_E_INVAL
    assert tgf.tgf_measure_noalloc(g, P(U.data_ptr()), -1.0, P(out.data_ptr()),
                                   P(s.cuda_stream)) == tgf.TGF_E_INVAL
    # unit links of the untwisted box: E = 0, plaquette 1
    tgf.check(tgf.tgf_measure_noalloc(g, P(U.data_ptr()), 0.0, P(out.data_ptr()),
                                      P(s.cuda_stream)))
    s.synchronize()
    got = out.cpu().numpy()
    assert got[COLS["E"]] == 0.0 and got[COLS["plaq"]] == 1.0
