"""The algorithmic work model behind the bench's roofline line (CPU only).

Bytes: every link and accumulator element an RK stage touches, once, with
ping-pong link buffers -- per site and RK3 step FP64 full 4 480 B, FP32 full
2 240 B, FP32 12-real 1 664 B.  Flops: the site formulation, about 3.7e4 per
site-step for 12-real storage.  Monte Carlo: 1 296 B and 3 402 flop per link
update.  SU(N): 640 N^2 B per site-step.
"""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bytes_per_site_step():
    # links: read + write 4 links of NE complex entries in each of 3 stages;
    # X: 4 links x 4 complex slots, written / read+written / read over the stages
    for storage, ne, cb in (("f64", 9, 16), ("f32", 9, 8), ("f32c12", 6, 8)):
        links = 3 * 2 * 4 * ne * cb
        x = (1 + 2 + 1) * 4 * 4 * cb
        assert bench.bytes_per_site_step(storage) == links + x
    assert bench.bytes_per_site_step("f64") == 4480
    assert bench.bytes_per_site_step("f32") == 2240
    assert bench.bytes_per_site_step("f32c12") == 1664
    # the LDS and plaquette-sharing variants move the same algorithmic bytes
    for v in ("site_alg_xcd", "site_lds", "site_lds_xcd", "site_plq_xcd"):
        assert bench.bytes_per_site_step("f32c12", v) == 1664


def test_flops_per_site_step():
    f = bench.flops_per_site_step("f32c12", "site_lds_xcd")
    assert f == 3 * 12404
    assert 3.5e4 < f < 3.9e4
    # one count for the site formulation, whatever the kernel variant
    for v in ("site_alg", "site_alg_xcd", "site_lds", "site_plq_xcd"):
        assert bench.flops_per_site_step("f32c12", v) == f
    # 12-real storage pays its third-row rebuilds on top of the FP32 full count
    assert bench.flops_per_site_step("f32", "site_lds_xcd") < f


def test_mc_and_sun_models():
    # a launch reads all 4V links (144 B each) and writes the V/2 updated ones
    assert bench.MC_BYTES_PER_LINK == pytest.approx((4 * 144 + 0.5 * 144) / 0.5)
    assert bench.MC_FLOPS_PER_LINK == 3402
    for n in (2, 3, 4, 8):
        assert bench.sun_bytes_per_site_step(n) == 640 * n * n


def test_kernel_source_hash_ignores_comments_only(tmp_path):
    """The hash that ties a profile to the kernel code: unchanged by comment
    and blank-line edits, changed by any edit of the code."""
    import shutil
    src = os.path.join(ROOT, "paper_2107_03747_amd", "csrc")
    dst = tmp_path / "paper_2107_03747_amd" / "csrc"
    shutil.copytree(src, dst)
    h0 = bench.kernel_source_hash(str(tmp_path))
    assert h0 == bench.kernel_source_hash()
    k = dst / "kernels.hip"
    text = k.read_text()
    k.write_text("// a new comment line\n\n" + text.replace("namespace tgf {", "namespace tgf {  /* x */", 1))
    assert bench.kernel_source_hash(str(tmp_path)) == h0
    k.write_text(text.replace("kRkA[3] = {0.0,", "kRkA[3] = {0.0 ,", 1))
    assert bench.kernel_source_hash(str(tmp_path)) != h0
