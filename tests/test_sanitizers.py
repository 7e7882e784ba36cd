"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Three builds, each run by a driver in tests/sanitize/: the FP64 oracle (flows,
measurements, Monte Carlo, SU(N), samplers on ragged, multiply twisted
lattices), the ensemble statistics, and the runtime's host code (layout and
workspace sizing, contexts over an untouched workspace, work-group shapes,
variants and every check that returns before a device call; device launchers
replaced by stubs, device code of the allocation-free entry point compiled but
never run).  Any sanitizer report ends the driver with a nonzero status.
The runtime build uses hipcc with the sanitizers on the host side only.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2107_03747_amd", "csrc")
INC = os.path.join(ROOT, "include")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def check_clean(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "Sanitizer" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    run([gcc, "-std=c11", "-O1", "-g", *SAN_FLAGS, "-fopenmp",
         os.path.join(ROOT, "oracle", "tgf_oracle.c"), os.path.join(ROOT, "oracle", "sun_oracle.c"),
         os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe])
    assert "0 failed checks" in check_clean(exe)


def test_stats_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "stats_san")
    run([gxx, "-std=c++17", "-O1", "-g", *SAN_FLAGS, "-I", INC,
         os.path.join(CSRC, "stats.cpp"), os.path.join(SAN, "stats_driver.cpp"), "-o", exe])
    assert "0 failed checks" in check_clean(exe)


def test_runtime_host_code_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    host_san = []
    for f in SAN_FLAGS:
        host_san += ["-Xarch_host", f]
    common = ["-std=c++17", "-O1", "-g", *host_san, "-I", INC, "-I", CSRC,
              "-Wno-unused-command-line-argument"]
    objs = []
    for src in (os.path.join(CSRC, "runtime.hip"), os.path.join(SAN, "launch_stubs.cpp"),
                os.path.join(SAN, "runtime_driver.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        run([hipcc, "--offload-host-only", "-x", "hip", "-c", *common, src, "-o", o])
        objs.append(o)
    # the allocation-free entry point holds kernels: its device code is built too
    o = str(tmp_path / "noalloc.o")
    run([hipcc, "--offload-arch=gfx950", "-c", *common, "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", os.path.join(CSRC, "noalloc.hip"), "-o", o])
    objs.append(o)
    exe = str(tmp_path / "runtime_san")
    run([hipcc, "--offload-arch=gfx950", *host_san, *objs, "-o", exe])
    assert "0 failed checks" in check_clean(exe)


def test_stage_index_audit(tmp_path):
    """Every access of the stage launches replayed on the host with the
    kernels' own index functions (tests/sanitize/index_audit.cpp): the
    LDS-staged kernel on per-configuration blocks (whole planes and 256 sites)
    and the tile-based site kernels, both block orders, all three storages,
    on the 4x4x12x12 box, the benchmark's extents, ragged and degenerate
    batches, and the first and last work-groups of boxes up to the site cap
    (2^28 - 256); no access may leave its buffer, LDS block or wave, and no
    32-bit per-lane byte offset may wrap."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "index_audit")
    host_san = []
    for f in SAN_FLAGS:
        host_san += ["-Xarch_host", f]
    run([hipcc, "--offload-host-only", "-x", "hip", "-std=c++17", "-O1", "-g", *host_san,
         "-I", INC, "-I", CSRC, "-Wno-unused-command-line-argument",
         os.path.join(SAN, "index_audit.cpp"), "-o", exe])
    out = check_clean(exe)
    assert " 0 violations" in out, out
