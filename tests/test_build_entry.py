"""The build step must import without the compiled library: on a fresh
checkout libtgf.so does not exist until build() has made it."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_module_imports_without_loading_the_library():
    code = ("import sys\n"
            "from paper_2107_03747_amd import build\n"
            "import __graft_entry__\n"
            "assert callable(build.build) and callable(__graft_entry__.build)\n"
            "assert 'paper_2107_03747_amd.tgf' not in sys.modules, 'build imported the binding'\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
