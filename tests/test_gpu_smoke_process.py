"""The entry point's smoke run in a fresh interpreter, where nothing imports torch before
the library is loaded (the order in which the library and torch could end up on
different HIP runtimes)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_smoke_in_fresh_process():
    code = "import __graft_entry__ as g; g.smoke()"
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    assert "smoke ok" in res.stdout
