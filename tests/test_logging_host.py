"""FFTRW_LOG diagnostics of the host functions: silent by default; level 1
reports errors, level 2 also order searches."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPT = """
from paper_1302_6189_amd import fftrw
fftrw.fft_order_search((8, 8, 8), 4)
try:
    fftrw.fft_decomp((4, 4, 4), 0, "abc", 0)
except fftrw.FftrwError:
    pass
"""


def _stderr(level):
    env = dict(os.environ)
    env.pop("FFTRW_LOG", None)
    if level is not None:
        env["FFTRW_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return [l for l in r.stderr.splitlines() if l.startswith("fftrw: ")]


def test_silent_by_default():
    assert _stderr(None) == [] and _stderr(0) == []


def test_levels():
    one = _stderr(1)
    assert one == ["fftrw: error -1: P must be >= 1"]
    two = _stderr(2)
    assert two[0] == "fftrw: order search M=3 P=4 ownership=0: least 384 (4 orders), largest 768 (4 orders)"
    assert two[1:] == one
