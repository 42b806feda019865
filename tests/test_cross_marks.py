"""The cross-tile marks of the relaxation (bit-parallel on whole tile rows) against a
per-node enumeration of the diamond neighbours, on the host: random, sparse, single-node
and full change masks for every tile of ragged grids and all 8 neighbouring tiles
(tests/host/cross_marks_check.cpp, compiled here with g++)."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cross_marks_match_enumeration():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "cross_marks_check")
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-Wno-unknown-pragmas", "-o", exe,
                               os.path.join(ROOT, "tests", "host", "cross_marks_check.cpp")])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cross marks: ok" in r.stdout
