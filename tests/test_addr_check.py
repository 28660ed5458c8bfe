"""The host-side address checker (tests/addrcheck/addr_check.cpp): every
global and LDS access of the screen, its operand preparation, the listed-
point rescan and the Lloyd update stays inside its buffer at the benchmark
shapes, every k-step count of the screen and the shapes of the screen
variants that were taken out after memory faults.  Run on the CPU: it replays
the kernels' index arithmetic with the library's own geometry header."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "addrcheck", "addr_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("addrcheck") / "addr_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe, SRC], check=True)
    return exe


def test_every_access_in_bounds(checker):
    r = subprocess.run([checker], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:]
    assert r.stdout.strip().endswith("0 violations")
    # the benchmark shapes and the removed variants' shapes were all covered
    for shape in ("C1 4.8M x 42", "C2 16M x 128", "C3 50M x 256", "removed FP8-vs-centers",
                  "removed norm-pruned", "removed batched", "Lloyd C3 50M x 256"):
        assert shape in r.stdout


def test_checker_catches_the_unwritten_sorted_positions(checker):
    # Before points without a valid center got a key of their own, the last
    # cluster's chunk ran to n and its sums read sorted positions the scatter
    # never wrote (then gathered X rows at whatever index they held).
    r = subprocess.run([checker, "--legacy-chunk-end"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 1
    assert "read before any scatter wrote them" in r.stdout
