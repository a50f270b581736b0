"""Host test of the paired search's work items (`csrc/rici_pairs.h`): item k
of a T x T tile grid must be the tile pair (I, J), I <= J, that the band order
puts k-th, for every item of every grid up to 300 tiles and of a few grids of
thousands of tiles (a set of 2^21 images has 8 192 tiles), and the items of a
grid must be exactly its pairs I <= J, each once.  The mapping is the closed
form of the kernel; the harness compares it with the order written out as
nested loops.  (A wrong mapping would skip or repeat tile pairs: ranks would
be off by whole tiles.)"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    out = tmp_path_factory.mktemp("pairs") / "pair_items"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2007_02306_amd", "csrc"),
                    os.path.join(HERE, "pair_items_harness.cpp"), "-o", str(out)], check=True)
    return str(out)


def test_every_item_of_small_grids(harness):
    r = subprocess.run([harness] + [str(t) for t in range(1, 301)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr + r.stdout


def test_large_grids(harness):
    r = subprocess.run([harness, "4095", "4096", "4099", "8191"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr + r.stdout


@pytest.mark.parametrize("T", [1, 7, 8, 9, 92, 257])
def test_items_are_the_pairs_once(harness, T):
    r = subprocess.run([harness, "-p", str(T)], capture_output=True, text=True, check=True)
    items = [tuple(map(int, line.split())) for line in r.stdout.split("\n") if line]
    assert len(items) == T * (T + 1) // 2
    assert sorted(items) == [(i, j) for i in range(T) for j in range(i, T)]
