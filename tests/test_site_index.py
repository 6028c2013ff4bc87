"""Host check of the device site numbering and tile choice (g++, no GPU)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

LATTICES = [
    (2, 2, 2, 2, 16384), (4, 4, 4, 4, 16384), (6, 2, 2, 2, 16384), (10, 6, 4, 6, 16384),
    (16, 16, 16, 32, 16384), (32, 32, 32, 64, 16384), (8, 8, 8, 8, 64),
    (12, 12, 12, 24, 16384), (20, 20, 20, 40, 16384), (24, 24, 24, 48, 16384),
    (16, 16, 16, 32, 512),
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("idx") / "site_index_check")
    src = os.path.join(HERE, "host", "site_index_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, src], check=True)
    return exe


@pytest.mark.parametrize("lat", LATTICES)
def test_site_numbering_is_a_bijection(checker, lat):
    r = subprocess.run([checker, *map(str, lat)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")


def test_production_tile_shape(checker):
    r = subprocess.run([checker, "32", "32", "32", "64", "16384"], capture_output=True,
                       text=True, timeout=300)
    # 2^15 sites per tile, split as evenly as the extents allow
    tiles = sorted(int(t) for t in r.stdout.split("tiles")[1].split())
    assert tiles == [8, 16, 16, 16]
