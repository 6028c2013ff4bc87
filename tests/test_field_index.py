"""Host check of the device field, link and clover-table index maps (g++, no GPU)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("fidx") / "field_index_check")
    src = os.path.join(HERE, "host", "field_index_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, src], check=True)
    return exe


@pytest.mark.parametrize("nblk", [1, 3, 17])
def test_index_maps_are_bijections_and_agree(checker, nblk):
    r = subprocess.run([checker, str(nblk)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
