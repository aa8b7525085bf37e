"""The serving queue protocol on the CPU: the server's producer half
(csrc/chem_serve_ring.h, the code the server runs) against threads that
follow the resident kernels' half, with a small ring, a small tile table and
a low tile limit so that full rings, reused table entries, rebases, idle and
quantum exits and relaunches all happen (tests/serve_ring_sim.cpp).  Every
cell of every box must be processed exactly once and every box complete once."""
import pathlib
import shutil
import subprocess

import pytest

HERE = pathlib.Path(__file__).resolve().parent


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("serve_ring") / "serve_ring_sim"
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-Wall", "-Werror", "-o", str(exe),
                    str(HERE / "serve_ring_sim.cpp")], check=True)
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_serve_queue_protocol(sim, seed):
    r = subprocess.run([str(sim), str(seed), "400"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    words = r.stdout.split()
    stats = dict(zip(words[0::2], (int(w) for w in words[1::2])))
    assert stats["errors"] == 0 and stats["boxes"] == 400
    assert stats["rebases"] >= 1 and stats["launches"] >= 2   # the paths meant to run did run
