"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (plain C) and the library's host-side loader (mechanism parser and
the generated lane-per-cell source) are built with the sanitizers and run on
the configuration mechanisms and on malformed texts; any report fails the
test.  Device code is never instrumented: the host driver passes every
sanitizer flag through -Xarch_host.
"""
import os
import shutil
import subprocess

import pytest

from paper_2405_05974_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2405_05974_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _mech_files(tmp_path):
    out = []
    for cfg in (1, 4, 3):
        p = tmp_path / f"cfg{cfg}.mech"
        p.write_text(synth.config_mechanism(cfg).to_text())
        out.append(str(p))
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-ffp-contract=off",
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "sanitize", "oracle_driver.c"),
                    "-o", str(exe), "-lm"], check=True, capture_output=True)
    for mech in _mech_files(tmp_path)[:2]:
        r = subprocess.run([str(exe), mech], capture_output=True, text=True, env=ENV, timeout=600)
        assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-3000:]
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_host_loader_under_sanitizers(tmp_path):
    objs = [os.path.join(CSRC, f) for f in ("chem_jit.cpp.o", "chem_kernels.hip.o", "chem_server.cpp.o")]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built")
    exe = tmp_path / "host_san"
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                 "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", flag]
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *san,
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
                    os.path.join(HERE, "sanitize", "host_driver.cpp"), "-o", str(tmp_path / "host_driver.o")],
                   check=True, capture_output=True)
    subprocess.run(["hipcc", "--offload-arch=gfx950", *san, str(tmp_path / "host_driver.o"), *objs,
                    "-o", str(exe), "-lhiprtc"], check=True, capture_output=True)
    for mech in _mech_files(tmp_path):
        r = subprocess.run([str(exe), mech], capture_output=True, text=True, env=ENV, timeout=300)
        assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-3000:]
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
