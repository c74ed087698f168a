"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
gcc/g++): the FP64 oracle driven through every rule, averaging lattice and
border kind (tests/cpp/oracle_driver.c), and the host checks of the tile
geometry and the graph replay plan, which compile the library's own
HIP-free headers."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe):
    subprocess.run(cmd, check=True)
    # verify_asan_link_order=0: the environment may preload a library ahead
    # of the ASan runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c99", "-Wall", *SAN, "-o", exe, os.path.join(HERE, "cpp", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"], exe)


@pytest.mark.parametrize("name", ["tiling_check", "plan_check"])
def test_host_checks_under_sanitizers(tmp_path, name):
    exe = str(tmp_path / name)
    _run(["g++", "-std=c++17", "-Wall", *SAN, "-o", exe, os.path.join(HERE, "cpp", name + ".cpp")], exe)
