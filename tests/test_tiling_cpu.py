"""Host-only check of the periodic wrap of the tile halos (no GPU): compiles
tests/cpp/tiling_check.cpp against the kernels' own tile-geometry header with
g++ and runs it.  For periodic sizes 1..400 in x (64-wide tiles) and in y (4, 8,
16 and 32-row tiles) every coordinate a tile touches must stay inside the
lattice on an interior tile, or wrap to its residue modulo the size."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_every_tile_halo_wraps_into_the_lattice(tmp_path):
    exe = str(tmp_path / "tiling_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe,
                    os.path.join(HERE, "cpp", "tiling_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
