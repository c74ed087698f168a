"""Host-only checks (no GPU).  The periodic wrap of the tile halos: compiles
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


def test_graph_replay_plan_keeps_the_diagnostics_cadence(tmp_path):
    """The step loops' graph replay plan (lbm_plan.hpp): refused exactly for
    graph lengths and diagnostic cadences that do not divide one another;
    otherwise every step runs once, replays start at multiples of the graph
    length, and the diagnostics run at (t + 1) % diag_every == 0 whatever the
    sequence of step calls."""
    exe = str(tmp_path / "plan_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe,
                    os.path.join(HERE, "cpp", "plan_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")
