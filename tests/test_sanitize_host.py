"""The library's host-side mesh setup (csrc/mesh.cpp: macro-primitive graph,
level layouts, ghost-copy table, coarse tables) built with AddressSanitizer
and UndefinedBehaviorSanitizer by the host compiler, and run on the seeded
meshes and on the inputs the setup must reject (CPU only, no device code).
Counts are compared with the oracle's numbering."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import hhg_inputs as hi
from oracle.mesh import Level, MacroMesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_10167_amd", "csrc")
GXX = shutil.which("g++")

pytestmark = pytest.mark.skipif(GXX is None or not os.path.isdir("/opt/rocm/include"),
                                reason="needs g++ and the ROCm headers")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / "mesh_driver")
    cmd = [GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
           os.path.join(ROOT, "tests", "sanitize", "mesh_driver.cpp"),
           os.path.join(CSRC, "mesh.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def run(driver, vxy, tri, L, lc):
    vxy, tri = np.asarray(vxy, float), np.asarray(tri, int)
    text = "%d %d %d %d\n" % (len(vxy), len(tri), L, lc)
    text += " ".join(repr(float(v)) for v in vxy.ravel()) + "\n"
    text += " ".join(str(int(t)) for t in tri.ravel()) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver], input=text, capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    return r.stdout.split("\n")


@pytest.mark.parametrize("name,L", [("square", 6), ("annulus64", 5), ("annulus128", 4)])
def test_setup_is_clean_and_counts_match(driver, name, L):
    vxy, tri = hi.mesh_by_name(name)
    out = run(driver, vxy, tri, L, 2)
    assert out[0] == "OK"
    m = MacroMesh(vxy, tri)
    for line in out[1:1 + L]:
        lvl, n_all, n_int, total, _ = map(int, line.split())
        lv = Level(m, lvl)
        assert (n_all, n_int) == (lv.n_all, lv.interior_count())
        assert total >= n_all


def test_fan_of_sixteen_edges_sets_up(driver):
    """A macro-vertex with 16 incident edges (the supported maximum)."""
    k = 16
    ang = 2 * np.pi * np.arange(k) / k
    vxy = np.vstack([[0.0, 0.0], np.c_[np.cos(ang), np.sin(ang)]])
    tri = [[0, 1 + i, 1 + (i + 1) % k] for i in range(k)]
    assert run(driver, vxy, tri, 3, 1)[0] == "OK"


@pytest.mark.parametrize("case", ["zero_area", "non_manifold", "bad_id", "level_high",
                                  "level_low", "coarse_above_fine", "degree17", "empty"])
def test_rejected_inputs_are_clean(driver, case):
    sq_v, sq_t = hi.unit_square()
    if case == "zero_area":
        args = ([[0, 0], [1, 0], [2, 0]], [[0, 1, 2]], 3, 2)
    elif case == "non_manifold":
        args = ([[0, 0], [1, 0], [0, 1], [0, -1], [1, 1]], [[0, 1, 2], [0, 3, 1], [0, 1, 4]], 3, 2)
    elif case == "bad_id":
        args = (sq_v, [[0, 1, 7], [0, 2, 3]], 3, 2)
    elif case == "level_high":
        args = (sq_v, sq_t, 13, 2)
    elif case == "level_low":
        args = (sq_v, sq_t, 0, 0)
    elif case == "coarse_above_fine":
        args = (sq_v, sq_t, 3, 4)
    elif case == "degree17":
        k = 17
        ang = 2 * np.pi * np.arange(k) / k
        args = (np.vstack([[0.0, 0.0], np.c_[np.cos(ang), np.sin(ang)]]),
                [[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], 3, 1)
    else:
        args = (np.zeros((0, 2)), np.zeros((0, 3), int), 3, 2)
    out = run(driver, *args)
    assert out[0].startswith("ERR "), out
