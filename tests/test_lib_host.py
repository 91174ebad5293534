"""Host-side checks of the C-ABI library that need no GPU: the shared
library loads, exports every symbol include/hhg.h declares, and its mesh setup
(host code only) agrees with the oracle's numbering and geometry."""
import os
import re

import numpy as np
import pytest

import hhg_inputs as hi
from oracle.mesh import Level, MacroMesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
P = pytest.importorskip("paper_1805_10167_amd")


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "hhg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hhg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("name", ["square", "annulus64", "annulus128"])
@pytest.mark.parametrize("level", [1, 2, 3, 5])
def test_counts_and_coordinates_match_oracle(name, level):
    vxy, tri = hi.mesh_by_name(name)
    h = P.hhg_setup_mesh(vxy, tri, max(level, 2), 1)
    try:
        lv = Level(MacroMesh(vxy, tri), level)
        ni, na = P.hhg_n_dofs(h, level)
        assert (ni, na) == (lv.interior_count(), lv.n_all)
        xy = P.hhg_coords(h, level)
        assert np.abs(xy - lv.xy).max() <= 1e-15
        assert P.hhg_field_elems(h, level) >= na
    finally:
        P.hhg_destroy_mesh(h)


@pytest.mark.parametrize("name,level", [("square", 3), ("annulus64", 4), ("annulus128", 2)])
def test_cell_centroids_match_oracle(name, level):
    """The library's canonical cell order and geometry (micro-triangle
    centroids) against the oracle's cell list."""
    from oracle import transport as tr
    vxy, tri = hi.mesh_by_name(name)
    h = P.hhg_setup_mesh(vxy, tri, max(level, 2), 1)
    try:
        c = tr.Cells(Level(MacroMesh(vxy, tri), level))
        xy = P.hhg_cell_coords(h, level, len(tri))
        assert xy.shape == c.centroid.shape
        assert np.abs(xy - c.centroid).max() <= 1e-15
    finally:
        P.hhg_destroy_mesh(h)


@pytest.mark.parametrize("name,level", [("square", 3), ("annulus64", 4), ("annulus128", 2)])
def test_ghost_table(name, level):
    """One entry per copy slot: face rings (3 corners and 3 (n-2) side
    points per face), edge end slots (2 per edge), ghost rows (n-1 per face
    of an interior edge), vertex ring slots (one per incident edge); every
    destination distinct and never an owned slot (owners are sources)."""
    vxy, tri = hi.mesh_by_name(name)
    m = MacroMesh(vxy, tri)
    h = P.hhg_setup_mesh(vxy, tri, max(level, 2), 1)
    try:
        dst, src = P.hhg_ghost_table(h, level)
        n = 2 ** level + 1
        interior_edges = [fs for e, fs in enumerate(m.edge_faces) if not m.edge_boundary[e]]
        degree = np.zeros(m.V, dtype=int)
        for a, b in m.edges:
            degree[a] += 1
            degree[b] += 1
        expect = m.F * (3 + 3 * (n - 2)) + 2 * m.E + sum(len(fs) for fs in interior_edges) * (n - 1) + degree.sum()
        assert len(dst) == expect
        assert len(np.unique(dst)) == len(dst)
        assert not np.isin(src, dst).any()
    finally:
        P.hhg_destroy_mesh(h)


def test_paper_count_at_level6():
    """2145 points per face at level 6 (sec. 5.2): n_all of one face."""
    vxy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    h = P.hhg_setup_mesh(vxy, [[0, 1, 2]], 6, 2)
    try:
        assert P.hhg_n_dofs(h, 6)[1] == 2145
    finally:
        P.hhg_destroy_mesh(h)


def test_setup_errors():
    with pytest.raises(P.HHGError) as e:
        P.hhg_setup_mesh([[0, 0], [1, 0], [2, 0]], [[0, 1, 2]], 3, 2)
    assert e.value.code == P.HHG_EINVAL
    vxy = [[0, 0], [1, 0], [0, 1], [0, -1], [1, 1]]
    with pytest.raises(P.HHGError):
        P.hhg_setup_mesh(vxy, [[0, 1, 2], [0, 1, 3], [0, 1, 4]], 3, 2)
    with pytest.raises(P.HHGError):
        P.hhg_setup_mesh(*hi.unit_square(), 13, 2)
    with pytest.raises(P.HHGError):
        P.hhg_setup_mesh(*hi.unit_square(), 4, 5)
    with pytest.raises(P.HHGError):
        P.hhg_setup_mesh([[0, 0], [1, 0], [0, 1]], [[0, 1, 7]], 3, 2)
    assert "out of range" in P.hhg_last_error()


def test_unbound_mesh_rejects_compute_calls():
    h = P.hhg_setup_mesh(*hi.unit_square(), 3, 2)
    try:
        assert P.hhg_workspace_bytes(h, P.HHG_FEAT_F64) > 0
        rc = P.lib().hhg_apply(h, 3, 0, 0, None, None, None)
        assert rc == P.HHG_ENOMEM
        with pytest.raises(P.HHGError):
            P.hhg_workspace_bytes(h, 1 << 7)
    finally:
        P.hhg_destroy_mesh(h)


def _fan(m):
    """m triangles around the origin (all sharing vertex 0), counter-clockwise."""
    import math
    vxy = [[0.0, 0.0]] + [[math.cos(2 * math.pi * k / m), math.sin(2 * math.pi * k / m)] for k in range(m)]
    tri = [[0, 1 + k, 1 + (k + 1) % m] for k in range(m)]
    return vxy, tri


def test_vertex_degree_limit():
    """A macro-vertex may have up to 16 macro-edges: a 16-triangle fan sets
    up, a 17-triangle fan is rejected with a clear message."""
    h = P.hhg_setup_mesh(*_fan(16), 3, 2)
    P.hhg_destroy_mesh(h)
    with pytest.raises(P.HHGError) as e:
        P.hhg_setup_mesh(*_fan(17), 3, 2)
    assert e.value.code == P.HHG_EINVAL
    assert "more than 16" in P.hhg_last_error()
