"""Pins of the oracle's refinement, numbering and geometry (CPU only)."""
import json
import os

import numpy as np
import pytest

import hhg_inputs as hi
from oracle.assemble import micro_triangles
from oracle.mesh import Level, MacroMesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_count_pin():
    """Sec. 5.2: 2145 unknowns per macro-face at refinement level 6."""
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    vxy, tri = hi.unit_square()
    lv = Level(MacroMesh(vxy, tri), g["level"])
    assert lv.points_per_face() == g["unknowns_per_face"]
    # the face-local map really holds that many distinct points per face
    for loc in lv.loc:
        assert len(np.unique(loc[loc >= 0])) == g["unknowns_per_face"]
    assert g["macro_faces"] * lv.points_per_face() >= g["total_at_least"]


@pytest.mark.parametrize("name,V,E,F,Eb", [("square", 4, 5, 2, 4),
                                           ("annulus64", 48, 112, 64, 32),
                                           ("annulus128", 96, 224, 128, 64)])
def test_macro_topology(name, V, E, F, Eb):
    m = MacroMesh(*hi.mesh_by_name(name))
    assert (m.V, m.E, m.F) == (V, E, F)
    assert m.edge_boundary.sum() == Eb
    # Euler characteristic: disc = 1, annulus = 0
    assert m.V - m.E + m.F == (1 if name == "square" else 0)


@pytest.mark.parametrize("name", ["square", "annulus64"])
@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_counts_and_coordinates(name, level):
    m = MacroMesh(*hi.mesh_by_name(name))
    lv = Level(m, level)
    n = lv.n
    # every canonical point is reached from some face map
    seen = np.zeros(lv.n_all, dtype=bool)
    for loc in lv.loc:
        seen[loc[loc >= 0]] = True
    assert seen.all()
    # coordinates of each face-local point agree with the affine face map
    for f, loc in enumerate(lv.loc):
        x0, x1, x2 = m.vxy[m.tri[f]]
        J, I = np.nonzero(loc >= 0)
        pts = x0 + np.outer(I / (n - 1), x1 - x0) + np.outer(J / (n - 1), x2 - x0)
        assert np.abs(lv.xy[loc[J, I]] - pts).max() < 1e-14
    # interior count: faces (n-2)(n-3)/2 + interior edges (n-2) + interior vertices
    Eint = (~m.edge_boundary).sum()
    Vint = (~m.vertex_boundary).sum()
    assert lv.interior_count() == m.F * (n - 2) * (n - 3) // 2 + Eint * (n - 2) + Vint


def test_orientation_and_micro_triangles():
    vxy, tri = hi.annulus(16)
    # input faces are clockwise by construction; the oracle reorients them
    x = vxy[tri]
    det_in = ((x[:, 1, 0] - x[:, 0, 0]) * (x[:, 2, 1] - x[:, 0, 1])
              - (x[:, 1, 1] - x[:, 0, 1]) * (x[:, 2, 0] - x[:, 0, 0]))
    assert (det_in < 0).all()
    m = MacroMesh(vxy, tri)
    lv = Level(m, 3)
    t = micro_triangles(lv)
    assert len(t) == m.F * (lv.n - 1) ** 2
    p = lv.xy[t]
    det = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
           - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    assert (det > 0).all()
    # the micro-triangles tile each macro-face exactly
    xm = m.vxy[m.tri]
    dm = ((xm[:, 1, 0] - xm[:, 0, 0]) * (xm[:, 2, 1] - xm[:, 0, 1])
          - (xm[:, 1, 1] - xm[:, 0, 1]) * (xm[:, 2, 0] - xm[:, 0, 0]))
    assert abs(det.sum() - dm.sum()) < 1e-12


def test_bad_meshes_rejected():
    with pytest.raises(ValueError):
        MacroMesh([[0, 0], [1, 0], [2, 0]], [[0, 1, 2]])
    # three faces on one edge
    vxy = [[0, 0], [1, 0], [0, 1], [0, -1], [1, 1]]
    with pytest.raises(ValueError):
        MacroMesh(vxy, [[0, 1, 2], [0, 1, 3], [0, 1, 4]])


def test_canonical_order():
    """Vertices, then edges sorted by (lo, hi) with k = 1..n-2 from lo to hi,
    then faces with interior points j-major."""
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, 3)
    n = lv.n
    assert (lv.kind[:m.V] == 0).all()
    for e, (a, b) in enumerate(m.edges):
        s = m.V + e * (n - 2)
        xa, xb = m.vxy[a], m.vxy[b]
        # k increases away from the lower vertex id
        d = np.linalg.norm(lv.xy[s:s + n - 2] - xa, axis=1)
        assert (np.diff(d) > 0).all()
        assert np.allclose(lv.xy[s], xa + (xb - xa) / (n - 1))
    f0 = lv.face_base
    assert (lv.jidx[f0:f0 + n - 3] == 1).all()
    assert (lv.kidx[f0:f0 + n - 3] == np.arange(1, n - 2)).all()
