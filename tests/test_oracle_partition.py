"""The oracle's virtual partition (one block per macro-primitive with explicit
ghost copies, refreshed in the four directions of the paper's Alg. 3)
against its global-vector mode (CPU only).

After the packer runs, every ghost slot must hold its owner's value exactly
(the slot's identity comes from the numbering, the value from the packer,
which works by position and orientation alone).  The blockwise apply, each
row evaluated inside its block from local values only and summed in the CSR
row's order, must then equal the global A u to 1e-15 (bitwise in practice).
A mesh whose faces are given in mixed clockwise/counter-clockwise order with
rotated starting vertices puts every side of a face, in both directions, on
some edge.  A packer with the direction flag ignored (a mistake planted in
the oracle) must fail the ghost check."""
import numpy as np
import pytest

import hhg_inputs as hi
from oracle import partition as PT
from oracle.assemble import assemble
from oracle.mesh import Level, MacroMesh


def mixed_orientation_annulus():
    vxy, tri = hi.mesh_by_name("annulus64")
    tri = np.array(tri)
    for f in range(len(tri)):
        a, b, c = tri[f]
        if f % 2:
            a, b, c = a, c, b          # clockwise input
        if f % 3 == 1:
            a, b, c = b, c, a          # another starting vertex
        elif f % 3 == 2:
            a, b, c = c, a, b
        tri[f] = (a, b, c)
    return vxy, tri


MESHES = {
    "annulus64": lambda: hi.mesh_by_name("annulus64"),
    "square": lambda: hi.mesh_by_name("square"),
    "mixed": mixed_orientation_annulus,
}


def ghost_mismatch(P, u):
    """Largest |ghost - owner| over every local slot of every block."""
    ids = P.slot_ids()
    worst = 0.0
    m = P.lv.mesh
    for kind, count in (("vert", m.V), ("edge", m.E), ("face", m.F)):
        for p in range(count):
            sid = ids[kind][p]
            loc = P.flat_local(kind, p)
            ok = sid >= 0
            worst = max(worst, float(np.abs(loc[ok] - u[sid[ok]]).max(initial=0.0)))
    return worst


@pytest.mark.parametrize("name,level", [("annulus64", 3), ("annulus64", 4), ("square", 4),
                                        ("mixed", 3), ("mixed", 4)])
def test_ghosts_hold_their_owners_values(name, level):
    lv = Level(MacroMesh(*MESHES[name]()), level)
    u = hi.uniform_vector(lv.n_all, 7)
    P = PT.Partition(lv)
    P.scatter(u)
    P.sync()
    assert ghost_mismatch(P, u) == 0.0


@pytest.mark.parametrize("name,level", [("annulus64", 3), ("square", 4), ("mixed", 4)])
def test_blockwise_apply_equals_global_apply(name, level):
    lv = Level(MacroMesh(*MESHES[name]()), level)
    A = assemble(lv, want=("A",))["A"]
    P = PT.Partition(lv)
    for seed in (1, 2):
        u = hi.uniform_vector(lv.n_all, seed)
        P.scatter(u)
        P.sync()
        y = P.apply(A)
        ref = A @ u
        assert np.abs(y - ref).max() <= 1e-15 * np.abs(ref).max()


def test_repeated_sweeps_through_the_packer():
    """Three damped Jacobi steps, each applying the operator blockwise after
    a fresh ghost exchange, follow the global iteration."""
    lv = Level(MacroMesh(*mixed_orientation_annulus()), 3)
    A = assemble(lv, want=("A",))["A"]
    d = A.diagonal()
    f = hi.uniform_vector(lv.n_all, 3)
    ug = np.zeros(lv.n_all)
    ub = np.zeros(lv.n_all)
    P = PT.Partition(lv)
    for _ in range(3):
        ug = ug + (2.0 / 3.0) * (f - A @ ug) / d
        P.scatter(ub)
        P.sync()
        ub = ub + (2.0 / 3.0) * (f - P.apply(A)) / d
    assert np.abs(ub - ug).max() <= 1e-14 * np.abs(ug).max()


def test_packer_without_orientation_fails():
    """Planted mistake: every face side taken as running along its edge."""
    lv = Level(MacroMesh(*mixed_orientation_annulus()), 3)
    u = hi.uniform_vector(lv.n_all, 7)
    P = PT.Partition(lv)
    P.face_sides = [[(e, True) for e, _ in sides] for sides in P.face_sides]
    P.edge_adj = [[(f, s, True) for f, s, _ in adj] for adj in P.edge_adj]
    P.scatter(u)
    P.sync()
    assert ghost_mismatch(P, u) > 0.1


def test_incomplete_ghost_layer_is_detected():
    """A stencil neighbour outside a block's slots is an error, not a zero."""
    lv = Level(MacroMesh(*hi.mesh_by_name("square")), 3)
    A = assemble(lv, want=("A",))["A"].tolil()
    A[lv.face_base, 3] = 1.0          # a row of face 0 reaching vertex 3, not on face 0
    P = PT.Partition(lv)
    P.scatter(np.ones(lv.n_all))
    P.sync()
    with pytest.raises(KeyError):
        P.apply(A.tocsr())
