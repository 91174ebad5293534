"""GPU parity of the P2 path (stencils of the four unknown types, interface
rows from the faces' element partials, damped Jacobi, p-multigrid solve)
against the oracle, through the C ABI.

FP64, 1e-12 relative (max norm) for apply, residual and Jacobi; the solve
follows the oracle's residual history to 1e-10 with equal cycle counts.  At
sizes beyond the oracle's assembly (a face grid larger than the launch's
face blocks, and the benchmark's level-9 size) the operator is checked by
its exactness on quadratics: zero rows for harmonic quadratics, and for
x^2 + y^2 the rows -4 times the basis integrals (0 for vertex unknowns,
|T| / 3 per adjacent micro-triangle for edge unknowns), to a rounding bound
of 1e-12 absolute (row sums of |weights| times |u| of order 10, times 64
unit roundoffs)."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import log, rel_err, to_np

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
_CACHE = {}


def _ring_coef(F):
    c = np.ones(F)
    c[::3] = 7.0
    return c


def setup(name, l, coef=False):
    import paper_1805_10167_amd as P
    from oracle import p2
    from oracle.mesh import MacroMesh
    from oracle.mg import Hierarchy
    key = (name, l, coef)
    if key not in _CACHE:
        vxy, tri = hi.mesh_by_name(name)
        m = MacroMesh(vxy, tri)
        fc = _ring_coef(m.F) if coef else None
        S = p2.P2(Hierarchy(m, l, 2, face_coef=fc), face_coef=fc)
        g = P.Mesh(vxy, tri, l + 1, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_P2)
        if coef:
            P.hhg_set_face_coefficient(g.h, fc)
        P.hhg_p2_setup(g.h)
        _CACHE[key] = (g, S)
    return _CACHE[key]


CASES = [("square", 3), ("annulus64", 3), ("annulus64", 5), ("annulus128", 4)]


@pytest.mark.parametrize("name,l", CASES)
def test_apply_and_residual(name, l):
    import paper_1805_10167_amd as P
    log("P2 apply %s l=%d" % (name, l))
    g, S = setup(name, l)
    x = hi.uniform_vector(S.N, 31)
    f = hi.uniform_vector(S.N, 32)
    xd, fd = g.from_canonical(l + 1, x), g.from_canonical(l + 1, f)
    y = g.field(l + 1)
    P.hhg_p2_apply(g.h, l, xd, y)
    err = rel_err(to_np(g.to_canonical(l + 1, y)), S.apply(x))
    log("  apply rel err %.2e" % err)
    assert err <= F64_TOL
    # copies are consistent: the P1 restriction of y (which reads ghost rows) equals the oracle's
    P.hhg_p2_residual(g.h, l, xd, fd, y)
    r = S.residual(x, f)
    assert rel_err(to_np(g.to_canonical(l + 1, y)), r) <= F64_TOL
    fc = g.field(l)
    P.hhg_restrict(g.h, l + 1, P.HHG_F64, y, fc)
    assert rel_err(to_np(g.to_canonical(l, fc)), S.restrict(r)) <= F64_TOL


@pytest.mark.parametrize("name,l", CASES)
def test_jacobi(name, l):
    import paper_1805_10167_amd as P
    g, S = setup(name, l)
    x = hi.uniform_vector(S.N, 33)
    f = hi.uniform_vector(S.N, 34)
    y = g.field(l + 1)
    P.hhg_p2_jacobi(g.h, l, 0.7, g.from_canonical(l + 1, x), g.from_canonical(l + 1, f), y)
    S.omega = 0.7
    assert rel_err(to_np(g.to_canonical(l + 1, y)), S.jacobi(x, f, 1)) <= F64_TOL


def test_face_coefficient():
    import paper_1805_10167_amd as P
    l = 4
    g, S = setup("annulus64", l, coef=True)
    x = hi.uniform_vector(S.N, 35)
    y = g.field(l + 1)
    P.hhg_p2_apply(g.h, l, g.from_canonical(l + 1, x), y)
    assert rel_err(to_np(g.to_canonical(l + 1, y)), S.apply(x)) <= F64_TOL


@pytest.mark.parametrize("name,l", [("square", 4), ("annulus64", 4), ("annulus128", 4)])
def test_pmg_solve(name, l):
    import paper_1805_10167_amd as P
    log("P2 p-multigrid solve %s l=%d" % (name, l))
    g, S = setup(name, l)
    f = hi.uniform_vector(S.N, 36)
    f[S.lv.dirichlet] = 0.0
    S.omega = 0.7
    uo, ho = S.solve(np.zeros(S.N), f, rtol=1e-8, nu1=3, nu2=3, vnu=(2, 2))
    u = g.field(l + 1)
    rc, st, hist = P.hhg_p2_solve(g.h, l, u, g.from_canonical(l + 1, f), rtol=1e-8, nu1=3, nu2=3,
                                  vnu1=2, vnu2=2, omega=0.7)
    log("  cycles %d (oracle %d), history rel err %.2e" % (st["iters"], len(ho) - 1,
                                                           rel_err(hist, ho[:len(hist)])))
    assert rc == 0 and st["iters"] == len(ho) - 1
    assert rel_err(hist, ho) <= 1e-10
    assert rel_err(to_np(g.to_canonical(l + 1, u)), uo) <= 1e-10


def _quadratic_check(name, l, n_tan=None):
    """Rows of A2 applied to interpolated quadratics (see the module
    docstring); returns the worst absolute deviation."""
    import torch

    import paper_1805_10167_amd as P
    from oracle.mesh import Level, MacroMesh
    vxy, tri = hi.mesh_by_name(name) if n_tan is None else hi.annulus(n_tan=n_tan)
    m = MacroMesh(vxy, tri)
    g = P.Mesh(vxy, tri, l + 1, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_P2)
    P.hhg_p2_setup(g.h)
    lv = Level(m, l + 1)
    xy = torch.tensor(lv.xy, dtype=torch.float64, device="cuda")
    x, y = xy[:, 0], xy[:, 1]
    interior = torch.tensor(~lv.dirichlet, device="cuda")
    # load of a unit source at each unknown: 0 for vertex unknowns; for edge
    # unknowns |T| / 3 per adjacent micro-triangle of level l (all of a face's
    # micro-triangles have its area / 4^l)
    P2v = lv.xy[m.tri]
    farea = 0.5 * np.abs((P2v[:, 1, 0] - P2v[:, 0, 0]) * (P2v[:, 2, 1] - P2v[:, 0, 1])
                         - (P2v[:, 1, 1] - P2v[:, 0, 1]) * (P2v[:, 2, 0] - P2v[:, 0, 0]))
    tri_area = farea / 4.0 ** l
    load = np.zeros(lv.n_all)
    # face interiors: kind 2, face-local (i, j): an edge unknown unless both even
    fi = np.flatnonzero(lv.kind == 2)
    ev = (lv.kidx[fi] % 2 == 0) & (lv.jidx[fi] % 2 == 0)
    load[fi[~ev]] = 2.0 * tri_area[lv.prim[fi[~ev]]] / 3.0
    # macro-edge points: odd k are edge unknowns, one micro-triangle per adjacent face
    ei = np.flatnonzero(lv.kind == 1)
    odd = lv.kidx[ei] % 2 == 1
    for e in range(m.E):
        sel = ei[odd & (lv.prim[ei] == e)]
        load[sel] = sum(tri_area[f] for f in m.edge_faces[e]) / 3.0
    load = torch.tensor(load, dtype=torch.float64, device="cuda")
    worst = 0.0
    out = g.field(l + 1)
    for u, ref in ((x * y, 0.0 * x), (x * x - y * y, 0.0 * x), (x * x + y * y, -4.0 * load)):
        P.hhg_p2_apply(g.h, l, g.from_canonical(l + 1, u), out)
        got = g.to_canonical(l + 1, out)
        worst = max(worst, float(((got - ref).abs() * interior).max().item()))
        del got
    return worst, float(load.max().item())


def test_quadratics_with_more_tiles_than_face_blocks():
    """64-face annulus, P2 level 7 (fields of level 8: 10,560 face tiles
    against 8,192 face blocks)."""
    worst, lmax = _quadratic_check("annulus64", 7)
    log("P2 quadratic exactness annulus64 l=7: worst %.2e (largest load %.2e)" % (worst, lmax))
    assert worst <= 1e-12


def test_quadratics_at_benchmark_size():
    """The benchmark's P2 configuration: 64-face annulus, P2 level 9 (33.5M
    unknowns, the level-10 point layout)."""
    worst, lmax = _quadratic_check("annulus64", 9)
    log("P2 quadratic exactness annulus64 l=9: worst %.2e (largest load %.2e)" % (worst, lmax))
    assert worst <= 1e-12


def test_solve_converges_with_capped_face_grid():
    import paper_1805_10167_amd as P
    l = 7
    vxy, tri = hi.mesh_by_name("annulus64")
    g = P.Mesh(vxy, tri, l + 1, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_P2)
    P.hhg_p2_setup(g.h)
    _, n_all = g.n_dofs(l + 1)
    f = g.from_canonical(l + 1, hi.uniform_vector(n_all, 37))
    u = g.field(l + 1)
    rc, st, hist = P.hhg_p2_solve(g.h, l, u, f, rtol=1e-8, nu1=3, nu2=3, omega=0.7)
    rate = (hist[-1] / hist[0]) ** (1.0 / max(st["iters"], 1))
    log("P2 solve annulus64 l=%d: %d cycles, rate %.3f" % (l, st["iters"], rate))
    assert rc == 0 and rate < 0.35


def test_rejects_bad_calls():
    import paper_1805_10167_amd as P
    g, S = setup("annulus64", 3)
    x = g.field(4)
    with pytest.raises(P.HHGError):
        P.hhg_p2_apply(g.h, 4, x, g.field(4))            # level + 1 beyond max_level
    with pytest.raises(P.HHGError):
        P.hhg_p2_apply(g.h, 3, x, x)                     # aliasing
    with pytest.raises(P.HHGError):
        P.hhg_p2_jacobi(g.h, 3, -1.0, x, g.field(4), g.field(4))
    h2 = P.Mesh(*hi.mesh_by_name("square"), 3, 2, P.HHG_FEAT_F64)
    with pytest.raises(P.HHGError):
        P.hhg_p2_setup(h2.h)                             # workspace without HHG_FEAT_P2
