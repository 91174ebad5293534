"""Pins of the oracle's P2 elements and p-multigrid (CPU only).

  * the element basis: rows of the element stiffness sum to zero, it is
    symmetric, and a vertex does not couple with the midpoint of the
    opposite edge (the integral of (4 lam_a - 1) lam_c vanishes);
  * exactness on quadratics: the P2 interpolant of a harmonic quadratic has
    A u = 0 on interior rows, and for u = x^2 + y^2 (-Lap u = -4) the rows are
    -4 times the integral of the basis function, which is 0 for vertex
    functions and |T| / 3 per element for edge functions (closed forms of
    the integrals of barycentric monomials);
  * the Galerkin identity P^T A2 P = A1 with the independently assembled P1
    stiffness (also with a coefficient per macro-face);
  * the embedding reproduces linear functions exactly;
  * the p-multigrid solve reaches the direct solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import hhg_inputs as hi
from oracle import p2
from oracle.mesh import MacroMesh
from oracle.mg import Hierarchy

_CACHE = {}


def system(name, l, coef=None):
    key = (name, l, coef is None)
    if key not in _CACHE:
        m = MacroMesh(*hi.mesh_by_name(name))
        fc = None if coef is None else coef(m)
        H = Hierarchy(m, l, 2, face_coef=fc)
        _CACHE[key] = p2.P2(H, face_coef=fc)
    return _CACHE[key]


def _ring_coef(m):
    c = np.ones(m.F)
    c[::3] = 7.0
    return c


def test_element_matrix_properties():
    rng = np.random.default_rng(0)
    for _ in range(20):
        P = rng.uniform(-1, 1, (3, 2))
        K = p2.element_stiffness(P)
        assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
        assert np.abs(K.sum(axis=1)).max() <= 1e-12 * np.abs(K).max()
        # vertex a and the midpoint of the opposite edge: (0, m12), (1, m02), (2, m01)
        for a, m in ((0, 4), (1, 5), (2, 3)):
            assert abs(K[a, m]) <= 1e-13 * np.abs(K).max()
        # positive semidefinite with the constants as the only null space
        w = np.linalg.eigvalsh(K)
        assert w[0] > -1e-12 and w[1] > 1e-8


@pytest.mark.parametrize("name,l", [("square", 3), ("annulus64", 3)])
def test_quadratics_are_reproduced(name, l):
    S = system(name, l)
    x, y = S.lv.xy[:, 0], S.lv.xy[:, 1]
    ii = S.lv.interior
    for u in (x * y, x * x - y * y, 3 * x * y - 2 * x + y):
        assert np.abs((S.A @ u)[ii]).max() <= 1e-11
    # -Lap(x^2 + y^2) = -4: load of a constant
    u = x * x + y * y
    load = np.zeros(S.N)
    nodes = S.nodes
    e1 = S.lv.xy[nodes[:, 1]] - S.lv.xy[nodes[:, 0]]
    e2 = S.lv.xy[nodes[:, 2]] - S.lv.xy[nodes[:, 0]]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    for k in range(3):
        np.add.at(load, nodes[:, 3 + k], area / 3.0)
    got = S.A @ u
    assert np.abs(got[ii] + 4.0 * load[ii]).max() <= 1e-11
    # vertex rows see no load at all
    vert = np.zeros(S.N, dtype=bool)
    vert[nodes[:, :3].ravel()] = True
    iv = np.intersect1d(ii, np.flatnonzero(vert))
    assert len(iv) > 0 and np.abs(got[iv]).max() <= 1e-11


@pytest.mark.parametrize("name,l,coef", [("square", 3, None), ("annulus64", 3, None),
                                         ("annulus64", 3, _ring_coef)])
def test_galerkin_identity(name, l, coef):
    S = system(name, l, coef)
    A1 = S.H.A[l]
    G = (S.P.T @ S.A @ S.P).toarray()
    assert np.abs(G - A1.toarray()).max() <= 1e-12 * abs(A1).max()


def test_embedding_reproduces_linear_functions():
    S = system("annulus64", 3)
    xc, yc = S.lc.xy[:, 0], S.lc.xy[:, 1]
    xf, yf = S.lv.xy[:, 0], S.lv.xy[:, 1]
    for a, b, c in ((1.0, 0.0, 0.0), (0.3, -2.0, 0.7), (0.0, 1.5, -4.0)):
        assert np.abs(S.P @ (a + b * xc + c * yc) - (a + b * xf + c * yf)).max() <= 1e-14
    # every row sums to one
    assert np.abs(np.asarray(S.P.sum(axis=1)).ravel() - 1.0).max() == 0.0


@pytest.mark.parametrize("name,l", [("square", 4), ("annulus64", 4)])
def test_pmg_solve_reaches_direct_solution(name, l):
    S = system(name, l)
    f = hi.uniform_vector(S.N, 5)
    f[S.lv.dirichlet] = 0.0
    u, hist = S.solve(np.zeros(S.N), f, rtol=1e-10, nu1=3, nu2=3)
    assert hist[-1] <= 1e-10 * hist[0]
    rate = (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1))
    assert rate < 0.5
    ii = S.lv.interior
    ref = spla.spsolve(S.A[ii][:, ii].tocsc(), f[ii])
    assert np.abs(u[ii] - ref).max() <= 1e-8 * np.abs(ref).max()
