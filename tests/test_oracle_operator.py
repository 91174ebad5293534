"""Pins of the oracle's assembled operators (CPU only).

Each pin comes from outside the oracle: a textbook matrix, a closed-form
eigenpair, the cotangent formula computed from angles, or an invariant."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import hhg_inputs as hi
from oracle.assemble import assemble
from oracle.mesh import Level, MacroMesh


def _square_grid_perm(lv):
    """Map interior canonical points of the unit square to a (n-2)^2 grid."""
    n = lv.n
    h = 1.0 / (n - 1)
    ii = lv.interior
    gx = np.rint(lv.xy[ii, 0] / h).astype(int) - 1
    gy = np.rint(lv.xy[ii, 1] / h).astype(int) - 1
    return ii, gy * (n - 2) + gx


@pytest.mark.parametrize("level", [2, 3, 4])
def test_unit_square_is_five_point_laplacian(level):
    """On the two right-angled faces the P1 stiffness matrix restricted to
    interior points is kron(I, T) + kron(T, I), T = tridiag(-1, 2, -1)."""
    lv = Level(MacroMesh(*hi.unit_square()), level)
    A = assemble(lv)["A"]
    ii, g = _square_grid_perm(lv)
    m = lv.n - 2
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    ref = (sp.kron(sp.eye(m), T) + sp.kron(T, sp.eye(m))).toarray()
    Aii = A[ii][:, ii].toarray()
    P = np.zeros((len(ii), len(ii)))
    P[np.arange(len(ii)), g] = 1.0
    assert np.abs(P.T @ Aii @ P - ref).max() < 1e-13


def test_unit_square_closed_form_eigenpair():
    """s(x,y) = sin(pi x) sin(pi y) on the grid is an eigenvector of the
    5-point operator: A s = 8 sin^2(pi h / 2) s at interior rows."""
    lv = Level(MacroMesh(*hi.unit_square()), 6)
    A = assemble(lv)["A"]
    s = hi.manufactured_u(lv.xy)
    h = 1.0 / (lv.n - 1)
    lam = 8.0 * math.sin(math.pi * h / 2) ** 2
    y = A @ s
    ii = lv.interior
    assert np.abs(y[ii] - lam * s[ii]).max() < 1e-13


def _angles(x):
    out = []
    for k in range(3):
        a = x[(k + 1) % 3] - x[k]
        b = x[(k + 2) % 3] - x[k]
        out.append(math.acos(a @ b / (np.linalg.norm(a) * np.linalg.norm(b))))
    return out


@pytest.mark.parametrize("level", [2, 3, 4])
def test_face_rows_equal_cotangent_stencil(level):
    """Face-interior rows carry the cotangent 7-point stencil: E/W -cot(t2),
    N/S -cot(t1), SE/NW -cot(t0), centre 2 sum cot (angles from arccos)."""
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, level)
    A = assemble(lv)["A"].tocsr()
    n = lv.n
    for f in range(0, m.F, 7):
        c = [1.0 / math.tan(t) for t in _angles(m.vxy[m.tri[f]])]
        loc = lv.loc[f]
        for j in range(1, n - 2):
            for i in range(1, n - 1 - j):
                p = loc[j, i]
                assert abs(A[p, p] - 2 * sum(c)) < 1e-12
                assert abs(A[p, loc[j, i + 1]] + c[2]) < 1e-12
                assert abs(A[p, loc[j, i - 1]] + c[2]) < 1e-12
                assert abs(A[p, loc[j + 1, i]] + c[1]) < 1e-12
                assert abs(A[p, loc[j - 1, i]] + c[1]) < 1e-12
                assert abs(A[p, loc[j - 1, i + 1]] + c[0]) < 1e-12
                assert abs(A[p, loc[j + 1, i - 1]] + c[0]) < 1e-12
                assert A[p].nnz == 7


def test_stencil_level_independent():
    """2D P1 stiffness is scale invariant, so a point's stencil does not
    depend on the level (same physical point at levels 3 and 4)."""
    m = MacroMesh(*hi.annulus(16))
    l3, l4 = Level(m, 3), Level(m, 4)
    A3, A4 = assemble(l3)["A"], assemble(l4)["A"]
    for p3 in range(0, l3.n_all, 11):
        if l3.dirichlet[p3]:
            continue
        p4 = np.flatnonzero(np.abs(l4.xy - l3.xy[p3]).sum(1) < 1e-12)[0]
        assert abs(A3[p3, p3] - A4[p4, p4]) < 1e-12
        assert abs(np.sort(A3[p3].data) - np.sort(A4[p4].data)).max() < 1e-12


@pytest.mark.parametrize("name", ["square", "annulus64"])
def test_row_sums_symmetry_and_mass(name):
    m = MacroMesh(*hi.mesh_by_name(name))
    lv = Level(m, 3)
    kap = np.exp(hi.grf_eval(lv.xy, seed=3))
    for kappa in (None, kap):
        mats = assemble(lv, kappa)
        A, M = mats["A"], mats["M"]
        assert np.abs(A @ np.ones(lv.n_all)).max() < 1e-12
        assert abs(A - A.T).max() < 1e-14
        # positive definite on interior points
        ii = lv.interior
        ev = np.linalg.eigvalsh(A[ii][:, ii].toarray())
        assert ev.min() > 0
    area = 1.0 if name == "square" else None
    one = np.ones(lv.n_all)
    tot = one @ (M @ one)
    xm = m.vxy[m.tri]
    dm = 0.5 * ((xm[:, 1, 0] - xm[:, 0, 0]) * (xm[:, 2, 1] - xm[:, 0, 1])
                - (xm[:, 1, 1] - xm[:, 0, 1]) * (xm[:, 2, 0] - xm[:, 0, 0])).__abs__().sum()
    assert abs(tot - dm) < 1e-12
    if area is not None:
        assert abs(tot - area) < 1e-14


def test_variable_k_constant_field_scales():
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, 3)
    A1 = assemble(lv)["A"]
    A7 = assemble(lv, np.full(lv.n_all, 7.0))["A"]
    assert abs(A7 - 7.0 * A1).max() < 1e-12


def test_variable_k_brute_force_quadrature():
    """k_T = mean of the nodal k is the exact integral of the P1 interpolant
    of k against constant gradients: compare with a 3-point edge-midpoint
    quadrature (exact for linear k) computed here triangle by triangle."""
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, 2)
    kap = 1.0 + np.random.default_rng(0).random(lv.n_all)
    A = assemble(lv, kap)["A"].toarray()
    from oracle.assemble import micro_triangles
    ref = np.zeros_like(A)
    for t in micro_triangles(lv):
        x = lv.xy[t]
        B = np.array([[x[1, 0] - x[0, 0], x[2, 0] - x[0, 0]],
                      [x[1, 1] - x[0, 1], x[2, 1] - x[0, 1]]])
        area = 0.5 * abs(np.linalg.det(B))
        G = np.linalg.inv(B).T @ np.array([[-1.0, 1.0, 0.0], [-1.0, 0.0, 1.0]])
        kq = np.mean([0.5 * (kap[t[a]] + kap[t[b]]) for a, b in ((0, 1), (1, 2), (0, 2))])
        ref[np.ix_(t, t)] += kq * area * (G.T @ G)
    assert np.abs(A - ref).max() < 1e-12


@pytest.mark.parametrize("variable_k", [False, True])
def test_rows_at_equals_assembled_rows(variable_k):
    """The sampled-row operator (for levels too large to assemble) equals the
    rows of the globally assembled stiffness."""
    from oracle.assemble import assemble, rows_at
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, 4)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(lv.n_all)
    pts = np.concatenate([np.arange(m.V), rng.choice(lv.n_all, 300, replace=False)])
    pts = np.unique(pts)
    kf = (lambda xy: np.exp(hi.grf_eval(xy, 3))) if variable_k else None
    A = assemble(lv, None if kf is None else kf(lv.xy))["A"]
    got = rows_at(lv, pts, x, kf)
    assert np.abs(got - (A @ x)[pts]).max() <= 1e-13 * np.abs(A @ x).max()
