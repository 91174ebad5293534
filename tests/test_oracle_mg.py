"""Pins of the oracle's multigrid pieces (CPU only)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import hhg_inputs as hi
from oracle.mesh import Level, MacroMesh
from oracle.mg import Hierarchy, pcg_jacobi, prolongation, stage_sets


@pytest.fixture(scope="module")
def ann4():
    return Hierarchy(MacroMesh(*hi.annulus(16)), 4, 2)


def test_prolongation_reproduces_linear_functions(ann4):
    for l in (3, 4):
        lf, lc = ann4.levels[l], ann4.levels[l - 1]
        for a, b, c in ((1.0, 0, 0), (0.3, -1.7, 2.2)):
            uc = a + b * lc.xy[:, 0] + c * lc.xy[:, 1]
            uf = a + b * lf.xy[:, 0] + c * lf.xy[:, 1]
            assert np.abs(ann4.P[l] @ uc - uf).max() < 1e-13
        # each fine row has weight sum 1 and at most two entries
        P = ann4.P[l]
        assert np.allclose(P @ np.ones(lc.n_all), 1.0)
        assert np.diff(P.indptr).max() <= 2


def test_galerkin_identity(ann4):
    """Nested P1 spaces with the same bilinear form: P^T A_f P = A_c."""
    for l in (3, 4):
        P = ann4.P[l]
        G = (P.T @ ann4.A[l] @ P - ann4.A[l - 1])
        assert abs(G).max() < 1e-12


def test_stages_cover_interior_and_are_independent(ann4):
    for l in (2, 3, 4):
        lv = ann4.levels[l]
        S = stage_sets(lv)
        allp = np.sort(np.concatenate(S))
        assert (allp == lv.interior).all()
        A = ann4.A[l].tocsr()
        for s, idx in enumerate(S):
            sub = A[idx][:, idx].tocoo()
            off = (sub.row != sub.col) & (np.abs(sub.data) > 1e-12)
            if s != 1:
                assert not off.any(), "stage %d not independent" % s
            else:
                # stage B: only the corner pairs of two edges meeting at a
                # vertex inside one face (both at distance one micro-edge)
                p, q = idx[sub.row[off]], idx[sub.col[off]]
                assert (lv.kind[p] == 1).all() and (lv.kind[q] == 1).all()
                assert (lv.prim[p] != lv.prim[q]).all()
                n = lv.n
                assert np.isin(lv.kidx[p], (1, n - 2)).all()
                assert np.isin(lv.kidx[q], (1, n - 2)).all()


def test_stage_update_solves_its_rows(ann4):
    """After an independent stage the residual on its points is zero."""
    l = 3
    lv = ann4.levels[l]
    rng = np.random.default_rng(5)
    u = rng.random(lv.n_all)
    f = rng.random(lv.n_all)
    d = ann4.diag[l]
    for s, (S, AS) in enumerate(ann4.stages[l]):
        u[S] += (f[S] - AS @ u) / d[S]
        if s != 1:
            assert np.abs((f - ann4.A[l] @ u)[S]).max() < 1e-12


def _red_black_textbook(u, f, m, backward=False):
    """Red-black Gauss-Seidel for the unscaled 5-point operator on an m x m
    grid with zero boundary, plain loops (red = (x + y) even first)."""
    u = u.copy()
    order = (1, 0) if backward else (0, 1)
    for colour in order:
        new = u.copy()
        for y in range(m):
            for x in range(m):
                if (x + y) % 2 != colour:
                    continue
                s = 0.0
                if x > 0: s += u[y, x - 1]
                if x < m - 1: s += u[y, x + 1]
                if y > 0: s += u[y - 1, x]
                if y < m - 1: s += u[y + 1, x]
                new[y, x] = (f[y, x] + s) / 4.0
        u = new
    return u


@pytest.mark.parametrize("backward", [False, True])
def test_unit_square_sweep_is_red_black(backward):
    H = Hierarchy(MacroMesh(*hi.unit_square()), 4, 2)
    lv = H.levels[4]
    n = lv.n
    m = n - 2
    h = 1.0 / (n - 1)
    ii = lv.interior
    gx = np.rint(lv.xy[ii, 0] / h).astype(int) - 1
    gy = np.rint(lv.xy[ii, 1] / h).astype(int) - 1
    rng = np.random.default_rng(2)
    u = np.zeros(lv.n_all)
    f = np.zeros(lv.n_all)
    u[ii] = rng.random(len(ii))
    f[ii] = rng.random(len(ii))
    ug = np.zeros((m, m)); fg = np.zeros((m, m))
    ug[gy, gx] = u[ii]; fg[gy, gx] = f[ii]
    ref = _red_black_textbook(ug, fg, m, backward)
    H.smooth(4, u, f, 1, backward=backward)
    assert np.abs(u[ii] - ref[gy, gx]).max() < 1e-14


def _dense_vcycle_error(H, l, nu1, nu2):
    """Error propagation of the V-cycle as a dense matrix on interior points:
    E = S_post (I - P_int B_{l-1} P_int^T A) S_pre, with B the (recursive)
    approximate coarse inverse and B_lc = A_lc^-1."""
    lv = H.levels[l]
    ii = lv.interior
    A = H.A[l].toarray()[np.ix_(ii, ii)]
    N = len(ii)
    if l == H.lc:
        return np.zeros((N, N)), np.linalg.inv(A)
    pos = -np.ones(lv.n_all, dtype=int)
    pos[ii] = np.arange(N)
    stage_mats = []
    for S, _ in H.stages[l]:
        Sm = np.eye(N)
        rows = pos[S]
        Sm[rows] -= A[rows] / np.diag(A)[rows][:, None]
        stage_mats.append(Sm)
    pre = np.eye(N)
    for Sm in stage_mats:
        pre = Sm @ pre
    post = np.eye(N)
    for Sm in stage_mats[::-1]:
        post = Sm @ post
    Spre = np.linalg.matrix_power(pre, nu1)
    Spost = np.linalg.matrix_power(post, nu2)
    _, Bc = _dense_vcycle_error(H, l - 1, nu1, nu2)
    ic = H.levels[l - 1].interior
    P = H.P[l].toarray()[np.ix_(ii, ic)]
    CG = np.eye(N) - P @ Bc @ P.T @ A
    E = Spost @ CG @ Spre
    B = (np.eye(N) - E) @ np.linalg.inv(A)
    return E, B


@pytest.fixture(scope="module")
def ann3c1():
    return Hierarchy(MacroMesh(*hi.annulus(16)), 3, 1)


@pytest.mark.parametrize("nu", [(1, 1), (3, 3), (2, 0)])
def test_vcycle_matches_dense_error_propagation(ann3c1, nu):
    """Three levels (3 -> 2 -> 1) against the dense recursive formula."""
    ann4 = ann3c1
    l = 3
    lv = ann4.levels[l]
    ii = lv.interior
    E, _ = _dense_vcycle_error(ann4, l, *nu)
    rng = np.random.default_rng(1)
    for trial in range(3):
        e0 = np.zeros(lv.n_all)
        e0[ii] = rng.standard_normal(len(ii))
        u = e0.copy()
        ann4.vcycle(l, u, np.zeros(lv.n_all), *nu)   # exact solution is 0
        assert np.abs(u[ii] - E @ e0[ii]).max() < 1e-12 * np.abs(e0).max()
    if nu[0] == nu[1]:
        A = ann4.A[l].toarray()[np.ix_(ii, ii)]
        AE = A @ E
        assert np.abs(AE - AE.T).max() < 1e-10


def test_pcg_matches_direct_solve(ann4):
    A = ann4.A_coarse
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    x, it = pcg_jacobi(A, b)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.abs(x - xd).max() < 1e-11 * np.abs(xd).max()
    assert np.linalg.norm(b - A @ x) <= 1e-14 * np.linalg.norm(b)
    assert it < 4 * len(b)
    assert pcg_jacobi(A, np.zeros(len(b)))[1] == 0


def test_coarse_solve_direct_and_pcg(ann4):
    """The direct coarse solve is the exact solution; the PCG alternative
    agrees within its stopping tolerance."""
    lvc = ann4.levels[ann4.lc]
    ic = lvc.interior
    rng = np.random.default_rng(4)
    f = np.zeros(lvc.n_all)
    f[ic] = rng.standard_normal(len(ic))
    u = np.zeros(lvc.n_all)
    assert ann4.coarse_solve(u, f) == 0
    xd = np.linalg.solve(ann4.A_coarse.toarray(), f[ic])
    assert np.abs(u[ic] - xd).max() <= 1e-13 * np.abs(xd).max()
    Hp = Hierarchy(ann4.mesh, ann4.lc + 1, ann4.lc, coarse="pcg")
    up = np.zeros(lvc.n_all)
    assert Hp.coarse_solve(up, f) > 0
    assert np.abs(up[ic] - xd).max() <= 1e-11 * np.abs(xd).max()


def test_solve_matches_sparse_direct():
    H = Hierarchy(MacroMesh(*hi.annulus(16)), 5, 2)
    lv = H.levels[5]
    f = hi.uniform_rhs(lv.n_all, 1)
    u, hist = H.solve(np.zeros(lv.n_all), f, rtol=1e-11)
    ii = lv.interior
    ud = spla.spsolve(H.A[5][ii][:, ii].tocsc(), f[ii])
    assert np.linalg.norm(u[ii] - ud) <= 1e-9 * np.linalg.norm(ud)
    rho = (hist[-1] / hist[2]) ** (1.0 / (len(hist) - 3))
    assert 0.08 < rho < 0.25


def test_manufactured_solution_second_order():
    """-Laplace u = 2 pi^2 sin sin on the unit square, b = M f_I, g = 0:
    the lumped-mass weighted nodal error falls by ~4 per level."""
    errs = []
    for l in range(3, 8):
        H = Hierarchy(MacroMesh(*hi.unit_square()), l, 2)
        lv = H.levels[l]
        b = H.M[l] @ hi.manufactured_f(lv.xy)
        u, _ = H.solve(np.zeros(lv.n_all), b, rtol=1e-12, nu1=2, nu2=2)
        mlump = np.asarray(H.M[l].sum(axis=1)).ravel()
        e = u - hi.manufactured_u(lv.xy)
        errs.append(math.sqrt((mlump * e * e).sum()))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert ((ratios > 3.6) & (ratios < 4.4)).all(), ratios


def test_dirichlet_values_preserved(ann4):
    lv = ann4.levels[4]
    rng = np.random.default_rng(9)
    u = rng.random(lv.n_all)
    d0 = u[lv.dirichlet].copy()
    ann4.vcycle(4, u, rng.random(lv.n_all), 2, 2)
    assert (u[lv.dirichlet] == d0).all()
