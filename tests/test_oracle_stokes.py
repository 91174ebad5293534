"""Pins of the oracle's Stokes system, block preconditioner and MINRES (CPU
only).  Each pin comes from outside the code it checks: exact integrals of
polynomials (the divergence and gradient blocks are exact on linear fields),
the closed-form stabilisation energy of a linear pressure, symmetry by dense
assembly, a manufactured smooth Stokes flow whose velocity error must fall
as h^2, a dense Krylov least-squares minimiser for MINRES, and a sparse
direct solve."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import hhg_inputs as hi
from oracle import stokes as S
from oracle.mesh import Level, MacroMesh


def mesh(name):
    return MacroMesh(*hi.mesh_by_name(name))


def test_face_viscosity_jumps_at_the_middle_ring():
    m = mesh("annulus64")
    mu = S.face_viscosity(m)
    assert sorted(set(mu.tolist())) == [1.0, 100.0]
    c = m.vxy[m.tri].mean(axis=1)
    r = np.hypot(c[:, 0], c[:, 1])
    # faces of the inner ring of quads (the first 2 * 16 faces) have mu = 1
    assert (mu[:32] == 1.0).all() and (mu[32:] == 100.0).all()
    assert r[:32].max() < 0.775 < r[32:].min()


@pytest.mark.parametrize("name,level", [("annulus64", 3), ("square", 4)])
def test_divergence_of_a_linear_velocity(name, level):
    """For u = (a + b x + c y, d + e x + g y), div u = b + g is constant, so
    (B u_I)_q = -int psi_q div u = -(b + g) int psi_q, and int psi_q is the
    row sum of the consistent mass matrix."""
    lv = Level(mesh(name), level)
    bl = S.assemble_stokes(lv, np.full(lv.mesh.F, 3.0))
    from oracle.assemble import assemble
    M = assemble(lv, want=("M",))["M"]
    x, y = lv.xy[:, 0], lv.xy[:, 1]
    ux = 0.3 + 1.7 * x - 0.4 * y
    uy = -1.1 + 0.6 * x + 2.9 * y
    got = bl["Bx"] @ ux + bl["By"] @ uy
    want = -(1.7 + 2.9) * np.asarray(M.sum(axis=1)).ravel()
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max() * 10


@pytest.mark.parametrize("name,level", [("annulus64", 3), ("square", 4)])
def test_gradient_of_a_linear_pressure(name, level):
    """(B^T p)_b = -int p div phi_b = int grad p . phi_b for a velocity test
    function phi_b that vanishes on the boundary (integration by parts), so
    for p = a + b x + c y: (Bx^T p)_b = b int phi_b, (By^T p)_b = c int phi_b
    at every interior point b."""
    lv = Level(mesh(name), level)
    bl = S.assemble_stokes(lv, np.ones(lv.mesh.F))
    from oracle.assemble import assemble
    M = assemble(lv, want=("M",))["M"]
    row = np.asarray(M.sum(axis=1)).ravel()
    p = 0.7 - 2.3 * lv.xy[:, 0] + 1.3 * lv.xy[:, 1]
    ii = lv.interior
    gx, gy = bl["Bx"].T @ p, bl["By"].T @ p
    assert np.abs(gx[ii] - (-2.3) * row[ii]).max() <= 1e-13 * row.max()
    assert np.abs(gy[ii] - 1.3 * row[ii]).max() <= 1e-13 * row.max()


@pytest.mark.parametrize("level", [2, 3, 4])
def test_stabilisation_energy_of_a_linear_pressure(level):
    """c(p, p) = delta sum_T h_T^2 / mu_T |T| |grad p|^2.  On the unit square
    every micro-triangle is right-angled with legs 2^-l, so h_T^2 = 2 4^-l
    and, for p = x with mu = 2, c(p, p) = delta * 2 * 4^-l / 2 * 1.  The
    stabilisation annihilates constants."""
    lv = Level(mesh("square"), level)
    bl = S.assemble_stokes(lv, np.full(2, 2.0))
    p = lv.xy[:, 0].copy()
    want = S.DELTA * 2.0 * 4.0 ** -level / 2.0
    assert abs(p @ (bl["C"] @ p) - want) <= 1e-14
    assert np.abs(bl["C"] @ np.ones(lv.n_all)).max() <= 1e-15


def test_lumped_pressure_mass_integrates_one_over_mu():
    m = mesh("annulus64")
    lv = Level(m, 3)
    mu = S.face_viscosity(m)
    bl = S.assemble_stokes(lv, mu)
    P = m.vxy[m.tri]
    area = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                        - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0]))
    assert abs(bl["m"].sum() - (area / mu).sum()) <= 1e-13
    assert (bl["m"] > 0).all()


@pytest.mark.parametrize("level", [3, 4])
def test_pressure_block_of_the_preconditioner_in_closed_form(level):
    """On the unit square every interior point sits in six right isosceles
    micro-triangles with legs h = 2^-level: lumped mass 6 (h^2/2) / 3 = h^2,
    P1 stiffness diagonal 4, longest edge sqrt(2) h, so diag(C) =
    (1/12) 2 h^2 4 = 2 h^2 / 3 and the pressure block m + 4 diag(C) is
    11 h^2 / 3 (mu = 1)."""
    st = S.Stokes(mesh("square"), level, 1)
    h2 = 4.0 ** -level
    inner = ~st.dir
    assert inner.sum() == (2 ** level - 1) ** 2
    assert np.abs(st.m[inner] - h2).max() <= 1e-14
    assert np.abs(st.s[inner] - 11.0 * h2 / 3.0).max() <= 1e-14
    # the preconditioner divides the pressure by that block
    e = np.zeros(3 * st.N)
    e[2 * st.N:] = 1.0
    assert np.abs(st.precond(e)[2 * st.N:][inner] - 3.0 / (11.0 * h2)).max() <= 1e-12 / h2


@pytest.mark.parametrize("name,level", [("annulus64", 2), ("square", 3)])
def test_stokes_matrix_is_symmetric_with_a_constant_pressure_kernel(name, level):
    st = S.Stokes(mesh(name), level, 1, S.face_viscosity(mesh(name)) if name != "square" else None)
    K = st.matrix().toarray()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    # the operator applied column by column equals the matrix (Dirichlet
    # velocity columns aside, where the matrix holds the identity)
    E = np.eye(3 * st.N)
    keep = np.concatenate([~st.dir, ~st.dir, np.ones(st.N, bool)])
    Kop = np.stack([st.apply(E[:, k]) for k in range(3 * st.N)], 1)
    assert np.abs((Kop - K)[np.ix_(keep, keep)]).max() <= 1e-14 * np.abs(K).max()
    ones_p = np.concatenate([np.zeros(2 * st.N), np.ones(st.N)])
    assert np.abs(st.apply(ones_p)).max() <= 1e-14 * np.abs(K).max()


def test_preconditioner_is_symmetric_positive_definite():
    st = S.Stokes(mesh("annulus64"), 3, 2, S.face_viscosity(mesh("annulus64")))
    keep = np.concatenate([~st.dir, ~st.dir, np.ones(st.N, bool)])
    idx = np.flatnonzero(keep)
    E = np.zeros(3 * st.N)
    cols = []
    for k in idx:
        E[k] = 1.0
        cols.append(st.precond(E)[idx])
        E[k] = 0.0
    Pinv = np.stack(cols, 1)
    assert np.abs(Pinv - Pinv.T).max() <= 1e-12 * np.abs(Pinv).max()
    assert np.linalg.eigvalsh(0.5 * (Pinv + Pinv.T)).min() > 0


def test_minres_iterates_minimise_the_residual_over_the_krylov_space():
    """x_k = x_0 + argmin over the Krylov space K_k(P^-1 K, P^-1 r_0) of the
    P^-1-norm of b - K x, found here by a dense least-squares solve over an
    orthonormalised Krylov basis (no Lanczos, no rotations)."""
    m = mesh("annulus64")
    st = S.Stokes(m, 2, 1, S.face_viscosity(m), nu=(1, 1))
    keep = np.concatenate([~st.dir, ~st.dir, np.ones(st.N, bool)])
    idx = np.flatnonzero(keep)
    n = 3 * st.N
    E = np.zeros(n)
    Pcols, Kcols = [], []
    for k in idx:
        E[k] = 1.0
        Pcols.append(st.precond(E)[idx])
        Kcols.append(st.apply(E)[idx])
        E[k] = 0.0
    Pinv = np.stack(Pcols, 1)
    Kd = np.stack(Kcols, 1)
    Pinv = 0.5 * (Pinv + Pinv.T)
    R = sla.cholesky(Pinv)                 # Pinv = R^T R
    rng = np.random.default_rng(3)
    b = np.zeros(n)
    b[idx] = rng.uniform(-1, 1, len(idx))
    b[2 * st.N:] = 0.0
    x0 = np.zeros(n)
    r0 = b[idx]
    basis = []
    q = Pinv @ r0
    for k in range(1, 7):
        basis.append(q)
        Q, _ = np.linalg.qr(np.stack(basis, 1))
        c, *_ = np.linalg.lstsq(R @ (Kd @ Q), R @ r0, rcond=None)
        want = Q @ c
        got, hist = S.minres(st.apply, st.precond, b, x0, rtol=0.0, max_iters=k)
        assert len(hist) == k + 1
        scale = np.abs(want).max()
        assert np.abs(got[idx] - want).max() <= 1e-9 * scale
        res = r0 - Kd @ want
        assert abs(hist[-1] - math.sqrt(res @ Pinv @ res)) <= 1e-9 * hist[0]
        q = Pinv @ (Kd @ q)


def test_minres_converges_to_the_direct_solution():
    m = mesh("annulus64")
    st = S.Stokes(m, 4, 2, S.face_viscosity(m))
    lv = st.lv
    T = hi.grf_eval(lv.xy, 500)
    r = np.hypot(lv.xy[:, 0], lv.xy[:, 1])
    b = st.rhs(-T * lv.xy[:, 0] / r, -T * lv.xy[:, 1] / r)
    x, hist = S.minres(st.apply, st.precond, b, np.zeros(3 * st.N), rtol=1e-12, max_iters=2000)
    assert hist[-1] <= 1e-12 * hist[0]
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))   # monotone
    # direct: pin the pressure at one point, then remove the weighted mean
    K = st.matrix().tolil()
    k0 = 2 * st.N
    K[k0, :] = 0.0
    K[k0, k0] = 1.0
    rhs = b.copy()
    rhs[k0] = 0.0
    xd = S.pressure_mean_free(st, spla.spsolve(K.tocsc(), rhs))
    # MINRES keeps the weighted pressure mean at zero by itself
    assert abs(st.s @ x[2 * st.N:]) <= 1e-10 * np.abs(st.s * x[2 * st.N:]).sum()
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()


def _manufactured(xy):
    """u = curl of psi = sin^2(pi x) sin^2(pi y) (zero with its gradient on
    the unit square's boundary, divergence free), p = sin(pi x) cos(pi y)
    (zero mean); f = -Laplace u + grad p."""
    x, y = xy[:, 0], xy[:, 1]
    pi = math.pi
    ux = pi * np.sin(pi * x) ** 2 * np.sin(2 * pi * y)
    uy = -pi * np.sin(2 * pi * x) * np.sin(pi * y) ** 2
    p = np.sin(pi * x) * np.cos(pi * y)
    fx = -2 * pi ** 3 * np.sin(2 * pi * y) * (2 * np.cos(2 * pi * x) - 1) + pi * np.cos(pi * x) * np.cos(pi * y)
    fy = 2 * pi ** 3 * np.sin(2 * pi * x) * (2 * np.cos(2 * pi * y) - 1) - pi * np.sin(pi * x) * np.sin(pi * y)
    return ux, uy, p, fx, fy


def test_manufactured_forcing_is_minus_laplacian_plus_gradient():
    """The hand-derived f against central differences of u and p."""
    rng = np.random.default_rng(0)
    xy = rng.uniform(0.1, 0.9, (50, 2))
    h = 1e-4
    ux, uy, p, fx, fy = _manufactured(xy)

    def at(dx, dy):
        return _manufactured(xy + np.array([dx, dy]))

    E, W, N, Sx = at(h, 0), at(-h, 0), at(0, h), at(0, -h)
    lap = [(E[c] + W[c] + N[c] + Sx[c] - 4 * (ux, uy)[c]) / h ** 2 for c in (0, 1)]
    gp = ((E[2] - W[2]) / (2 * h), (N[2] - Sx[2]) / (2 * h))
    assert np.abs(-lap[0] + gp[0] - fx).max() <= 1e-4 * np.abs(fx).max()
    assert np.abs(-lap[1] + gp[1] - fy).max() <= 1e-4 * np.abs(fy).max()
    div = (E[0] - W[0]) / (2 * h) + (N[1] - Sx[1]) / (2 * h)
    assert np.abs(div).max() <= 1e-6


def test_manufactured_stokes_velocity_error_falls_as_h_squared():
    """Nodal velocity error of the discrete solution (MINRES to 1e-11, block
    multigrid preconditioner) against the smooth flow: ratios between levels
    tend to 4 (second order); the pressure error falls too."""
    m = mesh("square")
    prev = None
    ratios = []
    for level in range(3, 7):
        st = S.Stokes(m, level, 2)
        ux, uy, p, fx, fy = _manufactured(st.lv.xy)
        x, _ = S.minres(st.apply, st.precond, st.rhs(fx, fy), np.zeros(3 * st.N), rtol=1e-11,
                        max_iters=1000)
        x = S.pressure_mean_free(st, x)
        eu = max(np.abs(x[:st.N] - ux).max(), np.abs(x[st.N:2 * st.N] - uy).max())
        pm = p - (st.s @ p) / st.s.sum()
        ep = np.abs(x[2 * st.N:] - pm).max()
        if prev is not None:
            ratios.append(prev[0] / eu)
            assert ep < prev[1]
        prev = (eu, ep)
    assert 3.5 <= ratios[-2] <= 4.5 and 3.7 <= ratios[-1] <= 4.3, ratios
