"""GPU parity of the Stokes path (face coefficient, Stokes operator, block
preconditioner, MINRES) against the oracle, through the C ABI.

FP64 operator, residual, preconditioner and dot: 1e-12 relative (max norm).
MINRES: the first iterations follow the oracle's to 1e-10 (each step divides
by the norms of nearly cancelling Lanczos vectors, so rounding differences of
1e-16 grow slowly with the step count); converged solutions agree within the
accuracy the stopping test guarantees.  Inputs: seeded uniform vectors on
the jittered annulus with a 1:100 viscosity jump and on the unit square."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import F32_VCYCLE_TOL, log, rel_err, to_np

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
_CACHE = {}


def setup(name, L, nu=(2, 2), lc=2):
    """(library mesh with Stokes set up, oracle Stokes system)."""
    import paper_1805_10167_amd as P
    from oracle import stokes as S
    from oracle.mesh import MacroMesh
    key = (name, L, nu, lc)
    if key not in _CACHE:
        vxy, tri = hi.mesh_by_name(name)
        m = MacroMesh(vxy, tri)
        mu = np.ones(m.F) if name == "square" else S.face_viscosity(m)
        st = S.Stokes(m, L, lc, mu, nu=nu)
        g = P.Mesh(vxy, tri, L, lc, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
        P.hhg_stokes_setup(g.h, mu, S.DELTA)
        _CACHE[key] = (g, st)
    return _CACHE[key]


def random_stokes(st, seed, dirichlet_zero=True):
    x = hi.uniform_vector(3 * st.N, seed)
    if dirichlet_zero:
        x[:st.N][st.dir] = 0.0
        x[st.N:2 * st.N][st.dir] = 0.0
    return x


CASES = [("annulus64", 4), ("annulus64", 6), ("square", 5), ("annulus128", 5)]


@pytest.mark.parametrize("name,L", CASES)
def test_face_coefficient_operator_and_vcycle(name, L):
    """HHG_OP_LAPLACE with a coefficient per macro-face against the oracle's
    assembly with the same coefficient: apply on several levels and one
    V(2,2) cycle (coarse operators, inverse and smoother all rebuilt)."""
    import paper_1805_10167_amd as P
    log("face coefficient %s L=%d" % (name, L))
    g, st = setup(name, L)
    H = st.H
    for lvl in sorted({L, L - 1, 2}):
        x = hi.uniform_vector(H.levels[lvl].n_all, 10 + lvl)
        y = g.field(lvl)
        P.hhg_apply(g.h, lvl, P.HHG_OP_LAPLACE, P.HHG_F64, g.from_canonical(lvl, x), y)
        assert rel_err(to_np(g.to_canonical(lvl, y)), H.apply(lvl, x)) <= F64_TOL
    lv = H.levels[L]
    u, f = hi.uniform_vector(lv.n_all, 5), hi.uniform_vector(lv.n_all, 6)
    uf, ff = g.from_canonical(L, u), g.from_canonical(L, f)
    P.hhg_vcycle(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, 2, 2)
    err = rel_err(to_np(g.to_canonical(L, uf)), H.vcycle(L, u.copy(), f, 2, 2))
    log("  V-cycle rel err %.2e" % err)
    assert err <= F64_TOL


def test_face_coefficient_of_ones_is_the_plain_operator():
    import torch

    import paper_1805_10167_amd as P
    vxy, tri = hi.mesh_by_name("annulus64")
    g = P.Mesh(vxy, tri, 4, 2, P.HHG_FEAT_F64)
    _, n_all = g.n_dofs(4)
    x = g.from_canonical(4, hi.uniform_vector(n_all, 3))
    y0, y1, y2 = g.field(4), g.field(4), g.field(4)
    P.hhg_apply(g.h, 4, P.HHG_OP_LAPLACE, P.HHG_F64, x, y0)
    P.hhg_set_face_coefficient(g.h, np.full(len(tri), 2.5))
    P.hhg_apply(g.h, 4, P.HHG_OP_LAPLACE, P.HHG_F64, x, y1)
    P.hhg_set_face_coefficient(g.h, np.ones(len(tri)))
    P.hhg_apply(g.h, 4, P.HHG_OP_LAPLACE, P.HHG_F64, x, y2)
    assert torch.equal(y0, y2)
    assert rel_err(to_np(y1), 2.5 * to_np(y0)) <= 1e-15
    with pytest.raises(P.HHGError):
        P.hhg_set_face_coefficient(g.h, np.r_[np.ones(len(tri) - 1), -1.0])


@pytest.mark.parametrize("name,L", CASES)
def test_stokes_apply_and_residual(name, L):
    """y = K x on several levels (the divergence/gradient blocks scale with
    h, the stabilisation with h^2) with non-zero boundary velocity data, and
    r = b - K x; both with consistent copies (the operator applied to the
    result through the library equals the oracle's on canonical values)."""
    import paper_1805_10167_amd as P
    from oracle import stokes as S
    from oracle.mesh import MacroMesh
    log("stokes apply %s L=%d" % (name, L))
    g, st = setup(name, L)
    m = MacroMesh(*hi.mesh_by_name(name))
    for lvl in sorted({L, L - 1, 2}):
        sl = st if lvl == L else S.Stokes(m, lvl, 1 if lvl <= 2 else 2, st.mu_face)
        x = random_stokes(sl, 40 + lvl, dirichlet_zero=False)
        xf, y = g.stokes_from_canonical(lvl, x), g.stokes_vector(lvl)
        P.hhg_stokes_apply(g.h, lvl, xf, y)
        ref = sl.apply(x)
        err = rel_err(to_np(g.stokes_to_canonical(lvl, y)), ref)
        assert err <= F64_TOL, (lvl, err)
        # copies of y are consistent
        y2 = g.stokes_vector(lvl)
        P.hhg_stokes_apply(g.h, lvl, y, y2)
        yc = to_np(g.stokes_to_canonical(lvl, y))
        assert rel_err(to_np(g.stokes_to_canonical(lvl, y2)), sl.apply(yc)) <= F64_TOL
    x = random_stokes(st, 50, dirichlet_zero=False)
    b = random_stokes(st, 51)
    r = g.stokes_vector(L)
    P.hhg_stokes_residual(g.h, L, g.stokes_from_canonical(L, x), g.stokes_from_canonical(L, b), r)
    ref = b - st.apply(x)
    ref[:st.N][st.dir] = 0.0
    ref[st.N:2 * st.N][st.dir] = 0.0
    assert rel_err(to_np(g.stokes_to_canonical(L, r)), ref) <= F64_TOL


@pytest.mark.parametrize("name,L", CASES)
def test_stokes_preconditioner_and_dot(name, L):
    import torch

    import paper_1805_10167_amd as P
    log("stokes precond %s L=%d" % (name, L))
    g, st = setup(name, L)
    r = random_stokes(st, 60)
    rf, z = g.stokes_from_canonical(L, r), g.stokes_vector(L)
    P.hhg_stokes_precond(g.h, P.HHG_F64, rf, z, 2, 2)
    zg = to_np(g.stokes_to_canonical(L, z))
    err = rel_err(zg, st.precond(r))
    log("  precond rel err %.2e" % err)
    assert err <= F64_TOL
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.hhg_stokes_dot(g.h, L, rf, z, out)
    ref = float(r @ zg)
    assert abs(out.item() - ref) <= 1e-13 * np.abs(r * zg).sum()
    # FP32 V-cycles in the velocity blocks: within the FP32 V-cycle bound
    z32 = g.stokes_vector(L)
    P.hhg_stokes_precond(g.h, P.HHG_F32, rf, z32, 2, 2)
    assert rel_err(to_np(g.stokes_to_canonical(L, z32)), st.precond(r)) <= F32_VCYCLE_TOL


@pytest.mark.parametrize("name,L,k", [("annulus64", 4, 12), ("square", 5, 12), ("annulus128", 5, 8)])
def test_minres_first_iterations_follow_the_oracle(name, L, k):
    import paper_1805_10167_amd as P
    from oracle import stokes as S
    log("minres %d steps %s L=%d" % (k, name, L))
    g, st = setup(name, L)
    b = random_stokes(st, 70)
    b[2 * st.N:] = 0.0
    x0 = random_stokes(st, 71) * 0.1
    xf, bf = g.stokes_from_canonical(L, x0), g.stokes_from_canonical(L, b)
    rc, stats, hist = P.hhg_stokes_solve(g.h, xf, bf, rtol=0.0, max_iters=k, nu1=2, nu2=2)
    assert rc == P.HHG_ENOTCONV and stats["iters"] == k
    xo, ho = S.minres(st.apply, st.precond, b, x0, rtol=0.0, max_iters=k)
    eh = rel_err(hist, ho)
    ex = rel_err(to_np(g.stokes_to_canonical(L, xf)), xo)
    log("  history rel err %.2e, iterate rel err %.2e" % (eh, ex))
    assert eh <= 1e-10 and ex <= 1e-10


@pytest.mark.parametrize("name,L", [("annulus64", 5), ("square", 6)])
def test_minres_solve_to_tolerance(name, L):
    """Solve to 1e-8 in the preconditioner's norm.  FP64 velocity cycles:
    the same iteration count as the oracle's MINRES and its solution within
    1e-8 (the two follow the same iterates, apart from rounding the Lanczos
    process amplifies slowly).  FP32 velocity cycles: converged, and within
    1e-5 of an oracle solve to 1e-12, as is the FP64 solution (the 1e-8
    residual bound times the norm of the preconditioned inverse, a few
    hundred here)."""
    import paper_1805_10167_amd as P
    from oracle import stokes as S
    log("minres solve %s L=%d" % (name, L))
    g, st = setup(name, L)
    lv = st.lv
    if name == "square":
        # the manufactured smooth flow's forcing
        from test_oracle_stokes import _manufactured
        _, _, _, fx, fy = _manufactured(lv.xy)
        b = st.rhs(fx, fy)
    else:
        # buoyancy -T r_hat from a seeded random temperature field
        T = hi.grf_eval(lv.xy, 500)
        rr = np.hypot(lv.xy[:, 0], lv.xy[:, 1])
        b = st.rhs(-T * lv.xy[:, 0] / rr, -T * lv.xy[:, 1] / rr)
    xo, ho = S.minres(st.apply, st.precond, b, np.zeros(3 * st.N), rtol=1e-8, max_iters=1000)
    xt, _ = S.minres(st.apply, st.precond, b, np.zeros(3 * st.N), rtol=1e-12, max_iters=2000)
    scale = np.abs(xt).max()
    bf = g.stokes_from_canonical(L, b)
    for prec in (P.HHG_F64, P.HHG_F32):
        xf = g.stokes_vector(L)
        rc, stats, hist = P.hhg_stokes_solve(g.h, xf, bf, precision=prec, rtol=1e-8, max_iters=1000)
        xg = to_np(g.stokes_to_canonical(L, xf))
        err = np.abs(xg - xt).max() / scale
        log("  prec %d: iters %d (oracle %d), rel res %.2e, error vs tight solve %.2e, %.1f ms"
            % (prec, stats["iters"], len(ho) - 1, stats["rel_res"], err, stats["ms"]))
        assert rc == 0 and stats["converged"] == 1 and stats["rel_res"] <= 1e-8
        if prec == P.HHG_F64:
            eo = np.abs(xg - xo).max() / np.abs(xo).max()
            log("  FP64 solution against the oracle's 1e-8 solve: %.2e" % eo)
            assert stats["iters"] == len(ho) - 1 and eo <= 1e-8
        assert err <= 1e-5
        # velocity boundary data untouched, pressure mean (weighted) zero
        assert np.array_equal(xg[:st.N][st.dir], np.zeros(st.dir.sum()))
        assert abs(st.s @ xg[2 * st.N:]) <= 1e-9 * np.abs(st.s * xg[2 * st.N:]).sum()


def test_stokes_errors():
    import paper_1805_10167_amd as P
    vxy, tri = hi.mesh_by_name("annulus64")
    g = P.Mesh(vxy, tri, 3, 2, P.HHG_FEAT_F64)
    x, y = g.stokes_vector(3), g.stokes_vector(3)
    with pytest.raises(P.HHGError) as e:
        P.hhg_stokes_apply(g.h, 3, x, y)
    assert e.value.code == P.HHG_ENOMEM
    g3 = P.Mesh(vxy, tri, 3, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_STOKES)
    P.hhg_stokes_setup(g3.h, np.ones(len(tri)), 1.0 / 12.0)
    _, n_all = g3.n_dofs(3)
    canon = np.zeros(3 * n_all)
    canon[n_all - 1] = float("nan")          # u_x at the last face-interior point
    bad = g3.stokes_from_canonical(3, canon)
    rc, stats, _ = P.hhg_stokes_solve(g3.h, g3.stokes_vector(3), bad)
    assert rc == P.HHG_ENOTCONV and stats["converged"] == 0
    g2 = P.Mesh(vxy, tri, 3, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_STOKES)
    x, y = g2.stokes_vector(3), g2.stokes_vector(3)
    with pytest.raises(P.HHGError) as e:
        P.hhg_stokes_apply(g2.h, 3, x, y)      # before setup
    assert e.value.code == P.HHG_EINVAL
    P.hhg_stokes_setup(g2.h, np.ones(len(tri)), 1.0 / 12.0)
    with pytest.raises(P.HHGError):
        P.hhg_stokes_apply(g2.h, 3, x, x)
    with pytest.raises(P.HHGError):
        P.hhg_stokes_precond(g2.h, P.HHG_F32, x, y, 2, 2)   # no FP32 hierarchy
    with pytest.raises(P.HHGError):
        P.hhg_stokes_setup(g2.h, np.ones(len(tri)), 0.0)


def test_operator_and_solve_with_more_tiles_than_face_blocks():
    """Level 8 of the 64-face annulus has 10,560 face tiles, more than the
    8,192 face blocks of a launch, so the face blocks loop over tiles: the
    operator against the oracle's assembly element by element, and a MINRES
    solve that converges in the level-independent iteration count (about
    225 at levels 5-7)."""
    import torch

    import paper_1805_10167_amd as P
    from oracle import stokes as S
    from oracle.mesh import Level, MacroMesh
    L = 8
    vxy, tri = hi.mesh_by_name("annulus64")
    m = MacroMesh(vxy, tri)
    mu = S.face_viscosity(m)
    log("stokes operator annulus64 L=%d (face grid capped)" % L)
    lv = Level(m, L)
    blk = S.assemble_stokes(lv, mu)
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
    P.hhg_stokes_setup(g.h, mu, S.DELTA)
    N = lv.n_all
    x = hi.uniform_vector(3 * N, 21)
    x[:N][lv.dirichlet] = 0.0
    x[N:2 * N][lv.dirichlet] = 0.0
    y = g.stokes_vector(L)
    P.hhg_stokes_apply(g.h, L, g.stokes_from_canonical(L, x), y)
    ux, uy, p = x[:N], x[N:2 * N], x[2 * N:]
    ref = np.concatenate([blk["A"] @ ux + blk["Bx"].T @ p, blk["A"] @ uy + blk["By"].T @ p,
                          blk["Bx"] @ ux + blk["By"] @ uy - blk["C"] @ p])
    ref[:N][lv.dirichlet] = 0.0
    ref[N:2 * N][lv.dirichlet] = 0.0
    err = rel_err(to_np(g.stokes_to_canonical(L, y)), ref)
    log("  rel err %.2e" % err)
    assert err <= F64_TOL
    b = g.stokes_vector(L)
    P.hhg_stokes_apply(g.h, L, g.stokes_from_canonical(L, x), b)
    z = g.stokes_vector(L)
    rc, st, hist = P.hhg_stokes_solve(g.h, z, b, rtol=1e-8, max_iters=600)
    log("  MINRES: %d iterations, rel %.2e" % (st["iters"], st["rel_res"]))
    assert rc == 0 and st["iters"] <= 300
    r = g.stokes_vector(L)
    P.hhg_stokes_residual(g.h, L, z, b, r)
    d = torch.zeros(2, dtype=torch.float64, device="cuda")
    P.hhg_stokes_dot(g.h, L, r, r, d[0:1])
    P.hhg_stokes_dot(g.h, L, b, b, d[1:2])
    dd = d.cpu().numpy()
    assert np.sqrt(dd[0] / dd[1]) <= 1e-5
