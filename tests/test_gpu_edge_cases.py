"""Degenerate and boundary cases of the method on the GPU against the
oracle: a single macro-face (no interior edges or vertices), coarse level 1,
a cycle that is only the coarse solve, level 1 (faces without interior
points), zero right-hand sides, an iteration cap of zero, non-finite input, a
diverging solve (indefinite coefficient), and argument errors of the C
ABI."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import log, rel_err, to_np

pytestmark = pytest.mark.gpu
F64_TOL = 1e-12


def one_face():
    return np.array([[0.0, 0.0], [1.0, 0.2], [0.3, 0.9]]), np.array([[0, 1, 2]], dtype=np.int32)


def meshes(vxy, tri, L, lc):
    import paper_1805_10167_amd as P
    from oracle.mesh import MacroMesh
    from oracle.mg import Hierarchy
    g = P.Mesh(vxy, tri, L, lc, P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
    return g, Hierarchy(MacroMesh(vxy, tri), L, lc)


def fan16():
    """16 triangles around the origin: a degree-16 interior macro-vertex (the
    most the layout holds) where 16 interior macro-edges meet."""
    t = 2 * np.pi * np.arange(16) / 16
    vxy = np.vstack([[0.0, 0.0], np.c_[np.cos(t), np.sin(t)]])
    tri = np.array([[0, 1 + k, 1 + (k + 1) % 16] for k in range(16)], dtype=np.int32)
    return vxy, tri


@pytest.mark.parametrize("case", ["one_face_L4", "square_lc1_L3", "annulus_lc_eq_L", "square_L1", "fan16_L5"])
def test_vcycle_and_apply_degenerate_hierarchies(case):
    import paper_1805_10167_amd as P
    if case == "one_face_L4":
        (vxy, tri), L, lc = one_face(), 4, 2
    elif case == "square_lc1_L3":
        (vxy, tri), L, lc = hi.unit_square(), 3, 1
    elif case == "annulus_lc_eq_L":
        (vxy, tri), L, lc = hi.annulus(16), 3, 3
    elif case == "fan16_L5":
        (vxy, tri), L, lc = fan16(), 5, 2
    else:
        (vxy, tri), L, lc = hi.unit_square(), 1, 1
    log("degenerate hierarchy %s" % case)
    g, H = meshes(vxy, tri, L, lc)
    lv = H.levels[L]
    u, f = hi.uniform_vector(lv.n_all, 1), hi.uniform_vector(lv.n_all, 2)
    uf, ff, y = g.from_canonical(L, u), g.from_canonical(L, f), g.field(L)
    P.hhg_apply(g.h, L, P.HHG_OP_LAPLACE, P.HHG_F64, uf, y)
    ref = H.apply(L, u)
    ref[lv.dirichlet] = 0.0
    assert rel_err(to_np(g.to_canonical(L, y)), ref) <= F64_TOL
    P.hhg_vcycle(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, 2, 2)
    assert rel_err(to_np(g.to_canonical(L, uf)), H.vcycle(L, u.copy(), f, 2, 2)) <= F64_TOL
    if L > lc:
        uf = g.from_canonical(L, u)
        P.hhg_smooth(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, 2, 1)
        assert rel_err(to_np(g.to_canonical(L, uf)), H.smooth(L, u.copy(), f, 2, backward=True)) <= F64_TOL


def test_solve_zero_rhs_and_zero_iterations():
    import paper_1805_10167_amd as P
    g, H = meshes(*hi.annulus(16), 4, 2)
    L = 4
    u, f = g.field(L), g.field(L)
    for mode in (P.HHG_MODE_PLAIN_FP64, P.HHG_MODE_MP_IR):
        rc, st, hist = P.hhg_solve(g.h, u, f, mode=mode, rtol=1e-8)
        assert rc == 0 and st["iters"] == 0 and st["converged"] == 1 and hist == [0.0]
    f = g.from_canonical(L, hi.uniform_rhs(H.levels[L].n_all, 1))
    rc, st, _ = P.hhg_solve(g.h, u, f, rtol=1e-8, max_iters=0)
    assert rc == P.HHG_ENOTCONV and st["iters"] == 0
    assert not u.any()
    assert "cap" in P.hhg_last_error()


def test_non_finite_input_is_reported():
    import torch

    import paper_1805_10167_amd as P
    g, H = meshes(*hi.annulus(16), 4, 2)
    L = 4
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 1)
    f[np.flatnonzero(~lv.dirichlet)[7]] = np.nan
    u, ff = g.field(L), g.from_canonical(L, f)
    for mode in (P.HHG_MODE_PLAIN_FP64, P.HHG_MODE_MP_IR):
        u.zero_()
        rc, st, _ = P.hhg_solve(g.h, u, ff, mode=mode, rtol=1e-8, max_iters=5)
        log("nan input, mode %d: rc %d iters %d" % (mode, rc, st["iters"]))
        assert rc == P.HHG_ENOTCONV and st["converged"] == 0
        assert not np.isfinite(st["rel_res"]) or st["iters"] <= 1
    assert torch.isfinite(g.field(L)).all()


def test_argument_errors():
    import torch

    import paper_1805_10167_amd as P
    g, H = meshes(*hi.annulus(16), 3, 2)
    x, y = g.field(3), g.field(3)
    cases = [
        lambda: P.hhg_apply(g.h, 4, P.HHG_OP_LAPLACE, P.HHG_F64, x, y),        # level out of range
        lambda: P.hhg_apply(g.h, 3, P.HHG_OP_LAPLACE, 7, x, y),                # dtype
        lambda: P.hhg_apply(g.h, 3, P.HHG_OP_DIFFUSION, P.HHG_F64, x, y),      # no coefficient
        lambda: P.hhg_apply(g.h, 3, P.HHG_OP_LAPLACE, P.HHG_F64, x, x),        # aliasing
        lambda: P.hhg_vcycle(g.h, 1, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F64, x, y, 1, 1),
        lambda: P.hhg_smooth(g.h, 3, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_NET, P.HHG_F32, x, y, 1, 0),
        lambda: P.hhg_solve(g.h, x, y, mode=P.HHG_MODE_LEARNED),               # no NET workspace
        lambda: P.hhg_restrict(g.h, 1, P.HHG_F64, x, y),
        lambda: P.hhg_convert(g.h, 3, P.HHG_F32, x, P.HHG_F32, y),
        lambda: P.hhg_net_set_weights(g.h, np.zeros(224, np.float32)),          # no NET workspace
    ]
    for k, call in enumerate(cases):
        with pytest.raises(P.HHGError) as e:
            call()
        log("case %d: %s" % (k, P.hhg_last_error()))
        assert e.value.code in (P.HHG_EINVAL, P.HHG_ENOMEM)
    assert torch.equal(x, torch.zeros_like(x))


@pytest.mark.parametrize("case", ["square_L2_lc1", "annulus_L3_lc2", "one_face_L5"])
def test_solve_history_small_levels(case):
    """Residual histories of small-level solves equal the oracle's: the
    norm-forming sweep at n = 5 has no face-core points, and on one face all
    edges are Dirichlet."""
    import paper_1805_10167_amd as P
    if case == "square_L2_lc1":
        (vxy, tri), L, lc = hi.unit_square(), 2, 1
    elif case == "annulus_L3_lc2":
        (vxy, tri), L, lc = hi.annulus(16), 3, 2
    else:
        (vxy, tri), L, lc = one_face(), 5, 2
    g, H = meshes(vxy, tri, L, lc)
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 3)
    uf, ff = g.field(L), g.from_canonical(L, f)
    rc, st, hist = P.hhg_solve(g.h, uf, ff, rtol=1e-10, max_iters=60)
    uo, ho = H.solve(np.zeros(lv.n_all), f, 1e-10, 3, 3)
    log("%s: iters %d (oracle %d)" % (case, st["iters"], len(ho) - 1))
    assert rc == 0 and st["iters"] == len(ho) - 1
    assert rel_err(hist, ho) <= 1e-10
    assert rel_err(to_np(g.to_canonical(L, uf)), uo) <= F64_TOL


def test_solve_stops_when_the_residual_keeps_growing():
    """An indefinite operator: k = -0.3 on a seeded fifth of the points that
    only the finest level has (so the injected coarse coefficients, and the
    coarse operators, stay positive), k = 1 elsewhere.  Gauss-Seidel then
    diverges (the oracle's residuals: 1.0e2, 2.0e9, 1.5e18, 1.1e27), and the
    solve loop stops after three cycles of rising residual with
    HHG_ENOTCONV, before max_iters, its history finite and rising."""
    import torch

    import paper_1805_10167_amd as P
    from oracle.mesh import Level, MacroMesh
    L = 5
    vxy, tri = hi.mesh_by_name("annulus64")
    lv = Level(MacroMesh(vxy, tri), L)
    fine_only = (((lv.kind == 2) & ((lv.kidx % 2 == 1) | (lv.jidx % 2 == 1)))
                 | ((lv.kind == 1) & (lv.kidx % 2 == 1)))
    kap = np.where(fine_only & (hi.uniform_vector(lv.n_all, 1) > 0.6), -0.3, 1.0)
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_VARK)
    P.hhg_set_coefficient(g.h, torch.tensor(kap, device="cuda"))
    f = hi.uniform_vector(lv.n_all, 3)
    f[lv.dirichlet] = 0.0
    u = g.field(L)
    rc, st, hist = P.hhg_solve(g.h, u, g.from_canonical(L, f), op=P.HHG_OP_DIFFUSION, rtol=1e-8,
                               max_iters=30)
    log("diverging solve: rc %d, %d cycles, history %s, error %r" % (rc, st["iters"], hist,
                                                                   P.hhg_last_error()))
    assert rc == P.HHG_ENOTCONV
    assert "grew" in P.hhg_last_error()
    assert st["iters"] == 3 and st["converged"] == 0
    assert np.all(np.isfinite(hist)) and hist[1] < hist[2] < hist[3]
