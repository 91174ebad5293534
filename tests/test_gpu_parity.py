"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

FP64 results must match the oracle to 1e-12 relative (max-norm); FP32
kernels are compared with the FP64 oracle to bounds derived from FP32
rounding (unit roundoff 6e-8 times a small growth factor of the stencil sums
and sweeps).  Inputs are seeded and synthetic: uniform random vectors on the
unit square and the jittered 64/128-face annulus."""
import numpy as np
import pytest

import hhg_inputs as hi
import gpu_util
from gpu_util import gpu_mesh, log, oracle_hierarchy, rel_err, to_np

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_VCYCLE_TOL, MP_TOL = gpu_util.F32_VCYCLE_TOL, gpu_util.MP_TOL
CASES = [("square", 5), ("annulus64", 4), ("annulus64", 6), ("annulus128", 4)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1805_10167_amd as P
    P.lib()


_MESHES = {}


def mesh(name, L, features=None):
    import paper_1805_10167_amd as P
    features = features or (P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
    key = (name, L, features)
    if key not in _MESHES:
        _MESHES[key] = gpu_mesh(name, L, 2, features)
    return _MESHES[key]


def canon_vec(lv, seed, dirichlet_zero=False):
    x = hi.uniform_vector(lv.n_all, seed)
    if dirichlet_zero:
        x[lv.dirichlet] = 0.0
    return x


@pytest.mark.parametrize("name,L", CASES)
def test_canonical_roundtrip(name, L):
    import paper_1805_10167_amd as P
    log("roundtrip %s L=%d" % (name, L))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    x = canon_vec(H.levels[L], 11)
    for dt in (P.HHG_F64, P.HHG_F32):
        f = g.from_canonical(L, x, dt)
        y = to_np(g.to_canonical(L, f, dt))
        ref = x if dt == P.HHG_F64 else x.astype(np.float32).astype(np.float64)
        assert np.array_equal(y, ref)


@pytest.mark.parametrize("name,L", CASES)
@pytest.mark.parametrize("op", ["A", "M"])
def test_apply_parity(name, L, op):
    import paper_1805_10167_amd as P
    log("apply %s L=%d op=%s" % (name, L, op))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    for lvl in sorted({L, L - 1, 2}):
        lv = H.levels[lvl]
        x = canon_vec(lv, 100 + lvl)
        xf = g.from_canonical(lvl, x)
        y = g.field(lvl)
        P.hhg_apply(g.h, lvl, P.HHG_OP_LAPLACE if op == "A" else P.HHG_OP_MASS, P.HHG_F64, xf, y)
        yg = to_np(g.to_canonical(lvl, y))
        assert rel_err(yg, H.apply(lvl, x, op)) <= F64_TOL


@pytest.mark.parametrize("name,L", CASES)
def test_residual_and_norm(name, L):
    import torch

    import paper_1805_10167_amd as P
    log("residual %s L=%d" % (name, L))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    lv = H.levels[L]
    u, f = canon_vec(lv, 1), canon_vec(lv, 2)
    uf, ff, r = g.from_canonical(L, u), g.from_canonical(L, f), g.field(L)
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.hhg_residual(g.h, L, P.HHG_OP_LAPLACE, P.HHG_F64, uf, ff, r, nrm)
    ro = H.residual(L, u, f)
    assert rel_err(to_np(g.to_canonical(L, r)), ro) <= F64_TOL
    assert abs(nrm.item() - np.linalg.norm(ro)) <= F64_TOL * np.linalg.norm(ro)
    # norm only: no residual field
    nrm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.hhg_residual(g.h, L, P.HHG_OP_LAPLACE, P.HHG_F64, uf, ff, None, nrm2)
    assert abs(nrm2.item() - np.linalg.norm(ro)) <= F64_TOL * np.linalg.norm(ro)


@pytest.mark.parametrize("name,L", CASES + [("annulus64", 7), ("square", 7)])
@pytest.mark.parametrize("backward,sweeps", [(0, 1), (1, 1), (0, 2), (1, 3)])
def test_smooth_parity(name, L, backward, sweeps):
    import paper_1805_10167_amd as P
    log("smooth %s L=%d bwd=%d sweeps=%d" % (name, L, backward, sweeps))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    lv = H.levels[L]
    u, f = canon_vec(lv, 3), canon_vec(lv, 4)
    uf, ff = g.from_canonical(L, u), g.from_canonical(L, f)
    P.hhg_smooth(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, sweeps, backward)
    ug = to_np(g.to_canonical(L, uf))
    uo = H.smooth(L, u.copy(), f, sweeps, backward=bool(backward))
    assert rel_err(ug, uo) <= F64_TOL
    # ghost copies stay consistent: A u through the library equals the
    # oracle's A applied to the canonical result
    y = g.field(L)
    P.hhg_apply(g.h, L, P.HHG_OP_LAPLACE, P.HHG_F64, uf, y)
    assert rel_err(to_np(g.to_canonical(L, y)), H.apply(L, ug)) <= F64_TOL


@pytest.mark.parametrize("name,L,nu", [("square", 5, (2, 2)), ("annulus64", 4, (1, 1)),
                                       ("annulus64", 6, (3, 3)), ("annulus128", 4, (3, 3)),
                                       ("annulus64", 6, (2, 0)), ("annulus64", 7, (3, 3)),
                                       ("annulus128", 7, (1, 2)), ("annulus64", 5, (0, 2))])
def test_vcycle_parity(name, L, nu):
    _vcycle_parity(name, L, nu, 2)


@pytest.mark.parametrize("name,L,lc,coarse", [("annulus64", 6, 3, "direct"), ("square", 6, 3, "direct"),
                                              ("annulus64", 5, 4, "pcg")])
def test_vcycle_parity_other_coarse_levels(name, L, lc, coarse):
    """The coarsest level is a parameter (sec. 4.3 fixes none).  Level 3 of
    the annulus (1,920 coarse unknowns) still takes the stored inverse; level
    4 (7,936) exceeds it and the library falls back to Jacobi-PCG, compared
    with the oracle's PCG option."""
    _vcycle_parity(name, L, (3, 3), lc, coarse)


def _vcycle_parity(name, L, nu, lc, coarse="direct"):
    import paper_1805_10167_amd as P
    from oracle.mesh import MacroMesh
    from oracle.mg import Hierarchy
    log("vcycle %s L=%d nu=%s lc=%d" % (name, L, nu, lc))
    g = mesh(name, L) if lc == 2 else gpu_mesh(name, L, lc, P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
    H = (oracle_hierarchy(name, L, lc) if coarse == "direct"
         else Hierarchy(MacroMesh(*hi.mesh_by_name(name)), L, lc, coarse="pcg"))
    lv = H.levels[L]
    u, f = canon_vec(lv, 5), canon_vec(lv, 6)
    uf, ff = g.from_canonical(L, u), g.from_canonical(L, f)
    P.hhg_vcycle(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, *nu)
    ug = to_np(g.to_canonical(L, uf))
    uo = H.vcycle(L, u.copy(), f, *nu)
    assert rel_err(ug, uo) <= F64_TOL
    # Dirichlet values are read, never written
    assert np.array_equal(ug[lv.dirichlet], u[lv.dirichlet])


_L8 = {}


@pytest.mark.parametrize("op,dtype", [("laplace", "f64"), ("laplace", "f32"), ("diffusion", "f64")])
def test_vcycle_parity_several_tile_columns(op, dtype):
    """Level 8 of the 64-face annulus (257 points along a macro-edge).  The
    smoother tiles (182 x 22 or 182 x 16 interior points in the sweep that
    restricts its residual, 186 x 24 or 186 x 16 otherwise) span two columns
    and up to seventeen rows per face with ragged last ones, so coarse points
    next to every kind of tile border are restricted inside the sweep.  FP64
    to 1e-12; FP32 on FP32-representable inputs within 1e-4, as at smaller
    sizes.  The variable coefficient is the seeded random field of the
    other variable-coefficient tests."""
    import torch

    import paper_1805_10167_amd as P
    L = 8
    log("vcycle several tile columns %s %s L=%d" % (op, dtype, L))
    if op not in _L8:
        ks = 7 if op == "diffusion" else None
        H = oracle_hierarchy("annulus64", L, 2, ks)
        g = gpu_mesh("annulus64", L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK)
        if ks is not None:
            P.hhg_set_coefficient(g.h, torch.tensor(H.kappa[L], dtype=torch.float64, device="cuda"))
        _L8[op] = (g, H)
    g, H = _L8[op]
    lv = H.levels[L]
    dt = P.HHG_F64 if dtype == "f64" else P.HHG_F32
    cast = (lambda x: x) if dtype == "f64" else (lambda x: x.astype(np.float32).astype(np.float64))
    u, f = cast(canon_vec(lv, 5)), cast(canon_vec(lv, 6))
    uf, ff = g.from_canonical(L, u, dt), g.from_canonical(L, f, dt)
    opc = P.HHG_OP_LAPLACE if op == "laplace" else P.HHG_OP_DIFFUSION
    P.hhg_vcycle(g.h, L, opc, P.HHG_SMOOTH_GS, dt, uf, ff, 3, 3)
    err = rel_err(to_np(g.to_canonical(L, uf, dt)), H.vcycle(L, u.copy(), f, 3, 3))
    log("  rel err %.2e" % err)
    assert err <= (F64_TOL if dtype == "f64" else F32_VCYCLE_TOL)


@pytest.mark.parametrize("name,L,nu,rtol", [("annulus64", 6, (3, 3), 1e-8),
                                            ("square", 6, (2, 2), 1e-10),
                                            ("square", 5, (1, 1), 1e-8),
                                            ("annulus64", 5, (1, 2), 1e-9)])
def test_solve_parity(name, L, nu, rtol):
    import paper_1805_10167_amd as P
    log("solve %s L=%d" % (name, L))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 1)
    u0 = np.zeros(lv.n_all)
    uf, ff = g.from_canonical(L, u0), g.from_canonical(L, f)
    rc, st, hist = P.hhg_solve(g.h, uf, ff, rtol=rtol, nu1=nu[0], nu2=nu[1])
    assert rc == 0 and st["converged"] == 1
    uo, ho = H.solve(u0.copy(), f, rtol, *nu)
    assert st["iters"] == len(ho) - 1
    assert rel_err(hist, ho) <= 1e-10
    assert rel_err(to_np(g.to_canonical(L, uf)), uo) <= F64_TOL
    assert st["rel_res"] <= rtol


@pytest.mark.parametrize("name,L", [("annulus64", 6), ("square", 5)])
def test_fp32_kernels_within_bounds(name, L):
    import paper_1805_10167_amd as P
    log("fp32 %s L=%d" % (name, L))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    lv = H.levels[L]
    x, f = canon_vec(lv, 7), canon_vec(lv, 8)
    F32 = P.HHG_F32
    xf, ff = g.from_canonical(L, x, F32), g.from_canonical(L, f, F32)
    y = g.field(L, F32)
    P.hhg_apply(g.h, L, P.HHG_OP_LAPLACE, F32, xf, y)
    assert rel_err(to_np(g.to_canonical(L, y, F32)), H.apply(L, x)) <= 2e-5
    P.hhg_smooth(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, F32, xf, ff, 1, 0)
    assert rel_err(to_np(g.to_canonical(L, xf, F32)), H.smooth(L, x.copy(), f, 1)) <= 2e-5
    x2 = canon_vec(lv, 9)
    xf = g.from_canonical(L, x2, F32)
    P.hhg_vcycle(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, F32, xf, ff, 3, 3)
    err = rel_err(to_np(g.to_canonical(L, xf, F32)), H.vcycle(L, x2.copy(), f, 3, 3))
    log("  fp32 V-cycle rel err %.2e" % err)
    assert err <= F32_VCYCLE_TOL


def test_mixed_precision_solve_reaches_fp64_tolerance():
    import paper_1805_10167_amd as P
    name, L = "annulus64", 6
    log("mp solve %s L=%d" % (name, L))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 1)
    uf, ff = g.from_canonical(L, np.zeros(lv.n_all)), g.from_canonical(L, f)
    rc, st, hist = P.hhg_solve(g.h, uf, ff, mode=P.HHG_MODE_MP_IR, rtol=1e-8)
    assert rc == 0 and st["converged"] == 1 and st["rel_res"] <= 1e-8
    uo, _ = H.solve(np.zeros(lv.n_all), f, 1e-12)
    err = rel_err(to_np(g.to_canonical(L, uf)), uo)
    log("mp iters %d final error vs oracle %.3e" % (st["iters"], err))
    assert err <= MP_TOL


@pytest.mark.parametrize("name,L", CASES + [("annulus64", 7)])
def test_restrict_and_prolong_parity(name, L):
    """hhg_restrict (P^T r, zero at coarse Dirichlet points) and
    hhg_prolong_add (u += P uc at interior points) against the oracle, for
    both precisions, with consistent copies in the outputs."""
    import paper_1805_10167_amd as P
    log("restrict/prolong %s L=%d" % (name, L))
    g = mesh(name, L)
    H = oracle_hierarchy(name, L, 2)
    lv, lc = H.levels[L], H.levels[L - 1]
    r = canon_vec(lv, 21, dirichlet_zero=True)
    u, uc = canon_vec(lv, 22), canon_vec(lc, 23)
    for dt, tol in ((P.HHG_F64, F64_TOL), (P.HHG_F32, 2e-6)):
        cast = (lambda x: x) if dt == P.HHG_F64 else (lambda x: x.astype(np.float32).astype(np.float64))
        rf, fc = g.from_canonical(L, cast(r), dt), g.field(L - 1, dt)
        P.hhg_restrict(g.h, L, dt, rf, fc)
        assert rel_err(to_np(g.to_canonical(L - 1, fc, dt)), H.restrict(L, cast(r))) <= tol
        uf, ucf = g.from_canonical(L, cast(u), dt), g.from_canonical(L - 1, cast(uc), dt)
        P.hhg_prolong_add(g.h, L, dt, ucf, uf)
        ug = to_np(g.to_canonical(L, uf, dt))
        assert rel_err(ug, H.prolong_add(L, cast(u).copy(), cast(uc))) <= tol
        # the output's copies are consistent: applying the operator to it
        # through the library equals the oracle's operator on the canonical values
        y = g.field(L, dt)
        P.hhg_apply(g.h, L, P.HHG_OP_LAPLACE, dt, uf, y)
        assert rel_err(to_np(g.to_canonical(L, y, dt)), H.apply(L, ug)) <= 10 * tol
    with pytest.raises(P.HHGError):
        P.hhg_restrict(g.h, 1, P.HHG_F64, rf, fc)


def test_convert_roundtrip():
    import torch

    import paper_1805_10167_amd as P
    g = mesh("annulus64", 4)
    H = oracle_hierarchy("annulus64", 4, 2)
    x = canon_vec(H.levels[4], 31)
    x64 = g.from_canonical(4, x)
    x32 = g.field(4, P.HHG_F32)
    P.hhg_convert(g.h, 4, P.HHG_F64, x64, P.HHG_F32, x32)
    assert torch.equal(x32, x64.float())
    back = g.field(4)
    P.hhg_convert(g.h, 4, P.HHG_F32, x32, P.HHG_F64, back)
    assert torch.equal(back, x32.double())
    with pytest.raises(P.HHGError):
        P.hhg_convert(g.h, 4, P.HHG_F64, x64, P.HHG_F64, back)
