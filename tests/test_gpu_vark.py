"""GPU parity of the variable-coefficient operator -div(k grad u), k = exp(g)
with g a seeded Gaussian random field evaluated at the oracle's canonical
coordinates; both sides receive the identical nodal k."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import F32_VCYCLE_TOL, MP_TOL, log, oracle_hierarchy, rel_err, to_np

pytestmark = pytest.mark.gpu
F64_TOL = 1e-12
KSEED = 7

_MESHES = {}


def mesh_k(name, L):
    import torch

    import paper_1805_10167_amd as P
    key = (name, L)
    if key not in _MESHES:
        feats = P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK
        vxy, tri = hi.mesh_by_name(name)
        g = P.Mesh(vxy, tri, L, 2, feats)
        H = oracle_hierarchy(name, L, 2, KSEED)
        k = torch.tensor(H.kappa[L], dtype=torch.float64, device="cuda")
        P.hhg_set_coefficient(g.h, k)
        _MESHES[key] = (g, H)
    return _MESHES[key]


CASES = [("annulus64", 4), ("annulus64", 6), ("annulus64", 7), ("square", 5)]


@pytest.mark.parametrize("name,L", CASES)
def test_diffusion_apply_and_residual(name, L):
    import paper_1805_10167_amd as P
    log("vark apply %s L=%d" % (name, L))
    g, H = mesh_k(name, L)
    for lvl in sorted({L, L - 1, 2}):
        lv = H.levels[lvl]
        x = hi.uniform_vector(lv.n_all, 20 + lvl)
        xf, y = g.from_canonical(lvl, x), g.field(lvl)
        P.hhg_apply(g.h, lvl, P.HHG_OP_DIFFUSION, P.HHG_F64, xf, y)
        assert rel_err(to_np(g.to_canonical(lvl, y)), H.apply(lvl, x)) <= F64_TOL
    lv = H.levels[L]
    u, f = hi.uniform_vector(lv.n_all, 1), hi.uniform_vector(lv.n_all, 2)
    uf, ff, r = g.from_canonical(L, u), g.from_canonical(L, f), g.field(L)
    P.hhg_residual(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_F64, uf, ff, r)
    ro = H.residual(L, u, f)
    assert rel_err(to_np(g.to_canonical(L, r)), ro) <= F64_TOL
    # every copy of r is consistent: A r through the library = A of canonical r
    y = g.field(L)
    P.hhg_apply(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_F64, r, y)
    assert rel_err(to_np(g.to_canonical(L, y)), H.apply(L, ro)) <= 1e-11


@pytest.mark.parametrize("name,L", CASES)
@pytest.mark.parametrize("backward", [0, 1])
def test_diffusion_smooth(name, L, backward):
    import paper_1805_10167_amd as P
    log("vark smooth %s L=%d bwd=%d" % (name, L, backward))
    g, H = mesh_k(name, L)
    lv = H.levels[L]
    u, f = hi.uniform_vector(lv.n_all, 3), hi.uniform_vector(lv.n_all, 4)
    uf, ff = g.from_canonical(L, u), g.from_canonical(L, f)
    P.hhg_smooth(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, 2, backward)
    assert rel_err(to_np(g.to_canonical(L, uf)), H.smooth(L, u.copy(), f, 2, bool(backward))) <= F64_TOL


@pytest.mark.parametrize("name,L", CASES)
def test_diffusion_vcycle(name, L):
    import paper_1805_10167_amd as P
    log("vark vcycle %s L=%d" % (name, L))
    g, H = mesh_k(name, L)
    lv = H.levels[L]
    u, f = hi.uniform_vector(lv.n_all, 5), hi.uniform_vector(lv.n_all, 6)
    uf, ff = g.from_canonical(L, u), g.from_canonical(L, f)
    P.hhg_vcycle(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_SMOOTH_GS, P.HHG_F64, uf, ff, 3, 3)
    assert rel_err(to_np(g.to_canonical(L, uf)), H.vcycle(L, u.copy(), f, 3, 3)) <= F64_TOL


def test_diffusion_solves_plain_and_mixed():
    import paper_1805_10167_amd as P
    name, L = "annulus64", 6
    log("vark solve %s L=%d" % (name, L))
    g, H = mesh_k(name, L)
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 1)
    uo, ho = H.solve(np.zeros(lv.n_all), f, 1e-8)
    uf, ff = g.from_canonical(L, np.zeros(lv.n_all)), g.from_canonical(L, f)
    rc, st, hist = P.hhg_solve(g.h, uf, ff, op=P.HHG_OP_DIFFUSION, rtol=1e-8)
    assert rc == 0 and st["iters"] == len(ho) - 1
    assert rel_err(hist, ho) <= 1e-10
    assert rel_err(to_np(g.to_canonical(L, uf)), uo) <= F64_TOL
    uref, _ = H.solve(np.zeros(lv.n_all), f, 1e-12)
    uf.zero_()
    rc, st, hist = P.hhg_solve(g.h, uf, ff, op=P.HHG_OP_DIFFUSION, mode=P.HHG_MODE_MP_IR, rtol=1e-8)
    assert rc == 0 and st["rel_res"] <= 1e-8
    err = rel_err(to_np(g.to_canonical(L, uf)), uref)
    log("vark mp iters %d error vs oracle %.2e" % (st["iters"], err))
    assert err <= MP_TOL


@pytest.mark.parametrize("name,L", [("annulus64", 6), ("square", 5)])
def test_diffusion_fp32_kernels(name, L):
    """FP32 variable-coefficient kernels (LDS coefficient tiles) against the
    FP64 oracle on FP32-representable inputs: apply, residual with and
    without the field, Jacobi scaling with and without f, forward and
    backward sweeps, and a V-cycle."""
    import torch

    import paper_1805_10167_amd as P
    from oracle import net as onet
    log("vark fp32 %s L=%d" % (name, L))
    g, H = mesh_k(name, L)
    lv = H.levels[L]
    F32, D = P.HHG_F32, P.HHG_OP_DIFFUSION

    def r32(v):
        return v.astype(np.float32).astype(np.float64)

    def back(x):
        return to_np(g.to_canonical(L, x, F32))

    u, f = r32(hi.uniform_vector(lv.n_all, 31)), r32(hi.uniform_vector(lv.n_all, 32))
    uf, ff, y = g.from_canonical(L, u, F32), g.from_canonical(L, f, F32), g.field(L, F32)
    P.hhg_apply(g.h, L, D, F32, uf, y)
    assert rel_err(back(y), H.apply(L, u)) <= 2e-5
    ro = H.residual(L, u, f)
    nrm = torch.zeros(2, dtype=torch.float64, device="cuda")
    P.hhg_residual(g.h, L, D, F32, uf, ff, y, nrm[0:1])
    assert rel_err(back(y), ro) <= 2e-5
    P.hhg_residual(g.h, L, D, F32, uf, ff, None, nrm[1:2])
    ref = np.linalg.norm(ro)
    assert abs(nrm[0].item() - ref) <= 2e-5 * ref and nrm[0].item() == nrm[1].item()
    P.hhg_jacobi(g.h, L, D, F32, uf, ff, y)
    assert rel_err(back(y), onet.jacobi_scale(H, L, ro)) <= 2e-5
    P.hhg_jacobi(g.h, L, D, F32, uf, None, y)
    assert rel_err(back(y), onet.jacobi_scale(H, L, u.copy())) <= 2e-5
    for backward in (0, 1):
        x = g.from_canonical(L, u, F32)
        P.hhg_smooth(g.h, L, D, P.HHG_SMOOTH_GS, F32, x, ff, 2, backward)
        assert rel_err(back(x), H.smooth(L, u.copy(), f, 2, bool(backward))) <= 2e-5
    x = g.from_canonical(L, u, F32)
    P.hhg_vcycle(g.h, L, D, P.HHG_SMOOTH_GS, F32, x, ff, 3, 3)
    err = rel_err(back(x), H.vcycle(L, u.copy(), f, 3, 3))
    log("fp32 vark V-cycle rel err %.2e" % err)
    assert err <= F32_VCYCLE_TOL
