"""Element-wise parity of the streamed FP32 face sweep against the oracle.

The plain FP32 sweep of the three-colour faces runs the streamed kernel on
levels with at least 4,096 smoother tiles (186 x 24 points); smaller levels
keep the tile kernel.  A 300-face annulus (50 sectors, 3 rings) at level 8
(257 points along a macro-edge, 9.9M unknowns) has 14 such tiles per face,
4,200 in all, so the streamed kernel runs on it; each face holds two strip
columns, so strips meet at their halos, and the hypotenuse cuts through
strip pieces.  Laplacian and variable coefficient, forward and backward
order, one and two sweeps, plus an FP32 V(3,3) cycle whose finest-level
plain sweeps are streamed.

Inputs are FP32-representable, so only the kernel's FP32 arithmetic differs
from the oracle's FP64.  A point update rounds a sum of seven products and a
scaling, and the three colour stages of two sweeps chain such updates, so
the result carries about 30 FP32 unit roundoffs (2^-24 = 6e-8): 2e-6
relative in the max norm (the measured errors are 1.5e-7 to 3.1e-7).  The
operator applied to the result in FP32 loses digits to cancellation, as in
the tile kernel's FP32 test: 2e-5.  The V-cycle takes the FP32 V-cycle
bound."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import F32_VCYCLE_TOL, log, rel_err, to_np

pytestmark = pytest.mark.gpu

L = 8
N_TAN, N_RAD = 50, 3
SWEEP_TOL = 2e-6
APPLY_TOL = 2e-5
_CACHE = {}


def tiles_per_face(n, ti_w=186, tj_h=24):
    """Smoother tiles of one face: origins (ti ti_w, tj tj_h) inside the
    triangle (the tile list of the halo-3 sweep)."""
    return sum(1 for ti in range(n) for tj in range(n) if ti * ti_w <= n - 1 and tj * tj_h <= n - 1
               and ti * ti_w + tj * tj_h <= n - 1)


def setup(op):
    import torch

    import paper_1805_10167_amd as P
    from oracle.mesh import Level, MacroMesh
    from oracle.mg import Hierarchy
    if op not in _CACHE:
        vxy, tri = hi.annulus(n_tan=N_TAN, n_rad=N_RAD)
        m = MacroMesh(vxy, tri)
        kap = None
        if op == "diffusion":
            kap = np.exp(hi.grf_eval(Level(m, L).xy, 8, m=64))
        log("streamed-sweep oracle hierarchy (%s, %d faces, level %d)" % (op, m.F, L))
        H = Hierarchy(m, L, 2, kap)
        feats = P.HHG_FEAT_F64 | P.HHG_FEAT_MP | (P.HHG_FEAT_VARK if kap is not None else 0)
        g = P.Mesh(vxy, tri, L, 2, feats)
        if kap is not None:
            P.hhg_set_coefficient(g.h, torch.tensor(kap, dtype=torch.float64, device="cuda"))
        _CACHE[op] = (g, H)
    return _CACHE[op]


def f32_vector(n, seed):
    return hi.uniform_vector(n, seed).astype(np.float32).astype(np.float64)


def _op(P, op):
    return P.HHG_OP_LAPLACE if op == "laplace" else P.HHG_OP_DIFFUSION


def test_level_runs_the_streamed_kernel():
    """The mesh is above the streamed kernel's tile threshold."""
    n = 2 ** L + 1
    assert tiles_per_face(n) == 14
    assert 2 * N_TAN * N_RAD * tiles_per_face(n) >= 4096


@pytest.mark.parametrize("op", ["laplace", "diffusion"])
@pytest.mark.parametrize("backward,sweeps", [(0, 1), (1, 1), (0, 2), (1, 2)])
def test_streamed_sweep(op, backward, sweeps):
    import paper_1805_10167_amd as P
    log("streamed FP32 sweep %s bwd=%d sweeps=%d" % (op, backward, sweeps))
    g, H = setup(op)
    lv = H.levels[L]
    u, f = f32_vector(lv.n_all, 11), f32_vector(lv.n_all, 12)
    uf, ff = g.from_canonical(L, u, P.HHG_F32), g.from_canonical(L, f, P.HHG_F32)
    P.hhg_smooth(g.h, L, _op(P, op), P.HHG_SMOOTH_GS, P.HHG_F32, uf, ff, sweeps, backward)
    got = to_np(g.to_canonical(L, uf, P.HHG_F32))
    ref = H.smooth(L, u.copy(), f, sweeps, backward=bool(backward))
    err = rel_err(got, ref)
    log("  rel err %.2e" % err)
    assert err <= SWEEP_TOL
    assert np.array_equal(got[lv.dirichlet], u[lv.dirichlet])
    # the copies are consistent: the operator on the result (which reads the
    # ghost rows) equals the oracle's operator on the canonical values
    y = g.field(L, P.HHG_F32)
    P.hhg_apply(g.h, L, _op(P, op), P.HHG_F32, uf, y)
    assert rel_err(to_np(g.to_canonical(L, y, P.HHG_F32)), H.apply(L, got)) <= APPLY_TOL


def test_streamed_vcycle():
    import paper_1805_10167_amd as P
    log("FP32 V(3,3) with streamed finest-level sweeps")
    g, H = setup("laplace")
    lv = H.levels[L]
    u, f = f32_vector(lv.n_all, 13), f32_vector(lv.n_all, 14)
    uf, ff = g.from_canonical(L, u, P.HHG_F32), g.from_canonical(L, f, P.HHG_F32)
    P.hhg_vcycle(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F32, uf, ff, 3, 3)
    err = rel_err(to_np(g.to_canonical(L, uf, P.HHG_F32)), H.vcycle(L, u.copy(), f, 3, 3))
    log("  rel err %.2e" % err)
    assert err <= F32_VCYCLE_TOL
