"""Element-wise parity of the streamed FP32 face sweep against the oracle.

The plain FP32 sweep of the three-colour faces runs the streamed kernel on
levels with at least 4,096 smoother tiles (186 x 24 points); smaller levels
keep the tile kernel.  A 300-face annulus (50 sectors, 3 rings) at level 8
(257 points along a macro-edge, 9.9M unknowns) has 14 such tiles per face,
4,200 in all, so the streamed kernel runs on it; each face holds two strip
columns, so strips meet at their halos, and the hypotenuse cuts through
strip pieces.  A 100-face annulus (one ring) at level 9 (513 points, 13M
unknowns) has 42 tiles per face, 4,200 in all, in three strip columns, with
tiles that touch neither a macro-edge nor the diagonal.  Laplacian and
variable coefficient, forward and backward order, one and two sweeps, plus
an FP32 V(3,3) cycle on the level-8 mesh whose finest-level plain sweeps
are streamed.

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

MESHES = [(8, 3), (9, 1)]   # (level, rings of the 50-sector annulus)
N_TAN = 50
SWEEP_TOL = 2e-6
APPLY_TOL = 2e-5
_CACHE = {}


def tiles_per_face(n, ti_w=186, tj_h=24):
    """Smoother tiles of one face: origins (ti ti_w, tj tj_h) inside the
    triangle (the tile list of the halo-3 sweep)."""
    return sum(1 for ti in range(n) for tj in range(n) if ti * ti_w <= n - 1 and tj * tj_h <= n - 1
               and ti * ti_w + tj * tj_h <= n - 1)


def setup(op, L, n_rad):
    import torch

    import paper_1805_10167_amd as P
    from oracle.mesh import Level, MacroMesh
    from oracle.mg import Hierarchy
    key = (op, L, n_rad)
    if key not in _CACHE:
        _CACHE.clear()                      # one hierarchy at a time
        vxy, tri = hi.annulus(n_tan=N_TAN, n_rad=n_rad)
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
        _CACHE[key] = (g, H)
    return _CACHE[key]


def f32_vector(n, seed):
    return hi.uniform_vector(n, seed).astype(np.float32).astype(np.float64)


def _op(P, op):
    return P.HHG_OP_LAPLACE if op == "laplace" else P.HHG_OP_DIFFUSION


def test_levels_run_the_streamed_kernel():
    """Both meshes are above the streamed kernel's tile threshold."""
    assert tiles_per_face(2 ** 8 + 1) == 14 and tiles_per_face(2 ** 9 + 1) == 42
    for L, n_rad in MESHES:
        assert 2 * N_TAN * n_rad * tiles_per_face(2 ** L + 1) >= 4096


def test_streamed_vcycle():
    """On the level-8 mesh (collected before the sweeps, which reuse its
    hierarchy)."""
    import paper_1805_10167_amd as P
    L, n_rad = MESHES[0]
    log("FP32 V(3,3) with streamed finest-level sweeps, level %d rings %d" % (L, n_rad))
    g, H = setup("laplace", L, n_rad)
    lv = H.levels[L]
    u, f = f32_vector(lv.n_all, 13), f32_vector(lv.n_all, 14)
    uf, ff = g.from_canonical(L, u, P.HHG_F32), g.from_canonical(L, f, P.HHG_F32)
    P.hhg_vcycle(g.h, L, P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS, P.HHG_F32, uf, ff, 3, 3)
    err = rel_err(to_np(g.to_canonical(L, uf, P.HHG_F32)), H.vcycle(L, u.copy(), f, 3, 3))
    log("  rel err %.2e" % err)
    assert err <= F32_VCYCLE_TOL


# mesh by mesh and operator by operator, so that each hierarchy is built once
SWEEP_CASES = [(L, n_rad, op, bw, sw) for L, n_rad in MESHES for op in ("laplace", "diffusion")
               for bw, sw in ((0, 1), (1, 1), (0, 2), (1, 2))]


@pytest.mark.parametrize("L,n_rad,op,backward,sweeps", SWEEP_CASES)
def test_streamed_sweep(L, n_rad, op, backward, sweeps):
    import paper_1805_10167_amd as P
    log("streamed FP32 sweep level %d rings %d %s bwd=%d sweeps=%d" % (L, n_rad, op, backward, sweeps))
    g, H = setup(op, L, n_rad)
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
