"""Run-to-run determinism: every reduction in the library sums in a fixed
order (per-block trees, then one fixed-order final pass) and no kernel uses
floating-point atomics, so repeating a solve in one process gives the same
bits: iterate, residual history and iteration count."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import gpu_mesh, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["plain", "mp"])
@pytest.mark.parametrize("op", ["laplace", "diffusion"])
def test_solve_is_bitwise_repeatable(mode, op):
    import torch

    import paper_1805_10167_amd as P
    name, L = "annulus64", 7
    log("determinism %s %s" % (mode, op))
    g = gpu_mesh(name, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK)
    _, n_all = g.n_dofs(L)
    if op == "diffusion":
        xy = g.coords(L)
        P.hhg_set_coefficient(g.h, torch.tensor(np.exp(hi.grf_eval(xy, 3, m=64)),
                                                 dtype=torch.float64, device="cuda"))
    f = g.from_canonical(L, hi.uniform_rhs(n_all, 1))
    m = P.HHG_MODE_PLAIN_FP64 if mode == "plain" else P.HHG_MODE_MP_IR
    o = P.HHG_OP_LAPLACE if op == "laplace" else P.HHG_OP_DIFFUSION
    runs = []
    for _ in range(2):
        u = g.field(L)
        rc, st, hist = P.hhg_solve(g.h, u, f, mode=m, op=o, rtol=1e-8)
        assert rc == 0
        runs.append((u.clone(), st["iters"], np.asarray(hist)))
    (u1, i1, h1), (u2, i2, h2) = runs
    assert i1 == i2
    assert np.array_equal(h1, h2)
    assert torch.equal(u1, u2)
