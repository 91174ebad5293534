"""Every copy slot of every output equals the value it copies, bit for bit,
after each public operation (the explicit ghost-copy check of a partitioned
layout, sec. 2.2 and 3.3): the copy table of the level (hhg_ghost_table)
lists each face-ring, edge-end, edge-ghost-row and vertex-ring slot with its
owner.  Fields come from seeded uniform data on the jittered annulus."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import gpu_mesh, log

pytestmark = pytest.mark.gpu

L = 6


def consistent(g, level, fld):
    import paper_1805_10167_amd as P
    dst, src = P.hhg_ghost_table(g.h, level)
    a = fld.detach().cpu().numpy()
    bad = np.flatnonzero(a[dst] != a[src])
    return len(bad), len(dst)


@pytest.fixture(scope="module")
def mesh():
    import paper_1805_10167_amd as P
    from oracle import stokes as S
    g = gpu_mesh("annulus64", L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK | P.HHG_FEAT_STOKES)
    _, n_all = g.n_dofs(L)
    vxy, tri = hi.mesh_by_name("annulus64")
    import torch
    P.hhg_set_coefficient(g.h, torch.tensor(np.exp(0.5 * hi.uniform_vector(n_all, 9)), device="cuda"))
    P.hhg_stokes_setup(g.h, np.ones(len(tri)), S.DELTA)
    return g


def _ops(g):
    """(name, level, dtype, callable returning the output field)."""
    import torch

    import paper_1805_10167_amd as P
    _, n_all = g.n_dofs(L)
    x = g.from_canonical(L, hi.uniform_vector(n_all, 1))
    f = g.from_canonical(L, hi.uniform_vector(n_all, 2))
    x32 = g.from_canonical(L, hi.uniform_vector(n_all, 1), P.HHG_F32)
    f32 = g.from_canonical(L, hi.uniform_vector(n_all, 2), P.HHG_F32)
    F64, F32 = P.HHG_F64, P.HHG_F32
    LAP, DIF, MASS = P.HHG_OP_LAPLACE, P.HHG_OP_DIFFUSION, P.HHG_OP_MASS

    def run(fn, level=L, dt=F64):
        y = g.field(level, dt)
        fn(y)
        return y

    def smooth(op, dt, bwd):
        def fn(y):
            y.copy_(x if dt == F64 else x32)
            P.hhg_smooth(g.h, L, op, P.HHG_SMOOTH_GS, dt, y, f if dt == F64 else f32, 2, bwd)
        return fn

    def vcycle(op, dt):
        def fn(y):
            y.copy_(x if dt == F64 else x32)
            P.hhg_vcycle(g.h, L, op, P.HHG_SMOOTH_GS, dt, y, f if dt == F64 else f32, 3, 3)
        return fn

    def solve(mode):
        def fn(y):
            y.zero_()
            P.hhg_solve(g.h, y, f, mode=mode, rtol=1e-6, max_iters=20, history=False)
        return fn

    fs = P.hhg_field_elems(g.h, L)
    sx = g.stokes_from_canonical(L, np.concatenate([hi.uniform_vector(n_all, 5), hi.uniform_vector(n_all, 6),
                                                    hi.uniform_vector(n_all, 7)]))
    sb = g.stokes_from_canonical(L, np.concatenate([hi.uniform_vector(n_all, 8), hi.uniform_vector(n_all, 9),
                                                    hi.uniform_vector(n_all, 10)]))

    def stokes(call):
        def fn():
            y = g.stokes_vector(L)
            call(y)
            return [y[k * fs:(k + 1) * fs] for k in range(3)]
        return fn

    return [
        ("from_canonical", L, lambda: [x]),
        ("apply laplace f64", L, lambda: [run(lambda y: P.hhg_apply(g.h, L, LAP, F64, x, y))]),
        ("apply mass f64", L, lambda: [run(lambda y: P.hhg_apply(g.h, L, MASS, F64, x, y))]),
        ("apply diffusion f32", L, lambda: [run(lambda y: P.hhg_apply(g.h, L, DIF, F32, x32, y), dt=F32)]),
        ("residual f64", L, lambda: [run(lambda y: P.hhg_residual(g.h, L, LAP, F64, x, f, y))]),
        ("smooth forward f64", L, lambda: [run(smooth(LAP, F64, 0))]),
        ("smooth backward diffusion f64", L, lambda: [run(smooth(DIF, F64, 1))]),
        ("smooth forward f32", L, lambda: [run(smooth(LAP, F32, 0), dt=F32)]),
        ("vcycle f64", L, lambda: [run(vcycle(LAP, F64))]),
        ("vcycle diffusion f64", L, lambda: [run(vcycle(DIF, F64))]),
        ("vcycle f32", L, lambda: [run(vcycle(LAP, F32), dt=F32)]),
        ("jacobi", L, lambda: [run(lambda y: P.hhg_jacobi(g.h, L, LAP, F64, x, f, y))]),
        ("restrict", L - 1, lambda: [run(lambda y: P.hhg_restrict(g.h, L, F64, x, y), level=L - 1)]),
        ("prolong_add", L, lambda: [run(lambda y: (y.copy_(x), P.hhg_prolong_add(
            g.h, L, F64, g.from_canonical(L - 1, hi.uniform_vector(g.n_dofs(L - 1)[1], 3)), y)))]),
        ("axpby", L, lambda: [run(lambda y: P.hhg_axpby(g.h, L, F64, 0.5, x, -2.0, f, y))]),
        ("convert f64 -> f32", L, lambda: [run(lambda y: P.hhg_convert(g.h, L, F64, x, F32, y), dt=F32)]),
        ("solve plain", L, lambda: [run(solve(P.HHG_MODE_PLAIN_FP64))]),
        ("solve mixed precision", L, lambda: [run(solve(P.HHG_MODE_MP_IR))]),
        ("stokes apply", L, stokes(lambda y: P.hhg_stokes_apply(g.h, L, sx, y))),
        ("stokes residual", L, stokes(lambda y: P.hhg_stokes_residual(g.h, L, sx, sb, y))),
        ("stokes precond", L, stokes(lambda y: P.hhg_stokes_precond(g.h, P.HHG_F64, sb, y, 2, 2))),
        ("buoyancy", L, stokes(lambda y: P.hhg_buoyancy(g.h, L, torch.ones(2 * fs, dtype=torch.float64,
                                                                           device="cuda"), 2.0, y))),
    ]


def test_every_copy_matches_its_owner(mesh):
    g = mesh
    failures = []
    for name, level, fn in _ops(g):
        for k, fld in enumerate(fn()):
            nbad, ncopies = consistent(g, level, fld)
            log("%-32s field %d: %d of %d copies differ" % (name, k, nbad, ncopies))
            if nbad:
                failures.append((name, k, nbad))
    assert not failures, failures


def test_p2_outputs_are_consistent():
    import paper_1805_10167_amd as P
    l = 4
    g = gpu_mesh("annulus64", l + 1, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_P2)
    P.hhg_p2_setup(g.h)
    _, n_all = g.n_dofs(l + 1)
    x = g.from_canonical(l + 1, hi.uniform_vector(n_all, 11))
    f = g.from_canonical(l + 1, hi.uniform_vector(n_all, 12))
    outs = []
    for name, call in (("p2 apply", lambda y: P.hhg_p2_apply(g.h, l, x, y)),
                       ("p2 residual", lambda y: P.hhg_p2_residual(g.h, l, x, f, y)),
                       ("p2 jacobi", lambda y: P.hhg_p2_jacobi(g.h, l, 0.7, x, f, y)),
                       ("p2 solve", lambda y: P.hhg_p2_solve(g.h, l, y, f, rtol=1e-6, history=False))):
        y = g.field(l + 1)
        call(y)
        nbad, ncopies = consistent(g, l + 1, y)
        log("%-32s %d of %d copies differ" % (name, nbad, ncopies))
        outs.append(nbad)
    assert outs == [0, 0, 0, 0]
