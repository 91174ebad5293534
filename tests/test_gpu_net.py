"""GPU parity of the learned smoother's kernels against the FP64 oracle.

The FP32 instantiation of the same tile kernels is held to 1e-5 (FP32
rounding of sums of ~100 terms); the BF16 MFMA path (inputs and weights
rounded to BF16, relative precision 2^-8, FP32 accumulation) to 2e-2 in the
forward pass and 5e-2 for weight gradients, relative in the 2-norm."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import log, oracle_hierarchy, rel_err, to_np
from oracle import net as onet

pytestmark = pytest.mark.gpu
KSEED = 11
_MESHES = {}


def mesh_net(name, L):
    import torch

    import paper_1805_10167_amd as P
    key = (name, L)
    if key not in _MESHES:
        feats = P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK | P.HHG_FEAT_NET
        vxy, tri = hi.mesh_by_name(name)
        g = P.Mesh(vxy, tri, L, 2, feats)
        H = oracle_hierarchy(name, L, 2, KSEED)
        P.hhg_set_coefficient(g.h, torch.tensor(H.kappa[L], dtype=torch.float64, device="cuda"))
        _MESHES[key] = (g, H)
    return _MESHES[key]


def rel2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def random_weights(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, (16, 7)), rng.normal(0, scale, (16, 7))


CASES = [("annulus64", 5), ("annulus64", 7), ("square", 6), ("annulus128", 4)]


@pytest.mark.parametrize("name,L", CASES)
@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_net_forward(name, L, precision):
    import paper_1805_10167_amd as P
    log("net forward %s L=%d %s" % (name, L, precision))
    g, H = mesh_net(name, L)
    lv = H.levels[L]
    W1, W2 = random_weights(1)
    w32 = onet.pack(W1, W2).astype(np.float32)
    P.hhg_net_set_weights(g.h, w32)
    P.hhg_net_set_options(g.h, P.HHG_F32 if precision == "f32" else P.HHG_BF16, 0)
    rho = hi.uniform_vector(lv.n_all, 31).astype(np.float32).astype(np.float64)
    rf, out = g.from_canonical(L, rho, P.HHG_F32), g.field(L, P.HHG_F32)
    P.hhg_net_forward(g.h, L, rf, out)
    got = to_np(g.to_canonical(L, out, P.HHG_F32))
    W1r, W2r = onet.unpack(w32.astype(np.float64))
    ref = onet.forward(lv, rho, W1r, W2r)
    if precision == "f32":
        assert rel_err(got, ref) <= 1e-5
    else:
        assert rel2(got, ref) <= 2e-2
    # copies of out are consistent (out is 0 off the face interiors): the
    # library's Laplacian of out equals the oracle's Laplacian of canonical out
    y = g.field(L, P.HHG_F32)
    P.hhg_apply(g.h, L, P.HHG_OP_LAPLACE, P.HHG_F32, out, y)
    lap = oracle_hierarchy(name, L, 2).apply(L, got)
    assert rel_err(to_np(g.to_canonical(L, y, P.HHG_F32)), lap) <= 2e-5


@pytest.mark.parametrize("name,L", CASES)
@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_net_backward(name, L, precision):
    import torch

    import paper_1805_10167_amd as P
    log("net backward %s L=%d %s" % (name, L, precision))
    g, H = mesh_net(name, L)
    lv = H.levels[L]
    W1, W2 = random_weights(2)
    w32 = onet.pack(W1, W2).astype(np.float32)
    P.hhg_net_set_weights(g.h, w32)
    P.hhg_net_set_options(g.h, P.HHG_F32 if precision == "f32" else P.HHG_BF16, 0)
    rho = hi.uniform_vector(lv.n_all, 32).astype(np.float32).astype(np.float64)
    gr = hi.uniform_vector(lv.n_all, 33).astype(np.float32).astype(np.float64)
    gr[lv.kind != 2] = 0.0
    rf, gf = g.from_canonical(L, rho, P.HHG_F32), g.from_canonical(L, gr, P.HHG_F32)
    dW = torch.zeros(224, dtype=torch.float32, device="cuda")
    P.hhg_net_backward(g.h, L, rf, gf, dW)
    P.hhg_net_backward(g.h, L, rf, gf, dW)        # accumulates
    got = dW.cpu().numpy().astype(np.float64) / 2.0
    ref = onet.pack(*onet.backward(lv, rho, gr, *onet.unpack(w32.astype(np.float64))))
    if precision == "f32":
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    else:
        assert rel2(got, ref) <= 5e-2


def test_jacobi_dot_axpby():
    import torch

    import paper_1805_10167_amd as P
    name, L = "annulus64", 6
    g, H = mesh_net(name, L)
    lv = H.levels[L]
    u, f = hi.uniform_vector(lv.n_all, 1), hi.uniform_vector(lv.n_all, 2)
    uf, ff, rho = g.from_canonical(L, u), g.from_canonical(L, f), g.field(L)
    P.hhg_jacobi(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_F64, uf, ff, rho)
    ref = onet.jacobi_scale(H, L, H.residual(L, u, f))
    assert rel_err(to_np(g.to_canonical(L, rho)), ref) <= 1e-12
    P.hhg_jacobi(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_F64, uf, None, rho)
    assert rel_err(to_np(g.to_canonical(L, rho)), onet.jacobi_scale(H, L, u.copy())) <= 1e-12
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.hhg_dot(g.h, L, P.HHG_F64, uf, ff, out)
    ii = lv.interior
    assert abs(out.item() - u[ii] @ f[ii]) <= 1e-12 * np.abs(u[ii] * f[ii]).sum()
    z = g.field(L)
    P.hhg_axpby(g.h, L, P.HHG_F64, 2.0, uf, -0.5, ff, z)
    assert rel_err(to_np(g.to_canonical(L, z)), 2.0 * u - 0.5 * f) <= 1e-15


@pytest.mark.parametrize("precision,tol", [("f32", 2e-5), ("bf16", 1e-2)])
def test_net_smoother_with_jacobi_init(precision, tol):
    import paper_1805_10167_amd as P
    name, L = "annulus64", 6
    log("net smoother %s" % precision)
    g, H = mesh_net(name, L)
    lv = H.levels[L]
    W1, W2 = onet.jacobi_init()
    P.hhg_net_set_weights(g.h, onet.pack(W1, W2).astype(np.float32))
    P.hhg_net_set_options(g.h, P.HHG_F32 if precision == "f32" else P.HHG_BF16, 0)
    u, f = hi.uniform_vector(lv.n_all, 3), hi.uniform_vector(lv.n_all, 4)
    u32, f32 = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
    uf, ff = g.from_canonical(L, u32, P.HHG_F32), g.from_canonical(L, f32, P.HHG_F32)
    for backward in (0, 1):
        P.hhg_smooth(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_SMOOTH_NET, P.HHG_F32, uf, ff, 1, backward)
    got = to_np(g.to_canonical(L, uf, P.HHG_F32))
    ref = onet.net_smooth(H, L, u32.copy(), f32, W1, W2, 1, False)
    ref = onet.net_smooth(H, L, ref, f32, W1, W2, 1, True)
    assert rel_err(got, ref) <= tol


def test_adam_step_matches_oracle():
    import torch

    import paper_1805_10167_amd as P
    g, H = mesh_net("annulus64", 5)
    w0 = onet.pack(*random_weights(5)).astype(np.float32)
    P.hhg_net_set_weights(g.h, w0)
    rng = np.random.default_rng(6)
    w, m, v = w0.astype(np.float64), np.zeros(224), np.zeros(224)
    for step in (1, 2, 3):
        gr = rng.normal(0, 1, 224).astype(np.float32)
        P.hhg_net_adam_step(g.h, torch.tensor(gr, device="cuda"), 1e-2, step)
        w, m, v = onet.adam(w, gr.astype(np.float64), m, v, step, lr=1e-2)
    got = P.hhg_net_get_weights(g.h).astype(np.float64)
    assert np.abs(got - w).max() <= 1e-6


def test_learned_solve_rejection_and_guard():
    import paper_1805_10167_amd as P
    name, L = "annulus64", 6
    g, H = mesh_net(name, L)
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 1)
    ff = g.from_canonical(L, f)
    # not accepted: plain Gauss-Seidel inside the refinement loop
    P.hhg_net_set_weights(g.h, onet.pack(*onet.jacobi_init()).astype(np.float32))
    P.hhg_net_set_options(g.h, P.HHG_BF16, 0)
    uf = g.field(L)
    rc, st, _ = P.hhg_solve(g.h, uf, ff, mode=P.HHG_MODE_LEARNED, op=P.HHG_OP_DIFFUSION, rtol=1e-8)
    assert rc == 0 and st["fallback"] == 1 and st["smoother_used"] == P.HHG_SMOOTH_GS
    # accepted Jacobi-initialised network converges on its own
    P.hhg_net_set_options(g.h, P.HHG_BF16, 1)
    uf.zero_()
    rc, st, hist = P.hhg_solve(g.h, uf, ff, mode=P.HHG_MODE_LEARNED, op=P.HHG_OP_DIFFUSION,
                               rtol=1e-8, max_iters=200)
    log("jacobi-init learned solve: iters %d fallback %d" % (st["iters"], st["fallback"]))
    assert rc == 0 and st["rel_res"] <= 1e-8
    # a destructive network is dropped after its first bad cycle
    bad = onet.pack(*random_weights(9, scale=3.0)).astype(np.float32)
    P.hhg_net_set_weights(g.h, bad)
    P.hhg_net_set_options(g.h, P.HHG_BF16, 1)
    uf.zero_()
    rc, st, hist = P.hhg_solve(g.h, uf, ff, mode=P.HHG_MODE_LEARNED, op=P.HHG_OP_DIFFUSION,
                               rtol=1e-8, max_iters=200)
    log("bad-net solve: iters %d fallback %d" % (st["iters"], st["fallback"]))
    assert rc == 0 and st["fallback"] == 1 and st["rel_res"] <= 1e-8


# the fused step streams strip pieces of 8 rows below level 9, 16 at level 9
# and 32 from level 10: the unit square at levels 9 and 10 (0.26M and 1M
# unknowns) reaches the taller pieces within the oracle's reach
SWEEP_CASES = CASES + [("square", 9), ("square", 10)]


@pytest.mark.parametrize("name,L", SWEEP_CASES)
@pytest.mark.parametrize("precision", ["f32", "bf16"])
@pytest.mark.parametrize("backward", [0, 1])
def test_net_smoother_with_random_weights(name, L, precision, backward):
    """The production learned sweep (hhg_smooth with HHG_SMOOTH_NET: edge
    and vertex stages, the fused face step that forms rho = D^-1 (f - A u)
    in its tile, runs the network and adds its output) against the oracle's
    net_smooth, with seeded random weights on all 7 taps of all 16 channels,
    so every tap offset, channel and the rho ring reach the output.  FP32
    arithmetic of the same kernels: 1e-5; BF16 MFMA operands: the increment
    u_new - u within 2e-2 in the 2-norm (the forward bound)."""
    import paper_1805_10167_amd as P
    log("net smoother random weights %s L=%d %s bwd=%d" % (name, L, precision, backward))
    g, H = mesh_net(name, L)
    lv = H.levels[L]
    W1, W2 = random_weights(4, scale=0.3)
    w32 = onet.pack(W1, W2).astype(np.float32)
    W1r, W2r = onet.unpack(w32.astype(np.float64))
    assert (W1r != 0).all() and (W2r != 0).all()
    P.hhg_net_set_weights(g.h, w32)
    P.hhg_net_set_options(g.h, P.HHG_F32 if precision == "f32" else P.HHG_BF16, 0)
    u = hi.uniform_vector(lv.n_all, 41).astype(np.float32).astype(np.float64)
    f = hi.uniform_vector(lv.n_all, 42).astype(np.float32).astype(np.float64)
    uf, ff = g.from_canonical(L, u, P.HHG_F32), g.from_canonical(L, f, P.HHG_F32)
    P.hhg_smooth(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_SMOOTH_NET, P.HHG_F32, uf, ff, 1, backward)
    got = to_np(g.to_canonical(L, uf, P.HHG_F32))
    ref = onet.net_smooth(H, L, u.copy(), f, W1r, W2r, 1, bool(backward))
    inc = rel2(got - u, ref - u)
    log("  max rel %.2e  increment rel2 %.2e" % (rel_err(got, ref), inc))
    if precision == "f32":
        assert rel_err(got, ref) <= 1e-5 and inc <= 1e-5
    else:
        assert inc <= 2e-2
    assert np.array_equal(got[lv.dirichlet], u[lv.dirichlet])
    # copies are consistent: the library's operator on the result equals the
    # oracle's operator on its canonical values
    y = g.field(L, P.HHG_F32)
    P.hhg_apply(g.h, L, P.HHG_OP_DIFFUSION, P.HHG_F32, uf, y)
    assert rel_err(to_np(g.to_canonical(L, y, P.HHG_F32)), H.apply(L, got)) <= 2e-5
