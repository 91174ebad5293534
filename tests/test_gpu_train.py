"""GPU tests of the learned smoother's training harness: captured pairs and
the composed training gradient against the FP64 oracle, then a short
training run with the acceptance rule and the gain over the Jacobi-initialised
network (the trained network itself has no oracle: parity unpinned)."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import log, oracle_hierarchy, rel_err, to_np
from oracle import net as onet

pytestmark = pytest.mark.gpu
NAME = "annulus64"


def make_mesh(L):
    import paper_1805_10167_amd as P
    vxy, tri = hi.mesh_by_name(NAME)
    feats = P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK | P.HHG_FEAT_NET
    return P.Mesh(vxy, tri, L, 2, feats)


def kappa_dev(g, L, seed):
    import torch
    return torch.tensor(np.exp(hi.grf_eval(g.coords(L), seed)), dtype=torch.float64,
                        device="cuda")


def test_capture_pairs_match_oracle():
    from paper_1805_10167_amd import train
    L, seed = 5, 3
    g = make_mesh(L)
    H = oracle_hierarchy(NAME, L, 2, seed)
    lv = H.levels[L]
    f = hi.uniform_rhs(lv.n_all, 1000 + seed)
    ps = train.capture_pairs(g, [kappa_dev(g, L, seed)], [f], cycles=4)
    ustar, _ = H.solve(np.zeros(lv.n_all), f, rtol=1e-13)
    u = np.zeros(lv.n_all)
    import paper_1805_10167_amd as P
    for c in range(4):
        r = H.residual(L, u, f)
        e = ustar - u
        got_r = to_np(g.to_canonical(L, ps.r[c], P.HHG_F32))
        got_e = to_np(g.to_canonical(L, ps.e[c], P.HHG_F32))
        log("cycle %d: r %.2e e %.2e" % (c, rel_err(got_r, r), rel_err(got_e, e)))
        assert rel_err(got_r, r) <= 1e-6
        assert rel_err(got_e, e) <= 1e-6
        assert abs(ps.energy[c] - e @ r) <= 1e-9 * abs(e @ r)
        H.vcycle(L, u, f, 3, 3)
    assert list(ps.sample) == [0, 0, 0, 0]


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_training_gradient_matches_oracle(precision):
    """One pair through the library's Jacobi scaling, forward, axpby,
    operator, dot and backward equals the oracle's loss and gradient."""
    import torch

    import paper_1805_10167_amd as P
    from paper_1805_10167_amd import train
    L, seed = 5, 11
    g = make_mesh(L)
    H = oracle_hierarchy(NAME, L, 2, seed)
    lv = H.levels[L]
    rng = np.random.default_rng(7)
    e = rng.standard_normal(lv.n_all)
    e[lv.dirichlet] = 0.0
    r = H.apply(L, e) + 0.1 * rng.standard_normal(lv.n_all)   # any residual works
    r[lv.dirichlet] = 0.0
    r32 = r.astype(np.float32).astype(np.float64)
    e32 = e.astype(np.float32).astype(np.float64)
    W1, W2 = rng.normal(0, 0.5, (16, 7)), rng.normal(0, 0.5, (16, 7))
    w32 = onet.pack(W1, W2).astype(np.float32)
    P.hhg_net_set_weights(g.h, w32)
    E0 = float(e32 @ r32)
    R = g.from_canonical(L, r32, P.HHG_F32).reshape(1, -1)
    E = g.from_canonical(L, e32, P.HHG_F32).reshape(1, -1)
    ps = train.PairSet(g, [kappa_dev(g, L, seed)], R, E, np.zeros(1, dtype=int), np.array([E0]))
    prec = P.HHG_F32 if precision == "f32" else P.HHG_BF16
    tr = train.Trainer(ps, precision=prec)
    loss = tr.gradient([0])[0]
    got = tr.dW.cpu().numpy().astype(np.float64)
    Lref, dW1, dW2 = onet.loss_and_grad(H, L, r32, e32, *onet.unpack(w32.astype(np.float64)))
    ref = onet.pack(dW1, dW2)
    log("%s: loss %.6f vs %.6f, grad rel %.2e" % (precision, loss, Lref, rel_err(got, ref)))
    if precision == "f32":
        assert abs(loss - Lref) <= 1e-5 * abs(Lref)
        assert rel_err(got, ref) <= 1e-4
    else:
        assert abs(loss - Lref) <= 2e-2 * abs(Lref)
        assert float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) <= 5e-2
    assert torch.isfinite(tr.dW).all()


def test_package_jacobi_init_is_damped_jacobi():
    """The package's initial weights make the network exactly 2/3 rho on face
    interiors (and equal the oracle's initialisation)."""
    import torch

    import paper_1805_10167_amd as P
    from paper_1805_10167_amd import train
    L = 5
    g = make_mesh(L)
    H = oracle_hierarchy(NAME, L, 2)
    lv = H.levels[L]
    w = train.jacobi_init()
    assert np.array_equal(w, onet.pack(*onet.jacobi_init()).astype(np.float32))
    P.hhg_net_set_weights(g.h, w)
    P.hhg_net_set_options(g.h, P.HHG_F32, 0)
    rho = hi.uniform_vector(lv.n_all, 12).astype(np.float32).astype(np.float64)
    out = g.field(L, P.HHG_F32)
    P.hhg_net_forward(g.h, L, g.from_canonical(L, rho, P.HHG_F32), out)
    got = to_np(g.to_canonical(L, out, P.HHG_F32))
    face = lv.kind == 2
    assert rel_err(got[face], (2.0 / 3.0) * rho[face]) <= 1e-6
    assert not got[~face].any()
    assert torch.isfinite(out).all()


def _train_short(g, L, kind, steps=300):
    import paper_1805_10167_amd as P
    from paper_1805_10167_amd import train
    _, n_all = g.n_dofs(L)
    seeds = list(range(8))
    kaps = [kappa_dev(g, L, s) for s in seeds]
    if kind == "noise":
        ps = train.noise_pairs(g, kaps, lambda s, j: hi.uniform_vector(n_all, 5000 + 100 * s + j),
                               per_field=4)
    else:
        ps = train.capture_pairs(g, kaps, [hi.uniform_rhs(n_all, 1000 + s) for s in seeds], cycles=4)
    w0 = onet.pack(*onet.jacobi_init()).astype(np.float32)
    P.hhg_net_set_weights(g.h, w0)
    tr = train.Trainer(ps, lr=3e-3, batch=4, seed=0)
    loss0 = tr.mean_loss()
    losses = tr.train(steps)
    loss1 = tr.mean_loss()
    log("%s pairs: training loss %.4f -> %.4f (first batches %.4f, last %.4f)"
        % (kind, loss0, loss1, losses[:20].mean(), losses[-20:].mean()))
    assert np.all(np.isfinite(losses))
    assert loss1 < 0.97 * loss0
    return tr, w0


def _held_out(g, L):
    _, n_all = g.n_dofs(L)
    held = [10000, 10001]
    return [kappa_dev(g, L, s) for s in held], [hi.uniform_rhs(n_all, 1000 + s) for s in held]


def test_noise_training_gain_and_acceptance(tmp_path):
    """A short run on noise pairs lowers the training loss below the
    Jacobi-initialised network's, converges in the cycle and gains over the
    initial network on held-out fields; the acceptance rule is applied as
    stated and the learned solve honours its decision."""
    import paper_1805_10167_amd as P
    from paper_1805_10167_amd import train
    L = 5
    g = make_mesh(L)
    tr, w0 = _train_short(g, L, "noise")
    w1 = tr.weights()
    path = str(tmp_path / "net.npz")
    tr.save(path)
    wl, step = train.load_weights(path)
    assert step == 300 and np.array_equal(wl, w1)

    hk, hr = _held_out(g, L)
    rho_init, fb0 = train.evaluate(g, hk, hr, w0)
    dec = train.accept(g, hk, hr, w1)
    log("held-out factors: GS %s, Jacobi init %s, trained %s, guard %d, accepted %s"
        % (np.round(dec["rho_gs"], 4), np.round(rho_init, 4), np.round(dec["rho_net"], 4),
           dec["guard_tripped"], dec["accepted"]))
    assert not fb0.any() and dec["guard_tripped"] == 0
    assert dec["accepted"] == (dec["rho_net_mean"] <= dec["rho_gs_mean"])
    assert dec["rho_net_mean"] < 0.9 * rho_init.mean()
    f = g.from_canonical(L, hr[0])
    P.hhg_set_coefficient(g.h, hk[0])
    u = g.field(L)
    rc, st, _ = P.hhg_solve(g.h, u, f, mode=P.HHG_MODE_LEARNED, op=P.HHG_OP_DIFFUSION,
                            rtol=1e-8, max_iters=100)
    assert rc == 0 and st["rel_res"] <= 1e-8
    expect = P.HHG_SMOOTH_NET if dec["accepted"] else P.HHG_SMOOTH_GS
    assert st["smoother_used"] == expect and st["fallback"] == (0 if dec["accepted"] else 1)


def test_cycle_pair_training_is_rejected():
    """Trained on cycle-start pairs alone (smooth errors) the network
    amplifies high frequencies: its first learned cycle raises the residual,
    the guard undoes it, and acceptance fails."""
    from paper_1805_10167_amd import train
    L = 5
    g = make_mesh(L)
    tr, _ = _train_short(g, L, "cycles")
    hk, hr = _held_out(g, L)
    dec = train.accept(g, hk, hr, tr.weights())
    log("cycle-pair network: guard tripped %d, accepted %s" % (dec["guard_tripped"], dec["accepted"]))
    assert dec["guard_tripped"] == 2 and not dec["accepted"]


def test_early_stopping_keeps_the_best_factor():
    """train_early_stopping keeps the weights of the chunk with the smallest
    validation factor, which they reproduce exactly, and refuses to validate
    on the training mesh."""
    from paper_1805_10167_amd import train
    L = 5
    g, gv = make_mesh(L), make_mesh(L)
    _, n_all = g.n_dofs(L)
    kaps = [kappa_dev(g, L, s) for s in range(8)]
    ps = train.noise_pairs(g, kaps, lambda s, j: hi.uniform_vector(n_all, 5000 + 100 * s + j), per_field=4)
    import paper_1805_10167_amd as P
    P.hhg_net_set_weights(g.h, train.jacobi_init())
    tr = train.Trainer(ps, lr=3e-3, batch=4, seed=0)
    vseeds = (20000, 20001)
    vk = [kappa_dev(gv, L, s) for s in vseeds]
    vf = [hi.uniform_rhs(n_all, 1000 + s) for s in vseeds]
    w, step, hist, losses = train.train_early_stopping(tr, 400, 100, gv, vk, vf, log=log)
    assert len(hist) == 4 and len(losses) == 400 and np.all(np.isfinite(losses))
    best = min(r for _, r in hist)
    assert np.isfinite(best) and step == next(s for s, r in hist if r == best)
    rho, fb = train.evaluate(gv, vk, vf, w)
    assert not fb.any() and float(rho.mean()) == best
    with pytest.raises(ValueError):
        train.train_early_stopping(tr, 100, 100, g, vk, vf)
