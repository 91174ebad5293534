"""Pins of the oracle's learned smoother (CPU only): finite differences,
the damped-Jacobi initialisation, homogeneity and Adam's first step."""
import numpy as np
import pytest

import hhg_inputs as hi
from oracle import net
from oracle.mesh import MacroMesh
from oracle.mg import Hierarchy


@pytest.fixture(scope="module")
def H3():
    vxy, tri = hi.annulus(16)
    m = MacroMesh(vxy, tri)
    from oracle.mesh import Level
    kap = np.exp(hi.grf_eval(Level(m, 3).xy, seed=4))
    return Hierarchy(m, 3, 2, kap)


def _pair(H, l, seed):
    lv = H.levels[l]
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(lv.n_all)
    e[lv.dirichlet] = 0.0
    r = H.apply(l, e)          # r = A e for the exact solution u* = u + e
    return r, e


def test_jacobi_init_is_damped_jacobi(H3):
    lv = H3.levels[3]
    W1, W2 = net.jacobi_init()
    rho = np.random.default_rng(0).standard_normal(lv.n_all)
    out = net.forward(lv, rho, W1, W2)
    face = lv.kind == 2
    assert np.array_equal(out[face], (2.0 / 3.0) * rho[face])
    assert not out[~face].any()


def test_net_smooth_with_jacobi_init(H3):
    """Stages A and B of Gauss-Seidel, then u_face += 2/3 D^-1 (f - A u)."""
    l = 3
    lv = H3.levels[l]
    rng = np.random.default_rng(1)
    u, f = rng.random(lv.n_all), rng.random(lv.n_all)
    W1, W2 = net.jacobi_init()
    got = net.net_smooth(H3, l, u.copy(), f, W1, W2)
    ref = u.copy()
    d = H3.diag[l]
    for S, AS in H3.stages[l][:2]:
        ref[S] += (f[S] - AS @ ref) / d[S]
    r = H3.residual(l, ref, f)
    face = lv.kind == 2
    ref[face] += (2.0 / 3.0) * r[face] / d[face]
    assert np.abs(got - ref).max() < 1e-13


def test_homogeneity(H3):
    lv = H3.levels[3]
    rng = np.random.default_rng(2)
    W1, W2 = rng.normal(size=(16, 7)), rng.normal(size=(16, 7))
    rho = rng.standard_normal(lv.n_all)
    a = net.forward(lv, rho, W1, W2)
    b = net.forward(lv, 3.5 * rho, W1, W2)
    assert np.abs(b - 3.5 * a).max() <= 1e-12 * np.abs(b).max()


def test_gradient_matches_central_differences(H3):
    l = 3
    rng = np.random.default_rng(3)
    W1, W2 = rng.normal(0, 0.5, (16, 7)), rng.normal(0, 0.5, (16, 7))
    r, e = _pair(H3, l, 5)
    L, dW1, dW2 = net.loss_and_grad(H3, l, r, e, W1, W2)
    grad = net.pack(dW1, dW2)
    w0 = net.pack(W1, W2)
    eps = 1e-6
    worst = 0.0
    for k in rng.choice(len(w0), 40, replace=False):
        wp, wm = w0.copy(), w0.copy()
        wp[k] += eps
        wm[k] -= eps
        Lp = net.loss_and_grad(H3, l, r, e, *net.unpack(wp))[0]
        Lm = net.loss_and_grad(H3, l, r, e, *net.unpack(wm))[0]
        fd = (Lp - Lm) / (2 * eps)
        worst = max(worst, abs(fd - grad[k]) / max(abs(grad).max(), 1e-30))
    assert worst <= 1e-6, worst


def test_loss_of_exact_correction_is_zero(H3):
    """If N reproduced e on faces and e vanished elsewhere, the loss is 0;
    with N = 0 the loss is 1."""
    l = 3
    r, e = _pair(H3, l, 6)
    zero = np.zeros((16, 7))
    L, _, _ = net.loss_and_grad(H3, l, r, e, zero, zero)
    assert abs(L - 1.0) < 1e-12


def test_adam_first_step():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.01, 0.0])
    w1, m, v = net.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    # bias-corrected first step: w - lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.1 * g / (np.abs(g) + 1e-8))
