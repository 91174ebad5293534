"""Learned face smoother: forward, backward, loss and Adam (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not in the paper: this is the smoother variant layered on the plain method
(two-layer hexagonal CNN on the triangular grid).  Readings:
  * input: one channel, rho = D^-1 r on the whole face array (ring included,
    where the ring holds the edge and vertex rho);
  * hidden layer: 16 channels, ReLU, defined on face-interior points only
    (zero elsewhere); output: one channel on face-interior points;
  * 7-tap kernels over the offsets C, E, W, N, S, SE, NW of face-local
    (i, j); no biases, so N(a rho) = a N(rho) for a > 0;
  * W1[c, t] (input -> hidden channel c), W2[c, t] (hidden c -> output);
  * initialisation: channels 0 and 1 carry +rho and -rho (centre tap),
    output w (h0 - h1) with w = 2/3 (damped Jacobi); the other 14 channels
    get W1 ~ N(0, 0.01^2) from seed 42 and W2 = 0;
  * smoother step: stages A and B of Gauss-Seidel on edges and vertices,
    then u += N(D^-1 (f - A u)) on face interiors (backward: reverse);
  * loss of a pair (r, e = u* - u): (d^T A d) / (e^T A e), d = e - N(D^-1 r)
    on face interiors, d = e elsewhere.
"""
import numpy as np

TAPS = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1)]   # (di, dj)
NCH = 16


def jacobi_init(omega=2.0 / 3.0, seed=42, nch=NCH):
    """(W1, W2) of the damped-Jacobi initialisation, shape [nch, 7] each."""
    W1 = np.zeros((nch, 7))
    W2 = np.zeros((nch, 7))
    W1[0, 0], W1[1, 0] = 1.0, -1.0
    W2[0, 0], W2[1, 0] = omega, -omega
    W1[2:] = np.random.default_rng(seed).normal(0.0, 0.01, size=(nch - 2, 7))
    return W1, W2


def pack(W1, W2):
    """Flat [W1 (row-major), W2 (row-major)] vector of 2 * nch * 7 values."""
    return np.concatenate([np.asarray(W1).ravel(), np.asarray(W2).ravel()])


def unpack(w, nch=NCH):
    w = np.asarray(w, dtype=np.float64)
    return w[:nch * 7].reshape(nch, 7), w[nch * 7:].reshape(nch, 7)


def _shift(G, di, dj):
    """S[j, i] = G[j + dj, i + di] (zero outside the array)."""
    n = G.shape[-1]
    S = np.zeros_like(G)
    js = slice(max(0, -dj), min(n, n - dj))
    is_ = slice(max(0, -di), min(n, n - di))
    jd = slice(max(0, dj), min(n, n + dj))
    id_ = slice(max(0, di), min(n, n + di))
    S[..., js, is_] = G[..., jd, id_]
    return S


def _face_grid(lv, f, x):
    loc = lv.loc[f]
    G = np.zeros((lv.n, lv.n))
    m = loc >= 0
    G[m] = x[loc[m]]
    return G


def _interior_mask(n):
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return (I >= 1) & (J >= 1) & (I + J <= n - 2)


def forward(lv, rho, W1, W2, keep=False):
    """out = N(rho) on face-interior points (canonical vector, zero elsewhere).
    With keep, also returns per-face (rho grid, a) for the backward pass."""
    out = np.zeros(lv.n_all)
    mask = _interior_mask(lv.n)
    saved = []
    for f in range(lv.mesh.F):
        R = _face_grid(lv, f, rho)
        taps = np.stack([_shift(R, di, dj) for di, dj in TAPS])       # [7, n, n]
        a = np.einsum("ct,tji->cji", W1, taps) * mask                  # [16, n, n]
        h = np.maximum(a, 0.0)
        o = np.zeros((lv.n, lv.n))
        for t, (di, dj) in enumerate(TAPS):
            o += np.einsum("c,cji->ji", W2[:, t], _shift(h, di, dj))
        o *= mask
        loc = lv.loc[f]
        out[loc[mask]] = o[mask]
        if keep:
            saved.append((taps, a, h))
    return (out, saved) if keep else out


def backward(lv, rho, g, W1, W2):
    """Gradients (dW1, dW2) of sum_p g(p) N(rho)(p) over face-interior p."""
    _, saved = forward(lv, rho, W1, W2, keep=True)
    mask = _interior_mask(lv.n)
    dW1 = np.zeros_like(W1)
    dW2 = np.zeros_like(W2)
    for f in range(lv.mesh.F):
        taps, a, h = saved[f]
        Gf = _face_grid(lv, f, g) * mask
        dh = np.zeros_like(h)
        for t, (di, dj) in enumerate(TAPS):
            # out(p) gets W2[c,t] h_c(p + d_t): pair h at q with g at q - d_t
            Gq = _shift(Gf, -di, -dj)
            dW2[:, t] += np.einsum("cji,ji->c", h, Gq)
            dh += W2[:, t][:, None, None] * Gq
        da = dh * (a > 0) * mask
        dW1 += np.einsum("cji,tji->ct", da, taps)
    return dW1, dW2


def jacobi_scale(H, l, r):
    """rho = D^-1 r at interior points, zero at Dirichlet points."""
    lv = H.levels[l]
    rho = r / H.diag[l]
    rho[lv.dirichlet] = 0.0
    return rho


def loss_and_grad(H, l, r, e, W1, W2):
    """Energy-norm loss of one (r, e) pair and its weight gradients."""
    lv = H.levels[l]
    A = H.A[l]
    rho = jacobi_scale(H, l, r)
    out = forward(lv, rho, W1, W2)
    d = e - out
    d[lv.dirichlet] = 0.0
    Ad = A @ d
    Ad[lv.dirichlet] = 0.0
    E0 = float(e @ r)
    L = float(d @ Ad) / E0
    g = -2.0 * Ad / E0
    dW1, dW2 = backward(lv, rho, g, W1, W2)
    return L, dW1, dW2


def adam(w, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), step counted from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def net_smooth(H, l, u, f, W1, W2, sweeps=1, backward_order=False):
    """Smoother step with the network on faces and GS stages A, B on edges
    and vertices; the backward order runs the face step first."""
    lv = H.levels[l]
    d = H.diag[l]
    A_st, B_st = H.stages[l][0], H.stages[l][1]

    def stage(S_AS):
        S, AS = S_AS
        if len(S):
            u[S] += (f[S] - AS @ u) / d[S]

    def faces():
        r = H.residual(l, u, f)
        u[:] += forward(lv, jacobi_scale(H, l, r), W1, W2)

    for _ in range(sweeps):
        if backward_order:
            faces(); stage(B_st); stage(A_st)
        else:
            stage(A_st); stage(B_st); faces()
    return u
