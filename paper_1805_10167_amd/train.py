"""Training and acceptance of the learned face smoother, driven through the
library's calls (the network itself is not part of the paper: it replaces the
face colour stages of the smoother of sec. 4.3 in the FP32 cycles of the
mixed-precision refinement loop).

Every arithmetic step runs in libhhg.so: plain V-cycles and solves capture the
training pairs, and the library's Jacobi scaling, network forward/backward,
operator, dot, axpby and Adam calls make one training step.  torch only holds
the buffers.

Training pairs, two kinds.  Noise pairs (the default training set): for a
coefficient field k, e = D^-1 xi with xi i.i.d. uniform on the interior
points (0 on Dirichlet points) and r = A e -- errors with the whole spectrum
in them, as a smoother meets them after a coarse-grid correction.  Cycle
pairs: for k and a right-hand side f, the exact discrete solution u* comes
from a plain FP64 solve; plain V-cycles from u = 0 then give, at the start of
each of the first cycles, r = f - A u and e = u* - u.  Those errors are
smooth, so a network trained on them alone is free to amplify the high
frequencies it never sees, and it does (the solver's guard then drops it);
they are kept for that comparison.

Loss of one pair, with rho = D^-1 r and d = e - N(rho):
    L = d^T A d / e^T A e,   dL/dN = -2 A d / e^T A e,
the energy-norm error left by one application of the network, relative to the
error it was given; e^T A e = e^T r is taken once at capture.  A batch
averages the losses of its pairs.

Model selection.  The loss measures one application of the network, the
acceptance a whole cycle; past a few hundred steps the first keeps falling
while the second gets worse.  train_early_stopping therefore measures the
convergence factor (below) on validation fields, whose seeds are disjoint
from the training and the acceptance fields, at regular intervals, and keeps
the weights with the smallest one.

Acceptance.  The convergence factor of V(nu1, nu2) cycles inside the
mixed-precision loop, (|r_last| / |r_first|)^(1 / (last - first)), with the
network and with Gauss-Seidel on held-out coefficient fields; the network is
accepted iff its mean factor is no larger and no learned cycle tripped the
solver's guard.
"""
import numpy as np

from ._lib import (HHG_BF16, HHG_F32, HHG_F64, HHG_MODE_LEARNED, HHG_MODE_MP_IR,
                   HHG_MODE_PLAIN_FP64, HHG_OK, HHG_OP_DIFFUSION, HHG_SMOOTH_GS,
                   hhg_apply, hhg_axpby, hhg_convert, hhg_dot, hhg_field_elems,
                   hhg_jacobi, hhg_net_adam_step, hhg_net_backward,
                   hhg_net_forward, hhg_net_get_weights, hhg_net_set_options,
                   hhg_net_set_weights, hhg_residual, hhg_set_coefficient, hhg_solve,
                   hhg_vcycle)

N_WEIGHTS = 224


def jacobi_init(omega=2.0 / 3.0, seed=42):
    """Initial weights (W1[16][7] then W2[16][7], FP32) that make the network
    exactly damped Jacobi on face interiors: hidden channels 0 and 1 carry
    +rho and -rho through their centre taps, the output is omega (h0 - h1)
    = omega rho; channels 2..15 start with small N(0, 0.01^2) input weights
    (default_rng(seed)) and zero output weights, so they change nothing yet
    can learn."""
    W1 = np.zeros((16, 7))
    W2 = np.zeros((16, 7))
    W1[0, 0], W1[1, 0] = 1.0, -1.0
    W2[0, 0], W2[1, 0] = omega, -omega
    W1[2:] = np.random.default_rng(seed).normal(0.0, 0.01, size=(14, 7))
    return np.concatenate([W1.ravel(), W2.ravel()]).astype(np.float32)


class PairSet:
    """(r, e) pairs in FP32 library layout on the finest level of `mesh`,
    with the index of the coefficient field each pair belongs to and its
    energy e^T r."""

    def __init__(self, mesh, kappas, r, e, sample, energy):
        self.mesh = mesh
        self.level = mesh.L
        self.kappas = kappas
        self.r = r
        self.e = e
        self.sample = sample
        self.energy = energy

    def __len__(self):
        return len(self.sample)


def capture_pairs(mesh, kappas, rhss, cycles=8, tol=1e-12, nu1=3, nu2=3, log=None):
    """Pairs from plain FP64 V(nu1, nu2) cycles on the finest level.

    kappas: device FP64 tensors of nodal coefficients (canonical order);
    rhss: right-hand sides (canonical order, host or device).  The mesh
    needs HHG_FEAT_F64 | HHG_FEAT_MP | HHG_FEAT_VARK."""
    import torch
    L, h, dev = mesh.L, mesh.h, mesh.device
    total = hhg_field_elems(h, L)
    n = len(kappas)
    R = torch.empty((n * cycles, total), dtype=torch.float32, device=dev)
    E = torch.empty_like(R)
    energy = torch.zeros(n * cycles, dtype=torch.float64, device=dev)
    ustar, u, r64, e64 = (mesh.field(L) for _ in range(4))
    for s in range(n):
        hhg_set_coefficient(h, kappas[s])
        ff = mesh.from_canonical(L, rhss[s])
        ustar.zero_()
        rc, st, _ = hhg_solve(h, ustar, ff, mode=HHG_MODE_PLAIN_FP64, op=HHG_OP_DIFFUSION,
                              rtol=tol, max_iters=200, nu1=nu1, nu2=nu2, history=False)
        if rc != HHG_OK:
            raise RuntimeError("reference solve of sample %d did not reach %g: %s" % (s, tol, st))
        u.zero_()
        for c in range(cycles):
            k = s * cycles + c
            hhg_residual(h, L, HHG_OP_DIFFUSION, HHG_F64, u, ff, r64)
            hhg_axpby(h, L, HHG_F64, 1.0, ustar, -1.0, u, e64)
            hhg_dot(h, L, HHG_F64, e64, r64, energy[k:k + 1])
            hhg_convert(h, L, HHG_F64, r64, HHG_F32, R[k])
            hhg_convert(h, L, HHG_F64, e64, HHG_F32, E[k])
            hhg_vcycle(h, L, HHG_OP_DIFFUSION, HHG_SMOOTH_GS, HHG_F64, u, ff, nu1, nu2)
        if log and (s + 1) % max(1, n // 8) == 0:
            log("captured %d/%d samples (reference solve: %d cycles)" % (s + 1, n, st["iters"]))
    return PairSet(mesh, kappas, R, E, np.repeat(np.arange(n), cycles),
                   energy.cpu().numpy())


def noise_pairs(mesh, kappas, draw, per_field=8):
    """Noise pairs on the finest level of `mesh`: for each coefficient field
    s and j < per_field, xi = draw(s, j) (canonical order, FP64, host or
    device), e = D^-1 xi (0 on Dirichlet points), r = A e."""
    import torch
    L, h, dev = mesh.L, mesh.h, mesh.device
    total = hhg_field_elems(h, L)
    n = len(kappas)
    R = torch.empty((n * per_field, total), dtype=torch.float32, device=dev)
    E = torch.empty_like(R)
    energy = torch.zeros(n * per_field, dtype=torch.float64, device=dev)
    r64, e64 = mesh.field(L), mesh.field(L)
    for s in range(n):
        hhg_set_coefficient(h, kappas[s])
        for j in range(per_field):
            k = s * per_field + j
            xi = mesh.from_canonical(L, draw(s, j))
            hhg_jacobi(h, L, HHG_OP_DIFFUSION, HHG_F64, xi, None, e64)
            hhg_apply(h, L, HHG_OP_DIFFUSION, HHG_F64, e64, r64)
            hhg_dot(h, L, HHG_F64, e64, r64, energy[k:k + 1])
            hhg_convert(h, L, HHG_F64, r64, HHG_F32, R[k])
            hhg_convert(h, L, HHG_F64, e64, HHG_F32, E[k])
    return PairSet(mesh, kappas, R, E, np.repeat(np.arange(n), per_field), energy.cpu().numpy())


class Trainer:
    """Adam on the network's 224 FP32 master weights held by the mesh."""

    def __init__(self, pairs, lr=1e-3, batch=4, seed=0, precision=HHG_BF16):
        import torch
        self.p = pairs
        m = pairs.mesh
        self.h, self.L = m.h, pairs.level
        self.lr, self.batch = lr, batch
        self.rng = np.random.default_rng(seed)
        self.seed = seed
        self.step = 0
        self.precision = precision
        self.rho, self.out, self.d, self.g = (m.field(self.L, HHG_F32) for _ in range(4))
        self.dW = torch.zeros(N_WEIGHTS, dtype=torch.float32, device=m.device)
        self._cur = None
        hhg_net_set_options(self.h, precision, 0)

    def _use(self, s):
        if self._cur != s:
            hhg_set_coefficient(self.h, self.p.kappas[s])
            self._cur = s

    def _pair(self, k, scale, loss_slot):
        """Accumulate scale * dL_k/dW into dW; d^T A d into loss_slot."""
        h, L, p = self.h, self.L, self.p
        self._use(int(p.sample[k]))
        hhg_jacobi(h, L, HHG_OP_DIFFUSION, HHG_F32, p.r[k], None, self.rho)
        hhg_net_forward(h, L, self.rho, self.out)
        hhg_axpby(h, L, HHG_F32, 1.0, p.e[k], -1.0, self.out, self.d)
        hhg_apply(h, L, HHG_OP_DIFFUSION, HHG_F32, self.d, self.g)
        hhg_dot(h, L, HHG_F32, self.d, self.g, loss_slot)
        hhg_axpby(h, L, HHG_F32, -2.0 * scale / p.energy[k], self.g, 0.0, self.g, self.g)
        hhg_net_backward(h, L, self.rho, self.g, self.dW)

    def gradient(self, idx):
        """Mean loss gradient of the pairs idx in dW; returns their losses."""
        import torch
        lb = torch.zeros(len(idx), dtype=torch.float64, device=self.dW.device)
        self.dW.zero_()
        for b, k in enumerate(idx):
            self._pair(k, 1.0 / len(idx), lb[b:b + 1])
        return lb.cpu().numpy() / self.p.energy[np.asarray(idx)]

    def train(self, steps, log=None, log_every=100):
        """`steps` Adam steps on random batches; returns the mean batch loss
        of every step."""
        import torch
        n = len(self.p)
        B = min(self.batch, n)
        lb = torch.zeros(steps * B, dtype=torch.float64, device=self.dW.device)
        order = []
        for t in range(steps):
            idx = self.rng.choice(n, B, replace=False)
            order.append(idx)
            self.dW.zero_()
            for b, k in enumerate(idx):
                j = t * B + b
                self._pair(k, 1.0 / B, lb[j:j + 1])
            self.step += 1
            hhg_net_adam_step(self.h, self.dW, self.lr, self.step)
            if log and (t + 1) % log_every == 0:
                last = lb[(t + 1 - log_every) * B:(t + 1) * B].cpu().numpy()
                en = self.p.energy[np.concatenate(order[t + 1 - log_every:t + 1])]
                log("step %d: mean loss %.4f" % (self.step, float(np.mean(last / en))))
        dAd = lb.cpu().numpy().reshape(steps, B)
        en = self.p.energy[np.stack(order)]
        return (dAd / en).mean(axis=1)

    def mean_loss(self, idx=None):
        """Mean loss of the current weights over the pairs idx (all by default)."""
        idx = np.arange(len(self.p)) if idx is None else np.asarray(idx)
        out = []
        for s in range(0, len(idx), 64):
            out.append(self.gradient(idx[s:s + 64]))
        return float(np.concatenate(out).mean())

    def weights(self):
        return hhg_net_get_weights(self.h)

    def save(self, path, losses=None):
        """Checkpoint: FP32 master weights, step count, batch seed and losses
        (Adam's moments restart from zero on load)."""
        np.savez(path, weights=self.weights(), step=self.step, seed=self.seed,
                 losses=np.zeros(0) if losses is None else np.asarray(losses))


def load_weights(path):
    with np.load(path, allow_pickle=False) as z:
        return z["weights"].astype(np.float32), int(z["step"])


def convergence_factor(mesh, f, mode, nu1=3, nu2=3, first=3, last=12):
    """Convergence factor of the solve loop of `mode` from u = 0 on the
    finest level, and the solve's stats."""
    u = mesh.field(mesh.L)
    rc, st, hist = hhg_solve(mesh.h, u, f, mode=mode, op=HHG_OP_DIFFUSION, rtol=0.0,
                             max_iters=last, nu1=nu1, nu2=nu2, history=True)
    if len(hist) <= last or not np.isfinite(hist[last]) or hist[first] <= 0:
        return float("inf"), st
    return float((hist[last] / hist[first]) ** (1.0 / (last - first))), st


def evaluate(mesh, kappas, rhss, weights=None, precision=HHG_BF16, nu1=3, nu2=3):
    """Per-field convergence factors of the mixed-precision loop with
    Gauss-Seidel (weights None) or with the given network.  The network's
    runs mark it accepted for their duration; the flag is cleared after."""
    if weights is not None:
        hhg_net_set_weights(mesh.h, weights)
        hhg_net_set_options(mesh.h, precision, 1)
    rho, fallback = [], []
    try:
        for kap, f in zip(kappas, rhss):
            hhg_set_coefficient(mesh.h, kap)
            ff = mesh.from_canonical(mesh.L, f)
            mode = HHG_MODE_MP_IR if weights is None else HHG_MODE_LEARNED
            r, st = convergence_factor(mesh, ff, mode, nu1, nu2)
            rho.append(r)
            fallback.append(int(st["fallback"]))
    finally:
        if weights is not None:
            hhg_net_set_options(mesh.h, precision, 0)
    return np.array(rho), np.array(fallback)


def train_early_stopping(trainer, steps, every, mesh, kappas, rhss, precision=HHG_BF16, log=None):
    """Model selection by the quantity the network is judged on (the
    convergence factor of Q22): `steps` Adam steps in chunks of `every`;
    after each chunk the mean convergence factor of the learned cycle on the
    validation fields (kappas, rhss: seeds disjoint from the training and the
    acceptance fields) is measured on `mesh`, which must not be the training
    mesh, and the weights with the smallest factor are kept.  The one-step
    energy loss goes on falling after this factor has turned, so training to
    the loss plateau gives a worse smoother.  Returns (weights, step,
    [(step, factor), ...], per-step losses); without a finite factor the
    initial weights and step 0 come back."""
    if mesh.h == trainer.h:
        raise ValueError("validation needs a mesh of its own")
    best_rho, best_step, best_w = float("inf"), 0, trainer.weights()
    history, losses = [], []
    for _ in range(max(1, steps // every)):
        losses.append(trainer.train(every))
        w = trainer.weights()
        rho, fb = evaluate(mesh, kappas, rhss, w, precision)
        r = float(rho.mean()) if np.all(np.isfinite(rho)) and not fb.any() else float("inf")
        history.append((trainer.step, r))
        if log:
            log("step %d: validation factor %.5f" % (trainer.step, r))
        if r < best_rho:
            best_rho, best_step, best_w = r, trainer.step, w
    return best_w, best_step, history, np.concatenate(losses)


def accept(mesh, kappas, rhss, weights, precision=HHG_BF16, nu1=3, nu2=3):
    """Acceptance of `weights` against Gauss-Seidel; leaves the network loaded
    on `mesh` with the decision as its accepted flag."""
    rho_gs, _ = evaluate(mesh, kappas, rhss, None, precision, nu1, nu2)
    rho_net, fb = evaluate(mesh, kappas, rhss, weights, precision, nu1, nu2)
    ok = bool(np.all(np.isfinite(rho_net)) and not fb.any() and rho_net.mean() <= rho_gs.mean())
    hhg_net_set_weights(mesh.h, weights)
    hhg_net_set_options(mesh.h, precision, int(ok))
    return {"accepted": ok, "rho_gs": rho_gs.tolist(), "rho_net": rho_net.tolist(),
            "rho_gs_mean": float(rho_gs.mean()), "rho_net_mean": float(rho_net.mean()),
            "guard_tripped": int(fb.sum())}
