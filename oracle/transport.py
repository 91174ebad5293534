"""Cell-centred finite-volume transport of the temperature and its coupling
to the Stokes flow (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's energy-transport example (sec. 5.2) advances the temperature T
with an explicit upwind finite-volume scheme, using the last computed
velocity, and solves the Stokes system (driven by the buoyancy -Ra T r_hat)
only after every three transport steps.  Finite-volume unknowns live on the
interiors of the micro-triangles (sec. 3.1).  The paper gives no parameter;
the readings are:

  * cells: every micro-triangle of every macro-face (up and down); T is one
    value per cell;
  * flux through a micro-edge e of cell c: F = |e| n . (u_a + u_b) / 2 with n
    the unit normal pointing out of c and u_a, u_b the P1 velocity at the
    edge's end points (the exact flux of the linear velocity along e);
  * one step: T_c <- T_c - dt / |c| sum_e F_e T_up(e), with T_up the value of
    c when F_e > 0 and of the neighbour across e otherwise;
  * no diffusion (the paper takes 1/Pe as negligible); micro-edges on the
    domain boundary carry no flux, since the velocity is zero there, so the
    prescribed wall temperatures act through the initial field only;
  * buoyancy load vector of the piecewise-constant T:
      b_i = -Ra r_hat(x_i) sum_{c contains i} T_c |c| / 3
    (the exact integral of T phi_i with r_hat frozen at the node);
  * time loop: a Stokes solve before transport steps 0, 3, 6, ... (warm
    started from the previous flow), then the transport step.

Cell order (canonical): per macro-face in input order, the up cells
{(i, j), (i+1, j), (i, j+1)} j-major, then the down cells
{(i+1, j), (i+1, j+1), (i, j+1)} j-major.
"""
import numpy as np
import scipy.sparse as sp


class Cells:
    """The cells of one level: point triples, areas, centroids, and for each
    cell and local edge k (opposite its k-th vertex) the neighbour cell across
    that edge (-1 on the domain boundary), found by matching point pairs."""

    def __init__(self, lv):
        n = lv.n
        tris, face, kind = [], [], []
        for f, loc in enumerate(lv.loc):
            for j in range(n - 1):
                for i in range(n - 1 - j):
                    tris.append((loc[j, i], loc[j, i + 1], loc[j + 1, i]))
                    face.append(f)
                    kind.append(0)
            for j in range(n - 2):
                for i in range(n - 2 - j):
                    tris.append((loc[j, i + 1], loc[j + 1, i + 1], loc[j + 1, i]))
                    face.append(f)
                    kind.append(1)
        self.tri = np.array(tris, dtype=np.int64)
        self.face = np.array(face)
        self.kind = np.array(kind)
        self.C = len(self.tri)
        p = lv.xy[self.tri]
        self.centroid = p.mean(axis=1)
        e1, e2 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]
        self.area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        # neighbour across local edge k = (vertex k+1, vertex k+2)
        owner = {}
        for c in range(self.C):
            for k in range(3):
                a, b = self.tri[c, (k + 1) % 3], self.tri[c, (k + 2) % 3]
                owner.setdefault((min(a, b), max(a, b)), []).append((c, k))
        self.nbr = -np.ones((self.C, 3), dtype=np.int64)
        for pairs in owner.values():
            assert len(pairs) <= 2
            if len(pairs) == 2:
                (c1, k1), (c2, k2) = pairs
                self.nbr[c1, k1] = c2
                self.nbr[c2, k2] = c1
        # outward normal times length of local edge k
        self.nlen = np.zeros((self.C, 3, 2))
        for k in range(3):
            a, b, o = p[:, (k + 1) % 3], p[:, (k + 2) % 3], p[:, k]
            d = b - a
            nv = np.stack([d[:, 1], -d[:, 0]], 1)            # |nv| = |e|
            flip = ((nv * (a - o)).sum(1) < 0)[:, None]       # point away from the opposite vertex
            self.nlen[:, k] = np.where(flip, -nv, nv)


def fluxes(cells, ux, uy):
    """F[c, k]: outward flux of the P1 velocity (ux, uy nodal, canonical)
    through local edge k of cell c; zero on the domain boundary."""
    F = np.zeros((cells.C, 3))
    for k in range(3):
        a, b = cells.tri[:, (k + 1) % 3], cells.tri[:, (k + 2) % 3]
        umx, umy = 0.5 * (ux[a] + ux[b]), 0.5 * (uy[a] + uy[b])
        F[:, k] = cells.nlen[:, k, 0] * umx + cells.nlen[:, k, 1] * umy
    F[cells.nbr < 0] = 0.0
    return F


def upwind_step(cells, T, F, dt):
    """One explicit upwind step of dT/dt + div(u T) = 0."""
    out = np.zeros(cells.C)
    for k in range(3):
        nb = cells.nbr[:, k]
        Tn = np.where(nb >= 0, T[np.maximum(nb, 0)], T)
        up = np.where(F[:, k] > 0, T, Tn)
        out += F[:, k] * up
    return T - dt / cells.area * out


def upwind_matrix(cells, F, dt):
    """The same step as a sparse matrix S with T_new = S T (for pins)."""
    rows, cols, vals = [np.arange(cells.C)], [np.arange(cells.C)], [np.ones(cells.C)]
    for k in range(3):
        s = dt / cells.area * F[:, k]
        out = F[:, k] > 0
        rows.append(np.flatnonzero(out)); cols.append(np.flatnonzero(out)); vals.append(-s[out])
        inn = (~out) & (cells.nbr[:, k] >= 0)
        rows.append(np.flatnonzero(inn)); cols.append(cells.nbr[inn, k]); vals.append(-s[inn])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(cells.C, cells.C))


def buoyancy(lv, cells, T, Ra):
    """Nodal load of -Ra T r_hat: b_i = -Ra r_hat(x_i) sum_{c ∋ i} T_c |c| / 3,
    zero at Dirichlet points (the velocity there is data)."""
    w = np.repeat((T * cells.area / 3.0)[:, None], 3, axis=1)
    s = np.bincount(cells.tri.ravel(), weights=w.ravel(), minlength=lv.n_all)
    r = np.hypot(lv.xy[:, 0], lv.xy[:, 1])
    bx = -Ra * s * lv.xy[:, 0] / r
    by = -Ra * s * lv.xy[:, 1] / r
    bx[lv.dirichlet] = 0.0
    by[lv.dirichlet] = 0.0
    return bx, by


def simulate(st, cells, T0, Ra, dt, steps, stokes_every=3, rtol=1e-8, max_iters=2000):
    """The coupled loop: before transport steps 0, stokes_every, ... solve
    Stokes (MINRES, warm start) with the buoyancy of the current T, then one
    upwind step with the current velocity.  Returns (T, Stokes vector,
    MINRES iteration counts)."""
    from .stokes import minres
    N = st.N
    x = np.zeros(3 * N)
    T = T0.copy()
    its = []
    F = None
    for k in range(steps):
        if k % stokes_every == 0:
            bx, by = buoyancy(st.lv, cells, T, Ra)
            b = np.concatenate([bx, by, np.zeros(N)])
            x, hist = minres(st.apply, st.precond, b, x, rtol=rtol, max_iters=max_iters)
            its.append(len(hist) - 1)
            F = fluxes(cells, x[:N], x[N:2 * N])
        T = upwind_step(cells, T, F, dt)
    return T, x, its
