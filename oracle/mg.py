"""Geometric multigrid on the refinement hierarchy (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (sec. 4.3) names the ingredients: pointwise smoothers that use the
diagonal, Gauss-Seidel needing a global update order (sec. 2.4) realised as a
multicolour Gauss-Seidel (sec. 3.2), interpolation and restriction as
non-square matrix-vector products, Krylov or direct solvers on the coarse
grid, and multigrid as a solver.  It fixes none of the parameters; the
readings used here are:

  * smoother stages, each updated simultaneously: A = interior macro-vertices
    and even-k edge points, B = odd-k edge points, then face colours
    (i - j) mod 3 = 0, 1, 2; a face with an exactly right angle uses two
    colours by the parity rule of the direction with zero weight.  The
    backward sweep runs the stages in reverse order;
  * restriction is the transpose of linear interpolation (weight 1 at the
    coincident point, 1/2 at each neighbour);
  * residual, correction and coarse right-hand side are zero at Dirichlet
    points;
  * coarse solve: direct (the exact solution of the coarse interior system,
    by a sparse LU factorisation) by default; the Krylov alternative is CG
    with Jacobi preconditioner from zero, stopping when |r| <= 1e-14 |b| or
    after 4 N iterations;
  * solve loop: relative residual |f - A u| / |f - A u0| over interior points
    after every cycle.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import assemble, inject
from .mesh import Level


def face_colouring(mesh, f, i, j):
    """Colour of face-local interior points (i, j) of face f, and the number
    of colours.  Every stencil offset changes i - j by +-1 or +-2, so
    (i - j) mod 3 is a proper colouring; with a right angle the direction of
    zero weight is dropped and a parity rule remains."""
    d0, d1, d2 = mesh.face_dot(f)
    if d0 == 0.0:
        return (i + j) % 2, 2
    if d1 == 0.0:
        return i % 2, 2
    if d2 == 0.0:
        return j % 2, 2
    return (i - j) % 3, 3


def stage_sets(lv):
    """Index arrays of the forward-sweep stages [A, B, F0, F1, F2]."""
    mesh = lv.mesh
    interior = ~lv.dirichlet
    is_v = (lv.kind == 0) & interior
    is_e = (lv.kind == 1) & interior
    even = (lv.kidx % 2) == 0
    A = np.flatnonzero(is_v | (is_e & even))
    B = np.flatnonzero(is_e & ~even)
    colour = np.full(lv.n_all, -1)
    for f in range(mesh.F):
        s = lv.face_base + f * lv.n_face
        idx = np.arange(s, s + lv.n_face)
        c, _ = face_colouring(mesh, f, lv.kidx[idx], lv.jidx[idx])
        colour[idx] = c
    F = [np.flatnonzero(colour == c) for c in range(3)]
    return [A, B] + F


def prolongation(lf, lc):
    """Linear interpolation from level lc to level lf = lc + 1 as a sparse
    [n_all(lf), n_all(lc)] matrix.  A fine point either coincides with a
    coarse point or is the midpoint of a coarse micro-edge."""
    rows, cols, vals = [], [], []
    n = lf.n
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m = I + J <= n - 1
    I, J = I[m], J[m]
    for locf, locc in zip(lf.loc, lc.loc):
        fine = locf[J, I]
        ie, je = I % 2 == 0, J % 2 == 0
        both = ie & je
        rows.append(fine[both]); cols.append(locc[J[both] // 2, I[both] // 2])
        vals.append(np.ones(both.sum()))
        # the two coarse endpoints of the coarse micro-edge through the point
        for sel, a_i, a_j, b_i, b_j in (
                (~ie & je, (I - 1) // 2, J // 2, (I + 1) // 2, J // 2),
                (ie & ~je, I // 2, (J - 1) // 2, I // 2, (J + 1) // 2),
                (~ie & ~je, (I + 1) // 2, (J - 1) // 2, (I - 1) // 2, (J + 1) // 2)):
            rows += [fine[sel], fine[sel]]
            cols += [locc[a_j[sel], a_i[sel]], locc[b_j[sel], b_i[sel]]]
            vals += [np.full(sel.sum(), 0.5), np.full(sel.sum(), 0.5)]
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    # points on shared edges/vertices appear once per face: keep one copy
    key = rows * lc.n_all + cols
    _, first = np.unique(key, return_index=True)
    return sp.csr_matrix((vals[first], (rows[first], cols[first])),
                         shape=(lf.n_all, lc.n_all))


def pcg_jacobi(A, b, tol=1e-14, maxit=None):
    """Jacobi-preconditioned CG from x = 0 (sec. 4.3 names PCG for SPD
    problems).  Returns (x, iterations)."""
    N = len(b)
    maxit = 4 * N if maxit is None else maxit
    x = np.zeros(N)
    bn = np.sqrt(b @ b)
    if bn == 0.0:
        return x, 0
    dinv = 1.0 / A.diagonal()
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.sqrt(r @ r) <= tol * bn:
            break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


class Hierarchy:
    """All levels lc..L of one macro mesh with their operators.

    op: "laplace" (k = 1) or "diffusion" (nodal k at the finest level,
    injected to coarser levels).  coarse: "direct" or "pcg" (sec. 4.3 allows
    either on the coarse grid).  face_coef[F]: a coefficient constant on each
    macro-face multiplying the stiffness on every level (the same on all
    levels, so the coarse operators stay the Galerkin products)."""

    def __init__(self, mesh, L, lc=2, kappa_fine=None, coarse="direct", face_coef=None):
        self.mesh = mesh
        self.L = L
        self.lc = lc
        if coarse not in ("direct", "pcg"):
            raise ValueError(coarse)
        self.coarse = coarse
        self.levels = {l: Level(mesh, l) for l in range(lc, L + 1)}
        self.kappa = {}
        if kappa_fine is not None:
            self.kappa[L] = np.asarray(kappa_fine, dtype=np.float64)
            for l in range(L - 1, lc - 1, -1):
                self.kappa[l] = inject(self.levels[l + 1], self.levels[l], self.kappa[l + 1])
        self.A = {}
        self.M = {}
        self.P = {}
        self.stages = {}
        self.diag = {}
        for l, lv in self.levels.items():
            mats = assemble(lv, self.kappa.get(l), face_coef=face_coef)
            self.A[l] = mats["A"]
            self.M[l] = mats["M"]
            self.diag[l] = self.A[l].diagonal()
            self.stages[l] = [(S, self.A[l][S]) for S in stage_sets(lv)]
            if l > lc:
                self.P[l] = prolongation(lv, self.levels[l - 1])
        lvc = self.levels[lc]
        ic = lvc.interior
        self.A_coarse = self.A[lc][ic][:, ic].tocsr()
        self._lu = spla.splu(self.A_coarse.tocsc()) if coarse == "direct" else None

    # ---- Alg. 3 semantics: y = A x on interior rows, 0 on Dirichlet rows
    def apply(self, l, x, op="A"):
        lv = self.levels[l]
        y = (self.A[l] if op == "A" else self.M[l]) @ x
        y[lv.dirichlet] = 0.0
        return y

    def residual(self, l, u, f):
        lv = self.levels[l]
        r = f - self.A[l] @ u
        r[lv.dirichlet] = 0.0
        return r

    def smooth(self, l, u, f, sweeps=1, backward=False):
        """Staged Gauss-Seidel: within a stage all points are updated at once,
        u_S += D_S^-1 (f - A u)_S (omega = 1)."""
        order = self.stages[l][::-1] if backward else self.stages[l]
        d = self.diag[l]
        for _ in range(sweeps):
            for S, AS in order:
                if len(S):
                    u[S] += (f[S] - AS @ u) / d[S]
        return u

    def restrict(self, l, r):
        """Coarse right-hand side P^T r, zero at coarse Dirichlet points."""
        fc = self.P[l].T @ r
        fc[self.levels[l - 1].dirichlet] = 0.0
        return fc

    def prolong_add(self, l, u, uc):
        """u += P uc at interior fine points (Dirichlet points untouched)."""
        c = self.P[l] @ uc
        ii = self.levels[l].interior
        u[ii] += c[ii]
        return u

    def coarse_solve(self, u, f):
        """u += A_int^-1 (f - A u)_int on the coarsest level (exactly, or by
        PCG); returns the PCG iterations (0 for the direct solve)."""
        lvc = self.levels[self.lc]
        r = self.residual(self.lc, u, f)
        b = r[lvc.interior]
        if self._lu is not None:
            x, it = self._lu.solve(b), 0
        else:
            x, it = pcg_jacobi(self.A_coarse, b)
        u[lvc.interior] += x
        return it

    def vcycle(self, l, u, f, nu1, nu2):
        """One V(nu1, nu2) cycle on level l (sec. 4.3: geometric multigrid on
        the nested hierarchy)."""
        if l == self.lc:
            self.coarse_solve(u, f)
            return u
        self.smooth(l, u, f, nu1, backward=False)
        r = self.residual(l, u, f)
        fc = self.restrict(l, r)
        uc = np.zeros(self.levels[l - 1].n_all)
        self.vcycle(l - 1, uc, fc, nu1, nu2)
        self.prolong_add(l, u, uc)
        self.smooth(l, u, f, nu2, backward=True)
        return u

    def res_norm(self, l, u, f):
        r = self.residual(l, u, f)
        return float(np.sqrt(r @ r))

    def solve(self, u, f, rtol=1e-8, nu1=3, nu2=3, max_iters=100):
        """Multigrid as a solver: V-cycles until the relative residual over
        interior points drops below rtol.  Returns (u, history)."""
        L = self.L
        r0 = self.res_norm(L, u, f)
        hist = [r0]
        if r0 == 0.0:
            return u, hist
        for _ in range(max_iters):
            self.vcycle(L, u, f, nu1, nu2)
            hist.append(self.res_norm(L, u, f))
            if hist[-1] <= rtol * r0:
                break
        return u, hist


def build_hierarchy(vxy, tri, L, lc=2, kappa_fine=None):
    from .mesh import MacroMesh
    return Hierarchy(MacroMesh(vxy, tri), L, lc, kappa_fine)
