"""Quadratic (P2) elements on the refined macro-faces and p-multigrid with
the linear (P1) elements of the same level (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references: second-order elements carry unknowns on the micro-vertices
and on the micro-edges, the edge unknowns forming three subgroups by edge
direction (sec. 3.1); a P2 stencil is a row of the P2 stiffness matrix, one
stencil shape for vertex unknowns and one for each edge direction (sec. 4.2,
Fig. 8); p-multigrid transfers between P1 and P2 on the same refinement
level (sec. 4.3).

Readings where the paper is silent (listed in the design notes):
  * the P2 unknowns of level l are the micro-vertices of level l + 1: the
    vertices of level l (even face-local indices) and the midpoints of its
    micro-edges (odd i: horizontal, odd j: vertical, both odd: diagonal
    edges), numbered canonically as level l + 1;
  * the operator is the Laplacian (times a coefficient constant on each
    macro-face), Dirichlet points as for P1;
  * smoother: damped point Jacobi u += omega D^-1 (f - A u) (a pointwise
    update with the stencil's diagonal);
  * p-multigrid cycle on level l: nu1 Jacobi sweeps, residual, restriction
    to P1 by the transpose of the P1 -> P2 embedding, one P1 V-cycle of the
    h-hierarchy from zero on level l, prolongation by the embedding,
    correction, nu2 Jacobi sweeps.

Parity status: `element_stiffness`, `assemble_p2` and `embedding` are pinned
(exactness on quadratics, the Galerkin identity with the P1 stiffness, the
closed-form integrals of the basis); the solver functions are pinned by
convergence to the direct solution.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import Level

# local node order of a P2 element: its vertices 0, 1, 2, then the midpoints
# of the edges (0, 1), (1, 2), (0, 2)
EDGES = ((0, 1), (1, 2), (0, 2))
# edge-midpoint quadrature (exact for polynomials of degree 2): barycentric
# coordinates of the three points, equal weights |T| / 3
QUAD = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])


def basis_gradients(P, lam):
    """Gradients of the six P2 Lagrange basis functions at the barycentric
    point lam of the triangle with vertices P[3, 2]:
      vertex a:    phi = lam_a (2 lam_a - 1)   -> (4 lam_a - 1) grad lam_a
      edge (a, b): phi = 4 lam_a lam_b         -> 4 (lam_b grad lam_a + lam_a grad lam_b)
    grad lam_a is the inward normal of the opposite side over twice the
    area."""
    x = P[:, 0]
    y = P[:, 1]
    det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0])
    gl = np.array([[y[1] - y[2], x[2] - x[1]],
                   [y[2] - y[0], x[0] - x[2]],
                   [y[0] - y[1], x[1] - x[0]]]) / det
    G = np.zeros((6, 2))
    for a in range(3):
        G[a] = (4.0 * lam[a] - 1.0) * gl[a]
    for k, (a, b) in enumerate(EDGES):
        G[3 + k] = 4.0 * (lam[b] * gl[a] + lam[a] * gl[b])
    return G, abs(det) / 2.0


def element_stiffness(P):
    """K[a, b] = integral of grad phi_a . grad phi_b over the triangle, by the
    edge-midpoint rule (the integrand is quadratic)."""
    K = np.zeros((6, 6))
    for lam in QUAD:
        G, area = basis_gradients(P, lam)
        K += (area / 3.0) * (G @ G.T)
    return K


def elements(lv_fine, lv_coarse):
    """P2 elements of level l: for every macro-face and every micro-triangle
    of level l (up triangles (a, b), then down triangles), the canonical
    level-(l+1) indices of its six nodes in the local order, the canonical
    level-l indices of its three vertices, and its face."""
    n = lv_coarse.n
    nodes, verts, face = [], [], []
    for f, (locf, locc) in enumerate(zip(lv_fine.loc, lv_coarse.loc)):
        for b in range(n - 1):
            for a in range(n - 1 - b):
                # up (a, b): vertices (a, b), (a+1, b), (a, b+1)
                V = [(a, b), (a + 1, b), (a, b + 1)]
                nodes.append(_p2_nodes(locf, V))
                verts.append([locc[j, i] for i, j in V])
                face.append(f)
        for b in range(n - 2):
            for a in range(n - 2 - b):
                # down (a, b): vertices (a+1, b), (a+1, b+1), (a, b+1)
                V = [(a + 1, b), (a + 1, b + 1), (a, b + 1)]
                nodes.append(_p2_nodes(locf, V))
                verts.append([locc[j, i] for i, j in V])
                face.append(f)
    return np.array(nodes, dtype=np.int64), np.array(verts, dtype=np.int64), np.array(face)


def _p2_nodes(locf, V):
    """Fine indices of the vertices (2i, 2j) and edge midpoints of a coarse
    triangle with vertices V (coarse face-local (i, j))."""
    out = [locf[2 * j, 2 * i] for i, j in V]
    for a, b in EDGES:
        (ia, ja), (ib, jb) = V[a], V[b]
        out.append(locf[ja + jb, ia + ib])
    return out


class P2:
    """P2 Laplacian on level l of a macro mesh (unknowns numbered as level
    l + 1), its p-multigrid cycle over the P1 hierarchy `H` (whose finest
    level is l), and the embedding of P1 into P2."""

    def __init__(self, H, face_coef=None, omega=0.6):
        self.H = H
        self.l = H.L
        self.lc = H.levels[H.L]
        self.lv = Level(H.mesh, H.L + 1)
        self.N = self.lv.n_all
        coef = np.ones(H.mesh.F) if face_coef is None else np.asarray(face_coef, dtype=np.float64)
        self.nodes, self.verts, self.face = elements(self.lv, self.lc)
        self.A = assemble_p2(self.lv, self.nodes, coef[self.face])
        self.P = embedding(self.lv, self.lc, self.nodes, self.verts)
        self.diag = self.A.diagonal()
        self.omega = omega

    def apply(self, x):
        y = self.A @ x
        y[self.lv.dirichlet] = 0.0
        return y

    def residual(self, u, f):
        r = f - self.A @ u
        r[self.lv.dirichlet] = 0.0
        return r

    def jacobi(self, u, f, sweeps=1):
        """Damped point Jacobi on the interior points (all updated at once
        from the old values)."""
        ii = self.lv.interior
        for _ in range(sweeps):
            r = f - self.A @ u
            u = u.copy()
            u[ii] += self.omega * r[ii] / self.diag[ii]
        return u

    def restrict(self, r):
        """P1 right-hand side P^T r, zero at Dirichlet points."""
        rc = self.P.T @ r
        rc[self.lc.dirichlet] = 0.0
        return rc

    def prolong_add(self, u, uc):
        c = self.P @ uc
        ii = self.lv.interior
        u = u.copy()
        u[ii] += c[ii]
        return u

    def cycle(self, u, f, nu1=2, nu2=2, vnu=(2, 2)):
        u = self.jacobi(u, f, nu1)
        rc = self.restrict(self.residual(u, f))
        ec = self.H.vcycle(self.l, np.zeros(self.lc.n_all), rc, *vnu)
        u = self.prolong_add(u, ec)
        return self.jacobi(u, f, nu2)

    def res_norm(self, u, f):
        r = self.residual(u, f)
        return float(np.sqrt(r @ r))

    def solve(self, u, f, rtol=1e-8, nu1=2, nu2=2, vnu=(2, 2), max_iters=200):
        """p-multigrid cycles until the residual over interior points has
        dropped by rtol.  Returns (u, history)."""
        r0 = self.res_norm(u, f)
        hist = [r0]
        if r0 == 0.0:
            return u, hist
        for _ in range(max_iters):
            u = self.cycle(u, f, nu1, nu2, vnu)
            hist.append(self.res_norm(u, f))
            if hist[-1] <= rtol * r0:
                break
        return u, hist


def assemble_p2(lv, nodes, coef):
    """Global P2 stiffness: sum over elements of coef_e K_e scattered to the
    element's nodes."""
    rows, cols, vals = [], [], []
    for e in range(len(nodes)):
        idx = nodes[e]
        # vertices of the element: its first three nodes' coordinates
        K = coef[e] * element_stiffness(lv.xy[idx[:3]])
        rows.append(np.repeat(idx, 6))
        cols.append(np.tile(idx, 6))
        vals.append(K.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(lv.n_all, lv.n_all))


def embedding(lv_fine, lv_coarse, nodes, verts):
    """The P1 function of level l with nodal values uc, written in the P2
    basis: P2 nodal values are the P1 function's values there, i.e. uc at
    vertices and the mean of the two end values at edge midpoints.  Sparse
    [n_all(l+1), n_all(l)]; nodes shared by elements are set once."""
    rows, cols, vals = [], [], []
    for e in range(len(nodes)):
        nd, vt = nodes[e], verts[e]
        for a in range(3):
            rows.append(nd[a]); cols.append(vt[a]); vals.append(1.0)
        for k, (a, b) in enumerate(EDGES):
            rows += [nd[3 + k], nd[3 + k]]
            cols += [vt[a], vt[b]]
            vals += [0.5, 0.5]
    rows = np.array(rows); cols = np.array(cols); vals = np.array(vals)
    key = rows * lv_coarse.n_all + cols
    _, first = np.unique(key, return_index=True)
    return sp.csr_matrix((vals[first], (rows[first], cols[first])),
                         shape=(lv_fine.n_all, lv_coarse.n_all))
