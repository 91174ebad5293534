"""Equal-order P1-P1 Stokes with pressure stabilisation, block-diagonal
multigrid preconditioner and preconditioned MINRES (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's energy-transport example (sec. 5.2) solves incompressible Stokes
flow, discretised with equal-order P1 elements for velocity and pressure plus
a Petrov-Galerkin pressure stabilisation, and sec. 4.3 names preconditioned
MINRES as the solver of symmetric indefinite systems, with multigrid usable
as a preconditioner.  The paper gives no parameters; the readings are:

  * viscous term: -div(mu grad u) for each velocity component (the paper's
    -Laplace u, with a viscosity mu constant on each macro-face);
  * weak form: a(u, v) + b(v, p) = (f, v), b(u, q) - c(p, q) = 0 with
      a(u, v) = sum_c int mu grad u_c . grad v_c,
      b(v, q) = -int q div v,
      c(p, q) = delta sum_T (h_T^2 / mu_T) int_T grad p . grad q,
    h_T the longest edge of micro-triangle T and delta = 1/12 (the
    Brezzi-Pitkaranta form of the stabilisation);
  * velocity: zero on every boundary macro-edge and its vertices (sec. 5.2
    uses homogeneous Dirichlet velocity); pressure: a P1 unknown at every
    point, boundary included; its constant is the kernel of the operator and
    is fixed by a zero mean weighted with the preconditioner's pressure
    block, which the MINRES iterates keep by construction;
  * preconditioner: blockdiag(V_A, V_A, S^-1) with V_A one V(nu1, nu2) cycle
    of the mu-weighted Laplacian from a zero start (forward stages before,
    backward stages after the coarse correction: a symmetric operator) and
    S the diagonal matrix m + sigma_C diag(C): m the lumped mass matrix
    weighted with 1/mu (the usual spectral equivalent of the pressure Schur
    complement B A^-1 B^T), plus the diagonal of the stabilisation block,
    which the Schur complement of the stabilised system also contains
    (S_exact = B A^-1 B^T + C).  C's eigenvalues reach several times its
    diagonal on oscillating pressures, hence the weight sigma_C = 4 (a
    measured choice: on the 64-face annulus at level 5 with the 1:100
    viscosity jump, sigma_C = 0, 1, 2, 3, 5, 8 took 197, 166, 155, 149,
    143, 140 MINRES steps to 1e-8);
  * MINRES: the Lanczos process of the preconditioned operator with a QR
    factorisation of its tridiagonal matrix by Givens rotations; the stopping
    test is on the residual measured in the norm of the inverse
    preconditioner, relative to its start.

A Stokes vector is one array [u_x | u_y | p] of 3 n_all values in the
canonical order of each component.
"""
import numpy as np
import scipy.sparse as sp

from .assemble import micro_triangle_faces, micro_triangles
from .mg import Hierarchy

DELTA = 1.0 / 12.0
SIGMA_C = 4.0


def face_viscosity(mesh, r_jump=0.775, mu_in=1.0, mu_out=100.0):
    """mu per macro-face (an input of the problem, from the shared input
    generators): a jump of mu_out / mu_in across the middle ring."""
    import hhg_inputs
    return hhg_inputs.face_viscosity(mesh.vxy, mesh.tri, r_jump, mu_in, mu_out)


def stokes_element_matrices(xy, tris, mu_t, delta=DELTA):
    """Element matrices of every micro-triangle, shape [T, 3, 3] each:
    K (mu-weighted stiffness), Bx and By (rows: pressure test function a,
    columns: velocity trial function b; B[a, b] = -int_T psi_a d_c phi_b),
    C (stabilisation) and the lumped 1/mu-weighted mass per vertex [T, 3]."""
    p = xy[tris]
    x, y = p[..., 0], p[..., 1]
    # d phi_a / dx = (y_{a+1} - y_{a+2}) / (2 signed area), d phi_a / dy = (x_{a+2} - x_{a+1}) / (2 signed area)
    gx = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], 1)
    gy = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], 1)
    two_a = gx[:, 0] * gy[:, 1] - gx[:, 1] * gy[:, 0]
    area = 0.5 * np.abs(two_a)
    gx = gx / two_a[:, None]
    gy = gy / two_a[:, None]
    stiff = area[:, None, None] * (gx[:, :, None] * gx[:, None, :] + gy[:, :, None] * gy[:, None, :])
    K = mu_t[:, None, None] * stiff
    # int_T psi_a = |T| / 3 and the derivative of phi_b is constant on T
    Bx = -(area / 3.0)[:, None, None] * np.broadcast_to(gx[:, None, :], (len(tris), 3, 3))
    By = -(area / 3.0)[:, None, None] * np.broadcast_to(gy[:, None, :], (len(tris), 3, 3))
    e = np.stack([p[:, 1] - p[:, 2], p[:, 2] - p[:, 0], p[:, 0] - p[:, 1]], 1)
    h2 = (e ** 2).sum(-1).max(axis=1)
    C = (delta * h2 / mu_t)[:, None, None] * stiff
    mlump = np.repeat((area / (3.0 * mu_t))[:, None], 3, axis=1)
    return K, Bx, By, C, mlump


def assemble_stokes(lv, mu_face, delta=DELTA):
    """Global blocks over all canonical points (no boundary treatment):
    A (mu-Laplacian), Bx, By (pressure rows, velocity columns), C, and the
    lumped pressure mass m (vector)."""
    tris = micro_triangles(lv)
    mu_t = np.asarray(mu_face, dtype=np.float64)[micro_triangle_faces(lv)]
    K, Bx, By, C, ml = stokes_element_matrices(lv.xy, tris, mu_t, delta)
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    N = lv.n_all
    csr = lambda E: sp.csr_matrix((E.ravel(), (rows, cols)), shape=(N, N))   # noqa: E731
    m = np.bincount(tris.ravel(), weights=ml.ravel(), minlength=N)
    return {"A": csr(K), "Bx": csr(Bx), "By": csr(By), "C": csr(C), "m": m}


class Stokes:
    """The Stokes system of one macro mesh at level L, its block
    preconditioner (multigrid hierarchy down to level lc) and MINRES."""

    def __init__(self, mesh, L, lc=2, mu_face=None, delta=DELTA, nu=(2, 2)):
        mu_face = np.ones(mesh.F) if mu_face is None else np.asarray(mu_face, dtype=np.float64)
        self.mu_face = mu_face
        self.L, self.nu = L, nu
        self.H = Hierarchy(mesh, L, lc, face_coef=mu_face)
        self.lv = self.H.levels[L]
        self.N = self.lv.n_all
        b = assemble_stokes(self.lv, mu_face, delta)
        self.A, self.Bx, self.By, self.C, self.m = b["A"], b["Bx"], b["By"], b["C"], b["m"]
        self.s = self.m + SIGMA_C * self.C.diagonal()   # pressure block of the preconditioner
        self.dir = self.lv.dirichlet

    def split(self, x):
        N = self.N
        return x[:N], x[N:2 * N], x[2 * N:]

    def apply(self, x):
        """y = K x: velocity rows zero at Dirichlet points (the velocity
        there is zero and not an unknown), pressure rows everywhere."""
        ux, uy, p = self.split(x)
        yx = self.A @ ux + self.Bx.T @ p
        yy = self.A @ uy + self.By.T @ p
        yp = self.Bx @ ux + self.By @ uy - self.C @ p
        yx[self.dir] = 0.0
        yy[self.dir] = 0.0
        return np.concatenate([yx, yy, yp])

    def precond(self, r):
        """z = P^-1 r: one V(nu1, nu2) cycle per velocity component from
        zero, the pressure divided by m + sigma_C diag(C)."""
        rx, ry, rp = self.split(r)
        zx = self.H.vcycle(self.L, np.zeros(self.N), rx, *self.nu)
        zy = self.H.vcycle(self.L, np.zeros(self.N), ry, *self.nu)
        return np.concatenate([zx, zy, rp / self.s])

    def rhs(self, fx, fy):
        """Load vector of nodal body-force values: (M f_x, M f_y, 0), zero at
        Dirichlet velocity points."""
        bx = self.H.M[self.L] @ fx
        by = self.H.M[self.L] @ fy
        bx[self.dir] = 0.0
        by[self.dir] = 0.0
        return np.concatenate([bx, by, np.zeros(self.N)])

    def matrix(self):
        """K as one sparse matrix over all 3 N entries (Dirichlet velocity
        rows and columns replaced by the identity), for direct solves."""
        keep = sp.diags((~self.dir).astype(float))
        I_d = sp.diags(self.dir.astype(float))
        A = keep @ self.A @ keep + I_d
        BxT = keep @ self.Bx.T
        ByT = keep @ self.By.T
        Z = sp.csr_matrix((self.N, self.N))
        return sp.bmat([[A, Z, BxT], [Z, A, ByT], [BxT.T, ByT.T, -self.C]]).tocsr()


def minres(apply, precond, b, x0, rtol=1e-8, max_iters=500, dot=np.dot):
    """Preconditioned MINRES for symmetric K and symmetric positive definite
    P (sec. 4.3).  Returns (x, history of the P^-1-norm of the residual).

    Lanczos on P^-1 K in the P^-1 inner product: v_1 = r_0 / beta_1,
    z_k = P^-1 v_k, alpha_k = z_k . K z_k,
    beta_{k+1} v_{k+1} = K z_k - alpha_k v_k - beta_k v_{k-1}, so that
    K Z_k = V_{k+1} T_k with T_k tridiagonal ((k+1) x k).  The iterate
    x_k = x_0 + Z_k y_k minimises |beta_1 e_1 - T_k y|, which is the P^-1-norm
    of b - K x_k.  T_k is reduced to upper triangular form by one Givens
    rotation per step; its columns (eps, delta, gamma) give the directions
    w_k = (z_k - delta w_{k-1} - eps w_{k-2}) / gamma, and the rotated right-
    hand side gives the step length and the residual norm."""
    x = x0.copy()
    r = b - apply(x)
    y = precond(r)
    beta = np.sqrt(dot(r, y))
    hist = [beta]
    if beta == 0.0:
        return x, hist
    v_old = np.zeros_like(b)
    v = r / beta
    z = y / beta
    w_old = np.zeros_like(b)
    w_older = np.zeros_like(b)
    c_old, s_old, c, s = 1.0, 0.0, 1.0, 0.0       # rotations k-2 and k-1
    eta = beta
    beta_k = 0.0                                  # beta_k, sub-diagonal entry of column k
    for _ in range(max_iters):
        Kz = apply(z)
        alpha = dot(z, Kz)
        r_next = Kz - alpha * v - beta_k * v_old
        y_next = precond(r_next)
        beta_next = np.sqrt(max(dot(r_next, y_next), 0.0))
        # previous rotations on column k: entries (rows k-2, k-1, k)
        eps = s_old * beta_k
        dbar = c_old * beta_k
        delta = c * dbar + s * alpha
        gbar = -s * dbar + c * alpha
        gamma = np.hypot(gbar, beta_next)
        c_new, s_new = gbar / gamma, beta_next / gamma
        w = (z - delta * w_old - eps * w_older) / gamma
        x += (c_new * eta) * w
        eta = -s_new * eta
        hist.append(abs(eta))
        if abs(eta) <= rtol * hist[0] or beta_next == 0.0:
            break
        w_older, w_old = w_old, w
        c_old, s_old, c, s = c, s, c_new, s_new
        v_old, v = v, r_next / beta_next
        z = y_next / beta_next
        beta_k = beta_next
    return x, hist


def pressure_mean_free(st, x):
    """x with its pressure shifted to a zero mean weighted with the
    preconditioner's pressure block s (the kernel direction of K removed)."""
    x = x.copy()
    p = x[2 * st.N:]
    p -= (st.s @ p) / st.s.sum()
    return x
