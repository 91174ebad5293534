"""Element-by-element P1 assembly (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states that a stencil entry is a non-zero of one row of the
stiffness matrix (sec. 1.1 and 4.2) and that a conventional solver obtains the
matrix through element matrices (sec. 4.2).  The oracle therefore assembles
the global matrix from P1 element matrices over every micro-triangle, which
is the plain definition of the operator the HIP stencils apply.

Element matrices (exact integration; reading for the variable coefficient:
the P1 interpolant of k integrates to the vertex mean k_T on each triangle):
  stiffness  K_T[a, b] = k_T * |T| * grad(phi_a) . grad(phi_b)
  mass       M_T[a, b] = |T| / 12 * (1 + delta_ab)
"""
import numpy as np
import scipy.sparse as sp


def micro_triangles(lv):
    """Canonical vertex triples of every micro-triangle of every face.

    Up triangles {(i,j), (i+1,j), (i,j+1)} for i+j <= n-2 and down triangles
    {(i+1,j), (i+1,j+1), (i,j+1)} for i+j <= n-3, per face (sec. 3.1: each
    refinement splits a triangle into four congruent ones, so a face at level
    l holds (n-1)^2 of them)."""
    n = lv.n
    J, I = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    up = I + J <= n - 2
    dn = I + J <= n - 3
    iu, ju = I[up], J[up]
    idn, jdn = I[dn], J[dn]
    tris = []
    for loc in lv.loc:
        tris.append(np.stack([loc[ju, iu], loc[ju, iu + 1], loc[ju + 1, iu]], 1))
        tris.append(np.stack([loc[jdn, idn + 1], loc[jdn + 1, idn + 1],
                              loc[jdn + 1, idn]], 1))
    t = np.concatenate(tris)
    assert (t >= 0).all()
    return t


def micro_triangle_faces(lv):
    """Macro-face of each micro-triangle, in the order of micro_triangles."""
    n = lv.n
    per_face = (n - 1) * n // 2 + (n - 2) * (n - 1) // 2     # up + down = (n - 1)^2
    return np.repeat(np.arange(len(lv.loc)), per_face)


def element_matrices(xy, tris, kappa=None, elem_coef=None):
    """Stiffness and mass element matrices, shape [T, 3, 3] each.  kappa:
    nodal coefficient (vertex mean per triangle); elem_coef: an extra factor
    per triangle (a coefficient constant on each macro-face)."""
    p = xy[tris]                       # [T, 3, 2]
    x, y = p[..., 0], p[..., 1]
    # b_a = y_{a+1} - y_{a+2}, c_a = x_{a+2} - x_{a+1}; grad phi_a = (b_a, c_a)/(2|T|)
    b = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], 1)
    c = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], 1)
    area = 0.5 * (b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0])
    area = np.abs(area)
    K = (b[:, :, None] * b[:, None, :] + c[:, :, None] * c[:, None, :]) / (4.0 * area)[:, None, None]
    if kappa is not None:
        kbar = kappa[tris].mean(axis=1)
        K = K * kbar[:, None, None]
    if elem_coef is not None:
        K = K * np.asarray(elem_coef, dtype=np.float64)[:, None, None]
    M = (area / 12.0)[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None]
    return K, M


def assemble(lv, kappa=None, want=("A", "M"), face_coef=None):
    """Global (Neumann, i.e. before any boundary treatment) stiffness A and
    mass M as CSR matrices over all canonical points.  face_coef[F]: a
    coefficient constant on each macro-face multiplying the stiffness,
    -div(face_coef grad u) (with kappa: -div(face_coef kappa grad u))."""
    tris = micro_triangles(lv)
    ec = None if face_coef is None else np.asarray(face_coef, dtype=np.float64)[micro_triangle_faces(lv)]
    K, M = element_matrices(lv.xy, tris, kappa, ec)
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    out = {}
    if "A" in want:
        out["A"] = sp.csr_matrix((K.ravel(), (rows, cols)), shape=(lv.n_all, lv.n_all))
    if "M" in want:
        out["M"] = sp.csr_matrix((M.ravel(), (rows, cols)), shape=(lv.n_all, lv.n_all))
    return out


def inject(lv_fine, lv_coarse, x_fine):
    """Coarse nodal values by injection: coarse (I, J) is fine (2I, 2J)."""
    out = np.zeros(lv_coarse.n_all)
    for locf, locc in zip(lv_fine.loc, lv_coarse.loc):
        nc = lv_coarse.n
        J, I = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
        m = I + J <= nc - 1
        out[locc[J[m], I[m]]] = x_fine[locf[2 * J[m], 2 * I[m]]]
    return out


def rows_at(lv, points, x, kappa=None):
    """(A x)[points] for the Neumann stiffness A, from the element matrices of
    the micro-triangles incident to each point only (the same definition as
    `assemble`, for levels too large to assemble).  kappa(xy) -> nodal k at
    the given coordinates, or None for k = 1."""
    n = lv.n
    points = np.asarray(points, dtype=np.int64)
    want = {int(p): k for k, p in enumerate(points)}
    # every occurrence (face, i, j) of the wanted points
    occ = []
    for f, loc in enumerate(lv.loc):
        J, I = np.nonzero(np.isin(loc, points))
        for j, i in zip(J.tolist(), I.tolist()):
            occ.append((f, i, j))
    tris = set()
    for f, i, j in occ:
        loc = lv.loc[f]
        for a, b in ((i, j), (i - 1, j), (i, j - 1)):           # up triangles
            if a >= 0 and b >= 0 and a + b <= n - 2:
                tris.add(tuple(sorted((loc[b, a], loc[b, a + 1], loc[b + 1, a]))) + (0,) +
                         (loc[b, a], loc[b, a + 1], loc[b + 1, a]))
        for a, b in ((i - 1, j - 1), (i - 1, j), (i, j - 1)):   # down triangles
            if a >= 0 and b >= 0 and a + b <= n - 3:
                tris.add(tuple(sorted((loc[b, a + 1], loc[b + 1, a + 1], loc[b + 1, a]))) + (1,) +
                         (loc[b, a + 1], loc[b + 1, a + 1], loc[b + 1, a]))
    T = np.array([t[4:] for t in tris], dtype=np.int64)
    kap = None
    if kappa is not None:
        uniq = np.unique(T)
        kv = np.zeros(lv.n_all)
        kv[uniq] = kappa(lv.xy[uniq])
        kap = kv
    K, _ = element_matrices(lv.xy, T, kap)
    out = np.zeros(len(points))
    for t in range(len(T)):
        for a in range(3):
            k = want.get(int(T[t, a]))
            if k is not None:
                out[k] += K[t, a] @ x[T[t]]
    return out
