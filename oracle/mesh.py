"""Macro mesh, structured refinement and canonical numbering (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references:
  * macro-primitives: one node per mesh vertex, edge and face (sec. 2.1);
  * uniform refinement by connecting edge midpoints, applied recursively, so a
    macro-edge at level l carries n = 2^l + 1 micro-vertices (sec. 1.1, 3.1);
  * each unknown is owned by exactly one primitive (sec. 2.2);
  * a fixed topological (i, j) enumeration per face (sec. 3.2).

Readings where the paper is silent (listed in the design notes):
  * faces are made counter-clockwise by swapping their 2nd and 3rd vertex;
    face-local micro-vertex (i, j) sits at x0 + i/(n-1)(x1-x0) + j/(n-1)(x2-x0);
  * an edge runs from its lower to its higher vertex id, interior points
    k = 1..n-2;
  * canonical order: macro-vertices by id, then edges sorted by (lo, hi) with
    k = 1..n-2, then faces in input order with interior points j-major
    (j = 1..n-3, i = 1..n-2-j);
  * every macro-edge with a single face is a Dirichlet boundary edge, and so
    are its two vertices.
"""
import numpy as np


class MacroMesh:
    """Macro mesh with oriented faces, edge list and boundary flags."""

    def __init__(self, vxy, tri):
        vxy = np.asarray(vxy, dtype=np.float64)
        tri = np.array(tri, dtype=np.int64)
        if vxy.ndim != 2 or vxy.shape[1] != 2 or tri.ndim != 2 or tri.shape[1] != 3:
            raise ValueError("bad mesh arrays")
        for f in range(len(tri)):
            a, b, c = tri[f]
            e1 = vxy[b] - vxy[a]
            e2 = vxy[c] - vxy[a]
            det = e1[0] * e2[1] - e1[1] * e2[0]
            if det == 0.0:
                raise ValueError("degenerate face %d" % f)
            if det < 0.0:
                tri[f] = (a, c, b)
        self.vxy = vxy
        self.tri = tri
        self.V = len(vxy)
        self.F = len(tri)
        faces_of = {}
        for f in range(self.F):
            v0, v1, v2 = tri[f]
            for p, q in ((v0, v1), (v0, v2), (v1, v2)):
                faces_of.setdefault((min(p, q), max(p, q)), []).append(f)
        self.edges = sorted(faces_of)
        self.E = len(self.edges)
        self.edge_id = {key: e for e, key in enumerate(self.edges)}
        self.edge_faces = [faces_of[key] for key in self.edges]
        if any(len(fs) > 2 for fs in self.edge_faces):
            raise ValueError("non-manifold edge")
        self.edge_boundary = np.array([len(fs) == 1 for fs in self.edge_faces])
        self.vertex_boundary = np.zeros(self.V, dtype=bool)
        for e, (a, b) in enumerate(self.edges):
            if self.edge_boundary[e]:
                self.vertex_boundary[a] = True
                self.vertex_boundary[b] = True

    def face_cot(self, f):
        """Cotangents (c0, c1, c2) of face f at its vertices x0, x1, x2.

        c_k = (a.b)/|a x b| with a, b the edge vectors leaving x_k."""
        x = self.vxy[self.tri[f]]
        out = []
        for k in range(3):
            a = x[(k + 1) % 3] - x[k]
            b = x[(k + 2) % 3] - x[k]
            dot = a[0] * b[0] + a[1] * b[1]
            crs = abs(a[0] * b[1] - a[1] * b[0])
            out.append(dot / crs)
        return tuple(out)

    def face_dot(self, f):
        """Dot products a.b at each vertex (exact zero = right angle)."""
        x = self.vxy[self.tri[f]]
        out = []
        for k in range(3):
            a = x[(k + 1) % 3] - x[k]
            b = x[(k + 2) % 3] - x[k]
            out.append(a[0] * b[0] + a[1] * b[1])
        return tuple(out)


class Level:
    """One refinement level: canonical numbering, coordinates, masks.

    Attributes:
      n        micro-vertices per macro-edge (2^l + 1)
      n_all    number of canonical points (every micro-vertex once)
      loc      list over faces of an (n, n) int64 array: loc[f][j, i] is the
               canonical index of face-local point (i, j), -1 outside
      xy       canonical coordinates [n_all, 2]
      dirichlet  boolean mask of Dirichlet points
      kind     0 vertex, 1 edge, 2 face-interior point
      prim     owning primitive id; kidx: edge k, or face-local i; jidx: face j
    """

    def __init__(self, mesh, level):
        if level < 1:
            raise ValueError("level >= 1 required")
        self.mesh = mesh
        self.level = level
        n = 2 ** level + 1
        self.n = n
        V, E, F = mesh.V, mesh.E, mesh.F
        ne = n - 2
        nf = (n - 2) * (n - 3) // 2
        self.n_edge = ne
        self.n_face = nf
        self.edge_base = V
        self.face_base = V + E * ne
        self.n_all = V + E * ne + F * nf

        kind = np.zeros(self.n_all, dtype=np.int8)
        prim = np.zeros(self.n_all, dtype=np.int64)
        kidx = np.zeros(self.n_all, dtype=np.int64)
        jidx = np.zeros(self.n_all, dtype=np.int64)
        xy = np.zeros((self.n_all, 2))
        dirichlet = np.zeros(self.n_all, dtype=bool)

        prim[:V] = np.arange(V)
        xy[:V] = mesh.vxy
        dirichlet[:V] = mesh.vertex_boundary
        t = np.arange(1, n - 1)
        for e, (a, b) in enumerate(mesh.edges):
            s = V + e * ne
            kind[s:s + ne] = 1
            prim[s:s + ne] = e
            kidx[s:s + ne] = t
            xa, xb = mesh.vxy[a], mesh.vxy[b]
            xy[s:s + ne] = xa + np.outer(t / (n - 1), xb - xa)
            dirichlet[s:s + ne] = mesh.edge_boundary[e]

        # face-local (i, j) grids
        J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        inside = I + J <= n - 1
        interior = (I >= 1) & (J >= 1) & (I + J <= n - 2)
        # j-major enumeration of interior points
        order = np.full((n, n), -1, dtype=np.int64)
        order[interior] = np.arange(nf)  # row-major over (j, i) == j-major
        self.loc = []
        for f in range(F):
            v0, v1, v2 = mesh.tri[f]
            loc = np.full((n, n), -1, dtype=np.int64)
            loc[interior] = self.face_base + f * nf + order[interior]
            loc[0, 0] = v0
            loc[0, n - 1] = v1
            loc[n - 1, 0] = v2
            # side j = 0 runs v0 -> v1 with parameter i
            self._fill_side(loc, v0, v1, [(i, 0) for i in range(1, n - 1)])
            # side i = 0 runs v0 -> v2 with parameter j
            self._fill_side(loc, v0, v2, [(0, j) for j in range(1, n - 1)])
            # hypotenuse runs v1 -> v2 with parameter j: point (n-1-j, j)
            self._fill_side(loc, v1, v2, [(n - 1 - j, j) for j in range(1, n - 1)])
            assert (loc[inside] >= 0).all()
            self.loc.append(loc)
            s = self.face_base + f * nf
            kind[s:s + nf] = 2
            prim[s:s + nf] = f
            ii = I[interior]
            jj = J[interior]
            kidx[s:s + nf] = ii
            jidx[s:s + nf] = jj
            x0, x1, x2 = mesh.vxy[v0], mesh.vxy[v1], mesh.vxy[v2]
            xy[s:s + nf] = (x0 + np.outer(ii / (n - 1), x1 - x0)
                            + np.outer(jj / (n - 1), x2 - x0))
        self.kind = kind
        self.prim = prim
        self.kidx = kidx
        self.jidx = jidx
        self.xy = xy
        self.dirichlet = dirichlet
        self.interior = np.flatnonzero(~dirichlet)

    def _fill_side(self, loc, p, q, pts):
        """Canonical ids of the interior points of the face side p -> q.

        pts[t-1] is the face-local (i, j) at parameter t = 1..n-2 from p."""
        n = self.n
        mesh = self.mesh
        e = mesh.edge_id[(min(p, q), max(p, q))]
        base = self.edge_base + e * self.n_edge
        for t, (i, j) in enumerate(pts, start=1):
            k = t if p < q else n - 1 - t
            loc[j, i] = base + k - 1

    def points_per_face(self):
        """All micro-vertices of one refined macro-face, ring included."""
        return self.n * (self.n + 1) // 2

    def interior_count(self):
        return int((~self.dirichlet).sum())
