"""Virtual partition of one refined macro mesh: every macro-primitive is a
separately owned block with explicit ghost copies (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper keeps each macro-primitive's unknowns in an array of its own,
surrounds it with ghost layers holding copies of the neighbouring
primitives' values (sec. 2.2), and refreshes those copies in four directions
before an operator is applied (Alg. 3: vertex to edge, edge to face, face to
edge, edge to vertex).  This module is that storage on the CPU, so that the
global-vector oracle can be checked against it:

  * face block f: an (n, n) array over face-local (i, j), j-major; the
    interior points are owned, the three sides and corners are ghosts;
  * edge block e (vertices a < b): an array over k = 0..n-1 from a to b,
    owned for 0 < k < n-1, ghosts at the two ends, plus, for each adjacent
    face, a ghost row of n-1 values: the face points next to the edge, the
    t-th lying between edge points t and t+1;
  * vertex block v: its own value and a ring of ghosts, the point next to v
    on each incident edge.

The packer moves values between blocks by position alone: the side of a face
an edge occupies, and whether the side runs along the edge's direction.  It
never consults the canonical numbering, so a wrong flip or side shows up as
a wrong ghost.  The canonical numbering is used only to scatter a global
vector into the owned entries, to gather the owned entries back, and to find
a stencil neighbour's slot in the block that applies the row.
"""
import numpy as np


def _side_points(n, side):
    """Face-local (i, j) of the points of a face side, t = 0..n-1 from the
    side's first vertex: side 0 runs v0 -> v1 (j = 0), side 1 v0 -> v2
    (i = 0), side 2 v1 -> v2 (i + j = n - 1)."""
    t = np.arange(n)
    if side == 0:
        return t, np.zeros(n, np.int64)
    if side == 1:
        return np.zeros(n, np.int64), t
    return n - 1 - t, t


def _near_points(n, side):
    """Face-local (i, j) of the face points next to a side, t = 0..n-2: the
    t-th touches side points t and t+1."""
    t = np.arange(n - 1)
    if side == 0:
        return t, np.ones(n - 1, np.int64)
    if side == 1:
        return np.ones(n - 1, np.int64), t
    return n - 2 - t, t


class Partition:
    """Blocks, packer and blockwise operator application of one level."""

    def __init__(self, lv):
        self.lv = lv
        m = lv.mesh
        n = self.n = lv.n
        # the side of each face an edge occupies and the side's direction
        self.face_sides = []                      # per face: [(edge, forward)] for sides 0, 1, 2
        self.edge_adj = [[] for _ in range(m.E)]  # per edge: [(face, side, forward)]
        for f in range(m.F):
            v0, v1, v2 = (int(x) for x in m.tri[f])
            sides = []
            for s, (p, q) in enumerate(((v0, v1), (v0, v2), (v1, v2))):
                e = m.edge_id[(min(p, q), max(p, q))]
                sides.append((e, p < q))
                self.edge_adj[e].append((f, s, p < q))
            self.face_sides.append(sides)
        # vertex rings: incident edges and which end of the edge the vertex is
        self.vert_ring = [[] for _ in range(m.V)]
        for e, (a, b) in enumerate(m.edges):
            self.vert_ring[a].append((e, 1))       # point next to a: k = 1
            self.vert_ring[b].append((e, n - 2))   # point next to b: k = n-2
        self.face = [np.zeros((n, n)) for _ in range(m.F)]
        self.edge = [np.zeros(n) for _ in range(m.E)]
        self.edge_ghost = [np.zeros((len(self.edge_adj[e]), n - 1)) for e in range(m.E)]
        self.vert = np.zeros(m.V)
        self.vert_ghost = [np.zeros(len(r)) for r in self.vert_ring]

    # ---------------------------------------------------------- owned data
    def scatter(self, u):
        """Owned entries from a global vector; ghosts are left alone."""
        lv = self.lv
        m = lv.mesh
        n = self.n
        self.vert[:] = u[:m.V]
        for e in range(m.E):
            s = lv.edge_base + e * lv.n_edge
            self.edge[e][1:n - 1] = u[s:s + lv.n_edge]
        J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        interior = (I >= 1) & (J >= 1) & (I + J <= n - 2)
        for f in range(m.F):
            self.face[f][interior] = u[lv.loc[f][interior]]

    def gather(self, y_blocks):
        """Global vector from per-block owned results (see apply)."""
        lv = self.lv
        out = np.zeros(lv.n_all)
        for ids, vals in y_blocks:
            out[ids] = vals
        return out

    # --------------------------------------------------------------- packer
    def sync(self):
        """Refresh every ghost copy from its owner, in the paper's order:
        vertex -> edge ends, edge -> face sides, face -> edge ghost rows,
        edge -> vertex rings."""
        m = self.lv.mesh
        n = self.n
        for e, (a, b) in enumerate(m.edges):          # (a) vertex -> edge
            self.edge[e][0] = self.vert[a]
            self.edge[e][n - 1] = self.vert[b]
        for f in range(m.F):                          # (b) edge -> face
            for s, (e, fwd) in enumerate(self.face_sides[f]):
                i, j = _side_points(n, s)
                self.face[f][j, i] = self.edge[e] if fwd else self.edge[e][::-1]
        for e in range(m.E):                          # (c) face -> edge
            for g, (f, s, fwd) in enumerate(self.edge_adj[e]):
                i, j = _near_points(n, s)
                row = self.face[f][j, i]
                self.edge_ghost[e][g] = row if fwd else row[::-1]
        for v in range(m.V):                          # (d) edge -> vertex
            for q, (e, k) in enumerate(self.vert_ring[v]):
                self.vert_ghost[v][q] = self.edge[e][k]

    # ------------------------------------------ canonical ids of local slots
    def slot_ids(self):
        """For every block, the canonical id each local slot (owned or ghost)
        stands for, laid out as flat_local() lays out its values.  Built from
        the numbering, independently of the packer, to check it."""
        lv = self.lv
        m = lv.mesh
        n = self.n
        out = {"vert": [], "edge": [], "face": []}
        for v in range(m.V):
            ring = [lv.edge_base + e * lv.n_edge + k - 1 for e, k in self.vert_ring[v]]
            out["vert"].append(np.array([v] + ring, np.int64))
        for e, (a, b) in enumerate(m.edges):
            own = np.concatenate([[a], lv.edge_base + e * lv.n_edge + np.arange(n - 2), [b]])
            rows = []
            for f, s, fwd in self.edge_adj[e]:
                i, j = _near_points(n, s)
                ids = lv.loc[f][j, i]
                rows.append(ids if fwd else ids[::-1])
            out["edge"].append(np.concatenate([own] + rows).astype(np.int64))
        for f in range(m.F):
            out["face"].append(lv.loc[f].ravel().copy())
        return out

    def flat_local(self, kind, p):
        """The local values of one block, slots in slot_ids() order."""
        if kind == "vert":
            return np.concatenate([[self.vert[p]], self.vert_ghost[p]])
        if kind == "edge":
            return np.concatenate([self.edge[p]] + list(self.edge_ghost[p]))
        return self.face[p].ravel()

    # ---------------------------------------------------- blockwise operator
    def apply(self, A):
        """y = A u row by row, each owned row evaluated inside its block from
        the block's local values only (owned and ghost), its terms summed in
        the order of the CSR row.  Raises if a stencil neighbour has no slot
        in the block (an incomplete ghost layer)."""
        A = A.tocsr()
        lv = self.lv
        m = lv.mesh
        n = self.n
        ids = self.slot_ids()
        res = []
        blocks = []
        for v in range(m.V):
            blocks.append(("vert", v, np.array([v], np.int64)))
        for e in range(m.E):
            blocks.append(("edge", e, lv.edge_base + e * lv.n_edge + np.arange(n - 2)))
        for f in range(m.F):
            s = lv.face_base + f * lv.n_face
            blocks.append(("face", f, np.arange(s, s + lv.n_face)))
        for kind, p, own in blocks:
            if own.size == 0:
                continue
            where = {int(c): s for s, c in enumerate(ids[kind][p]) if c >= 0}
            local = self.flat_local(kind, p)
            y = np.zeros(own.size)
            for r, gi in enumerate(own):
                lo, hi = A.indptr[gi], A.indptr[gi + 1]
                acc = 0.0
                for c, w in zip(A.indices[lo:hi], A.data[lo:hi]):
                    if int(c) not in where:
                        raise KeyError("row %d of %s %d: neighbour %d has no local slot" % (gi, kind, p, c))
                    acc += w * local[where[int(c)]]
                y[r] = acc
            res.append((own, y))
        return self.gather(res)
