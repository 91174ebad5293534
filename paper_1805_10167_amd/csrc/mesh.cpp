// Host setup of the macro-primitive graph (sec. 2.1), the per-level field
// layouts (sec. 3.1, 3.2) and the ghost-copy table (sec. 2.2, 3.3).
//
// Layout of one field of level l (n = 2^l + 1 points per macro-edge):
//   faces    : F blocks; face-local row j (n - j points, i = 0..n-1-j) starts
//              at row_off[j], rows padded to 16 elements.  The ring (i = 0,
//              j = 0, i + j = n - 1) holds ghost copies of edge and vertex
//              values, the interior is owned by the face.
//   edges    : E blocks of [main: k = 0..n-1 | ghost row 0 | ghost row 1].
//              k = 1..n-2 are owned, k = 0 and n-1 are copies of the two
//              vertices.  Ghost row s holds the n-1 near-row points of the
//              edge's s-th face, in edge order: g[m] touches edge points m
//              and m+1.
//   vertices : V blocks of [value | one copy per incident edge of the edge
//              point next to the vertex].
// Every copy has exactly one owner; the ghost table lists (copy, owner)
// offset pairs grouped by the kind of owner, so that each smoother stage can
// refresh just the copies of the points it changed.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>

#include "hhg_mesh.hpp"

namespace hhg {

void MeshData::side_point(int side, int t, int d, int n, int& i, int& j) {
    if (side == 0) {
        i = t; j = d;
    } else if (side == 1) {
        i = d; j = t;
    } else {
        i = n - 1 - d - t; j = t;
    }
}

static inline int side_start(int side) { return side == 2 ? 1 : 0; }
static inline int side_end(int side) { return side == 0 ? 1 : 2; }
static inline int side_third(int side) { return 2 - side; }

Owner MeshData::owner_of(int f, int i, int j, int n) const {
    const FaceInfo& fi = faces[f];
    Owner o{0, 0, 0, i, j};
    if (i == 0 && j == 0) { o.kind = 0; o.prim = fi.vtx[0]; return o; }
    if (i == n - 1 && j == 0) { o.kind = 0; o.prim = fi.vtx[1]; return o; }
    if (i == 0 && j == n - 1) { o.kind = 0; o.prim = fi.vtx[2]; return o; }
    int side = -1, t = 0;
    if (j == 0) { side = 0; t = i; }
    else if (i == 0) { side = 1; t = j; }
    else if (i + j == n - 1) { side = 2; t = j; }
    if (side < 0) { o.kind = 2; o.prim = f; return o; }
    o.kind = 1;
    o.prim = fi.edge[side];
    o.k = fi.rev[side] ? n - 1 - t : t;
    return o;
}

int64_t MeshData::owner_offset(const LevelHost& L, const Owner& o) const {
    if (o.kind == 0) return vert_off(L, o.prim, 0);
    if (o.kind == 1) return edge_off(L, o.prim, o.k);
    return face_off(L, o.prim, o.i, o.j);
}

int64_t MeshData::canonical_of(const LevelHost& L, const Owner& o) const {
    const int n = L.n;
    if (o.kind == 0) return o.prim;
    if (o.kind == 1) {
        if (o.k == 0) return edges[o.prim].a;
        if (o.k == n - 1) return edges[o.prim].b;
        return L.can_edge_base + (int64_t)o.prim * (n - 2) + (o.k - 1);
    }
    const int64_t nfi = (int64_t)(n - 2) * (n - 3) / 2;
    const int64_t j = o.j;
    const int64_t before = (j - 1) * (n - 2) - (j - 1) * j / 2;
    return L.can_face_base + (int64_t)o.prim * nfi + before + (o.i - 1);
}

std::string MeshData::build(const double* in_vxy, int nv, const int32_t* in_tri,
                            int nf, int max_level, int coarse_level) {
    if (nv < 3 || nf < 1) return "need at least 3 vertices and 1 face";
    if (max_level < 1 || max_level > MAXLEVEL) return "max_level must be in 1..12";
    if (coarse_level < 1 || coarse_level > max_level)
        return "coarse_level must be in 1..max_level";
    V = nv; F = nf; L = max_level; lc = coarse_level;
    vxy.assign(in_vxy, in_vxy + 2 * (size_t)nv);
    tri.resize(nf);
    for (int f = 0; f < nf; ++f) {
        int a = in_tri[3 * f], b = in_tri[3 * f + 1], c = in_tri[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            return "vertex id out of range in face " + std::to_string(f);
        if (a == b || b == c || a == c) return "repeated vertex in face " + std::to_string(f);
        double e1x = vxy[2 * b] - vxy[2 * a], e1y = vxy[2 * b + 1] - vxy[2 * a + 1];
        double e2x = vxy[2 * c] - vxy[2 * a], e2y = vxy[2 * c + 1] - vxy[2 * a + 1];
        double det = e1x * e2y - e1y * e2x;
        if (det == 0.0 || !std::isfinite(det)) return "zero-area face " + std::to_string(f);
        if (det < 0.0) std::swap(b, c);   // make it counter-clockwise
        tri[f] = {a, b, c};
    }
    // macro-edges from sorted vertex pairs (sec. 2.1)
    std::map<std::pair<int, int>, std::vector<int>> faces_of;
    for (int f = 0; f < nf; ++f)
        for (int s = 0; s < 3; ++s) {
            int p = tri[f][side_start(s)], q = tri[f][side_end(s)];
            faces_of[{std::min(p, q), std::max(p, q)}].push_back(f);
        }
    E = (int)faces_of.size();
    std::map<std::pair<int, int>, int> edge_id;
    edge_v.clear();
    edges.assign(E, EdgeInfo{});
    for (auto& kv : faces_of) {
        if (kv.second.size() > 2) return "non-manifold macro-edge";
        int e = (int)edge_v.size();
        edge_id[kv.first] = e;
        edge_v.push_back({kv.first.first, kv.first.second});
        EdgeInfo& ei = edges[e];
        ei.a = kv.first.first;
        ei.b = kv.first.second;
        ei.nf = (int)kv.second.size();
        ei.boundary = ei.nf == 1;
    }
    std::vector<char> vbnd(V, 0);
    for (int e = 0; e < E; ++e)
        if (edges[e].boundary) { vbnd[edges[e].a] = 1; vbnd[edges[e].b] = 1; }

    faces.assign(F, FaceInfo{});
    nfaces2 = 0;
    std::vector<int> fill(E, 0);
    for (int f = 0; f < F; ++f) {
        FaceInfo& fi = faces[f];
        double x[3][2];
        for (int k = 0; k < 3; ++k) {
            fi.vtx[k] = tri[f][k];
            x[k][0] = vxy[2 * tri[f][k]];
            x[k][1] = vxy[2 * tri[f][k] + 1];
        }
        double dots[3];
        for (int k = 0; k < 3; ++k) {
            const double* p0 = x[k];
            const double* p1 = x[(k + 1) % 3];
            const double* p2 = x[(k + 2) % 3];
            double ax = p1[0] - p0[0], ay = p1[1] - p0[1];
            double bx = p2[0] - p0[0], by = p2[1] - p0[1];
            double dot = ax * bx + ay * by;
            double crs = std::fabs(ax * by - ay * bx);
            dots[k] = dot;
            fi.cot[k] = dot / crs;
        }
        {
            double e1x = x[1][0] - x[0][0], e1y = x[1][1] - x[0][1];
            double e2x = x[2][0] - x[0][0], e2y = x[2][1] - x[0][1];
            fi.area = 0.5 * std::fabs(e1x * e2y - e1y * e2x);
        }
        // multicolour ordering: 3 colours (i - j) mod 3, or the parity rule of
        // the lattice direction whose weight vanishes at an exact right angle
        if (dots[0] == 0.0) { fi.colour_rule = 1; fi.ncolours = 2; }
        else if (dots[1] == 0.0) { fi.colour_rule = 2; fi.ncolours = 2; }
        else if (dots[2] == 0.0) { fi.colour_rule = 3; fi.ncolours = 2; }
        else { fi.colour_rule = 0; fi.ncolours = 3; }
        if (fi.ncolours == 2) ++nfaces2;
        for (int s = 0; s < 3; ++s) {
            int p = tri[f][side_start(s)], q = tri[f][side_end(s)];
            int e = edge_id[{std::min(p, q), std::max(p, q)}];
            EdgeInfo& ei = edges[e];
            int slot = fill[e]++;
            fi.edge[s] = e;
            fi.slot[s] = slot;
            fi.rev[s] = (p != ei.a);
            fi.bside[s] = ei.boundary;
            ei.face[slot] = f;
            ei.side[slot] = s;
            ei.rev[slot] = fi.rev[s];
            int la = (p == ei.a) ? side_start(s) : side_end(s);
            int lb = (p == ei.a) ? side_end(s) : side_start(s);
            ei.cA[slot] = fi.cot[side_third(s)];
            ei.cL[slot] = fi.cot[la];
            ei.cH[slot] = fi.cot[lb];
            ei.area[slot] = fi.area;
        }
        for (int k = 0; k < 3; ++k) fi.bvtx[k] = vbnd[fi.vtx[k]];
    }
    // macro-vertices and their incident edges (sorted by edge id)
    verts.assign(V, VertexInfo{});
    maxdeg = 0;
    for (int e = 0; e < E; ++e) {
        for (int end = 0; end < 2; ++end) {
            int v = end == 0 ? edges[e].a : edges[e].b;
            VertexInfo& vi = verts[v];
            if (vi.deg >= MAXDEG) return "a macro-vertex has more than 16 macro-edges";
            edges[e].vslot[end] = vi.deg;
            vi.edge[vi.deg] = e;
            vi.at_a[vi.deg] = (end == 0);
            vi.nfe[vi.deg] = edges[e].nf;
            vi.deg++;
        }
    }
    for (int v = 0; v < V; ++v) {
        VertexInfo& vi = verts[v];
        vi.boundary = vbnd[v];
        if (vi.deg == 0) return "isolated vertex " + std::to_string(v);
        maxdeg = std::max(maxdeg, vi.deg);
        for (int q = 0; q < vi.deg; ++q) {
            const EdgeInfo& ei = edges[vi.edge[q]];
            for (int s = 0; s < 2; ++s) {
                vi.partner[q][s] = -1;
                vi.cA[q][s] = 0.0;
                vi.area[q][s] = 0.0;
                if (s >= ei.nf) continue;
                const FaceInfo& fi = faces[ei.face[s]];
                // the other side of that face through v
                int other = -1;
                for (int s2 = 0; s2 < 3; ++s2) {
                    if (s2 == ei.side[s]) continue;
                    if (tri[ei.face[s]][side_start(s2)] == v || tri[ei.face[s]][side_end(s2)] == v)
                        other = fi.edge[s2];
                }
                int pslot = -1;
                for (int q2 = 0; q2 < vi.deg; ++q2)
                    if (vi.edge[q2] == other) pslot = q2;
                if (pslot < 0) return "inconsistent vertex fan";
                vi.partner[q][s] = pslot;
                vi.cA[q][s] = ei.cA[s];
                vi.area[q][s] = ei.area[s];
            }
        }
    }
    // ghost-row corner entries held by the other edge of each face
    for (int e = 0; e < E; ++e) {
        EdgeInfo& ei = edges[e];
        for (int s = 0; s < 2; ++s)
            for (int end = 0; end < 2; ++end) {
                ei.cg_edge[s][end] = -1;
                ei.cg_slot[s][end] = 0;
                ei.cg_first[s][end] = 0;
                if (s >= ei.nf) continue;
                const int f = ei.face[s];
                const int v = end == 0 ? ei.a : ei.b;
                for (int s2 = 0; s2 < 3; ++s2) {
                    if (s2 == ei.side[s]) continue;
                    if (tri[f][side_start(s2)] != v && tri[f][side_end(s2)] != v) continue;
                    const int e2 = faces[f].edge[s2];
                    if (edges[e2].boundary) continue;
                    ei.cg_edge[s][end] = e2;
                    ei.cg_slot[s][end] = faces[f].slot[s2];
                    ei.cg_first[s][end] = (edges[e2].a == v);
                }
            }
    }
    // faces around each vertex and the vertex's corner in them
    for (int v = 0; v < V; ++v) verts[v].nfc = 0;
    for (int f = 0; f < F; ++f)
        for (int c = 0; c < 3; ++c) {
            VertexInfo& vi = verts[tri[f][c]];
            if (vi.nfc >= MAXDEG) return "a macro-vertex has more than 16 macro-faces";
            vi.fc_face[vi.nfc] = f;
            vi.fc_corner[vi.nfc] = c;
            vi.nfc++;
        }
    iedges.clear();
    iverts.clear();
    for (int e = 0; e < E; ++e)
        if (!edges[e].boundary) iedges.push_back(e);
    for (int v = 0; v < V; ++v)
        if (!verts[v].boundary) iverts.push_back(v);

    faces0 = faces;
    edges0 = edges;
    verts0 = verts;
    face_coef.assign(F, 1.0);
    sfaces.clear();
    sedges.clear();
    sverts.clear();
    lv.assign(L + 1, LevelHost{});
    for (int l = 1; l <= L; ++l) build_level(l);
    build_coarse();
    return "";
}

std::string MeshData::set_face_coef(const double* coef) {
    for (int f = 0; f < F; ++f)
        if (!(coef[f] > 0.0) || !std::isfinite(coef[f]))
            return "face coefficient " + std::to_string(f) + " is not a positive finite number";
    face_coef.assign(coef, coef + F);
    faces = faces0;
    edges = edges0;
    verts = verts0;
    // every stiffness weight is -1/2 cot(angle) of one micro-triangle, and
    // every micro-triangle lies in one macro-face: scale by that face's value
    for (int f = 0; f < F; ++f)
        for (int k = 0; k < 3; ++k) faces[f].cot[k] *= face_coef[f];
    for (int e = 0; e < E; ++e)
        for (int s = 0; s < edges[e].nf; ++s) {
            const double c = face_coef[edges[e].face[s]];
            edges[e].cA[s] *= c;
            edges[e].cL[s] *= c;
            edges[e].cH[s] *= c;
        }
    for (int v = 0; v < V; ++v) {
        VertexInfo& vi = verts[v];
        for (int q = 0; q < vi.deg; ++q) {
            const EdgeInfo& ei = edges[vi.edge[q]];
            for (int s = 0; s < ei.nf; ++s) vi.cA[q][s] *= face_coef[ei.face[s]];
        }
    }
    return "";
}

namespace {

// P1 element contributions of one triangle with vertex positions P[3] (any
// orientation) to the row stencils of the point at local vertex r; slot[a]
// is the stencil neighbour of local vertex a.  Definitions (per triangle T):
//   A[r][b]   = mu |T| grad phi_r . grad phi_b
//   BX[r][b]  = -int_T psi_r d phi_b / dx = -|T|/3 d phi_b / dx  (pressure row r)
//   BXT[r][a] = BX[a][r] = -|T|/3 d phi_r / dx                    (velocity row r)
//   C[r][b]   = delta h_T^2 / mu |T| grad phi_r . grad phi_b, h_T the longest edge
//   m        += |T| / (3 mu)  (lumped 1/mu-weighted mass; the caller adds
//               a multiple of C's centre weight afterwards)
template <int W>
void add_triangle(const double P[3][2], int r, const int slot[3], double mu, double delta,
                  double (&w)[SB_N][W], double& m) {
    double gx[3], gy[3];
    for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        gx[a] = P[a1][1] - P[a2][1];
        gy[a] = P[a2][0] - P[a1][0];
    }
    const double two_a = gx[0] * gy[1] - gx[1] * gy[0];   // twice the signed area
    const double area = 0.5 * std::fabs(two_a);
    for (int a = 0; a < 3; ++a) {
        gx[a] /= two_a;
        gy[a] /= two_a;
    }
    double h2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3;
        const double dx = P[a1][0] - P[a][0], dy = P[a1][1] - P[a][1];
        h2 = std::max(h2, dx * dx + dy * dy);
    }
    for (int b = 0; b < 3; ++b) {
        const double st = area * (gx[r] * gx[b] + gy[r] * gy[b]);
        w[SB_A][slot[b]] += mu * st;
        w[SB_C][slot[b]] += delta * h2 / mu * st;
        w[SB_BX][slot[b]] += -area / 3.0 * gx[b];
        w[SB_BY][slot[b]] += -area / 3.0 * gy[b];
        w[SB_BXT][slot[b]] += -area / 3.0 * gx[r];
        w[SB_BYT][slot[b]] += -area / 3.0 * gy[r];
    }
    m += area / (3.0 * mu);
}

}  // namespace

namespace {

// P2 element stiffness of a face from the cotangents c[k] of its angles
// (already times the face coefficient), local order v0 v1 v2 m01 m12 m02.
// With the P1 element stiffness K1 (K1_aa = (c_b + c_c) / 2, K1_ab = -c_c / 2,
// c the angle opposite the edge ab) and the integrals of barycentric
// monomials over the triangle, the quadratic basis lam_a (2 lam_a - 1) and
// 4 lam_a lam_b gives:
//   vertex a, itself:          K1_aa
//   vertices a, b:             -K1_ab / 3          =  c_c / 6
//   vertex a, midpoint of ab:  4 K1_ab / 3         = -2 c_c / 3
//   vertex a, midpoint of bc:  0
//   midpoint of ab, itself:    8 (K1_aa + K1_bb + K1_ab) / 3 = 4 (c_0 + c_1 + c_2) / 3
//   midpoints of ab and bc:    8 K1_ac / 3         = -4 c_b / 3 (b the shared vertex)
void p2_element(const double c[3], double K[6][6]) {
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) K[a][b] = 0.0;
    const int mid[3][3] = {{-1, 3, 5}, {3, -1, 4}, {5, 4, -1}};   // node of the midpoint of (a, b)
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, cc = (a + 2) % 3;
        K[a][a] = 0.5 * (c[b] + c[cc]);
        K[a][b] = K[b][a] = c[cc] / 6.0;
        // vertex a with the midpoints of its two edges
        K[a][mid[a][b]] = K[mid[a][b]][a] = -2.0 * c[cc] / 3.0;
        K[a][mid[a][cc]] = K[mid[a][cc]][a] = -2.0 * c[b] / 3.0;
    }
    const double all = c[0] + c[1] + c[2];
    for (int m = 3; m < 6; ++m) K[m][m] = 4.0 * all / 3.0;
    // pairs of midpoints and their shared vertex: (m01, m12) at 1, (m01, m02) at 0, (m12, m02) at 2
    const int pr[3][3] = {{3, 4, 1}, {3, 5, 0}, {4, 5, 2}};
    for (auto& q : pr) K[q[0]][q[1]] = K[q[1]][q[0]] = -4.0 * c[q[2]] / 3.0;
}

// Level-(l+1) offsets of the local nodes of the up (kind 0) and down (kind
// 1) element of coarse position (a, b), relative to (2a, 2b).
const int P2OFF[2][6][2] = {{{0, 0}, {2, 0}, {0, 2}, {1, 0}, {1, 1}, {0, 1}},
                            {{2, 2}, {0, 2}, {2, 0}, {1, 2}, {1, 1}, {2, 1}}};

// Row of point (I, J) of a face with nc coarse points per side, restricted
// to the face's own elements: weight per neighbour offset, summed over the
// elements containing the point.
std::map<std::pair<int, int>, double> p2_face_row(const double K[6][6], int nc, int I, int J) {
    std::map<std::pair<int, int>, double> w;
    for (int kind = 0; kind < 2; ++kind)
        for (int r = 0; r < 6; ++r) {
            const int dx = I - P2OFF[kind][r][0], dy = J - P2OFF[kind][r][1];
            if ((dx & 1) || (dy & 1)) continue;
            const int a = dx / 2, b = dy / 2;
            if (a < 0 || b < 0 || a + b > nc - 2 - kind) continue;
            for (int q = 0; q < 6; ++q)
                w[{2 * a + P2OFF[kind][q][0] - I, 2 * b + P2OFF[kind][q][1] - J}] += K[r][q];
        }
    return w;
}

}  // namespace

std::string MeshData::p2_tables() {
    p2faces.assign(F, P2Face{});
    p2ediag.assign(2 * (size_t)E, 0.0);
    p2vdiag.assign(V, 0.0);
    // stencil slots: C E W N S SE NW, and the vertex type's far vertices
    const int hex[7][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, -1}, {-1, 1}};
    const int far[6][2] = {{2, 0}, {-2, 0}, {0, 2}, {0, -2}, {2, -2}, {-2, 2}};
    const int NC = 65, NV = 2 * NC - 1;   // a face large enough that interior rows see all elements
    std::vector<std::array<double, 3>> corner_d(F);
    std::vector<std::array<std::array<double, 2>, 3>> side_d(F);
    for (int f = 0; f < F; ++f) {
        P2Face& t = p2faces[f];
        p2_element(faces[f].cot, t.K);
        for (int type = 0; type < 4; ++type) {
            auto w = p2_face_row(t.K, NC, 16 + (type & 1), 16 + (type >> 1));
            for (int s = 0; s < 7; ++s) {
                auto it = w.find({hex[s][0], hex[s][1]});
                t.hex[type][s] = it == w.end() ? 0.0 : it->second;
                if (it != w.end()) w.erase(it);
            }
            for (int s = 0; s < 6; ++s) {
                auto it = w.find({far[s][0], far[s][1]});
                const double v = it == w.end() ? 0.0 : it->second;
                if (it != w.end()) w.erase(it);
                if (type == 0) t.far[s] = v;
                else if (v != 0.0) return "P2 edge stencil reaches a far vertex";
            }
            for (auto& kv : w)
                if (kv.second != 0.0) return "P2 stencil has an unexpected neighbour";
        }
        // diagonals of the face's share of boundary rows: side points (even,
        // odd parameter) and corners
        for (int side = 0; side < 3; ++side)
            for (int par = 0; par < 2; ++par) {
                int I, J;
                side_point(side, 2 + par, 0, NV, I, J);
                side_d[f][side][par] = p2_face_row(t.K, NC, I, J)[{0, 0}];
            }
        corner_d[f][0] = p2_face_row(t.K, NC, 0, 0)[{0, 0}];
        corner_d[f][1] = p2_face_row(t.K, NC, NV - 1, 0)[{0, 0}];
        corner_d[f][2] = p2_face_row(t.K, NC, 0, NV - 1)[{0, 0}];
    }
    for (int e = 0; e < E; ++e) {
        const EdgeInfo& ei = edges[e];
        for (int par = 0; par < 2; ++par)
            for (int s = 0; s < ei.nf; ++s) p2ediag[2 * e + par] += side_d[ei.face[s]][ei.side[s]][par];
    }
    for (int v = 0; v < V; ++v) {
        const VertexInfo& vi = verts[v];
        for (int c = 0; c < vi.nfc; ++c) p2vdiag[v] += corner_d[vi.fc_face[c]][vi.fc_corner[c]];
    }
    return "";
}

void MeshData::fv_tables() {
    fvfaces.assign(F, FvFace{});
    auto X = [&](int v, int c) { return vxy[2 * v + c]; };
    for (int f = 0; f < F; ++f) {
        FvFace& t = fvfaces[f];
        const int* v = tri[f].data();
        // side vectors taken as differences of the two vertices of the side,
        // so that the two faces of a macro-edge get exactly negated normals
        double s0[2], s1[2], s2[2];
        for (int c = 0; c < 2; ++c) {
            s0[c] = X(v[1], c) - X(v[0], c);
            s1[c] = X(v[2], c) - X(v[0], c);
            s2[c] = X(v[2], c) - X(v[1], c);
            t.x0[c] = X(v[0], c);
            t.e1[c] = s0[c];
            t.e2[c] = s1[c];
        }
        // counter-clockwise face: the outside of the up cell is to the right
        // of side 0 and of side 2, and to the left of side 1
        t.nb[0] = s0[1];  t.nb[1] = -s0[0];
        t.nl[0] = -s1[1]; t.nl[1] = s1[0];
        t.nd[0] = s2[1];  t.nd[1] = -s2[0];
        t.area = 0.5 * std::fabs(s0[0] * s1[1] - s0[1] * s1[0]);
        for (int s = 0; s < 3; ++s) {
            const FaceInfo& fi = faces[f];
            const EdgeInfo& ei = edges[fi.edge[s]];
            t.nbr_face[s] = -1;
            t.nbr_side[s] = 0;
            t.nbr_flip[s] = 0;
            if (ei.nf < 2) continue;
            const int other = 1 - fi.slot[s];
            t.nbr_face[s] = ei.face[other];
            t.nbr_side[s] = ei.side[other];
            t.nbr_flip[s] = (ei.rev[other] != fi.rev[s]) ? 1 : 0;
        }
    }
}

void MeshData::stokes_tables(double delta) {
    sfaces.assign(F, StokesFace{});
    sedges.assign(E, StokesEdge{});
    sverts.assign(V, StokesVert{});
    auto X = [&](int v, int c) { return vxy[2 * v + c]; };
    // face interior: the six micro-triangles around (i, j), as offsets
    // (di, dj); neighbour slots C, E, W, N, S, SE, NW
    const int off[7][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, -1}, {-1, 1}};
    auto slot_of = [&](int di, int dj) {
        for (int t = 0; t < 7; ++t)
            if (off[t][0] == di && off[t][1] == dj) return t;
        return -1;
    };
    const int ftri[6][3][2] = {
        {{0, 0}, {1, 0}, {0, 1}},      // up (i, j)
        {{-1, 0}, {0, 0}, {-1, 1}},    // up (i-1, j)
        {{0, -1}, {1, -1}, {0, 0}},    // up (i, j-1)
        {{0, -1}, {0, 0}, {-1, 0}},    // down (i-1, j-1)
        {{0, 0}, {0, 1}, {-1, 1}},     // down (i-1, j)
        {{1, -1}, {1, 0}, {0, 0}}};    // down (i, j-1)
    for (int f = 0; f < F; ++f) {
        const int* t = tri[f].data();
        const double e1[2] = {X(t[1], 0) - X(t[0], 0), X(t[1], 1) - X(t[0], 1)};
        const double e2[2] = {X(t[2], 0) - X(t[0], 0), X(t[2], 1) - X(t[0], 1)};
        StokesFace& sf = sfaces[f];
        for (int k = 0; k < 6; ++k) {
            double P[3][2];
            int slot[3], r = -1;
            for (int a = 0; a < 3; ++a) {
                const int di = ftri[k][a][0], dj = ftri[k][a][1];
                P[a][0] = di * e1[0] + dj * e2[0];
                P[a][1] = di * e1[1] + dj * e2[1];
                slot[a] = slot_of(di, dj);
                if (di == 0 && dj == 0) r = a;
            }
            add_triangle<7>(P, r, slot, face_coef[f], delta, sf.w, sf.m);
        }
    }
    // edge point k: slots 0 = k, 1 = k-1, 2 = k+1, 3 + 2s = g_s[k-1],
    // 4 + 2s = g_s[k]; on face s with third vertex c the micro-triangle
    // (k, k+1, g_s[k]) is the macro-face (a, b, c) scaled and translated
    for (int e = 0; e < E; ++e) {
        const EdgeInfo& ei = edges[e];
        const double de[2] = {X(ei.b, 0) - X(ei.a, 0), X(ei.b, 1) - X(ei.a, 1)};
        StokesEdge& se = sedges[e];
        for (int s = 0; s < ei.nf; ++s) {
            const int f = ei.face[s];
            int c = -1;
            for (int k = 0; k < 3; ++k)
                if (tri[f][k] != ei.a && tri[f][k] != ei.b) c = tri[f][k];
            const double ds[2] = {X(c, 0) - X(ei.a, 0), X(c, 1) - X(ei.a, 1)};
            // positions relative to point k of the slots used on this side
            double pos[7][2] = {{0, 0}, {-de[0], -de[1]}, {de[0], de[1]}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
            pos[3 + 2 * s][0] = ds[0] - de[0];
            pos[3 + 2 * s][1] = ds[1] - de[1];
            pos[4 + 2 * s][0] = ds[0];
            pos[4 + 2 * s][1] = ds[1];
            const int etri[3][3] = {{0, 2, 4 + 2 * s}, {1, 0, 3 + 2 * s}, {0, 4 + 2 * s, 3 + 2 * s}};
            for (int k = 0; k < 3; ++k) {
                double P[3][2];
                int r = -1;
                for (int a = 0; a < 3; ++a) {
                    P[a][0] = pos[etri[k][a]][0];
                    P[a][1] = pos[etri[k][a]][1];
                    if (etri[k][a] == 0) r = a;
                }
                add_triangle<7>(P, r, etri[k], face_coef[f], delta, se.w, se.m);
            }
        }
    }
    // vertex: one corner micro-triangle per incident face, (v, ring q1,
    // ring q2) with q1, q2 the face's two edges through v
    for (int v = 0; v < V; ++v) {
        const VertexInfo& vi = verts[v];
        StokesVert& sv = sverts[v];
        for (int c = 0; c < vi.nfc; ++c) {
            const int f = vi.fc_face[c], cr = vi.fc_corner[c];
            const int sa = cr == 2 ? 1 : 0, sb = cr == 0 ? 1 : 2;   // sides through the corner
            int slot[3] = {0, -1, -1};
            double P[3][2] = {{0, 0}, {0, 0}, {0, 0}};
            const int es[2] = {faces[f].edge[sa], faces[f].edge[sb]};
            for (int k = 0; k < 2; ++k) {
                for (int q = 0; q < vi.deg; ++q)
                    if (vi.edge[q] == es[k]) slot[1 + k] = 1 + q;
                const EdgeInfo& ek = edges[es[k]];
                const int other = ek.a == v ? ek.b : ek.a;
                P[1 + k][0] = X(other, 0) - X(v, 0);
                P[1 + k][1] = X(other, 1) - X(v, 1);
            }
            add_triangle<1 + MAXDEG>(P, 0, slot, face_coef[f], delta, sv.w, sv.m);
        }
    }
    // Pressure block of the preconditioner: the exact Schur complement of the
    // stabilised system is B A^-1 B^T + C.  The lumped mass stands for the
    // first term; the diagonal of C, weighted by kStabWeight because C's
    // largest eigenvalues are several times its diagonal on oscillating
    // pressures, stands for the second.  The centre is slot 0 everywhere.
    constexpr double kStabWeight = 4.0;
    for (StokesFace& sf : sfaces) sf.m += kStabWeight * sf.w[SB_C][0];
    for (StokesEdge& se : sedges) se.m += kStabWeight * se.w[SB_C][0];
    for (StokesVert& sv : sverts) sv.m += kStabWeight * sv.w[SB_C][0];
}

void MeshData::build_level(int level) {
    LevelHost& H = lv[level];
    const int n = (1 << level) + 1;
    H.level = level;
    H.n = n;
    H.row_off.assign(n + 1, 0);
    for (int j = 0; j < n; ++j) H.row_off[j + 1] = H.row_off[j] + (int32_t)pad_up(n - j, PAD);
    H.face_stride = H.row_off[n];
    H.ghost_off = (int32_t)pad_up(n, PAD);
    H.ghost_stride = (int32_t)pad_up(n - 1, PAD);
    H.edge_stride = H.ghost_off + 2 * (int64_t)H.ghost_stride;
    H.vert_stride = pad_up(1 + maxdeg, PAD);
    H.face_base = 0;
    H.edge_base = (int64_t)F * H.face_stride;
    H.vert_base = H.edge_base + (int64_t)E * H.edge_stride;
    H.total = pad_up(H.vert_base + (int64_t)V * H.vert_stride, 64);
    const int64_t nfi = (int64_t)(n - 2) * (n - 3) / 2;
    H.n_all = V + (int64_t)E * (n - 2) + (int64_t)F * nfi;
    H.n_int = (int64_t)iverts.size() + (int64_t)iedges.size() * (n - 2) + (int64_t)F * nfi;
    H.can_edge_base = V;
    H.can_face_base = V + (int64_t)E * (n - 2);

    // tiles of TILE_I x TILE_J face-local points covering the whole face
    H.tiles.clear();
    for (int tj = 0; tj * TILE_J <= n - 1; ++tj)
        for (int ti = 0; ti * TILE_I <= n - 1; ++ti)
            if (ti * TILE_I + tj * TILE_J <= n - 1) H.tiles.push_back(make_int2(ti, tj));

    // smoother tiles over the whole face triangle (ring included), column by
    // column so that consecutive tiles are vertical neighbours
    const int halos[GS_NHALO] = {GS_H, GS_HE, GS_HR};
    for (int e = 0; e < GS_NHALO; ++e)
        for (int t = 0; t < 2; ++t) {
            const int ti_w = gs_tile_width(halos[e]), tj_h = t ? GS_TJ16 : (e == 2 ? GS_TJR : GS_TJ);
            std::vector<int2>& tl = H.gs_tl[e][t];
            tl.clear();
            for (int ti = 0; ti * ti_w <= n - 1; ++ti)
                for (int tj = 0; tj * tj_h <= n - 1; ++tj)
                    if (ti * ti_w + tj * tj_h <= n - 1) tl.push_back(make_int2(ti, tj));
        }

    // learned-smoother output tiles that contain interior points
    H.net_tiles.clear();
    for (int ti = 0; ti * NET_TI <= n - 3; ++ti)
        for (int tj = 0; tj * NET_TJ <= n - 3; ++tj) {
            int imin = std::max(ti * NET_TI, 1), jmin = std::max(tj * NET_TJ, 1);
            if (imin + jmin <= n - 2) H.net_tiles.push_back(make_int2(ti, tj));
        }
    // learned-step strip pieces (NET_TI columns, net_strip_rows rows) that
    // contain interior points; a strip's pieces are consecutive, bottom to top
    H.net_strips.clear();
    const int sr = net_strip_rows(n);
    for (int ti = 0; ti * NET_TI <= n - 3; ++ti)
        for (int tj = 0; tj * sr <= n - 3; ++tj) {
            int imin = std::max(ti * NET_TI, 1), jmin = std::max(tj * sr, 1);
            if (imin + jmin <= n - 2) H.net_strips.push_back(make_int2(ti, tj));
        }

    // ghost table
    std::vector<std::tuple<int, int64_t, int64_t>> ent;
    auto cls_of = [&](const Owner& o) {
        if (o.kind == 0) return (int)G_VERT;
        if (o.kind == 1) return (o.k % 2 == 0) ? (int)G_EEVEN : (int)G_EODD;
        return (int)G_FACE;
    };
    for (int f = 0; f < F; ++f) {
        // ring: corners and the three sides
        int ci[3] = {0, n - 1, 0}, cj[3] = {0, 0, n - 1};
        for (int c = 0; c < 3; ++c) {
            Owner o = owner_of(f, ci[c], cj[c], n);
            ent.emplace_back(G_VERT, face_off(H, f, ci[c], cj[c]), owner_offset(H, o));
        }
        for (int s = 0; s < 3; ++s)
            for (int t = 1; t <= n - 2; ++t) {
                int i, j;
                side_point(s, t, 0, n, i, j);
                Owner o = owner_of(f, i, j, n);
                ent.emplace_back(cls_of(o), face_off(H, f, i, j), owner_offset(H, o));
            }
    }
    for (int e = 0; e < E; ++e) {
        const EdgeInfo& ei = edges[e];
        ent.emplace_back(G_VERT, edge_off(H, e, 0), vert_off(H, ei.a, 0));
        ent.emplace_back(G_VERT, edge_off(H, e, n - 1), vert_off(H, ei.b, 0));
        if (ei.boundary) continue;
        for (int s = 0; s < ei.nf; ++s) {
            for (int g = 0; g <= n - 2; ++g) {
                int t = ei.rev[s] ? n - 2 - g : g;
                int i, j;
                side_point(ei.side[s], t, 1, n, i, j);
                Owner o = owner_of(ei.face[s], i, j, n);
                ent.emplace_back(cls_of(o), ghost_off(H, e, s, g), owner_offset(H, o));
            }
        }
    }
    for (int v = 0; v < V; ++v) {
        const VertexInfo& vi = verts[v];
        for (int q = 0; q < vi.deg; ++q) {
            int k = vi.at_a[q] ? 1 : n - 2;
            ent.emplace_back(G_EODD, vert_off(H, v, 1 + q), edge_off(H, vi.edge[q], k));
        }
    }
    std::stable_sort(ent.begin(), ent.end());
    H.gdst.resize(ent.size());
    H.gsrc.resize(ent.size());
    for (int c = 0; c <= G_NCLS; ++c) H.gcls[c] = 0;
    for (size_t x = 0; x < ent.size(); ++x) {
        H.gdst[x] = std::get<1>(ent[x]);
        H.gsrc[x] = std::get<2>(ent[x]);
        H.gcls[std::get<0>(ent[x]) + 1] = (int64_t)x + 1;
    }
    for (int c = 1; c <= G_NCLS; ++c) H.gcls[c] = std::max(H.gcls[c], H.gcls[c - 1]);
}

void MeshData::build_coarse() {
    const LevelHost& H = lv[lc];
    const int n = H.n;
    Wc = std::max(7, 1 + maxdeg);
    std::vector<int32_t> compact(H.n_all, -1);
    c_owner.clear(); c_kind.clear(); c_prim.clear(); c_pa.clear(); c_pb.clear();
    auto add = [&](const Owner& o) {
        compact[canonical_of(H, o)] = (int32_t)c_owner.size();
        c_owner.push_back(owner_offset(H, o));
        c_kind.push_back(o.kind);
        c_prim.push_back(o.prim);
        c_pa.push_back(o.kind == 1 ? o.k : o.i);
        c_pb.push_back(o.j);
    };
    // canonical order restricted to interior points
    for (int v = 0; v < V; ++v)
        if (!verts[v].boundary) add(Owner{0, v, 0, 0, 0});
    for (int e = 0; e < E; ++e)
        if (!edges[e].boundary)
            for (int k = 1; k <= n - 2; ++k) add(Owner{1, e, k, 0, 0});
    for (int f = 0; f < F; ++f)
        for (int j = 1; j <= n - 3; ++j)
            for (int i = 1; i <= n - 2 - j; ++i) add(Owner{2, f, 0, i, j});
    Nc = (int32_t)c_owner.size();
    c_cols.assign((size_t)Nc * Wc, -1);
    auto col = [&](const Owner& o) { return compact[canonical_of(H, o)]; };
    auto edge_pt = [&](int e, int k) {
        if (k == 0) return Owner{0, edges[e].a, 0, 0, 0};
        if (k == n - 1) return Owner{0, edges[e].b, 0, 0, 0};
        return Owner{1, e, k, 0, 0};
    };
    for (int p = 0; p < Nc; ++p) {
        int32_t* cp = &c_cols[(size_t)p * Wc];
        cp[0] = p;
        if (c_kind[p] == 0) {
            const VertexInfo& vi = verts[c_prim[p]];
            for (int q = 0; q < vi.deg; ++q)
                cp[1 + q] = col(edge_pt(vi.edge[q], vi.at_a[q] ? 1 : n - 2));
        } else if (c_kind[p] == 1) {
            int e = c_prim[p], k = c_pa[p];
            const EdgeInfo& ei = edges[e];
            cp[1] = col(edge_pt(e, k - 1));
            cp[2] = col(edge_pt(e, k + 1));
            for (int s = 0; s < 2; ++s)
                for (int d = 0; d < 2; ++d) {
                    int g = k - 1 + d;
                    int t = ei.rev[s] ? n - 2 - g : g;
                    int i, j;
                    side_point(ei.side[s], t, 1, n, i, j);
                    cp[3 + 2 * s + d] = col(owner_of(ei.face[s], i, j, n));
                }
        } else {
            int f = c_prim[p], i = c_pa[p], j = c_pb[p];
            const int di[6] = {1, -1, 0, 0, 1, -1}, dj[6] = {0, 0, 1, -1, -1, 1};
            for (int w = 0; w < 6; ++w) cp[1 + w] = col(owner_of(f, i + di[w], j + dj[w], n));
        }
    }
}

}  // namespace hhg
