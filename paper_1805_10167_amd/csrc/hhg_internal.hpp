// Internal data structures of the HHG P1 library: macro-primitive tables
// (sec. 2.1-2.3 of the paper), per-level layouts (sec. 3.1-3.2) and the ghost
// copy table that realises the process-local direct-copy path of the
// communication layer (sec. 2.4, 3.3).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace hhg {

constexpr int MAXDEG = 16;      // incident macro-edges per macro-vertex
constexpr int MAXLEVEL = 12;
constexpr int PAD = 16;         // row/segment padding in elements
constexpr int TILE_I = 64;      // generic face tile: 64 (i) x 4 (j) points
constexpr int TILE_J = 4;
// fused smoother tile: TI x TJ updated points plus a halo of H on every
// side, so that an LDS row holds TI + 2 H = GS_W values (three per lane of a
// wave); H = GS_H for the sweep, GS_HE for the sweep that also forms the
// residual, GS_HR for the sweep that also restricts it (residuals one point
// beyond the tile on its low-i and low-j sides)
constexpr int GS_W = 192;
constexpr int GS_H = 3;
constexpr int GS_HE = 4;
constexpr int GS_HR = 5;
constexpr int GS_NHALO = 3;   // tile lists kept per level: halo GS_H, GS_HE, GS_HR
constexpr int GS_TJ = 24;
constexpr int GS_TJ16 = 16;   // tile height of the variable-coefficient FP64 smoother
constexpr int GS_TJR = 22;    // tile height of the restricting sweep (GS_HR), so that its
                              // tile has as many LDS rows as the residual sweep's
constexpr int gs_tile_width(int halo) { return GS_W - 2 * halo; }
// learned-smoother tile: NET_TI x NET_TJ output points
constexpr int NET_TI = 58;
constexpr int NET_TJ = 12;
// fused learned step: one wave streams the output rows of a piece of a
// NET_TI-wide strip; tall pieces on large levels (fewer start-up rows per
// row), short ones on small levels (a wave's chain of row steps is their
// latency)
inline int net_strip_rows(int n) { return n >= 1025 ? 32 : (n >= 513 ? 16 : 8); }
constexpr int COARSE_DENSE_MAXN = 2048;   // coarse systems solved with a stored inverse
constexpr int NET_NW = 224;     // weights: W1[16][7] then W2[16][7]

inline int64_t pad_up(int64_t x, int64_t p) { return (x + p - 1) / p * p; }

// Ghost-copy classes, by the kind of the owning point.  A stage of the
// smoother refreshes only the copies of the points it changed.
enum GhostClass { G_VERT = 0, G_EEVEN = 1, G_EODD = 2, G_FACE = 3, G_NCLS = 4 };
enum { GM_VERT = 1, GM_EEVEN = 2, GM_EODD = 4, GM_FACE = 8, GM_ALL = 15 };

// Face sides: 0 = v0->v1 (j = 0), 1 = v0->v2 (i = 0), 2 = v1->v2 (i+j = n-1).
struct FaceInfo {
    double cot[3];        // cotangent of the angle at v0, v1, v2
    double area;          // macro-face area
    int32_t vtx[3];
    int32_t edge[3];      // macro-edge on each side
    int32_t slot[3];      // which ghost row of that edge this face fills
    int32_t rev[3];       // 1: edge parameter k runs against the side
    int32_t bside[3];     // side is a Dirichlet edge
    int32_t bvtx[3];      // vertex is Dirichlet
    int32_t colour_rule;  // 0: (i-j) mod 3, 1: (i+j) mod 2, 2: i mod 2, 3: j mod 2
    int32_t ncolours;     // 3, or 2 for a face with an exact right angle
};

// A macro-edge runs from a to b (a < b).  For each adjacent face s the
// micro-triangle (k, k+1, g_s[k]) is a translate of the scaled macro-face,
// with angles cL at k (= angle at a), cH at k+1 (= angle at b) and cA at the
// apex g_s[k] (the third vertex).  g_s[m] is the near-row point adjacent to
// edge points m and m+1.
struct EdgeInfo {
    int32_t a, b;
    int32_t nf;           // adjacent faces: 1 = boundary (Dirichlet), 2 = interior
    int32_t boundary;
    int32_t face[2];
    int32_t side[2];
    int32_t rev[2];
    double cA[2], cL[2], cH[2];
    double area[2];       // macro-face areas
    int32_t vslot[2];     // ghost slot of this edge at vertex a and at vertex b
    // In face s the edge point next to vertex a (end 0) or b (end 1) is the
    // first/last entry of the ghost row of the other edge of that face
    // through the vertex: edge id (-1 if it is a boundary edge), its ghost
    // row, and 1 if that entry is position 0 (else n-2).
    int32_t cg_edge[2][2];
    int32_t cg_slot[2][2];
    int32_t cg_first[2][2];
    int32_t pad_;
};

// A macro-vertex keeps one ghost copy per incident edge: the edge point one
// micro-edge away from it.  For edge q and each face s of that edge, the
// corner micro-triangle (v, q-point, partner-point) has angle cA opposite
// the micro-edge v -> q-point.
struct VertexInfo {
    int32_t deg;
    int32_t boundary;
    int32_t edge[MAXDEG];
    int32_t at_a[MAXDEG];
    int32_t nfe[MAXDEG];
    int32_t partner[MAXDEG][2];
    double cA[MAXDEG][2];
    double area[MAXDEG][2];
    int32_t nfc;                  // incident faces and the vertex's corner in each
    int32_t fc_face[MAXDEG];
    int32_t fc_corner[MAXDEG];    // 0: (0,0), 1: (n-1,0), 2: (0,n-1)
    int32_t pad_;
};

// Equal-order P1-P1 Stokes stencils (blocks of the saddle-point operator),
// at the unit scale of the macro-face (one micro-step = one macro-edge):
// level l scales the divergence/gradient blocks by 2^-l and the pressure
// stabilisation and lumped pressure mass by 4^-l; the viscous block is
// level independent.  Row stencils of one point over its neighbours:
//   A   mu-weighted stiffness, velocity row, velocity neighbours
//   BX  divergence (x part), pressure row, velocity neighbours
//   BY  divergence (y part), pressure row, velocity neighbours
//   BXT gradient (x part) = transpose of BX, velocity row, pressure neighbours
//   BYT gradient (y part), velocity row, pressure neighbours
//   C   pressure stabilisation, pressure row, pressure neighbours
enum { SB_A = 0, SB_BX = 1, SB_BY = 2, SB_BXT = 3, SB_BYT = 4, SB_C = 5, SB_N = 6 };
// face-interior point: neighbours C, E, W, N, S, SE, NW of face-local (i, j)
struct StokesFace { double w[SB_N][7]; double m; };
// edge point k: k, k-1, k+1, then for face s = 0, 1 the near-row points
// g_s[k-1], g_s[k] (zero weights for the missing face of a boundary edge)
struct StokesEdge { double w[SB_N][7]; double m; };
// vertex: the vertex, then ring slot q (edge point next to it on edge q)
struct StokesVert { double w[SB_N][1 + MAXDEG]; double m; };

// Finite-volume cells of a macro-face (the micro-triangles) at unit scale,
// one micro-step = one macro-edge: outward normal times length of the three
// edges of an up cell {(i,j), (i+1,j), (i,j+1)}: bottom (along side 0),
// left (along side 1), diagonal (along side 2); a down cell is the point
// reflection, with the negated normals.  Level l scales normals by 2^-l and
// the cell area by 4^-l.  Per side, the face across it (-1 on the domain
// boundary), that face's side, and whether position t along this side is
// position n-2-t on the other.  x0, e1, e2 give point coordinates,
// x(i, j) = x0 + 2^-l (i e1 + j e2).
struct FvFace {
    double nb[2], nl[2], nd[2];
    double area;
    double x0[2], e1[2], e2[2];
    int32_t nbr_face[3];
    int32_t nbr_side[3];
    int32_t nbr_flip[3];
    int32_t pad_;
};

// P2 stencils of one macro-face (Laplacian times the face coefficient) on
// the level-(l+1) layout that holds P2 fields of level l: per point type
// (0 vertex, 1 i-direction edge, 2 j-direction edge, 3 diagonal edge) the
// weights of the hexagonal neighbours C, E, W, N, S, SE, NW; the vertex
// type's couplings with the vertices two steps away ((2,0), (-2,0), (0,2),
// (0,-2), (2,-2), (-2,2)); and the element matrix (local order v0 v1 v2
// m01 m12 m02) for the faces' shares of boundary rows.
struct P2Face {
    double hex[4][7];
    double far[6];
    double K[6][6];
};

// Per-level view passed to kernels by value.
struct LevelDev {
    int32_t level, n;
    int32_t F, E, V;
    int32_t ghost_off, ghost_stride, vert_stride;
    int32_t ntiles, n_iedges, n_iverts, n_net_tiles, n_net_strips, net_sr;
    int32_t n_gs_tl[GS_NHALO][2];    // smoother tiles per face, [halo][GS_TJ16 rows]
    int64_t face_stride, edge_stride;
    int64_t face_base, edge_base, vert_base, total;
    int64_t gcls[G_NCLS + 1];
    int64_t can_edge_base, can_face_base, n_all;
    double inv4l;                     // 1 / 4^level: micro/macro area ratio
    const int32_t* row_off;           // [n + 1] start of row j inside a face
    const int2* tiles;                // 64 x 4 tiles covering the whole face
    const int2* gs_tl[GS_NHALO][2];   // smoother tiles covering the whole face
    const int2* net_tiles;            // learned-smoother tiles meeting the interior
    const int2* net_strips;           // learned-step strip pieces meeting the interior
    const FaceInfo* faces;
    const EdgeInfo* edges;
    const VertexInfo* verts;
    const int32_t* iedges;            // interior edge ids
    const int32_t* iverts;            // interior vertex ids
    const int64_t* gdst;              // ghost copies: field[gdst] = field[gsrc]
    const int64_t* gsrc;
    const StokesFace* sfaces;         // Stokes stencils (null unless set up)
    const StokesEdge* sedges;
    const StokesVert* sverts;
    const FvFace* fvfaces;            // finite-volume cell geometry (null unless set up)
    const double* vxy;                // macro-vertex coordinates [2 V]
    const P2Face* p2faces;            // P2 stencils (null unless set up)
    const double* p2ediag;            // P2 diagonal of edge points [2 E]: even, odd k
    const double* p2vdiag;            // P2 diagonal of vertices [V]
};

// Coarse-level Jacobi-PCG data: interior points in canonical order, each
// with up to W stencil neighbours in an ELL table (column -1 = Dirichlet).
struct CoarseDev {
    int32_t N, W;
    const int64_t* owner;     // [N] field offset of the owned value
    const int32_t* kind;      // [N] 0 vertex, 1 edge, 2 face
    const int32_t* prim;      // [N] primitive id
    const int32_t* pa;        // [N] face i / edge k
    const int32_t* pb;        // [N] face j
    const int32_t* cols;      // [N * W]
    double* vals;             // [N * W] filled on the device per operator
    double* vec;              // [5 * N] CG scratch (x, r, z, p, q)
};

struct LevelHost {
    int level = 0, n = 0;
    int64_t face_stride = 0, edge_stride = 0, vert_stride = 0;
    int64_t face_base = 0, edge_base = 0, vert_base = 0, total = 0;
    int32_t ghost_off = 0, ghost_stride = 0;
    std::vector<int32_t> row_off;
    std::vector<int2> tiles;
    std::vector<int2> gs_tl[GS_NHALO][2];   // [halo][GS_TJ16 rows]
    std::vector<int2> net_tiles;
    std::vector<int2> net_strips;
    std::vector<int64_t> gdst, gsrc;
    int64_t gcls[G_NCLS + 1] = {0, 0, 0, 0, 0};
    int64_t n_all = 0, n_int = 0, can_edge_base = 0, can_face_base = 0;
    // device copies (inside the bound workspace)
    int32_t* d_row_off = nullptr;
    int2* d_tiles = nullptr;
    int2* d_gs_tl[GS_NHALO][2] = {};
    int2* d_net_tiles = nullptr;
    int2* d_net_strips = nullptr;
    int64_t* d_gdst = nullptr;
    int64_t* d_gsrc = nullptr;
};

}  // namespace hhg
