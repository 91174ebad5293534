// Host-side mesh object behind the opaque hhg_mesh handle.
#pragma once

#include <array>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "hhg_internal.hpp"

namespace hhg {

// Bump allocator over the caller's workspace (or a dry run to size it).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    void* take(size_t bytes) {
        off = (size_t)pad_up((int64_t)off, 256);
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// Owner of a face-local point: the primitive that holds the unique value.
struct Owner {
    int kind;   // 0 vertex, 1 edge point, 2 face interior
    int prim;   // vertex / edge / face id
    int k;      // edge parameter (kind 1)
    int i, j;   // face-local coordinates (kind 2)
};

struct MeshData {
    int V = 0, E = 0, F = 0, L = 0, lc = 0, maxdeg = 0;
    int nfaces2 = 0;   // faces smoothed with two colours (exact right angle)
    std::vector<double> vxy;
    std::vector<std::array<int, 3>> tri;            // counter-clockwise
    std::vector<std::array<int, 2>> edge_v;         // (a, b), a < b
    std::vector<FaceInfo> faces;
    std::vector<EdgeInfo> edges;
    std::vector<VertexInfo> verts;
    // the same tables before a face coefficient scaled their stiffness
    // weights (cotangents), and the coefficient itself (1 by default)
    std::vector<FaceInfo> faces0;
    std::vector<EdgeInfo> edges0;
    std::vector<VertexInfo> verts0;
    std::vector<double> face_coef;
    // Stokes stencils at unit scale (empty until stokes_tables runs)
    std::vector<StokesFace> sfaces;
    std::vector<StokesEdge> sedges;
    std::vector<StokesVert> sverts;
    std::vector<FvFace> fvfaces;
    // P2 stencils and interface diagonals (empty until p2_tables runs)
    std::vector<P2Face> p2faces;
    std::vector<double> p2ediag, p2vdiag;
    std::vector<int32_t> iedges, iverts;
    std::vector<LevelHost> lv;                      // index = level

    // coarse-level CG tables (host)
    int32_t Nc = 0, Wc = 0;
    std::vector<int64_t> c_owner;
    std::vector<int32_t> c_kind, c_prim, c_pa, c_pb, c_cols;

    // ---- geometry/indexing helpers (host)
    static void side_point(int side, int t, int d, int n, int& i, int& j);
    Owner owner_of(int f, int i, int j, int n) const;
    int64_t owner_offset(const LevelHost& L, const Owner& o) const;
    int64_t canonical_of(const LevelHost& L, const Owner& o) const;
    int64_t face_off(const LevelHost& L, int f, int i, int j) const {
        return L.face_base + (int64_t)f * L.face_stride + L.row_off[j] + i;
    }
    int64_t edge_off(const LevelHost& L, int e, int k) const {
        return L.edge_base + (int64_t)e * L.edge_stride + k;
    }
    int64_t ghost_off(const LevelHost& L, int e, int s, int g) const {
        return L.edge_base + (int64_t)e * L.edge_stride + L.ghost_off +
               (int64_t)s * L.ghost_stride + g;
    }
    int64_t vert_off(const LevelHost& L, int v, int slot) const {
        return L.vert_base + (int64_t)v * L.vert_stride + slot;
    }

    // Build everything; returns "" on success or an error message.
    std::string build(const double* vxy, int nv, const int32_t* tri, int nf,
                      int max_level, int coarse_level);
    void build_level(int level);
    void build_coarse();
    // Scale the stiffness weights of face f (and its share of the edge and
    // vertex weights) by coef[f] > 0; "" or an error message.
    std::string set_face_coef(const double* coef);
    // Stokes stencils from the geometry and the face coefficient (the
    // viscosity), stabilisation parameter delta.
    void stokes_tables(double delta);
    // Finite-volume cell geometry and face-to-face neighbours.
    void fv_tables();
    // P2 stencils from the face cotangents (times the face coefficient);
    // "" or an error message.
    std::string p2_tables();
};

}  // namespace hhg

// Workspace-resident state of one mesh.
struct hhg_mesh {
    hhg::MeshData m;
    uint32_t features = 0;
    bool bound = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // device tables
    hhg::FaceInfo* d_faces = nullptr;
    hhg::EdgeInfo* d_edges = nullptr;
    hhg::VertexInfo* d_verts = nullptr;
    hhg::StokesFace* d_sfaces = nullptr;
    hhg::StokesEdge* d_sedges = nullptr;
    hhg::StokesVert* d_sverts = nullptr;
    bool stokes_ready = false;
    double stokes_delta = 0.0;
    // MINRES vectors of the finest level (HHG_FEAT_STOKES): 7 Stokes vectors
    // of 3 fields each
    double* s_vec[7] = {};
    double* s_state = nullptr;   // MINRES scalars
    hhg::FvFace* d_fvfaces = nullptr;
    double* d_vxy = nullptr;
    double* t_cells = nullptr;   // second cell field of the transport loop
    double* b_stokes = nullptr;  // buoyancy right-hand side of the transport loop
    // P2 (HHG_FEAT_P2): tables and the faces' partial boundary rows
    hhg::P2Face* d_p2faces = nullptr;
    double* d_p2ediag = nullptr;
    double* d_p2vdiag = nullptr;
    double* p2part = nullptr;     // [F][3][n of the finest level]
    bool p2_ready = false;
    int32_t* d_iedges = nullptr;
    int32_t* d_iverts = nullptr;
    hhg::CoarseDev coarse{};              // vals: Laplace operator
    double* coarse_vals_diff = nullptr;   // diffusion operator
    // explicit inverses of the coarse interior operator (Laplace, diffusion),
    // rebuilt on the GPU before the first coarse solve after a change
    double* coarse_inv[2] = {nullptr, nullptr};
    mutable bool inv_ok[2] = {false, false};
    // fields per level (index = level); finest-level u, f come from the caller
    void* u64[hhg::MAXLEVEL + 1] = {};
    void* f64[hhg::MAXLEVEL + 1] = {};
    void* r64[hhg::MAXLEVEL + 1] = {};
    void* u32[hhg::MAXLEVEL + 1] = {};
    void* f32[hhg::MAXLEVEL + 1] = {};
    void* r32[hhg::MAXLEVEL + 1] = {};
    void* a64[hhg::MAXLEVEL + 1] = {};   // second buffer of the ping-pong smoother
    void* a32[hhg::MAXLEVEL + 1] = {};
    double* kap64[hhg::MAXLEVEL + 1] = {};
    float* kap32[hhg::MAXLEVEL + 1] = {};
    bool kappa_set = false;
    // learned smoother: FP32 master weights, Adam moments, scratch
    float* net_w = nullptr;
    float* net_m = nullptr;
    float* net_v = nullptr;
    float* net_partials = nullptr;
    bool net_loaded = false;
    bool net_accepted = false;
    bool net_mfma = true;         // BF16 MFMA forward (false: FP32, for tests)
    double* partials = nullptr;   // reduction partial sums
    int64_t n_partials = 0;
    double* dscalars = nullptr;   // small device scalars (norms, dots)
    // the solve loop's residual norm: pinned host memory mapped into the
    // device address space, written by the reduction kernel itself, so that
    // reading it needs no copy after the stream synchronisation
    double* h_norm = nullptr;
    double* h_norm_dev = nullptr;
    // timing of finest-level face smoother launches
    bool timing = false;
    int64_t t_launches = 0;
    double t_ms = 0.0;
    std::vector<std::pair<void*, void*>> t_events;

    hhg::LevelDev dev(int level) const;
};
