// C ABI of the HHG P1 library and the host drivers of the multigrid cycle
// (sec. 4.3): V-cycle recursion, solve loop and mixed-precision iterative
// refinement.  All device work is done by the kernels in kernels.hip.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <new>
#include <utility>
#include <string>

#include "../../include/hhg.h"
#include "hhg_kernels.hpp"
#include "hhg_mesh.hpp"

using namespace hhg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(HHG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_CHECK(expr, where)                          \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

// Lay out (or size, with a null base) everything the workspace holds.
void carve(hhg_mesh* M, uint32_t feat, Carver& c) {
    MeshData& m = M->m;
    M->d_faces = (FaceInfo*)c.take(sizeof(FaceInfo) * m.F);
    M->d_edges = (EdgeInfo*)c.take(sizeof(EdgeInfo) * m.E);
    M->d_verts = (VertexInfo*)c.take(sizeof(VertexInfo) * m.V);
    M->d_iedges = (int32_t*)c.take(sizeof(int32_t) * (m.iedges.size() + 1));
    M->d_iverts = (int32_t*)c.take(sizeof(int32_t) * (m.iverts.size() + 1));
    for (int l = 1; l <= m.L; ++l) {
        LevelHost& H = m.lv[l];
        H.d_row_off = (int32_t*)c.take(sizeof(int32_t) * H.row_off.size());
        H.d_tiles = (int2*)c.take(sizeof(int2) * (H.tiles.size() + 1));
        for (int e = 0; e < GS_NHALO; ++e)
            for (int t = 0; t < 2; ++t)
                H.d_gs_tl[e][t] = (int2*)c.take(sizeof(int2) * (H.gs_tl[e][t].size() + 1));
        H.d_net_tiles = (int2*)c.take(sizeof(int2) * (H.net_tiles.size() + 1));
        H.d_net_strips = (int2*)c.take(sizeof(int2) * (H.net_strips.size() + 1));
        H.d_gdst = (int64_t*)c.take(sizeof(int64_t) * (H.gdst.size() + 1));
        H.d_gsrc = (int64_t*)c.take(sizeof(int64_t) * (H.gsrc.size() + 1));
    }
    CoarseDev& C = M->coarse;
    C.N = m.Nc;
    C.W = m.Wc;
    const size_t NW = (size_t)m.Nc * m.Wc;
    C.owner = (const int64_t*)c.take(sizeof(int64_t) * m.Nc);
    C.kind = (const int32_t*)c.take(sizeof(int32_t) * m.Nc);
    C.prim = (const int32_t*)c.take(sizeof(int32_t) * m.Nc);
    C.pa = (const int32_t*)c.take(sizeof(int32_t) * m.Nc);
    C.pb = (const int32_t*)c.take(sizeof(int32_t) * m.Nc);
    C.cols = (const int32_t*)c.take(sizeof(int32_t) * NW);
    C.vals = (double*)c.take(sizeof(double) * NW);                  // Laplace
    M->coarse_vals_diff = (double*)c.take(sizeof(double) * NW);     // diffusion
    M->coarse_inv[0] = M->coarse_inv[1] = nullptr;
    M->inv_ok[0] = M->inv_ok[1] = false;
    if (m.Nc > 0 && m.Nc <= COARSE_DENSE_MAXN) {
        const size_t NN = (size_t)m.Nc * m.Nc;
        M->coarse_inv[0] = (double*)c.take(sizeof(double) * NN);
        if (feat & HHG_FEAT_VARK) M->coarse_inv[1] = (double*)c.take(sizeof(double) * NN);
    }
    C.vec = (double*)c.take(sizeof(double) * 5 * (size_t)m.Nc);
    M->n_partials = 1024;
    for (int l = 1; l <= m.L; ++l)
        M->n_partials = std::max({M->n_partials, sweep_norm_partials(M, l), face_loop_partials(M, l)});
    if (feat & HHG_FEAT_STOKES) M->n_partials = std::max(M->n_partials, stokes_partials());
    M->partials = (double*)c.take(sizeof(double) * M->n_partials);
    M->dscalars = (double*)c.take(sizeof(double) * 64);
    for (int l = 0; l <= MAXLEVEL; ++l) {
        M->u64[l] = M->f64[l] = M->r64[l] = nullptr;
        M->u32[l] = M->f32[l] = M->r32[l] = nullptr;
        M->kap64[l] = nullptr;
        M->kap32[l] = nullptr;
        M->a64[l] = M->a32[l] = nullptr;
    }
    auto fld = [&](int l, size_t esz) { return c.take(esz * (size_t)m.lv[l].total); };
    if (feat & (HHG_FEAT_F64 | HHG_FEAT_MP)) M->r64[m.L] = fld(m.L, 8);
    if (feat & HHG_FEAT_F64) {
        for (int l = m.lc; l < m.L; ++l) {
            M->u64[l] = fld(l, 8);
            M->f64[l] = fld(l, 8);
            M->r64[l] = fld(l, 8);
        }
    }
    if (feat & HHG_FEAT_MP) {
        if (!(feat & HHG_FEAT_F64))
            for (int l = m.lc; l <= m.L; ++l)
                if (!M->r64[l]) M->r64[l] = fld(l, 8);   // FP64 coarse residual
        for (int l = 1; l <= m.L; ++l) {
            if (l >= m.lc) {
                M->u32[l] = fld(l, 4);
                M->f32[l] = fld(l, 4);
            }
            M->r32[l] = fld(l, 4);
        }
    }
    for (int l = 1; l <= m.L; ++l) {
        if (feat & HHG_FEAT_F64) M->a64[l] = fld(l, 8);
        if (feat & HHG_FEAT_MP) M->a32[l] = fld(l, 4);
    }
    M->net_w = M->net_m = M->net_v = M->net_partials = nullptr;
    if (feat & HHG_FEAT_NET) {
        M->net_w = (float*)c.take(sizeof(float) * NET_NW);
        M->net_m = (float*)c.take(sizeof(float) * NET_NW);
        M->net_v = (float*)c.take(sizeof(float) * NET_NW);
        size_t maxb = 1;
        for (int l = 1; l <= m.L; ++l) maxb = std::max(maxb, (size_t)m.F * m.lv[l].net_tiles.size());
        M->net_partials = (float*)c.take(sizeof(float) * NET_NW * maxb);
    }
    if (feat & HHG_FEAT_VARK) {
        for (int l = 1; l <= m.L; ++l) {
            M->kap64[l] = (double*)fld(l, 8);
            if (feat & HHG_FEAT_MP) M->kap32[l] = (float*)fld(l, 4);
        }
    }
    M->d_sfaces = nullptr;
    M->d_sedges = nullptr;
    M->d_sverts = nullptr;
    M->s_state = nullptr;
    M->d_fvfaces = nullptr;
    M->d_vxy = nullptr;
    M->b_stokes = nullptr;
    M->t_cells = nullptr;
    for (auto& v : M->s_vec) v = nullptr;
    if (feat & HHG_FEAT_STOKES) {
        M->d_sfaces = (StokesFace*)c.take(sizeof(StokesFace) * m.F);
        M->d_sedges = (StokesEdge*)c.take(sizeof(StokesEdge) * m.E);
        M->d_sverts = (StokesVert*)c.take(sizeof(StokesVert) * m.V);
        M->s_state = (double*)c.take(sizeof(double) * 64);
        for (auto& v : M->s_vec) v = (double*)c.take(sizeof(double) * 3 * (size_t)m.lv[m.L].total);
        M->d_fvfaces = (FvFace*)c.take(sizeof(FvFace) * m.F);
        M->d_vxy = (double*)c.take(sizeof(double) * 2 * m.V);
        M->b_stokes = (double*)c.take(sizeof(double) * 3 * (size_t)m.lv[m.L].total);
        M->t_cells = (double*)c.take(sizeof(double) * 2 * (size_t)m.lv[m.L].total);
    }
    M->d_p2faces = nullptr;
    M->d_p2ediag = M->d_p2vdiag = M->p2part = nullptr;
    if (feat & HHG_FEAT_P2) {
        M->d_p2faces = (P2Face*)c.take(sizeof(P2Face) * m.F);
        M->d_p2ediag = (double*)c.take(sizeof(double) * 2 * (size_t)m.E);
        M->d_p2vdiag = (double*)c.take(sizeof(double) * m.V);
        M->p2part = (double*)c.take(sizeof(double) * 3 * (size_t)m.F * m.lv[m.L].n);
    }
}

template <class V>
hipError_t upload(void* dst, const V& v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice, s);
}

bool level_ok(const hhg_mesh* M, int level) { return level >= 1 && level <= M->m.L; }
bool dtype_ok(int dt) { return dt == HHG_F64 || dt == HHG_F32; }
bool op_ok(const hhg_mesh* M, int op) {
    if (op == HHG_OP_LAPLACE || op == HHG_OP_MASS) return true;
    return op == HHG_OP_DIFFUSION && M->kappa_set;
}

int check_common(const hhg_mesh* M, int level, int dtype) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    if (!dtype_ok(dtype)) return fail(HHG_EINVAL, "dtype must be HHG_F64 or HHG_F32");
    return HHG_OK;
}

int check_op(const hhg_mesh* M, int op, int dtype) {
    if (op == HHG_OP_DIFFUSION && !M->kappa_set)
        return fail(HHG_EINVAL, "HHG_OP_DIFFUSION needs hhg_set_coefficient first");
    if (op == HHG_OP_DIFFUSION && dtype == HHG_F32 && !(M->features & HHG_FEAT_MP))
        return fail(HHG_EINVAL, "FP32 diffusion needs a workspace bound with HHG_FEAT_MP");
    if (!op_ok(M, op)) return fail(HHG_EINVAL, "unknown operator");
    return HHG_OK;
}

int check_smoother(const hhg_mesh* M, int smoother, int dtype) {
    if (smoother == HHG_SMOOTH_GS) return HHG_OK;
    if (smoother != HHG_SMOOTH_NET) return fail(HHG_EINVAL, "unknown smoother");
    if (!(M->features & HHG_FEAT_NET)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_NET");
    if (!M->net_loaded) return fail(HHG_EINVAL, "no network weights set");
    if (dtype != HHG_F32) return fail(HHG_EINVAL, "the learned smoother runs on FP32 fields");
    return HHG_OK;
}

// fields of the hierarchy for a dtype
void* level_u(const hhg_mesh* M, int l, int dt) { return dt == HHG_F64 ? M->u64[l] : M->u32[l]; }
void* level_f(const hhg_mesh* M, int l, int dt) { return dt == HHG_F64 ? M->f64[l] : M->f32[l]; }
void* level_r(const hhg_mesh* M, int l, int dt) { return dt == HHG_F64 ? M->r64[l] : M->r32[l]; }

void* level_alt(const hhg_mesh* M, int l, int dt) { return dt == HHG_F64 ? M->a64[l] : M->a32[l]; }

// Learned-smoother sweep (FP32), x -> y: Gauss-Seidel stages A and B on
// edges and vertices (in place on x, then a refresh of the stage-B corner
// copies), then the face step y = x + N(D^-1 (f - A x)) on face interiors
// with the ring values of D^-1 (f - A x) from an edge/vertex pass; the
// backward sweep runs the face step first and the stages on y after it.
int net_sweep(const hhg_mesh* M, int level, int op, void* x_, void* y_, const void* f_, int backward,
              hipStream_t s) {
    float* x = (float*)x_;
    float* y = (float*)y_;
    const float* f = (const float*)f_;
    float* rho = (float*)M->r32[level];
    auto face_step = [&]() -> int {
        HIP_CHECK(launch_jacobi_low(M, level, op, x, f, rho, s), "net rho");
        HIP_CHECK(launch_net_step(M, level, op, x, y, f, rho, M->net_mfma, s), "net step");
        return HHG_OK;
    };
    int rc;
    if (backward) {
        if ((rc = face_step())) return rc;
        HIP_CHECK(launch_low_gs(M, level, op, HHG_F32, y, f, 1, s), "stage");
        HIP_CHECK(launch_low_gs(M, level, op, HHG_F32, y, f, 0, s), "stage");
        return HHG_OK;
    }
    HIP_CHECK(launch_low_gs(M, level, op, HHG_F32, x, f, 0, s), "stage");
    HIP_CHECK(launch_low_gs(M, level, op, HHG_F32, x, f, 1, s), "stage");
    // stage B left the ghost-row corner copies to its successor
    HIP_CHECK(launch_low_gs(M, level, op, HHG_F32, x, f, 2, s), "corner copies");
    return face_step();
}

int smooth_pp(const hhg_mesh* M, int level, int op, int smoother, int dt, void* x, void* y,
              const void* f, int sweeps, int backward, hipStream_t s, void** out) {
    for (int i = 0; i < sweeps; ++i) {
        if (smoother == HHG_SMOOTH_NET) {
            int rc = net_sweep(M, level, op, x, y, f, backward, s);
            if (rc) return rc;
            std::swap(x, y);
            continue;
        }
        HIP_CHECK(launch_gs_sweep(M, level, op, dt, x, y, f, backward, s), "smooth");
        std::swap(x, y);
    }
    *out = x;
    return HHG_OK;
}

int copy_field(const hhg_mesh* M, int level, int dt, void* dst, const void* src, hipStream_t s) {
    const size_t bytes = (size_t)M->m.lv[level].total * (dt == HHG_F64 ? 8 : 4);
    HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "copy");
    return HHG_OK;
}

// One V-cycle on `level`.  norm != nullptr: also |f - A u|_2 of the result
// into the device double *norm, formed by the last post-smoothing sweep when
// there is one besides the sweep that carries the prolongation, else by a
// residual pass.  u_zero: u is known to be 0 (the coarse corrections, which
// the restriction zeroes).
int vcycle_rec(const hhg_mesh* M, int level, int op, int smoother, int dt, void* u, const void* f,
               int nu1, int nu2, hipStream_t s, double* norm = nullptr, bool u_zero = false) {
    const int lc = M->m.lc;
    const double* vals = op == HHG_OP_DIFFUSION ? M->coarse_vals_diff : M->coarse.vals;
    if (level == lc) {
        HIP_CHECK(launch_coarse_solve(M, op, dt, u, f, vals, s, u_zero), "coarse solve");
        if (norm) HIP_CHECK(launch_residual(M, level, op, dt, u, f, nullptr, norm, s), "residual norm");
        return HHG_OK;
    }
    void* alt = level_alt(M, level, dt);
    void* cur = nullptr;
    // with Gauss-Seidel the last pre-smoothing sweep also forms and restricts the residual
    const bool sweep_res = smoother == HHG_SMOOTH_GS && nu1 > 0;
    int rc = smooth_pp(M, level, op, smoother, dt, u, alt, f, sweep_res ? nu1 - 1 : nu1, 0, s, &cur);
    if (rc) return rc;
    void* other = cur == u ? alt : u;
    void* r = level_r(M, level, dt);
    void* uc = level_u(M, level - 1, dt);
    void* fc = level_f(M, level - 1, dt);
    if (sweep_res) {
        HIP_CHECK(launch_gs_sweep_restrict(M, level, op, dt, cur, other, f, r, fc, uc, s),
                  "smooth + residual + restrict");
        std::swap(cur, other);
    } else {
        HIP_CHECK(launch_residual(M, level, op, dt, cur, f, r, nullptr, s), "residual");
        HIP_CHECK(launch_restrict(M, level, dt, r, fc, uc, s), "restrict");
    }
    rc = vcycle_rec(M, level - 1, op, smoother, dt, uc, fc, nu1, nu2, s, nullptr, true);
    if (rc) return rc;
    void* fin = nullptr;
    if (smoother == HHG_SMOOTH_GS && nu2 > 0) {
        // prolongation folded into the first post-smoothing sweep: cur -> other
        HIP_CHECK(launch_gs_sweep_prolong(M, level, op, dt, cur, other, f, uc, s), "prolong + smooth");
        const bool sweep_norm = norm && nu2 >= 2;
        rc = smooth_pp(M, level, op, smoother, dt, other, cur, f, sweep_norm ? nu2 - 2 : nu2 - 1, 1, s, &fin);
        if (rc) return rc;
        if (sweep_norm) {
            void* y = fin == other ? cur : other;
            HIP_CHECK(launch_gs_sweep_norm(M, level, op, dt, fin, y, f, norm, s), "smooth + norm");
            fin = y;
            norm = nullptr;
        }
    } else {
        HIP_CHECK(launch_prolong_add(M, level, dt, uc, cur, s), "prolong");
        rc = smooth_pp(M, level, op, smoother, dt, cur, other, f, nu2, 1, s, &fin);
        if (rc) return rc;
    }
    if (fin != u && (rc = copy_field(M, level, dt, u, fin, s))) return rc;
    if (norm) HIP_CHECK(launch_residual(M, level, op, dt, u, f, nullptr, norm, s), "residual norm");
    return HHG_OK;
}

// The solve loop's norm slot: 64 bytes of pinned, coherent host memory
// mapped into the device address space, allocated when the first workspace
// is bound and kept until the mesh is destroyed.
static int solve_norm_slot(hhg_mesh* M) {
    if (M->h_norm) return HHG_OK;
    void* h = nullptr;
    void* d = nullptr;
    HIP_CHECK(hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent), "pinned norm slot");
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipHostFree(h);
        return fail(HHG_EHIP, "pinned norm slot has no device address");
    }
    M->h_norm = (double*)h;
    M->h_norm_dev = (double*)d;
    return HHG_OK;
}

// Value of the norm slot once the stream has drained.
static int read_norm_slot(const hhg_mesh* M, double* h, hipStream_t s) {
    HIP_CHECK(hipStreamSynchronize(s), "norm readback");
    *h = *(volatile const double*)M->h_norm;
    return HHG_OK;
}


}  // namespace

hhg::LevelDev hhg_mesh::dev(int level) const {
    const LevelHost& H = m.lv[level];
    LevelDev L{};
    L.level = level;
    L.n = H.n;
    L.F = m.F; L.E = m.E; L.V = m.V;
    L.ghost_off = H.ghost_off;
    L.ghost_stride = H.ghost_stride;
    L.vert_stride = (int32_t)H.vert_stride;
    L.ntiles = (int32_t)H.tiles.size();
    for (int e = 0; e < GS_NHALO; ++e)
        for (int t = 0; t < 2; ++t) {
            L.n_gs_tl[e][t] = (int32_t)H.gs_tl[e][t].size();
            L.gs_tl[e][t] = H.d_gs_tl[e][t];
        }
    L.n_net_tiles = (int32_t)H.net_tiles.size();
    L.n_net_strips = (int32_t)H.net_strips.size();
    L.net_sr = net_strip_rows(H.n);
    L.n_iedges = (int32_t)m.iedges.size();
    L.n_iverts = (int32_t)m.iverts.size();
    L.face_stride = H.face_stride;
    L.edge_stride = H.edge_stride;
    L.face_base = H.face_base;
    L.edge_base = H.edge_base;
    L.vert_base = H.vert_base;
    L.total = H.total;
    for (int c = 0; c <= G_NCLS; ++c) L.gcls[c] = H.gcls[c];
    L.can_edge_base = H.can_edge_base;
    L.can_face_base = H.can_face_base;
    L.n_all = H.n_all;
    L.inv4l = std::ldexp(1.0, -2 * level);
    L.row_off = H.d_row_off;
    L.tiles = H.d_tiles;
    L.net_tiles = H.d_net_tiles;
    L.net_strips = H.d_net_strips;
    L.faces = d_faces;
    L.edges = d_edges;
    L.verts = d_verts;
    L.iedges = d_iedges;
    L.iverts = d_iverts;
    L.gdst = H.d_gdst;
    L.gsrc = H.d_gsrc;
    L.sfaces = d_sfaces;
    L.sedges = d_sedges;
    L.sverts = d_sverts;
    L.fvfaces = d_fvfaces;
    L.p2faces = d_p2faces;
    L.p2ediag = d_p2ediag;
    L.p2vdiag = d_p2vdiag;
    L.vxy = d_vxy;
    return L;
}

extern "C" {

const char* hhg_last_error(void) { return g_err.c_str(); }

int hhg_setup_mesh(const double* vxy, int32_t n_vertices, const int32_t* tri, int32_t n_faces,
                   int32_t max_level, int32_t coarse_level, hhg_mesh** out) {
    if (!vxy || !tri || !out) return fail(HHG_EINVAL, "null argument");
    *out = nullptr;
    hhg_mesh* M = new (std::nothrow) hhg_mesh();
    if (!M) return fail(HHG_ENOMEM, "host allocation failed");
    std::string err;
    try {
        err = M->m.build(vxy, n_vertices, tri, n_faces, max_level, coarse_level);
    } catch (const std::exception& ex) {
        err = std::string("setup failed: ") + ex.what();
    }
    if (!err.empty()) {
        delete M;
        return fail(HHG_EINVAL, err);
    }
    *out = M;
    return HHG_OK;
}

void hhg_destroy_mesh(hhg_mesh* mesh) {
    if (!mesh) return;
    if (mesh->h_norm) (void)hipHostFree(mesh->h_norm);
    for (auto& ev : mesh->t_events) {
        (void)hipEventDestroy((hipEvent_t)ev.first);
        (void)hipEventDestroy((hipEvent_t)ev.second);
    }
    delete mesh;
}

int hhg_workspace_bytes(const hhg_mesh* mesh, uint32_t features, size_t* bytes) {
    if (!mesh || !bytes) return fail(HHG_EINVAL, "null argument");
    if (features & ~(HHG_FEAT_F64 | HHG_FEAT_MP | HHG_FEAT_VARK | HHG_FEAT_NET | HHG_FEAT_STOKES | HHG_FEAT_P2))
        return fail(HHG_EINVAL, "unknown feature bits");
    if ((features & HHG_FEAT_STOKES) && !(features & HHG_FEAT_F64))
        return fail(HHG_EINVAL, "HHG_FEAT_STOKES needs HHG_FEAT_F64 (the preconditioner's hierarchy)");
    if ((features & HHG_FEAT_P2) && !(features & HHG_FEAT_F64))
        return fail(HHG_EINVAL, "HHG_FEAT_P2 needs HHG_FEAT_F64 (the P1 hierarchy of the p-multigrid cycle)");
    if ((features & HHG_FEAT_NET) && !(features & HHG_FEAT_MP))
        return fail(HHG_EINVAL, "HHG_FEAT_NET needs HHG_FEAT_MP (the learned smoother runs in FP32)");
    hhg_mesh tmp;
    tmp.m = mesh->m;
    Carver c(nullptr);
    carve(&tmp, features, c);
    *bytes = c.off + 256;
    return HHG_OK;
}

int hhg_bind_workspace(hhg_mesh* M, uint32_t features, void* dptr, size_t bytes, void* stream) {
    if (!M || !dptr) return fail(HHG_EINVAL, "null argument");
    size_t need = 0;
    int rc = hhg_workspace_bytes(M, features, &need);
    if (rc) return rc;
    if (bytes < need) return fail(HHG_ENOMEM, "workspace too small: need " + std::to_string(need));
    if ((uintptr_t)dptr % 256) return fail(HHG_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    // zero once, so that entries no kernel writes (row and block padding)
    // hold zeros in every workspace field, whatever the memory held before
    HIP_CHECK(hipMemsetAsync(dptr, 0, need, s), "workspace clear");
    if ((rc = solve_norm_slot(M))) return rc;
    HIP_CHECK(scratch_init(), "static scratch");
    Carver c(dptr);
    carve(M, features, c);
    MeshData& m = M->m;
    HIP_CHECK(upload(M->d_faces, m.faces, s), "upload");
    HIP_CHECK(upload(M->d_edges, m.edges, s), "upload");
    HIP_CHECK(upload(M->d_verts, m.verts, s), "upload");
    HIP_CHECK(upload(M->d_iedges, m.iedges, s), "upload");
    HIP_CHECK(upload(M->d_iverts, m.iverts, s), "upload");
    for (int l = 1; l <= m.L; ++l) {
        LevelHost& H = m.lv[l];
        HIP_CHECK(upload(H.d_row_off, H.row_off, s), "upload");
        HIP_CHECK(upload(H.d_tiles, H.tiles, s), "upload");
        for (int e = 0; e < GS_NHALO; ++e)
            for (int t = 0; t < 2; ++t) HIP_CHECK(upload(H.d_gs_tl[e][t], H.gs_tl[e][t], s), "upload");
        HIP_CHECK(upload(H.d_net_tiles, H.net_tiles, s), "upload");
        HIP_CHECK(upload(H.d_net_strips, H.net_strips, s), "upload");
        HIP_CHECK(upload(H.d_gdst, H.gdst, s), "upload");
        HIP_CHECK(upload(H.d_gsrc, H.gsrc, s), "upload");
    }
    CoarseDev& C = M->coarse;
    HIP_CHECK(upload((void*)C.owner, m.c_owner, s), "upload");
    HIP_CHECK(upload((void*)C.kind, m.c_kind, s), "upload");
    HIP_CHECK(upload((void*)C.prim, m.c_prim, s), "upload");
    HIP_CHECK(upload((void*)C.pa, m.c_pa, s), "upload");
    HIP_CHECK(upload((void*)C.pb, m.c_pb, s), "upload");
    HIP_CHECK(upload((void*)C.cols, m.c_cols, s), "upload");
    M->ws = (char*)dptr;
    M->ws_bytes = bytes;
    M->features = features;
    M->bound = true;
    M->kappa_set = false;
    M->net_loaded = false;
    M->net_accepted = false;
    M->stokes_ready = false;
    HIP_CHECK(launch_coarse_extract(M, OP_LAPLACE, C.vals, s), "coarse operator");
    HIP_CHECK(hipStreamSynchronize(s), "bind");
    return HHG_OK;
}

int hhg_field_elems(const hhg_mesh* M, int32_t level, int64_t* n) {
    if (!M || !n) return fail(HHG_EINVAL, "null argument");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    *n = M->m.lv[level].total;
    return HHG_OK;
}

int hhg_n_dofs(const hhg_mesh* M, int32_t level, int64_t* n_interior, int64_t* n_all) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    if (n_interior) *n_interior = M->m.lv[level].n_int;
    if (n_all) *n_all = M->m.lv[level].n_all;
    return HHG_OK;
}

int hhg_coords(const hhg_mesh* M, int32_t level, double* xy) {
    if (!M || !xy) return fail(HHG_EINVAL, "null argument");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    const MeshData& m = M->m;
    const LevelHost& H = m.lv[level];
    const int n = H.n;
    for (int v = 0; v < m.V; ++v) {
        xy[2 * v] = m.vxy[2 * v];
        xy[2 * v + 1] = m.vxy[2 * v + 1];
    }
    for (int e = 0; e < m.E; ++e) {
        const double* a = &m.vxy[2 * m.edges[e].a];
        const double* b = &m.vxy[2 * m.edges[e].b];
        for (int k = 1; k <= n - 2; ++k) {
            const double t = (double)k / (n - 1);
            const int64_t c = H.can_edge_base + (int64_t)e * (n - 2) + (k - 1);
            xy[2 * c] = a[0] + t * (b[0] - a[0]);
            xy[2 * c + 1] = a[1] + t * (b[1] - a[1]);
        }
    }
    const int64_t nfi = (int64_t)(n - 2) * (n - 3) / 2;
    for (int f = 0; f < m.F; ++f) {
        const double* x0 = &m.vxy[2 * m.tri[f][0]];
        const double* x1 = &m.vxy[2 * m.tri[f][1]];
        const double* x2 = &m.vxy[2 * m.tri[f][2]];
        int64_t c = H.can_face_base + (int64_t)f * nfi;
        for (int j = 1; j <= n - 3; ++j)
            for (int i = 1; i <= n - 2 - j; ++i, ++c) {
                const double si = (double)i / (n - 1), sj = (double)j / (n - 1);
                xy[2 * c] = x0[0] + si * (x1[0] - x0[0]) + sj * (x2[0] - x0[0]);
                xy[2 * c + 1] = x0[1] + si * (x1[1] - x0[1]) + sj * (x2[1] - x0[1]);
            }
    }
    return HHG_OK;
}

int hhg_ghost_table(const hhg_mesh* M, int32_t level, int64_t* n_copies, int64_t* dst, int64_t* src) {
    if (!M || !n_copies) return fail(HHG_EINVAL, "null argument");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    const LevelHost& H = M->m.lv[level];
    *n_copies = (int64_t)H.gdst.size();
    if (dst) std::copy(H.gdst.begin(), H.gdst.end(), dst);
    if (src) std::copy(H.gsrc.begin(), H.gsrc.end(), src);
    return HHG_OK;
}

int hhg_from_canonical(const hhg_mesh* M, int32_t level, int32_t dtype, const void* canon,
                       void* field, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (!canon || !field) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_canon(M, level, dtype, canon, field, 0, (hipStream_t)stream), "from_canonical");
    return HHG_OK;
}

int hhg_to_canonical(const hhg_mesh* M, int32_t level, int32_t dtype, const void* field,
                     void* canon, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (!canon || !field) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_canon(M, level, dtype, field, canon, 1, (hipStream_t)stream), "to_canonical");
    return HHG_OK;
}

int hhg_set_coefficient(hhg_mesh* M, const double* k_canon, void* stream) {
    if (!M || !k_canon) return fail(HHG_EINVAL, "null argument");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!(M->features & HHG_FEAT_VARK)) return fail(HHG_EINVAL, "workspace lacks HHG_FEAT_VARK");
    hipStream_t s = (hipStream_t)stream;
    const int L = M->m.L;
    HIP_CHECK(launch_canon(M, L, HHG_F64, k_canon, M->kap64[L], 0, s), "coefficient");
    for (int l = L; l > 1; --l) HIP_CHECK(launch_inject(M, l, HHG_F64, M->kap64[l], M->kap64[l - 1], s), "inject");
    if (M->features & HHG_FEAT_MP)
        for (int l = 1; l <= L; ++l)
            HIP_CHECK(launch_f64_to_f32(M->kap64[l], M->kap32[l], M->m.lv[l].total, s), "coefficient f32");
    M->kappa_set = true;
    HIP_CHECK(launch_coarse_extract(M, OP_DIFFUSION, M->coarse_vals_diff, s), "coarse operator");
    M->inv_ok[1] = false;
    return HHG_OK;
}

int hhg_apply(const hhg_mesh* M, int32_t level, int32_t op, int32_t dtype, const void* x, void* y,
              void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if ((rc = check_op(M, op, dtype))) return rc;
    if (!x || !y || x == y) return fail(HHG_EINVAL, "x and y must be distinct buffers");
    HIP_CHECK(launch_apply(M, level, op, dtype, x, y, (hipStream_t)stream), "apply");
    return HHG_OK;
}

int hhg_residual(const hhg_mesh* M, int32_t level, int32_t op, int32_t dtype, const void* u,
                 const void* f, void* r, double* norm, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if ((rc = check_op(M, op, dtype))) return rc;
    if (op == HHG_OP_MASS) return fail(HHG_EINVAL, "residual needs a stiffness operator");
    if (!u || !f || (!r && !norm)) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_residual(M, level, op, dtype, u, f, r, norm, (hipStream_t)stream), "residual");
    return HHG_OK;
}

int hhg_smooth(const hhg_mesh* M, int32_t level, int32_t op, int32_t smoother, int32_t dtype,
               void* u, const void* f, int32_t sweeps, int32_t backward, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if ((rc = check_op(M, op, dtype))) return rc;
    if (op == HHG_OP_MASS) return fail(HHG_EINVAL, "smoothing needs a stiffness operator");
    if ((rc = check_smoother(M, smoother, dtype))) return rc;
    if (sweeps < 0 || !u || !f) return fail(HHG_EINVAL, "bad arguments");
    void* alt = level_alt(M, level, dtype);
    if (!alt) return fail(HHG_ENOMEM, dtype == HHG_F64 ? "workspace lacks HHG_FEAT_F64"
                                                       : "workspace lacks HHG_FEAT_MP");
    hipStream_t s = (hipStream_t)stream;
    void* fin = nullptr;
    if ((rc = smooth_pp(M, level, op, smoother, dtype, u, alt, f, sweeps, backward != 0, s, &fin))) return rc;
    if (fin != u) return copy_field(M, level, dtype, u, fin, s);
    return HHG_OK;
}

int hhg_vcycle(const hhg_mesh* M, int32_t level, int32_t op, int32_t smoother, int32_t dtype,
               void* u, const void* f, int32_t nu1, int32_t nu2, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if ((rc = check_op(M, op, dtype))) return rc;
    if (op == HHG_OP_MASS) return fail(HHG_EINVAL, "multigrid needs a stiffness operator");
    if ((rc = check_smoother(M, smoother, dtype))) return rc;
    if (level < M->m.lc) return fail(HHG_EINVAL, "level below the coarse level");
    if (dtype == HHG_F64 && !(M->features & HHG_FEAT_F64))
        return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_F64");
    if (dtype == HHG_F32 && !(M->features & HHG_FEAT_MP))
        return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_MP");
    if (nu1 < 0 || nu2 < 0 || !u || !f) return fail(HHG_EINVAL, "bad arguments");
    return vcycle_rec(M, level, op, smoother, dtype, u, f, nu1, nu2, (hipStream_t)stream);
}

int hhg_solve(hhg_mesh* M, const hhg_solve_opts* o, void* u, const void* f, hhg_solve_stats* st,
              void* stream) {
    if (!M || !o || !u || !f || !st) return fail(HHG_EINVAL, "null argument");
    auto t0 = std::chrono::steady_clock::now();
    std::memset(st, 0, sizeof(*st));
    g_err.clear();
    const int L = M->m.L;
    int rc = check_common(M, L, HHG_F64);
    if (rc) return rc;
    if ((rc = check_op(M, o->op, HHG_F64))) return rc;
    if (o->op == HHG_OP_MASS) return fail(HHG_EINVAL, "solve needs a stiffness operator");
    if (o->mode != HHG_MODE_PLAIN_FP64 && o->mode != HHG_MODE_MP_IR && o->mode != HHG_MODE_LEARNED)
        return fail(HHG_EINVAL, "unknown solve mode");
    if (o->mode == HHG_MODE_LEARNED && !(M->features & HHG_FEAT_NET))
        return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_NET");
    if (o->mode == HHG_MODE_PLAIN_FP64 && !(M->features & HHG_FEAT_F64))
        return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_F64");
    if (o->mode != HHG_MODE_PLAIN_FP64 && !(M->features & HHG_FEAT_MP))
        return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_MP");
    if (o->max_iters < 0 || o->nu1 < 0 || o->nu2 < 0 || !(o->rtol >= 0))
        return fail(HHG_EINVAL, "bad solve options");
    if (o->op == HHG_OP_DIFFUSION && o->mode == HHG_MODE_MP_IR && !M->kap32[L])
        return fail(HHG_EINVAL, "FP32 coefficient missing");
    hipStream_t s = (hipStream_t)stream;
    if (!M->h_norm) return fail(HHG_ENOMEM, "no norm slot: bind a workspace first");
    double* dnorm = M->h_norm_dev;
    const int64_t nL = M->m.lv[L].total;
    const bool mp = o->mode != HHG_MODE_PLAIN_FP64;
    // Plain: u in place, norm-only residuals.  Mixed precision: the fused
    // outer step writes u + e into the other FP64 buffer (ping-pong with the
    // level's FP64 scratch field) together with the FP32 residual, which is
    // the next cycle's right-hand side.
    double* cur = (double*)u;
    double* alt = (double*)M->r64[L];
    float* r32 = (float*)M->f32[L];
    float* e32 = (float*)M->u32[L];
    auto first_norm = [&](double* out) -> int {
        if (mp) HIP_CHECK(launch_mp_step(M, L, o->op, cur, nullptr, (const double*)f, nullptr, r32, dnorm, s),
                          "residual");
        else HIP_CHECK(launch_residual(M, L, o->op, HHG_F64, cur, f, nullptr, dnorm, s), "residual");
        return read_norm_slot(M, out, s);
    };
    auto finish = [&](int status) -> int {
        if (cur != (double*)u)
            HIP_CHECK(hipMemcpyAsync(u, cur, sizeof(double) * nL, hipMemcpyDeviceToDevice, s), "copy back");
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return status;
    };
    double r0 = 0.0;
    if ((rc = first_norm(&r0))) return rc;
    st->res0 = r0;
    // the learned smoother runs only when a network is loaded and accepted
    int smoother = HHG_SMOOTH_GS;
    if (o->mode == HHG_MODE_LEARNED) {
        if (M->net_loaded && M->net_accepted) smoother = HHG_SMOOTH_NET;
        else st->fallback = 1;
    }
    st->smoother_used = smoother;
    if (o->res_history && o->history_capacity > 0) o->res_history[0] = r0;
    if (r0 == 0.0) {
        st->converged = 1;
        st->rel_res = 0.0;
        return finish(HHG_OK);
    }
    double prev = r0;
    int rising = 0;
    int status = HHG_ENOTCONV;
    for (int it = 0; it < o->max_iters; ++it) {
        double rn = 0.0;
        const bool learned = smoother == HHG_SMOOTH_NET;
        if (!mp) {
            if ((rc = vcycle_rec(M, L, o->op, HHG_SMOOTH_GS, HHG_F64, u, f, o->nu1, o->nu2, s, dnorm)))
                return rc;
            if ((rc = read_norm_slot(M, &rn, s))) return rc;
        } else {
            HIP_CHECK(launch_fill(e32, nL, HHG_F32, 0.0, s), "fill");
            if ((rc = vcycle_rec(M, L, o->op, smoother, HHG_F32, e32, r32, o->nu1, o->nu2, s))) return rc;
            HIP_CHECK(launch_mp_step(M, L, o->op, cur, e32, (const double*)f, alt, r32, dnorm, s), "update");
            if ((rc = read_norm_slot(M, &rn, s))) return rc;
            if (learned && !(rn <= prev)) {
                // learned smoother guard: the cycle did not lower the residual
                // (or made it non-finite): keep the previous iterate, rebuild
                // its residual and go on with Gauss-Seidel
                if ((rc = first_norm(&rn))) return rc;
                smoother = HHG_SMOOTH_GS;
                st->fallback = 1;
                st->smoother_used = HHG_SMOOTH_GS;
            } else {
                std::swap(cur, alt);
            }
        }
        st->iters = it + 1;
        st->rel_res = rn / r0;
        if (o->res_history && it + 1 < o->history_capacity) o->res_history[it + 1] = rn;
        if (!std::isfinite(rn)) {
            g_err = "residual is not finite";
            break;
        }
        if (rn <= o->rtol * r0) {
            st->converged = 1;
            status = HHG_OK;
            break;
        }
        rising = (rn > prev) ? rising + 1 : 0;
        if (rising >= 3) {
            g_err = "residual grew in 3 consecutive cycles";
            break;
        }
        prev = rn;
    }
    if (status == HHG_ENOTCONV && g_err.empty()) g_err = "iteration cap reached";
    return finish(status);
}

int hhg_jacobi(const hhg_mesh* M, int32_t level, int32_t op, int32_t dtype, const void* u,
               const void* f, void* rho, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if ((rc = check_op(M, op, dtype))) return rc;
    if (op == HHG_OP_MASS) return fail(HHG_EINVAL, "needs a stiffness operator");
    if (!u || !rho || u == rho || (f && f == rho)) return fail(HHG_EINVAL, "bad buffers");
    HIP_CHECK(launch_jacobi(M, level, op, dtype, u, f, rho, (hipStream_t)stream), "jacobi");
    return HHG_OK;
}

int hhg_dot(const hhg_mesh* M, int32_t level, int32_t dtype, const void* x, const void* y,
            double* out, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (!x || !y || !out) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_dot(M, level, dtype, x, y, out, (hipStream_t)stream), "dot");
    return HHG_OK;
}

int hhg_dot_noalloc(const hhg_mesh* M, int32_t level, int32_t dtype, const void* x, const void* y,
                    double* out, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (!x || !y || !out) return fail(HHG_EINVAL, "null buffer");
    if (!dot_noalloc_fits(M, level))
        return fail(HHG_EINVAL, "dot needs more partial sums than the static scratch holds");
    HIP_CHECK(launch_dot_noalloc(M, level, dtype, x, y, out, (hipStream_t)stream), "dot (static scratch)");
    return HHG_OK;
}

int hhg_axpby(const hhg_mesh* M, int32_t level, int32_t dtype, double alpha, const void* x,
              double beta, const void* y, void* z, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (!x || !y || !z) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_axpby(M->m.lv[level].total, dtype, alpha, x, beta, y, z, (hipStream_t)stream), "axpby");
    return HHG_OK;
}

int hhg_restrict(const hhg_mesh* M, int32_t level, int32_t dtype, const void* r, void* fc, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (level < 2) return fail(HHG_EINVAL, "restriction needs level >= 2");
    if (!r || !fc || r == fc) return fail(HHG_EINVAL, "bad buffers");
    HIP_CHECK(launch_restrict(M, level, dtype, r, fc, nullptr, (hipStream_t)stream), "restrict");
    // the kernel writes owned coarse values (all the V-cycle reads); the call
    // also leaves fc's copies consistent
    HIP_CHECK(launch_sync(M, level - 1, dtype, fc, GM_ALL, (hipStream_t)stream), "restrict copies");
    return HHG_OK;
}

int hhg_prolong_add(const hhg_mesh* M, int32_t level, int32_t dtype, const void* uc, void* u, void* stream) {
    int rc = check_common(M, level, dtype);
    if (rc) return rc;
    if (level < 2) return fail(HHG_EINVAL, "prolongation needs level >= 2");
    if (!uc || !u || uc == u) return fail(HHG_EINVAL, "bad buffers");
    HIP_CHECK(launch_prolong_add(M, level, dtype, uc, u, (hipStream_t)stream), "prolong");
    return HHG_OK;
}

int hhg_convert(const hhg_mesh* M, int32_t level, int32_t src_dtype, const void* src, int32_t dst_dtype,
                void* dst, void* stream) {
    int rc = check_common(M, level, src_dtype);
    if (rc) return rc;
    if (!src || !dst) return fail(HHG_EINVAL, "null buffer");
    const int64_t n = M->m.lv[level].total;
    hipStream_t s = (hipStream_t)stream;
    if (src_dtype == HHG_F64 && dst_dtype == HHG_F32)
        HIP_CHECK(launch_f64_to_f32((const double*)src, (float*)dst, n, s), "convert");
    else if (src_dtype == HHG_F32 && dst_dtype == HHG_F64)
        HIP_CHECK(launch_f32_to_f64((const float*)src, (double*)dst, n, s), "convert");
    else
        return fail(HHG_EINVAL, "only F64 <-> F32 conversions");
    return HHG_OK;
}

static int check_net(const hhg_mesh* M) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!(M->features & HHG_FEAT_NET)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_NET");
    return HHG_OK;
}

int hhg_net_set_weights(hhg_mesh* M, const float* w, int32_t n, void* stream) {
    int rc = check_net(M);
    if (rc) return rc;
    if (!w || n != NET_NW) return fail(HHG_EINVAL, "expected 224 weights");
    hipStream_t s = (hipStream_t)stream;
    HIP_CHECK(hipMemcpyAsync(M->net_w, w, sizeof(float) * NET_NW, hipMemcpyHostToDevice, s), "weights");
    HIP_CHECK(launch_fill(M->net_m, NET_NW, HHG_F32, 0.0, s), "adam state");
    HIP_CHECK(launch_fill(M->net_v, NET_NW, HHG_F32, 0.0, s), "adam state");
    HIP_CHECK(hipStreamSynchronize(s), "weights");
    M->net_loaded = true;
    return HHG_OK;
}

int hhg_net_get_weights(const hhg_mesh* M, float* w, int32_t n, void* stream) {
    int rc = check_net(M);
    if (rc) return rc;
    if (!w || n != NET_NW) return fail(HHG_EINVAL, "expected 224 weights");
    hipStream_t s = (hipStream_t)stream;
    HIP_CHECK(hipMemcpyAsync(w, M->net_w, sizeof(float) * NET_NW, hipMemcpyDeviceToHost, s), "weights");
    HIP_CHECK(hipStreamSynchronize(s), "weights");
    return HHG_OK;
}

int hhg_net_set_options(hhg_mesh* M, int32_t precision, int32_t accepted) {
    int rc = check_net(M);
    if (rc) return rc;
    if (precision != HHG_BF16 && precision != HHG_F32) return fail(HHG_EINVAL, "precision must be BF16 or F32");
    M->net_mfma = precision == HHG_BF16;
    M->net_accepted = accepted != 0;
    return HHG_OK;
}

int hhg_net_forward(const hhg_mesh* M, int32_t level, const void* rho, void* out, void* stream) {
    int rc = check_net(M);
    if (rc) return rc;
    if ((rc = check_common(M, level, HHG_F32))) return rc;
    if (!M->net_loaded) return fail(HHG_EINVAL, "no network weights set");
    if (!rho || !out || rho == out) return fail(HHG_EINVAL, "bad buffers");
    hipStream_t s = (hipStream_t)stream;
    HIP_CHECK(launch_fill(out, M->m.lv[level].total, HHG_F32, 0.0, s), "net forward");
    HIP_CHECK(launch_net_forward(M, level, (const float*)rho, (float*)out, 0, M->net_mfma, s), "net forward");
    return HHG_OK;
}

int hhg_net_backward(const hhg_mesh* M, int32_t level, const void* rho, const void* g, float* dW,
                     void* stream) {
    int rc = check_net(M);
    if (rc) return rc;
    if ((rc = check_common(M, level, HHG_F32))) return rc;
    if (!M->net_loaded) return fail(HHG_EINVAL, "no network weights set");
    if (!rho || !g || !dW) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_net_backward(M, level, (const float*)rho, (const float*)g, dW, M->net_mfma,
                                  (hipStream_t)stream), "net backward");
    return HHG_OK;
}

int hhg_net_adam_step(hhg_mesh* M, const float* grad, float lr, int32_t step, void* stream) {
    int rc = check_net(M);
    if (rc) return rc;
    if (!grad || step < 1 || !(lr > 0.f)) return fail(HHG_EINVAL, "bad Adam arguments");
    HIP_CHECK(launch_net_adam(M, grad, lr, step, (hipStream_t)stream), "adam");
    return HHG_OK;
}

int hhg_set_face_coefficient(hhg_mesh* M, const double* coef, void* stream) {
    if (!M || !coef) return fail(HHG_EINVAL, "null argument");
    const std::string err = M->m.set_face_coef(coef);
    if (!err.empty()) return fail(HHG_EINVAL, err);
    M->stokes_ready = false;
    M->p2_ready = false;
    if (!M->bound) return HHG_OK;
    hipStream_t s = (hipStream_t)stream;
    const MeshData& m = M->m;
    HIP_CHECK(upload(M->d_faces, m.faces, s), "upload");
    HIP_CHECK(upload(M->d_edges, m.edges, s), "upload");
    HIP_CHECK(upload(M->d_verts, m.verts, s), "upload");
    HIP_CHECK(launch_coarse_extract(M, OP_LAPLACE, M->coarse.vals, s), "coarse operator");
    if (M->kappa_set) HIP_CHECK(launch_coarse_extract(M, OP_DIFFUSION, M->coarse_vals_diff, s), "coarse operator");
    M->inv_ok[0] = M->inv_ok[1] = false;
    HIP_CHECK(hipStreamSynchronize(s), "face coefficient");
    return HHG_OK;
}

int hhg_stokes_setup(hhg_mesh* M, const double* viscosity, double delta, void* stream) {
    if (!M || !viscosity) return fail(HHG_EINVAL, "null argument");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!(M->features & HHG_FEAT_STOKES)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_STOKES");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(HHG_EINVAL, "delta must be positive");
    int rc = hhg_set_face_coefficient(M, viscosity, stream);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    MeshData& m = M->m;
    m.stokes_tables(delta);
    m.fv_tables();
    HIP_CHECK(upload(M->d_sfaces, m.sfaces, s), "upload");
    HIP_CHECK(upload(M->d_sedges, m.sedges, s), "upload");
    HIP_CHECK(upload(M->d_sverts, m.sverts, s), "upload");
    HIP_CHECK(upload(M->d_fvfaces, m.fvfaces, s), "upload");
    HIP_CHECK(upload(M->d_vxy, m.vxy, s), "upload");
    HIP_CHECK(hipStreamSynchronize(s), "stokes setup");
    M->stokes_delta = delta;
    M->stokes_ready = true;
    return HHG_OK;
}

namespace {

int check_stokes(const hhg_mesh* M, int level) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!(M->features & HHG_FEAT_STOKES)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_STOKES");
    if (!M->stokes_ready) return fail(HHG_EINVAL, "hhg_stokes_setup has not been called");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    return HHG_OK;
}

// Velocity blocks of the preconditioner: z_c = one V(nu1, nu2) cycle of the
// viscous operator from zero on r_c, for c = x, y (FP64, or FP32 cycles on
// the rounded residual with the result raised to FP64).
int stokes_vel_precond(const hhg_mesh* M, int prec, const double* r, double* z, int nu1, int nu2,
                       hipStream_t s) {
    const int L = M->m.L;
    const int64_t fs = M->m.lv[L].total;
    for (int c = 0; c < 2; ++c) {
        const double* rc_ = r + c * fs;
        double* zc = z + c * fs;
        if (prec == HHG_F64) {
            HIP_CHECK(launch_fill(zc, fs, HHG_F64, 0.0, s), "precond");
            int rc = vcycle_rec(M, L, HHG_OP_LAPLACE, HHG_SMOOTH_GS, HHG_F64, zc, rc_, nu1, nu2, s);
            if (rc) return rc;
        } else {
            float* u32 = (float*)M->u32[L];
            float* f32 = (float*)M->f32[L];
            HIP_CHECK(launch_f64_to_f32(rc_, f32, fs, s), "precond");
            HIP_CHECK(launch_fill(u32, fs, HHG_F32, 0.0, s), "precond");
            int rc = vcycle_rec(M, L, HHG_OP_LAPLACE, HHG_SMOOTH_GS, HHG_F32, u32, f32, nu1, nu2, s);
            if (rc) return rc;
            HIP_CHECK(launch_f32_to_f64(u32, zc, fs, s), "precond");
        }
    }
    return HHG_OK;
}

int check_stokes_prec(const hhg_mesh* M, int prec, int nu1, int nu2) {
    if (prec != HHG_F64 && prec != HHG_F32) return fail(HHG_EINVAL, "precision must be HHG_F64 or HHG_F32");
    if (prec == HHG_F32 && !(M->features & HHG_FEAT_MP))
        return fail(HHG_ENOMEM, "FP32 preconditioner needs HHG_FEAT_MP");
    if (nu1 < 0 || nu2 < 0 || nu1 + nu2 == 0) return fail(HHG_EINVAL, "need at least one smoothing sweep");
    return HHG_OK;
}

}  // namespace

int hhg_stokes_apply(const hhg_mesh* M, int32_t level, const void* x, void* y, void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!x || !y || x == y) return fail(HHG_EINVAL, "x and y must be distinct buffers");
    HIP_CHECK(launch_stokes_apply(M, level, 0, (const double*)x, nullptr, (double*)y, M->partials, nullptr,
                                  (hipStream_t)stream), "stokes apply");
    return HHG_OK;
}

int hhg_stokes_residual(const hhg_mesh* M, int32_t level, const void* x, const void* b, void* r,
                        void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!x || !b || !r || r == x || r == b) return fail(HHG_EINVAL, "r must be distinct from x and b");
    HIP_CHECK(launch_stokes_apply(M, level, 2, (const double*)x, (const double*)b, (double*)r, M->partials,
                                  nullptr, (hipStream_t)stream), "stokes residual");
    return HHG_OK;
}

int hhg_stokes_precond(const hhg_mesh* M, int32_t precision, const void* r, void* z, int32_t nu1,
                       int32_t nu2, void* stream) {
    const int L = M ? M->m.L : 0;
    int rc = check_stokes(M, L);
    if (rc) return rc;
    if ((rc = check_stokes_prec(M, precision, nu1, nu2))) return rc;
    if (!r || !z || r == z) return fail(HHG_EINVAL, "r and z must be distinct buffers");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = stokes_vel_precond(M, precision, (const double*)r, (double*)z, nu1, nu2, s))) return rc;
    HIP_CHECK(launch_stokes_pscale_dot(M, L, (const double*)r, (double*)z, M->partials, nullptr, s), "precond");
    return HHG_OK;
}

int hhg_stokes_dot(const hhg_mesh* M, int32_t level, const void* a, const void* b, double* out,
                   void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!a || !b || !out) return fail(HHG_EINVAL, "null buffer");
    hipStream_t s = (hipStream_t)stream;
    int64_t np = 0;
    HIP_CHECK(launch_stokes_dot(M, level, (const double*)a, (const double*)b, M->partials, &np, s), "dot");
    HIP_CHECK(launch_reduce(M->partials, np, out, s), "dot");
    return HHG_OK;
}

namespace {

// MINRES on the finest level (see hhg_stokes_solve); arguments checked.
int stokes_minres(hhg_mesh* M, const hhg_stokes_opts* o, void* x_, const void* b_, hhg_stokes_stats* st,
                  hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    *st = hhg_stokes_stats{};
    const int L = M->m.L;
    int rc = 0;
    double* x = (double*)x_;
    const double* b = (const double*)b_;
    const int64_t n3 = 3 * M->m.lv[L].total;
    double* R[2] = {M->s_vec[0], M->s_vec[1]};   // r_k, r_{k-1} (then r_{k+1})
    double* Y[2] = {M->s_vec[2], M->s_vec[3]};   // y_k = P^-1 r_k, y_{k+1}
    double* KY = M->s_vec[4];
    double* W[2] = {M->s_vec[5], M->s_vec[6]};   // w_{k-1}, w_{k-2}
    double* sst = M->s_state;
    double* slot = M->h_norm_dev;
    volatile const double* hslot = M->h_norm;
    int64_t np = 0;
    for (double* v : {R[1], W[0], W[1]}) HIP_CHECK(launch_fill(v, n3, HHG_F64, 0.0, s), "solve");
    HIP_CHECK(launch_stokes_apply(M, L, 2, x, b, R[0], M->partials, nullptr, s), "residual");
    if ((rc = stokes_vel_precond(M, o->precision, R[0], Y[0], o->nu1, o->nu2, s))) return rc;
    HIP_CHECK(launch_stokes_pscale_dot(M, L, R[0], Y[0], M->partials, &np, s), "precond");
    HIP_CHECK(launch_minres_scalars(0, M->partials, np, sst, slot, s), "minres");
    HIP_CHECK(hipStreamSynchronize(s), "minres");
    const double beta1 = hslot[2];
    st->res0 = beta1;
    int hist_n = 0;
    auto record = [&](double v) {
        if (o->res_history && hist_n < o->history_capacity) o->res_history[hist_n] = v;
        ++hist_n;
    };
    record(beta1);
    auto finish = [&](int status) {
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return status;
    };
    if (!std::isfinite(beta1)) return finish(fail(HHG_ENOTCONV, "non-finite initial residual"));
    if (!(beta1 > 0.0)) {
        st->converged = 1;
        return finish(HHG_OK);
    }
    double rel = 1.0;
    for (int k = 1; k <= o->max_iters; ++k) {
        HIP_CHECK(launch_stokes_apply(M, L, 1, Y[0], nullptr, KY, M->partials, &np, s), "minres apply");
        HIP_CHECK(launch_minres_scalars(1, M->partials, np, sst, slot, s), "minres");
        HIP_CHECK(launch_minres_rupdate(n3, KY, R[0], R[1], sst, s), "minres");
        if ((rc = stokes_vel_precond(M, o->precision, R[1], Y[1], o->nu1, o->nu2, s))) return finish(rc);
        HIP_CHECK(launch_stokes_pscale_dot(M, L, R[1], Y[1], M->partials, &np, s), "minres precond");
        HIP_CHECK(launch_minres_scalars(2, M->partials, np, sst, slot, s), "minres");
        HIP_CHECK(launch_minres_wupdate(n3, Y[0], W[0], W[1], x, sst, s), "minres");
        HIP_CHECK(hipStreamSynchronize(s), "minres");
        const double eta = hslot[0], bnext = hslot[1];
        rel = eta / beta1;
        record(eta);
        st->iters = k;
        st->rel_res = rel;
        if (!std::isfinite(eta)) return finish(fail(HHG_ENOTCONV, "non-finite residual"));
        if (rel <= o->rtol || bnext == 0.0) {
            st->converged = 1;
            return finish(HHG_OK);
        }
        std::swap(R[0], R[1]);
        std::swap(Y[0], Y[1]);
        std::swap(W[0], W[1]);
    }
    return finish(fail(HHG_ENOTCONV, "MINRES iteration cap reached"));
}

int check_stokes_opts(const hhg_mesh* M, const hhg_stokes_opts* o) {
    int rc = check_stokes_prec(M, o->precision, o->nu1, o->nu2);
    if (rc) return rc;
    if (o->max_iters < 0 || !(o->rtol >= 0)) return fail(HHG_EINVAL, "bad solve options");
    if (!M->h_norm) return fail(HHG_ENOMEM, "no norm slot: bind a workspace first");
    return HHG_OK;
}

}  // namespace

int hhg_stokes_solve(hhg_mesh* M, const hhg_stokes_opts* o, void* x_, const void* b_, hhg_stokes_stats* st,
                     void* stream) {
    if (!o || !st) return fail(HHG_EINVAL, "null argument");
    *st = hhg_stokes_stats{};
    const int L = M ? M->m.L : 0;
    int rc = check_stokes(M, L);
    if (rc) return rc;
    if ((rc = check_stokes_opts(M, o))) return rc;
    if (!x_ || !b_ || x_ == b_) return fail(HHG_EINVAL, "x and b must be distinct buffers");
    return stokes_minres(M, o, x_, b_, st, (hipStream_t)stream);
}

int hhg_cell_coords(const hhg_mesh* M, int32_t level, double* xy) {
    if (!M || !xy) return fail(HHG_EINVAL, "null argument");
    if (!level_ok(M, level)) return fail(HHG_EINVAL, "level out of range");
    const MeshData& m = M->m;
    const int n = m.lv[level].n;
    int64_t c = 0;
    for (int f = 0; f < m.F; ++f) {
        const double* x0 = &m.vxy[2 * m.tri[f][0]];
        const double* x1 = &m.vxy[2 * m.tri[f][1]];
        const double* x2 = &m.vxy[2 * m.tri[f][2]];
        // up cells, then down cells, j-major: centroid at (i + 1/3, j + 1/3)
        // and (i + 2/3, j + 2/3) in face-local steps
        for (int kind = 0; kind < 2; ++kind)
            for (int j = 0; j <= n - 2 - kind; ++j)
                for (int i = 0; i <= n - 2 - kind - j; ++i, ++c) {
                    const double o = kind ? 2.0 / 3.0 : 1.0 / 3.0;
                    const double si = (i + o) / (n - 1), sj = (j + o) / (n - 1);
                    xy[2 * c] = x0[0] + si * (x1[0] - x0[0]) + sj * (x2[0] - x0[0]);
                    xy[2 * c + 1] = x0[1] + si * (x1[1] - x0[1]) + sj * (x2[1] - x0[1]);
                }
    }
    return HHG_OK;
}

int hhg_cells_from_canonical(const hhg_mesh* M, int32_t level, const double* canon, double* cells,
                             void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!canon || !cells) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_cell_canon(M, level, canon, cells, 0, (hipStream_t)stream), "cells");
    return HHG_OK;
}

int hhg_cells_to_canonical(const hhg_mesh* M, int32_t level, const double* cells, double* canon,
                           void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!canon || !cells) return fail(HHG_EINVAL, "null buffer");
    HIP_CHECK(launch_cell_canon(M, level, cells, canon, 1, (hipStream_t)stream), "cells");
    return HHG_OK;
}

int hhg_transport_step(const hhg_mesh* M, int32_t level, const double* x, const double* T_in,
                       double* T_out, double dt, void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!x || !T_in || !T_out || T_in == T_out) return fail(HHG_EINVAL, "T_in and T_out must be distinct");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(HHG_EINVAL, "bad time step");
    const int64_t fs = M->m.lv[level].total;
    HIP_CHECK(launch_fv_step(M, level, x, x + fs, T_in, T_out, dt, (hipStream_t)stream), "transport");
    return HHG_OK;
}

int hhg_buoyancy(const hhg_mesh* M, int32_t level, const double* T, double Ra, double* b, void* stream) {
    int rc = check_stokes(M, level);
    if (rc) return rc;
    if (!T || !b) return fail(HHG_EINVAL, "null buffer");
    hipStream_t s = (hipStream_t)stream;
    const int64_t fs = M->m.lv[level].total;
    HIP_CHECK(launch_fill(b + 2 * fs, fs, HHG_F64, 0.0, s), "buoyancy");
    HIP_CHECK(launch_fv_buoyancy(M, level, T, Ra, b, s), "buoyancy");
    return HHG_OK;
}

int hhg_energy_run(hhg_mesh* M, const hhg_energy_opts* o, void* x, void* T, hhg_energy_stats* st,
                   void* stream) {
    if (!o || !st) return fail(HHG_EINVAL, "null argument");
    *st = hhg_energy_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    const int L = M ? M->m.L : 0;
    int rc = check_stokes(M, L);
    if (rc) return rc;
    if ((rc = check_stokes_opts(M, &o->stokes))) return rc;
    if (!x || !T) return fail(HHG_EINVAL, "null buffer");
    if (o->steps < 0 || o->stokes_every < 1 || !(o->dt >= 0.0) || !std::isfinite(o->dt) || !std::isfinite(o->Ra))
        return fail(HHG_EINVAL, "bad energy options");
    hipStream_t s = (hipStream_t)stream;
    const int64_t fs = M->m.lv[L].total;
    double* cur = (double*)T;
    double* other = M->t_cells;
    double* xs = (double*)x;
    hhg_stokes_opts so = o->stokes;
    so.res_history = nullptr;
    so.history_capacity = 0;
    for (int k = 0; k < o->steps; ++k) {
        if (k % o->stokes_every == 0) {
            HIP_CHECK(launch_fill(M->b_stokes + 2 * fs, fs, HHG_F64, 0.0, s), "buoyancy");
            HIP_CHECK(launch_fv_buoyancy(M, L, cur, o->Ra, M->b_stokes, s), "buoyancy");
            hhg_stokes_stats ss;
            rc = stokes_minres(M, &so, xs, M->b_stokes, &ss, s);
            st->stokes_solves++;
            st->minres_iters += ss.iters;
            st->worst_rel_res = std::max(st->worst_rel_res, ss.rel_res);
            if (rc) break;
        }
        HIP_CHECK(launch_fv_step(M, L, xs, xs + fs, cur, other, o->dt, s), "transport");
        std::swap(cur, other);
        st->steps = k + 1;
    }
    if (cur != (double*)T) HIP_CHECK(hipMemcpyAsync(T, cur, sizeof(double) * 2 * fs, hipMemcpyDeviceToDevice, s),
                                     "copy back");
    HIP_CHECK(hipStreamSynchronize(s), "energy run");
    st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

// ------------------------------------------------------------------ P2

namespace {

int check_p2(const hhg_mesh* M, int level) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!(M->features & HHG_FEAT_P2)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_P2");
    if (!M->p2_ready) return fail(HHG_EINVAL, "hhg_p2_setup has not been called since the last coefficient change");
    if (level < 1 || level + 1 > M->m.L) return fail(HHG_EINVAL, "P2 level must satisfy 1 <= level < max_level");
    return HHG_OK;
}

// `sweeps` Jacobi sweeps ping-ponging between x and y; *out: the buffer
// holding the result.
int p2_jacobi_pp(const hhg_mesh* M, int fl, double omega, double* x, double* y, const double* f, int sweeps,
                 hipStream_t s, double** out) {
    double* cur = x;
    double* other = y;
    for (int k = 0; k < sweeps; ++k) {
        HIP_CHECK(launch_p2(M, fl, 2, cur, f, other, M->p2part, omega, s), "P2 Jacobi");
        std::swap(cur, other);
    }
    *out = cur;
    return HHG_OK;
}

}  // namespace

int hhg_p2_setup(hhg_mesh* M, void* stream) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    if (!M->bound) return fail(HHG_ENOMEM, "no workspace bound");
    if (!(M->features & HHG_FEAT_P2)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_P2");
    const std::string err = M->m.p2_tables();
    if (!err.empty()) return fail(HHG_EINVAL, err);
    hipStream_t s = (hipStream_t)stream;
    HIP_CHECK(upload(M->d_p2faces, M->m.p2faces, s), "upload");
    HIP_CHECK(upload(M->d_p2ediag, M->m.p2ediag, s), "upload");
    HIP_CHECK(upload(M->d_p2vdiag, M->m.p2vdiag, s), "upload");
    HIP_CHECK(hipStreamSynchronize(s), "P2 setup");
    M->p2_ready = true;
    return HHG_OK;
}

int hhg_p2_apply(const hhg_mesh* M, int32_t level, const void* x, void* y, void* stream) {
    int rc = check_p2(M, level);
    if (rc) return rc;
    if (!x || !y || x == y) return fail(HHG_EINVAL, "x and y must be distinct buffers");
    HIP_CHECK(launch_p2(M, level + 1, 0, (const double*)x, nullptr, (double*)y, M->p2part, 0.0,
                        (hipStream_t)stream), "P2 apply");
    return HHG_OK;
}

int hhg_p2_residual(const hhg_mesh* M, int32_t level, const void* x, const void* f, void* r, void* stream) {
    int rc = check_p2(M, level);
    if (rc) return rc;
    if (!x || !f || !r || r == x || r == f) return fail(HHG_EINVAL, "r must be distinct from x and f");
    HIP_CHECK(launch_p2(M, level + 1, 1, (const double*)x, (const double*)f, (double*)r, M->p2part, 0.0,
                        (hipStream_t)stream), "P2 residual");
    return HHG_OK;
}

int hhg_p2_jacobi(const hhg_mesh* M, int32_t level, double omega, const void* x, const void* f, void* y,
                  void* stream) {
    int rc = check_p2(M, level);
    if (rc) return rc;
    if (!x || !f || !y || y == x || y == f) return fail(HHG_EINVAL, "y must be distinct from x and f");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(HHG_EINVAL, "omega must be positive");
    HIP_CHECK(launch_p2(M, level + 1, 2, (const double*)x, (const double*)f, (double*)y, M->p2part, omega,
                        (hipStream_t)stream), "P2 Jacobi");
    return HHG_OK;
}

int hhg_p2_solve(hhg_mesh* M, const hhg_p2_opts* o, void* x_, const void* f_, hhg_p2_stats* st, void* stream) {
    if (!M || !o || !x_ || !f_ || !st) return fail(HHG_EINVAL, "null argument");
    auto t0 = std::chrono::steady_clock::now();
    std::memset(st, 0, sizeof(*st));
    g_err.clear();
    const int l = o->level, fl = l + 1;
    int rc = check_p2(M, l);
    if (rc) return rc;
    if (!(M->features & HHG_FEAT_F64)) return fail(HHG_ENOMEM, "workspace lacks HHG_FEAT_F64");
    if (l < M->m.lc) return fail(HHG_EINVAL, "P2 level below the coarse level");
    if (o->max_iters < 0 || o->nu1 < 0 || o->nu2 < 0 || o->vnu1 < 0 || o->vnu2 < 0 || !(o->rtol >= 0) ||
        !(o->omega > 0.0) || !std::isfinite(o->omega))
        return fail(HHG_EINVAL, "bad P2 solve options");
    if (o->vnu1 + o->vnu2 == 0 && l > M->m.lc) return fail(HHG_EINVAL, "the P1 cycle needs a smoothing sweep");
    hipStream_t s = (hipStream_t)stream;
    double* x = (double*)x_;
    const double* f = (const double*)f_;
    double* tmp = (double*)level_alt(M, fl, HHG_F64);
    double* r = (double*)level_r(M, fl, HHG_F64);
    void* uc = level_u(M, l, HHG_F64);
    void* fc = level_f(M, l, HHG_F64);
    const int64_t nfl = M->m.lv[fl].total;
    auto res_norm = [&](const double* u, double* out) -> int {
        HIP_CHECK(launch_p2(M, fl, 1, u, f, r, M->p2part, 0.0, s), "P2 residual");
        HIP_CHECK(launch_dot(M, fl, HHG_F64, r, r, M->h_norm_dev, s), "P2 norm");
        double sq = 0.0;
        if ((rc = read_norm_slot(M, &sq, s))) return rc;
        *out = std::sqrt(sq);
        return HHG_OK;
    };
    double r0 = 0.0;
    if ((rc = res_norm(x, &r0))) return rc;
    st->res0 = r0;
    if (o->res_history && o->history_capacity > 0) o->res_history[0] = r0;
    int status = HHG_ENOTCONV;
    if (r0 == 0.0) {
        st->converged = 1;
        status = HHG_OK;
    }
    for (int it = 0; status != HHG_OK && it < o->max_iters; ++it) {
        // nu1 Jacobi sweeps, residual, restriction to P1 (zeroes uc), one P1
        // V-cycle from zero, prolongation and correction, nu2 Jacobi sweeps
        double* cur = nullptr;
        if ((rc = p2_jacobi_pp(M, fl, o->omega, x, tmp, f, o->nu1, s, &cur))) return rc;
        HIP_CHECK(launch_p2(M, fl, 1, cur, f, r, M->p2part, 0.0, s), "P2 residual");
        HIP_CHECK(launch_restrict(M, fl, HHG_F64, r, fc, uc, s), "P2 -> P1");
        if ((rc = vcycle_rec(M, l, HHG_OP_LAPLACE, HHG_SMOOTH_GS, HHG_F64, uc, fc, o->vnu1, o->vnu2, s, nullptr,
                             true)))
            return rc;
        HIP_CHECK(launch_prolong_add(M, fl, HHG_F64, uc, cur, s), "P1 -> P2");
        double* fin = nullptr;
        if ((rc = p2_jacobi_pp(M, fl, o->omega, cur, cur == x ? tmp : x, f, o->nu2, s, &fin))) return rc;
        if (fin != x)
            HIP_CHECK(hipMemcpyAsync(x, fin, sizeof(double) * nfl, hipMemcpyDeviceToDevice, s), "copy back");
        double rn = 0.0;
        if ((rc = res_norm(x, &rn))) return rc;
        st->iters = it + 1;
        st->rel_res = rn / r0;
        if (o->res_history && it + 1 < o->history_capacity) o->res_history[it + 1] = rn;
        if (!std::isfinite(rn)) {
            g_err = "residual is not finite";
            break;
        }
        if (rn <= o->rtol * r0) {
            st->converged = 1;
            status = HHG_OK;
        }
    }
    if (status == HHG_ENOTCONV && g_err.empty()) g_err = "iteration cap reached";
    st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

int hhg_timing_enable(hhg_mesh* M, int32_t enable) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    M->timing = enable != 0;
    return HHG_OK;
}

int hhg_timing_read(hhg_mesh* M, int64_t* launches, double* total_ms, int32_t reset) {
    if (!M) return fail(HHG_EINVAL, "null mesh");
    double tot = 0.0;
    for (int64_t i = 0; i < M->t_launches; ++i) {
        hipEvent_t a = (hipEvent_t)M->t_events[i].first, b = (hipEvent_t)M->t_events[i].second;
        HIP_CHECK(hipEventSynchronize(b), "timing");
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, a, b), "timing");
        tot += ms;
    }
    if (launches) *launches = M->t_launches;
    if (total_ms) *total_ms = tot;
    if (reset) M->t_launches = 0;
    return HHG_OK;
}

}  // extern "C"
