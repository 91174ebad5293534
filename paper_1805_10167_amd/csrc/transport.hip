// HIP kernels (gfx950) of the energy-transport coupling of the paper's
// example application (sec. 5.2): the temperature lives on the interiors of
// the micro-triangles (finite-volume unknowns, sec. 3.1) and is advanced by
// an explicit upwind step with the P1 velocity of the last Stokes solve; the
// Stokes solve is driven by the buoyancy load of that temperature.
//
// A cell field of level l is two point-layout fields, [up | down], each of
// the level's field length: the up cell {(i,j), (i+1,j), (i,j+1)} of a face
// is kept at the slot of point (i, j) of the first, the down cell
// {(i+1,j), (i+1,j+1), (i,j+1)} at the slot of point (i, j) of the second.
// Only face slots are used.  Canonical cell order: per face in input order,
// the up cells j-major, then the down cells j-major ((n-1)^2 per face).
//
// Flux through a micro-edge of a cell: |e| n . (u_a + u_b) / 2 with n the
// outward unit normal (the exact flux of the linear velocity along e); the
// two cells of an edge compute it from the same values with negated normals,
// so their fluxes cancel exactly.  Micro-edges on the domain boundary carry
// no flux (the velocity vanishes there).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "hhg_device.hpp"

namespace hhg {

// Slot of the up cell at position t along side s of a face (the cell whose
// edge is the micro-edge between side positions t and t+1).
__device__ __forceinline__ int64_t side_up_cell(const LevelDev& L, int face, int s, int t) {
    const int n = L.n;
    int i, j;
    if (s == 0) { i = t; j = 0; }
    else if (s == 1) { i = 0; j = t; }
    else { i = n - 2 - t; j = t; }
    return face_base(L, face) + row_start(n, j) + i;
}

// Temperature across side s of face `face` at position t (the up cell of the
// neighbouring face), or the cell's own value on the domain boundary (its
// flux is zero there anyway).
__device__ __forceinline__ double across(const LevelDev& L, const FvFace& fv, int s, int t,
                                         const double* __restrict__ Tup, double own) {
    const int nf = fv.nbr_face[s];
    if (nf < 0) return own;
    const int tt = fv.nbr_flip[s] ? L.n - 2 - t : t;
    return Tup[side_up_cell(L, nf, fv.nbr_side[s], tt)];
}

// Outward flux h n . (u_a + u_b) / 2 (n: unit-scale normal times length).
__device__ __forceinline__ double flux(const double* n, double h, double uxa, double uya, double uxb,
                                       double uyb) {
    return h * (n[0] * (0.5 * (uxa + uxb)) + n[1] * (0.5 * (uya + uyb)));
}

// One explicit upwind step Tout = Tin - dt / |c| sum_e F_e T_up(e) on every
// cell; ux, uy are the velocity point fields.  A thread takes the up cell
// and the down cell of one face-local (i, j).
__global__ __launch_bounds__(NT) void k_fv_step(LevelDev L, const double* __restrict__ ux,
                                                const double* __restrict__ uy, const double* __restrict__ Tin,
                                                double* __restrict__ Tout, int64_t fs, double dt) {
    const double* Tup = Tin;
    const double* Tdn = Tin + fs;
    const double h = ldexp(1.0, -L.level);
    FACE_ALL_LOOP(L, gridDim.x)
    (void)interior;
    (void)fi;
    if (i + j > n - 2) continue;
    const FvFace& fv = L.fvfaces[face];
    const int64_t up = row_start(n, j + 1) - row_start(n, j);
    const int64_t dn = j > 0 ? row_start(n, j) - row_start(n, j - 1) : 0;
    const double rc = dt / (h * h * fv.area);
    // velocities at (i,j), (i+1,j), (i,j+1)
    const double x0 = ux[p], y0 = uy[p], x1 = ux[p + 1], y1 = uy[p + 1];
    const double x2 = ux[p + up], y2 = uy[p + up];
    const double Tc = Tup[p];
    const double Fb = j > 0 || fv.nbr_face[0] >= 0 ? flux(fv.nb, h, x0, y0, x1, y1) : 0.0;
    const double Fl = i > 0 || fv.nbr_face[1] >= 0 ? flux(fv.nl, h, x0, y0, x2, y2) : 0.0;
    const double Fd = i + j < n - 2 || fv.nbr_face[2] >= 0 ? flux(fv.nd, h, x1, y1, x2, y2) : 0.0;
    const double Tb = j > 0 ? Tdn[p - dn] : across(L, fv, 0, i, Tup, Tc);
    const double Tl = i > 0 ? Tdn[p - 1] : across(L, fv, 1, j, Tup, Tc);
    const double Td = i + j < n - 2 ? Tdn[p] : across(L, fv, 2, j, Tup, Tc);
    const double sum = Fb * (Fb > 0.0 ? Tc : Tb) + Fl * (Fl > 0.0 ? Tc : Tl) + Fd * (Fd > 0.0 ? Tc : Td);
    Tout[p] = Tc - rc * sum;
    if (i + j <= n - 3) {
        // down cell: diagonal (shared with this up cell), top (up cell
        // (i, j+1)), right (up cell (i+1, j)); all neighbours in the face
        const double x3 = ux[p + up + 1], y3 = uy[p + up + 1];
        const double Td0 = Tdn[p];
        const double Gd = -Fd;
        const double Gt = -flux(fv.nb, h, x2, y2, x3, y3);
        const double Gr = -flux(fv.nl, h, x1, y1, x3, y3);
        const double s2 = Gd * (Gd > 0.0 ? Td0 : Tc) + Gt * (Gt > 0.0 ? Td0 : Tup[p + up]) +
                          Gr * (Gr > 0.0 ? Td0 : Tup[p + 1]);
        Tout[fs + p] = Td0 - rc * s2;
    }
    }
}

// Sum of T |c| / 3 over the cells around face-local point (i, j) of a face
// (the up cells (i,j), (i-1,j), (i,j-1) and the down cells (i-1,j-1),
// (i-1,j), (i,j-1) that exist).
__device__ __forceinline__ double cell_gather(const LevelDev& L, int face, int i, int j, const double* Tup,
                                              const double* Tdn, double third_area) {
    const int n = L.n;
    const int64_t fb = face_base(L, face);
    auto at = [&](int a, int b) { return fb + row_start(n, b) + a; };
    double s = 0.0;
    if (i + j <= n - 2) s += Tup[at(i, j)];
    if (i >= 1 && i - 1 + j <= n - 2) s += Tup[at(i - 1, j)];
    if (j >= 1 && i + j - 1 <= n - 2) s += Tup[at(i, j - 1)];
    if (i >= 1 && j >= 1 && i + j - 2 <= n - 3) s += Tdn[at(i - 1, j - 1)];
    if (i >= 1 && i - 1 + j <= n - 3) s += Tdn[at(i - 1, j)];
    if (j >= 1 && i + j - 1 <= n - 3) s += Tdn[at(i, j - 1)];
    return s * third_area;
}

// Buoyancy load b = -Ra r_hat(x_p) sum_{c around p} T_c |c| / 3 in the
// velocity fields of the Stokes vector b (copies written; zero at Dirichlet
// points); the pressure field is left to the caller.
__global__ __launch_bounds__(NT) void k_fv_buoyancy(LevelDev L, const double* __restrict__ T, double Ra,
                                                    double* __restrict__ b, int64_t fs, int gf) {
    const double* Tup = T;
    const double* Tdn = T + fs;
    const double h = ldexp(1.0, -L.level);
    double* bx = b;
    double* by = b + fs;
    if ((int)blockIdx.x < gf) {
        FACE_TILE_LOOP(L, gf)
        (void)up;
        (void)dn;
        const FvFace& fv = L.fvfaces[face];
        const double s = cell_gather(L, face, i, j, Tup, Tdn, h * h * fv.area / 3.0);
        const double x = fv.x0[0] + h * (i * fv.e1[0] + j * fv.e2[0]);
        const double y = fv.x0[1] + h * (i * fv.e1[1] + j * fv.e2[1]);
        const double r = sqrt(x * x + y * y);
        const double vx = -Ra * s * x / r, vy = -Ra * s * y / r;
        bx[p] = vx;
        by[p] = vy;
        push_face_near(L, bx, fi, i, j, vx);
        push_face_near(L, by, fi, i, j, vy);
        FACE_TILE_END
    } else {
        LOW_LOOP(L, gf) {
            double vx = 0.0, vy = 0.0;
            if (t < ne_) {
                const int e = (int)(t / (nl_ - 2)), k = (int)(t % (nl_ - 2)) + 1;
                const EdgeInfo& ei = L.edges[e];
                if (!ei.boundary) {
                    double s = 0.0;
                    for (int q = 0; q < ei.nf; ++q) {
                        const int f = ei.face[q], sd = ei.side[q];
                        const int tt = ei.rev[q] ? nl_ - 1 - k : k;
                        int i, j;
                        if (sd == 0) { i = tt; j = 0; }
                        else if (sd == 1) { i = 0; j = tt; }
                        else { i = nl_ - 1 - tt; j = tt; }
                        s += cell_gather(L, f, i, j, Tup, Tdn, h * h * L.fvfaces[f].area / 3.0);
                    }
                    const double xa = L.vxy[2 * ei.a], ya = L.vxy[2 * ei.a + 1];
                    const double x = xa + (double)k / (nl_ - 1) * (L.vxy[2 * ei.b] - xa);
                    const double y = ya + (double)k / (nl_ - 1) * (L.vxy[2 * ei.b + 1] - ya);
                    const double r = sqrt(x * x + y * y);
                    vx = -Ra * s * x / r;
                    vy = -Ra * s * y / r;
                }
                const int64_t m = edge_main(L, e) + k;
                bx[m] = vx;
                by[m] = vy;
                push_edge(L, bx, ei, k, vx, true);
                push_edge(L, by, ei, k, vy, true);
            } else {
                const int v = (int)(t - ne_);
                const VertexInfo& vi = L.verts[v];
                if (!vi.boundary) {
                    double s = 0.0;
                    for (int c = 0; c < vi.nfc; ++c) {
                        const int f = vi.fc_face[c], cr = vi.fc_corner[c];
                        const int i = cr == 1 ? nl_ - 1 : 0, j = cr == 2 ? nl_ - 1 : 0;
                        s += cell_gather(L, f, i, j, Tup, Tdn, h * h * L.fvfaces[f].area / 3.0);
                    }
                    const double x = L.vxy[2 * v], y = L.vxy[2 * v + 1];
                    const double r = sqrt(x * x + y * y);
                    vx = -Ra * s * x / r;
                    vy = -Ra * s * y / r;
                }
                const int64_t vb = vert_off(L, v);
                bx[vb] = vx;
                by[vb] = vy;
                push_vertex(L, bx, vi, vx);
                push_vertex(L, by, vi, vy);
            }
        }
    }
}

// Canonical cell order <-> cell field (to_canon = 1: field -> canonical).
__global__ __launch_bounds__(NT) void k_cell_canon(LevelDev L, const double* __restrict__ src,
                                                   double* __restrict__ dst, int64_t fs, int to_canon) {
    FACE_ALL_LOOP(L, gridDim.x)
    (void)interior;
    (void)fi;
    if (i + j > n - 2) continue;
    const int64_t per = (int64_t)(n - 1) * (n - 1), nup = (int64_t)n * (n - 1) / 2;
    const int64_t cu = face * per + (int64_t)j * (n - 1) - (int64_t)j * (j - 1) / 2 + i;
    if (to_canon) dst[cu] = src[p];
    else dst[p] = src[cu];
    if (i + j <= n - 3) {
        const int64_t cd = face * per + nup + (int64_t)j * (n - 2) - (int64_t)j * (j - 1) / 2 + i;
        if (to_canon) dst[cd] = src[fs + p];
        else dst[fs + p] = src[cd];
    }
    }
}

// ------------------------------------------------------------------ launchers

static inline int fv_grid(const LevelDev& L) {
    const int64_t g = (int64_t)L.F * L.ntiles;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, MAX_FACE_BLOCKS));
}

hipError_t launch_fv_step(const hhg_mesh* M, int level, const double* ux, const double* uy, const double* Tin,
                          double* Tout, double dt, hipStream_t s) {
    const LevelDev L = M->dev(level);
    k_fv_step<<<fv_grid(L), NT, 0, s>>>(L, ux, uy, Tin, Tout, L.total, dt);
    return hipGetLastError();
}

hipError_t launch_fv_buoyancy(const hhg_mesh* M, int level, const double* T, double Ra, double* b,
                              hipStream_t s) {
    const LevelDev L = M->dev(level);
    const int gf = fv_grid(L);
    int64_t gl = ((int64_t)L.E * (L.n - 2) + L.V + NT - 1) / NT;
    gl = std::max<int64_t>(1, std::min<int64_t>(gl, MAX_LOW_BLOCKS));
    k_fv_buoyancy<<<gf + (int)gl, NT, 0, s>>>(L, T, Ra, b, L.total, gf);
    return hipGetLastError();
}

hipError_t launch_cell_canon(const hhg_mesh* M, int level, const double* src, double* dst, int to_canon,
                             hipStream_t s) {
    const LevelDev L = M->dev(level);
    k_cell_canon<<<fv_grid(L), NT, 0, s>>>(L, src, dst, L.total, to_canon);
    return hipGetLastError();
}

}  // namespace hhg
