// HIP kernels (gfx950) of quadratic (P2) elements on the refined
// macro-faces (sec. 3.1: unknowns on micro-vertices and micro-edges, the edge
// unknowns in three subgroups by edge direction; sec. 4.2: one stencil per
// unknown type) and the Jacobi smoother of the p-multigrid cycle (sec. 4.3).
//
// The P2 unknowns of level l are the points of level l + 1, so a P2 field is
// a field of the level-(l+1) layout (owned values and every ghost copy), and
// the P2 <-> P1 transfers of level l are the level-(l+1) <-> level-l transfers
// of the P1 hierarchy.  A face point (i, j) of the level-(l+1) layout is of
// type (i odd) + 2 (j odd): 0 a vertex of level l, 1 the midpoint of an
// i-direction micro-edge, 2 of a j-direction one, 3 of a diagonal one.
//
// Face-interior rows: the hexagonal 7-point stencil of the point's type (the
// same neighbour offsets as P1), plus, for vertex points, the six vertices two
// steps away.  All of it lies in the face's own array (boundary points
// included as copies), so face rows need no ghost rows.
//
// Edge and vertex rows: each face adds the contributions of its own elements
// to its boundary points (element matrix times the element's values, from
// the face array) into a partial array [face][side][t]; the edge/vertex
// kernel sums the partials of the faces around the point (the finite-element
// assembly of the interface rows), so no second ghost row is needed either.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "hhg_device.hpp"

namespace hhg {

// Local nodes of the up and down element of coarse position (a, b), as
// level-(l+1) offsets from (2a, 2b), in the order v0 v1 v2 m01 m12 m02 (the
// down element is the point reflection of the up one, so the same element
// matrix applies with its v0 at (2, 2), v1 at (0, 2), v2 at (2, 0)).
__device__ __forceinline__ int p2_off(int kind, int r, int c) {
    // [kind][r][c]
    constexpr int OFF[2][6][2] = {{{0, 0}, {2, 0}, {0, 2}, {1, 0}, {1, 1}, {0, 1}},
                                  {{2, 2}, {0, 2}, {2, 0}, {1, 2}, {1, 1}, {2, 1}}};
    return OFF[kind][r][c];
}

// Contribution of the face's own elements to row (I, J) of the face (a
// boundary point): sum over elements containing the point of its element
// matrix row times the element's values.
__device__ __forceinline__ double p2_elem_rows(const LevelDev& L, const P2Face& pf, const double* __restrict__ x,
                                               int face, int I, int J) {
    const int n = L.n, nc = (n + 1) / 2;
    const int64_t fb = face_base(L, face);
    double acc = 0.0;
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const int dx = I - p2_off(kind, r, 0), dy = J - p2_off(kind, r, 1);
            if ((dx | dy) & 1) continue;
            const int a = dx >> 1, b = dy >> 1;
            if (a < 0 || b < 0 || a + b > nc - 2 - kind) continue;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                s += pf.K[r][q] * x[fb + row_start(n, 2 * b + p2_off(kind, q, 1)) + 2 * a + p2_off(kind, q, 0)];
            acc += s;
        }
    }
    return acc;
}

// Face tiles: the smoother's TI x TJ tiles (halo-3 tile list, TI = 186,
// TJ = 24) loaded with a two-point halo into LDS in one round of independent
// loads (f of the block's points into registers alongside), every interior
// row then formed from LDS.  A row (fixed j) holds two point types, chosen
// per lane by selects.
constexpr int P2_NT = 512, P2_NW = P2_NT / 64, P2_H = 2;
constexpr int P2_TJ = GS_TJ, P2_TI = GS_W - 2 * GS_H;
constexpr int P2_RA = P2_TJ + 2 * P2_H, P2_RPW = (P2_RA + P2_NW - 1) / P2_NW, P2_KR = P2_TJ / P2_NW;
static_assert(P2_TI + 2 * P2_H <= GS_W, "tile with halo must fit an LDS row");
static_assert(P2_TJ % P2_NW == 0, "tile rows must split evenly over the waves");

// MODE 0: y = A x; 1: y = f - A x; 2: y = x + omega D^-1 (f - A x).  Blocks
// [0, gt) take face tiles (interior rows, with their ghost-row copies), the
// rest the boundary partials of every face.
template <int MODE>
__global__ __launch_bounds__(P2_NT) void k_p2_face(LevelDev L, const double* __restrict__ x,
                                                   const double* __restrict__ f, double* __restrict__ y,
                                                   double* __restrict__ part, double omega, int ntiles, int gt) {
    __shared__ double xs[P2_RA][GS_W];
    const int b = blockIdx.x, n = L.n;
    if (b < gt) {
        const int logical = (b & 7) * (gt >> 3) + (b >> 3);   // contiguous tiles per XCD
        if (logical >= ntiles) return;
        const int wv = wave_id(), lane = threadIdx.x & 63;
        const int ntl = L.n_gs_tl[0][0];
        const int face = logical / ntl;
        const FaceInfo& fi = L.faces[face];
        const FaceGhosts gh = face_ghosts(L, fi);
        const P2Face& pf = L.p2faces[face];
        const int2 tl = L.gs_tl[0][0][logical % ntl];
        const int i0 = tl.x * P2_TI - P2_H, j0 = tl.y * P2_TJ - P2_H;   // LDS origin
        const int64_t fb = face_base(L, face);
        double xr[P2_RPW][3];
#pragma unroll
        for (int q = 0; q < P2_RPW; ++q) {
            const int r = wv + P2_NW * q, j = j0 + r;
            const int64_t rb = fb + row_start(n, j < 0 ? 0 : (j > n ? n : j));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int tx = lane + 64 * c, i = i0 + tx;
                const bool in = r < P2_RA && tx < P2_TI + 2 * P2_H && j >= 0 && j < n && i >= 0 && i <= n - 1 - j;
                xr[q][c] = in ? x[rb + i] : 0.0;
            }
        }
        double fr[P2_KR][3];
#pragma unroll
        for (int k = 0; k < P2_KR; ++k) {
            const int r = P2_H + wv + P2_NW * k, j = j0 + r;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int tx = lane + 64 * c, i = i0 + tx;
                const bool pt = MODE >= 1 && tx >= P2_H && tx < P2_H + P2_TI && j >= 1 && i >= 1 && i + j <= n - 2;
                fr[k][c] = pt ? f[fb + row_start(n, pt ? j : 0) + i] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < P2_RPW; ++q) {
            const int r = wv + P2_NW * q;
            if (r >= P2_RA) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) xs[r][lane + 64 * c] = xr[q][c];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < P2_KR; ++k) {
            const int r = P2_H + wv + P2_NW * k, j = j0 + r;
            // the row's two types (wave-uniform): even rows vertex / i-edge,
            // odd rows j-edge / diagonal; lanes pick by the parity of i
            const int ta = (j & 1) << 1;
            double wa[7], wb[7];
#pragma unroll
            for (int t = 0; t < 7; ++t) {
                wa[t] = pf.hex[ta][t];
                wb[t] = pf.hex[ta | 1][t];
            }
            const bool even_row = (j & 1) == 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int tx0 = lane + 64 * c, i = i0 + tx0;
                // lanes outside the tile read inside it (their result is dropped)
                const int tx = tx0 >= P2_H && tx0 < P2_H + P2_TI ? tx0 : P2_H;
                const bool odd_i = (i & 1) != 0;
                double w[7];
#pragma unroll
                for (int t = 0; t < 7; ++t) w[t] = odd_i ? wb[t] : wa[t];
                double ax = w[0] * xs[r][tx] + w[1] * xs[r][tx + 1] + w[2] * xs[r][tx - 1] + w[3] * xs[r + 1][tx] +
                            w[4] * xs[r - 1][tx] + w[5] * xs[r - 1][tx + 1] + w[6] * xs[r + 1][tx - 1];
                if (even_row) {
                    const double far = pf.far[0] * xs[r][tx + 2] + pf.far[1] * xs[r][tx - 2] +
                                       pf.far[2] * xs[r + 2][tx] + pf.far[3] * xs[r - 2][tx] +
                                       pf.far[4] * xs[r - 2][tx + 2] + pf.far[5] * xs[r + 2][tx - 2];
                    ax += odd_i ? 0.0 : far;
                }
                double v;
                if (MODE == 0) v = ax;
                else if (MODE == 1) v = fr[k][c] - ax;
                else v = xs[r][tx] + omega * (fr[k][c] - ax) / w[0];
                if (!(tx0 >= P2_H && tx0 < P2_H + P2_TI && j >= 1 && i >= 1 && i + j <= n - 2)) continue;
                y[fb + row_start(n, j) + i] = v;
                push_face_near(gh, n, y, i, j, v);
            }
        }
    } else {
        const int64_t nb = (int64_t)L.F * 3 * n;
        for (int64_t t = (int64_t)(b - gt) * P2_NT + threadIdx.x; t < nb;
             t += (int64_t)(gridDim.x - gt) * P2_NT) {
            const int face = (int)(t / (3 * n)), side = (int)(t / n % 3), s = (int)(t % n);
            int I, J;
            side_point0(side, s, n, I, J);
            part[t] = p2_elem_rows(L, L.p2faces[face], x, face, I, J);
        }
    }
}

// Edge and vertex rows from the faces' partials (fixed order over the faces),
// with every copy.  Dirichlet points: 0 for MODE 0 and 1, unchanged for 2.
template <int MODE>
__global__ __launch_bounds__(NT) void k_p2_low(LevelDev L, const double* __restrict__ x,
                                               const double* __restrict__ f, double* __restrict__ y,
                                               const double* __restrict__ part, double omega) {
    LOW_LOOP(L, 0) {
        const int n = nl_;
        if (t < ne_) {
            const int e = (int)(t / (n - 2)), k = (int)(t % (n - 2)) + 1;
            const EdgeInfo& ei = L.edges[e];
            const int64_t m = edge_main(L, e) + k;
            double v;
            if (ei.boundary) {
                v = MODE == 2 ? x[m] : 0.0;
            } else {
                double ax = 0.0;
                for (int q = 0; q < ei.nf; ++q)
                    ax += part[((int64_t)ei.face[q] * 3 + ei.side[q]) * n + (ei.rev[q] ? n - 1 - k : k)];
                if (MODE == 0) v = ax;
                else if (MODE == 1) v = f[m] - ax;
                else v = x[m] + omega * (f[m] - ax) / L.p2ediag[2 * e + (k & 1)];
            }
            y[m] = v;
            push_edge(L, y, ei, k, v, true);
        } else {
            const int vtx = (int)(t - ne_);
            const VertexInfo& vi = L.verts[vtx];
            const int64_t vb = vert_off(L, vtx);
            double v;
            if (vi.boundary) {
                v = MODE == 2 ? x[vb] : 0.0;
            } else {
                double ax = 0.0;
                for (int c = 0; c < vi.nfc; ++c) {
                    // corner 0: side 0 at t = 0; corner 1: side 0 at n-1; corner 2: side 1 at n-1
                    const int cr = vi.fc_corner[c];
                    ax += part[((int64_t)vi.fc_face[c] * 3 + (cr == 2 ? 1 : 0)) * n + (cr == 0 ? 0 : n - 1)];
                }
                if (MODE == 0) v = ax;
                else if (MODE == 1) v = f[vb] - ax;
                else v = x[vb] + omega * (f[vb] - ax) / L.p2vdiag[vtx];
            }
            y[vb] = v;
            push_vertex(L, y, vi, v);
        }
    }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_p2(const hhg_mesh* M, int fine_level, int mode, const double* x, const double* f, double* y,
                     double* part, double omega, hipStream_t s) {
    const LevelDev L = M->dev(fine_level);
    // one block per tile (a multiple of 8 for the XCD order), then partial blocks
    const int ntiles = L.F * L.n_gs_tl[0][0];
    const int gt = (ntiles + 7) / 8 * 8;
    const int64_t nb = (int64_t)L.F * 3 * L.n;
    const int gb = (int)std::max<int64_t>(1, std::min<int64_t>((nb + P2_NT - 1) / P2_NT, MAX_LOW_BLOCKS));
    int64_t gl = ((int64_t)L.E * (L.n - 2) + L.V + NT - 1) / NT;
    gl = std::max<int64_t>(1, std::min<int64_t>(gl, MAX_LOW_BLOCKS));
    if (mode == 0) {
        k_p2_face<0><<<gt + gb, P2_NT, 0, s>>>(L, x, f, y, part, omega, ntiles, gt);
        k_p2_low<0><<<(int)gl, NT, 0, s>>>(L, x, f, y, part, omega);
    } else if (mode == 1) {
        k_p2_face<1><<<gt + gb, P2_NT, 0, s>>>(L, x, f, y, part, omega, ntiles, gt);
        k_p2_low<1><<<(int)gl, NT, 0, s>>>(L, x, f, y, part, omega);
    } else {
        k_p2_face<2><<<gt + gb, P2_NT, 0, s>>>(L, x, f, y, part, omega, ntiles, gt);
        k_p2_low<2><<<(int)gl, NT, 0, s>>>(L, x, f, y, part, omega);
    }
    return hipGetLastError();
}

}  // namespace hhg
